/*
 * distance_oracle.c -- CPU oracle for the exact Euclidean distance transform
 * and the Pre-Watershed markers built on it.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; only the tests, the smoke check and the benchmark do.  It
 * shares no code, header or table with the GPU path.
 *
 * What it computes
 * ----------------
 * Table 1 of the paper (Sec. V-A) builds its Pre-Watershed operation on
 * morphological reconstruction and a distance transformation, without
 * restating either, so the oracle takes these definitions:
 *
 *   dist2(p) = min over pixels q of the image with value 0 of |p - q|^2
 *              (squared Euclidean distance, an exact integer; pixels outside
 *              the image are not background; 2^31 - 1 if the image has no
 *              0 pixel);
 *   D8(p)    = min(floor(sqrt(dist2(p))), 255);
 *   markers  = the regional maxima of D8 (255 / 0, connectivity conn), i.e.
 *              255 where the 1-dome of D8 is positive.
 *
 * Method, in the plainest exact form: first, per column, the distance to the
 * nearest 0 pixel of that column (a scan down and a scan up); then, per
 * pixel, the minimum over the pixels x' of its row of (x - x')^2 + g(x')^2,
 * searched outward from x and stopped once (x - x')^2 alone reaches the best
 * value found (no farther column can do better).  The regional maxima come
 * from the reconstruction oracle (recon_oracle.c).
 */
#include <stdint.h>
#include <stdlib.h>

int oracle_regional_max(const uint8_t *img, uint8_t *out, int64_t height, int64_t width, int conn);

/* dist2: h*w int32.  Returns 0, or -1 on a bad argument / allocation failure. */
int oracle_distance2(const uint8_t *img, int32_t *dist2, int64_t h, int64_t w) {
    if (!img || !dist2 || h < 1 || w < 1) return -1;
    const int64_t none = -1;   /* no 0 pixel in that column */
    int64_t *g = (int64_t *)malloc((size_t)(h * w) * sizeof(int64_t));
    if (!g) return -1;
    for (int64_t x = 0; x < w; ++x) {
        int64_t d = none;
        for (int64_t y = 0; y < h; ++y) {
            if (img[y * w + x] == 0) d = 0;
            else if (d != none) d += 1;
            g[y * w + x] = d;
        }
        d = none;
        for (int64_t y = h - 1; y >= 0; --y) {
            if (img[y * w + x] == 0) d = 0;
            else if (d != none) d += 1;
            if (d != none && (g[y * w + x] == none || d < g[y * w + x])) g[y * w + x] = d;
        }
    }
    for (int64_t y = 0; y < h; ++y) {
        const int64_t *gr = g + y * w;
        for (int64_t x = 0; x < w; ++x) {
            int64_t best = -1;
            for (int64_t step = 0; step < w; ++step) {
                if (best >= 0 && step * step >= best) break;
                for (int side = 0; side < 2; ++side) {
                    if (step == 0 && side == 1) break;
                    const int64_t xx = side == 0 ? x - step : x + step;
                    if (xx < 0 || xx >= w || gr[xx] == none) continue;
                    const int64_t v = step * step + gr[xx] * gr[xx];
                    if (best < 0 || v < best) best = v;
                }
            }
            dist2[y * w + x] = best < 0 || best > INT32_MAX ? INT32_MAX : (int32_t)best;
        }
    }
    free(g);
    return 0;
}

static int64_t isqrt64(int64_t v) {
    int64_t r = 0;
    while ((r + 1) * (r + 1) <= v) ++r;   /* plain: values here are at most ~2^31 only via the cap */
    return r;
}

/* D8 = min(floor(sqrt(dist2)), 255).  out: h*w uint8.  Returns 0 or -1. */
int oracle_distance8(const uint8_t *img, uint8_t *out, int64_t h, int64_t w) {
    int32_t *d2 = (int32_t *)malloc((size_t)(h * w) * sizeof(int32_t));
    if (!d2) return -1;
    if (oracle_distance2(img, d2, h, w) != 0) {
        free(d2);
        return -1;
    }
    for (int64_t p = 0; p < h * w; ++p)
        out[p] = d2[p] >= 255 * 255 ? 255 : (uint8_t)isqrt64(d2[p]);
    free(d2);
    return 0;
}

/* Pre-Watershed markers: regional maxima of D8.  out: h*w uint8. */
int oracle_pre_watershed(const uint8_t *img, uint8_t *out, int64_t h, int64_t w, int conn) {
    uint8_t *d8 = (uint8_t *)malloc((size_t)(h * w));
    if (!d8) return -1;
    int rc = oracle_distance8(img, d8, h, w);
    if (rc == 0) rc = oracle_regional_max(d8, out, h, w, conn);
    free(d8);
    return rc;
}
