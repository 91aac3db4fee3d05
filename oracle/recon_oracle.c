/*
 * recon_oracle.c -- CPU oracle for grayscale morphological reconstruction.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do.  It shares no code, header or table with the GPU path.
 *
 * What it computes
 * ----------------
 * The paper (Table 1 in Sec. V-A, and the paragraph after it on irregular
 * operations) builds its ReconToNuclei,
 * FillHoles, Pre-Watershed and RBC-detection operations on morphological
 * reconstruction (MR) and names Vincent's wave-propagation algorithm as the
 * fast CPU method.  The paper does not restate the definition, so the oracle
 * takes the textbook one:
 *
 *   rho_I(J) = fixed point of  J_{n+1} = min(delta_B(J_n), I),  J_0 = min(J, I)
 *
 * where delta_B is the flat dilation by the unit square (8-connectivity) or
 * the unit cross (4-connectivity), truncated at the image border (pixels
 * outside the image do not exist; equivalent to zero padding for the max).
 *
 * The oracle follows Vincent's hybrid sequential algorithm, which reaches that
 * fixed point exactly:
 *   1. clip the marker under the mask;
 *   2. one raster scan (top-to-bottom, left-to-right) taking, for each pixel,
 *      the max over itself and its already-visited neighbours, clipped by the
 *      mask;
 *   3. one anti-raster scan doing the same with the neighbours visited
 *      from the other side, and putting into a FIFO every pixel that could
 *      still raise one of those neighbours;
 *   4. FIFO propagation: pop p, raise every neighbour q with J(q) < J(p) and
 *      J(q) < I(q) to min(J(p), I(q)), and push q.
 *
 * Fill-holes is the reconstruction of the complement (the FillHoles operation
 * of Table 1):  F = 255 - rho_{255-X}(m),  m = 255-X on the one-pixel image
 * frame and 0 inside.  `conn` is the connectivity of that reconstruction,
 * i.e. of the background.
 *
 * Reconstruction by erosion (the dual operation, the first of the operations
 * built next on the same propagation):
 *
 *   rho^e_I(J) = fixed point of  J_{n+1} = max(eps_B(J_n), I),  J_0 = max(J, I)
 *
 * with eps_B the flat erosion (pixels outside the image do not exist: 255
 * padding for the min).  The oracle runs Vincent's hybrid algorithm for it
 * directly, with min and max exchanged -- not through the complement -- so
 * that the duality rho^e_I(J) = 255 - rho_{255-I}(255-J) is a check between
 * two independent codes.
 *
 * The h-dome of I (Vincent's regional-maxima machinery, used by the paper's
 * ReconToNuclei step):  D_h(I) = I - rho_I(max(I - h, 0)),  h >= 1.  Regional
 * maxima: the pixels where D_1(I) > 0 (255 there, 0 elsewhere); a plateau at
 * value 0 is never reported (with any nonzero pixel present it borders a
 * higher one; an all-zero image has no reported maximum -- a reading).
 *
 * Images are dense row-major uint8 arrays of height*width bytes.
 * Return value: 0 on success, -1 on bad arguments, -2 on allocation failure.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---- a growable FIFO of pixel indices --------------------------------- */
typedef struct {
    int64_t *buf;
    int64_t cap, head, count;
} fifo_t;

static int fifo_init(fifo_t *q, int64_t cap)
{
    if (cap < 16) cap = 16;
    q->buf = (int64_t *)malloc((size_t)cap * sizeof(int64_t));
    q->cap = cap;
    q->head = 0;
    q->count = 0;
    return q->buf ? 0 : -1;
}

static int fifo_push(fifo_t *q, int64_t v)
{
    if (q->count == q->cap) {
        int64_t ncap = q->cap * 2;
        int64_t *nb = (int64_t *)malloc((size_t)ncap * sizeof(int64_t));
        if (!nb) return -1;
        for (int64_t i = 0; i < q->count; ++i)
            nb[i] = q->buf[(q->head + i) % q->cap];
        free(q->buf);
        q->buf = nb;
        q->cap = ncap;
        q->head = 0;
    }
    q->buf[(q->head + q->count) % q->cap] = v;
    q->count++;
    return 0;
}

static int64_t fifo_pop(fifo_t *q)
{
    int64_t v = q->buf[q->head];
    q->head = (q->head + 1) % q->cap;
    q->count--;
    return v;
}

/* ---- neighbourhoods ---------------------------------------------------- */
/* Offsets (dy, dx).  The "earlier" half holds the neighbours a raster scan
 * has already visited when it reaches a pixel; the "later" half is its mirror
 * image, visited earlier by the anti-raster scan. */
static const int EARLY8[4][2] = {{0, -1}, {-1, -1}, {-1, 0}, {-1, 1}};
static const int LATE8[4][2]  = {{0, 1}, {1, 1}, {1, 0}, {1, -1}};
static const int EARLY4[2][2] = {{0, -1}, {-1, 0}};
static const int LATE4[2][2]  = {{0, 1}, {1, 0}};

static int inside(int64_t y, int64_t x, int64_t h, int64_t w)
{
    return y >= 0 && y < h && x >= 0 && x < w;
}

static uint8_t u8min(uint8_t a, uint8_t b) { return a < b ? a : b; }
static uint8_t u8max(uint8_t a, uint8_t b) { return a > b ? a : b; }

/* Reconstruction by dilation of mask I from marker J, in place on J. */
static int recon_in_place(uint8_t *J, const uint8_t *I, int64_t h, int64_t w, int conn)
{
    const int (*early)[2] = conn == 8 ? EARLY8 : EARLY4;
    const int (*late)[2] = conn == 8 ? LATE8 : LATE4;
    const int nhalf = conn == 8 ? 4 : 2;
    const int64_t n = h * w;

    /* 1. marker clipped under the mask */
    for (int64_t i = 0; i < n; ++i)
        J[i] = u8min(J[i], I[i]);

    /* 2. raster scan */
    for (int64_t y = 0; y < h; ++y) {
        for (int64_t x = 0; x < w; ++x) {
            uint8_t m = J[y * w + x];
            for (int k = 0; k < nhalf; ++k) {
                int64_t qy = y + early[k][0], qx = x + early[k][1];
                if (inside(qy, qx, h, w)) m = u8max(m, J[qy * w + qx]);
            }
            J[y * w + x] = u8min(m, I[y * w + x]);
        }
    }

    /* 3. anti-raster scan, seeding the FIFO */
    fifo_t q;
    if (fifo_init(&q, n / 8 + 16) != 0) return -2;
    for (int64_t y = h - 1; y >= 0; --y) {
        for (int64_t x = w - 1; x >= 0; --x) {
            const int64_t p = y * w + x;
            uint8_t m = J[p];
            for (int k = 0; k < nhalf; ++k) {
                int64_t qy = y + late[k][0], qx = x + late[k][1];
                if (inside(qy, qx, h, w)) m = u8max(m, J[qy * w + qx]);
            }
            J[p] = u8min(m, I[p]);
            for (int k = 0; k < nhalf; ++k) {
                int64_t qy = y + late[k][0], qx = x + late[k][1];
                if (!inside(qy, qx, h, w)) continue;
                const int64_t r = qy * w + qx;
                if (J[r] < J[p] && J[r] < I[r]) {
                    if (fifo_push(&q, p) != 0) { free(q.buf); return -2; }
                    break;
                }
            }
        }
    }

    /* 4. FIFO propagation over the full neighbourhood */
    while (q.count > 0) {
        const int64_t p = fifo_pop(&q);
        const int64_t y = p / w, x = p % w;
        for (int half = 0; half < 2; ++half) {
            const int (*nb)[2] = half == 0 ? early : late;
            for (int k = 0; k < nhalf; ++k) {
                int64_t qy = y + nb[k][0], qx = x + nb[k][1];
                if (!inside(qy, qx, h, w)) continue;
                const int64_t r = qy * w + qx;
                if (J[r] < J[p] && J[r] != I[r]) {
                    J[r] = u8min(J[p], I[r]);
                    if (fifo_push(&q, r) != 0) { free(q.buf); return -2; }
                }
            }
        }
    }
    free(q.buf);
    return 0;
}

/* rho_mask(marker) into out (out may alias marker, not mask). */
int oracle_recon_dilate(const uint8_t *marker, const uint8_t *mask, uint8_t *out,
                        int64_t height, int64_t width, int conn)
{
    if (!marker || !mask || !out || height < 1 || width < 1) return -1;
    if (conn != 4 && conn != 8) return -1;
    if (out != marker) memcpy(out, marker, (size_t)(height * width));
    return recon_in_place(out, mask, height, width, conn);
}

/* Fill-holes as the reconstruction of the complement, into out. */
int oracle_fill_holes(const uint8_t *img, uint8_t *out, int64_t height, int64_t width, int conn)
{
    if (!img || !out || height < 1 || width < 1) return -1;
    if (conn != 4 && conn != 8) return -1;
    const int64_t n = height * width;
    uint8_t *comp = (uint8_t *)malloc((size_t)n);
    if (!comp) return -2;
    for (int64_t i = 0; i < n; ++i) comp[i] = (uint8_t)(255 - img[i]);
    for (int64_t y = 0; y < height; ++y)
        for (int64_t x = 0; x < width; ++x) {
            const int on_frame = y == 0 || y == height - 1 || x == 0 || x == width - 1;
            out[y * width + x] = on_frame ? comp[y * width + x] : 0;
        }
    int rc = recon_in_place(out, comp, height, width, conn);
    free(comp);
    if (rc != 0) return rc;
    for (int64_t i = 0; i < n; ++i) out[i] = (uint8_t)(255 - out[i]);
    return 0;
}

/* Many same-shaped reconstructions, one after another (used by exhaustive
 * tests to avoid one foreign call per tiny image). */
int oracle_recon_dilate_many(const uint8_t *markers, const uint8_t *masks, uint8_t *outs,
                             int64_t count, int64_t height, int64_t width, int conn)
{
    const int64_t n = height * width;
    for (int64_t i = 0; i < count; ++i) {
        int rc = oracle_recon_dilate(markers + i * n, masks + i * n, outs + i * n,
                                     height, width, conn);
        if (rc != 0) return rc;
    }
    return 0;
}

/* Reconstruction by erosion of mask I from marker J, in place on J: Vincent's
 * hybrid algorithm with min and max exchanged. */
static int recon_erode_in_place(uint8_t *J, const uint8_t *I, int64_t h, int64_t w, int conn)
{
    const int (*early)[2] = conn == 8 ? EARLY8 : EARLY4;
    const int (*late)[2] = conn == 8 ? LATE8 : LATE4;
    const int nhalf = conn == 8 ? 4 : 2;
    const int64_t n = h * w;

    /* 1. marker raised over the mask */
    for (int64_t i = 0; i < n; ++i)
        J[i] = u8max(J[i], I[i]);

    /* 2. raster scan: min over the pixel and its already-visited neighbours, floored by the mask */
    for (int64_t y = 0; y < h; ++y) {
        for (int64_t x = 0; x < w; ++x) {
            uint8_t m = J[y * w + x];
            for (int k = 0; k < nhalf; ++k) {
                int64_t qy = y + early[k][0], qx = x + early[k][1];
                if (inside(qy, qx, h, w)) m = u8min(m, J[qy * w + qx]);
            }
            J[y * w + x] = u8max(m, I[y * w + x]);
        }
    }

    /* 3. anti-raster scan, seeding the FIFO with pixels that can still lower a later neighbour */
    fifo_t q;
    if (fifo_init(&q, n / 8 + 16) != 0) return -2;
    for (int64_t y = h - 1; y >= 0; --y) {
        for (int64_t x = w - 1; x >= 0; --x) {
            const int64_t p = y * w + x;
            uint8_t m = J[p];
            for (int k = 0; k < nhalf; ++k) {
                int64_t qy = y + late[k][0], qx = x + late[k][1];
                if (inside(qy, qx, h, w)) m = u8min(m, J[qy * w + qx]);
            }
            J[p] = u8max(m, I[p]);
            for (int k = 0; k < nhalf; ++k) {
                int64_t qy = y + late[k][0], qx = x + late[k][1];
                if (!inside(qy, qx, h, w)) continue;
                const int64_t r = qy * w + qx;
                if (J[r] > J[p] && J[r] > I[r]) {
                    if (fifo_push(&q, p) != 0) { free(q.buf); return -2; }
                    break;
                }
            }
        }
    }

    /* 4. FIFO propagation over the full neighbourhood */
    while (q.count > 0) {
        const int64_t p = fifo_pop(&q);
        const int64_t y = p / w, x = p % w;
        for (int half = 0; half < 2; ++half) {
            const int (*nb)[2] = half == 0 ? early : late;
            for (int k = 0; k < nhalf; ++k) {
                int64_t qy = y + nb[k][0], qx = x + nb[k][1];
                if (!inside(qy, qx, h, w)) continue;
                const int64_t r = qy * w + qx;
                if (J[r] > J[p] && J[r] != I[r]) {
                    J[r] = u8max(J[p], I[r]);
                    if (fifo_push(&q, r) != 0) { free(q.buf); return -2; }
                }
            }
        }
    }
    free(q.buf);
    return 0;
}

/* rho^e_mask(marker) into out (out may alias marker, not mask). */
int oracle_recon_erode(const uint8_t *marker, const uint8_t *mask, uint8_t *out,
                       int64_t height, int64_t width, int conn)
{
    if (!marker || !mask || !out || height < 1 || width < 1) return -1;
    if (conn != 4 && conn != 8) return -1;
    if (out != marker) memcpy(out, marker, (size_t)(height * width));
    return recon_erode_in_place(out, mask, height, width, conn);
}

/* h-dome D_h(I) = I - rho_I(max(I - h, 0)) into out; h in 1..255. */
int oracle_hdome(const uint8_t *img, uint8_t *out, int64_t height, int64_t width, int hval, int conn)
{
    if (!img || !out || height < 1 || width < 1 || hval < 1 || hval > 255) return -1;
    if (conn != 4 && conn != 8) return -1;
    const int64_t n = height * width;
    for (int64_t i = 0; i < n; ++i) out[i] = (uint8_t)(img[i] > hval ? img[i] - hval : 0);
    int rc = recon_in_place(out, img, height, width, conn);
    if (rc != 0) return rc;
    for (int64_t i = 0; i < n; ++i) out[i] = (uint8_t)(img[i] - out[i]);
    return 0;
}

/* Regional maxima: 255 where D_1(I) > 0, else 0. */
int oracle_regional_max(const uint8_t *img, uint8_t *out, int64_t height, int64_t width, int conn)
{
    int rc = oracle_hdome(img, out, height, width, 1, conn);
    if (rc != 0) return rc;
    const int64_t n = height * width;
    for (int64_t i = 0; i < n; ++i) out[i] = out[i] ? 255 : 0;
    return 0;
}
