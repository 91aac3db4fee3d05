/*
 * label_oracle.c -- CPU oracle for connected-component labelling (BWLabel)
 * and the area filter (AreaThreshold) of binary uint8 images.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; only the tests, the smoke check and the benchmark do.  It
 * shares no code, header or table with the GPU path.
 *
 * What it computes
 * ----------------
 * Table 1 of the paper (Sec. V-A) lists BWLabel and AreaThreshold among the
 * segmentation operations with their own CPU and GPU implementations; the
 * paper does not restate them, so the oracle takes the usual definitions:
 *
 *   BWLabel: the foreground is the set of nonzero pixels; two foreground
 *   pixels are connected if a path of foreground pixels joins them, each step
 *   to one of the 4 edge neighbours (conn = 4) or 8 edge-and-corner
 *   neighbours (conn = 8); pixels outside the image do not exist.  Each
 *   connected component gets one label; background pixels get 0.  Labels are
 *   1..n, numbered in raster order (row by row, left to right) of each
 *   component's first pixel.
 *
 *   AreaThreshold: the area of a component is its pixel count; the output is
 *   255 on the pixels of components whose area lies in [min_area, max_area]
 *   (both inclusive) and 0 elsewhere.
 *
 * Method: a raster scan finds the first pixel of every unlabelled component
 * and labels the whole component from it by a breadth-first flood over the
 * connectivity's neighbours (an explicit FIFO of pixel indices), so labels
 * come out in raster order of first pixels by construction.  The area filter
 * counts the pixels of every label, then writes each pixel's result.
 */
#include <stdint.h>
#include <stdlib.h>

/* labels: h*w int32, dense rows.  Returns the number of components, or -1 on
 * a bad argument or allocation failure. */
int64_t oracle_label(const uint8_t *img, int32_t *labels, int64_t h, int64_t w, int conn) {
    if (!img || !labels || h < 1 || w < 1 || (conn != 4 && conn != 8)) return -1;
    const int64_t n = h * w;
    int64_t *fifo = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!fifo) return -1;
    for (int64_t p = 0; p < n; ++p) labels[p] = 0;
    static const int dy8[8] = {-1, -1, -1, 0, 0, 1, 1, 1}, dx8[8] = {-1, 0, 1, -1, 1, -1, 0, 1};
    static const int dy4[4] = {-1, 0, 0, 1}, dx4[4] = {0, -1, 1, 0};
    const int *dy = conn == 8 ? dy8 : dy4, *dx = conn == 8 ? dx8 : dx4;
    int32_t next = 0;
    for (int64_t s = 0; s < n; ++s) {
        if (img[s] == 0 || labels[s] != 0) continue;
        labels[s] = ++next;
        int64_t head = 0, tail = 0;
        fifo[tail++] = s;
        while (head < tail) {
            const int64_t p = fifo[head++];
            const int64_t y = p / w, x = p % w;
            for (int k = 0; k < conn; ++k) {
                const int64_t yy = y + dy[k], xx = x + dx[k];
                if (yy < 0 || yy >= h || xx < 0 || xx >= w) continue;
                const int64_t q = yy * w + xx;
                if (img[q] != 0 && labels[q] == 0) {
                    labels[q] = next;
                    fifo[tail++] = q;
                }
            }
        }
    }
    free(fifo);
    return next;
}

/* out: h*w uint8 (255 kept, 0 otherwise).  Returns the number of components
 * kept, or -1. */
int64_t oracle_area_threshold(const uint8_t *img, uint8_t *out, int64_t h, int64_t w, int conn,
                              int64_t min_area, int64_t max_area) {
    if (!img || !out || h < 1 || w < 1) return -1;
    const int64_t n = h * w;
    int32_t *labels = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!labels) return -1;
    const int64_t nl = oracle_label(img, labels, h, w, conn);
    if (nl < 0) {
        free(labels);
        return -1;
    }
    int64_t *area = (int64_t *)calloc((size_t)nl + 1, sizeof(int64_t));
    if (!area) {
        free(labels);
        return -1;
    }
    for (int64_t p = 0; p < n; ++p) area[labels[p]] += 1;
    int64_t kept = 0;
    for (int64_t l = 1; l <= nl; ++l)
        if (area[l] >= min_area && area[l] <= max_area) kept += 1;
    for (int64_t p = 0; p < n; ++p) {
        const int32_t l = labels[p];
        out[p] = (l != 0 && area[l] >= min_area && area[l] <= max_area) ? 255 : 0;
    }
    free(area);
    free(labels);
    return kept;
}
