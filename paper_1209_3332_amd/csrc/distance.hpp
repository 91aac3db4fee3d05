// distance.hpp -- device code of the exact Euclidean distance transform and
// the distance map of the Pre-Watershed operation (Table 1 of the paper,
// Sec. V-A: Pre-Watershed is built on a distance transformation and
// morphological reconstruction), for AMD MI355X (gfx950).
//
// dist2(p) = min over the 0 pixels q of the image of |p - q|^2 (an exact
// integer; pixels outside the image are not background; 2^31 - 1 when the
// image has no 0 pixel).  D8(p) = min(floor(sqrt(dist2(p))), 255).  The
// Pre-Watershed markers are the regional maxima of D8, computed by the
// reconstruction kernels (the 1-dome) on the D8 plane.
//
// Separable, in two passes:
//   edt_zeros per column segment of EDT_SEG rows: the first and the last row
//             holding a 0 pixel (-1 if none);
//   edt_cols  g(y, x) = distance along column x from row y to the nearest 0
//             pixel of that column (EDT_NONE if none).  A thread owns one
//             column of one segment: it holds the segment's pixels in
//             registers, takes the nearest 0 above and below the segment from
//             the other segments' summaries (the nearest segment that has
//             one), scans down and up and writes g once.
//   edt_rows  one workgroup per row: the row of g is staged in LDS, then
//             every pixel takes min over x' of (x - x')^2 + g(x')^2,
//             searched outward from x and stopped once (x - x')^2 alone
//             reaches the best value (no farther column can do better; the
//             pixel's own column bounds the search by g(x)), inside the
//             columns its segment's anchors found (the minimising column
//             moves right with x).  Writes dist2 (int32) or D8 (uint8), in
//             place over the row it read.
#pragma once
#include "kernels.hpp"

namespace rk {

typedef int32_t i32x4 __attribute__((ext_vector_type(4)));

constexpr int32_t EDT_NONE = 0x3fffffff;   // no 0 pixel in the column
constexpr int EDT_SEG = 16;                // rows per column segment (held in registers)
constexpr int EDT_MAX_W = 16384;           // widest row staged in LDS

struct EdtArgs {
    const uint8_t *img;    // input (0 = background)
    int64_t pitch_img;     // bytes
    int32_t *g;            // column distances, then (mode 0) dist2 in place
    int64_t pitch_g;       // elements
    uint8_t *d8;           // mode 1: D8 output (may be the input image)
    int64_t pitch_d8;      // bytes
    int32_t h, w;
    int32_t mode;          // 0: dist2 into g; 1: D8 into d8
    int32_t *zfirst;       // per (segment, column): first row of the segment with a 0 pixel, or -1
    int32_t *zlast;        // ... last such row, or -1
};

// Column-segment summaries.  Grid-stride over (segment, column), consecutive
// threads on consecutive columns; with dword-aligned rows a thread takes 4
// adjacent columns at once (dword loads).
__global__ void edt_zeros(EdtArgs a) {
    const int64_t n_seg = (a.h + EDT_SEG - 1) / EDT_SEG;
    if (((((uintptr_t)a.img) | (uintptr_t)a.pitch_img | (uintptr_t)a.w) & 3u) == 0) {
        const int w4 = a.w / 4;
        const int64_t n4 = n_seg * w4;
        for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n4; q += (int64_t)gridDim.x * blockDim.x) {
            const int x = (int)(q % w4) * 4;
            const int64_t s = q / w4;
            const int y0 = (int)s * EDT_SEG;
            const RK_GLOBAL uint32_t *col = (const RK_GLOBAL uint32_t *)(gp(a.img) + x);
            uint32_t v[EDT_SEG];
#pragma unroll
            for (int r = 0; r < EDT_SEG; ++r)
                v[r] = y0 + r < a.h ? col[(int64_t)(y0 + r) * (a.pitch_img / 4)] : 0x01010101u;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                int first = -1, last = -1;
#pragma unroll
                for (int r = 0; r < EDT_SEG; ++r)
                    if (((v[r] >> (8 * c)) & 0xffu) == 0u) {
                        if (first < 0) first = y0 + r;
                        last = y0 + r;
                    }
                a.zfirst[s * a.w + x + c] = first;
                a.zlast[s * a.w + x + c] = last;
            }
        }
        return;
    }
    const int64_t n = n_seg * a.w;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(q % a.w);
        const int y0 = (int)(q / a.w) * EDT_SEG;
        const RK_GLOBAL uint8_t *col = gp(a.img) + x;
        uint8_t v[EDT_SEG];
#pragma unroll
        for (int r = 0; r < EDT_SEG; ++r) v[r] = y0 + r < a.h ? col[(int64_t)(y0 + r) * a.pitch_img] : 1;
        int first = -1, last = -1;
#pragma unroll
        for (int r = 0; r < EDT_SEG; ++r)
            if (v[r] == 0) {
                if (first < 0) first = y0 + r;
                last = y0 + r;
            }
        a.zfirst[q] = first;
        a.zlast[q] = last;
    }
}

// Column pass.  Grid-stride over (segment, column) with consecutive threads on
// consecutive columns (coalesced byte loads and int32 stores); with dword-
// aligned image rows a thread takes 4 adjacent columns at once (dword loads,
// and 16-byte stores where the distance plane allows them).
__global__ void edt_cols(EdtArgs a) {
    const int n_seg = (a.h + EDT_SEG - 1) / EDT_SEG;
    if (((((uintptr_t)a.img) | (uintptr_t)a.pitch_img | (uintptr_t)a.w) & 3u) == 0) {
        const int w4 = a.w / 4;
        const int64_t n4 = (int64_t)n_seg * w4;
        const bool vec = ((((uintptr_t)a.g) | (uintptr_t)(a.pitch_g * 4)) & 15u) == 0;
        for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n4; q += (int64_t)gridDim.x * blockDim.x) {
            const int x = (int)(q % w4) * 4;
            const int s = (int)(q / w4);
            const int y0 = s * EDT_SEG, y1 = min(a.h, y0 + EDT_SEG);
            const RK_GLOBAL uint32_t *col = (const RK_GLOBAL uint32_t *)(gp(a.img) + x);
            uint32_t v[EDT_SEG];
#pragma unroll
            for (int r = 0; r < EDT_SEG; ++r)
                v[r] = y0 + r < a.h ? col[(int64_t)(y0 + r) * (a.pitch_img / 4)] : 0x01010101u;
            int g[EDT_SEG][4];
            const int last = y1 - 1 - y0;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                int above = EDT_NONE, below = EDT_NONE;
                for (int t = s - 1; t >= 0; --t) {
                    const int z = a.zlast[(int64_t)t * a.w + x + c];
                    if (z >= 0) {
                        above = y0 - z;
                        break;
                    }
                }
                for (int t = s + 1; t < n_seg; ++t) {
                    const int z = a.zfirst[(int64_t)t * a.w + x + c];
                    if (z >= 0) {
                        below = z - (y1 - 1);
                        break;
                    }
                }
                int d = above;
#pragma unroll
                for (int r = 0; r < EDT_SEG; ++r) {
                    if (((v[r] >> (8 * c)) & 0xffu) == 0u) d = 0;
                    else if (r > 0 && d != EDT_NONE) d += 1;
                    g[r][c] = d;
                }
                d = below;
#pragma unroll
                for (int r = EDT_SEG - 1; r >= 0; --r) {
                    if (r > last) continue;
                    if (((v[r] >> (8 * c)) & 0xffu) == 0u) d = 0;
                    else if (r < last && d != EDT_NONE) d += 1;
                    if (d < g[r][c]) g[r][c] = d;
                }
            }
#pragma unroll
            for (int r = 0; r < EDT_SEG; ++r) {
                if (y0 + r >= a.h) continue;
                int32_t *row = a.g + (int64_t)(y0 + r) * a.pitch_g + x;
                if (vec) {
                    i32x4 o;
                    o.x = g[r][0];
                    o.y = g[r][1];
                    o.z = g[r][2];
                    o.w = g[r][3];
                    *(RK_GLOBAL i32x4 *)row = o;
                } else {
#pragma unroll
                    for (int c = 0; c < 4; ++c) ((RK_GLOBAL int32_t *)row)[c] = g[r][c];
                }
            }
        }
        return;
    }
    const int64_t n = (int64_t)n_seg * a.w;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(q % a.w);
        const int s = (int)(q / a.w);
        const int y0 = s * EDT_SEG, y1 = min(a.h, y0 + EDT_SEG);
        const RK_GLOBAL uint8_t *col = gp(a.img) + x;
        uint8_t v[EDT_SEG];
#pragma unroll
        for (int r = 0; r < EDT_SEG; ++r) v[r] = y0 + r < a.h ? col[(int64_t)(y0 + r) * a.pitch_img] : 1;
        // nearest 0 above row y0 and below row y1 - 1, from the summaries
        int above = EDT_NONE, below = EDT_NONE;
        for (int t = s - 1; t >= 0; --t) {
            const int z = a.zlast[(int64_t)t * a.w + x];
            if (z >= 0) {
                above = y0 - z;
                break;
            }
        }
        for (int t = s + 1; t < n_seg; ++t) {
            const int z = a.zfirst[(int64_t)t * a.w + x];
            if (z >= 0) {
                below = z - (y1 - 1);
                break;
            }
        }
        int g[EDT_SEG];
        int d = above;   // distance from row y0 + r to the nearest 0 at or above it
#pragma unroll
        for (int r = 0; r < EDT_SEG; ++r) {
            if (v[r] == 0) d = 0;
            else if (r > 0 && d != EDT_NONE) d += 1;
            g[r] = d;
        }
        d = below;       // ... at or below it (rows past the image are never 0)
        const int last = y1 - 1 - y0;
#pragma unroll
        for (int r = EDT_SEG - 1; r >= 0; --r) {
            if (r > last) continue;
            if (v[r] == 0) d = 0;
            else if (r < last && d != EDT_NONE) d += 1;
            if (d < g[r]) g[r] = d;
        }
        RK_GLOBAL int32_t *gc = (RK_GLOBAL int32_t *)a.g + x;
#pragma unroll
        for (int r = 0; r < EDT_SEG; ++r)
            if (y0 + r < a.h) gc[(int64_t)(y0 + r) * a.pitch_g] = g[r];
    }
}

__device__ __forceinline__ uint32_t isqrt_cap255(int64_t v) {
    if (v >= 255 * 255) return 255u;
    int64_t r = (int64_t)sqrt((double)v);
    while (r * r > v) --r;
    while ((r + 1) * (r + 1) <= v) ++r;
    return (uint32_t)r;
}

// Row pass.  One workgroup (any size) per row, grid-stride over rows; dynamic
// LDS: w * 4 bytes.
//
// Every pixel x takes min over columns i of f_i(x) = (x - i)^2 + g(i)^2,
// searched outward from its own column and stopped once (x - i)^2 alone
// reaches the best value.  That search is as long as the pixel's distance, so
// it is first tried with EDT_TRY steps, which settles every pixel of ordinary
// images.  A row with pixels left over (few 0 pixels, long distances) bounds
// their searches with anchors: for i < j, f_i - f_j = (j - i)(2x - i - j) +
// g(i)^2 - g(j)^2 grows strictly with x, so every minimising column of a pixel
// lies at or right of every minimising column of any pixel to its left (and
// at or left of those of any pixel to its right).  The row is cut into
// segments of EDT_ANCHOR pixels:
//   1. the anchors (the first pixel of every segment, and the last pixel of
//      the row) search without bound and store a minimising column in the g
//      row, over their own entry (the row itself is in LDS by then);
//   2. every pixel left over searches only inside [column of its segment's
//      anchor, column of the next anchor];
//   3. the anchors' own values follow from their columns.
// The anchors alone pay the long searches (17 of them in a 4096-pixel row).
constexpr int EDT_ANCHOR = 256;
constexpr int EDT_TRY = 64;          // outward steps tried before a pixel is left over
constexpr int EDT_MAX_PER_THREAD = 64;   // pixels per thread and row (16384 / 256); a mask bit each

// In LDS a column distance takes 16 bits (it is below the height, at most
// 16384); EDT_NONE16 marks a column without a 0 pixel.
constexpr uint32_t EDT_NONE16 = 0xffffu;

__device__ __forceinline__ int64_t edt_f(RK_LDS const uint16_t *row, int x, int i) {
    const uint32_t v = row[i];
    return v == EDT_NONE16 ? INT64_MAX : (int64_t)(x - i) * (x - i) + (int64_t)v * v;
}

// Minimum of f_i(x) over i in [lo, hi], visiting columns by increasing |x - i|
// and stopping once (x - i)^2 reaches the best value found, or after
// max_steps distances; *arg receives a minimising column (-1 if every visited
// column is EDT_NONE) and *done whether the search ended by itself (the
// minimum is exact) rather than at max_steps.
__device__ __forceinline__ int64_t edt_search(RK_LDS const uint16_t *row, int x, int lo, int hi, int max_steps,
                                              int *arg, bool *done) {
    int64_t best = INT64_MAX;
    int at = -1;
    auto take = [&](int i) {
        const int64_t f = edt_f(row, x, i);
        if (f < best) {
            best = f;
            at = i;
        }
    };
    bool finished = true;
    if (x < lo) {
        for (int i = lo; i <= hi && (int64_t)(i - x) * (i - x) < best; ++i) take(i);
    } else if (x > hi) {
        for (int i = hi; i >= lo && (int64_t)(x - i) * (x - i) < best; --i) take(i);
    } else {
        take(x);
        int step = 1;
        for (; (x - step >= lo || x + step <= hi) && (int64_t)step * step < best; ++step) {
            if (step > max_steps) {
                finished = false;
                break;
            }
            if (x - step >= lo) take(x - step);
            if (x + step <= hi) take(x + step);
        }
    }
    *arg = at;
    *done = finished;
    return best;
}

__device__ __forceinline__ void edt_put(const EdtArgs &a, RK_GLOBAL int32_t *gr, int y, int x, int64_t best) {
    if (a.mode == 0)
        gr[x] = best == INT64_MAX ? 0x7fffffff : (int32_t)best;
    else
        gp(a.d8)[(int64_t)y * a.pitch_d8 + x] = (uint8_t)(best == INT64_MAX ? 255u : isqrt_cap255(best));
}

__global__ void edt_rows(EdtArgs a) {
    const int w = a.w;
    // the row of column distances, 16 bits each, then (rows wider than
    // EDT_TRY, the only ones that can leave pixels over) two flag words: all
    // inside the w * 4 bytes of dynamic LDS, so the kernel needs no static LDS
    // (which would cost a workgroup per CU of occupancy)
    RK_LDS uint16_t *row = (RK_LDS uint16_t *)dyn_lds();
    RK_LDS int *left_over = (RK_LDS int *)(dyn_lds() + ((2 * w + 3) & ~3));
    const bool may_leave = w > EDT_TRY;
    const int last = w - 1;
    const int n_seg = (w + EDT_ANCHOR - 1) / EDT_ANCHOR;
    // anchors: k * EDT_ANCHOR for k < n_seg, and w - 1 (index n_seg) unless it is one already
    const bool extra = (n_seg - 1) * EDT_ANCHOR != last;
    const int n_anchor = n_seg + (extra ? 1 : 0);
    auto anchor_x = [&](int k) { return k < n_seg ? k * EDT_ANCHOR : last; };
    // "some pixel of the row is left over", one word per parity of the row
    // count: a row's word is cleared during the row before it (after that
    // row's staging barrier, by which every thread has read the word for the
    // row before), set during its first pass and read after the barrier that
    // ends the pass; one barrier, where a workgroup reduction takes three
    if (may_leave && threadIdx.x == 0) {
        left_over[0] = 0;
        left_over[1] = 0;
    }
    int it = 0;
    for (int y = blockIdx.x; y < a.h; y += gridDim.x, ++it) {
        RK_GLOBAL int32_t *gr = (RK_GLOBAL int32_t *)a.g + (int64_t)y * a.pitch_g;
        for (int x = threadIdx.x; x < w; x += blockDim.x) {
            const int32_t v = gr[x];
            row[x] = (uint16_t)(v == EDT_NONE ? EDT_NONE16 : (uint32_t)v);
        }
        __syncthreads();
        if (may_leave && threadIdx.x == 0) left_over[(it + 1) & 1] = 0;
        // every pixel: a short outward search; the pixels it does not settle are left over
        uint64_t open = 0;   // bit m: this thread's m-th pixel (threadIdx.x + m * blockDim.x) is left over
        int m = 0;
        for (int x = threadIdx.x; x < w; x += blockDim.x, ++m) {
            const uint32_t gx = row[x];
            int64_t best = gx == EDT_NONE16 ? INT64_MAX : (int64_t)gx * gx;
            int step = 1;
            for (; step < w && (int64_t)step * step < best && step <= EDT_TRY; ++step) {
                if (x - step >= 0) {
                    const uint32_t v = row[x - step];
                    if (v != EDT_NONE16 && (int64_t)step * step + (int64_t)v * v < best)
                        best = (int64_t)step * step + (int64_t)v * v;
                }
                if (x + step < w) {
                    const uint32_t v = row[x + step];
                    if (v != EDT_NONE16 && (int64_t)step * step + (int64_t)v * v < best)
                        best = (int64_t)step * step + (int64_t)v * v;
                }
            }
            if (step >= w || (int64_t)step * step >= best) edt_put(a, gr, y, x, best);
            else open |= 1ull << m;
        }
        if (open) left_over[it & 1] = 1;   // (only rows wider than EDT_TRY can leave a pixel over)
        // this barrier also orders the settled pixels' stores (anchors' among
        // them) before the anchor entries below, and, when nothing is left
        // over, this row's reads of the LDS row before the next row's staging
        __syncthreads();
        if (may_leave && left_over[it & 1]) {
            // 1. the anchors' columns, kept in the g row
            for (int k = threadIdx.x; k < n_anchor; k += blockDim.x) {
                int arg;
                bool done;
                const int ax = anchor_x(k);
                (void)edt_search(row, ax, 0, last, w, &arg, &done);
                gr[ax] = arg;
            }
            __syncthreads();
            // 2. the pixels left over, each inside its segment's pair of anchor columns
            m = 0;
            for (int x = threadIdx.x; x < w; x += blockDim.x, ++m) {
                const int k = x / EDT_ANCHOR;
                if (!((open >> m) & 1ull) || x == k * EDT_ANCHOR || (extra && x == last)) continue;
                const int lo = gr[k * EDT_ANCHOR];
                const int hi = gr[anchor_x(k + 1)];
                int arg;
                bool done;
                const int64_t best = lo < 0 ? INT64_MAX : edt_search(row, x, lo, hi, w, &arg, &done);
                edt_put(a, gr, y, x, best);
            }
            __syncthreads();
            // 3. the anchors' values (every anchor: the entry of a settled one was overwritten in 1.)
            for (int k = threadIdx.x; k < n_anchor; k += blockDim.x) {
                const int ax = anchor_x(k);
                const int col = gr[ax];
                edt_put(a, gr, y, ax, col < 0 ? INT64_MAX : edt_f(row, ax, col));
            }
            __syncthreads();
        }
    }
}

}  // namespace rk
