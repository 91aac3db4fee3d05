// label.hpp -- device code of connected-component labelling (BWLabel) and the
// area filter (AreaThreshold) of binary uint8 images, for AMD MI355X (gfx950).
//
// Both are listed in Table 1 of the paper (Sec. V-A) among the segmentation
// operations.  Definitions: the foreground is the set of nonzero pixels; two
// foreground pixels are connected through foreground paths of 4- or
// 8-neighbour steps (pixels outside the image do not exist); each component
// gets one label 1..n, numbered in raster order of its first pixel; the
// background gets 0.  The area filter keeps (255) the pixels of components
// whose pixel count lies in [min_area, max_area] and clears the rest.
//
// Method (union-find on the label plane itself, then a rank relabelling):
//   label_local     one wave per 16 x 256 tile: each row's runs of
//                   foreground pixels become depth-one trees, then one
//                   union-find link (LDS atomic min: the larger root under
//                   the smaller) per pair of touching runs of adjacent rows,
//                   path compression, then every foreground pixel's node id
//                   is written: the pitched index + 1 of its tile root (0 on
//                   the background);
//   label_merge     one wave per tile: the tile's top row and left column
//                   against the neighbouring tiles' pixels, as a global
//                   union-find with agent-scope atomic min on the label plane
//                   (lock-free: a link only ever lowers a root's parent);
//   label_flatten   every pixel's node id becomes its root's; a root (the
//                   component's smallest pitched index, i.e. its raster-first
//                   pixel) sets its bit in a bitmap over pitched indices;
//   rank_*          exclusive prefix count of the bitmap words (per-segment
//                   sums, one wave scanning the segments, per-word offsets);
//   label_final     label = (roots before the pixel's root) + 1.
// Node ids are pitched indices (y * pitch + x) + 1, so the order of ids is the
// raster order and the parent of id a is stored at element a - 1.
#pragma once
#include "kernels.hpp"

namespace rk {

constexpr int LT_H = 16;     // rows of a labelling tile
constexpr int LT_W = 256;    // columns (64 lanes x 4 pixels)
constexpr uint32_t LT_BG = 0xffffffffu;
constexpr int RANK_SEG = 1024;   // bitmap words per scan segment (64 lanes x 16)

struct LabelArgs {
    const uint8_t *img;     // input image (nonzero = foreground)
    int64_t pitch_img;      // bytes
    int32_t *lab;           // label plane (int32), written in place
    int64_t pitch_lab;      // elements
    int32_t h, w;
    int32_t conn;
    int32_t tiles_x;        // tiles per row of tiles
    uint32_t *bits;         // root bitmap over pitched indices (null: no ranks wanted)
    uint32_t *word_off;     // roots before each bitmap word
    uint32_t *seg_sum;      // roots per segment of RANK_SEG words
    uint32_t n_words;
    uint32_t n_segs;
    int32_t *count;         // receives the number of components (may be null)
    int32_t lab_vec;        // 1: the label plane allows 16-byte accesses (base and row pitch)
    int32_t fg_inv;         // 1: the foreground is the pixels below 255 (the complement's nonzero pixels)
};

typedef int32_t i32x4 __attribute__((ext_vector_type(4)));

// 4 label elements at columns x..x+3 of a row (x a multiple of 4); elements
// at or past w read 0 and are not written.
__device__ __forceinline__ void lab_load4(const int32_t *row, int x, int w, int vec, int32_t v[4]) {
    if (vec && x + 4 <= w) {
        const i32x4 q = *(const RK_GLOBAL i32x4 *)(row + x);
        v[0] = q.x;
        v[1] = q.y;
        v[2] = q.z;
        v[3] = q.w;
        return;
    }
    for (int k = 0; k < 4; ++k) v[k] = x + k < w ? ((const RK_GLOBAL int32_t *)row)[x + k] : 0;
}

__device__ __forceinline__ void lab_store4(int32_t *row, int x, int w, int vec, const int32_t v[4]) {
    if (vec && x + 4 <= w) {
        i32x4 q;
        q.x = v[0];
        q.y = v[1];
        q.z = v[2];
        q.w = v[3];
        *(RK_GLOBAL i32x4 *)(row + x) = q;
        return;
    }
    for (int k = 0; k < 4; ++k)
        if (x + k < w) ((RK_GLOBAL int32_t *)row)[x + k] = v[k];
}

// ---- tile-local union-find in LDS (indices within the tile)

__device__ __forceinline__ uint32_t lds_find(RK_LDS uint32_t *par, uint32_t a) {
    while (true) {
        const uint32_t p = __hip_atomic_load(par + a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (p == a) return a;
        a = p;
    }
}

__device__ __forceinline__ void lds_union(RK_LDS uint32_t *par, uint32_t a, uint32_t b) {
    while (true) {
        a = lds_find(par, a);
        b = lds_find(par, b);
        if (a == b) return;
        if (a < b) {
            const uint32_t t = a;
            a = b;
            b = t;
        }
        // a is (or was) a root above b: hang it under b unless someone linked it meanwhile
        const uint32_t old = __hip_atomic_fetch_min(par + a, b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (old == a) return;
        a = old;
    }
}

// ---- global union-find on the label plane (node ids: pitched index + 1)

// Find with path halving: every other node on the path is pointed at its
// grandparent (an atomic minimum: a parent always has the smaller id, so the
// entry only moves up its own tree, whatever other waves write meanwhile).
// Without it, a component spanning many tiles (a background, a corridor)
// builds chains as long as the tiles it crosses, each step a round trip to
// the device-coherent level.
__device__ __forceinline__ int32_t g_find(int32_t *lab, int32_t a) {
    while (true) {
        const int32_t p = __hip_atomic_load((RK_GLOBAL int32_t *)(lab + (a - 1)), __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
        if (p == a) return a;
        const int32_t gp = __hip_atomic_load((RK_GLOBAL int32_t *)(lab + (p - 1)), __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
        if (gp == p) return p;
        __hip_atomic_fetch_min((RK_GLOBAL int32_t *)(lab + (a - 1)), gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        a = gp;
    }
}

__device__ __forceinline__ void g_union(int32_t *lab, int32_t a, int32_t b) {
    while (true) {
        a = g_find(lab, a);
        b = g_find(lab, b);
        if (a == b) return;
        if (a < b) {
            const int32_t t = a;
            a = b;
            b = t;
        }
        const int32_t old = __hip_atomic_fetch_min((RK_GLOBAL int32_t *)(lab + (a - 1)), b, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
        if (old == a) return;
        a = old;
    }
}

__device__ __forceinline__ int img_aligned(const LabelArgs &a) {
    return (((uintptr_t)a.img | (uintptr_t)a.pitch_img) & 3u) == 0;
}

// inclusive prefix maximum over the 64 lanes of a wave (unsigned values; 0
// is the identity): DPP row shifts inside each 16-lane row, then the totals of
// the rows before through readlane
__device__ __forceinline__ uint32_t wave_prefix_max(uint32_t v) {
    v = max(v, dpp_or<DPP_ROW_SHR + 1>(0u, v));
    v = max(v, dpp_or<DPP_ROW_SHR + 2>(0u, v));
    v = max(v, dpp_or<DPP_ROW_SHR + 4>(0u, v));
    v = max(v, dpp_or<DPP_ROW_SHR + 8>(0u, v));
    const uint32_t r0 = (uint32_t)__builtin_amdgcn_readlane((int)v, 15);
    const uint32_t r1 = max(r0, (uint32_t)__builtin_amdgcn_readlane((int)v, 31));
    const uint32_t r2 = max(r1, (uint32_t)__builtin_amdgcn_readlane((int)v, 47));
    return max(v, sel_row(lane_id() >> 4, 0u, r0, r1, r2));
}

// The 4 pixels at columns x..x+3 of row y as foreground bytes: nonzero where
// the pixel is foreground (fg_inv: below 255), 0 elsewhere and past the image.
__device__ __forceinline__ uint32_t fg_load4(const LabelArgs &a, int y, int x, int valid, int aligned) {
    uint32_t v = gload4(a.img + (int64_t)y * a.pitch_img, x, valid, aligned);
    if (a.fg_inv) {
        const uint32_t keep = valid >= 4 ? 0xffffffffu : (valid <= 0 ? 0u : ((1u << (8 * valid)) - 1u));
        v = (~v) & keep;
    }
    return v;
}

// Phase 1: tile-local labelling.  Grid: one 64-lane workgroup per tile
// (grid-stride); dynamic LDS: LT_H * LT_W * 4 bytes.  Lane l holds columns
// 4l..4l+3 of every row.
//   a. runs: every foreground pixel's parent is the first pixel of its run of
//      foreground pixels in the row (one prefix maximum over the lanes of the
//      last background column), so a run is a tree of depth one;
//   b. unions between each run and every run of the row above that touches
//      it, issued once per pair of runs: by the pixel under (4-conn) or
//      diagonally under (8-conn) the upper run's first pixel inside the
//      window the run can reach;
//   c. path compression; d. node ids out.
// label_tile is one tile (all lanes of the wave; `par` holds LT_H * LT_W
// words of LDS); label_local runs it over the tiles of one image.
__device__ void label_tile(const LabelArgs &a, RK_LDS uint32_t *par, int y0, int x0, int aligned) {
    const int ln = lane_id();
    const int c = 4 * ln;
    {
        const int th = min(LT_H, a.h - y0), tw = min(LT_W, a.w - x0);
        const int valid = min(4, tw - c);
        uint64_t fg = 0;   // bit 4r+k: pixel (r, c+k) is foreground
        uint32_t rows[LT_H];   // all loads in flight together
#pragma unroll
        for (int r = 0; r < LT_H; ++r)
            rows[r] = r < th ? fg_load4(a, y0 + r, x0 + c, valid, aligned) : 0u;
#pragma unroll
        for (int r = 0; r < LT_H; ++r) {
            const uint32_t v = rows[r];
            int lb = -1;          // last background column so far in this lane
            int lbk[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const bool f = ((v >> (8 * k)) & 0xffu) != 0u;
                fg |= (uint64_t)(f ? 1u : 0u) << (4 * r + k);
                if (!f) lb = c + k;
                lbk[k] = lb;
            }
            // last background column before this lane (-1: none), through
            // values shifted by one so that 0 is the identity
            const int excl = (int)from_lower(wave_prefix_max((uint32_t)(lb + 1))) - 1;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t i = (uint32_t)(r * LT_W + c + k);
                const bool f = (fg >> (4 * r + k)) & 1u;
                par[i] = f ? (uint32_t)(r * LT_W + max(excl, lbk[k]) + 1) : LT_BG;
            }
        }
        __syncthreads();
        // the neighbouring lanes' foreground bits: 6-bit windows per row with
        // bit 0 = column c-1, bits 1..4 = columns c..c+3, bit 5 = column c+4
        // (no neighbour inside the tile: background; the tile borders are
        // joined by label_merge)
        const uint64_t fl = ((uint64_t)__shfl_up((uint32_t)(fg >> 32), 1u) << 32) | __shfl_up((uint32_t)fg, 1u);
        const uint64_t fr = ((uint64_t)__shfl_down((uint32_t)(fg >> 32), 1u) << 32) | __shfl_down((uint32_t)fg, 1u);
        auto window = [&](int r) -> uint32_t {
            const uint32_t own = (uint32_t)(fg >> (4 * r)) & 15u;
            const uint32_t l = ln > 0 ? (uint32_t)(fl >> (4 * r + 3)) & 1u : 0u;
            const uint32_t rt = ln < LANES - 1 ? (uint32_t)(fr >> (4 * r)) & 1u : 0u;
            return l | (own << 1) | (rt << 5);
        };
        uint32_t wup = window(0);
        for (int r = 1; r < th; ++r) {
            const uint32_t wr = window(r);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (!((wr >> (k + 1)) & 1u)) continue;
                const uint32_t i = (uint32_t)(r * LT_W + c + k);
                const uint32_t u = i - LT_W;   // the pixel above
                const bool left = (wr >> k) & 1u;
                const bool up_left = (wup >> k) & 1u;
                const bool up = (wup >> (k + 1)) & 1u;
                const bool up_right = (wup >> (k + 2)) & 1u;
                if (a.conn == 8) {
                    if (!left) {                                   // the run's first pixel
                        if (up_left) lds_union(par, i, u - 1);
                        else if (up) lds_union(par, i, u);
                    }
                    if (!up && up_right) lds_union(par, i, u + 1);
                } else if (up && (!left || !up_left)) {
                    lds_union(par, i, u);
                }
            }
            wup = wr;
        }
        __syncthreads();
        // path compression of the run starts (every other pixel's parent is its
        // run's start, so afterwards its root is two steps away)
        for (int r = 0; r < th; ++r) {
            const uint32_t wr = window(r);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (((wr >> (k + 1)) & 1u) && !((wr >> k) & 1u)) {
                    const uint32_t i = (uint32_t)(r * LT_W + c + k);
                    par[i] = lds_find(par, i);
                }
            }
        }
        __syncthreads();
        for (int r = 0; r < th; ++r) {
            int32_t ids[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                ids[k] = 0;
                if ((fg >> (4 * r + k)) & 1u) {
                    const uint32_t root = par[par[r * LT_W + c + k]];
                    const int ry = (int)(root / LT_W), rx = (int)(root % LT_W);
                    ids[k] = (int32_t)((int64_t)(y0 + ry) * a.pitch_lab + x0 + rx + 1);
                }
            }
            lab_store4(a.lab + (int64_t)(y0 + r) * a.pitch_lab, x0 + c, a.w, a.lab_vec, ids);
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(64) void label_local(LabelArgs a) {
    RK_LDS uint32_t *par = (RK_LDS uint32_t *)dyn_lds();
    const int n_tiles = a.tiles_x * ((a.h + LT_H - 1) / LT_H);
    const int aligned = img_aligned(a);
    for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x)
        label_tile(a, par, (tile / a.tiles_x) * LT_H, (tile % a.tiles_x) * LT_W, aligned);
}

// Phase 2: unions across tile borders.  One 64-lane workgroup per tile
// (grid-stride).  The top row meets the row above (the tiles above), the left
// column meets the column to the left; with 8-connectivity the diagonal
// neighbours too.  Every pair of adjacent pixels in different tiles is met at
// least once.
// Unions across the tile's top row and left column, issued once per pair of
// touching runs (the rule label_tile uses inside a tile): along the top row,
// pixel x of the tile's row (c) and the row above (a); a pixel whose left
// neighbour c[x-1] is foreground joins a[x-1] and a[x] through it, and a[x+1]
// through a[x] when that is foreground; so with 8-connectivity c[x] links
// a[x-1] (or else a[x]) only if it starts a run, and a[x+1] only if a[x] is
// background; with 4-connectivity a[x] only if c[x-1] and a[x-1] are not both
// foreground.  The left column is the same along the rows (a: column x0 - 1).
// A skip relies on c[x-1] joined to c[x] and a[x-1] to a[x], so it is taken
// only where c[x-1] lies inside this tile (label_tile joined the run); the
// first pixel of the row (or column) always links explicitly.  Then every
// implied link rests on links inside one tile, and a pair of diagonal or
// cross-corner neighbours in other tiles is always linked explicitly.  A
// component spanning many tiles (a background) costs a few unions per tile
// instead of one per border pixel.
__device__ void merge_tile(const LabelArgs &a, int y0, int x0) {
    const int ln = lane_id();
    const int th = min(LT_H, a.h - y0), tw = min(LT_W, a.w - x0);
    auto fg = [&](int y, int x) -> bool {
        return y >= 0 && y < a.h && x >= 0 && x < a.w && a.lab[(int64_t)y * a.pitch_lab + x] != 0;
    };
    auto node = [&](int y, int x) -> int32_t { return a.lab[(int64_t)y * a.pitch_lab + x]; };
    if (y0 > 0) {
        for (int k = 0; k < 4; ++k) {
            const int x = x0 + 4 * ln + k;
            if (x >= x0 + tw || !fg(y0, x)) continue;
            const bool in = x - 1 >= x0;   // c[x-1] inside this tile
            const bool cl = in && fg(y0, x - 1), al = fg(y0 - 1, x - 1), au = fg(y0 - 1, x), ar = fg(y0 - 1, x + 1);
            const int32_t self = node(y0, x);
            if (a.conn == 8) {
                if (!cl) {
                    if (al) g_union(a.lab, self, node(y0 - 1, x - 1));
                    else if (au) g_union(a.lab, self, node(y0 - 1, x));
                }
                if (!au && ar) g_union(a.lab, self, node(y0 - 1, x + 1));
            } else if (au && (!cl || !(in && al))) {
                g_union(a.lab, self, node(y0 - 1, x));
            }
        }
    }
    if (x0 > 0) {
        for (int r = ln; r < th; r += LANES) {
            const int y = y0 + r;
            if (!fg(y, x0)) continue;
            const bool in = r >= 1;   // the pixel above inside this tile
            const bool cl = in && fg(y - 1, x0), al = fg(y - 1, x0 - 1), au = fg(y, x0 - 1), ar = fg(y + 1, x0 - 1);
            const int32_t self = node(y, x0);
            if (a.conn == 8) {
                if (!cl) {
                    if (al) g_union(a.lab, self, node(y - 1, x0 - 1));
                    else if (au) g_union(a.lab, self, node(y, x0 - 1));
                }
                if (!au && ar) g_union(a.lab, self, node(y + 1, x0 - 1));
            } else if (au && (!cl || !(in && al))) {
                g_union(a.lab, self, node(y, x0 - 1));
            }
        }
    }
}

__global__ __launch_bounds__(64) void label_merge(LabelArgs a) {
    const int n_tiles = a.tiles_x * ((a.h + LT_H - 1) / LT_H);
    for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x)
        merge_tile(a, (tile / a.tiles_x) * LT_H, (tile % a.tiles_x) * LT_W);
}

// Clear a word array (a fill kernel rather than a memset node).
__global__ void clear_words(uint32_t *p, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}

// Phase 3: every foreground pixel takes its root's id; roots set their bit.
// Grid-stride over (row, 256-column chunk), 64 lanes x 4 pixels.
__global__ __launch_bounds__(64) void label_flatten(LabelArgs a) {
    const int ln = lane_id();
    const int chunks = (a.w + LT_W - 1) / LT_W;
    const int64_t n = (int64_t)a.h * chunks;
    for (int64_t q = blockIdx.x; q < n; q += gridDim.x) {
        const int y = (int)(q / chunks), x0 = (int)(q % chunks) * LT_W;
        int32_t *row = a.lab + (int64_t)y * a.pitch_lab;
        const int xl = x0 + 4 * ln;
        int32_t v[4];
        lab_load4(row, xl, a.w, a.lab_vec, v);
        bool any = false;
        for (int k = 0; k < 4; ++k) {
            if (v[k] == 0) continue;
            const int32_t root = g_find(a.lab, v[k]);
            any |= root != v[k];
            v[k] = root;
            const int32_t self = (int32_t)((int64_t)y * a.pitch_lab + xl + k + 1);
            if (root == self && a.bits) {
                const uint32_t bit = (uint32_t)(self - 1);
                __hip_atomic_fetch_or(a.bits + (bit >> 5), 1u << (bit & 31u), __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        if (any) lab_store4(row, xl, a.w, a.lab_vec, v);
    }
}

// inclusive prefix sum over the 64 lanes of a wave
__device__ __forceinline__ uint32_t wave_prefix(uint32_t v) {
    const int ln = lane_id();
#pragma unroll
    for (int d = 1; d < LANES; d <<= 1) {
        const uint32_t o = __shfl_up(v, (unsigned)d);
        if (ln >= d) v += o;
    }
    return v;
}

// Phase 4a: roots per segment of RANK_SEG bitmap words.
__global__ __launch_bounds__(64) void rank_segments(LabelArgs a) {
    const int ln = lane_id();
    for (uint32_t s = blockIdx.x; s < a.n_segs; s += gridDim.x) {
        uint32_t sum = 0;
        const uint32_t w0 = s * RANK_SEG + (uint32_t)ln * 16u;
        for (uint32_t j = 0; j < 16u; ++j)
            if (w0 + j < a.n_words) sum += (uint32_t)__popc(a.bits[w0 + j]);
        const uint32_t tot = __shfl(wave_prefix(sum), LANES - 1);
        if (ln == 0) a.seg_sum[s] = tot;
    }
}

// Phase 4b: one wave turns the segment sums into exclusive offsets (in place)
// and writes the number of components.
__global__ __launch_bounds__(64) void rank_scan(LabelArgs a) {
    const int ln = lane_id();
    uint32_t carry = 0;
    for (uint32_t s0 = 0; s0 < a.n_segs; s0 += LANES) {
        const uint32_t s = s0 + (uint32_t)ln;
        const uint32_t v = s < a.n_segs ? a.seg_sum[s] : 0u;
        const uint32_t inc = wave_prefix(v);
        if (s < a.n_segs) a.seg_sum[s] = carry + inc - v;
        carry += __shfl(inc, LANES - 1);
    }
    if (ln == 0 && a.count) *a.count = (int32_t)carry;
}

// Phase 4c: roots before every bitmap word.
__global__ __launch_bounds__(64) void rank_words(LabelArgs a) {
    const int ln = lane_id();
    for (uint32_t s = blockIdx.x; s < a.n_segs; s += gridDim.x) {
        const uint32_t w0 = s * RANK_SEG + (uint32_t)ln * 16u;
        uint32_t cnt[16];
        uint32_t sum = 0;
        for (uint32_t j = 0; j < 16u; ++j) {
            cnt[j] = w0 + j < a.n_words ? (uint32_t)__popc(a.bits[w0 + j]) : 0u;
            sum += cnt[j];
        }
        uint32_t run = a.seg_sum[s] + wave_prefix(sum) - sum;
        for (uint32_t j = 0; j < 16u; ++j) {
            if (w0 + j < a.n_words) a.word_off[w0 + j] = run;
            run += cnt[j];
        }
    }
}

// Phase 5: final labels 1..n in raster order of the roots.
__global__ __launch_bounds__(64) void label_final(LabelArgs a) {
    const int ln = lane_id();
    const int chunks = (a.w + LT_W - 1) / LT_W;
    const int64_t n = (int64_t)a.h * chunks;
    for (int64_t q = blockIdx.x; q < n; q += gridDim.x) {
        const int y = (int)(q / chunks), x0 = (int)(q % chunks) * LT_W;
        int32_t *row = a.lab + (int64_t)y * a.pitch_lab;
        const int xl = x0 + 4 * ln;
        int32_t v[4];
        lab_load4(row, xl, a.w, a.lab_vec, v);
        if ((v[0] | v[1] | v[2] | v[3]) == 0) continue;
        for (int k = 0; k < 4; ++k) {
            if (v[k] == 0) continue;
            const uint32_t r = (uint32_t)(v[k] - 1);
            const uint32_t below = a.bits[r >> 5] & ((1u << (r & 31u)) - 1u);
            v[k] = (int32_t)(a.word_off[r >> 5] + (uint32_t)__popc(below) + 1u);
        }
        lab_store4(row, xl, a.w, a.lab_vec, v);
    }
}

// ---- area filter (on a flattened label plane: every foreground pixel holds
// its component's root id, so no rank relabelling is needed)

struct AreaArgs {
    const int32_t *lab;
    int64_t pitch_lab;
    int32_t lab_vec;
    uint32_t *area;         // pixel count per root id (index 0 unused)
    uint8_t *out;           // the image, overwritten with 255 / 0
    int64_t pitch_out;
    int32_t out_aligned;    // 1: the image allows dword accesses
    int32_t h, w;
    int64_t min_area, max_area;
};

// Pixel counts per root id: runs of equal ids inside a lane's 4 pixels are
// added with one atomic each.
__global__ __launch_bounds__(64) void area_count(AreaArgs a) {
    const int ln = lane_id();
    const int chunks = (a.w + LT_W - 1) / LT_W;
    const int64_t n = (int64_t)a.h * chunks;
    for (int64_t q = blockIdx.x; q < n; q += gridDim.x) {
        const int y = (int)(q / chunks), x0 = (int)(q % chunks) * LT_W;
        const int32_t *row = a.lab + (int64_t)y * a.pitch_lab;
        int32_t vv[4];
        lab_load4(row, x0 + 4 * ln, a.w, a.lab_vec, vv);
        int32_t cur = 0;
        uint32_t run = 0;
        for (int k = 0; k < 4; ++k) {
            const int32_t v = vv[k];
            if (v != cur) {
                if (cur != 0) __hip_atomic_fetch_add(a.area + cur, run, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                cur = v;
                run = 0;
            }
            run += 1;
        }
        if (cur != 0) __hip_atomic_fetch_add(a.area + cur, run, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__global__ __launch_bounds__(64) void area_apply(AreaArgs a) {
    const int ln = lane_id();
    const int chunks = (a.w + LT_W - 1) / LT_W;
    const int64_t n = (int64_t)a.h * chunks;
    for (int64_t q = blockIdx.x; q < n; q += gridDim.x) {
        const int y = (int)(q / chunks), x0 = (int)(q % chunks) * LT_W;
        const int32_t *row = a.lab + (int64_t)y * a.pitch_lab;
        uint8_t *orow = a.out + (int64_t)y * a.pitch_out;
        const int xl = x0 + 4 * ln;
        int32_t vv[4];
        lab_load4(row, xl, a.w, a.lab_vec, vv);
        uint32_t out = 0;
        for (int k = 0; k < 4; ++k) {
            const int32_t v = vv[k];
            const int64_t ar = v != 0 ? (int64_t)a.area[v] : -1;
            if (v != 0 && ar >= a.min_area && ar <= a.max_area) out |= 0xffu << (8 * k);
        }
        gstore4(orow, xl, min(4, a.w - xl), a.out_aligned, out);
    }
}

}  // namespace rk
