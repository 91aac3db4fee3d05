// kernels.hpp -- gfx950 kernels for grayscale reconstruction by dilation.
//
// The reconstruction rho_I(J) is the fixed point of J <- min(dilate(J), I)
// started from min(J, I) (the morphological reconstruction the paper's
// segmentation operations are built on: Table 1 and the paragraph after it,
// Sec. V-A).  Any order of monotone updates J(q) <- max(J(q), min(J(p), I(q)))
// over neighbour pairs converges to it, which is what lets the work below run
// in parallel and out of order.
//
// Work decomposition
//   A tile (H x W) is cut into blocks of BH x 256 pixels.  One wave (64 lanes,
//   4 pixels per lane across a row) owns a block while it works on it; the
//   block's mask I and marker J, plus a one-pixel ring of neighbour values
//   (the "halo"), sit in LDS.  Only the owning wave writes a block's pixels,
//   so uint8 pixels never need atomics in global memory.
//
//   K1 dense_pass     every block once, independently, with an empty halo:
//                     clip, `scan_rounds` rounds of directional passes
//                     (down, up, right, left: one-dimensional recursive max/min
//                     filters, diagonal neighbours included for
//                     8-connectivity), then an LDS queue drained to local
//                     convergence.  The result is exactly the reconstruction
//                     of each block on its own.  No coordination at all.
//   K2 border_seed    for every block, compare its border with the adjacent
//                     pixels of its neighbours and request a visit of each
//                     neighbour that the border can still raise.
//   K3 revisit_drain  a persistent grid of waves pulls requested blocks from a
//                     device ring, reloads them with a fresh halo, seeds an
//                     LDS queue from every pixel a neighbour can raise, drains
//                     it, writes back the changed rows and requests the
//                     neighbours its border can still raise.  Per-block state
//                     bits keep a block in the ring at most once and owned by
//                     one wave at a time (a block requested while owned is
//                     re-run by its owner).  The grid exits when the count of
//                     outstanding visits reaches zero.
//
// Values read from another block may be stale, but never too high: a halo or
// neighbour value is always clipped under its own mask, and owners only ever
// raise pixels.  So any read gives a valid lower bound, and a missed update is
// always caught by the border check of the block that made it.
//
// Fill-holes runs the same kernels on the implicit mask 255 - X with the
// marker held in a scratch plane: K1 computes the initial marker (255 - X on
// the image frame, 0 inside) on the fly, and fill_finish writes 255 - J back
// into the image.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rk {

constexpr int LANES = 64;
constexpr int BW = 256;      // block width: 64 lanes x 4 pixels
constexpr int JP = 268;      // LDS row pitch of J incl. halo columns (67 dwords: odd)
constexpr int JOFF = 4;      // byte offset of column 0 inside a J row (column -1 at 3)
constexpr int IP = 260;      // LDS row pitch of I (65 dwords: odd)
constexpr int MAX_INLINE_TASKS = 12;

// block state bits (revisit scheduler)
constexpr uint32_t ST_R = 2u;  // a wave owns the block
constexpr uint32_t ST_D = 4u;  // visit requested (queued, or re-run pending)

enum { OP_DILATE = 0, OP_FILL = 1 };

struct TaskDev {
    uint8_t *j;            // marker plane (dilate) or fill scratch plane
    const uint8_t *i;      // mask plane (dilate) or the image X (fill: mask = 255 - X)
    uint8_t *img;          // fill: image receiving 255 - J at the end; dilate: unused
    int64_t pitch_j;
    int64_t pitch_i;
    int32_t h, w;
    int32_t conn;
    int32_t op;
    int32_t nby, nbx;
    uint32_t block0;       // first global block id of this task
    int32_t aligned;       // 1 if both planes allow dword access (4-aligned base and pitch)
    int32_t scan_rounds;   // directional pass rounds on the dense pass
    int32_t qcap;          // LDS queue entries (<= the launch's LDS allocation)
};

// Batch header in device memory, in front of a device task table.
struct BatchHdr {
    uint32_t n_tasks;
    uint32_t total_blocks;
    uint32_t ring_cap;
    uint32_t any_fill;
    uint32_t pad[12];
};

// The task list of a launch: up to MAX_INLINE_TASKS tasks travel by value in
// the kernel arguments; larger batches live in device memory (hdr != null).
struct TaskTable {
    const BatchHdr *hdr;
    const TaskDev *ext;
    uint32_t n_inline;
    uint32_t total_inline;
    uint32_t ring_cap_inline;
    uint32_t pad;
    TaskDev inl[MAX_INLINE_TASKS];
};

struct Work {
    uint32_t pending;        // outstanding revisits (queued + running)
    uint32_t ring_head;
    uint32_t ring_tail;
    uint32_t abort;          // set by the watchdog: the launch gave up (results incomplete)
    uint32_t progress;       // completed revisits (watchdog heartbeat)
    uint32_t pad0[3];
    unsigned long long stat_dense;
    unsigned long long stat_revisit;
    unsigned long long stat_rerun;
    unsigned long long stat_overflow;
    unsigned long long stat_request;
    unsigned long long pad1[3];
};

struct KArgs {
    Work *work;
    uint32_t *state;
    uint32_t *ring;
    uint32_t *tile_pending;
    uint32_t *tile_done;
    int32_t qcap;
    int32_t scan_rounds;
    uint64_t watchdog_ticks;   // wall-clock ticks without progress before giving up
};

// ---------------------------------------------------------------------------
// task table access (all indices wave-uniform)

__device__ __forceinline__ uint32_t n_tasks_of(const TaskTable &tt) {
    return tt.hdr ? tt.hdr->n_tasks : tt.n_inline;
}
__device__ __forceinline__ uint32_t total_blocks_of(const TaskTable &tt) {
    return tt.hdr ? tt.hdr->total_blocks : tt.total_inline;
}
__device__ __forceinline__ uint32_t ring_cap_of(const TaskTable &tt) {
    return tt.hdr ? tt.hdr->ring_cap : tt.ring_cap_inline;
}
__device__ __forceinline__ uint32_t block0_of(const TaskTable &tt, int k) {
    return tt.hdr ? tt.ext[k].block0 : tt.inl[k].block0;
}
__device__ __forceinline__ TaskDev task_of(const TaskTable &tt, int k) {
    return tt.hdr ? tt.ext[k] : tt.inl[k];
}

__device__ __forceinline__ int find_task(const TaskTable &tt, uint32_t gblock) {
    int lo = 0, hi = (int)n_tasks_of(tt) - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (block0_of(tt, mid) <= gblock) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint32_t uniform(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

// ---------------------------------------------------------------------------
// byte-lane helpers (4 pixels per 32-bit word)
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t bmax4(uint32_t a, uint32_t b) {
    u16x2 e = __builtin_elementwise_max(__builtin_bit_cast(u16x2, a & 0x00ff00ffu),
                                        __builtin_bit_cast(u16x2, b & 0x00ff00ffu));
    u16x2 o = __builtin_elementwise_max(__builtin_bit_cast(u16x2, (a >> 8) & 0x00ff00ffu),
                                        __builtin_bit_cast(u16x2, (b >> 8) & 0x00ff00ffu));
    return __builtin_bit_cast(uint32_t, e) | (__builtin_bit_cast(uint32_t, o) << 8);
}

__device__ __forceinline__ uint32_t bmin4(uint32_t a, uint32_t b) {
    u16x2 e = __builtin_elementwise_min(__builtin_bit_cast(u16x2, a & 0x00ff00ffu),
                                        __builtin_bit_cast(u16x2, b & 0x00ff00ffu));
    u16x2 o = __builtin_elementwise_min(__builtin_bit_cast(u16x2, (a >> 8) & 0x00ff00ffu),
                                        __builtin_bit_cast(u16x2, (b >> 8) & 0x00ff00ffu));
    return __builtin_bit_cast(uint32_t, e) | (__builtin_bit_cast(uint32_t, o) << 8);
}

__device__ __forceinline__ uint32_t byte_of(uint32_t v, int j) { return (v >> (8 * j)) & 0xffu; }

__device__ __forceinline__ uint32_t set_byte(uint32_t v, int j, uint32_t b) {
    return (v & ~(0xffu << (8 * j))) | (b << (8 * j));
}

// one bit per byte whose value differs between a and b
__device__ __forceinline__ uint32_t diff_bytes(uint32_t a, uint32_t b) {
    const uint32_t d = a ^ b;
    return ((d & 0x000000ffu) ? 1u : 0u) | ((d & 0x0000ff00u) ? 2u : 0u) |
           ((d & 0x00ff0000u) ? 4u : 0u) | ((d & 0xff000000u) ? 8u : 0u);
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Whole-wave shifts by one lane through DPP (a single VALU operation):
// from_lower(v) gives lane i the value of lane i-1 (lane 0 gets 0);
// from_upper(v) gives lane i the value of lane i+1 (lane 63 gets 0).
constexpr int DPP_WAVE_SHL1 = 0x130;
constexpr int DPP_WAVE_SHR1 = 0x138;
__device__ __forceinline__ uint32_t from_lower(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, DPP_WAVE_SHR1, 0xf, 0xf, true);
}
__device__ __forceinline__ uint32_t from_upper(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, DPP_WAVE_SHL1, 0xf, 0xf, true);
}

__device__ __forceinline__ uint32_t prefix_count(unsigned long long mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// ---------------------------------------------------------------------------
// global memory access of the 4 pixels at columns x..x+3 of a row with
// `valid` (0..4) of them inside the image; bytes past the image read 0.
__device__ __forceinline__ uint32_t gload4(const uint8_t *row, int x, int valid, int aligned) {
    if (valid <= 0) return 0u;
    if (aligned && valid == 4) return *(const uint32_t *)(row + x);
    uint32_t v = 0;
    for (int k = 0; k < valid && k < 4; ++k) v |= (uint32_t)row[x + k] << (8 * k);
    return v;
}

__device__ __forceinline__ void gstore4(uint8_t *row, int x, int valid, int aligned, uint32_t v) {
    if (valid <= 0) return;
    if (aligned && valid == 4) {
        *(uint32_t *)(row + x) = v;
        return;
    }
    for (int k = 0; k < valid && k < 4; ++k) row[x + k] = (uint8_t)(v >> (8 * k));
}

// mask value of 4 pixels: I, or 255 - X for fill-holes (0 outside the image)
__device__ __forceinline__ uint32_t mask4(const TaskDev &t, int gy, int gx, int valid) {
    uint32_t v = gload4(t.i + (int64_t)gy * t.pitch_i, gx, valid, t.aligned);
    if (t.op == OP_FILL) {
        const uint32_t keep = valid >= 4 ? 0xffffffffu : (valid <= 0 ? 0u : ((1u << (8 * valid)) - 1u));
        v = (~v) & keep;
    }
    return v;
}

__device__ __forceinline__ uint32_t mask1(const TaskDev &t, int gy, int gx) {
    const uint32_t v = t.i[(int64_t)gy * t.pitch_i + gx];
    return t.op == OP_FILL ? 255u - v : v;
}

// current marker value of one pixel, clipped under its mask
__device__ __forceinline__ uint32_t marker1(const TaskDev &t, int gy, int gx) {
    return min((uint32_t)t.j[(int64_t)gy * t.pitch_j + gx], mask1(t, gy, gx));
}

// current marker of 4 pixels, clipped under their mask
__device__ __forceinline__ uint32_t marker4(const TaskDev &t, int gy, int gx, int valid) {
    return bmin4(gload4(t.j + (int64_t)gy * t.pitch_j, gx, valid, t.aligned), mask4(t, gy, gx, valid));
}

// initial fill-holes marker of 4 pixels: the mask on the image frame, 0 inside
__device__ __forceinline__ uint32_t fill_init4(const TaskDev &t, int gy, int gx, int valid, uint32_t mask) {
    if (gy == 0 || gy == t.h - 1) return mask;
    uint32_t v = 0;
    if (gx == 0 && valid > 0) v |= mask & 0xffu;
    const int last = t.w - 1 - gx;   // byte index of column w-1 inside this word
    if (last >= 0 && last < 4 && last < valid) v |= mask & (0xffu << (8 * last));
    return v;
}

// ---------------------------------------------------------------------------
// per-visit LDS layout
template <int BH>
struct Lds {
    uint8_t *J;          // (BH + 2) rows of JP bytes; pixel (y, x) at (y + 1) * JP + JOFF + x
    uint8_t *I;          // BH rows of IP bytes
    uint8_t *rowdirty;   // BH bytes
    uint16_t *Q;         // queue ring
    __device__ __forceinline__ uint32_t *Jw(int y, int d) {  // dword d of row y (y in -1..BH)
        return (uint32_t *)(J + (y + 1) * JP + JOFF + 4 * d);
    }
    __device__ __forceinline__ uint32_t *Iw(int y, int d) { return (uint32_t *)(I + y * IP + 4 * d); }
    __device__ __forceinline__ uint8_t &Jb(int y, int x) { return J[(y + 1) * JP + JOFF + x]; }
    __device__ __forceinline__ uint8_t &Ib(int y, int x) { return I[y * IP + x]; }
};

template <int BH>
__host__ __device__ constexpr size_t lds_bytes(int qcap) {
    return (size_t)(BH + 2) * JP + (size_t)BH * IP + (size_t)((BH + 15) & ~15) + 2u * (size_t)qcap;
}

// Base of the workgroup's dynamic LDS.  (A host build of these kernels for
// emulated testing supplies its own definition.)
#ifndef RK_DYN_LDS_PROVIDED
__device__ __forceinline__ uint8_t *dyn_lds() {
    extern __shared__ __align__(16) uint8_t rk_smem[];
    return rk_smem;
}
#endif

template <int BH>
__device__ __forceinline__ Lds<BH> lds_layout() {
    Lds<BH> L;
    L.J = dyn_lds();
    L.I = L.J + (BH + 2) * JP;
    L.rowdirty = L.I + BH * IP;
    L.Q = (uint16_t *)(L.rowdirty + ((BH + 15) & ~15));
    return L;
}

struct BlockGeom {
    int y0, x0, bh, bw;
    int has_n, has_s, has_w, has_e;   // neighbouring blocks exist
};

template <int BH>
__device__ __forceinline__ BlockGeom geom(const TaskDev &t, int by, int bx) {
    BlockGeom g;
    g.y0 = by * BH;
    g.x0 = bx * BW;
    g.bh = min(BH, t.h - g.y0);
    g.bw = min(BW, t.w - g.x0);
    g.has_n = by > 0;
    g.has_s = by + 1 < t.nby;
    g.has_w = bx > 0;
    g.has_e = bx + 1 < t.nbx;
    return g;
}

// Load I and J of the block into LDS (J clipped under I; for the first visit
// of a fill-holes block, J is the initial frame marker).  Outside the image: 0.
template <int BH>
__device__ void load_block(const TaskDev &t, const BlockGeom &g, Lds<BH> &L, bool fill_initial) {
    const int ln = lane_id();
    const int x = 4 * ln;
    const int valid = min(4, g.bw - x);
    for (int r = 0; r < BH; ++r) {
        uint32_t iv = 0, jv = 0;
        if (r < g.bh && valid > 0) {
            const int gy = g.y0 + r;
            iv = mask4(t, gy, g.x0 + x, valid);
            if (fill_initial)
                jv = fill_init4(t, gy, g.x0 + x, valid, iv);
            else
                jv = bmin4(gload4(t.j + (int64_t)gy * t.pitch_j, g.x0 + x, valid, t.aligned), iv);
        }
        *L.Iw(r, ln) = iv;
        *L.Jw(r, ln) = jv;
    }
}

// Set the halo ring to 0 (no neighbour information).
template <int BH>
__device__ void clear_halo(Lds<BH> &L) {
    const int ln = lane_id();
    *L.Jw(-1, ln) = 0u;
    *L.Jw(BH, ln) = 0u;
    for (int r = ln - 1; r <= BH; r += LANES) {
        L.Jb(r, -1) = 0;
        L.Jb(r, BW) = 0;
    }
}

// Load the one-pixel ring of neighbour marker values, each clipped under its
// own mask (0 outside the image).
template <int BH>
__device__ void load_halo(const TaskDev &t, const BlockGeom &g, Lds<BH> &L) {
    const int ln = lane_id();
    const int x = 4 * ln;
    const int valid = min(4, g.bw - x);
    uint32_t top = 0, bot = 0;
    if (g.has_n) top = marker4(t, g.y0 - 1, g.x0 + x, valid);
    if (g.has_s) bot = marker4(t, g.y0 + BH, g.x0 + x, valid);
    *L.Jw(-1, ln) = top;
    *L.Jw(BH, ln) = bot;
    // columns -1 and 256 for rows -1..BH (lane k handles row k-1)
    const bool west = g.has_w;
    const bool east = g.has_e;
    for (int r = ln - 1; r <= BH; r += LANES) {
        const bool row_in = (r >= 0 && r < g.bh) || (r == -1 && g.has_n) || (r == BH && g.has_s);
        const int gy = g.y0 + r;
        uint32_t wv = 0, ev = 0;
        if (row_in && west) wv = marker1(t, gy, g.x0 - 1);
        if (row_in && east) ev = marker1(t, gy, g.x0 + BW);
        L.Jb(r, -1) = (uint8_t)wv;
        L.Jb(r, BW) = (uint8_t)ev;
    }
}

// neighbour bytes of a dword row across lanes: left = pixel x-1, right = pixel x+4
template <int BH>
__device__ __forceinline__ void side_bytes(Lds<BH> &L, int y, uint32_t v, uint32_t &left,
                                           uint32_t &right) {
    const int ln = lane_id();
    const uint32_t up = from_lower(v);
    const uint32_t dn = from_upper(v);
    left = ln == 0 ? (uint32_t)L.Jb(y, -1) : (up >> 24);
    right = ln == LANES - 1 ? (uint32_t)L.Jb(y, BW) : (dn & 0xffu);
}

// vertical pass (down if dir > 0, up otherwise); returns true if anything changed
template <int BH>
__device__ bool vpass(Lds<BH> &L, int conn, int dir) {
    const int ln = lane_id();
    const int r0 = dir > 0 ? 0 : BH - 1;
    const int rprev = dir > 0 ? -1 : BH;
    uint32_t prev = *L.Jw(rprev, ln);
    uint32_t pl, pr;
    side_bytes(L, rprev, prev, pl, pr);
    bool changed = false;
    for (int k = 0; k < BH; ++k) {
        const int r = r0 + dir * k;
        const uint32_t cur = *L.Jw(r, ln);
        uint32_t m = bmax4(cur, prev);
        if (conn == 8) {
            m = bmax4(m, (prev << 8) | pl);
            m = bmax4(m, (prev >> 8) | (pr << 24));
        }
        const uint32_t nv = bmin4(m, *L.Iw(r, ln));
        if (nv != cur) {
            *L.Jw(r, ln) = nv;
            changed = true;
        }
        prev = nv;
        side_bytes(L, r, prev, pl, pr);
    }
    return changed;
}

// horizontal pass (right if dir > 0, left otherwise): lane y walks row y
template <int BH>
__device__ bool hpass(Lds<BH> &L, int conn, int dir) {
    const int ln = lane_id();
    const int y = ln < BH ? ln : BH - 1;   // idle lanes shadow the last row (never store)
    const bool active = ln < BH;
    uint32_t prev = dir > 0 ? (uint32_t)L.Jb(y, -1) : (uint32_t)L.Jb(y, BW);
    bool changed = false;
    for (int k = 0; k < BW / 4; ++k) {
        const int d = dir > 0 ? k : BW / 4 - 1 - k;
        uint32_t cur = *L.Jw(y, d);
        const uint32_t iv = *L.Iw(y, d);
        const uint32_t cur0 = cur;
        for (int s = 0; s < 4; ++s) {
            const int j = dir > 0 ? s : 3 - s;
            const int x = 4 * d + j;
            uint32_t m = max(byte_of(cur, j), prev);
            if (conn == 8) {
                uint32_t up = from_lower(prev);
                uint32_t dn = from_upper(prev);
                const int xs = x - dir;   // column the diagonal neighbours sit in
                if (ln == 0) up = L.Jb(-1, xs);
                if (ln == BH - 1) dn = L.Jb(BH, xs);
                m = max(m, max(up, dn));
            }
            const uint32_t v = min(m, byte_of(iv, j));
            cur = set_byte(cur, j, v);
            prev = v;
        }
        if (active && cur != cur0) {
            *L.Jw(y, d) = cur;
            changed = true;
        }
    }
    return changed;
}

// push the pixels flagged by `pred` (one per lane) onto the LDS ring;
// returns false (and pushes nothing) if they do not fit.
__device__ __forceinline__ bool push_bits(uint16_t *Q, int qcap, uint32_t head, uint32_t &tail,
                                          bool pred, uint32_t pix) {
    const unsigned long long m = __ballot(pred);
    if (m == 0) return true;
    const uint32_t cnt = (uint32_t)__popcll(m);
    if (tail - head + cnt > (uint32_t)qcap) return false;
    if (pred) Q[(tail + prefix_count(m)) % (uint32_t)qcap] = (uint16_t)pix;
    tail += cnt;
    return true;
}

// Seed pass: raise every pixel that a neighbour (block or halo) can raise and push it.
template <int BH>
__device__ void seed_pass(Lds<BH> &L, int conn, int qcap, uint32_t head, uint32_t &tail,
                          bool &overflow, bool &changed) {
    const int ln = lane_id();
    for (int r = 0; r < BH; ++r) {
        const uint32_t a = *L.Jw(r - 1, ln);
        const uint32_t c = *L.Jw(r, ln);
        const uint32_t b = *L.Jw(r + 1, ln);
        uint32_t al, ar, cl, cr, bl, br;
        side_bytes(L, r - 1, a, al, ar);
        side_bytes(L, r, c, cl, cr);
        side_bytes(L, r + 1, b, bl, br);
        uint32_t m = bmax4(c, bmax4(a, b));
        m = bmax4(m, bmax4((c << 8) | cl, (c >> 8) | (cr << 24)));
        if (conn == 8) {
            m = bmax4(m, bmax4((a << 8) | al, (a >> 8) | (ar << 24)));
            m = bmax4(m, bmax4((b << 8) | bl, (b >> 8) | (br << 24)));
        }
        const uint32_t nv = bmin4(m, *L.Iw(r, ln));
        const uint32_t dm = diff_bytes(nv, c);
        if (dm) {
            *L.Jw(r, ln) = nv;
            L.rowdirty[r] = 1;
        }
        if (__ballot(dm != 0)) changed = true;
        for (int j = 0; j < 4; ++j) {
            const bool p = (dm >> j) & 1u;
            if (!push_bits(L.Q, qcap, head, tail, p, (uint32_t)(r * BW + 4 * ln + j))) overflow = true;
        }
    }
}

// Raise J(y, x) to `target` if lower; returns true if this lane raised it.
template <int BH>
__device__ __forceinline__ bool raise_px(Lds<BH> &L, int y, int x, uint32_t target) {
    const int off = (y + 1) * JP + JOFF + x;
    uint32_t *wp = (uint32_t *)(L.J + (off & ~3));
    const int sh = 8 * (off & 3);
    uint32_t old = *wp;
    while (true) {
        if (((old >> sh) & 0xffu) >= target) return false;
        const uint32_t nw = (old & ~(0xffu << sh)) | (target << sh);
        const uint32_t prev = atomicCAS(wp, old, nw);
        if (prev == old) return true;
        old = prev;
    }
}

// Border seed: after the halo has been refreshed, only pixels on the block's
// border can be raised by a neighbour (the interior was left converged by the
// previous visit, and only the owner writes it).  Raise and push exactly those.
template <int BH>
__device__ void seed_border(Lds<BH> &L, int conn, int bh, int bw, int qcap, uint32_t head, uint32_t &tail,
                            bool &overflow, bool &changed) {
    const int ln = lane_id();
    // rows 0 and bh-1 (each once): lanes across columns, like the dense seed pass
    for (int pass = 0; pass < 2; ++pass) {
        const int r = pass == 0 ? 0 : bh - 1;
        if (pass == 1 && r == 0) break;
        const uint32_t a = *L.Jw(r - 1, ln);
        const uint32_t c = *L.Jw(r, ln);
        const uint32_t b = *L.Jw(r + 1, ln);
        uint32_t al, ar, cl, cr, bl, br;
        side_bytes(L, r - 1, a, al, ar);
        side_bytes(L, r, c, cl, cr);
        side_bytes(L, r + 1, b, bl, br);
        uint32_t m = bmax4(c, bmax4(a, b));
        m = bmax4(m, bmax4((c << 8) | cl, (c >> 8) | (cr << 24)));
        if (conn == 8) {
            m = bmax4(m, bmax4((a << 8) | al, (a >> 8) | (ar << 24)));
            m = bmax4(m, bmax4((b << 8) | bl, (b >> 8) | (br << 24)));
        }
        const uint32_t nv = bmin4(m, *L.Iw(r, ln));
        const uint32_t dm = diff_bytes(nv, c);
        if (dm) {
            *L.Jw(r, ln) = nv;
            L.rowdirty[r] = 1;
        }
        if (__ballot(dm != 0)) changed = true;
        for (int j = 0; j < 4; ++j) {
            const bool p = (dm >> j) & 1u;
            if (!push_bits(L.Q, qcap, head, tail, p, (uint32_t)(r * BW + 4 * ln + j))) overflow = true;
        }
    }
    __syncthreads();
    // columns 0 and bw-1, rows 1..bh-2: lane r handles row r
    for (int side = 0; side < 2; ++side) {
        const int x = side == 0 ? 0 : bw - 1;
        if (side == 1 && x == 0) break;
        bool raised = false;
        const int r = ln;
        if (r >= 1 && r < bh - 1) {
            uint32_t m = L.Jb(r, x);
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    if (dx == 0 && dy == 0) continue;
                    if (conn == 4 && dx != 0 && dy != 0) continue;
                    m = max(m, (uint32_t)L.Jb(r + dy, x + dx));
                }
            const uint32_t nv = min(m, (uint32_t)L.Ib(r, x));
            if (nv > (uint32_t)L.Jb(r, x)) raised = raise_px(L, r, x, nv);
            if (raised) L.rowdirty[r] = 1;
        }
        if (__ballot(raised)) changed = true;
        if (!push_bits(L.Q, qcap, head, tail, raised, (uint32_t)(r * BW + x))) overflow = true;
        __syncthreads();
    }
}

// Drain the LDS ring to empty; *overflow set if pushes had to be dropped.
template <int BH>
__device__ void drain(Lds<BH> &L, int conn, int qcap, uint32_t &head, uint32_t &tail,
                      bool &overflow) {
    const int ln = lane_id();
    const int ndir = conn == 8 ? 8 : 4;
    const int dys[8] = {-1, 1, 0, 0, -1, -1, 1, 1};
    const int dxs[8] = {0, 0, -1, 1, -1, 1, -1, 1};
    while (head != tail) {
        const uint32_t n = min(tail - head, (uint32_t)LANES);
        const bool valid = (uint32_t)ln < n;
        uint32_t p = 0;
        if (valid) p = L.Q[(head + ln) % (uint32_t)qcap];
        head += n;
        __syncthreads();
        const int y = (int)(p >> 8), x = (int)(p & 255u);
        const uint32_t v = valid ? (uint32_t)L.Jb(y, x) : 0u;
        for (int k = 0; k < ndir; ++k) {
            const int ny = y + dys[k], nx = x + dxs[k];
            bool raised = false;
            if (valid && ny >= 0 && ny < BH && nx >= 0 && nx < BW) {
                const uint32_t tgt = min(v, (uint32_t)L.Ib(ny, nx));
                if ((uint32_t)L.Jb(ny, nx) < tgt) {
                    raised = raise_px(L, ny, nx, tgt);
                    if (raised) L.rowdirty[ny] = 1;
                }
            }
            if (!push_bits(L.Q, qcap, head, tail, raised, (uint32_t)(ny * BW + nx))) overflow = true;
        }
        __syncthreads();
    }
}

// Seed and drain until no queue overflow is left; returns true if anything changed.
// border_only: the first seed looks at the block's border only (valid when the
// interior is already converged and only the halo changed); re-seeds after a
// queue overflow are always dense.
template <int BH>
__device__ bool converge_block(Lds<BH> &L, int conn, int qcap, Work *w, bool border_only, int bh, int bw) {
    bool changed = false;
    for (int round = 0; round <= (1 << 16); ++round) {   // each round raises pixels; bounded anyway
        uint32_t head = 0, tail = 0;
        bool overflow = false;
        if (border_only && round == 0)
            seed_border<BH>(L, conn, bh, bw, qcap, head, tail, overflow, changed);
        else
            seed_pass<BH>(L, conn, qcap, head, tail, overflow, changed);
        __syncthreads();
        drain<BH>(L, conn, qcap, head, tail, overflow);
        __syncthreads();
        if (!__ballot(overflow)) break;
        if (lane_id() == 0)
            __hip_atomic_fetch_add(&w->stat_overflow, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    for (int r = 0; r < BH; ++r)
        if (L.rowdirty[r]) changed = true;
    return __ballot(changed) != 0;
}

// Write back the rows flagged dirty (all rows if `all`).
template <int BH>
__device__ void store_block(const TaskDev &t, const BlockGeom &g, Lds<BH> &L, bool all) {
    const int ln = lane_id();
    const int x = 4 * ln;
    const int valid = min(4, g.bw - x);
    for (int r = 0; r < g.bh; ++r) {
        if (!all && !L.rowdirty[r]) continue;
        gstore4(t.j + (int64_t)(g.y0 + r) * t.pitch_j, g.x0 + x, valid, t.aligned, *L.Jw(r, ln));
    }
}

// ---------------------------------------------------------------------------
// scheduling (revisits)

__device__ __forceinline__ bool expired(const KArgs &a, uint64_t start) {
    return wall_clock64() - start > a.watchdog_ticks;
}

// Idle back-off: about 2^min(k, 6) x 256 cycles, so that hundreds of idle waves
// do not hammer the scheduler's counters while a few waves work.
__device__ __forceinline__ void backoff(int k) {
    const int n = 1 << (k < 6 ? k : 6);
    for (int i = 0; i < n; ++i) __builtin_amdgcn_s_sleep(4);
}

// Request a visit of global block `nb` of task `ti`.  Called by all lanes with
// wave-uniform arguments; lane 0 performs the atomics.  Returns false if the
// watchdog expired while waiting for a ring slot.
__device__ bool request_block(const KArgs &a, uint32_t ring_cap, int ti, uint32_t nb) {
    const int ln = lane_id();
    int pos = -1;
    if (ln == 0) {
        const uint32_t old = __hip_atomic_fetch_or(a.state + nb, ST_D, __ATOMIC_ACQ_REL,
                                                   __HIP_MEMORY_SCOPE_AGENT);
        if (!(old & (ST_R | ST_D))) {   // the block was idle: queue it
            __hip_atomic_fetch_add(a.tile_pending + ti, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&a.work->pending, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&a.work->stat_request, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            pos = (int)(__hip_atomic_fetch_add(&a.work->ring_tail, 1u, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT) % ring_cap);
        }
    }
    pos = uniform(pos);
    if (pos < 0) return true;
    // the slot is free unless its previous occupant has not been taken out yet
    const uint64_t t0 = wall_clock64();
    while (true) {
        int busy = 0;
        if (ln == 0) busy = __hip_atomic_load(a.ring + pos, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
        if (!uniform(busy)) break;
        if (expired(a, t0)) return false;
        __builtin_amdgcn_s_sleep(1);
    }
    if (ln == 0) __hip_atomic_store(a.ring + pos, nb + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    return true;
}

// Border checks: request every neighbouring block whose pixels the block's
// border (in LDS rows 0 / bh-1 and columns 0 / bw-1) can still raise.
// Neighbour pixels are read from global memory, clipped under their mask.
template <int BH>
__device__ bool check_neighbours(const KArgs &a, uint32_t ring_cap, int ti, const TaskDev &t,
                                 const BlockGeom &g, int by, int bx, Lds<BH> &L) {
    const int ln = lane_id();
    const int conn = t.conn;
    const uint32_t gb = t.block0 + (uint32_t)(by * t.nbx + bx);
    uint32_t want = 0;   // bit k: request neighbour k (N, S, W, E, NW, NE, SW, SE)
    {   // N and S edges: lane handles columns 4ln..4ln+3
        const int x = 4 * ln;
        const int valid = min(4, g.bw - x);
        for (int side = 0; side < 2; ++side) {
            const bool exists = side == 0 ? g.has_n : g.has_s;
            if (!exists) continue;
            const int r = side == 0 ? 0 : g.bh - 1;
            const int gy = side == 0 ? g.y0 - 1 : g.y0 + BH;
            const uint32_t c = *L.Jw(r, ln);
            uint32_t out = c;
            if (conn == 8) {
                const uint32_t up = from_lower(c), dn = from_upper(c);
                const uint32_t l = ln == 0 ? 0u : (up >> 24);          // our pixel x-1 (none at x=0)
                const uint32_t rr = ln == LANES - 1 ? 0u : (dn & 0xffu);
                out = bmax4(out, bmax4((c << 8) | l, (c >> 8) | (rr << 24)));
            }
            bool viol = false;
            if (valid > 0) {
                const uint32_t ni = mask4(t, gy, g.x0 + x, valid);
                const uint32_t nj = bmin4(gload4(t.j + (int64_t)gy * t.pitch_j, g.x0 + x, valid, t.aligned), ni);
                viol = bmax4(nj, bmin4(out, ni)) != nj;
            }
            if (__ballot(viol)) want |= 1u << side;
        }
    }
    {   // W and E edges: lane r handles row r
        const int r = ln;
        for (int side = 0; side < 2; ++side) {
            const bool exists = side == 0 ? g.has_w : g.has_e;
            if (!exists) continue;
            const int cx = side == 0 ? 0 : g.bw - 1;
            const int gx = side == 0 ? g.x0 - 1 : g.x0 + BW;
            bool viol = false;
            if (r < g.bh) {
                uint32_t out = L.Jb(r, cx);
                if (conn == 8) {
                    if (r > 0) out = max(out, (uint32_t)L.Jb(r - 1, cx));
                    if (r + 1 < g.bh) out = max(out, (uint32_t)L.Jb(r + 1, cx));
                }
                const int gy = g.y0 + r;
                viol = marker1(t, gy, gx) < min(out, mask1(t, gy, gx));
            }
            if (__ballot(viol)) want |= 4u << side;
        }
    }
    if (conn == 8) {   // corners: lanes 0..3
        bool viol = false;
        if (ln < 4) {
            const bool north = ln < 2, west = (ln & 1) == 0;
            const bool ex = (north ? g.has_n : g.has_s) && (west ? g.has_w : g.has_e);
            if (ex) {
                const int r = north ? 0 : g.bh - 1;
                const int cx = west ? 0 : g.bw - 1;
                const int gy = north ? g.y0 - 1 : g.y0 + BH;
                const int gx = west ? g.x0 - 1 : g.x0 + BW;
                viol = marker1(t, gy, gx) < min((uint32_t)L.Jb(r, cx), mask1(t, gy, gx));
            }
        }
        want |= (uint32_t)(__ballot(viol) & 0xfull) << 4;
    }
    want = uniform(want);
    const int nbx = t.nbx;
    const int offs[8] = {-nbx, nbx, -1, 1, -nbx - 1, -nbx + 1, nbx - 1, nbx + 1};
    for (int k = 0; k < 8; ++k)
        if (want & (1u << k))
            if (!request_block(a, ring_cap, ti, (uint32_t)((int)gb + offs[k]))) return false;
    return true;
}

// ---------------------------------------------------------------------------
// K1: dense pass.  Every block once, independently (empty halo).

template <int BH>
__global__ __launch_bounds__(64) void dense_pass(TaskTable tt, KArgs a) {
    Lds<BH> L = lds_layout<BH>();
    const int ln = lane_id();
    const uint32_t total = total_blocks_of(tt);
    for (uint32_t gb = blockIdx.x; gb < total; gb += gridDim.x) {
        const int ti = uniform(find_task(tt, gb));
        const TaskDev t = task_of(tt, ti);
        const int lb = (int)(gb - t.block0);
        const int by = lb / t.nbx, bx = lb % t.nbx;
        const BlockGeom g = geom<BH>(t, by, bx);
        load_block<BH>(t, g, L, t.op == OP_FILL);
        clear_halo<BH>(L);
        for (int r = ln; r < BH; r += LANES) L.rowdirty[r] = 0;
        __syncthreads();
        for (int k = 0; k < t.scan_rounds; ++k) {
            bool c = vpass<BH>(L, t.conn, +1);
            c |= vpass<BH>(L, t.conn, -1);
            __syncthreads();
            c |= hpass<BH>(L, t.conn, +1);
            c |= hpass<BH>(L, t.conn, -1);
            __syncthreads();
            if (!__ballot(c)) break;
        }
        converge_block<BH>(L, t.conn, t.qcap, a.work, false, g.bh, g.bw);
        store_block<BH>(t, g, L, true);
        if (ln == 0)
            __hip_atomic_fetch_add(&a.work->stat_dense, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
    }
}

// K2: border seeding.  Each block's border against its neighbours.

template <int BH>
__global__ __launch_bounds__(64) void border_seed(TaskTable tt, KArgs a) {
    Lds<BH> L = lds_layout<BH>();
    const int ln = lane_id();
    const uint32_t total = total_blocks_of(tt);
    const uint32_t ring_cap = ring_cap_of(tt);
    for (uint32_t gb = blockIdx.x; gb < total; gb += gridDim.x) {
        const int ti = uniform(find_task(tt, gb));
        const TaskDev t = task_of(tt, ti);
        const int lb = (int)(gb - t.block0);
        const int by = lb / t.nbx, bx = lb % t.nbx;
        const BlockGeom g = geom<BH>(t, by, bx);
        // border rows and columns of the block's current marker into LDS
        const int x = 4 * ln;
        const int valid = min(4, g.bw - x);
        *L.Jw(0, ln) = marker4(t, g.y0, g.x0 + x, valid);
        *L.Jw(g.bh - 1, ln) = marker4(t, g.y0 + g.bh - 1, g.x0 + x, valid);
        for (int r = ln; r < g.bh; r += LANES) {
            L.Jb(r, 0) = (uint8_t)marker1(t, g.y0 + r, g.x0);
            L.Jb(r, g.bw - 1) = (uint8_t)marker1(t, g.y0 + r, g.x0 + g.bw - 1);
        }
        __syncthreads();
        if (!check_neighbours<BH>(a, ring_cap, ti, t, g, by, bx, L)) {
            if (ln == 0) __hip_atomic_store(&a.work->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
        __syncthreads();
    }
}

// K3: revisit scheduler.

template <int BH>
__global__ __launch_bounds__(64) void revisit_drain(TaskTable tt, KArgs a) {
    Lds<BH> L = lds_layout<BH>();
    const int ln = lane_id();
    Work *w = a.work;
    const uint32_t ring_cap = ring_cap_of(tt);

    while (true) {
        // ---- acquire a ring position (or learn that everything is done)
        int pos = -1;   // >= 0: ring position we own; -2: exit
        {
            uint32_t seen = 0;
            if (ln == 0) seen = __hip_atomic_load(&w->progress, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            seen = uniform(seen);
            uint64_t since = wall_clock64();
            for (int spin = 0;; ++spin) {
                int r = -1;
                uint32_t pr = 0;
                if (ln == 0) {
                    if (__hip_atomic_load(&w->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                        r = -2;
                    } else {
                        uint32_t h = __hip_atomic_load(&w->ring_head, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                        const uint32_t tl = __hip_atomic_load(&w->ring_tail, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                        if (h != tl) {
                            if (__hip_atomic_compare_exchange_strong(&w->ring_head, &h, h + 1u, __ATOMIC_ACQ_REL,
                                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                                r = (int)(h % ring_cap);
                        } else if (__hip_atomic_load(&w->pending, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == 0u) {
                            r = -2;
                        }
                    }
                    pr = __hip_atomic_load(&w->progress, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                r = uniform(r);
                pr = uniform(pr);
                if (r != -1) {
                    pos = r;
                    break;
                }
                const uint64_t now = wall_clock64();
                if (pr != seen) {
                    seen = pr;
                    since = now;
                } else if (now - since > a.watchdog_ticks) {
                    if (ln == 0) __hip_atomic_store(&w->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    pos = -2;
                    break;
                }
                backoff(spin);
            }
        }
        if (pos == -2) break;
        // ---- take the block id out of the slot (its producer may still be writing it)
        int gsel = -1;
        {
            const uint64_t t0 = wall_clock64();
            while (true) {
                int v = 0;
                if (ln == 0)
                    v = (int)__hip_atomic_exchange(a.ring + pos, 0u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
                v = uniform(v);
                if (v != 0) {
                    gsel = v - 1;
                    break;
                }
                if (expired(a, t0)) break;
                __builtin_amdgcn_s_sleep(1);
            }
        }
        if (gsel < 0) {
            if (ln == 0) __hip_atomic_store(&w->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
        }

        const uint32_t gb = (uint32_t)gsel;
        const int ti = uniform(find_task(tt, gb));
        const TaskDev t = task_of(tt, ti);
        const int lb = (int)(gb - t.block0);
        const int by = lb / t.nbx, bx = lb % t.nbx;
        const BlockGeom g = geom<BH>(t, by, bx);

        // ---- claim: clear D, set R
        if (ln == 0) {
            uint32_t s = __hip_atomic_load(a.state + gb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            for (int k = 0; k < 1024; ++k) {
                if (__hip_atomic_compare_exchange_strong(a.state + gb, &s, (s & ~ST_D) | ST_R,
                                                         __ATOMIC_ACQ_REL, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT))
                    break;
            }
            __hip_atomic_fetch_add(&w->stat_revisit, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __threadfence();
        __syncthreads();

        load_block<BH>(t, g, L, false);
        bool ok = true;
        while (true) {
            load_halo<BH>(t, g, L);
            for (int r = ln; r < BH; r += LANES) L.rowdirty[r] = 0;
            __syncthreads();
            if (converge_block<BH>(L, t.conn, t.qcap, w, true, g.bh, g.bw)) {
                store_block<BH>(t, g, L, false);
                __threadfence();
                ok = check_neighbours<BH>(a, ring_cap, ti, t, g, by, bx, L);
            }
            // ---- finish: re-run if requested meanwhile, else release
            int rerun = 0;
            if (ln == 0) {
                uint32_t s = __hip_atomic_load(a.state + gb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                for (int k = 0; k < 1024; ++k) {
                    const uint32_t ns = (s & ST_D) ? (s & ~ST_D) : (s & ~ST_R);
                    if (__hip_atomic_compare_exchange_strong(a.state + gb, &s, ns, __ATOMIC_ACQ_REL,
                                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                        rerun = (s & ST_D) ? 1 : 0;
                        break;
                    }
                }
                if (rerun)
                    __hip_atomic_fetch_add(&w->stat_rerun, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            rerun = uniform(rerun);
            __threadfence();
            __syncthreads();
            if (!rerun || !ok) break;
        }
        // ---- the visit is complete
        if (ln == 0) {
            const uint32_t left = __hip_atomic_fetch_sub(a.tile_pending + ti, 1u, __ATOMIC_ACQ_REL,
                                                         __HIP_MEMORY_SCOPE_AGENT);
            if (left == 1u)
                __hip_atomic_store(a.tile_done + ti, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_sub(&w->pending, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&w->progress, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (!ok) __hip_atomic_store(&w->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (!ok) break;
    }
}

// ---------------------------------------------------------------------------
// set-up and finishing kernels (grid-stride)

// Copy a task table from host-visible memory into the device table.
__global__ void copy_table(const uint8_t *src, uint8_t *dst, uint32_t bytes) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < bytes; i += gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// Reset the scheduling state of the batch.
__global__ void reset_work(TaskTable tt, Work *w, uint32_t *state, uint32_t *ring,
                           uint32_t *tile_pending, uint32_t *tile_done) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t nth = gridDim.x * blockDim.x;
    const uint32_t n_tasks = n_tasks_of(tt), total = total_blocks_of(tt), ring_cap = ring_cap_of(tt);
    if (tid == 0) {
        w->pending = 0;
        w->ring_head = 0;
        w->ring_tail = 0;
        w->abort = 0;
        w->progress = 0;
        w->stat_dense = w->stat_revisit = w->stat_rerun = w->stat_overflow = w->stat_request = 0;
    }
    for (uint32_t i = tid; i < total; i += nth) state[i] = 0;
    for (uint32_t i = tid; i < ring_cap; i += nth) ring[i] = 0;
    for (uint32_t i = tid; i < n_tasks; i += nth) {
        tile_pending[i] = 0;
        tile_done[i] = 0;
    }
}

// Fill-holes result: image = 255 - J.
__global__ void fill_finish(TaskTable tt) {
    const uint32_t n = n_tasks_of(tt);
    for (uint32_t ti = 0; ti < n; ++ti) {
        const TaskDev t = task_of(tt, (int)ti);
        if (t.op != OP_FILL) continue;
        const int64_t npx = (int64_t)t.h * t.w;
        for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < npx;
             p += (int64_t)gridDim.x * blockDim.x) {
            const int y = (int)(p / t.w), x = (int)(p % t.w);
            t.img[(int64_t)y * t.pitch_i + x] = (uint8_t)(255u - t.j[(int64_t)y * t.pitch_j + x]);
        }
    }
}

// Self-test (checks that this code object runs and that the one-lane DPP
// shifts move data the way the kernels assume):
//   out[i] = 3 i + 1,  out[n + i] = from_lower(i + 100),  out[2n + i] = from_upper(i + 100)
// for i < n, with n a multiple of the block size (all lanes active).
__global__ void self_test(uint32_t *out, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t lo = from_lower(i + 100u), hi = from_upper(i + 100u);
    if (i < n) {
        out[i] = i * 3u + 1u;
        out[n + i] = lo;
        out[2 * n + i] = hi;
    }
}

}  // namespace rk
