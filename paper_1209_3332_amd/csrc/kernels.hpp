// kernels.hpp -- gfx950 kernels for grayscale reconstruction by dilation.
//
// The reconstruction rho_I(J) is the fixed point of J <- min(dilate(J), I)
// (the morphological reconstruction the paper's segmentation operations are
// built on, Table 1 and the paragraph after it, Sec. V-A).  Any order of
// monotone updates J(q) <- max(J(q), min(J(p), I(q))) over neighbour pairs
// converges to it, which is what lets the work below run out of order.
//
// Work decomposition
//   A tile (H x W) is cut into blocks of BH x 256 pixels.  One wave (64 lanes)
//   owns a block while it works on it: the block's mask I and marker J, plus a
//   one-pixel ring of the neighbours' J (the "halo"), sit in LDS.  Only the
//   owning wave writes a block's pixels, so uint8 pixels never need atomics
//   in global memory.
//   A visit of a block:
//     1. loads I, J (clipped under I) and the halo into LDS;
//     2. on the first visit, runs `scan_rounds` rounds of directional passes
//        (down, up, right, left), each a one-dimensional recursive max/min
//        filter with the diagonal neighbours included for 8-connectivity;
//     3. seeds an LDS queue with every pixel that a neighbour (in the block or
//        in the halo) can still raise, raising it;
//     4. drains the queue (pop p; raise each in-block neighbour q with
//        J(q) < min(J(p), I(q)); push q); on queue overflow it re-seeds;
//     5. writes the changed rows back and, for each neighbouring block whose
//        pixels its border can still raise, requests a visit of that block.
//   A persistent grid of waves pulls first visits from a counter and later
//   visits from a device ring of block ids.  Per-block state bits make sure a
//   block is queued at most once and worked on by one wave at a time; a block
//   requested while it is being worked on is re-run in place by its owner.
//   Termination: a global count of outstanding visits reaching zero; a count
//   per tile reports each tile's convergence.
//
// Fill-holes runs the same machinery on the implicit mask 255 - X with the
// marker held in a scratch plane (initialised to 255 - X on the image frame,
// 0 inside); a final pass writes 255 - J back into the image.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rk {

constexpr int LANES = 64;
constexpr int BW = 256;      // block width: 64 lanes x 4 pixels
constexpr int JP = 268;      // LDS row pitch of J incl. halo columns (67 dwords: odd)
constexpr int JOFF = 4;      // byte offset of column 0 inside a J row (column -1 at 3)
constexpr int IP = 260;      // LDS row pitch of I (65 dwords: odd)

// block state bits
constexpr uint32_t ST_P = 1u;  // first visit not yet started
constexpr uint32_t ST_R = 2u;  // a wave is working on the block
constexpr uint32_t ST_D = 4u;  // visit requested (queued, or re-run pending)

enum { OP_DILATE = 0, OP_FILL = 1 };

struct TaskDev {
    uint8_t *j;            // marker plane (dilate) or fill scratch plane
    const uint8_t *i;      // mask plane (dilate) or the image X (fill; mask = 255 - X)
    uint8_t *img;          // fill: image to receive 255 - J at the end; dilate: unused
    int64_t pitch_j;
    int64_t pitch_i;
    int32_t h, w;
    int32_t conn;
    int32_t op;
    int32_t nby, nbx;
    uint32_t block0;       // first global block id of this task
    int32_t aligned;       // 1 if both planes allow dword access (4-aligned base and pitch)
};

struct Work {
    uint32_t n_tasks;
    uint32_t total_blocks;
    uint32_t next_dense;
    uint32_t pending;
    uint32_t ring_head;
    uint32_t ring_tail;
    uint32_t ring_cap;
    uint32_t abort;          // set by the watchdog: the launch gave up (results incomplete)
    uint32_t progress;       // completed visits (watchdog heartbeat)
    uint32_t pad0[3];
    unsigned long long stat_dense;
    unsigned long long stat_revisit;
    unsigned long long stat_rerun;
    unsigned long long stat_overflow;
    unsigned long long stat_spill;
    unsigned long long pad1[3];
};

struct KArgs {
    const TaskDev *tasks;
    Work *work;
    uint32_t *state;
    uint32_t *ring;
    uint32_t *tile_pending;
    uint32_t *tile_done;
    int32_t qcap;
    int32_t scan_rounds;
    uint64_t watchdog_ticks;   // idle wall-clock ticks without any completed visit before giving up
};

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

// mask of bytes whose value differs between a and b (one bit per byte)
__device__ __forceinline__ uint32_t diff_bytes(uint32_t a, uint32_t b) {
    uint32_t d = a ^ b, m = 0;
    m |= (d & 0x000000ffu) ? 1u : 0u;
    m |= (d & 0x0000ff00u) ? 2u : 0u;
    m |= (d & 0x00ff0000u) ? 4u : 0u;
    m |= (d & 0xff000000u) ? 8u : 0u;
    return m;
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t prefix_count(unsigned long long mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// ---------------------------------------------------------------------------
// global memory access of one dword of 4 pixels at columns x..x+3 of a row,
// with `valid` (0..4) pixels inside the image; bytes past the image read 0.
__device__ __forceinline__ uint32_t gload4(const uint8_t *row, int x, int valid, int aligned) {
    if (valid <= 0) return 0u;
    if (aligned && valid == 4) return *(const uint32_t *)(row + x);
    uint32_t v = 0;
    for (int k = 0; k < valid && k < 4; ++k) v |= (uint32_t)row[x + k] << (8 * k);
    return v;
}

__device__ __forceinline__ void gstore4(uint8_t *row, int x, int valid, int aligned, uint32_t v) {
    if (valid <= 0) return;
    if (aligned && valid == 4) { *(uint32_t *)(row + x) = v; return; }
    for (int k = 0; k < valid && k < 4; ++k) row[x + k] = (uint8_t)(v >> (8 * k));
}

// mask value of one dword: I, or 255 - X for fill-holes (0 outside the image)
__device__ __forceinline__ uint32_t mask4(const TaskDev &t, int gy, int gx, int valid) {
    uint32_t v = gload4(t.i + (int64_t)gy * t.pitch_i, gx, valid, t.aligned);
    if (t.op == OP_FILL) {
        uint32_t keep = valid >= 4 ? 0xffffffffu : ((1u << (8 * valid)) - 1u);
        v = (~v) & keep;
    }
    return v;
}

__device__ __forceinline__ uint32_t mask1(const TaskDev &t, int gy, int gx) {
    uint32_t v = t.i[(int64_t)gy * t.pitch_i + gx];
    return t.op == OP_FILL ? 255u - v : v;
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

struct BlockGeom {
    int y0, x0, bh, bw;
    int has_n, has_s, has_w, has_e;   // neighbouring blocks exist (and touch the block)
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

// Load I and J of the block (J clipped under I) into LDS; bytes outside the image are 0.
template <int BH>
__device__ void load_block(const TaskDev &t, const BlockGeom &g, Lds<BH> &L) {
    const int ln = lane_id();
    const int x = 4 * ln;
    const int valid = min(4, g.bw - x);
    for (int r = 0; r < BH; ++r) {
        uint32_t iv = 0, jv = 0;
        if (r < g.bh && valid > 0) {
            const int gy = g.y0 + r;
            iv = mask4(t, gy, g.x0 + x, valid);
            jv = gload4(t.j + (int64_t)gy * t.pitch_j, g.x0 + x, valid, t.aligned);
            jv = bmin4(jv, iv);
        }
        *L.Iw(r, ln) = iv;
        *L.Jw(r, ln) = jv;
    }
}

// Load the one-pixel ring of neighbour J values around the block (0 outside the image).
template <int BH>
__device__ void load_halo(const TaskDev &t, const BlockGeom &g, Lds<BH> &L) {
    const int ln = lane_id();
    const int x = 4 * ln;
    const int valid = min(4, g.bw - x);
    // rows -1 and BH (columns 0..255)
    uint32_t top = 0, bot = 0;
    if (g.y0 > 0) top = gload4(t.j + (int64_t)(g.y0 - 1) * t.pitch_j, g.x0 + x, valid, t.aligned);
    if (g.bh == BH && g.y0 + BH < t.h)
        bot = gload4(t.j + (int64_t)(g.y0 + BH) * t.pitch_j, g.x0 + x, valid, t.aligned);
    *L.Jw(-1, ln) = top;
    *L.Jw(BH, ln) = bot;
    // columns -1 and 256 for rows -1..BH (lane r handles row r-1 for r = 0..BH+1)
    const bool west = g.x0 > 0;
    const bool east = g.bw == BW && g.x0 + BW < t.w;
    for (int r = ln - 1; r <= BH; r += LANES) {
        const int gy = g.y0 + r;
        const bool row_in = gy >= 0 && gy < t.h && (r < g.bh || r == BH || r == -1) &&
                            !(r == BH && g.bh < BH);
        uint8_t wv = 0, ev = 0;
        if (row_in && west) wv = t.j[(int64_t)gy * t.pitch_j + g.x0 - 1];
        if (row_in && east) ev = t.j[(int64_t)gy * t.pitch_j + g.x0 + BW];
        L.Jb(r, -1) = wv;
        L.Jb(r, BW) = ev;
    }
}

// neighbour bytes of a dword row across lanes: left = pixel x-1, right = pixel x+4
template <int BH>
__device__ __forceinline__ void side_bytes(Lds<BH> &L, int y, uint32_t v, uint32_t &left,
                                           uint32_t &right) {
    const int ln = lane_id();
    uint32_t up = __shfl_up(v, 1);
    uint32_t dn = __shfl_down(v, 1);
    left = ln == 0 ? (uint32_t)L.Jb(y, -1) : (up >> 24);
    right = ln == LANES - 1 ? (uint32_t)L.Jb(y, BW) : (dn & 0xffu);
}

// vertical pass (down if dir > 0, up otherwise); returns nonzero if anything changed
template <int BH>
__device__ bool vpass(Lds<BH> &L, int conn, int dir) {
    const int ln = lane_id();
    int r0 = dir > 0 ? 0 : BH - 1;
    int rprev = dir > 0 ? -1 : BH;
    uint32_t prev = *L.Jw(rprev, ln);
    uint32_t pl, pr;
    side_bytes(L, rprev, prev, pl, pr);
    bool changed = false;
    for (int k = 0; k < BH; ++k) {
        const int r = r0 + dir * k;
        uint32_t cur = *L.Jw(r, ln);
        uint32_t m = bmax4(cur, prev);
        if (conn == 8) {
            m = bmax4(m, (prev << 8) | pl);
            m = bmax4(m, (prev >> 8) | (pr << 24));
        }
        uint32_t nv = bmin4(m, *L.Iw(r, ln));
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
                uint32_t up = __shfl_up(prev, 1);
                uint32_t dn = __shfl_down(prev, 1);
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

// push the pixels flagged in `bits` (one per lane) onto the LDS ring.
// Returns false (and pushes nothing) if they do not fit.
__device__ __forceinline__ bool push_bits(uint16_t *Q, int qcap, uint32_t head, uint32_t &tail,
                                          bool pred, uint32_t pix) {
    const unsigned long long m = __ballot(pred);
    if (m == 0) return true;
    const uint32_t cnt = __popcll(m);
    if (tail - head + cnt > (uint32_t)qcap) return false;
    if (pred) Q[(tail + prefix_count(m)) % (uint32_t)qcap] = (uint16_t)pix;
    tail += cnt;
    return true;
}

// Seed pass: raise every pixel that a neighbour (block or halo) can raise and push it.
// Returns the number of pushed pixels; sets *overflow if some could not be pushed.
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

// Drain the LDS ring.  Returns with the ring empty; *overflow set if pushes were dropped.
template <int BH>
__device__ void drain(Lds<BH> &L, int conn, int qcap, uint32_t &head, uint32_t &tail,
                      bool &overflow) {
    const int ln = lane_id();
    const int ndir = conn == 8 ? 8 : 4;
    const int dys[8] = {-1, 1, 0, 0, -1, -1, 1, 1};
    const int dxs[8] = {0, 0, -1, 1, -1, 1, -1, 1};
    uint32_t iters = 0;
    while (head != tail) {
        if (++iters > (1u << 24)) {   // cannot happen: the raises are bounded; guard anyway
            overflow = false;
            head = tail;
            break;
        }
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

// Write back the dirty rows of J.
template <int BH>
__device__ void store_block(const TaskDev &t, const BlockGeom &g, Lds<BH> &L) {
    const int ln = lane_id();
    const int x = 4 * ln;
    const int valid = min(4, g.bw - x);
    for (int r = 0; r < g.bh; ++r) {
        if (!L.rowdirty[r]) continue;
        gstore4(t.j + (int64_t)(g.y0 + r) * t.pitch_j, g.x0 + x, valid, t.aligned, *L.Jw(r, ln));
    }
}

// ---------------------------------------------------------------------------
// scheduling

__device__ __forceinline__ int find_task(const TaskDev *tasks, int n, uint32_t gblock) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tasks[mid].block0 <= gblock) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Set the abort flag and report true once `start` is older than the watchdog
// budget (or another wave has already aborted).  Every wait in the kernels
// polls this, so every wave exits in bounded time even if the scheduler had
// a bug.
__device__ __forceinline__ bool expired(const KArgs &a, uint64_t start) {
    if (__hip_atomic_load(&a.work->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return true;
    if (wall_clock64() - start > a.watchdog_ticks) {
        __hip_atomic_store(&a.work->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return true;
    }
    return false;
}

__device__ __forceinline__ uint32_t ld_acq(uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

// Request a visit of global block `nb` of task `ti` (called by one lane).
__device__ void request_block(const KArgs &a, int ti, uint32_t nb) {
    const uint32_t old = __hip_atomic_fetch_or(a.state + nb, ST_D, __ATOMIC_ACQ_REL,
                                               __HIP_MEMORY_SCOPE_AGENT);
    if (old & (ST_P | ST_R | ST_D)) return;
    // the block was idle: queue it
    __hip_atomic_fetch_add(a.tile_pending + ti, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add(&a.work->pending, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t pos = __hip_atomic_fetch_add(&a.work->ring_tail, 1u, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
    uint32_t *slot = a.ring + pos % a.work->ring_cap;
    const uint64_t t0 = wall_clock64();
    while (__hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
        if (expired(a, t0)) return;
        __builtin_amdgcn_s_sleep(1);
    }
    __hip_atomic_store(slot, nb + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Border checks after a visit: request every neighbouring block whose pixels
// our border can still raise.  All lanes take part; requests are made by lane 0.
template <int BH>
__device__ void check_neighbours(const KArgs &a, int ti, const TaskDev &t, const BlockGeom &g,
                                 int by, int bx, Lds<BH> &L) {
    const int ln = lane_id();
    const int conn = t.conn;
    const uint32_t gb = t.block0 + (uint32_t)(by * t.nbx + bx);
    bool want[8] = {false, false, false, false, false, false, false, false};
    // N and S edges: lane handles columns 4ln..4ln+3
    {
        const int x = 4 * ln;
        const int valid = min(4, g.bw - x);
        for (int side = 0; side < 2; ++side) {
            const bool exists = side == 0 ? g.has_n : (g.has_s && g.bh == BH);
            if (!exists) continue;
            const int r = side == 0 ? 0 : g.bh - 1;      // our border row
            const int gy = side == 0 ? g.y0 - 1 : g.y0 + BH;
            uint32_t c = *L.Jw(r, ln);
            uint32_t out = c;
            if (conn == 8) {
                uint32_t up = __shfl_up(c, 1), dn = __shfl_down(c, 1);
                uint32_t l = ln == 0 ? 0u : (up >> 24);          // our pixel x-1 (none at x=0)
                uint32_t rr = (ln == LANES - 1) ? 0u : (dn & 0xffu);
                out = bmax4(out, bmax4((c << 8) | l, (c >> 8) | (rr << 24)));
            }
            bool viol = false;
            if (valid > 0) {
                const uint32_t nj = gload4(t.j + (int64_t)gy * t.pitch_j, g.x0 + x, valid, t.aligned);
                const uint32_t ni = mask4(t, gy, g.x0 + x, valid);
                const uint32_t tgt = bmin4(out, ni);
                const uint32_t raised = bmax4(nj, tgt);
                viol = raised != nj;
            }
            if (__ballot(viol)) want[side] = true;
        }
    }
    // W and E edges: lane r handles row r
    {
        const int r = ln;
        for (int side = 0; side < 2; ++side) {
            const bool exists = side == 0 ? g.has_w : (g.has_e && g.bw == BW);
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
                const uint32_t nj = t.j[(int64_t)gy * t.pitch_j + gx];
                const uint32_t tgt = min(out, mask1(t, gy, gx));
                viol = nj < tgt;
            }
            if (__ballot(viol)) want[2 + side] = true;
        }
    }
    // corners (8-connectivity only): lane 0
    if (conn == 8 && ln == 0) {
        for (int c = 0; c < 4; ++c) {
            const bool north = c < 2, west = (c & 1) == 0;
            const bool ex = (north ? g.has_n : (g.has_s && g.bh == BH)) &&
                            (west ? g.has_w : (g.has_e && g.bw == BW));
            if (!ex) continue;
            const int r = north ? 0 : g.bh - 1;
            const int cx = west ? 0 : g.bw - 1;
            const int gy = north ? g.y0 - 1 : g.y0 + BH;
            const int gx = west ? g.x0 - 1 : g.x0 + BW;
            const uint32_t out = L.Jb(r, cx);
            const uint32_t nj = t.j[(int64_t)gy * t.pitch_j + gx];
            if (nj < min(out, mask1(t, gy, gx))) want[4 + c] = true;
        }
    }
    if (ln == 0) {
        const int nbx = t.nbx;
        const int offs[8] = {-nbx, nbx, -1, 1, -nbx - 1, -nbx + 1, nbx - 1, nbx + 1};
        for (int k = 0; k < 8; ++k)
            if (want[k]) request_block(a, ti, (uint32_t)((int)gb + offs[k]));
    }
}

// ---------------------------------------------------------------------------
// the persistent kernel

template <int BH>
__global__ __launch_bounds__(64) void recon_persistent(KArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    Lds<BH> L;
    L.J = smem;
    L.I = smem + (BH + 2) * JP;
    L.rowdirty = L.I + BH * IP;
    L.Q = (uint16_t *)(L.rowdirty + ((BH + 15) & ~15));
    const int ln = lane_id();
    Work *w = a.work;
    const uint32_t total = w->total_blocks;
    const int ntasks = (int)w->n_tasks;

    while (true) {
        // ---- acquire a work item (lane 0), broadcast
        int gsel = -1, dense = 0;
        if (ln == 0) {
            uint32_t seen = __hip_atomic_load(&w->progress, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            uint64_t since = wall_clock64();
            while (true) {
                if (__hip_atomic_load(&w->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
                const uint32_t h = ld_acq(&w->ring_head);
                const uint32_t tl = ld_acq(&w->ring_tail);
                if (h != tl) {
                    uint32_t hh = h;
                    if (__hip_atomic_compare_exchange_strong(&w->ring_head, &hh, h + 1u,
                                                             __ATOMIC_ACQ_REL, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT)) {
                        uint32_t *slot = a.ring + h % w->ring_cap;
                        uint32_t v;
                        const uint64_t t0 = wall_clock64();
                        bool gave_up = false;
                        while ((v = __hip_atomic_exchange(slot, 0u, __ATOMIC_ACQ_REL,
                                                          __HIP_MEMORY_SCOPE_AGENT)) == 0u) {
                            if (expired(a, t0)) { gave_up = true; break; }
                            __builtin_amdgcn_s_sleep(1);
                        }
                        if (gave_up) break;
                        gsel = (int)(v - 1u);
                        dense = 0;
                        break;
                    }
                    continue;
                }
                if (ld_acq(&w->next_dense) < total) {
                    const uint32_t d = __hip_atomic_fetch_add(&w->next_dense, 1u, __ATOMIC_ACQ_REL,
                                                              __HIP_MEMORY_SCOPE_AGENT);
                    if (d < total) {
                        gsel = (int)d;
                        dense = 1;
                        break;
                    }
                }
                if (ld_acq(&w->pending) == 0u) break;
                if (__hip_atomic_load(&w->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
                // watchdog: give up if no visit anywhere completes for too long
                const uint32_t pr = __hip_atomic_load(&w->progress, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const uint64_t now = wall_clock64();
                if (pr != seen) {
                    seen = pr;
                    since = now;
                } else if (now - since > a.watchdog_ticks) {
                    __hip_atomic_store(&w->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        gsel = __shfl(gsel, 0);
        dense = __shfl(dense, 0);
        if (gsel < 0) break;

        const uint32_t gb = (uint32_t)gsel;
        const int ti = find_task(a.tasks, ntasks, gb);
        const TaskDev t = a.tasks[ti];
        const int lb = (int)(gb - t.block0);
        const int by = lb / t.nbx, bx = lb % t.nbx;
        const BlockGeom g = geom<BH>(t, by, bx);

        // ---- claim the block: clear P/D, set R
        if (ln == 0) {
            uint32_t s = __hip_atomic_load(a.state + gb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            while (!__hip_atomic_compare_exchange_weak(a.state + gb, &s, (s & ~(ST_P | ST_D)) | ST_R,
                                                       __ATOMIC_ACQ_REL, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT)) {
            }
            __hip_atomic_fetch_add(dense ? &w->stat_dense : &w->stat_revisit, 1ull,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __threadfence();
        __syncthreads();

        load_block<BH>(t, g, L);
        bool first = true;
        while (true) {
            load_halo<BH>(t, g, L);
            for (int r = ln; r < BH; r += LANES) L.rowdirty[r] = (first && dense) ? 1 : 0;
            __syncthreads();
            bool changed = first && dense;
            if (first && dense) {
                for (int k = 0; k < a.scan_rounds; ++k) {
                    bool c = vpass<BH>(L, t.conn, +1);
                    c |= vpass<BH>(L, t.conn, -1);
                    __syncthreads();
                    c |= hpass<BH>(L, t.conn, +1);
                    c |= hpass<BH>(L, t.conn, -1);
                    __syncthreads();
                    if (!__ballot(c)) break;
                }
            }
            // seed + drain until no overflow
            for (int round = 0;; ++round) {
                if (round > (1 << 16)) {   // cannot happen (each round raises pixels); guard anyway
                    if (ln == 0)
                        __hip_atomic_store(&w->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                uint32_t head = 0, tail = 0;
                bool overflow = false;
                seed_pass<BH>(L, t.conn, a.qcap, head, tail, overflow, changed);
                __syncthreads();
                drain<BH>(L, t.conn, a.qcap, head, tail, overflow);
                __syncthreads();
                if (!__ballot(overflow)) break;
                if (ln == 0)
                    __hip_atomic_fetch_add(&w->stat_overflow, 1ull, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
            }
            // rows raised by the drain also count as changes
            for (int r = 0; r < BH; ++r)
                if (L.rowdirty[r]) changed = true;
            changed = __ballot(changed) != 0;
            if (changed) {
                store_block<BH>(t, g, L);
                __threadfence();
                check_neighbours<BH>(a, ti, t, g, by, bx, L);
            }
            // ---- finish: re-run if requested meanwhile, else release
            int rerun = 0;
            if (ln == 0) {
                uint32_t s = __hip_atomic_load(a.state + gb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                while (true) {
                    const uint32_t ns = (s & ST_D) ? (s & ~ST_D) : (s & ~ST_R);
                    if (__hip_atomic_compare_exchange_weak(a.state + gb, &s, ns, __ATOMIC_ACQ_REL,
                                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                        rerun = (s & ST_D) ? 1 : 0;
                        break;
                    }
                }
                if (rerun)
                    __hip_atomic_fetch_add(&w->stat_rerun, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            rerun = __shfl(rerun, 0);
            __threadfence();
            __syncthreads();
            first = false;
            if (!rerun) break;
        }
        // ---- the visit is complete
        if (ln == 0) {
            const uint32_t left = __hip_atomic_fetch_sub(a.tile_pending + ti, 1u, __ATOMIC_ACQ_REL,
                                                         __HIP_MEMORY_SCOPE_AGENT);
            if (left == 1u)
                __hip_atomic_store(a.tile_done + ti, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            __hip_atomic_fetch_sub(&w->pending, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&w->progress, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// ---------------------------------------------------------------------------
// set-up and finishing kernels (grid-stride)

// Batch header copied in front of the task table; the set-up kernels and the
// persistent kernel read the batch size from it, so a captured launch sequence
// serves every batch that fits the workspace.
struct BatchHdr {
    uint32_t n_tasks;
    uint32_t total_blocks;
    uint32_t ring_cap;
    uint32_t any_fill;
    uint32_t pad[12];
};

// Reset the scheduling state for the tasks of the batch.
__global__ void reset_work(const BatchHdr *hdr, const TaskDev *tasks, Work *w, uint32_t *state,
                           uint32_t *ring, uint32_t *tile_pending, uint32_t *tile_done) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t nth = gridDim.x * blockDim.x;
    const uint32_t n_tasks = hdr->n_tasks, total_blocks = hdr->total_blocks, ring_cap = hdr->ring_cap;
    if (tid == 0) {
        w->n_tasks = n_tasks;
        w->total_blocks = total_blocks;
        w->next_dense = 0;
        w->pending = total_blocks;
        w->ring_head = 0;
        w->ring_tail = 0;
        w->ring_cap = ring_cap;
        w->abort = 0;
        w->progress = 0;
        w->stat_dense = w->stat_revisit = w->stat_rerun = w->stat_overflow = w->stat_spill = 0;
    }
    for (uint32_t i = tid; i < total_blocks; i += nth) state[i] = ST_P;
    for (uint32_t i = tid; i < ring_cap; i += nth) ring[i] = 0;
    for (uint32_t i = tid; i < n_tasks; i += nth) {
        tile_pending[i] = (uint32_t)(tasks[i].nby * tasks[i].nbx);
        tile_done[i] = 0;
    }
}

// Fill-holes marker: 255 - X on the image frame, 0 inside (into the scratch plane).
__global__ void fill_init(const BatchHdr *hdr, const TaskDev *tasks) {
    if (!hdr->any_fill) return;
    for (uint32_t ti = 0; ti < hdr->n_tasks; ++ti) {
        const TaskDev t = tasks[ti];
        if (t.op != OP_FILL) continue;
        const int64_t n = (int64_t)t.h * t.w;
        for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
             p += (int64_t)gridDim.x * blockDim.x) {
            const int y = (int)(p / t.w), x = (int)(p % t.w);
            const bool frame = y == 0 || y == t.h - 1 || x == 0 || x == t.w - 1;
            t.j[(int64_t)y * t.pitch_j + x] =
                frame ? (uint8_t)(255u - t.i[(int64_t)y * t.pitch_i + x]) : (uint8_t)0;
        }
    }
}

// Fill-holes result: image = 255 - J.
__global__ void fill_finish(const BatchHdr *hdr, const TaskDev *tasks) {
    if (!hdr->any_fill) return;
    for (uint32_t ti = 0; ti < hdr->n_tasks; ++ti) {
        const TaskDev t = tasks[ti];
        if (t.op != OP_FILL) continue;
        const int64_t n = (int64_t)t.h * t.w;
        for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
             p += (int64_t)gridDim.x * blockDim.x) {
            const int y = (int)(p / t.w), x = (int)(p % t.w);
            t.img[(int64_t)y * t.pitch_i + x] = (uint8_t)(255u - t.j[(int64_t)y * t.pitch_j + x]);
        }
    }
}

}  // namespace rk
