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
// The other operations run the same kernels on a transformed pair (the
// transform is applied when the mask is read, and by init_marker to the
// marker plane before the first visit; finish_result maps the fixed point
// back):
//   fill-holes       mask 255 - X, marker in a scratch plane: 255 - X on the
//                    image frame, 0 inside; result 255 - J into the image;
//   erosion          mask 255 - I, marker 255 - J complemented in place in the
//                    caller's marker plane; result 255 - J in the same plane
//                    (reconstruction by erosion is the dual of dilation);
//   h-dome           mask I, marker max(I - h, 0) in a scratch plane; result
//                    I - J into the image;
//   regional maxima  the 1-dome, result 255 where it is positive, else 0.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// Address spaces of LDS and global pointers (the host emulation of these
// kernels defines both empty).  Image planes reach the kernels as plain
// pointers; accesses go through gp(), so that they are global (not flat)
// instructions and never wait on, or delay, LDS traffic.
#ifndef RK_LDS
#define RK_LDS __attribute__((address_space(3)))
#define RK_GLOBAL __attribute__((address_space(1)))
#endif

namespace rk {

constexpr int LANES = 64;
constexpr int BW = 256;      // block width: 64 lanes x 4 pixels
constexpr int JP = 268;      // LDS row pitch of J incl. halo columns (67 dwords: odd)
constexpr int JOFF = 4;      // byte offset of column 0 inside a J row (column -1 at 3)
constexpr int MAX_INLINE_TASKS = 12;
constexpr int RING_STRIDE = 16;       // ring slots are 64 bytes apart (one waiter per slot line)
constexpr int STATE_STRIDE = 32;      // block state words are 128 bytes apart (no shared atomic lines)
constexpr int MAX_DRAIN_GRID = 4096;  // upper bound of the revisit kernel's grid

// block state bits (revisit scheduler)
constexpr uint32_t ST_R = 2u;  // a wave owns the block
constexpr uint32_t ST_D = 4u;  // visit requested (queued, or re-run pending)
constexpr uint32_t ST_V = 8u;  // the block has had its first (dense) visit

enum { OP_DILATE = 0, OP_FILL = 1, OP_ERODE = 2, OP_HDOME = 3, OP_RMAX = 4 };

struct TaskDev {
    uint8_t *j;            // marker plane: the caller's (dilate, erode) or a scratch plane
    const uint8_t *i;      // mask plane, or the image the mask is derived from
    uint8_t *img;          // plane receiving the mapped result at the end (unused by dilate)
    int64_t pitch_j;
    int64_t pitch_i;
    int64_t pitch_img;
    int32_t h, w;
    int32_t conn;
    int32_t op;
    int32_t minv;          // 1: the mask is 255 - (the plane i) (fill-holes, erosion)
    int32_t hval;          // h-dome height (h-dome: h, regional maxima: 1)
    int32_t nby, nbx;
    uint32_t block0;       // first global block id of this task
    int32_t aligned;       // 1 if both planes allow dword access (4-aligned base and pitch)
    int32_t scan_rounds;   // directional pass rounds on the dense pass
    int32_t qcap;          // LDS queue entries (<= the launch's LDS allocation)
    int32_t *lab;          // int32 label plane of the component route (null: the task never takes it)
    int64_t pitch_lab;     // its row pitch in elements (a multiple of 4)
};

// Batch header in device memory, in front of a device task table.
struct BatchHdr {
    uint32_t n_tasks;
    uint32_t total_blocks;
    uint32_t ring_cap;
    uint32_t any_mapped;   // some task needs init_marker / finish_result
    uint32_t launch_seq;   // the launch's number (marks the per-launch flags of Work)
    uint32_t pad[11];
};

// The task list of a launch: up to MAX_INLINE_TASKS tasks travel by value in
// the kernel arguments; larger batches live in device memory (hdr != null).
struct TaskTable {
    const BatchHdr *hdr;
    const TaskDev *ext;
    uint32_t n_inline;
    uint32_t total_inline;
    uint32_t ring_cap_inline;
    uint32_t seq_inline;
    TaskDev inl[MAX_INLINE_TASKS];
};

// Scheduler counters.  Each group sits in a 128-byte line of its own so that
// waiters polling one of them do not delay updates of the others.
struct Work {
    uint32_t pending;        // outstanding revisits (queued + running)
    uint32_t abort;          // set by the watchdog: the launch gave up (results incomplete)
    uint32_t done;           // set when the last outstanding visit completes
    uint32_t pad0[29];
    uint32_t ring_head;      // next ticket handed to a waiting wave
    uint32_t pad1[31];
    uint32_t ring_tail;      // next ring position a request is written to
    uint32_t pad2[31];
    uint32_t progress;       // completed revisits (watchdog heartbeat)
    uint32_t pad3[31];
    unsigned long long stat_dense;
    unsigned long long stat_revisit;
    unsigned long long stat_rerun;
    unsigned long long stat_overflow;
    unsigned long long stat_request;
    unsigned long long stat_route;   // tasks reconstructed by the component route
    unsigned long long stat_spill;   // queue entries pushed to a global spill queue
    uint32_t route_any;              // = the launch's number: some task takes the component route
    uint32_t has_grey;               // = the launch's number: some task keeps the block route whatever it looks like
    uint32_t classify_done;          // workgroups of the classification that have finished
    uint32_t classify_skip;          // = the launch's number: the samples decided every route (no classification)
    uint32_t pad5[2];
    unsigned long long sample_word;  // (launch number << 32) | tasks sampled so far in that launch
    unsigned long long pad4[5];
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
    int32_t drain_budget;        // queue rounds of a revisit before a sweep round takes over
    int32_t binary_drain_budget; // the same for blocks whose mask is binary (0 / 255)
    int32_t test_fault;          // test hook: 1 = every claim's compare-and-swap is made to fail
    uint32_t *route;             // ROUTE_WORDS per task (below)
    int32_t route_policy;        // 0: the component route where it pays (auto); 1: for every two-valued mask
    uint16_t *spill;             // global spill queues: spill_cap entries per wave of the grid (null: none)
    uint32_t spill_cap;
    uint32_t launch_seq;         // this launch's number (serving: written into host_done)
    uint32_t *host_done;         // host-visible per-task completion words (null: none)
};

// Route words of a task: [0] OR and [1] AND of its nonzero mask values (the
// component route's classification), [2] the ring position of its first block,
// [3] 1 if the task takes the component route (decided by queue_tasks),
// [4] 1 if its sampled foreground is thin (runs of at most ~32 pixels on average).
constexpr int ROUTE_WORDS = 8;

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
// the launch's number: Work flags holding it were set by this launch (no reset needed)
__device__ __forceinline__ uint32_t seq_of(const TaskTable &tt) {
    return tt.hdr ? tt.hdr->launch_seq : tt.seq_inline;
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

// Whether task k takes the component route (component.hpp), as queue_tasks
// decided: its mask holds at most one nonzero value (two_valued: by the OR and
// AND of its nonzero mask values that comp_classify left in its route words),
// and the route pays.  Read only by kernels launched after queue_tasks.
__device__ __forceinline__ bool two_valued(const uint32_t *route, int k) {
    const uint32_t o = route[ROUTE_WORDS * k], n = route[ROUTE_WORDS * k + 1];
    return o == 0u || o == n;
}
__device__ __forceinline__ bool on_component_route(const uint32_t *route, const TaskDev &t, int k) {
    return t.lab && route && route[ROUTE_WORDS * k + 3] == 1u;
}
__device__ __forceinline__ bool on_component_route(const KArgs &a, const TaskDev &t, int k) {
    return on_component_route(a.route, t, k);
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
__device__ __forceinline__ const RK_GLOBAL uint8_t *gp(const uint8_t *p) { return (const RK_GLOBAL uint8_t *)p; }
__device__ __forceinline__ RK_GLOBAL uint8_t *gp(uint8_t *p) { return (RK_GLOBAL uint8_t *)p; }

// global memory access of the 4 pixels at columns x..x+3 of a row with
// `valid` (0..4) of them inside the image; bytes past the image read 0.
__device__ __forceinline__ uint32_t gload4(const uint8_t *row_, int x, int valid, int aligned) {
    const RK_GLOBAL uint8_t *row = gp(row_);
    if (valid <= 0) return 0u;
    if (aligned && valid == 4) return *(const RK_GLOBAL uint32_t *)(row + x);
    uint32_t v = 0;
    for (int k = 0; k < valid && k < 4; ++k) v |= (uint32_t)row[x + k] << (8 * k);
    return v;
}

__device__ __forceinline__ void gstore4(uint8_t *row_, int x, int valid, int aligned, uint32_t v) {
    RK_GLOBAL uint8_t *row = gp(row_);
    if (valid <= 0) return;
    if (aligned && valid == 4) {
        *(RK_GLOBAL uint32_t *)(row + x) = v;
        return;
    }
    for (int k = 0; k < valid && k < 4; ++k) row[x + k] = (uint8_t)(v >> (8 * k));
}

// Marker-plane accesses of the revisit kernel go to the device-coherent level
// (agent-scope atomic loads and stores): a wave on one XCD then reads what a
// wave on another wrote, with no L2 write-back or invalidation.  A writer
// waits for its stores to complete (vm_sync) before the scheduler atomics that
// let another wave read them; a reader issues its loads only after the atomic
// that handed it the block has returned.
__device__ __forceinline__ uint32_t cload32(const uint8_t *p) {
    return __hip_atomic_load((RK_GLOBAL uint32_t *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t cload8(const uint8_t *p) {
    return __hip_atomic_load((RK_GLOBAL uint8_t *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void cstore32(uint8_t *p, uint32_t v) {
    __hip_atomic_store((RK_GLOBAL uint32_t *)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void cstore8(uint8_t *p, uint32_t v) {
    __hip_atomic_store((RK_GLOBAL uint8_t *)p, (uint8_t)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// wait until every memory operation this wave issued has completed
__device__ __forceinline__ void vm_sync() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

__device__ __forceinline__ uint32_t cload4(const uint8_t *row, int x, int valid, int aligned) {
    if (valid <= 0) return 0u;
    if (aligned && valid == 4) return cload32(row + x);
    uint32_t v = 0;
    for (int k = 0; k < valid && k < 4; ++k) v |= cload8(row + x + k) << (8 * k);
    return v;
}

__device__ __forceinline__ void cstore4(uint8_t *row, int x, int valid, int aligned, uint32_t v) {
    if (valid <= 0) return;
    if (aligned && valid == 4) {
        cstore32(row + x, v);
        return;
    }
    for (int k = 0; k < valid && k < 4; ++k) cstore8(row + x + k, v >> (8 * k));
}

// mask value of 4 pixels: I, or 255 - I for a complemented mask (0 outside the image)
__device__ __forceinline__ uint32_t mask4(const TaskDev &t, int gy, int gx, int valid) {
    uint32_t v = gload4(t.i + (int64_t)gy * t.pitch_i, gx, valid, t.aligned);
    if (t.minv) {
        const uint32_t keep = valid >= 4 ? 0xffffffffu : (valid <= 0 ? 0u : ((1u << (8 * valid)) - 1u));
        v = (~v) & keep;
    }
    return v;
}

__device__ __forceinline__ uint32_t mask1(const TaskDev &t, int gy, int gx) {
    const uint32_t v = gp(t.i)[(int64_t)gy * t.pitch_i + gx];
    return t.minv ? 255u - v : v;
}

// current marker value of one pixel, clipped under its mask
__device__ __forceinline__ uint32_t marker1(const TaskDev &t, int gy, int gx) {
    return min((uint32_t)gp(t.j)[(int64_t)gy * t.pitch_j + gx], mask1(t, gy, gx));
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

// Per-wave statistics (meaningful in lane 0), added to the global counters
// once when the wave leaves a kernel.
struct WaveStats {
    unsigned long long dense = 0, revisit = 0, rerun = 0, overflow = 0, request = 0;
};

// ---------------------------------------------------------------------------
// per-visit LDS layout
// J and I share one geometry: (BH + 2) rows of JP bytes, pixel (y, x) at
// (y + 1) * JP + JOFF + x for y in -1..BH and x in -1..BW (the halo ring holds
// the neighbours' marker, clipped, and mask).
// The pointers carry the LDS address space, so that every access (volatile
// ones included) is a DS instruction.
template <int BH>
struct Lds {
    RK_LDS uint8_t *J;
    RK_LDS uint8_t *I;
    RK_LDS uint8_t *rowdirty;   // BH bytes
    RK_LDS uint16_t *Q;         // queue ring (power-of-two entries)
    // The wave's global spill queue (the second level under the LDS ring):
    // pushes that do not fit the ring go there, and the drain takes them back
    // when the ring runs empty.  Its state sits in LDS, read only on those
    // cold paths: sp[0..1] the queue's base address, sp[2] its capacity,
    // sp[3] the entries it holds.
    RK_LDS uint32_t *sp;
    __device__ __forceinline__ RK_LDS uint32_t *Jw(int y, int d) {  // dword d of row y (y in -1..BH)
        return (RK_LDS uint32_t *)(J + (y + 1) * JP + JOFF + 4 * d);
    }
    __device__ __forceinline__ RK_LDS uint32_t *Iw(int y, int d) {
        return (RK_LDS uint32_t *)(I + (y + 1) * JP + JOFF + 4 * d);
    }
    __device__ __forceinline__ RK_LDS uint8_t &Jb(int y, int x) { return J[(y + 1) * JP + JOFF + x]; }
    __device__ __forceinline__ RK_LDS uint8_t &Ib(int y, int x) { return I[(y + 1) * JP + JOFF + x]; }
};

template <int BH>
__host__ __device__ constexpr size_t lds_bytes(int qcap) {
    return 2 * (size_t)(BH + 2) * JP + (size_t)((BH + 15) & ~15) + 32u + 2u * (size_t)qcap;
}

// Lockstep point: the lanes of a wave execute in lockstep on the GPU, so this
// is empty there; the host emulation of these kernels (which runs lanes one
// after another between cross-lane operations) switches lanes here.
#ifndef RK_LANE_SYNC
#define RK_LANE_SYNC() ((void)0)
#endif

// Base of the workgroup's dynamic LDS.  (A host build of these kernels for
// emulated testing supplies its own definition.)
#ifndef RK_DYN_LDS_PROVIDED
__device__ __forceinline__ RK_LDS uint8_t *dyn_lds() {
    extern __shared__ __align__(16) uint8_t rk_smem[];
    return (RK_LDS uint8_t *)rk_smem;
}
#endif

template <int BH>
__device__ __forceinline__ Lds<BH> lds_layout() {
    Lds<BH> L;
    L.J = dyn_lds();
    L.I = L.J + (BH + 2) * JP;
    L.rowdirty = L.I + (BH + 2) * JP;
    L.sp = (RK_LDS uint32_t *)(L.rowdirty + ((BH + 15) & ~15));
    L.Q = (RK_LDS uint16_t *)(L.rowdirty + ((BH + 15) & ~15) + 32);
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
// COH: marker read from the device-coherent level (revisits).
template <int BH, bool COH>
__device__ __forceinline__ void load_block(const TaskDev &t, const BlockGeom &g, Lds<BH> &L, bool fill_initial) {
    const int ln = lane_id();
    const int x = 4 * ln;
    const int valid = min(4, g.bw - x);
    constexpr int CH = BH < 16 ? BH : 16;   // rows whose loads are in flight together
    if (t.aligned && g.bw == BW) {
        // whole-width block of a dword-aligned tile: one dword per lane and row,
        // issued without branches (rows past the image re-read the last row
        // and are zeroed afterwards)
        const RK_GLOBAL uint8_t *ip = gp(t.i) + g.x0 + x;
        const RK_GLOBAL uint8_t *jp = gp(t.j) + g.x0 + x;
        for (int r0 = 0; r0 < BH; r0 += CH) {
            uint32_t iv[CH], jr[CH];
#pragma unroll
            for (int k = 0; k < CH; ++k) {
                const int64_t gy = g.y0 + min(r0 + k, g.bh - 1);
                iv[k] = *(const RK_GLOBAL uint32_t *)(ip + gy * t.pitch_i);
                if (fill_initial)
                    jr[k] = 0u;
                else if (COH)
                    jr[k] = cload32(t.j + g.x0 + x + gy * t.pitch_j);
                else
                    jr[k] = *(const RK_GLOBAL uint32_t *)(jp + gy * t.pitch_j);
            }
#pragma unroll
            for (int k = 0; k < CH; ++k) {
                const int r = r0 + k;
                const bool in = r < g.bh;
                const uint32_t m = in ? (t.minv ? ~iv[k] : iv[k]) : 0u;
                *L.Iw(r, ln) = m;
                *L.Jw(r, ln) = fill_initial ? fill_init4(t, g.y0 + r, g.x0 + x, in ? 4 : 0, m) : bmin4(jr[k], m);
            }
        }
        return;
    }
    for (int r0 = 0; r0 < BH; r0 += CH) {
        uint32_t iv[CH], jr[CH];
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            const int r = r0 + k;
            iv[k] = 0;
            jr[k] = 0;
            if (r < g.bh && valid > 0) {
                const int gy = g.y0 + r;
                iv[k] = mask4(t, gy, g.x0 + x, valid);
                if (!fill_initial)
                    jr[k] = COH ? cload4(t.j + (int64_t)gy * t.pitch_j, g.x0 + x, valid, t.aligned)
                                : gload4(t.j + (int64_t)gy * t.pitch_j, g.x0 + x, valid, t.aligned);
            }
        }
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            const int r = r0 + k;
            *L.Iw(r, ln) = iv[k];
            *L.Jw(r, ln) = fill_initial ? fill_init4(t, g.y0 + r, g.x0 + x, valid, iv[k]) : bmin4(jr[k], iv[k]);
        }
    }
}

// Set the halo ring to 0 (no neighbour information).
template <int BH>
__device__ __forceinline__ void clear_halo(Lds<BH> &L) {
    const int ln = lane_id();
    *L.Jw(-1, ln) = 0u;
    *L.Jw(BH, ln) = 0u;
    *L.Iw(-1, ln) = 0u;
    *L.Iw(BH, ln) = 0u;
    for (int r = ln - 1; r <= BH; r += LANES) {
        L.Jb(r, -1) = 0;
        L.Jb(r, BW) = 0;
        L.Ib(r, -1) = 0;
        L.Ib(r, BW) = 0;
    }
}

// The one-pixel ring of neighbour pixels: mask, and marker clipped under it
// (both 0 outside the image; the marker from the device-coherent level).
// Loads into registers first (halo_issue), LDS stores after (halo_store), so a
// caller can have other loads in flight meanwhile.
struct HaloRegs {
    uint32_t ti, tj, bi, bj;
    uint32_t wi[2], wj[2], ei[2], ej[2];
};

template <int BH>
__device__ __forceinline__ void halo_issue(const TaskDev &t, const BlockGeom &g, HaloRegs &h) {
    const int ln = lane_id();
    const int x = 4 * ln;
    const int valid = min(4, g.bw - x);
    h.ti = h.tj = h.bi = h.bj = 0;
    if (g.has_n && valid > 0) {
        h.ti = mask4(t, g.y0 - 1, g.x0 + x, valid);
        h.tj = cload4(t.j + (int64_t)(g.y0 - 1) * t.pitch_j, g.x0 + x, valid, t.aligned);
    }
    if (g.has_s && valid > 0) {
        h.bi = mask4(t, g.y0 + BH, g.x0 + x, valid);
        h.bj = cload4(t.j + (int64_t)(g.y0 + BH) * t.pitch_j, g.x0 + x, valid, t.aligned);
    }
    // columns -1 and 256 for rows -1..BH (lane k handles row k-1)
    for (int k = 0; k < 2; ++k) {
        h.wi[k] = h.wj[k] = h.ei[k] = h.ej[k] = 0;
        const int r = ln - 1 + k * LANES;
        const bool row_in = (r >= 0 && r < g.bh) || (r == -1 && g.has_n) || (r == BH && g.has_s);
        const int gy = g.y0 + r;
        if (row_in && g.has_w) {
            h.wi[k] = mask1(t, gy, g.x0 - 1);
            h.wj[k] = cload8(t.j + (int64_t)gy * t.pitch_j + g.x0 - 1);
        }
        if (row_in && g.has_e) {
            h.ei[k] = mask1(t, gy, g.x0 + BW);
            h.ej[k] = cload8(t.j + (int64_t)gy * t.pitch_j + g.x0 + BW);
        }
    }
}

template <int BH>
__device__ __forceinline__ void halo_store(const HaloRegs &h, Lds<BH> &L) {
    const int ln = lane_id();
    *L.Iw(-1, ln) = h.ti;
    *L.Jw(-1, ln) = bmin4(h.tj, h.ti);
    *L.Iw(BH, ln) = h.bi;
    *L.Jw(BH, ln) = bmin4(h.bj, h.bi);
    for (int k = 0; k < 2; ++k) {
        const int r = ln - 1 + k * LANES;
        if (r > BH) break;
        L.Ib(r, -1) = (uint8_t)h.wi[k];
        L.Jb(r, -1) = (uint8_t)min(h.wj[k], h.wi[k]);
        L.Ib(r, BW) = (uint8_t)h.ei[k];
        L.Jb(r, BW) = (uint8_t)min(h.ej[k], h.ei[k]);
    }
}

template <int BH>
__device__ __forceinline__ void load_halo(const TaskDev &t, const BlockGeom &g, Lds<BH> &L) {
    HaloRegs h;
    halo_issue<BH>(t, g, h);
    halo_store<BH>(h, L);
}

// true if every byte of v is 0 or 255 (all bits of each byte equal)
__device__ __forceinline__ bool binary4(uint32_t v) { return ((v ^ (v >> 1)) & 0x7f7f7f7fu) == 0u; }

// Whether the block's mask (in LDS) is binary, 0 / 255 only: there a raise
// floods whole regions, which sweeps move faster than the queue.
template <int BH>
__device__ __forceinline__ bool mask_is_binary(Lds<BH> &L) {
    const int ln = lane_id();
    bool bin = true;
    for (int r = 0; r < BH; ++r) bin = bin && binary4(*L.Iw(r, ln));
    return __ballot(!bin) == 0;
}

// A visit's load: the block (mask, and marker from the device-coherent
// level) and its halo, with all loads of a whole-width aligned block of up to
// 32 rows in flight together.
template <int BH>
__device__ __forceinline__ void load_visit(const TaskDev &t, const BlockGeom &g, Lds<BH> &L) {
    if (!(t.aligned && g.bw == BW && BH <= 32)) {
        load_block<BH, true>(t, g, L, false);
        load_halo<BH>(t, g, L);
        return;
    }
    const int ln = lane_id();
    const int x = 4 * ln;
    HaloRegs h;
    halo_issue<BH>(t, g, h);
    uint32_t iv[BH], jr[BH];
#pragma unroll
    for (int k = 0; k < BH; ++k) {
        const int64_t gy = g.y0 + min(k, g.bh - 1);
        iv[k] = *(const RK_GLOBAL uint32_t *)(gp(t.i) + g.x0 + x + gy * t.pitch_i);
        jr[k] = cload32(t.j + g.x0 + x + gy * t.pitch_j);
    }
#pragma unroll
    for (int k = 0; k < BH; ++k) {
        const bool in = k < g.bh;
        const uint32_t m = in ? (t.minv ? ~iv[k] : iv[k]) : 0u;
        *L.Iw(k, ln) = m;
        *L.Jw(k, ln) = bmin4(jr[k], m);
    }
    halo_store<BH>(h, L);
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

// the same with the row's two halo bytes (hl = pixel -1, hr = pixel BW) given
__device__ __forceinline__ void side_from(uint32_t v, uint32_t hl, uint32_t hr, uint32_t &left, uint32_t &right) {
    const int ln = lane_id();
    const uint32_t up = from_lower(v);
    const uint32_t dn = from_upper(v);
    left = ln == 0 ? hl : (up >> 24);
    right = ln == LANES - 1 ? hr : (dn & 0xffu);
}

// ---------------------------------------------------------------------------
// Directional sweeps with row closure.
//
// In a raster pass a pixel takes v = clamp(u, lo, hi): u is the value reaching
// it from its predecessor along the row, lo = min(J', I) with J' the pixel and
// its neighbours in the row already swept, hi = I.  A map v -> clamp(v, lo, hi)
// (lo <= hi) composed with another such map is again one (the clamp of the
// inner bounds into the outer interval), so a whole row is a prefix scan of
// maps: across the 4 pixels of a lane, then across the lanes of a 16-lane DPP
// row, then across the 4 DPP rows through readlane.  Running it from both ends
// and taking the larger value closes the row: everything that reaches a pixel
// along the row from either side arrives in the same step.

constexpr int DPP_ROW_SHL = 0x100;   // + n: lane i reads lane i + n of its 16-lane row
constexpr int DPP_ROW_SHR = 0x110;   // + n: lane i reads lane i - n of its 16-lane row

__device__ __forceinline__ uint32_t clampu(uint32_t v, uint32_t lo, uint32_t hi) { return min(max(v, lo), hi); }

// lane i gets `v` of the lane selected by CTRL, or keeps `old` where there is none
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_or(uint32_t old, uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, 0xf, 0xf, false);
}

// one step of an inclusive scan of maps (a, b) within 16-lane rows: compose
// this lane's map after the one of the lane CTRL selects (identity (0, 255)
// where there is none)
template <int CTRL>
__device__ __forceinline__ void map_scan_step(uint32_t &a, uint32_t &b) {
    const uint32_t ta = dpp_or<CTRL>(0u, a), tb = dpp_or<CTRL>(255u, b);
    const uint32_t na = clampu(ta, a, b), nb = clampu(tb, a, b);
    a = na;
    b = nb;
}

// e_row for the lane's DPP row (row = lane / 16), without branches
__device__ __forceinline__ uint32_t sel_row(int row, uint32_t e0, uint32_t e1, uint32_t e2, uint32_t e3) {
    const uint32_t m1 = 0u - (uint32_t)(row & 1), m2 = 0u - (uint32_t)(row >> 1);
    const uint32_t lo = e0 ^ ((e0 ^ e1) & m1), hi = e2 ^ ((e2 ^ e3) & m1);
    return lo ^ ((lo ^ hi) & m2);
}

// Row closure of the 256 pixels held 4 per lane (byte j of lane l = pixel 4l+j):
// per pixel maps (byte j of lo4, hi4, lo <= hi), `vl` entering pixel 0 from the
// left and `vr` entering pixel 255 from the right (both wave-uniform).  Returns
// the pixels' values: max of the left-to-right and right-to-left scans.
__device__ __forceinline__ uint32_t row_closure(uint32_t lo4, uint32_t hi4, uint32_t vl, uint32_t vr) {
    const int ln = lane_id();
    const int row = ln >> 4;
    uint32_t lo[4], hi[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        lo[j] = byte_of(lo4, j);
        hi[j] = byte_of(hi4, j);
    }
    vl = uniform(vl);
    vr = uniform(vr);
    uint32_t out[4];
    {   // left to right
        uint32_t a = lo[0], b = hi[0];
#pragma unroll
        for (int j = 1; j < 4; ++j) {
            a = clampu(a, lo[j], hi[j]);
            b = clampu(b, lo[j], hi[j]);
        }
        map_scan_step<DPP_ROW_SHR + 1>(a, b);
        map_scan_step<DPP_ROW_SHR + 2>(a, b);
        map_scan_step<DPP_ROW_SHR + 4>(a, b);
        map_scan_step<DPP_ROW_SHR + 8>(a, b);
        // value entering each DPP row: through the totals of the rows before it
        const uint32_t e0 = vl;
        const uint32_t e1 = clampu(e0, (uint32_t)__builtin_amdgcn_readlane((int)a, 15),
                                   (uint32_t)__builtin_amdgcn_readlane((int)b, 15));
        const uint32_t e2 = clampu(e1, (uint32_t)__builtin_amdgcn_readlane((int)a, 31),
                                   (uint32_t)__builtin_amdgcn_readlane((int)b, 31));
        const uint32_t e3 = clampu(e2, (uint32_t)__builtin_amdgcn_readlane((int)a, 47),
                                   (uint32_t)__builtin_amdgcn_readlane((int)b, 47));
        // through the lanes before this one in its row
        const uint32_t xa = dpp_or<DPP_ROW_SHR + 1>(0u, a), xb = dpp_or<DPP_ROW_SHR + 1>(255u, b);
        uint32_t v = clampu(sel_row(row, e0, e1, e2, e3), xa, xb);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            v = clampu(v, lo[j], hi[j]);
            out[j] = v;
        }
    }
    {   // right to left
        uint32_t a = lo[3], b = hi[3];
#pragma unroll
        for (int j = 2; j >= 0; --j) {
            a = clampu(a, lo[j], hi[j]);
            b = clampu(b, lo[j], hi[j]);
        }
        map_scan_step<DPP_ROW_SHL + 1>(a, b);
        map_scan_step<DPP_ROW_SHL + 2>(a, b);
        map_scan_step<DPP_ROW_SHL + 4>(a, b);
        map_scan_step<DPP_ROW_SHL + 8>(a, b);
        const uint32_t e3 = vr;
        const uint32_t e2 = clampu(e3, (uint32_t)__builtin_amdgcn_readlane((int)a, 48),
                                   (uint32_t)__builtin_amdgcn_readlane((int)b, 48));
        const uint32_t e1 = clampu(e2, (uint32_t)__builtin_amdgcn_readlane((int)a, 32),
                                   (uint32_t)__builtin_amdgcn_readlane((int)b, 32));
        const uint32_t e0 = clampu(e1, (uint32_t)__builtin_amdgcn_readlane((int)a, 16),
                                   (uint32_t)__builtin_amdgcn_readlane((int)b, 16));
        const uint32_t xa = dpp_or<DPP_ROW_SHL + 1>(0u, a), xb = dpp_or<DPP_ROW_SHL + 1>(255u, b);
        uint32_t v = clampu(sel_row(row, e0, e1, e2, e3), xa, xb);
#pragma unroll
        for (int j = 3; j >= 0; --j) {
            v = clampu(v, lo[j], hi[j]);
            out[j] = max(out[j], v);
        }
    }
    return out[0] | (out[1] << 8) | (out[2] << 16) | (out[3] << 24);
}

// Sweep down (dir > 0) or up over the block's rows: each row takes the swept
// row before it (and, for 8-connectivity, its diagonal neighbours there) and is
// then closed along its length, with the halo pixels at both ends as inputs.
// This is a raster (or anti-raster) pass in which every row run is complete.
// Returns true if anything changed.
//
// The row's own loads do not depend on the row before it (only row r is
// written while row r is closed), so each row's marker, mask and halo bytes are
// read one row ahead and their latency overlaps the closure of the row before.
// After the last block row the read-ahead lands on the halo row, which exists.
template <int BH, int CONN, int DIR>
__device__ __forceinline__ bool sweep(Lds<BH> &L) {
    constexpr int dir = DIR;
    constexpr int conn = CONN;
    const int ln = lane_id();
    const int r0 = dir > 0 ? 0 : BH - 1;
    const int rprev = dir > 0 ? -1 : BH;
    uint32_t prev = *L.Jw(rprev, ln);
    uint32_t pl, pr;
    side_bytes(L, rprev, prev, pl, pr);
    uint32_t ncur = *L.Jw(r0, ln), nhi = *L.Iw(r0, ln);
    uint32_t nvl = L.Jb(r0, -1), nvr = L.Jb(r0, BW);
    bool changed = false;
    for (int k = 0; k < BH; ++k) {
        const int r = r0 + dir * k;
        const uint32_t cur = ncur, hi = nhi, vl = nvl, vr = nvr;
        const int rn = r + dir;   // -1 .. BH
        ncur = *L.Jw(rn, ln);
        nhi = *L.Iw(rn, ln);
        nvl = L.Jb(rn, -1);
        nvr = L.Jb(rn, BW);
        __builtin_amdgcn_sched_barrier(0);   // keep the read-ahead issued here, before the closure
        uint32_t m = bmax4(cur, prev);
        if (conn == 8) {
            m = bmax4(m, (prev << 8) | pl);
            m = bmax4(m, (prev >> 8) | (pr << 24));
        }
        const uint32_t nv = row_closure(bmin4(m, hi), hi, vl, vr);
        if (nv != cur) {
            *L.Jw(r, ln) = nv;
            L.rowdirty[r] = 1;
            changed = true;
        }
        prev = nv;
        side_from(prev, vl, vr, pl, pr);
    }
    return changed;
}

// A round of sweeps: down, then up, each with its direction a compile-time
// constant (every LDS offset of the unrolled rows an immediate).  A block
// visit has one call site of it (converge_block), which serves both a first
// visit's sweep rounds and a revisit's fallback.  Returns true if anything
// changed.
template <int BH, int CONN>
__device__ __forceinline__ bool sweep_round(Lds<BH> &L) {
    bool c = sweep<BH, CONN, +1>(L);
    __syncthreads();
    c |= sweep<BH, CONN, -1>(L);
    __syncthreads();
    return c;
}

// The spill queue's base address (state in LDS, see Lds::sp)
__device__ __forceinline__ uint16_t *spill_base(const volatile RK_LDS uint32_t *sp) {
    return (uint16_t *)(((uint64_t)sp[1] << 32) | (uint64_t)sp[0]);
}

// Push the pixels flagged by `pred` (one per lane) onto the LDS ring of qcap
// (a power of two) entries.  Returns false (and pushes nothing) if they do not
// fit: the caller then keeps them aside and hands them to spill() once its
// unit of work (a drain round, a seeded row) is done, so that the cold spill
// path exists once per unit instead of at every push site.
template <int BH>
__device__ __forceinline__ bool push(Lds<BH> &L, int qcap, uint32_t head, uint32_t &tail, bool pred, uint32_t pix) {
    const unsigned long long m = __ballot(pred);
    if (m == 0) return true;
    const uint32_t cnt = (uint32_t)__popcll(m);
    if (tail - head + cnt > (uint32_t)qcap) return false;
    if (pred) ((volatile RK_LDS uint16_t *)L.Q)[(tail + prefix_count(m)) & (uint32_t)(qcap - 1)] = (uint16_t)pix;
    tail += cnt;
    return true;
}

// Push the pixels flagged by `pred` to the wave's global spill queue; false
// (nothing pushed) if it has no room.  The spill is written and read back by
// its own wave only, at the device-coherent level (so that no cache level can
// hold an older copy of an entry the wave rewrote), and read only after a wait
// for the writes (drain).
template <int BH>
__device__ __forceinline__ bool spill(Lds<BH> &L, bool pred, uint32_t pix) {
    const unsigned long long m = __ballot(pred);
    if (m == 0) return true;
    const uint32_t cnt = (uint32_t)__popcll(m);
    volatile RK_LDS uint32_t *sp = L.sp;
    const uint32_t n = uniform(sp[3]);
    if (n + cnt > uniform(sp[2])) return false;
    if (pred)
        __hip_atomic_store((RK_GLOBAL uint16_t *)(spill_base(sp) + n + prefix_count(m)), (uint16_t)pix,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    RK_LANE_SYNC();   // every lane has read the count before it moves
    if (lane_id() == 0) sp[3] = n + cnt;
    return true;
}

// Marker byte of LDS pixel (y, x) for the queue phase.  A wave's LDS operations
// execute in issue order; volatile keeps the compiler from reordering these
// accesses among themselves, so a load issued after another lane's store of
// the same byte (in an earlier statement) sees that store, with no wait.
template <int BH>
__device__ __forceinline__ volatile RK_LDS uint8_t &jv(Lds<BH> &L, int y, int x) {
    return *(volatile RK_LDS uint8_t *)&L.Jb(y, x);
}

// Seed pass: raise every pixel that a neighbour (block or halo) can raise and push it.
// Rows r-1, r and r+1 are carried from one row to the next (row r+1 is not
// written while row r is seeded, row r is carried as written), so each row
// reads one new marker row, read a row ahead, and its mask row.
template <int BH, int CONN>
__device__ __forceinline__ void seed_pass(Lds<BH> &L, int qcap, uint32_t head, uint32_t &tail,
                          bool &overflow, bool &changed) {
    constexpr int conn = CONN;
    const int ln = lane_id();
    uint32_t a = *L.Jw(-1, ln), c = *L.Jw(0, ln), b = *L.Jw(1, ln);
    uint32_t ahl = L.Jb(-1, -1), ahr = L.Jb(-1, BW), chl = L.Jb(0, -1), chr = L.Jb(0, BW);
    uint32_t bhl = L.Jb(1, -1), bhr = L.Jb(1, BW);
    for (int r = 0; r < BH; ++r) {
        const int rn = min(r + 2, BH);   // the row after b (the halo row at most)
        const uint32_t nb = *L.Jw(rn, ln), nbhl = L.Jb(rn, -1), nbhr = L.Jb(rn, BW);
        const uint32_t hi = *L.Iw(r, ln);
        __builtin_amdgcn_sched_barrier(0);   // keep the read-ahead issued here
        uint32_t al, ar, cl, cr, bl, br;
        side_from(a, ahl, ahr, al, ar);
        side_from(c, chl, chr, cl, cr);
        side_from(b, bhl, bhr, bl, br);
        uint32_t m = bmax4(c, bmax4(a, b));
        m = bmax4(m, bmax4((c << 8) | cl, (c >> 8) | (cr << 24)));
        if (conn == 8) {
            m = bmax4(m, bmax4((a << 8) | al, (a >> 8) | (ar << 24)));
            m = bmax4(m, bmax4((b << 8) | bl, (b >> 8) | (br << 24)));
        }
        const uint32_t nv = bmin4(m, hi);
        const uint32_t dm = diff_bytes(nv, c);
        if (dm) {
            *L.Jw(r, ln) = nv;
            L.rowdirty[r] = 1;
        }
        if (__ballot(dm != 0)) {
            changed = true;
            uint32_t lost = 0;      // bit j: this lane's pixel j did not fit the ring
            bool any_lost = false;  // (a push fails for the whole wave: a uniform branch)
            for (int j = 0; j < 4; ++j) {
                const bool p = (dm >> j) & 1u;
                if (!push(L, qcap, head, tail, p, (uint32_t)(r * BW + 4 * ln + j))) {
                    any_lost = true;
                    lost |= (p ? 1u : 0u) << j;
                }
            }
            if (any_lost)
                for (int j = 0; j < 4; ++j)
                    if (!spill(L, (lost >> j) & 1u, (uint32_t)(r * BW + 4 * ln + j))) overflow = true;
        }
        a = nv;
        ahl = chl;
        ahr = chr;
        c = b;
        chl = bhl;
        chr = bhr;
        b = nb;
        bhl = nbhl;
        bhr = nbhr;
    }
}

// Raise J(y, x) to `target` if lower; returns true if this lane raised it.
// A byte store: within one call site the lanes of the wave write distinct
// pixels (or the same pixel with the same value), and successive call sites
// are ordered through jv(), so no raise is ever lost.
template <int BH>
__device__ __forceinline__ bool raise_px(Lds<BH> &L, int y, int x, uint32_t target) {
    volatile RK_LDS uint8_t &b = jv(L, y, x);
    if ((uint32_t)b >= target) return false;
    b = (uint8_t)target;
    return true;
}

// Border seed: after the halo has been refreshed, only pixels on the block's
// border can be raised by a neighbour (the interior was left converged by the
// previous visit, and only the owner writes it).  Raise and push exactly those.
template <int BH, int CONN>
__device__ __forceinline__ void seed_border(Lds<BH> &L, int bh, int bw, int qcap, uint32_t head, uint32_t &tail,
                            bool &overflow, bool &changed) {
    constexpr int conn = CONN;
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
        if (__ballot(dm != 0)) {
            changed = true;
            uint32_t lost = 0;
            bool any_lost = false;
            for (int j = 0; j < 4; ++j) {
                const bool p = (dm >> j) & 1u;
                if (!push(L, qcap, head, tail, p, (uint32_t)(r * BW + 4 * ln + j))) {
                    any_lost = true;
                    lost |= (p ? 1u : 0u) << j;
                }
            }
            if (any_lost)
                for (int j = 0; j < 4; ++j)
                    if (!spill(L, (lost >> j) & 1u, (uint32_t)(r * BW + 4 * ln + j))) overflow = true;
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
        if (!push(L, qcap, head, tail, raised, (uint32_t)(r * BW + x)) && !spill(L, raised, (uint32_t)(r * BW + x)))
            overflow = true;
        __syncthreads();
    }
}

// neighbour k of a pixel (N, S, W, E, then NW, NE, SW, SE): row and column step
__host__ __device__ constexpr int nb_dy(int k) { return k == 0 || k == 4 || k == 5 ? -1 : (k == 1 || k >= 6 ? 1 : 0); }
__host__ __device__ constexpr int nb_dx(int k) { return k == 2 || k == 4 || k == 6 ? -1 : (k == 3 || k == 5 || k == 7 ? 1 : 0); }

// Drain the LDS ring, and the wave's spill queue behind it, to empty;
// *overflow set if pushes had to be dropped (the ring full, the spill queue
// too, or a ring too small for a round).
// Each round pops up to 64 pixels (one per lane) and offers every popped
// pixel's value to its neighbours, one direction at a time.
// At most `budget` rounds (no limit if negative); returns false if the ring was
// not empty when the budget ran out.
template <int BH, int CONN>
__device__ __forceinline__ bool drain(Lds<BH> &L, int qcap, uint32_t &head, uint32_t &tail, bool &overflow, int budget) {
    const int ln = lane_id();
    volatile RK_LDS uint16_t *Qv = L.Q;
    volatile RK_LDS uint8_t *Jv = L.J;
    // room a round may need: up to 64 popped pixels x CONN pushes (at most
    // half the ring, for small rings)
    const uint32_t room = min((uint32_t)(LANES * CONN), (uint32_t)qcap / 2u);
    while (true) {
        if (tail - head + room > (uint32_t)qcap) {
            // nearly full: the newest entries go to the spill queue first, so
            // that no push of the round fails (cold; the round itself stays as
            // it is without a spill)
            volatile RK_LDS uint32_t *sp = L.sp;
            const uint32_t held = uniform(sp[3]), cap = uniform(sp[2]);
            const uint32_t m = min(tail - head + room - (uint32_t)qcap, cap - held);
            for (uint32_t i = (uint32_t)ln; i < m; i += LANES)
                __hip_atomic_store((RK_GLOBAL uint16_t *)(spill_base(sp) + held + i),
                                   (uint16_t)Qv[(tail - m + i) & (uint32_t)(qcap - 1)], __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            tail -= m;
            RK_LANE_SYNC();   // every lane has read the count before it moves
            if (ln == 0) sp[3] = held + m;
        }
        if (head == tail) {
            volatile RK_LDS uint32_t *sp = L.sp;
            const uint32_t held = uniform(sp[3]);
            if (held == 0) break;
            // the ring ran empty: take the spill's last entries back into it
            const uint32_t n = min(held, (uint32_t)qcap);
            const uint32_t base = held - n;
            vm_sync();   // the spill's stores have completed
            for (uint32_t i = (uint32_t)ln; i < n; i += LANES)
                Qv[(tail + i) & (uint32_t)(qcap - 1)] =
                    __hip_atomic_load((RK_GLOBAL uint16_t *)(spill_base(sp) + base + i), __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
            tail += n;
            RK_LANE_SYNC();   // every lane has read the count before it moves
            if (ln == 0) {
                sp[3] = base;
                sp[4] += n;   // entries taken back (statistics)
            }
        }
        if (budget-- == 0) return false;
        RK_LANE_SYNC();
        const uint32_t n = min(tail - head, (uint32_t)LANES);
        const bool valid = (uint32_t)ln < n;
        const uint32_t p = valid ? (uint32_t)Qv[(head + ln) & (uint32_t)(qcap - 1)] : 0u;
        head += n;
        const int y = (int)(p >> 8), x = (int)(p & 255u);
        const int a = (y + 1) * JP + JOFF + x;   // offset of pixel (y, x) in the J and I planes
        const uint32_t v = Jv[a];
        const bool ok_n = valid && y > 0, ok_s = valid && y < BH - 1;
        const bool ok_w = valid && x > 0, ok_e = valid && x < BW - 1;
        // the mask never changes: all neighbours' mask values up front (a
        // block pixel's neighbours lie in the LDS planes, the halo ring at worst)
        uint32_t iv[CONN];
#pragma unroll
        for (int k = 0; k < CONN; ++k) iv[k] = L.I[a + nb_dy(k) * JP + nb_dx(k)];
        // Direction k's neighbour is read right after direction k-1's store (so
        // it sees that raise), and direction k-1's push, which touches only the
        // ring, is issued while that read is in flight.
        bool prev_raised = false;
#pragma unroll
        for (int k = 0; k < CONN; ++k) {
            const int off = nb_dy(k) * JP + nb_dx(k);
            const bool in = (nb_dy(k) < 0 ? ok_n : nb_dy(k) > 0 ? ok_s : valid) &&
                            (nb_dx(k) < 0 ? ok_w : nb_dx(k) > 0 ? ok_e : true);
            const uint32_t tgt = min(v, iv[k]);
            RK_LANE_SYNC();   // every lane's store of direction k-1 is issued before this read
            const uint32_t cur = Jv[a + off];
            if (k > 0 && !push(L, qcap, head, tail, prev_raised, p + (uint32_t)(nb_dy(k - 1) * BW + nb_dx(k - 1))))
                overflow = true;
            const bool raised = in && cur < tgt;
            if (raised) {
                Jv[a + off] = (uint8_t)tgt;
                L.rowdirty[y + nb_dy(k)] = 1;
            }
            prev_raised = raised;
        }
        if (!push(L, qcap, head, tail, prev_raised, p + (uint32_t)(nb_dy(CONN - 1) * BW + nb_dx(CONN - 1))))
            overflow = true;
    }
    return true;
}

// Seed and drain until no queue overflow is left; returns true if anything changed.
// border_only: the first seed looks at the block's border only (valid when the
// interior is already converged and only the halo changed); re-seeds after a
// queue overflow are always dense.
// On a revisit, a drain that is still running after `budget` rounds is
// following long paths (a flood or a corridor entering the block) one pixel
// per round; it is cut short and a round of sweeps (which move whole row and
// column runs at once) takes over, followed by a dense seed, at most
// SWEEP_FALLBACKS times.  A first visit starts with up to `pre_sweeps` sweep
// rounds (while they change something) and then drains to the end.
constexpr int SWEEP_FALLBACKS = 4;
// A border seed that queues at least this many pixels (a wave's worth) is a
// wide front entering the block: it goes straight to a sweep round, which
// carries a front across the block in one pass, instead of draining it one
// pixel step per round first.  That shortens the chains of visits a launch
// waits on, at the price of the extra sweep work, so it is applied only when
// the launch is latency-bound: at most WIDE_FRONT_LOAD blocks per wave of the
// grid (a single tile); a launch with many more blocks than waves (a large
// batch) is throughput-bound and drains first.
constexpr uint32_t WIDE_FRONT = 64;
constexpr uint32_t WIDE_FRONT_LOAD = 4;

template <int BH, int CONN>
__device__ __forceinline__ bool converge_block(Lds<BH> &L, int qcap, WaveStats &st, bool border_only, int bh, int bw,
                                               int budget, bool wide_first, int pre_sweeps) {
    bool changed = false;
    int fallbacks = border_only ? SWEEP_FALLBACKS : 0;
    bool sweep_next = pre_sweeps > 0;
    for (int round = 0; round <= (1 << 16);) {   // each round raises pixels; bounded anyway
        if (sweep_next) {
            // the first visit's sweep rounds (again while they change
            // something, at most pre_sweeps), or one fallback round
            const bool c = __ballot(sweep_round<BH, CONN>(L)) != 0;
            sweep_next = pre_sweeps > 1 && c;
            pre_sweeps = pre_sweeps > 0 ? pre_sweeps - 1 : 0;
            if (sweep_next) continue;
            pre_sweeps = 0;
        }
        uint32_t head = 0, tail = 0;
        bool overflow = false;
        if (lane_id() == 0) ((volatile RK_LDS uint32_t *)L.sp)[3] = 0u;   // a round starts with empty queues
        __syncthreads();                                                  // (a seed finds every raisable pixel again)
        if (border_only && round == 0)
            seed_border<BH, CONN>(L, bh, bw, qcap, head, tail, overflow, changed);
        else
            seed_pass<BH, CONN>(L, qcap, head, tail, overflow, changed);
        __syncthreads();
        const bool wide = wide_first && border_only && round == 0 && fallbacks > 0 && tail - head >= WIDE_FRONT;
        const bool drained = !wide && drain<BH, CONN>(L, qcap, head, tail, overflow, fallbacks > 0 ? budget : -1);
        __syncthreads();
        ++round;
        if (!drained) {
            --fallbacks;
            sweep_next = true;
            continue;
        }
        if (!__ballot(overflow)) break;
        st.overflow += 1;
    }
    for (int r = 0; r < BH; ++r)
        if (L.rowdirty[r]) changed = true;
    return __ballot(changed) != 0;
}

// Write back the rows flagged dirty (all rows if `all`).
// COH: to the device-coherent level (revisits).
template <int BH, bool COH>
__device__ __forceinline__ void store_block(const TaskDev &t, const BlockGeom &g, Lds<BH> &L, bool all) {
    const int ln = lane_id();
    const int x = 4 * ln;
    const int valid = min(4, g.bw - x);
    for (int r = 0; r < g.bh; ++r) {
        if (!all && !L.rowdirty[r]) continue;
        if (COH)
            cstore4(t.j + (int64_t)(g.y0 + r) * t.pitch_j, g.x0 + x, valid, t.aligned, *L.Jw(r, ln));
        else
            gstore4(t.j + (int64_t)(g.y0 + r) * t.pitch_j, g.x0 + x, valid, t.aligned, *L.Jw(r, ln));
    }
}

// ---------------------------------------------------------------------------
// scheduling (revisits)

__device__ __forceinline__ uint32_t *state_word(const KArgs &a, uint32_t block) {
    return a.state + (size_t)block * STATE_STRIDE;
}

__device__ __forceinline__ bool expired(const KArgs &a, uint64_t start) {
    return wall_clock64() - start > a.watchdog_ticks;
}

// Idle back-off of a waiter polling its own ring slot: about 2^min(k, 3) x 512
// cycles (under 2 us), so a block handed to it is picked up quickly.
__device__ __forceinline__ void backoff(int k) {
    const int n = 1 << (k < 3 ? k : 3);
    for (int i = 0; i < n; ++i) __builtin_amdgcn_s_sleep(8);
}

constexpr uint32_t SLOT_EXIT = 0xffffffffu;   // ring slot value: no more work will come
// Compare-and-swap attempts on a block state word before a launch gives up.
// Only the owner, requesters (setting D) and the claim touch a word, so a
// retry fails only while another wave's update lands in between; this many
// failures in a row means something is wrong, and the launch is abandoned
// (abort flag, RECON_EDEVICE on the host) rather than run unowned.
constexpr int CAS_TRIES = 1024;

__device__ __forceinline__ void flush_stats(Work *w, const WaveStats &st) {
    if (lane_id() != 0) return;
    if (st.dense) __hip_atomic_fetch_add(&w->stat_dense, st.dense, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (st.revisit) __hip_atomic_fetch_add(&w->stat_revisit, st.revisit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (st.rerun) __hip_atomic_fetch_add(&w->stat_rerun, st.rerun, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (st.overflow)
        __hip_atomic_fetch_add(&w->stat_overflow, st.overflow, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (st.request)
        __hip_atomic_fetch_add(&w->stat_request, st.request, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);

}

// Request visits of the neighbouring blocks flagged in `want` (bit k:
// neighbour k of N, S, W, E, NW, NE, SW, SE) of block `gb` of task `ti`.
// Called by all lanes with wave-uniform arguments; lane k handles neighbour k,
// so the requests go out together.  When `keep` points to -1, the first
// flagged neighbour is claimed for the calling wave's next visit if it is idle
// (compare-and-swap idle -> owned): no ring round trip, and the calling visit's
// count of outstanding work passes to it unchanged.  Every other neighbour gets
// its requested bit; one that was idle is counted and written to the ring.  The
// caller's marker stores have completed before (vm_sync), so all atomics here
// are relaxed.  Returns false if the watchdog expired while waiting for a ring
// slot.
__device__ __forceinline__ bool request_neighbours(const KArgs &a, uint32_t ring_cap, int ti, uint32_t gb, int nbx, uint32_t want,
                                   int *keep, WaveStats &st) {
    const int ln = lane_id();
    const int k = ln & 7;
    const int off = k == 0 ? -nbx : k == 1 ? nbx : k == 2 ? -1 : k == 3 ? 1 : k == 4 ? -nbx - 1
                  : k == 5 ? -nbx + 1 : k == 6 ? nbx - 1 : nbx + 1;
    const uint32_t nb = (uint32_t)((int)gb + off);
    const bool mine = ln < 8 && ((want >> ln) & 1u);
    const int cand = (keep != nullptr && *keep < 0 && want != 0u) ? (int)__builtin_ctz(want) : -1;
    bool kept = false, queue = false;
    if (mine) {
        uint32_t old;
        if (ln == cand) {
            uint32_t expected = ST_V;   // idle: visited, not owned, not requested
            kept = __hip_atomic_compare_exchange_strong(state_word(a, nb), &expected, ST_V | ST_R, __ATOMIC_RELAXED,
                                                        __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            old = kept ? 0u : __hip_atomic_fetch_or(state_word(a, nb), ST_D, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            old = __hip_atomic_fetch_or(state_word(a, nb), ST_D, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        queue = !kept && !(old & (ST_R | ST_D));   // this request made an idle block pending
    }
    if (__ballot(kept)) {
        *keep = (int)((int)gb + (cand == 0 ? -nbx : cand == 1 ? nbx : cand == 2 ? -1 : cand == 3 ? 1
                      : cand == 4 ? -nbx - 1 : cand == 5 ? -nbx + 1 : cand == 6 ? nbx - 1 : nbx + 1));
        if (ln == 0) st.request += 1;
    }
    const unsigned long long qm = __ballot(queue);
    if (qm == 0) return true;
    const uint32_t nq = (uint32_t)__popcll(qm);
    uint32_t base = 0;
    if (ln == 0) {
        __hip_atomic_fetch_add(a.tile_pending + ti, nq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&a.work->pending, nq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        base = __hip_atomic_fetch_add(&a.work->ring_tail, nq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        st.request += nq;
    }
    base = uniform(base);
    uint32_t *slot = a.ring + (size_t)((base + prefix_count(qm)) % ring_cap) * RING_STRIDE;
    // a slot is free unless its previous occupant has not been taken out yet
    const uint64_t t0 = wall_clock64();
    while (true) {
        const bool busy = queue && __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
        if (!__ballot(busy)) break;
        if (expired(a, t0)) return false;
        __builtin_amdgcn_s_sleep(1);
    }
    if (queue) __hip_atomic_store(slot, nb + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return true;
}

// Border checks from LDS: request every neighbouring block that a pixel of
// this block's border (rows 0 / bh-1, columns 0 / bw-1) can still raise,
// judged against the halo ring (neighbour marker clipped under its mask, as
// loaded).  A halo value may be older than the neighbour's current one, but
// never higher, so a needed request is never missed; a stale one only costs a
// visit that finds nothing to do.
template <int BH>
__device__ __forceinline__ bool check_neighbours(const KArgs &a, uint32_t ring_cap, int ti, const TaskDev &t,
                                 const BlockGeom &g, int by, int bx, Lds<BH> &L, int *keep,
                                 WaveStats &st) {
    const int ln = lane_id();
    const int conn = t.conn;
    const uint32_t gb = t.block0 + (uint32_t)(by * t.nbx + bx);
    uint32_t want = 0;   // bit k: request neighbour k (N, S, W, E, NW, NE, SW, SE)
    {   // N and S edges: lane handles columns 4ln..4ln+3
        for (int side = 0; side < 2; ++side) {
            const bool exists = side == 0 ? g.has_n : g.has_s;
            if (!exists) continue;
            const int r = side == 0 ? 0 : g.bh - 1;
            const int hr = side == 0 ? -1 : BH;
            const uint32_t c = *L.Jw(r, ln);
            uint32_t out = c;
            if (conn == 8) {
                const uint32_t up = from_lower(c), dn = from_upper(c);
                const uint32_t l = ln == 0 ? 0u : (up >> 24);          // our pixel x-1 (none at x=0)
                const uint32_t rr = ln == LANES - 1 ? 0u : (dn & 0xffu);
                out = bmax4(out, bmax4((c << 8) | l, (c >> 8) | (rr << 24)));
            }
            const uint32_t nj = *L.Jw(hr, ln);
            const bool viol = bmax4(nj, bmin4(out, *L.Iw(hr, ln))) != nj;
            if (__ballot(viol)) want |= 1u << side;
        }
    }
    {   // W and E edges: lane r handles row r
        const int r = ln;
        for (int side = 0; side < 2; ++side) {
            const bool exists = side == 0 ? g.has_w : g.has_e;
            if (!exists) continue;
            const int cx = side == 0 ? 0 : g.bw - 1;
            const int hx = side == 0 ? -1 : BW;
            bool viol = false;
            if (r < g.bh) {
                uint32_t out = L.Jb(r, cx);
                if (conn == 8) {
                    if (r > 0) out = max(out, (uint32_t)L.Jb(r - 1, cx));
                    if (r + 1 < g.bh) out = max(out, (uint32_t)L.Jb(r + 1, cx));
                }
                viol = (uint32_t)L.Jb(r, hx) < min(out, (uint32_t)L.Ib(r, hx));
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
                const int hr = north ? -1 : BH;
                const int hx = west ? -1 : BW;
                viol = (uint32_t)L.Jb(hr, hx) < min((uint32_t)L.Jb(r, cx), (uint32_t)L.Ib(hr, hx));
            }
        }
        want |= (uint32_t)(__ballot(viol) & 0xfull) << 4;
    }
    want = uniform(want);
    if (want == 0u) return true;
    return request_neighbours(a, ring_cap, ti, gb, t.nbx, want, keep, st);
}

// ---------------------------------------------------------------------------
// K1: dense pass.  Every block once, independently (empty halo).

// A block loaded with an empty halo: sweep rounds, then seed and drain.
template <int BH, int CONN>
__device__ __forceinline__ void dense_block(const TaskDev &t, const BlockGeom &g, Lds<BH> &L, WaveStats &st) {
    converge_block<BH, CONN>(L, t.qcap, st, false, g.bh, g.bw, -1, false, t.scan_rounds);
}

// One visit's work on the loaded block: dense (a first visit: sweep rounds,
// then a dense seed and a drain to the end) or from the border (a later
// visit, with the revisit budget and fallbacks).  Returns whether anything
// changed (a dense visit always writes its block back).
template <int BH, int CONN>
__device__ __forceinline__ bool visit_block(const TaskDev &t, Lds<BH> &L, WaveStats &st, bool dense, int bh, int bw,
                                            int budget, bool wide_first) {
    return converge_block<BH, CONN>(L, t.qcap, st, !dense, bh, bw, dense ? -1 : budget, wide_first && !dense,
                                    dense ? t.scan_rounds : 0);
}

template <int BH>
__global__ __launch_bounds__(64) void dense_pass(TaskTable tt, KArgs a) {
    Lds<BH> L = lds_layout<BH>();
    const int ln = lane_id();
    const uint32_t total = total_blocks_of(tt);
    WaveStats st;
    for (uint32_t gb = blockIdx.x; gb < total; gb += gridDim.x) {
        const int ti = uniform(find_task(tt, gb));
        const TaskDev t = task_of(tt, ti);
        const int lb = (int)(gb - t.block0);
        const int by = lb / t.nbx, bx = lb % t.nbx;
        const BlockGeom g = geom<BH>(t, by, bx);
        load_block<BH, false>(t, g, L, t.op == OP_FILL);
        clear_halo<BH>(L);
        for (int r = ln; r < BH; r += LANES) L.rowdirty[r] = 0;
        __syncthreads();
        if (t.conn == 8)
            dense_block<BH, 8>(t, g, L, st);
        else
            dense_block<BH, 4>(t, g, L, st);
        store_block<BH, false>(t, g, L, true);
        st.dense += 1;
        __syncthreads();
    }
    flush_stats(a.work, st);
}

// K2: border seeding.  Each block's border against its neighbours.

template <int BH>
__global__ __launch_bounds__(64) void border_seed(TaskTable tt, KArgs a) {
    Lds<BH> L = lds_layout<BH>();
    const int ln = lane_id();
    const uint32_t total = total_blocks_of(tt);
    const uint32_t ring_cap = ring_cap_of(tt);
    WaveStats st;
    for (uint32_t gb = blockIdx.x; gb < total; gb += gridDim.x) {
        const int ti = uniform(find_task(tt, gb));
        const TaskDev t = task_of(tt, ti);
        const int lb = (int)(gb - t.block0);
        const int by = lb / t.nbx, bx = lb % t.nbx;
        const BlockGeom g = geom<BH>(t, by, bx);
        // border rows and columns of the block's current marker, and the halo
        const int x = 4 * ln;
        const int valid = min(4, g.bw - x);
        const uint32_t top = marker4(t, g.y0, g.x0 + x, valid);
        const uint32_t bot = marker4(t, g.y0 + g.bh - 1, g.x0 + x, valid);
        uint32_t lft[2] = {0, 0}, rgt[2] = {0, 0};
        for (int k = 0; k < 2; ++k) {
            const int r = ln + k * LANES;
            if (r < g.bh) {
                lft[k] = marker1(t, g.y0 + r, g.x0);
                rgt[k] = marker1(t, g.y0 + r, g.x0 + g.bw - 1);
            }
        }
        load_halo<BH>(t, g, L);
        *L.Jw(0, ln) = top;
        *L.Jw(g.bh - 1, ln) = bot;
        for (int k = 0; k < 2; ++k) {
            const int r = ln + k * LANES;
            if (r < g.bh) {
                L.Jb(r, 0) = (uint8_t)lft[k];
                L.Jb(r, g.bw - 1) = (uint8_t)rgt[k];
            }
        }
        __syncthreads();
        if (!check_neighbours<BH>(a, ring_cap, ti, t, g, by, bx, L, nullptr, st)) {
            if (ln == 0) __hip_atomic_store(&a.work->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
        }
        __syncthreads();
    }
    flush_stats(a.work, st);
}

// K3: revisit scheduler.
//
// A wave without a block of its own takes a ticket (the next ring position)
// and waits on that position's slot alone, so idle waves spread their polling
// over separate lines.  The wave that completes the last outstanding visit
// sets `done` and writes SLOT_EXIT into the slot of every ticket handed out so
// far; a wave that takes a ticket later sees `done` right after taking it (the
// two updates of ring_head are ordered, and `done` is written before).

// Wait for the block id at ticket `ticket`.  Returns the global block id, -1
// when all work is done, -2 on abort (watchdog).
__device__ __forceinline__ int wait_ticket(const KArgs &a, uint32_t ring_cap, uint32_t ticket) {
    const int ln = lane_id();
    Work *w = a.work;
    uint32_t *slot = a.ring + (size_t)(ticket % ring_cap) * RING_STRIDE;
    int state = 0;
    if (ln == 0 && __hip_atomic_load(&w->done, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT)) state = 1;
    if (uniform(state)) return -1;
    uint32_t seen = 0;
    if (ln == 0) seen = __hip_atomic_load(&w->progress, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    seen = uniform(seen);
    uint64_t since = wall_clock64();
    for (int spin = 0;; ++spin) {
        uint32_t v = 0;
        if (ln == 0) {
            v = __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (v != 0u && v != SLOT_EXIT) __hip_atomic_store(slot, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        v = uniform(v);
        if (v == SLOT_EXIT) return -1;
        if (v != 0u) return (int)(v - 1u);
        if ((spin & 63) == 63) {   // abort flag and watchdog: no visit completed for too long
            uint32_t pr = 0, ab = 0;
            if (ln == 0) {
                pr = __hip_atomic_load(&w->progress, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ab = __hip_atomic_load(&w->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            pr = uniform(pr);
            if (uniform(ab)) return -2;
            const uint64_t now = wall_clock64();
            if (pr != seen) {
                seen = pr;
                since = now;
            } else if (now - since > a.watchdog_ticks) {
                if (ln == 0) __hip_atomic_store(&w->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return -2;
            }
        }
        backoff(spin);
    }
}

// The last outstanding visit is complete: release every waiting ticket holder.
__device__ __forceinline__ void release_waiters(const KArgs &a, uint32_t ring_cap) {
    const int ln = lane_id();
    Work *w = a.work;
    uint32_t h = 0, tl = 0;
    if (ln == 0) {
        __hip_atomic_store(&w->done, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        h = __hip_atomic_fetch_add(&w->ring_head, 0u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        tl = __hip_atomic_load(&w->ring_tail, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    }
    h = uniform(h);
    tl = uniform(tl);
    // tickets below ring_tail were all served; the others wait for a block
    for (uint32_t pos = tl + (uint32_t)ln; (int32_t)(h - pos) > 0; pos += LANES)
        __hip_atomic_store(a.ring + (size_t)(pos % ring_cap) * RING_STRIDE, SLOT_EXIT, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

template <int BH>
__global__ __launch_bounds__(64) void revisit_drain(TaskTable tt, KArgs a) {
    Lds<BH> L = lds_layout<BH>();
    if (lane_id() == 0) {   // this wave's spill queue (capacity 0: none)
        const uint64_t sb = (uint64_t)(uintptr_t)(a.spill ? a.spill + (size_t)blockIdx.x * a.spill_cap : nullptr);
        volatile RK_LDS uint32_t *sp = L.sp;
        sp[0] = (uint32_t)sb;
        sp[1] = (uint32_t)(sb >> 32);
        sp[2] = a.spill ? a.spill_cap : 0u;
        sp[3] = 0u;
        sp[4] = 0u;
    }
    __syncthreads();
    const int ln = lane_id();
    Work *w = a.work;
    const uint32_t ring_cap = ring_cap_of(tt);
    WaveStats st;
    int keep = -1;   // block this wave requested and keeps for its next visit
    const bool wide_first = total_blocks_of(tt) <= WIDE_FRONT_LOAD * gridDim.x;   // latency-bound launch
    {   // nothing was requested at all: no visit will ever complete, leave now
        uint32_t pend = 0;
        if (ln == 0) pend = __hip_atomic_load(&w->pending, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        if (uniform(pend) == 0u) return;
    }

    int cur_ti = -1;      // task of the last visit and its descriptor (most visits stay in one task)
    TaskDev t{};
    uint32_t t_end = 0;
    while (true) {
        int gsel = keep;
        keep = -1;
        const bool claimed = gsel >= 0;   // a kept block was claimed when it was requested
        if (gsel < 0) {
            uint32_t ticket = 0;
            if (ln == 0)
                ticket = __hip_atomic_fetch_add(&w->ring_head, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            ticket = uniform(ticket);
            gsel = wait_ticket(a, ring_cap, ticket);
            if (gsel < 0) break;
        }

        const uint32_t gb = (uint32_t)gsel;
        if (cur_ti < 0 || gb < t.block0 || gb >= t_end) {
            cur_ti = uniform(find_task(tt, gb));
            t = task_of(tt, cur_ti);
            t_end = t.block0 + (uint32_t)(t.nby * t.nbx);
        }
        const int ti = cur_ti;
        const int lb = (int)(gb - t.block0);
        const int by = lb / t.nbx, bx = lb % t.nbx;
        const BlockGeom g = geom<BH>(t, by, bx);

        // ---- claim: clear D, set R (a kept block is owned already).  The previous owner and every requester
        // completed their (coherent) stores before updating the state word, so
        // loads issued after the claim returned see them.
        int first = 0;   // the block's first visit: a dense pass
        int lost = 0;    // the claim's compare-and-swap failed CAS_TRIES times in a row
        if (ln == 0) {
            if (!claimed) {
                uint32_t s = __hip_atomic_load(state_word(a, gb), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                lost = 1;
                // (the test hook expects a bit no state word has, so that every attempt fails)
                const uint32_t skew = a.test_fault == 1 ? 0x80000000u : 0u;
                for (int k = 0; k < CAS_TRIES; ++k) {
                    uint32_t e = s ^ skew;
                    if (__hip_atomic_compare_exchange_strong(state_word(a, gb), &e, (s & ~ST_D) | ST_R,
                                                             __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT)) {
                        lost = 0;
                        break;
                    }
                    s = e;
                }
                first = (s & ST_V) ? 0 : 1;
            }
            if (lost)
                __hip_atomic_store(&w->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            else if (first)
                st.dense += 1;
            else
                st.revisit += 1;
        }
        // never work on a block this wave does not own: give the launch up
        // instead (the host call reports RECON_EDEVICE)
        if (uniform(lost)) break;
        first = uniform(first);
        __syncthreads();
        __atomic_signal_fence(__ATOMIC_SEQ_CST);

        load_visit<BH>(t, g, L);
        __syncthreads();
        const int budget = mask_is_binary<BH>(L) ? a.binary_drain_budget : a.drain_budget;
        bool ok = true;
        for (int pass = 0;; ++pass) {
            if (pass > 0) load_halo<BH>(t, g, L);   // a re-run: neighbours changed meanwhile
            for (int r = ln; r < BH; r += LANES) L.rowdirty[r] = 0;
            __syncthreads();
            const bool dense = first && pass == 0;
            // a first visit: sweeps, dense seed and drain, with the halo as it
            // is now; a later one: the interior is converged, seed from the
            // border (one call site per connectivity keeps the kernel small)
            bool changed = t.conn == 8 ? visit_block<BH, 8>(t, L, st, dense, g.bh, g.bw, budget, wide_first)
                                       : visit_block<BH, 4>(t, L, st, dense, g.bh, g.bw, budget, wide_first);
            if (dense) changed = true;
            if (changed) {
                store_block<BH, true>(t, g, L, dense);
                vm_sync();   // the stores are complete before any request below
                ok = check_neighbours<BH>(a, ring_cap, ti, t, g, by, bx, L, &keep, st);
            }
            // ---- finish: re-run if requested meanwhile, else release
            int rerun = 0, stuck = 1;
            if (ln == 0) {
                uint32_t s = __hip_atomic_load(state_word(a, gb), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                for (int k = 0; k < CAS_TRIES; ++k) {
                    const uint32_t ns = ((s & ST_D) ? (s & ~ST_D) : (s & ~ST_R)) | ST_V;
                    if (__hip_atomic_compare_exchange_strong(state_word(a, gb), &s, ns, __ATOMIC_RELAXED,
                                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                        rerun = (s & ST_D) ? 1 : 0;
                        stuck = 0;
                        break;
                    }
                }
                if (rerun) st.rerun += 1;
            }
            rerun = uniform(rerun);
            // a block that could not be released stays owned: the launch gives up
            if (uniform(stuck)) ok = false;
            __syncthreads();
            if (!rerun || !ok) break;
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
        }
        // ---- the visit is complete.  A kept block inherits this visit's count
        // of outstanding work; otherwise the counts go down.  The watchdog
        // heartbeat is bumped on every eighth visit of a wave.
        int last = 0;
        if (ln == 0) {
            if ((st.revisit & 7u) == 0u)
                __hip_atomic_fetch_add(&w->progress, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (!ok) __hip_atomic_store(&w->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (keep < 0) {
                const uint32_t left = __hip_atomic_fetch_sub(a.tile_pending + ti, 1u, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT);
                const uint32_t all = __hip_atomic_fetch_sub(&w->pending, 1u, __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_AGENT);
                if (left == 1u) {
                    __hip_atomic_store(a.tile_done + ti, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    // the task's last visit: every visit of it wrote its blocks back
                    // and waited for the stores before its count went down, so the
                    // host may take the result now (serving completes the ticket
                    // without waiting for the rest of the launch)
                    if (a.host_done)
                        __hip_atomic_store(a.host_done + ti, a.launch_seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
                }
                last = all == 1u;
            }
        }
        if (uniform(last)) release_waiters(a, ring_cap);
        if (!ok) break;
    }
    if (lane_id() == 0) {   // entries that went through the spill queue
        const uint32_t taken = ((volatile RK_LDS uint32_t *)L.sp)[4];
        if (taken) __hip_atomic_fetch_add(&w->stat_spill, (unsigned long long)taken, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
    }
    flush_stats(w, st);
}

// ---------------------------------------------------------------------------
// set-up and finishing kernels (grid-stride)

// Copy a task table from host-visible memory into the device table.
__global__ void copy_table(const uint8_t *src, uint8_t *dst, uint32_t bytes) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < bytes; i += gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// The outcome of a launch for the host, without a wait: 1 if the scheduler of
// any of its (up to three) block-height groups gave up, else 0, stored into
// pinned host memory.
__global__ void launch_outcome(const Work *w0, const Work *w1, const Work *w2, uint32_t *out) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    uint32_t ab = 0;
    const Work *ws[3] = {w0, w1, w2};
    for (int k = 0; k < 3; ++k)
        if (ws[k]) ab |= __hip_atomic_load((uint32_t *)&ws[k]->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(out, ab ? 1u : 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Reset the scheduling state of the batch.
//   RESET_STAGED     the scheduler starts empty (the dense and border kernels
//                    of the staged pipeline run first);
//   RESET_QUEUE_ALL  every block starts requested and in the ring (in block
//                    order), so that the persistent revisit kernel makes each
//                    block's first visit itself;
//   RESET_ROUTE      counters only, and a first look at every task's mask for
//                    the component route (sample_route); the ring is filled by
//                    prepare after the routes are decided, with the blocks of
//                    the tasks that do not take the route.  When the samples
//                    alone show that no task can take it (every mask grey, or
//                    thick beside grey work), the last sampling wave decides
//                    every route and the classification is skipped.
enum { RESET_STAGED = 0, RESET_QUEUE_ALL = 1, RESET_ROUTE = 2 };
// Up to this many tasks, one wave samples them all (RESET_ROUTE).
constexpr uint32_t SAMPLE_ONE_WAVE = 8;

__device__ void decide_tasks(const TaskTable &tt, const KArgs &a);

// A first look at task k's mask for the component route, by one wave: 1024
// pixels spread over the image (16 rows of 64 columns), the OR and AND of
// the nonzero values found, and how thin the foreground is: the share of
// sampled foreground pixels that start a horizontal run (whose left neighbour
// is background) -- about 1 / (mean run length); at least 1/32 counts as thin
// (a corridor, noise), as does a sample without foreground.  The task's route
// words are written whole here (their identities plus what the sample saw).
// A grey mask nearly always shows two different nonzero values in the sample,
// and the classification then skips it whole; it, or a task without a label
// plane, marks the launch as having block-route work (has_grey).
__device__ void sample_route(const TaskTable &tt, const TaskDev &t, int k, uint32_t *route, Work *w) {
    const int ln = lane_id();
    uint32_t o = 0, an = 0xffu, fg = 0, starts = 0;
    if (t.lab) {
        // every sampled pixel and its left neighbour loaded together (one
        // round trip instead of one per sampled row)
        const int x = (int)(((int64_t)(2 * ln + 1) * t.w) / 128), xl = x > 0 ? x - 1 : x;
        uint32_t b[16], l[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int y = (int)(((int64_t)(2 * r + 1) * t.h) / 32);
            b[r] = mask1(t, y, x);
            l[r] = x > 0 ? mask1(t, y, xl) : 0u;
        }
#pragma unroll
        for (int r = 0; r < 16; ++r)
            if (b[r]) {
                o |= b[r];
                an &= b[r];
                fg += 1;
                if (l[r] == 0u) starts += 1;
            }
    }
    for (int d = 1; d < LANES; d <<= 1) {
        o |= (uint32_t)__shfl_xor((int)o, d);
        an &= (uint32_t)__shfl_xor((int)an, d);
        fg += (uint32_t)__shfl_xor((int)fg, d);
        starts += (uint32_t)__shfl_xor((int)starts, d);
    }
    if (ln == 0) {
        uint32_t *rw = route + ROUTE_WORDS * k;
        rw[0] = o;
        rw[1] = an;
        for (int q = 2; q < ROUTE_WORDS; ++q) rw[q] = 0u;
        rw[4] = (fg == 0u || 32u * starts >= fg) ? 1u : 0u;
        if (!t.lab || (o != 0u && o != an)) w->has_grey = seq_of(tt);   // (any writer, same value)
    }
}

// Counts one sampled task of the launch (lane 0 of the sampling wave, after
// its route words are written): the count lives in the low half of a word
// whose high half is the launch's number, so that no other kernel has to clear
// it between launches.  The release orders the sample's writes (and, in the
// wave holding thread 0, the counter resets) before the count; uniform true in
// the wave whose count completes the launch's samples.
__device__ __forceinline__ bool count_sample(const TaskTable &tt, Work *w, uint32_t n_tasks) {
    uint32_t last = 0;
    if (lane_id() == 0) {
        const unsigned long long seq = seq_of(tt);
        unsigned long long cur = __hip_atomic_load(&w->sample_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        unsigned long long nxt;
        do {
            nxt = (cur >> 32) == seq ? cur + 1ull : (seq << 32) | 1ull;
        } while (!__hip_atomic_compare_exchange_weak(&w->sample_word, &cur, nxt, __ATOMIC_RELEASE, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT));
        last = (uint32_t)nxt == n_tasks ? 1u : 0u;
    }
    return uniform(last) != 0u;
}

// After every sample (one wave): can some task still take the component
// route?  Only a mask whose sample shows at most one nonzero value, and then
// only when it is thin, or no task keeps the block route anyway, or the
// policy asks for the route for every two-valued mask (as decide_tasks).
__device__ __forceinline__ bool route_possible(const TaskTable &tt, const KArgs &a) {
    const uint32_t n_tasks = n_tasks_of(tt);
    const bool grey_work = __hip_atomic_load(&a.work->has_grey, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == seq_of(tt);
    int any = 0;
    for (uint32_t i = (uint32_t)lane_id(); i < n_tasks; i += LANES) {
        const TaskDev t = task_of(tt, (int)i);
        uint32_t *rw = a.route + ROUTE_WORDS * i;
        const uint32_t o = __hip_atomic_load(rw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t an = __hip_atomic_load(rw + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t thin = __hip_atomic_load(rw + 4, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        any |= (t.lab && (o == 0u || o == an) && (a.route_policy == 1 || !grey_work || thin != 0u)) ? 1 : 0;
    }
    return __ballot(any != 0) != 0ull;
}

__global__ void reset_work(TaskTable tt, KArgs a, int mode) {
    Work *w = a.work;
    uint32_t *state = a.state, *ring = a.ring, *tile_pending = a.tile_pending, *tile_done = a.tile_done;
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t nth = gridDim.x * blockDim.x;
    const uint32_t n_tasks = n_tasks_of(tt), total = total_blocks_of(tt), ring_cap = ring_cap_of(tt);
    const bool queue_all = mode == RESET_QUEUE_ALL;
    if (tid == 0) {
        w->pending = queue_all ? total : 0u;
        w->done = 0;
        w->ring_head = 0;
        w->ring_tail = queue_all ? total : 0u;
        w->abort = 0;
        w->progress = 0;
        w->stat_dense = w->stat_revisit = w->stat_rerun = w->stat_overflow = w->stat_request = 0;
        w->stat_route = 0;
        w->stat_spill = 0;
        w->classify_done = 0;
    }
    if (mode != RESET_ROUTE) {
        // (without queue_all the dense pass visits every block first)
        for (uint32_t i = tid; i < total; i += nth) state[(size_t)i * STATE_STRIDE] = queue_all ? ST_D : ST_V;
        for (uint32_t i = tid; i < ring_cap; i += nth)
            ring[(size_t)i * RING_STRIDE] = queue_all && i < total ? i + 1u : 0u;
    }
    if (mode != RESET_ROUTE) {
        for (uint32_t i = tid; i < n_tasks; i += nth) {
            const TaskDev t = task_of(tt, (int)i);
            tile_pending[i] = queue_all ? (uint32_t)(t.nby * t.nbx) : 0u;
            tile_done[i] = 0;
        }
        return;
    }
    if (n_tasks <= SAMPLE_ONE_WAVE) {
        // few tasks: the wave holding thread 0 samples them all in turn and
        // decides at once (no counting across waves, no fences)
        if (tid >= (uint32_t)LANES) return;
        for (uint32_t k = 0; k < n_tasks; ++k) {
            if (lane_id() == 0) {
                tile_pending[k] = 0u;
                tile_done[k] = 0u;
            }
            sample_route(tt, task_of(tt, (int)k), (int)k, a.route, w);
        }
        vm_sync();   // lane 0's writes are complete before the other lanes read them
        RK_LANE_SYNC();
        if (!route_possible(tt, a)) {
            decide_tasks(tt, a);
            if (lane_id() == 0) w->classify_skip = seq_of(tt);
        }
        return;
    }
    // one wave per task (grid-stride over the waves of the grid); the wave
    // holding thread 0 takes task 0 first, so its resets above are released
    // with that task's count
    for (uint32_t k = tid / LANES; k < n_tasks; k += nth / LANES) {
        if (lane_id() == 0) {
            tile_pending[k] = 0u;
            tile_done[k] = 0u;
        }
        sample_route(tt, task_of(tt, (int)k), (int)k, a.route, w);
        if (count_sample(tt, w, n_tasks)) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            if (!route_possible(tt, a)) {
                decide_tasks(tt, a);
                if (lane_id() == 0) w->classify_skip = seq_of(tt);
            }
        }
    }
}

// After the classification (RESET_ROUTE), the route of every task, decided
// by one wave (the last workgroup of comp_classify).  A two-valued mask takes
// the component route when its foreground is thin (there block visits would
// chain along corridors), when the launch has no task that keeps the block
// route anyway (nothing for its visits to overlap with), or when the policy
// asks for it for every two-valued mask; a thick two-valued mask in a launch
// with grey tasks stays on the block route, whose visits then fill the
// compute units the grey tasks' dependency chains leave idle.  Each task that
// keeps the block route reserves a range of ring positions for its blocks and
// counts them as outstanding; a task on the component route is complete as
// far as the block scheduler is concerned, and marks the launch as having one
// (route_any, so that the route's kernels return at once when no task takes it).
__device__ void decide_tasks(const TaskTable &tt, const KArgs &a) {
    const uint32_t n_tasks = n_tasks_of(tt), seq = seq_of(tt);
    const int ln = lane_id();
    const bool grey_work = __hip_atomic_load(&a.work->has_grey, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == seq;
    // the ring ranges follow task order: an exclusive prefix sum of the
    // block counts of the tasks that keep the block route (one wave, 64 tasks
    // per step; `base` carries the sum of the steps before)
    uint32_t base = 0;
    bool any_route = false;
    for (uint32_t i0 = 0; i0 < n_tasks; i0 += LANES) {
        const uint32_t i = i0 + (uint32_t)ln;
        uint32_t nb = 0;
        bool take = false;
        if (i < n_tasks) {
            const TaskDev t = task_of(tt, (int)i);
            uint32_t *rw = a.route + ROUTE_WORDS * i;
            const uint32_t o = __hip_atomic_load(rw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t an = __hip_atomic_load(rw + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t thin = __hip_atomic_load(rw + 4, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            take = t.lab && (o == 0u || o == an) && (a.route_policy == 1 || !grey_work || thin != 0u);
            rw[3] = take ? 1u : 0u;
            if (take) a.tile_done[i] = 1u;
            else nb = (uint32_t)(t.nby * t.nbx);
        }
        uint32_t incl = nb;   // inclusive prefix sum over the wave
        for (int d = 1; d < LANES; d <<= 1) {
            const uint32_t o = __shfl_up(incl, (unsigned)d);
            if (ln >= d) incl += o;
        }
        if (i < n_tasks && !take) {
            a.route[ROUTE_WORDS * i + 2] = base + incl - nb;
            a.tile_pending[i] = nb;
        }
        base += __shfl(incl, LANES - 1);
        any_route |= __ballot(take) != 0ull;
    }
    if (ln == 0) {
        a.work->ring_tail = base;
        a.work->pending = base;
        if (any_route) a.work->route_any = seq;
    }
}

// The initial marker of 4 pixels of a task that is not a plain dilation:
// fill-holes 255 - X on the image frame and 0 inside; erosion 255 - J (the
// caller's marker); h-dome and regional maxima max(I - h, 0) bytewise (I -
// min(I, h) never borrows across bytes).  `jrow` is the marker row.
__device__ __forceinline__ uint32_t initial_marker4(const TaskDev &t, const uint8_t *jrow, int y, int x, int valid) {
    if (t.op == OP_FILL) {   // (only a word on the image frame reads the image)
        const bool frame = y == 0 || y == t.h - 1 || x == 0 || x + 4 >= t.w;
        return frame ? fill_init4(t, y, x, valid, mask4(t, y, x, valid)) : 0u;
    }
    if (t.op == OP_ERODE) return ~gload4(jrow, x, valid, t.aligned);
    const uint32_t iv = gload4(t.i + (int64_t)y * t.pitch_i, x, valid, t.aligned);
    return iv - bmin4(iv, (uint32_t)t.hval * 0x01010101u);
}

// The result of 4 pixels from the fixed point jv: fill-holes and erosion
// 255 - J; h-dome I - J (J <= I bytewise, so the dword difference never
// borrows across bytes); regional maxima 255 where I - J > 0, else 0.
__device__ __forceinline__ uint32_t mapped_result4(const TaskDev &t, uint32_t jv, int y, int x, int valid) {
    if (t.op == OP_FILL || t.op == OP_ERODE) return ~jv;
    const uint32_t d = gload4(t.i + (int64_t)y * t.pitch_i, x, valid, t.aligned) - jv;
    if (t.op == OP_HDOME) return d;
    // 0x80 in every byte of d that is nonzero, then 0x01 -> 0xff
    const uint32_t nz = (d | ((d & 0x7f7f7f7fu) + 0x7f7f7f7fu)) & 0x80808080u;
    return (nz >> 7) * 0xffu;
}

// Row-strided walk over a task's plane, 16 bytes per thread: workgroup b
// takes rows b, b + gridDim.x, ..., its threads a row's consecutive 16-byte
// chunks (coalesced, no division of a flat index).  f(y, x, n): the chunk at
// column x of row y, n (1..16) of its pixels inside the image.
template <typename F>
__device__ __forceinline__ void for_each_chunk(const TaskDev &t, F f) {
    for (int y = (int)blockIdx.x; y < t.h; y += (int)gridDim.x)
        for (int x = 16 * (int)threadIdx.x; x < t.w; x += 16 * (int)blockDim.x) f(y, x, min(16, t.w - x));
}

__device__ __forceinline__ bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0u; }
typedef uint32_t u32x4 __attribute__((vector_size(16)));   // one 16-byte access

// Initial marker plane of every task that is not a plain dilation, written
// before any block is visited (so that any block can read any other's marker
// before that block's first visit).  Tasks on the component route are
// skipped (their kernels derive the marker themselves; `route` null: no
// task takes it).  A whole aligned chunk is one 16-byte store.
__device__ void init_marker_all(const TaskTable &tt, const uint32_t *route) {
    const uint32_t n = n_tasks_of(tt);
    for (uint32_t k = 0; k < n; ++k) {
        const TaskDev t = task_of(tt, (int)k);
        if (t.op == OP_DILATE || on_component_route(route, t, (int)k)) continue;
        for_each_chunk(t, [&](int y, int x, int nx) {
            uint8_t *jrow = t.j + (int64_t)y * t.pitch_j;
            uint32_t v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int valid = min(4, nx - 4 * q);
                v[q] = valid > 0 ? initial_marker4(t, jrow, y, x + 4 * q, valid) : 0u;
            }
            if (nx == 16 && aligned16(jrow + x)) {
                *(RK_GLOBAL u32x4 *)gp(jrow + x) = u32x4{v[0], v[1], v[2], v[3]};
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) gstore4(jrow, x + 4 * q, min(4, nx - 4 * q), t.aligned, v[q]);
            }
        });
    }
}

__global__ void init_marker(TaskTable tt, const uint32_t *route) { init_marker_all(tt, route); }

// Map the fixed point J back to each task's result (mapped_result4), except
// for tasks on the component route, whose kernels write their result.  Whole
// aligned chunks are one 16-byte load and one 16-byte store.
__global__ void finish_result(TaskTable tt, const uint32_t *route) {
    const uint32_t n = n_tasks_of(tt);
    for (uint32_t k = 0; k < n; ++k) {
        const TaskDev t = task_of(tt, (int)k);
        if (t.op == OP_DILATE || on_component_route(route, t, (int)k)) continue;
        for_each_chunk(t, [&](int y, int x, int nx) {
            const uint8_t *jrow = t.j + (int64_t)y * t.pitch_j;
            uint8_t *orow = t.img + (int64_t)y * t.pitch_img;
            const bool vec = nx == 16 && aligned16(jrow + x) && aligned16(orow + x);
            uint32_t jv[4];
            if (vec) {
                const u32x4 q4 = *(const RK_GLOBAL u32x4 *)gp(jrow + x);
#pragma unroll
                for (int q = 0; q < 4; ++q) jv[q] = q4[q];
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) jv[q] = gload4(jrow, x + 4 * q, min(4, nx - 4 * q), t.aligned);
            }
            uint32_t o[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int valid = min(4, nx - 4 * q);
                o[q] = valid > 0 ? mapped_result4(t, jv[q], y, x + 4 * q, valid) : 0u;
            }
            if (vec) {
                *(RK_GLOBAL u32x4 *)gp(orow + x) = u32x4{o[0], o[1], o[2], o[3]};
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) gstore4(orow, x + 4 * q, min(4, nx - 4 * q), t.aligned, o[q]);
            }
        });
    }
}

// After the route decisions (RESET_ROUTE): every block requested and in its
// task's ring range, or idle (a task on the component route, whose blocks
// nobody ever requests), ring positions past the queued blocks cleared; then
// the marker planes of the tasks that keep the block route (as init_marker).
__global__ void prepare(TaskTable tt, KArgs a, int any_mapped) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t nth = gridDim.x * blockDim.x;
    const uint32_t total = total_blocks_of(tt), ring_cap = ring_cap_of(tt);
    const uint32_t queued = a.work->ring_tail;
    for (uint32_t gb = tid; gb < total; gb += nth) {
        const int k = find_task(tt, gb);
        const TaskDev t = task_of(tt, k);
        if (on_component_route(a, t, k)) {
            a.state[(size_t)gb * STATE_STRIDE] = ST_V;
        } else {
            a.state[(size_t)gb * STATE_STRIDE] = ST_D;
            a.ring[(size_t)(a.route[ROUTE_WORDS * k + 2] + (gb - t.block0)) * RING_STRIDE] = gb + 1u;
        }
    }
    for (uint32_t i = queued + tid; i < ring_cap; i += nth) a.ring[(size_t)i * RING_STRIDE] = 0u;
    if (any_mapped) init_marker_all(tt, a.route);
}

// Self-test input pattern for the row closure (shared with the host check).
__host__ __device__ inline uint32_t self_test_mask(uint32_t p) {
    const uint32_t h = p * 2654435761u;
    return (h >> 13) % 5u == 0u ? (h >> 20) % 40u : 120u + (h >> 8) % 136u;   // dips cut runs
}
__host__ __device__ inline uint32_t self_test_low(uint32_t p, uint32_t mask) {
    const uint32_t h = (p + 977u) * 2246822519u;
    const uint32_t v = (h >> 17) % 64u;
    return (h >> 11) % 61u == 0u || v > mask ? mask : v;    // a few sources at the mask
}

// Self-test (checks that this code object runs and that the DPP lane moves
// and the row closure work the way the kernels assume):
//   out[i] = 3 i + 1,  out[n + i] = from_lower(i + 100),  out[2n + i] = from_upper(i + 100)
// for i < n, with n a multiple of the block size (all lanes active).
__global__ void self_test(uint32_t *out, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t lo = from_lower(i + 100u), hi = from_upper(i + 100u);
    uint32_t m4 = 0, l4 = 0;
    for (int j = 0; j < 4; ++j) {
        const uint32_t p = 4u * i + (uint32_t)j;
        const uint32_t mh = self_test_mask(p), ml = self_test_low(p, mh);
        m4 |= mh << (8 * j);
        l4 |= ml << (8 * j);
    }
    const uint32_t wave = i / 64u;
    const uint32_t rc = row_closure(l4, m4, (wave * 37u) & 255u, (wave * 91u + 7u) & 255u);
    if (i < n) {
        out[i] = i * 3u + 1u;
        out[n + i] = lo;
        out[2 * n + i] = hi;
        out[3 * n + i] = rc;
    }
}

}  // namespace rk
