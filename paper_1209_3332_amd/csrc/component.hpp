// component.hpp -- the component route of the reconstruction kernels: tasks
// whose mask takes at most two values, 0 and one c > 0, reconstructed through
// connected-component labelling instead of block visits.
//
// For such a mask the reconstruction has a closed form.  By its bottleneck-
// path characterisation (rho(p) is the largest, over sources q and paths from
// q to p, of min(J(q), the smallest mask value on the path)), a path through a
// pixel of mask 0 contributes 0, and a path inside one connected component C
// of {I = c} contributes min(J(q), c).  A path from outside C into C must pass
// a pixel of mask 0, so
//     rho(p) = 0                                    where I(p) = 0,
//     rho(p) = max over q in C(p) of min(J(q), c)   where I(p) = c.
// That is a labelling of {I != 0} followed by a maximum per component: work
// proportional to the pixels, with no chain of dependent block visits.  A
// 1-pixel corridor winding across a 4096 x 4096 tile, which the block
// scheduler can only follow one block at a time (hundreds of thousands of
// visits in sequence), takes a few labelling passes here.  The bytes are the
// same as the block route's (the reconstruction is unique); the route is only
// faster.
//
// Kernels (one 64-lane wave per workgroup, grid-stride over the blocks of all
// tasks of the launch, in the scheduler's block numbering: a block of BH x 256
// pixels is BH / 16 labelling tiles of 16 x 256, or BH rows of 256 pixels),
// after reset_work has sampled every task's mask (sample_route):
//   comp_classify     OR and AND of the nonzero (transformed) mask values of
//                     every task, into two words per task: the mask is
//                     two-valued when they are equal (one nonzero value) or the
//                     OR is 0 (an all-zero mask).  A wave skips the rows of a
//                     task already known to hold two different nonzero values,
//                     or that cannot take the route whatever its values.
//                     The last workgroup decides every task's route
//                     (decide_tasks), and prepare then fills the ring with the
//                     blocks of the others.  The whole kernel returns at once
//                     when the samples already decided every route;
//   comp_label_local  tile-local labelling of {I != 0} (label.hpp's label_tile)
//                     into the task's int32 label plane;
//   comp_label_merge  unions across tile borders (merge_tile);
//   comp_flatten_max  every pixel's node id becomes its root's, and each pixel
//                     offers min(J, I) to its root: an atomic maximum on the
//                     root's own entry of the label plane, encoded as
//                     ENC + value (ENC is above every node id, so a root
//                     entry at or above ENC marks a root that has an offer);
//   comp_write        the reconstruction: 0 on mask 0, else the value its
//                     root's entry holds (0 for a root without any offer),
//                     written as the task's result (into the caller's marker
//                     for a dilation, mapped as finish_result would otherwise).
// These tasks need no marker plane (the offers derive their initial marker
// as init_marker would), and none of their blocks is ever queued: init_marker,
// the ring and finish_result skip them.
#pragma once
#include "kernels.hpp"
#include "label.hpp"

namespace rk {

constexpr int32_t COMP_ENC = 0x40000000;   // above every node id (pitched index + 1 < 2^30)

// Labelling arguments of a task's (transformed) mask and label plane.
__device__ __forceinline__ LabelArgs comp_label_args(const TaskDev &t) {
    LabelArgs la{};
    la.img = t.i;
    la.pitch_img = t.pitch_i;
    la.lab = t.lab;
    la.pitch_lab = t.pitch_lab;
    la.h = t.h;
    la.w = t.w;
    la.conn = t.conn;
    la.tiles_x = t.nbx;     // LT_W == BW: a block column is a tile column
    la.bits = nullptr;
    la.lab_vec = 1;   // the planes are 256-byte aligned with a pitch of a multiple of 4 elements
    la.fg_inv = t.minv;
    return la;
}

// Walks the global index space of the launch's blocks: unit u of `per` units
// per block -> task, block row / column.  cur caches the last task.
struct UnitWalk {
    int cur = -1;
    TaskDev t{};
    uint32_t t_end = 0;
    __device__ __forceinline__ void at(const TaskTable &tt, uint32_t gb) {
        if (cur < 0 || gb < t.block0 || gb >= t_end) {
            cur = uniform(find_task(tt, gb));
            t = task_of(tt, cur);
            t_end = t.block0 + (uint32_t)(t.nby * t.nbx);
        }
    }
};

// Classification: one wave per block (grid-stride), the block's rows loaded
// together; each lane keeps the OR and AND of its nonzero mask bytes, the
// wave combines them once per task it leaves, and only a combination that
// changes a task's words is written.  A wave skips the blocks of a task whose
// words already show two different nonzero values (it can never take the
// route); the words are read with plain loads there, a stale copy only
// skipping less.
template <int BH>
__global__ __launch_bounds__(64) void comp_classify(TaskTable tt, KArgs a) {
    if (a.work->classify_skip == seq_of(tt)) return;   // the samples decided every route
    const int ln = lane_id();
    const uint32_t n = total_blocks_of(tt);
    UnitWalk wk;
    int acc_k = -1;                 // task whose partial OR / AND this wave holds
    uint32_t acc_or = 0, acc_and = 0xffu;
    const uint32_t seq = seq_of(tt);
    bool wrote = false;             // (lane 0) this workgroup changed a route word or has_grey
    auto flush = [&]() {
        if (acc_k < 0) return;
        for (int d = 1; d < LANES; d <<= 1) {
            acc_or |= (uint32_t)__shfl_xor((int)acc_or, d);
            acc_and &= (uint32_t)__shfl_xor((int)acc_and, d);
        }
        if (ln == 0) {
            uint32_t *wo = a.route + ROUTE_WORDS * acc_k, *wa = wo + 1;
            const uint32_t co = __hip_atomic_load(wo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((co | acc_or) != co) __hip_atomic_fetch_or(wo, acc_or, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t ca = __hip_atomic_load(wa, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((ca & acc_and) != ca) __hip_atomic_fetch_and(wa, acc_and, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t no = co | acc_or, na = ca & acc_and;
            wrote |= (no != co) || (na != ca);
            // this task is grey (any writer, same value; a plain load first so
            // that a line already holding it is not written again by every wave)
            if (no != 0u && no != na && a.work->has_grey != seq) {
                a.work->has_grey = seq;
                wrote = true;
            }
        }
        acc_or = 0;
        acc_and = 0xffu;
    };
    for (uint32_t gb = blockIdx.x; gb < n; gb += gridDim.x) {
        wk.at(tt, gb);
        const TaskDev &t = wk.t;
        if (!t.lab) continue;
        if (wk.cur != acc_k) {
            flush();
            acc_k = wk.cur;
        }
        const uint32_t *rw = a.route + ROUTE_WORDS * wk.cur;
        const uint32_t seen_or = rw[0], seen_and = rw[1];
        if (uniform(seen_or != 0u && seen_or != seen_and ? 1 : 0)) continue;
        // a thick mask beside grey work keeps the block route whatever its
        // values (decide_tasks), so it is not read either
        if (uniform(a.route_policy != 1 && rw[4] == 0u && a.work->has_grey == seq ? 1 : 0)) continue;
        const int lb = (int)(gb - t.block0);
        const BlockGeom g = geom<BH>(t, lb / t.nbx, lb % t.nbx);
        const int x = g.x0 + 4 * ln;
        const int valid = min(4, g.bw - 4 * ln);
        uint32_t m[BH];
#pragma unroll
        for (int r = 0; r < BH; ++r) m[r] = (r < g.bh && valid > 0) ? mask4(t, g.y0 + r, x, valid) : 0u;
#pragma unroll
        for (int r = 0; r < BH; ++r)
            for (int j = 0; j < 4; ++j) {
                const uint32_t b = byte_of(m[r], j);
                if (b) {
                    acc_or |= b;
                    acc_and &= b;
                }
            }
    }
    flush();
    // the last workgroup to finish decides every task's route (decide_tasks):
    // a workgroup that wrote releases its writes with its count, and the last
    // one acquires them all (an agent-scope release or acquire writes back or
    // invalidates this XCD's L2, so the others neither fence nor acquire)
    uint32_t prior = 0;
    if (ln == 0) {
        uint32_t *cnt = &a.work->classify_done;
        prior = wrote ? __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT)
                      : __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (uniform(prior) + 1u == gridDim.x) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        decide_tasks(tt, a);
    }
}

template <int BH>
__global__ __launch_bounds__(64) void comp_label_local(TaskTable tt, KArgs a) {
    if (a.work->route_any != seq_of(tt)) return;   // no task of the launch takes the route
    RK_LDS uint32_t *par = (RK_LDS uint32_t *)dyn_lds();
    constexpr int PER = BH / LT_H;
    const uint64_t n = (uint64_t)total_blocks_of(tt) * PER;
    UnitWalk wk;
    for (uint64_t u = blockIdx.x; u < n; u += gridDim.x) {
        const uint32_t gb = (uint32_t)(u / PER);
        wk.at(tt, gb);
        if (!on_component_route(a, wk.t, wk.cur)) continue;
        const int lb = (int)(gb - wk.t.block0);
        const int y0 = (lb / wk.t.nbx) * BH + (int)(u % PER) * LT_H, x0 = (lb % wk.t.nbx) * BW;
        if (y0 >= wk.t.h) continue;
        const LabelArgs la = comp_label_args(wk.t);
        label_tile(la, par, y0, x0, img_aligned(la));
    }
}

template <int BH>
__global__ __launch_bounds__(64) void comp_label_merge(TaskTable tt, KArgs a) {
    if (a.work->route_any != seq_of(tt)) return;   // no task of the launch takes the route
    constexpr int PER = BH / LT_H;
    const uint64_t n = (uint64_t)total_blocks_of(tt) * PER;
    UnitWalk wk;
    for (uint64_t u = blockIdx.x; u < n; u += gridDim.x) {
        const uint32_t gb = (uint32_t)(u / PER);
        wk.at(tt, gb);
        if (!on_component_route(a, wk.t, wk.cur)) continue;
        const int lb = (int)(gb - wk.t.block0);
        const int y0 = (lb / wk.t.nbx) * BH + (int)(u % PER) * LT_H, x0 = (lb % wk.t.nbx) * BW;
        if (y0 >= wk.t.h) continue;
        merge_tile(comp_label_args(wk.t), y0, x0);
    }
}

// The root of node id a: every find ends at a root, an entry equal to its own
// id or at or above COMP_ENC (which only a root's entry becomes).  Plain loads:
// while this runs, entries only change to an ancestor (a pixel's own final
// root) or, at roots, to COMP_ENC + offer, so a stale value still leads to the
// root.  (No path compression here: a pixel's entry must end as its root.)
__device__ __forceinline__ int32_t comp_find(const int32_t *lab, int32_t a) {
    while (true) {
        const int32_t p = ((const RK_GLOBAL int32_t *)lab)[a - 1];
        if (p == a || p >= COMP_ENC) return a;
        a = p;
    }
}

template <int BH>
__global__ __launch_bounds__(64) void comp_flatten_max(TaskTable tt, KArgs a) {
    if (a.work->route_any != seq_of(tt)) return;   // no task of the launch takes the route
    const int ln = lane_id();
    const uint64_t n = (uint64_t)total_blocks_of(tt) * BH;
    UnitWalk wk;
    for (uint64_t u = blockIdx.x; u < n; u += gridDim.x) {
        const uint32_t gb = (uint32_t)(u / BH);
        wk.at(tt, gb);
        const TaskDev &t = wk.t;
        if (!on_component_route(a, t, wk.cur)) continue;
        const int lb = (int)(gb - t.block0);
        const int y = (lb / t.nbx) * BH + (int)(u % BH), x0 = (lb % t.nbx) * BW;
        if (y >= t.h) continue;
        const int x = x0 + 4 * ln;
        const int valid = min(4, t.w - x);
        int32_t *row = t.lab + (int64_t)y * t.pitch_lab;
        int32_t v[4] = {0, 0, 0, 0};
        if (valid > 0) lab_load4(row, x, t.w, 1, v);   // label rows are 16-byte aligned (pitch a multiple of 4)
        // the offers: min(J, I) of the foreground pixels, J the task's initial
        // marker (the caller's for a dilation, else derived here: no marker
        // plane is prepared for a task on this route)
        uint32_t jm = 0;
        if (valid > 0) {
            const uint8_t *jrow = t.j + (int64_t)y * t.pitch_j;
            const uint32_t j0 = t.op == OP_DILATE ? gload4(jrow, x, valid, t.aligned) : initial_marker4(t, jrow, y, x, valid);
            jm = bmin4(j0, mask4(t, y, x, valid));
        }
        int32_t root = 0;       // the lane's current root and the largest offer made to it
        uint32_t best = 0;
        int32_t last_v = 0, last_r = 0;   // the lane's pixels mostly share one tile root: one find for them
        for (int k = 0; k < 4 && k < valid; ++k) {
            if (v[k] == 0) continue;   // mask 0
            const int32_t self = (int32_t)((int64_t)y * t.pitch_lab + x + k + 1);
            // v[k] at or above COMP_ENC: this pixel is a root that already has an offer
            int32_t r;
            if (v[k] >= COMP_ENC) {
                r = self;
            } else if (v[k] == last_v) {
                r = last_r;
            } else {
                r = comp_find(t.lab, v[k]);
                last_v = v[k];
                last_r = r;
            }
            if (r != v[k] && v[k] < COMP_ENC)   // a non-root points straight at its root
                __hip_atomic_store((RK_GLOBAL int32_t *)(row + x + k), r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t off = byte_of(jm, k);
            if (r != root) {
                if (root != 0 && best != 0)
                    __hip_atomic_fetch_max((RK_GLOBAL int32_t *)(t.lab + (root - 1)), COMP_ENC + (int32_t)best,
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                root = r;
                best = 0;
            }
            best = max(best, off);
        }
        // a zero offer never raises anything: only positive ones reach the root,
        // and only when above what its entry shows already
        if (root != 0 && best != 0) {
            int32_t *slot = t.lab + (root - 1);
            const int32_t seen = __hip_atomic_load((RK_GLOBAL int32_t *)slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (seen < COMP_ENC + (int32_t)best)
                __hip_atomic_fetch_max((RK_GLOBAL int32_t *)slot, COMP_ENC + (int32_t)best, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

template <int BH>
__global__ __launch_bounds__(64) void comp_write(TaskTable tt, KArgs a) {
    if (a.work->route_any != seq_of(tt)) return;   // no task of the launch takes the route
    const int ln = lane_id();
    const uint64_t n = (uint64_t)total_blocks_of(tt) * BH;
    UnitWalk wk;
    for (uint64_t u = blockIdx.x; u < n; u += gridDim.x) {
        const uint32_t gb = (uint32_t)(u / BH);
        wk.at(tt, gb);
        const TaskDev &t = wk.t;
        if (!on_component_route(a, t, wk.cur)) continue;
        const int lb = (int)(gb - t.block0);
        const int y = (lb / t.nbx) * BH + (int)(u % BH), x0 = (lb % t.nbx) * BW;
        if (y >= t.h) continue;
        if (lb == 0 && u % BH == 0 && ln == 0)   // one count per task that took the route
            __hip_atomic_fetch_add(&a.work->stat_route, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int x = x0 + 4 * ln;
        const int valid = min(4, t.w - x);
        if (valid <= 0) continue;
        const int32_t *row = t.lab + (int64_t)y * t.pitch_lab;
        int32_t ev[4];
        lab_load4(row, x, t.w, 1, ev);
        uint32_t out = 0;
        for (int k = 0; k < 4 && k < valid; ++k) {
            const int32_t e = ev[k];
            if (e == 0) continue;                   // mask 0
            const int32_t r = e >= COMP_ENC ? e : t.lab[e - 1];   // own entry (a root) or the root's
            if (r >= COMP_ENC) out |= (uint32_t)(r - COMP_ENC) << (8 * k);
        }
        // the result itself: the reconstruction into the caller's marker for a
        // dilation, else mapped into the task's result plane
        if (t.op == OP_DILATE)
            gstore4(t.j + (int64_t)y * t.pitch_j, x, valid, t.aligned, out);
        else
            gstore4(t.img + (int64_t)y * t.pitch_img, x, valid, t.aligned, mapped_result4(t, out, y, x, valid));
    }
}

}  // namespace rk
