// recon.hip -- host runtime and C ABI of librecon (see include/recon.h).
//
// A context owns the device workspace of the block scheduler (block states,
// visit ring, counters, per-tile counts), the fill-holes scratch planes, a
// pinned staging area, and one captured HIP graph per block shape for
// recon_batch.  A launch sequence is
//     [copy task table] -> reset -> K1 dense pass -> K2 border seeding
//     -> K3 revisit drain -> [fill-holes result]
// Up to MAX_INLINE_TASKS tasks travel by value in the kernel arguments; larger
// batches are copied into device memory by a kernel that reads the pinned
// staging buffer.  The library itself issues no hipMemcpy: every transfer is
// a kernel, so every step of the sequence is ordered on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/recon.h"
#include "kernels.hpp"
#include "label.hpp"
#include "component.hpp"
#include "distance.hpp"

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(RECON_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));  \
    } while (0)

using rk::BatchHdr;
static_assert(sizeof(BatchHdr) == 64, "header size");

constexpr int kVariants = 3;   // block rows 16, 32, 64
constexpr int kTimingRing = 64; // launches whose timing marks are kept
constexpr int kBlockRows[kVariants] = {16, 32, 64};

int variant_of(int rows) {
    for (int v = 0; v < kVariants; ++v)
        if (kBlockRows[v] == rows) return v;
    return -1;
}

size_t lds_for(int v, int qcap) {
    switch (v) {
        case 0: return rk::lds_bytes<16>(qcap);
        case 1: return rk::lds_bytes<32>(qcap);
        default: return rk::lds_bytes<64>(qcap);
    }
}

const void *drain_fn(int v) {
    switch (v) {
        case 0: return reinterpret_cast<const void *>(&rk::revisit_drain<16>);
        case 1: return reinterpret_cast<const void *>(&rk::revisit_drain<32>);
        default: return reinterpret_cast<const void *>(&rk::revisit_drain<64>);
    }
}

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Wait for `ev` with a deadline; RECON_ETIMEDOUT if it does not complete.
int wait_event(hipEvent_t ev, double seconds, const char *what) {
    const auto t0 = std::chrono::steady_clock::now();
    while (true) {
        hipError_t q = hipEventQuery(ev);
        if (q == hipSuccess) return RECON_OK;
        if (q != hipErrorNotReady) return fail(RECON_EDEVICE, "%s failed: %s", what, hipGetErrorString(q));
        if (std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() > seconds)
            return fail(RECON_ETIMEDOUT, "%s has not completed after %.0f s", what, seconds);
        std::this_thread::sleep_for(std::chrono::microseconds(100));
    }
}

// ---- the fixed workspace of recon_dilate_noalloc
// A file-scope device array holds the scheduler workspace of one launch of at
// most NOALLOC_MAX_BLOCKS blocks: the counters, the per-tile counts, one state
// word per block and the visit ring.  Every GPU the library runs on holds its
// own copy until the process ends.  Host code never passes the array's name to
// a kernel (on the host it is only a stand-in for the symbol): recon_create
// looks up each device's address once with hipGetSymbolAddress, and launches
// use that address.
constexpr size_t NOALLOC_MAX_BLOCKS = 8192;
constexpr size_t align256(size_t x) { return (x + 255) / 256 * 256; }
constexpr size_t NOALLOC_TILE_OFF = align256(sizeof(rk::Work));
constexpr size_t NOALLOC_STATE_OFF = NOALLOC_TILE_OFF + 256;   // tile_pending, tile_done
constexpr size_t NOALLOC_RING_OFF =
    NOALLOC_STATE_OFF + align256(NOALLOC_MAX_BLOCKS * rk::STATE_STRIDE * sizeof(uint32_t));
constexpr size_t NOALLOC_BYTES =
    NOALLOC_RING_OFF +
    align256((NOALLOC_MAX_BLOCKS + rk::MAX_DRAIN_GRID + 1) * rk::RING_STRIDE * sizeof(uint32_t));

__device__ __align__(256) uint8_t scratch[NOALLOC_BYTES];

}  // namespace

struct recon_ctx {
    int device = 0;
    int cus = 0;
    recon_config cfg{};
    uint64_t watchdog_ticks = 0;
    // scheduler workspace
    uint8_t *d_table = nullptr;       // BatchHdr + TaskDev[cap_tasks]
    size_t cap_tasks = 0;
    rk::Work *d_work = nullptr;
    uint32_t *d_state = nullptr;
    uint32_t *d_ring = nullptr;
    size_t cap_blocks = 0;
    uint32_t *d_tile_pending = nullptr;
    uint32_t *d_tile_done = nullptr;
    uint32_t *d_route = nullptr;      // route words per task (component route)
    uint16_t *d_spill = nullptr;      // global spill queues of the revisit kernel's waves
    uint8_t *d_scratch = nullptr;     // fill-holes marker planes
    size_t cap_scratch = 0;
    // pinned staging (task table in, statistics out)
    uint8_t *h_table = nullptr;
    size_t cap_h_table = 0;
    rk::Work *h_work = nullptr;
    hipEvent_t table_used = nullptr;  // the last copy out of h_table has finished
    hipEvent_t last_done = nullptr;
    // timing marks of the last kTimingRing launches (before K1, after K1, K2, K3, the launch)
    // [5] opens the launch, [0]..[4] close its steps, [6] closes the component route (after [0])
    hipEvent_t tev[kTimingRing][7] = {};
    bool tev_graph[kTimingRing] = {};   // that launch replayed a graph (only its total is marked)
    bool tev_route[kTimingRing] = {};   // that launch ran the component route (on the second stream)
    bool tev_merged[kTimingRing] = {};  // that launch ran the persistent pipeline (marks around K3 only)
    uint64_t launches = 0;              // launch sequences enqueued so far
    bool have_last = false;
    rk::Work *last_work = nullptr;      // the counters of the last launch (context or fixed workspace)
    uint8_t *noalloc = nullptr;         // this device's fixed workspace (recon_dilate_noalloc)
    bool last_was_graph = false;   // the last launch replayed a graph (only its total is timed)
    int resident[kVariants] = {0, 0, 0};
    // captured batch graphs per variant
    hipStream_t cap_stream = nullptr;
    // the component route's labelling kernels run on a second stream beside
    // the revisit kernel (fork and join events, also inside captured graphs)
    hipStream_t aux_stream = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    hipGraphExec_t graph[kVariants] = {nullptr, nullptr, nullptr};
    size_t graph_cap_blocks[kVariants] = {0, 0, 0};
    size_t graph_cap_tasks[kVariants] = {0, 0, 0};
    size_t graph_cap_scratch[kVariants] = {0, 0, 0};
    // serving (created on the first recon_submit)
    struct Serve;
    Serve *serve = nullptr;
    bool is_lane = false;   // a serving lane's private context
    // serving lanes: host-visible completion word per task of a launch (the
    // revisit kernel writes the launch number there when the task's last
    // visit completes) and the number of the lane's current launch
    uint32_t *h_done = nullptr;
    uint32_t launch_seq = 0;
    // recon_batch with tasks of several block heights: one context per height
    // (its own workspace and graphs) whose launch runs on a stream forked from
    // the caller's; `last_shapes` (bit v) names those that ran the last batch
    recon_ctx *shape_ctx[kVariants] = {nullptr, nullptr, nullptr};
    hipStream_t shape_stream[kVariants] = {nullptr, nullptr, nullptr};
    hipEvent_t shape_join[kVariants] = {nullptr, nullptr, nullptr};
    hipEvent_t shape_fork = nullptr;
    unsigned last_shapes = 0;
};

namespace {

// Launch numbers, unique in the process and never 0 (the value of device
// memory never written): the device-side flags keyed by them, in a context's
// workspace or in the no-allocation entry point's, which every context on a
// device shares, never take one launch's value for another's.
std::atomic<uint32_t> g_launch_seq{0};
uint32_t next_launch_seq() {
    uint32_t v;
    do {
        v = g_launch_seq.fetch_add(1u, std::memory_order_relaxed) + 1u;
    } while (v == 0u);
    return v;
}

int ensure_device(recon_ctx *c) {
    HIP_TRY(hipSetDevice(c->device));
    return RECON_OK;
}

// Ring positions for a workspace of n_blocks blocks: every block is in the ring
// at most once, and each wave of the revisit grid may hold one ticket ahead.
size_t ring_slots(size_t n_blocks) { return n_blocks + rk::MAX_DRAIN_GRID + 1; }

int resident_wgs(recon_ctx *c, int v) {
    if (c->resident[v] == 0) {
        int per_cu = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, drain_fn(v), 64,
                                                                    lds_for(v, c->cfg.queue_capacity));
        if (e != hipSuccess || per_cu <= 0) per_cu = 1;
        if (c->cfg.wg_per_cu > 0) per_cu = std::min(per_cu, c->cfg.wg_per_cu);
        c->resident[v] = per_cu * c->cus;
    }
    return c->resident[v];
}

void free_workspace(recon_ctx *c) {
    (void)hipFree(c->d_table);
    (void)hipFree(c->d_work);
    (void)hipFree(c->d_state);
    (void)hipFree(c->d_ring);
    (void)hipFree(c->d_tile_pending);
    (void)hipFree(c->d_tile_done);
    (void)hipFree(c->d_route);
    (void)hipFree(c->d_spill);
    c->d_spill = nullptr;
    (void)hipFree(c->d_scratch);
    c->d_table = nullptr;
    c->d_work = nullptr;
    c->d_state = c->d_ring = c->d_tile_pending = c->d_tile_done = c->d_route = nullptr;
    c->d_scratch = nullptr;
    c->cap_tasks = c->cap_blocks = c->cap_scratch = 0;
}

void drop_graphs(recon_ctx *c) {
    for (int v = 0; v < kVariants; ++v) {
        if (c->graph[v]) (void)hipGraphExecDestroy(c->graph[v]);
        c->graph[v] = nullptr;
        c->graph_cap_blocks[v] = c->graph_cap_tasks[v] = c->graph_cap_scratch[v] = 0;
    }
}

// Grow the workspace to hold n_tasks tasks, n_blocks blocks and `area_bytes`
// bytes of scratch planes.  Growing synchronises the device and drops the
// captured graphs (they hold the old pointers).
int ensure_capacity(recon_ctx *c, size_t n_tasks, size_t n_blocks, size_t area_bytes) {
    if (n_tasks <= c->cap_tasks && n_blocks <= c->cap_blocks && area_bytes <= c->cap_scratch)
        return RECON_OK;
    HIP_TRY(hipDeviceSynchronize());
    drop_graphs(c);
    const size_t nt = std::max(c->cap_tasks, std::max<size_t>(n_tasks, 64));
    const size_t nb = std::max(c->cap_blocks, std::max<size_t>(n_blocks, 4096));
    const size_t ns = std::max(c->cap_scratch, area_bytes);
    free_workspace(c);
    const size_t table = sizeof(BatchHdr) + nt * sizeof(rk::TaskDev);
    if (hipMalloc(&c->d_table, table) != hipSuccess ||
        hipMalloc(&c->d_work, sizeof(rk::Work)) != hipSuccess ||
        hipMalloc(&c->d_state, nb * rk::STATE_STRIDE * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&c->d_ring, ring_slots(nb) * rk::RING_STRIDE * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&c->d_tile_pending, nt * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&c->d_tile_done, nt * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&c->d_route, rk::ROUTE_WORDS * nt * sizeof(uint32_t)) != hipSuccess ||
        (c->cfg.spill_capacity > 0 &&
         hipMalloc(&c->d_spill, (size_t)rk::MAX_DRAIN_GRID * c->cfg.spill_capacity * sizeof(uint16_t)) != hipSuccess) ||
        (ns > 0 && hipMalloc(&c->d_scratch, ns) != hipSuccess)) {
        free_workspace(c);
        return fail(RECON_ENOMEM, "workspace allocation (%zu tasks, %zu blocks, %zu scratch bytes) failed",
                    nt, nb, ns);
    }
    // the scheduler words start at 0: the flags keyed by a launch number must
    // not find a stale number that some earlier owner of this memory left
    HIP_TRY(hipMemset(c->d_work, 0, sizeof(rk::Work)));
    c->cap_tasks = nt;
    c->cap_blocks = nb;
    c->cap_scratch = ns;
    if (c->cap_h_table < table) {
        if (c->h_table) (void)hipHostFree(c->h_table);
        c->h_table = nullptr;
        if (hipHostMalloc((void **)&c->h_table, table, hipHostMallocDefault) != hipSuccess)
            return fail(RECON_ENOMEM, "pinned task table allocation failed");
        c->cap_h_table = table;
    }
    return RECON_OK;
}

int check_image(const recon_image *im, const char *what) {
    if (!im) return fail(RECON_EINVAL, "%s: null image", what);
    if (!im->data) return fail(RECON_EINVAL, "%s: null data pointer", what);
    if (im->height < 1 || im->width < 1)
        return fail(RECON_EINVAL, "%s: shape %dx%d is empty", what, im->height, im->width);
    if (im->pitch < im->width)
        return fail(RECON_EINVAL, "%s: pitch %lld < width %d", what, (long long)im->pitch, im->width);
    return RECON_OK;
}

bool overlaps(const recon_image &a, const recon_image &b) {
    const uintptr_t a0 = (uintptr_t)a.data, a1 = a0 + (uintptr_t)((a.height - 1) * a.pitch + a.width);
    const uintptr_t b0 = (uintptr_t)b.data, b1 = b0 + (uintptr_t)((b.height - 1) * b.pitch + b.width);
    return a0 < b1 && b0 < a1;
}

// ops whose marker and mask are two caller images (the others derive both from one)
bool two_planes(int op) { return op == RECON_OP_DILATE || op == RECON_OP_ERODE; }

int check_task(const recon_task &t, const recon_config *cfg = nullptr) {
    if (t.op < RECON_OP_DILATE || t.op > RECON_OP_REGIONAL_MAX)
        return fail(RECON_EINVAL, "unknown op %d", t.op);
    if (t.op == RECON_OP_HDOME && (t.h < 1 || t.h > 255))
        return fail(RECON_EINVAL, "h-dome height must be in 1..255, got %d", t.h);
    if (t.scan_rounds < -1 || t.scan_rounds > 8) return fail(RECON_EINVAL, "task scan_rounds must be in -1..8");
    if (t.queue_capacity != 0 &&
        (t.queue_capacity < 64 || (cfg && t.queue_capacity > cfg->queue_capacity) ||
         (t.queue_capacity & (t.queue_capacity - 1)) != 0))
        return fail(RECON_EINVAL, "task queue_capacity must be a power of two in 64..%d",
                    cfg ? cfg->queue_capacity : 8192);
    if (t.conn != 4 && t.conn != 8) return fail(RECON_EINVAL, "conn must be 4 or 8, got %d", t.conn);
    if (t.block_rows != 0 && variant_of(t.block_rows) < 0)
        return fail(RECON_EINVAL, "task block_rows must be 0, 16, 32 or 64, got %d", t.block_rows);
    int rc = check_image(&t.image, two_planes(t.op) ? "marker" : "image");
    if (rc) return rc;
    if (two_planes(t.op)) {
        rc = check_image(&t.mask, "mask");
        if (rc) return rc;
        if (t.mask.height != t.image.height || t.mask.width != t.image.width)
            return fail(RECON_EINVAL, "marker %dx%d and mask %dx%d differ in shape", t.image.height,
                        t.image.width, t.mask.height, t.mask.width);
        if (overlaps(t.image, t.mask)) return fail(RECON_EINVAL, "marker and mask overlap");
    }
    return RECON_OK;
}

bool aligned4(const void *p, int64_t pitch) { return ((uintptr_t)p % 4 == 0) && (pitch % 4 == 0); }

// Host-side task table for `n` tasks (fill scratch planes as offsets, patched later).
// Device task table of a launch.  Tasks that need a scratch marker plane get
// its offset into the context's scratch area in `j` (relocated by the caller
// once the area is allocated) and uses_scratch[k] = 1.
// With `with_route`, every task whose node ids fit also gets an int32 label
// plane for the component route (its offset in lab_off, else SIZE_MAX).
void build_table(const recon_config &cfg, const recon_task *tasks, int n, int bh, std::vector<rk::TaskDev> &out,
                 std::vector<char> &uses_scratch, uint32_t &total_blocks, size_t &scratch_bytes,
                 bool &any_mapped, bool with_route, std::vector<size_t> &lab_off) {
    out.resize(n);
    uses_scratch.assign(n, 0);
    lab_off.assign(n, SIZE_MAX);
    total_blocks = 0;
    scratch_bytes = 0;
    any_mapped = false;
    for (int k = 0; k < n; ++k) {
        const recon_task &t = tasks[k];
        rk::TaskDev d{};
        d.h = t.image.height;
        d.w = t.image.width;
        d.conn = t.conn;
        d.nby = (d.h + bh - 1) / bh;
        d.nbx = (d.w + rk::BW - 1) / rk::BW;
        d.block0 = total_blocks;
        total_blocks += (uint32_t)(d.nby * d.nbx);
        d.scan_rounds = t.scan_rounds == 0 ? cfg.scan_rounds : (t.scan_rounds < 0 ? 0 : t.scan_rounds);
        d.qcap = t.queue_capacity == 0 ? cfg.queue_capacity : t.queue_capacity;
        d.minv = (t.op == RECON_OP_FILL_HOLES || t.op == RECON_OP_ERODE) ? 1 : 0;
        d.hval = t.op == RECON_OP_HDOME ? t.h : (t.op == RECON_OP_REGIONAL_MAX ? 1 : 0);
        if (two_planes(t.op)) {
            // marker in place in the caller's plane (erosion complements it
            // before and after the reconstruction)
            d.op = t.op == RECON_OP_DILATE ? rk::OP_DILATE : rk::OP_ERODE;
            d.j = t.image.data;
            d.pitch_j = t.image.pitch;
            d.i = t.mask.data;
            d.pitch_i = t.mask.pitch;
            d.img = t.op == RECON_OP_DILATE ? nullptr : t.image.data;
            d.pitch_img = t.image.pitch;
            d.aligned = aligned4(d.j, d.pitch_j) && aligned4(d.i, d.pitch_i);
        } else {
            d.op = t.op == RECON_OP_FILL_HOLES ? rk::OP_FILL : (t.op == RECON_OP_HDOME ? rk::OP_HDOME : rk::OP_RMAX);
            d.i = t.image.data;
            d.pitch_i = t.image.pitch;
            d.img = t.image.data;
            d.pitch_img = t.image.pitch;
            d.pitch_j = (int64_t)round_up((size_t)d.w, 4);
            d.j = (uint8_t *)(uintptr_t)scratch_bytes;   // offset into the scratch area
            scratch_bytes += round_up((size_t)d.pitch_j * d.h, 256);
            d.aligned = aligned4(d.i, d.pitch_i);
            uses_scratch[k] = 1;
        }
        if (t.op != RECON_OP_DILATE) any_mapped = true;
        d.lab = nullptr;
        d.pitch_lab = (int64_t)round_up((size_t)d.w, 4);
        if (with_route && (uint64_t)d.h * (uint64_t)d.pitch_lab < (uint64_t)rk::COMP_ENC) {
            lab_off[k] = scratch_bytes;
            scratch_bytes += round_up((size_t)d.pitch_lab * d.h * 4, 256);
        }
        out[k] = d;
    }
}

// The scheduler workspace a launch runs on: the context's (allocated by
// ensure_capacity) or the fixed device array of recon_dilate_noalloc.
struct Workspace {
    rk::Work *work;
    uint32_t *state;
    uint32_t *ring;
    uint32_t *tile_pending;
    uint32_t *tile_done;
    uint32_t *route;     // mask classification words (null: no task takes the component route)
    uint16_t *spill;     // spill queues, MAX_DRAIN_GRID x spill_cap entries (null: none)
    size_t cap_blocks;   // blocks the state words and the ring hold
};

Workspace ctx_workspace(const recon_ctx *c) {
    return Workspace{c->d_work, c->d_state, c->d_ring, c->d_tile_pending, c->d_tile_done, c->d_route,
                     c->d_spill, c->cap_blocks};
}

// Enqueue the kernels of one launch sequence on `s`.
int enqueue_kernels(recon_ctx *c, const Workspace &ws, int v, const rk::TaskTable &tt, uint32_t total_blocks,
                    uint32_t n_tasks_host, bool any_mapped, bool route, bool dynamic_sizes, hipStream_t s) {
    if (route && dynamic_sizes && !c->aux_stream) {
        HIP_TRY(hipStreamCreateWithFlags(&c->aux_stream, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
        HIP_TRY(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
    }
    rk::KArgs ka;
    ka.work = ws.work;
    ka.state = ws.state;
    ka.ring = ws.ring;
    ka.tile_pending = ws.tile_pending;
    ka.tile_done = ws.tile_done;
    ka.qcap = c->cfg.queue_capacity;
    ka.scan_rounds = c->cfg.scan_rounds;
    ka.watchdog_ticks = c->watchdog_ticks;
    ka.drain_budget = c->cfg.drain_budget;
    ka.binary_drain_budget = c->cfg.binary_drain_budget;
    ka.test_fault = c->cfg.test_fault;
    ka.route = route ? ws.route : nullptr;
    ka.route_policy = c->cfg.component_route == 1 ? 1 : 0;
    ka.spill = ws.spill;
    ka.spill_cap = ws.spill ? (uint32_t)c->cfg.spill_capacity : 0u;
    ka.launch_seq = c->launch_seq;
    ka.host_done = dynamic_sizes ? nullptr : c->h_done;   // (never inside a captured graph)
    const size_t lds = lds_for(v, c->cfg.queue_capacity);
    const int resident = resident_wgs(c, v);
    // K1/K2 are grid-stride: with sizes known only on the device (captured
    // graphs), launch enough workgroups for the largest batch the workspace holds.
    const uint32_t nblk = dynamic_sizes ? (uint32_t)ws.cap_blocks : total_blocks;
    const int grid12 = (int)std::max<uint32_t>(1u, std::min<uint32_t>(nblk, 65535u));
    const int grid3 = std::max(1, std::min<int>(std::min(resident, rk::MAX_DRAIN_GRID),
                                                (int)std::max<uint32_t>(1u, nblk)));
    const int stop = c->cfg.stop_after_stage;
    // per-kernel timing marks on plain launches only: events recorded inside a
    // captured graph cannot be timed (a graph launch is timed as a whole)
    const bool timing = c->cfg.timing != 0 && !dynamic_sizes;
    // stop 0: the persistent pipeline (every block's first visit inside the
    // revisit kernel); 1-3: the staged pipeline (dense pass, border seeding,
    // revisits as separate kernels), stopped after that stage (test hooks)
    const bool merged = stop == 0;
    hipEvent_t *tev = c->tev[c->launches % kTimingRing];
    c->tev_route[c->launches % kTimingRing] = route;
    c->tev_merged[c->launches % kTimingRing] = merged;
    if (timing) HIP_TRY(hipEventRecord(tev[5], s));
    const int reset_mode = !merged ? rk::RESET_STAGED : (route ? rk::RESET_ROUTE : rk::RESET_QUEUE_ALL);
    hipLaunchKernelGGL(rk::reset_work, dim3(64), dim3(256), 0, s, tt, ka, reset_mode);
    // (a mark between two kernels costs the gap of its own packet: the
    // persistent pipeline marks only the revisit kernel, the route's end and
    // the launch; the staged one every stage)
    if (timing && !merged) HIP_TRY(hipEventRecord(tev[0], s));
    // the stream of the block route's kernels: with the component route, a
    // second stream forked after the classification
    hipStream_t d = s;
    if (route) {
        // the component route: classify every task's mask (unless the samples
        // reset_work took already decided every route), then label and
        // reconstruct the two-valued ones (the others' waves exit at once)
        const int bh = kBlockRows[v];
        const int g_rows = (int)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)nblk * bh, 4096));
        const int g_tiles = (int)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)nblk * (bh / rk::LT_H), 4096));
        const size_t lds_lab = (size_t)rk::LT_H * rk::LT_W * sizeof(uint32_t);
#define RK_COMP(K, GRID, LDS)                                                                     \
    switch (v) {                                                                                  \
        case 0: hipLaunchKernelGGL(rk::K<16>, dim3(GRID), dim3(64), LDS, s, tt, ka); break;      \
        case 1: hipLaunchKernelGGL(rk::K<32>, dim3(GRID), dim3(64), LDS, s, tt, ka); break;      \
        default: hipLaunchKernelGGL(rk::K<64>, dim3(GRID), dim3(64), LDS, s, tt, ka); break;     \
    }
        RK_COMP(comp_classify, (int)std::max<uint32_t>(1u, std::min<uint32_t>(nblk, 1024u)), 0);
        // A large batch (a replayed graph) forks: the ring and marker planes
        // (prepare) and the revisit kernel of the tasks that keep the block
        // route go to the second stream, while the route's labelling and
        // maxima stay on this one, so that the route's work runs beside the
        // revisit kernel (which leaves most compute units idle on
        // latency-bound tiles).  The route's kernels are dispatched first:
        // they need LDS (comp_label_local) that the persistent revisit kernel
        // would otherwise hold until it ends.  A direct launch (at most 12
        // tasks) runs everything on one stream: the route's kernels first
        // (when no task takes the route they return at once), then the block
        // route; the fork and join each cost more than that.
        if (dynamic_sizes) {
            HIP_TRY(hipEventRecord(c->ev_fork, s));
            HIP_TRY(hipStreamWaitEvent(c->aux_stream, c->ev_fork, 0));
            d = c->aux_stream;
        }
        RK_COMP(comp_label_local, g_tiles, lds_lab);
        RK_COMP(comp_label_merge, g_tiles, 0);
        RK_COMP(comp_flatten_max, g_rows, 0);
        RK_COMP(comp_write, g_rows, 0);
#undef RK_COMP
        if (timing) HIP_TRY(hipEventRecord(tev[6], s));
        hipLaunchKernelGGL(rk::prepare, dim3(1024), dim3(256), 0, d, tt, ka, any_mapped ? 1 : 0);
    } else if (any_mapped) {
        hipLaunchKernelGGL(rk::init_marker, dim3(1024), dim3(256), 0, s, tt, ka.route);
    }
    if (timing && !route && !merged) HIP_TRY(hipEventRecord(tev[6], s));
#define RK_LAUNCH(K, GRID)                                                                        \
    switch (v) {                                                                                  \
        case 0: hipLaunchKernelGGL(rk::K<16>, dim3(GRID), dim3(64), lds, d, tt, ka); break;      \
        case 1: hipLaunchKernelGGL(rk::K<32>, dim3(GRID), dim3(64), lds, d, tt, ka); break;      \
        default: hipLaunchKernelGGL(rk::K<64>, dim3(GRID), dim3(64), lds, d, tt, ka); break;     \
    }
    if (!merged) RK_LAUNCH(dense_pass, grid12);
    if (timing && !merged) HIP_TRY(hipEventRecord(tev[1], d));
    if (stop >= 2) RK_LAUNCH(border_seed, grid12);
    if (timing) HIP_TRY(hipEventRecord(tev[2], d));
    if (merged || stop >= 3) RK_LAUNCH(revisit_drain, grid3);
    if (timing) HIP_TRY(hipEventRecord(tev[3], d));
#undef RK_LAUNCH
    if (d != s) {   // join the block route's stream
        HIP_TRY(hipEventRecord(c->ev_join, d));
        HIP_TRY(hipStreamWaitEvent(s, c->ev_join, 0));
    }
    if (any_mapped) hipLaunchKernelGGL(rk::finish_result, dim3(1024), dim3(256), 0, s, tt, ka.route);
    if (timing) HIP_TRY(hipEventRecord(tev[4], s));
    HIP_TRY(hipGetLastError());
    return RECON_OK;
}

// Enqueue one launch sequence for `tasks` on `stream`.  use_graph replays the
// context's captured graph for the block shape (the task table then always
// lives in device memory).
int run_tasks(recon_ctx *c, const recon_task *tasks, int n, hipStream_t stream, bool use_graph) {
    int rc = ensure_device(c);
    if (rc) return rc;
    const int bh = c->cfg.block_rows;
    const int v = variant_of(bh);
    std::vector<rk::TaskDev> table;
    std::vector<char> uses_scratch;
    std::vector<size_t> lab_off;
    uint32_t total_blocks = 0;
    size_t scratch_need = 0;
    bool any_mapped = false;
    const bool with_route = c->cfg.component_route >= 0 && c->cfg.stop_after_stage == 0;
    build_table(c->cfg, tasks, n, bh, table, uses_scratch, total_blocks, scratch_need, any_mapped, with_route,
                lab_off);
    rc = ensure_capacity(c, (size_t)n, (size_t)total_blocks, scratch_need);
    if (rc) return rc;
    for (int k = 0; k < n; ++k) {
        rk::TaskDev &d = table[k];
        if (uses_scratch[k]) {
            d.j = c->d_scratch + (uintptr_t)d.j;
            if (!aligned4(d.j, d.pitch_j)) d.aligned = 0;
        }
        if (lab_off[k] != SIZE_MAX) d.lab = (int32_t *)(c->d_scratch + lab_off[k]);
    }

    c->launch_seq = next_launch_seq();   // numbers the launch (serving lanes: the value the kernel reports per task)
    rk::TaskTable tt{};
    const bool inline_table = !use_graph && n <= rk::MAX_INLINE_TASKS;
    if (inline_table) {
        tt.hdr = nullptr;
        tt.ext = nullptr;
        tt.n_inline = (uint32_t)n;
        tt.total_inline = total_blocks;
        tt.ring_cap_inline = (uint32_t)ring_slots(c->cap_blocks);
        tt.seq_inline = c->launch_seq;
        for (int k = 0; k < n; ++k) tt.inl[k] = table[k];
    } else {
        tt.hdr = (const BatchHdr *)c->d_table;
        tt.ext = (const rk::TaskDev *)(c->d_table + sizeof(BatchHdr));
        // stage the table in pinned memory once the previous copy out of it is done
        rc = wait_event(c->table_used, 60.0, "the previous task-table copy");
        if (rc) return rc;
        BatchHdr hdr{};
        hdr.n_tasks = (uint32_t)n;
        hdr.total_blocks = total_blocks;
        hdr.ring_cap = (uint32_t)ring_slots(c->cap_blocks);
        hdr.any_mapped = any_mapped ? 1u : 0u;
        hdr.launch_seq = c->launch_seq;
        std::memcpy(c->h_table, &hdr, sizeof(hdr));
        std::memcpy(c->h_table + sizeof(hdr), table.data(), table.size() * sizeof(rk::TaskDev));
    }
    const uint32_t table_bytes = (uint32_t)(sizeof(BatchHdr) + table.size() * sizeof(rk::TaskDev));

    if (use_graph) {
        if (!c->graph[v] || c->graph_cap_blocks[v] != c->cap_blocks || c->graph_cap_tasks[v] != c->cap_tasks ||
            c->graph_cap_scratch[v] != c->cap_scratch) {
            if (c->graph[v]) (void)hipGraphExecDestroy(c->graph[v]);
            c->graph[v] = nullptr;
            if (!c->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
            hipGraph_t g = nullptr;
            HIP_TRY(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
            const uint32_t max_bytes = (uint32_t)(sizeof(BatchHdr) + c->cap_tasks * sizeof(rk::TaskDev));
            hipLaunchKernelGGL(rk::copy_table, dim3(16), dim3(256), 0, c->cap_stream, c->h_table, c->d_table,
                               max_bytes);
            rc = enqueue_kernels(c, ctx_workspace(c), v, tt, total_blocks, (uint32_t)n, true, with_route, true,
                                 c->cap_stream);
            hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
            if (rc) return rc;
            if (e != hipSuccess) return fail(RECON_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
            e = hipGraphInstantiate(&c->graph[v], g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) return fail(RECON_EDEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
            c->graph_cap_blocks[v] = c->cap_blocks;
            c->graph_cap_tasks[v] = c->cap_tasks;
            c->graph_cap_scratch[v] = c->cap_scratch;
        }
        hipEvent_t *tev = c->tev[c->launches % kTimingRing];
        if (c->cfg.timing) HIP_TRY(hipEventRecord(tev[5], stream));
        HIP_TRY(hipGraphLaunch(c->graph[v], stream));
        if (c->cfg.timing) HIP_TRY(hipEventRecord(tev[4], stream));
        HIP_TRY(hipEventRecord(c->table_used, stream));
    } else {
        if (!inline_table) {
            hipLaunchKernelGGL(rk::copy_table, dim3(16), dim3(256), 0, stream, c->h_table, c->d_table,
                               table_bytes);
            HIP_TRY(hipEventRecord(c->table_used, stream));
        }
        rc = enqueue_kernels(c, ctx_workspace(c), v, tt, total_blocks, (uint32_t)n, any_mapped, with_route, false,
                             stream);
        if (rc) return rc;
    }
    HIP_TRY(hipEventRecord(c->last_done, stream));
    c->have_last = true;
    c->last_work = c->d_work;
    c->last_was_graph = use_graph;
    c->tev_graph[c->launches % kTimingRing] = use_graph;
    c->launches += 1;
    return RECON_OK;
}

// Run the self-test kernel: it writes into pinned host memory, which the host
// checks once the kernel's event has completed (within `seconds`).
int self_test(double seconds) {
    const uint32_t n = 1024;
    uint32_t *h = nullptr;
    hipEvent_t ev = nullptr;
    if (hipHostMalloc((void **)&h, 4 * n * sizeof(uint32_t), hipHostMallocDefault) != hipSuccess)
        return fail(RECON_ENOMEM, "self-test pinned allocation failed");
    std::memset(h, 0, 4 * n * sizeof(uint32_t));
    int rc = RECON_OK;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        rc = fail(RECON_EDEVICE, "self-test event creation failed");
    } else {
        hipLaunchKernelGGL(rk::self_test, dim3((n + 255) / 256), dim3(256), 0, nullptr, h, n);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) rc = fail(RECON_EDEVICE, "self-test launch failed: %s", hipGetErrorString(e));
        else if (hipEventRecord(ev, nullptr) != hipSuccess) rc = fail(RECON_EDEVICE, "self-test event record failed");
        else rc = wait_event(ev, seconds, "the self-test kernel");
        const volatile uint32_t *v = h;
        if (rc == RECON_OK)
            for (uint32_t i = 0; i < n; ++i) {
                const uint32_t lane = i % 64u;
                const uint32_t want_lo = lane > 0 ? i - 1u + 100u : 0u;
                const uint32_t want_hi = lane < 63 ? i + 1u + 100u : 0u;
                if (v[i] != i * 3u + 1u || v[n + i] != want_lo || v[2 * n + i] != want_hi) {
                    rc = fail(RECON_EDEVICE,
                              "self-test mismatch at %u: wrote %u/%u/%u, expected %u/%u/%u (lane shifts)", i,
                              v[i], v[n + i], v[2 * n + i], i * 3u + 1u, want_lo, want_hi);
                    break;
                }
            }
        // row closure: each wave closes one row of 256 pixels; check it pixel by
        // pixel against the two sequential scans
        for (uint32_t w = 0; rc == RECON_OK && w < n / 64u; ++w) {
            uint32_t lo[256], hi[256], lr[256];
            for (uint32_t x = 0; x < 256; ++x) {
                hi[x] = rk::self_test_mask(256u * w + x);
                lo[x] = rk::self_test_low(256u * w + x, hi[x]);
            }
            uint32_t u = (w * 37u) & 255u;
            for (uint32_t x = 0; x < 256; ++x) lr[x] = u = std::min(std::max(u, lo[x]), hi[x]);
            u = (w * 91u + 7u) & 255u;
            for (int x = 255; x >= 0; --x) {
                u = std::min(std::max(u, lo[x]), hi[x]);
                const uint32_t want = std::max(lr[x], u);
                const uint32_t got = (v[3 * n + 64u * w + (uint32_t)x / 4u] >> (8 * (x % 4))) & 0xffu;
                if (got != want) {
                    rc = fail(RECON_EDEVICE, "self-test mismatch in the row closure: row %u pixel %d is %u, "
                              "expected %u (DPP row moves)", w, x, got, want);
                    break;
                }
            }
        }
        if (rc != RECON_ETIMEDOUT) (void)hipEventDestroy(ev);
    }
    if (rc != RECON_ETIMEDOUT) (void)hipHostFree(h);   // never free memory a live kernel may write
    return rc == RECON_ETIMEDOUT ? RECON_EDEVICE : rc;
}

// Allocate a context (no self-test): events, pinned statistics buffer, watchdog.
int make_ctx(recon_ctx **out, int device, const recon_config &c) {
    recon_ctx *ctx = new recon_ctx();
    ctx->device = device;
    ctx->cfg = c;
    if (hipDeviceGetAttribute(&ctx->cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->table_used, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->last_done, hipEventDisableTiming) != hipSuccess ||
        hipHostMalloc((void **)&ctx->h_work, sizeof(rk::Work), hipHostMallocDefault) != hipSuccess) {
        delete ctx;
        return fail(RECON_EDEVICE, "device query / event / pinned allocation failed");
    }
    if (c.timing)
        for (auto &set : ctx->tev)
            for (auto &ev : set)
                if (hipEventCreate(&ev) != hipSuccess) {
                    delete ctx;
                    return fail(RECON_EDEVICE, "timing event creation failed");
                }
    int clock_khz = 0;
    if (hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, device) != hipSuccess || clock_khz <= 0)
        clock_khz = 100000;
    ctx->watchdog_ticks = (uint64_t)clock_khz * 1000ull * 8ull;   // 8 s without progress
    // the table event must be "complete" before its first use
    if (hipEventRecord(ctx->table_used, nullptr) != hipSuccess) {
        delete ctx;
        return fail(RECON_EDEVICE, "event record failed");
    }
    *out = ctx;
    return RECON_OK;
}

// recon_batch of tasks with several block heights: each height's tasks run
// as one launch sequence on that height's context, on a stream forked from
// `stream`; `stream` waits for every group.  The call is timed as a whole on
// the caller's context (a launch whose only mark is its total).
int run_shape_groups(recon_ctx *c, const recon_task *tasks, int n, unsigned shapes, hipStream_t stream) {
    int rc = ensure_device(c);
    if (rc) return rc;
    if (!c->shape_fork) HIP_TRY(hipEventCreateWithFlags(&c->shape_fork, hipEventDisableTiming));
    const int v_ctx = variant_of(c->cfg.block_rows);
    std::vector<recon_task> group[kVariants];
    for (int k = 0; k < n; ++k)
        group[tasks[k].block_rows ? variant_of(tasks[k].block_rows) : v_ctx].push_back(tasks[k]);
    for (int v = 0; v < kVariants; ++v) {
        if (!(shapes & (1u << v)) || c->shape_ctx[v]) continue;
        recon_config cfg = c->cfg;
        cfg.block_rows = kBlockRows[v];
        cfg.timing = 0;
        rc = make_ctx(&c->shape_ctx[v], c->device, cfg);
        if (rc) return rc;
        c->shape_ctx[v]->noalloc = c->noalloc;
        if (hipStreamCreateWithFlags(&c->shape_stream[v], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&c->shape_join[v], hipEventDisableTiming) != hipSuccess)
            return fail(RECON_EDEVICE, "stream / event creation for block height %d failed", kBlockRows[v]);
    }
    hipEvent_t *tev = c->tev[c->launches % kTimingRing];
    if (c->cfg.timing) HIP_TRY(hipEventRecord(tev[5], stream));
    HIP_TRY(hipEventRecord(c->shape_fork, stream));
    for (int v = 0; v < kVariants; ++v) {
        if (!(shapes & (1u << v))) continue;
        HIP_TRY(hipStreamWaitEvent(c->shape_stream[v], c->shape_fork, 0));
        const int m = (int)group[v].size();
        rc = run_tasks(c->shape_ctx[v], group[v].data(), m, c->shape_stream[v], m > rk::MAX_INLINE_TASKS);
        if (rc) return rc;
        HIP_TRY(hipEventRecord(c->shape_join[v], c->shape_stream[v]));
        HIP_TRY(hipStreamWaitEvent(stream, c->shape_join[v], 0));
    }
    if (c->cfg.timing) HIP_TRY(hipEventRecord(tev[4], stream));
    HIP_TRY(hipEventRecord(c->last_done, stream));
    c->have_last = true;
    c->last_work = nullptr;
    c->last_shapes = shapes;
    c->last_was_graph = true;
    c->tev_graph[c->launches % kTimingRing] = true;
    c->launches += 1;
    return RECON_OK;
}

// Device bytes a serving request holds while admitted: its images, its scratch
// marker plane and, with the component route, its label plane.
size_t task_bytes(const recon_task &t, const recon_config &cfg) {
    size_t b = (size_t)t.image.height * (size_t)t.image.pitch;
    if (two_planes(t.op)) b += (size_t)t.mask.height * (size_t)t.mask.pitch;
    else b += round_up((size_t)round_up((size_t)t.image.width, 4) * t.image.height, 256);
    if (cfg.component_route >= 0) b += round_up(round_up((size_t)t.image.width, 4) * t.image.height * 4, 256);
    return b;
}

}  // namespace

// ============================================================================
// Serving: a request loop that admits tasks by device memory and slots and runs
// them as continuous batches.  A worker thread owns `kLanes` lanes, each a
// private context (its own scheduler workspace, kept resident) with its own
// stream.  Whenever a lane is free and requests are waiting, the lane takes
// every waiting request (up to its batch limit) and launches the pipeline on
// them; lanes run concurrently, so requests admitted while others are on the
// GPU start as soon as a lane frees up and overlap with the work in flight.
struct recon_ctx::Serve {
    static constexpr int kLanes = 3;
    static constexpr int kMaxPerLaunch = 64;
    struct Req {
        uint64_t ticket;
        recon_task task;
        size_t bytes;
        bool finished = false;   // completed before its launch ended (its own tile converged)
    };
    struct Lane {
        recon_ctx *sub = nullptr;
        hipStream_t stream = nullptr;
        hipEvent_t done = nullptr;
        std::vector<Req> reqs;
        uint32_t seq = 0;        // the launch number its tasks' completion words will show
        bool busy = false;
    };
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Req> waiting;
    std::unordered_map<uint64_t, int> status;   // 0 waiting, 1 running, 2 done, -1 failed
    uint64_t next_ticket = 1;
    size_t bytes_admitted = 0;
    size_t bytes_fixed = 0;      // the lanes' own resident workspace, counted against the cap
    int slots_admitted = 0;
    recon_serve_counters stats{};
    bool stop = false;
    int error = RECON_OK;
    std::string error_msg;
    Lane lanes[kLanes];
    std::thread worker;
    int device = 0;
};

namespace {

void serve_loop(recon_ctx *ctx) {
    recon_ctx::Serve *S = ctx->serve;
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    while (true) {
        bool any_busy = false;
        // harvest finished lanes, and single tasks that finished inside a running launch
        for (auto &L : S->lanes) {
            if (!L.busy) continue;
            const hipError_t q = hipEventQuery(L.done);
            if (q == hipErrorNotReady) {
                any_busy = true;
                const volatile uint32_t *hd = L.sub->h_done;
                for (size_t i = 0; i < L.reqs.size(); ++i) {
                    recon_ctx::Serve::Req &r = L.reqs[i];
                    // a reconstruction by dilation is complete when its last visit
                    // is (other operations still map their result at the end)
                    if (r.finished || r.task.op != RECON_OP_DILATE || hd[i] != L.seq) continue;
                    r.finished = true;
                    S->status[r.ticket] = 2;
                    S->bytes_admitted -= r.bytes;
                    S->slots_admitted -= 1;
                    S->stats.early_completions += 1;
                    S->cv_done.notify_all();
                }
                continue;
            }
            // the launch's counters were copied into the lane's pinned buffer
            // ahead of its completion event: a launch its watchdog gave up
            // fails every request it had not completed
            const bool gave_up = q == hipSuccess && L.sub->h_work->abort != 0;
            const int st = q == hipSuccess && !gave_up ? 2 : -1;
            if (q != hipSuccess) {
                S->error = RECON_EDEVICE;
                S->error_msg = std::string("serving launch failed: ") + hipGetErrorString(q);
            } else if (gave_up) {
                S->error = RECON_EDEVICE;
                S->error_msg = "serving launch: scheduler watchdog expired, the launch did not converge";
            }
            for (auto &r : L.reqs) {
                // completed already (its tile's last visit was done and its
                // status handed out, perhaps taken by a wait)
                if (r.finished) continue;
                S->status[r.ticket] = st;
                S->bytes_admitted -= r.bytes;
                S->slots_admitted -= 1;
            }
            L.reqs.clear();
            L.busy = false;
            S->cv_done.notify_all();
        }
        // launch waiting requests on free lanes
        for (auto &L : S->lanes) {
            if (L.busy || S->waiting.empty()) continue;
            std::vector<recon_task> tasks;
            while (!S->waiting.empty() && (int)L.reqs.size() < recon_ctx::Serve::kMaxPerLaunch) {
                L.reqs.push_back(S->waiting.front());
                S->waiting.pop_front();
            }
            for (auto &r : L.reqs) {
                tasks.push_back(r.task);
                S->status[r.ticket] = 1;
            }
            int rc = run_tasks(L.sub, tasks.data(), (int)tasks.size(), L.stream, false);
            L.seq = L.sub->launch_seq;
            if (rc == RECON_OK) {
                hipLaunchKernelGGL(rk::copy_table, dim3(1), dim3(64), 0, L.stream, (const uint8_t *)L.sub->last_work,
                                   (uint8_t *)L.sub->h_work, (uint32_t)sizeof(rk::Work));
                if (hipGetLastError() != hipSuccess || hipEventRecord(L.done, L.stream) != hipSuccess)
                    rc = RECON_EDEVICE;
            }
            if (rc != RECON_OK) {
                S->error = rc;
                S->error_msg = g_err;
                for (auto &r : L.reqs) {
                    S->status[r.ticket] = -1;
                    S->bytes_admitted -= r.bytes;
                    S->slots_admitted -= 1;
                }
                L.reqs.clear();
                S->cv_done.notify_all();
                continue;
            }
            L.busy = true;
            any_busy = true;
            S->stats.launches += 1;
            S->stats.requests += (int64_t)L.reqs.size();
            S->stats.max_batch = std::max<int64_t>(S->stats.max_batch, (int64_t)L.reqs.size());
        }
        int busy_now = 0;
        for (auto &L : S->lanes) busy_now += L.busy ? 1 : 0;
        S->stats.max_busy_lanes = std::max<int64_t>(S->stats.max_busy_lanes, busy_now);
        if (S->stop && S->waiting.empty() && !any_busy) break;
        if (any_busy)
            S->cv_work.wait_for(lk, std::chrono::microseconds(20));
        else
            S->cv_work.wait_for(lk, std::chrono::milliseconds(5));
    }
}

int serve_start(recon_ctx *ctx) {
    if (ctx->serve) return RECON_OK;
    auto *S = new recon_ctx::Serve();
    S->device = ctx->device;
    recon_config c = ctx->cfg;
    c.timing = 0;
    for (auto &L : S->lanes) {
        int rc = make_ctx(&L.sub, ctx->device, c);
        if (rc == RECON_OK) {
            L.sub->is_lane = true;
            if (hipHostMalloc((void **)&L.sub->h_done, recon_ctx::Serve::kMaxPerLaunch * sizeof(uint32_t),
                              hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess)
                rc = fail(RECON_ENOMEM, "serving lane completion words: pinned allocation failed");
            else
                std::memset(L.sub->h_done, 0, recon_ctx::Serve::kMaxPerLaunch * sizeof(uint32_t));
        }
        if (rc == RECON_OK) {
            if (hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&L.done, hipEventDisableTiming) != hipSuccess)
                rc = fail(RECON_EDEVICE, "serving lane stream/event creation failed");
        }
        if (rc != RECON_OK) {
            for (auto &M : S->lanes) {
                if (M.sub) recon_destroy(M.sub);
                if (M.stream) (void)hipStreamDestroy(M.stream);
                if (M.done) (void)hipEventDestroy(M.done);
            }
            delete S;
            return rc;
        }
    }
    // the lanes' resident workspace (spill queues, scheduler state for the
    // largest launch) counts against the admission cap too
    S->bytes_fixed = (size_t)recon_ctx::Serve::kLanes *
                     ((size_t)rk::MAX_DRAIN_GRID * (size_t)std::max(0, c.spill_capacity) * sizeof(uint16_t) +
                      ((size_t)4096 + (size_t)rk::MAX_DRAIN_GRID) * 256);
    ctx->serve = S;
    S->worker = std::thread(serve_loop, ctx);
    return RECON_OK;
}

}  // namespace

extern "C" {

const char *recon_last_error(void) { return g_err.c_str(); }

int recon_create(recon_ctx **out, int device, const recon_config *cfg) {
    if (!out) return fail(RECON_EINVAL, "null output pointer");
    *out = nullptr;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev == 0) return fail(RECON_EDEVICE, "no HIP device available");
    if (device < 0 || device >= ndev) return fail(RECON_EINVAL, "device %d out of range (%d devices)", device, ndev);
    recon_config c{};
    if (cfg) c = *cfg;
    if (c.block_rows == 0) c.block_rows = 32;
    if (variant_of(c.block_rows) < 0) return fail(RECON_EINVAL, "block_rows must be 16, 32 or 64");
    if (c.queue_capacity == 0) c.queue_capacity = 2048;
    if (c.queue_capacity < 64 || c.queue_capacity > 8192 || (c.queue_capacity & (c.queue_capacity - 1)) != 0)
        return fail(RECON_EINVAL, "queue_capacity must be a power of two in 64..8192");
    if (c.scan_rounds < -1 || c.scan_rounds > 8) return fail(RECON_EINVAL, "scan_rounds must be in -1..8");
    if (c.drain_budget == 0) c.drain_budget = 128;
    if (c.binary_drain_budget == 0) c.binary_drain_budget = 4;
    if (c.drain_budget < 1 || c.drain_budget > 4096 || c.binary_drain_budget < 1 || c.binary_drain_budget > 4096)
        return fail(RECON_EINVAL, "drain_budget and binary_drain_budget must be in 1..4096");
    if (c.scan_rounds == 0) c.scan_rounds = 3;
    if (c.scan_rounds < 0) c.scan_rounds = 0;
    if (c.wg_per_cu < 0) return fail(RECON_EINVAL, "wg_per_cu must be >= 0");
    if (c.stop_after_stage < 0 || c.stop_after_stage > 3) return fail(RECON_EINVAL, "stop_after_stage must be 0..3");
    if (c.test_fault < 0 || c.test_fault > 1) return fail(RECON_EINVAL, "test_fault must be 0 or 1");
    if (c.spill_capacity == 0) c.spill_capacity = 8192;
    if (c.spill_capacity < -1 || (c.spill_capacity > 0 && (c.spill_capacity < 64 || c.spill_capacity > 65536)))
        return fail(RECON_EINVAL, "spill_capacity must be -1 (none), 0 (default 8192) or 64..65536");
    if (c.spill_capacity < 0) c.spill_capacity = 0;
    if (c.component_route < -1 || c.component_route > 1)
        return fail(RECON_EINVAL, "component_route must be 0 (where it pays), 1 (every two-valued mask) or -1 (off)");
    if (c.serve_mem_cap < 0 || c.serve_slots < 0) return fail(RECON_EINVAL, "serving limits must be >= 0");
    if (c.serve_mem_cap == 0) c.serve_mem_cap = (int64_t)64 << 30;
    if (c.serve_slots == 0) c.serve_slots = 256;
    e = hipSetDevice(device);
    if (e != hipSuccess) return fail(RECON_EDEVICE, "hipSetDevice failed: %s", hipGetErrorString(e));
    // once per device, with it current: the self-test, and the address of this
    // device's copy of the fixed workspace
    static std::mutex tested_mu;
    static std::vector<int> tested;
    static std::unordered_map<int, uint8_t *> noalloc_ptr;
    uint8_t *fixed = nullptr;
    {
        std::lock_guard<std::mutex> lk(tested_mu);
        if (std::find(tested.begin(), tested.end(), device) == tested.end()) {
            int rc = self_test(20.0);
            if (rc) {
                std::string m = g_err;
                return fail(rc, "device self-test failed: %s", m.c_str());
            }
            void *ptr = nullptr;
            e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !ptr)
                return fail(RECON_EDEVICE, "hipGetSymbolAddress of the fixed workspace failed: %s",
                            hipGetErrorString(e));
            noalloc_ptr[device] = (uint8_t *)ptr;
            tested.push_back(device);
        }
        fixed = noalloc_ptr[device];
    }
    int rc = make_ctx(out, device, c);
    if (rc == RECON_OK) (*out)->noalloc = fixed;
    return rc;
}

int recon_destroy(recon_ctx *ctx) {
    if (!ctx) return fail(RECON_EINVAL, "null context");
    if (ctx->serve) (void)recon_serve_stop(ctx);
    (void)hipSetDevice(ctx->device);
    if (ctx->have_last && wait_event(ctx->last_done, 60.0, "the last launch") != RECON_OK)
        return RECON_ETIMEDOUT;   // leak rather than free memory a running kernel may use
    drop_graphs(ctx);
    free_workspace(ctx);
    if (ctx->h_table) (void)hipHostFree(ctx->h_table);
    if (ctx->h_work) (void)hipHostFree(ctx->h_work);
    if (ctx->h_done) (void)hipHostFree(ctx->h_done);
    if (ctx->table_used) (void)hipEventDestroy(ctx->table_used);
    if (ctx->last_done) (void)hipEventDestroy(ctx->last_done);
    for (auto &set : ctx->tev)
        for (auto &ev : set)
            if (ev) (void)hipEventDestroy(ev);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    if (ctx->aux_stream) (void)hipStreamDestroy(ctx->aux_stream);
    if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
    if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
    for (int v = 0; v < kVariants; ++v) {
        if (ctx->shape_ctx[v]) (void)recon_destroy(ctx->shape_ctx[v]);
        if (ctx->shape_stream[v]) (void)hipStreamDestroy(ctx->shape_stream[v]);
        if (ctx->shape_join[v]) (void)hipEventDestroy(ctx->shape_join[v]);
    }
    if (ctx->shape_fork) (void)hipEventDestroy(ctx->shape_fork);
    delete ctx;
    return RECON_OK;
}

int recon_dilate(recon_ctx *ctx, recon_image *marker, const recon_image *mask, int conn, void *stream) {
    if (!ctx) return fail(RECON_EINVAL, "null context");
    if (!marker || !mask) return fail(RECON_EINVAL, "null image");
    recon_task t{};
    t.op = RECON_OP_DILATE;
    t.conn = conn;
    t.image = *marker;
    t.mask = *mask;
    int rc = check_task(t);
    if (rc) return rc;
    return run_tasks(ctx, &t, 1, (hipStream_t)stream, false);
}

int recon_dilate_noalloc(recon_ctx *ctx, recon_image *marker, const recon_image *mask, int conn, void *stream) {
    if (!ctx) return fail(RECON_EINVAL, "null context");
    if (!marker || !mask) return fail(RECON_EINVAL, "null image");
    if (!ctx->noalloc) return fail(RECON_EDEVICE, "the fixed workspace of this device was not set up");
    if (ctx->cfg.stop_after_stage != 0)
        return fail(RECON_EINVAL, "recon_dilate_noalloc runs the persistent pipeline only (stop_after_stage = 0)");
    recon_task t{};
    t.op = RECON_OP_DILATE;
    t.conn = conn;
    t.image = *marker;
    t.mask = *mask;
    int rc = check_task(t);
    if (rc) return rc;
    const int bh = ctx->cfg.block_rows;
    const size_t blocks = (size_t)((t.image.height + bh - 1) / bh) * (size_t)((t.image.width + rk::BW - 1) / rk::BW);
    if (blocks > NOALLOC_MAX_BLOCKS)
        return fail(RECON_EINVAL,
                    "recon_dilate_noalloc: a %dx%d image has %zu blocks of %dx%d pixels, above the fixed "
                    "workspace's %zu", t.image.height, t.image.width, blocks, bh, rk::BW, NOALLOC_MAX_BLOCKS);
    rc = ensure_device(ctx);
    if (rc) return rc;
    std::vector<rk::TaskDev> table;
    std::vector<char> uses_scratch;
    uint32_t total_blocks = 0;
    size_t scratch_bytes = 0;
    bool any_mapped = false;
    std::vector<size_t> lab_off;
    build_table(ctx->cfg, &t, 1, bh, table, uses_scratch, total_blocks, scratch_bytes, any_mapped, false, lab_off);
    uint8_t *base = ctx->noalloc;
    Workspace ws;
    ws.work = (rk::Work *)base;
    ws.tile_pending = (uint32_t *)(base + NOALLOC_TILE_OFF);
    ws.tile_done = ws.tile_pending + 1;
    ws.state = (uint32_t *)(base + NOALLOC_STATE_OFF);
    ws.ring = (uint32_t *)(base + NOALLOC_RING_OFF);
    ws.route = nullptr;   // no label plane: the block route only
    ws.spill = nullptr;   // no spill queues: a full LDS queue re-seeds the block
    ws.cap_blocks = total_blocks;
    rk::TaskTable tt{};
    tt.hdr = nullptr;
    tt.ext = nullptr;
    tt.n_inline = 1;
    tt.total_inline = total_blocks;
    tt.ring_cap_inline = (uint32_t)ring_slots(total_blocks);
    ctx->launch_seq = next_launch_seq();
    tt.seq_inline = ctx->launch_seq;
    tt.inl[0] = table[0];
    const hipStream_t s = (hipStream_t)stream;
    rc = enqueue_kernels(ctx, ws, variant_of(bh), tt, total_blocks, 1u, false, false, false, s);
    if (rc) return rc;
    HIP_TRY(hipEventRecord(ctx->last_done, s));
    ctx->have_last = true;
    ctx->last_work = ws.work;
    ctx->last_was_graph = false;
    ctx->tev_graph[ctx->launches % kTimingRing] = false;
    ctx->launches += 1;
    return RECON_OK;
}

int recon_fill_holes(recon_ctx *ctx, recon_image *img, int conn, void *stream) {
    if (!ctx) return fail(RECON_EINVAL, "null context");
    if (!img) return fail(RECON_EINVAL, "null image");
    recon_task t{};
    t.op = RECON_OP_FILL_HOLES;
    t.conn = conn;
    t.image = *img;
    int rc = check_task(t);
    if (rc) return rc;
    return run_tasks(ctx, &t, 1, (hipStream_t)stream, false);
}

int recon_erode(recon_ctx *ctx, recon_image *marker, const recon_image *mask, int conn, void *stream) {
    if (!ctx) return fail(RECON_EINVAL, "null context");
    if (!marker || !mask) return fail(RECON_EINVAL, "null image");
    recon_task t{};
    t.op = RECON_OP_ERODE;
    t.conn = conn;
    t.image = *marker;
    t.mask = *mask;
    int rc = check_task(t);
    if (rc) return rc;
    return run_tasks(ctx, &t, 1, (hipStream_t)stream, false);
}

int recon_hdome(recon_ctx *ctx, recon_image *img, int h, int conn, void *stream) {
    if (!ctx) return fail(RECON_EINVAL, "null context");
    if (!img) return fail(RECON_EINVAL, "null image");
    recon_task t{};
    t.op = RECON_OP_HDOME;
    t.conn = conn;
    t.h = h;
    t.image = *img;
    int rc = check_task(t);
    if (rc) return rc;
    return run_tasks(ctx, &t, 1, (hipStream_t)stream, false);
}

int recon_regional_max(recon_ctx *ctx, recon_image *img, int conn, void *stream) {
    if (!ctx) return fail(RECON_EINVAL, "null context");
    if (!img) return fail(RECON_EINVAL, "null image");
    recon_task t{};
    t.op = RECON_OP_REGIONAL_MAX;
    t.conn = conn;
    t.image = *img;
    int rc = check_task(t);
    if (rc) return rc;
    return run_tasks(ctx, &t, 1, (hipStream_t)stream, false);
}

// ---- connected-component labelling and the area filter

// Scratch bytes of the labelling phases for an h x w image whose label plane
// has `pitch_lab` elements per row: the root bitmap, per-word offsets and
// per-segment sums.
static void label_layout(int h, int w, int64_t pitch_lab, uint32_t &n_words, uint32_t &n_segs, size_t &bytes) {
    const uint64_t nbits = (uint64_t)(h - 1) * (uint64_t)pitch_lab + (uint64_t)w;
    n_words = (uint32_t)((nbits + 31) / 32);
    n_segs = (n_words + rk::RANK_SEG - 1) / rk::RANK_SEG;
    bytes = round_up((size_t)n_words * 4, 256) * 2 + round_up((size_t)n_segs * 4, 256);
}

// true if the int32 plane (h rows of pitch elements, w used) overlaps the image's bytes
static bool plane_overlaps(const recon_image &img, const int32_t *plane, int64_t pitch) {
    recon_image p{};
    p.data = (uint8_t *)plane;
    p.height = img.height;
    p.width = img.width * 4;
    p.pitch = pitch * 4;
    return overlaps(img, p);
}

static int check_label_args(const recon_image *img, int64_t pitch_lab, int conn) {
    int rc = check_image(img, "image");
    if (rc) return rc;
    if (conn != 4 && conn != 8) return fail(RECON_EINVAL, "conn must be 4 or 8, got %d", conn);
    if (pitch_lab < img->width)
        return fail(RECON_EINVAL, "label pitch %lld < width %d", (long long)pitch_lab, img->width);
    if ((uint64_t)img->height * (uint64_t)pitch_lab >= (uint64_t)INT32_MAX)
        return fail(RECON_EINVAL, "height x label pitch must stay below 2^31 (node ids are int32)");
    return RECON_OK;
}

// Enqueue the labelling phases: labels of `img` into `lab` (pitch_lab
// elements per row); `area` holds label_layout's bytes.  With ranks =
// false the phases stop after flattening: every foreground pixel then holds
// its component's root id (the pitched index + 1 of its raster-first pixel).
static int enqueue_label(const recon_image &img, int32_t *lab, int64_t pitch_lab, int conn, int32_t *count,
                         uint8_t *area, bool ranks, hipStream_t s) {
    rk::LabelArgs a{};
    a.img = img.data;
    a.pitch_img = img.pitch;
    a.lab = lab;
    a.pitch_lab = pitch_lab;
    a.h = img.height;
    a.w = img.width;
    a.conn = conn;
    a.tiles_x = (img.width + rk::LT_W - 1) / rk::LT_W;
    size_t bytes = 0;
    label_layout(img.height, img.width, pitch_lab, a.n_words, a.n_segs, bytes);
    a.bits = ranks ? (uint32_t *)area : nullptr;
    a.word_off = (uint32_t *)(area + round_up((size_t)a.n_words * 4, 256));
    a.seg_sum = (uint32_t *)(area + 2 * round_up((size_t)a.n_words * 4, 256));
    a.count = count;
    a.lab_vec = (((uintptr_t)lab | (uintptr_t)(pitch_lab * 4)) & 15u) == 0 ? 1 : 0;
    const int64_t n_tiles = (int64_t)a.tiles_x * ((img.height + rk::LT_H - 1) / rk::LT_H);
    const int64_t n_rows = (int64_t)img.height * a.tiles_x;
    const int g_tiles = (int)std::min<int64_t>(n_tiles, 65535);
    const int g_rows = (int)std::min<int64_t>(n_rows, 65535);
    const int g_segs = (int)std::min<uint32_t>(a.n_segs, 65535u);
    const int g_clear = (int)std::min<uint32_t>((a.n_words + 255) / 256, 4096u);
    const size_t lds = (size_t)rk::LT_H * rk::LT_W * sizeof(uint32_t);
    if (ranks) hipLaunchKernelGGL(rk::clear_words, dim3(g_clear), dim3(256), 0, s, a.bits, a.n_words);
    hipLaunchKernelGGL(rk::label_local, dim3(g_tiles), dim3(64), lds, s, a);
    hipLaunchKernelGGL(rk::label_merge, dim3(g_tiles), dim3(64), 0, s, a);
    hipLaunchKernelGGL(rk::label_flatten, dim3(g_rows), dim3(64), 0, s, a);
    if (!ranks) {
        HIP_TRY(hipGetLastError());
        return RECON_OK;
    }
    hipLaunchKernelGGL(rk::rank_segments, dim3(g_segs), dim3(64), 0, s, a);
    hipLaunchKernelGGL(rk::rank_scan, dim3(1), dim3(64), 0, s, a);
    hipLaunchKernelGGL(rk::rank_words, dim3(g_segs), dim3(64), 0, s, a);
    hipLaunchKernelGGL(rk::label_final, dim3(g_rows), dim3(64), 0, s, a);
    HIP_TRY(hipGetLastError());
    return RECON_OK;
}

int recon_label(recon_ctx *ctx, const recon_image *img, int32_t *labels, int64_t label_pitch, int conn,
                int32_t *count, void *stream) {
    if (!ctx) return fail(RECON_EINVAL, "null context");
    if (!labels) return fail(RECON_EINVAL, "null label plane");
    int rc = check_label_args(img, label_pitch, conn);
    if (rc) return rc;
    if (plane_overlaps(*img, labels, label_pitch)) return fail(RECON_EINVAL, "label plane and image overlap");
    rc = ensure_device(ctx);
    if (rc) return rc;
    uint32_t nw = 0, ns = 0;
    size_t bytes = 0;
    label_layout(img->height, img->width, label_pitch, nw, ns, bytes);
    rc = ensure_capacity(ctx, 0, 0, bytes);
    if (rc) return rc;
    return enqueue_label(*img, labels, label_pitch, conn, count, ctx->d_scratch, true, (hipStream_t)stream);
}

int recon_area_threshold(recon_ctx *ctx, recon_image *img, int conn, int64_t min_area, int64_t max_area,
                         void *stream) {
    if (!ctx) return fail(RECON_EINVAL, "null context");
    if (!img) return fail(RECON_EINVAL, "null image");
    if (min_area < 0 || max_area < min_area)
        return fail(RECON_EINVAL, "area bounds must satisfy 0 <= min_area <= max_area");
    const int64_t pitch_lab = (int64_t)round_up((size_t)img->width, 64);
    int rc = check_label_args(img, pitch_lab, conn);
    if (rc) return rc;
    rc = ensure_device(ctx);
    if (rc) return rc;
    // the label plane holds root ids (pitched index + 1 of each component's
    // first pixel), which index the area counts directly: no ranks needed
    const size_t plane = round_up((size_t)img->height * (size_t)pitch_lab * 4, 256);
    const size_t n_area = (size_t)img->height * (size_t)pitch_lab + 1;
    const size_t abytes = round_up(n_area * 4, 256);
    rc = ensure_capacity(ctx, 0, 0, plane + abytes);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    int32_t *lab = (int32_t *)ctx->d_scratch;
    uint32_t *area = (uint32_t *)(ctx->d_scratch + plane);
    rc = enqueue_label(*img, lab, pitch_lab, conn, nullptr, nullptr, false, s);
    if (rc) return rc;
    rk::AreaArgs a{};
    a.lab = lab;
    a.pitch_lab = pitch_lab;
    a.lab_vec = (((uintptr_t)lab | (uintptr_t)(pitch_lab * 4)) & 15u) == 0 ? 1 : 0;
    a.out_aligned = aligned4(img->data, img->pitch) ? 1 : 0;
    a.area = area;
    a.out = img->data;
    a.pitch_out = img->pitch;
    a.h = img->height;
    a.w = img->width;
    a.min_area = min_area;
    a.max_area = max_area;
    const int64_t n_rows = (int64_t)img->height * ((img->width + rk::LT_W - 1) / rk::LT_W);
    const int g_rows = (int)std::min<int64_t>(n_rows, 65535);
    hipLaunchKernelGGL(rk::clear_words, dim3((unsigned)std::min<size_t>((n_area + 255) / 256, 4096)), dim3(256), 0,
                       s, area, (uint32_t)n_area);
    hipLaunchKernelGGL(rk::area_count, dim3(g_rows), dim3(64), 0, s, a);
    hipLaunchKernelGGL(rk::area_apply, dim3(g_rows), dim3(64), 0, s, a);
    HIP_TRY(hipGetLastError());
    return RECON_OK;
}

// ---- exact distance transform and Pre-Watershed markers

static int check_edt_image(const recon_image *img) {
    int rc = check_image(img, "image");
    if (rc) return rc;
    if (img->width > rk::EDT_MAX_W || img->height > rk::EDT_MAX_W)
        return fail(RECON_EINVAL, "distance transform: height and width must be at most %d", rk::EDT_MAX_W);
    return RECON_OK;
}

// Scratch bytes of the column-segment summaries.
static size_t edt_summary_bytes(int h, int w) {
    const size_t n = (size_t)((h + rk::EDT_SEG - 1) / rk::EDT_SEG) * (size_t)w;
    return 2 * round_up(n * 4, 256);
}

// `summary` holds edt_summary_bytes.
static int enqueue_edt(rk::EdtArgs a, uint8_t *summary, hipStream_t s) {
    const int64_t n_cols = ((int64_t)(a.h + rk::EDT_SEG - 1) / rk::EDT_SEG) * a.w;
    a.zfirst = (int32_t *)summary;
    a.zlast = (int32_t *)(summary + round_up((size_t)n_cols * 4, 256));
    const int g_cols = (int)std::min<int64_t>((n_cols + 255) / 256, 65535);
    hipLaunchKernelGGL(rk::edt_zeros, dim3(g_cols), dim3(256), 0, s, a);
    hipLaunchKernelGGL(rk::edt_cols, dim3(g_cols), dim3(256), 0, s, a);
    hipLaunchKernelGGL(rk::edt_rows, dim3(std::min(a.h, 65535)), dim3(256), (size_t)a.w * sizeof(int32_t), s, a);
    HIP_TRY(hipGetLastError());
    return RECON_OK;
}

int recon_distance(recon_ctx *ctx, const recon_image *img, int32_t *dist2, int64_t dist_pitch, void *stream) {
    if (!ctx) return fail(RECON_EINVAL, "null context");
    if (!dist2) return fail(RECON_EINVAL, "null distance plane");
    int rc = check_edt_image(img);
    if (rc) return rc;
    if (dist_pitch < img->width)
        return fail(RECON_EINVAL, "distance pitch %lld < width %d", (long long)dist_pitch, img->width);
    if (plane_overlaps(*img, dist2, dist_pitch)) return fail(RECON_EINVAL, "distance plane and image overlap");
    rc = ensure_device(ctx);
    if (rc) return rc;
    rc = ensure_capacity(ctx, 0, 0, edt_summary_bytes(img->height, img->width));
    if (rc) return rc;
    rk::EdtArgs a{};
    a.img = img->data;
    a.pitch_img = img->pitch;
    a.g = dist2;
    a.pitch_g = dist_pitch;
    a.h = img->height;
    a.w = img->width;
    a.mode = 0;
    return enqueue_edt(a, ctx->d_scratch, (hipStream_t)stream);
}

int recon_pre_watershed(recon_ctx *ctx, recon_image *img, int conn, void *stream) {
    if (!ctx) return fail(RECON_EINVAL, "null context");
    int rc = check_edt_image(img);
    if (rc) return rc;
    if (conn != 4 && conn != 8) return fail(RECON_EINVAL, "conn must be 4 or 8, got %d", conn);
    rc = ensure_device(ctx);
    if (rc) return rc;
    const int64_t pitch_g = (int64_t)round_up((size_t)img->width, 64);
    const size_t plane = round_up((size_t)img->height * (size_t)pitch_g * 4, 256);
    rc = ensure_capacity(ctx, 0, 0, plane + edt_summary_bytes(img->height, img->width));
    if (rc) return rc;
    rk::EdtArgs a{};
    a.img = img->data;
    a.pitch_img = img->pitch;
    a.g = (int32_t *)ctx->d_scratch;
    a.pitch_g = pitch_g;
    a.d8 = img->data;     // D8 replaces the image (its input is read by edt_cols only)
    a.pitch_d8 = img->pitch;
    a.h = img->height;
    a.w = img->width;
    a.mode = 1;
    rc = enqueue_edt(a, ctx->d_scratch + plane, (hipStream_t)stream);
    if (rc) return rc;
    // the regional maxima of D8, in place (the reconstruction reuses the
    // scratch area once the row pass, earlier on the stream, has read it)
    recon_task t{};
    t.op = RECON_OP_REGIONAL_MAX;
    t.conn = conn;
    t.image = *img;
    rc = check_task(t);
    if (rc) return rc;
    return run_tasks(ctx, &t, 1, (hipStream_t)stream, false);
}

int recon_batch(recon_ctx *ctx, const recon_task *tasks, int32_t n, void *stream) {
    if (!ctx) return fail(RECON_EINVAL, "null context");
    if (n < 0 || (n > 0 && !tasks)) return fail(RECON_EINVAL, "bad task list");
    if (n == 0) return RECON_OK;
    for (int k = 0; k < n; ++k) {
        int rc = check_task(tasks[k], &ctx->cfg);
        if (rc) {
            std::string m = g_err;
            return fail(rc, "task %d: %s", k, m.c_str());
        }
    }
    const int v_ctx = variant_of(ctx->cfg.block_rows);
    unsigned shapes = 0;
    for (int k = 0; k < n; ++k)
        shapes |= 1u << (tasks[k].block_rows ? variant_of(tasks[k].block_rows) : v_ctx);
    if (shapes == (1u << v_ctx)) {
        // a batch that fits the kernel arguments is launched directly (its table
        // travels inline: no table copy, and fewer packets than a graph replay,
        // which on this runtime costs more than the launches it saves); larger
        // batches replay the context's captured graph
        ctx->last_shapes = 0;
        const bool use_graph = n > rk::MAX_INLINE_TASKS;
        return run_tasks(ctx, tasks, n, (hipStream_t)stream, use_graph);
    }
    return run_shape_groups(ctx, tasks, n, shapes, (hipStream_t)stream);
}

// Durations (ms) of a recent launch from its timing marks: K1, K2, K3, whole
// launch (from before the scheduler reset to after the result mapping); -1
// where a mark was not recorded (graph replays mark only the whole).
static void launch_times(recon_ctx *ctx, int back, float t[5]) {
    const int i = (int)((ctx->launches - 1 - (uint64_t)back) % kTimingRing);
    hipEvent_t *tev = ctx->tev[i];
    t[0] = t[1] = t[2] = t[3] = t[4] = -1.f;
    float ms = 0.f;
    if (!ctx->tev_graph[i]) {
        if (ctx->tev_merged[i]) {
            // the persistent pipeline: no dense pass and no border kernel;
            // the route's mark (tev[6], its own stream) closes its kernels,
            // counted from the start of the launch
            t[0] = t[1] = 0.f;
            t[4] = 0.f;
            if (ctx->tev_route[i] && hipEventElapsedTime(&ms, tev[5], tev[6]) == hipSuccess) t[4] = ms;
        } else {
            if (hipEventElapsedTime(&ms, tev[6], tev[1]) == hipSuccess) t[0] = ms;
            if (hipEventElapsedTime(&ms, tev[1], tev[2]) == hipSuccess) t[1] = ms;
        }
        if (hipEventElapsedTime(&ms, tev[2], tev[3]) == hipSuccess) t[2] = ms;
    }
    if (hipEventElapsedTime(&ms, tev[5], tev[4]) == hipSuccess) t[3] = ms;
    (void)hipGetLastError();   // a mark that was not recorded must not leave an error behind
}

}  // extern "C"

namespace {

// The scheduler counters of `work` (device memory of ctx's device), read
// through a kernel into ctx's pinned buffer once ctx's last launch is done.
int read_work(recon_ctx *ctx, const rk::Work *work, rk::Work &w) {
    hipLaunchKernelGGL(rk::copy_table, dim3(1), dim3(64), 0, nullptr, (const uint8_t *)work,
                       (uint8_t *)ctx->h_work, (uint32_t)sizeof(rk::Work));
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventRecord(ctx->last_done, nullptr));
    int rc = wait_event(ctx->last_done, 60.0, "the statistics read-back");
    if (rc) return rc;
    std::memcpy(&w, (const void *)ctx->h_work, sizeof(w));
    return RECON_OK;
}

}  // namespace

extern "C" {

int recon_last_stats(recon_ctx *ctx, recon_stats *out) {
    if (!ctx || !out) return fail(RECON_EINVAL, "null argument");
    std::memset(out, 0, sizeof(*out));
    if (!ctx->have_last) return RECON_OK;
    int rc = ensure_device(ctx);
    if (rc) return rc;
    rc = wait_event(ctx->last_done, 60.0, "the last launch");
    if (rc) return rc;
    // the counters of the last launch, summed over its block-height groups
    std::vector<std::pair<recon_ctx *, const rk::Work *>> parts;
    if (ctx->last_shapes) {
        for (int v = 0; v < kVariants; ++v)
            if ((ctx->last_shapes & (1u << v)) && ctx->shape_ctx[v])
                parts.emplace_back(ctx->shape_ctx[v], ctx->shape_ctx[v]->last_work);
    } else {
        parts.emplace_back(ctx, ctx->last_work);
    }
    bool aborted = false;
    for (auto &pt : parts) {
        rk::Work w;
        rc = read_work(pt.first, pt.second, w);
        if (rc) return rc;
        out->dense_visits += (int64_t)w.stat_dense;
        out->revisits += (int64_t)w.stat_revisit;
        out->reruns += (int64_t)w.stat_rerun;
        out->queue_overflows += (int64_t)w.stat_overflow;
        out->requests += (int64_t)w.stat_request;
        out->aborted |= (int64_t)w.abort;
        out->component_tasks += (int64_t)w.stat_route;
        out->queue_spills += (int64_t)w.stat_spill;
        aborted |= w.abort != 0;
    }
    if (ctx->cfg.timing) {
        float t[5];
        launch_times(ctx, 0, t);
        out->dense_ms = t[0];
        out->seed_ms = t[1];
        out->drain_ms = t[2];
        out->total_ms = t[3];
        out->route_ms = t[4];
    }
    if (aborted) return fail(RECON_EDEVICE, "scheduler watchdog expired: the last launch did not converge");
    return RECON_OK;
}

int recon_enqueue_status(recon_ctx *ctx, uint32_t *host_flag, void *stream) {
    if (!ctx || !host_flag) return fail(RECON_EINVAL, "null argument");
    int rc = ensure_device(ctx);
    if (rc) return rc;
    // the Work records of the last launch (one per block-height group)
    const rk::Work *w[3] = {nullptr, nullptr, nullptr};
    int n = 0;
    if (ctx->have_last) {
        if (ctx->last_shapes) {
            for (int v = 0; v < kVariants && n < 3; ++v)
                if ((ctx->last_shapes & (1u << v)) && ctx->shape_ctx[v]) w[n++] = ctx->shape_ctx[v]->last_work;
        } else {
            w[n++] = ctx->last_work;
        }
    }
    hipLaunchKernelGGL(rk::launch_outcome, dim3(1), dim3(64), 0, (hipStream_t)stream, w[0], w[1], w[2], host_flag);
    HIP_TRY(hipGetLastError());
    return RECON_OK;
}

int recon_launch_times(recon_ctx *ctx, int back, float *dense_ms, float *seed_ms, float *drain_ms,
                       float *total_ms, float *route_ms) {
    if (!ctx || !dense_ms || !seed_ms || !drain_ms || !total_ms || !route_ms)
        return fail(RECON_EINVAL, "null argument");
    if (!ctx->cfg.timing) return fail(RECON_EINVAL, "the context was created without timing");
    if (back < 0 || back >= kTimingRing || (uint64_t)back >= ctx->launches)
        return fail(RECON_EINVAL, "launch %d back is not kept (%llu launches, %d kept)", back,
                    (unsigned long long)ctx->launches, kTimingRing);
    int rc = ensure_device(ctx);
    if (rc) return rc;
    hipEvent_t *tev = ctx->tev[(ctx->launches - 1 - (uint64_t)back) % kTimingRing];
    rc = wait_event(tev[4], 60.0, "the timed launch");
    if (rc) return rc;
    float t[5];
    launch_times(ctx, back, t);
    *dense_ms = t[0];
    *seed_ms = t[1];
    *drain_ms = t[2];
    *total_ms = t[3];
    *route_ms = t[4];
    return RECON_OK;
}

int recon_submit(recon_ctx *ctx, const recon_task *task, uint64_t *ticket) {
    if (!ctx || !task || !ticket) return fail(RECON_EINVAL, "null argument");
    int rc = check_task(*task, &ctx->cfg);
    if (rc) return rc;
    rc = ensure_device(ctx);
    if (rc) return rc;
    if (!ctx->serve) {
        rc = serve_start(ctx);
        if (rc) return rc;
    }
    recon_ctx::Serve *S = ctx->serve;
    const size_t bytes = task_bytes(*task, ctx->cfg);
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stop) return fail(RECON_EINVAL, "serving has been stopped");
        if ((int64_t)(bytes + S->bytes_fixed) > ctx->cfg.serve_mem_cap)
            return fail(RECON_EINVAL, "task needs %zu bytes, above the admission cap", bytes);
        if ((int64_t)(S->bytes_fixed + S->bytes_admitted + bytes) > ctx->cfg.serve_mem_cap ||
            S->slots_admitted >= ctx->cfg.serve_slots)
            return fail(RECON_EAGAIN, "admission full (%zu bytes, %d slots in flight)", S->bytes_admitted,
                        S->slots_admitted);
        const uint64_t tk = S->next_ticket++;
        S->waiting.push_back({tk, *task, bytes});
        S->status[tk] = 0;
        S->bytes_admitted += bytes;
        S->slots_admitted += 1;
        *ticket = tk;
    }
    S->cv_work.notify_one();
    return RECON_OK;
}

int recon_poll(recon_ctx *ctx, uint64_t ticket, int *done) {
    if (!ctx || !done) return fail(RECON_EINVAL, "null argument");
    *done = 0;
    if (!ctx->serve) return fail(RECON_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    recon_ctx::Serve *S = ctx->serve;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->status.find(ticket);
    if (it == S->status.end()) return fail(RECON_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    if (it->second == -1) {
        S->status.erase(it);
        return fail(S->error ? S->error : RECON_EDEVICE, "%s", S->error_msg.c_str());
    }
    if (it->second == 2) {
        *done = 1;
        S->status.erase(it);
    }
    return RECON_OK;
}

int recon_wait(recon_ctx *ctx, uint64_t ticket, int64_t timeout_us) {
    if (!ctx) return fail(RECON_EINVAL, "null context");
    if (!ctx->serve) return fail(RECON_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    recon_ctx::Serve *S = ctx->serve;
    std::unique_lock<std::mutex> lk(S->mu);
    const auto deadline = std::chrono::steady_clock::now() + std::chrono::microseconds(timeout_us < 0 ? 0 : timeout_us);
    while (true) {
        auto it = S->status.find(ticket);
        if (it == S->status.end()) return fail(RECON_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
        if (it->second == 2) {
            S->status.erase(it);
            return RECON_OK;
        }
        if (it->second == -1) {
            S->status.erase(it);
            return fail(S->error ? S->error : RECON_EDEVICE, "%s", S->error_msg.c_str());
        }
        if (timeout_us < 0) {
            S->cv_done.wait_for(lk, std::chrono::milliseconds(10));
        } else {
            if (std::chrono::steady_clock::now() >= deadline)
                return fail(RECON_ETIMEDOUT, "ticket %llu not done after %lld us", (unsigned long long)ticket,
                            (long long)timeout_us);
            S->cv_done.wait_until(lk, std::min(deadline, std::chrono::steady_clock::now() + std::chrono::milliseconds(10)));
        }
    }
}

int recon_serve_stats(recon_ctx *ctx, recon_serve_counters *out) {
    if (!ctx || !out) return fail(RECON_EINVAL, "null argument");
    std::memset(out, 0, sizeof(*out));
    recon_ctx::Serve *S = ctx->serve;
    if (!S) return RECON_OK;
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->stats;
    return RECON_OK;
}

int recon_serve_stop(recon_ctx *ctx) {
    if (!ctx) return fail(RECON_EINVAL, "null context");
    recon_ctx::Serve *S = ctx->serve;
    if (!S) return RECON_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    if (S->worker.joinable()) S->worker.join();
    int rc = RECON_OK;
    for (auto &L : S->lanes) {
        if (L.sub && recon_destroy(L.sub) != RECON_OK) rc = RECON_ETIMEDOUT;
        if (L.stream) (void)hipStreamDestroy(L.stream);
        if (L.done) (void)hipEventDestroy(L.done);
    }
    delete S;
    ctx->serve = nullptr;
    return rc;
}

}  // extern "C"
