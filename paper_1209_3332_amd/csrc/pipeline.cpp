// pipeline.cpp -- co-scheduling of a per-tile operation pipeline over the host
// cores and the GPU (see recon_pipeline_run in include/recon.h).
//
// The paper's Worker turns every tile into a graph of operation instances, the
// (tile, operation) tuples, and maps each ready instance to an idle CPU core or
// GPU (Sec. IV-B).  First-come-first-served hands the oldest ready instance to
// whichever device asks.  PATS keeps the ready instances sorted by their
// estimated GPU-over-CPU speedup: an idle CPU core takes the one with the
// lowest estimate, an idle GPU the one with the highest.  Data locality
// (Sec. IV-C) lets the GPU prefer an instance whose inputs are already in
// device memory, unless a non-resident one is expected to gain more than the
// transfers cost it.  The Worker holds a bounded number of tiles in flight
// (the demand-driven window of Sec. III-B): a finished tile frees a slot for
// the next one.
//
// Threads: one GPU manager thread (it calls the library's operations on its
// own stream, keeps up to `gpu_inflight` instances enqueued there and retires
// each when the stream has passed it), `cpu_workers` CPU threads (each
// runs the CPU variants of host_ops.cpp on one core) and `io_threads` threads
// that bring finished tiles' results out and the next tiles' images in.  Every tile slot owns
// pinned host planes and device planes for the tile's data; a per-plane bit
// set records where a valid copy lives, and a device moves a plane only when
// it lacks a valid copy.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <deque>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/recon.h"
#include "host_ops.hpp"

namespace {

using Clock = std::chrono::steady_clock;

thread_local std::string g_pipe_err;   // message of the calling thread's last failed pipeline call

double ms_since(Clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
}

// The tile's planes: A carries the image through the dome, fill-holes and area
// operations (each in place); B the markers; L the labels (int32) and the count.
enum Plane { PA = 0, PB = 1, PL = 2, NPLANES = 3 };
enum : uint8_t { ON_HOST = 1, ON_DEV = 2 };

struct OpShape {
    uint8_t in_mask;    // planes read
    uint8_t out_mask;   // planes written
    int next[2];        // dependent operations (-1: none)
    int deps;           // operations it waits for
};

// hdome -> fill-holes -> area -> {markers, labels}
constexpr OpShape kOps[RECON_PIPE_NOPS] = {
    {1u << PA, 1u << PA, {RECON_PIPE_FILL, -1}, 0},
    {1u << PA, 1u << PA, {RECON_PIPE_AREA, -1}, 1},
    {1u << PA, 1u << PA, {RECON_PIPE_MARKERS, RECON_PIPE_LABEL}, 1},
    {1u << PA, 1u << PB, {-1, -1}, 1},
    {1u << PA, 1u << PL, {-1, -1}, 1},
};

struct Slot {
    int tile = -1;                       // tile in the slot, -1 when free
    uint8_t *h[NPLANES] = {};            // pinned host planes
    uint8_t *d[NPLANES] = {};            // device planes
    int32_t *d_count = nullptr;          // device component count
    int32_t h_count = 0;
    // ON_HOST | ON_DEV per plane: written under xfer_mu, read by the scheduler
    // without it (a stale read only changes a placement preference)
    std::atomic<uint8_t> where[NPLANES];
    std::mutex xfer_mu;                  // one transfer of a slot's planes at a time
    int waiting[RECON_PIPE_NOPS] = {};   // unfinished dependencies per operation
    int left = 0;                        // unfinished operations of the tile
    Slot() {
        for (auto &w : where) w.store(0);
    }
};

struct Ready {
    int slot, op;
    uint64_t seq;   // order of becoming ready (FCFS)
    float speedup;
};

struct Device {
    bool gpu;
    int id = 0;   // 0: the GPU, 1 + k: CPU worker k
    hipStream_t stream = nullptr;
    hipStream_t xfer = nullptr;   // the GPU manager's plane transfers (its stream computes)
    hostops::Scratch *scratch = nullptr;
};

struct Run {
    recon_ctx *ctx;
    const recon_pipe_tile *tiles;
    int n;
    recon_pipe_config cfg;
    int H = 0, W = 0;            // plane geometry of the slots (largest tile)
    int64_t pitch = 0;           // bytes per row of the uint8 planes
    int64_t lpitch = 0;          // elements per row of the label plane
    std::unique_ptr<Slot[]> slots;
    int nslots = 0;
    std::vector<Ready> ready;
    std::vector<int> finished;   // slots whose tile's last operation completed
    std::mutex mu;
    std::condition_variable cv;
    uint64_t seq = 0;
    int next_tile = 0, done_tiles = 0;
    double gpu_left_ms = 0.0;    // estimated GPU time of the instances not started yet (cpu_guard)
    std::atomic<uint64_t> ready_gen{0};   // bumped whenever instances become ready (read without r.mu)
    Clock::time_point t0;        // start of the run (trace times)
    int err = RECON_OK;
    std::string err_msg;
    recon_pipe_stats st{};
    int device = 0;

    size_t plane_bytes(int p) const { return p == PL ? (size_t)H * lpitch * 4 : (size_t)H * pitch; }
};

int set_err(Run &r, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    std::lock_guard<std::mutex> g(r.mu);
    if (r.err == RECON_OK) {
        r.err = code;
        r.err_msg = buf;
    }
    r.cv.notify_all();
    return code;
}

#define PIPE_HIP(run, expr)                                                                  \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return set_err(run, RECON_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// Wait for the stream's work with a deadline: polled without sleeping for the
// first 2 ms (an operation or a plane copy usually ends within that, and a
// sleep of the host scheduler would add more than the wait itself), then with
// short sleeps.
int sync_stream(Run &r, hipStream_t s) {
    const auto t0 = Clock::now();
    while (true) {
        hipError_t q = hipStreamQuery(s);
        if (q == hipSuccess) return RECON_OK;
        if (q != hipErrorNotReady)
            return set_err(r, RECON_EDEVICE, "pipeline stream failed: %s", hipGetErrorString(q));
        const double ms = ms_since(t0);
        if (ms > 60000.0) return set_err(r, RECON_ETIMEDOUT, "pipeline stream wait exceeded 60 s");
        if (ms > 2.0) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}

// Copy plane p of the slot to the device or to the host on stream s (not waited for).
int move_plane(Run &r, Slot &sl, int p, bool to_dev, hipStream_t s) {
    const int th = r.tiles[sl.tile].height, tw = r.tiles[sl.tile].width;
    const size_t row = p == PL ? (size_t)tw * 4 : (size_t)tw;
    const size_t pitch = p == PL ? (size_t)r.lpitch * 4 : (size_t)r.pitch;
    if (to_dev)
        PIPE_HIP(r, hipMemcpy2DAsync(sl.d[p], pitch, sl.h[p], pitch, row, th, hipMemcpyHostToDevice, s));
    else
        PIPE_HIP(r, hipMemcpy2DAsync(sl.h[p], pitch, sl.d[p], pitch, row, th, hipMemcpyDeviceToHost, s));
    if (p == PL && !to_dev)
        PIPE_HIP(r, hipMemcpyAsync(&sl.h_count, sl.d_count, 4, hipMemcpyDeviceToHost, s));
    return RECON_OK;
}

// Make the planes in `mask` valid on the host (to_dev false) or on the device,
// copying those that lack a valid copy there (under the slot's transfer lock,
// so two devices never move the same plane at once).  `exclusive` leaves the
// copies only where they were brought (the basic mode, which reuses nothing).
int stage(Run &r, Slot &sl, uint8_t mask, bool to_dev, hipStream_t s, bool exclusive = false) {
    const uint8_t want = to_dev ? ON_DEV : ON_HOST;
    std::lock_guard<std::mutex> xg(sl.xfer_mu);
    uint8_t moved = 0;
    const auto t0 = Clock::now();
    int64_t bytes = 0;
    for (int p = 0; p < NPLANES; ++p) {
        if (!(mask & (1u << p)) || (sl.where[p].load() & want)) continue;
        int rc = move_plane(r, sl, p, to_dev, s);
        if (rc) return rc;
        moved |= (uint8_t)(1u << p);
        bytes += (int64_t)r.tiles[sl.tile].height * r.tiles[sl.tile].width * (p == PL ? 4 : 1);
    }
    if (!moved) return RECON_OK;
    int rc = sync_stream(r, s);
    if (rc) return rc;
    for (int p = 0; p < NPLANES; ++p)
        if (moved & (1u << p)) sl.where[p].store(exclusive ? want : (uint8_t)(sl.where[p].load() | want));
    const double ms = ms_since(t0);
    std::lock_guard<std::mutex> g(r.mu);
    const int n = __builtin_popcount(moved);
    if (to_dev) {
        r.st.uploads += n;
        r.st.upload_bytes += bytes;
    } else {
        r.st.downloads += n;
        r.st.download_bytes += bytes;
    }
    r.st.transfer_ms += ms;
    return RECON_OK;
}

recon_image dev_image(Run &r, Slot &sl, int p) {
    recon_image im;
    im.data = sl.d[p];
    im.height = r.tiles[sl.tile].height;
    im.width = r.tiles[sl.tile].width;
    im.pitch = r.pitch;
    return im;
}

// Enqueue the GPU variant of op on stream s (nothing waits for it).
int gpu_enqueue(Run &r, Slot &sl, int op, hipStream_t s) {
    const recon_pipe_config &c = r.cfg;
    recon_image a = dev_image(r, sl, PA);
    int rc = RECON_OK;
    switch (op) {
        case RECON_PIPE_HDOME: rc = recon_hdome(r.ctx, &a, c.h, c.conn, s); break;
        case RECON_PIPE_FILL: rc = recon_fill_holes(r.ctx, &a, c.conn, s); break;
        case RECON_PIPE_AREA: rc = recon_area_threshold(r.ctx, &a, c.conn, c.area_min, c.area_max, s); break;
        case RECON_PIPE_MARKERS: {
            recon_image b = dev_image(r, sl, PB);
            PIPE_HIP(r, hipMemcpy2DAsync(b.data, r.pitch, a.data, r.pitch, a.width, a.height,
                                         hipMemcpyDeviceToDevice, s));
            rc = recon_pre_watershed(r.ctx, &b, c.conn, s);
            break;
        }
        case RECON_PIPE_LABEL:
            rc = recon_label(r.ctx, &a, (int32_t *)sl.d[PL], r.lpitch, c.conn, sl.d_count, s);
            break;
    }
    if (rc) return set_err(r, rc, "GPU operation %d failed: %s", op, recon_last_error());
    return RECON_OK;
}

// Enqueue one launch of op (h-dome or fill-holes) over the slots' A planes.
int gpu_enqueue_batch(Run &r, const std::vector<int> &slots, int op, hipStream_t s) {
    std::vector<recon_task> tasks(slots.size());
    for (size_t k = 0; k < slots.size(); ++k) {
        recon_task &t = tasks[k];
        t = recon_task{};
        t.op = op == RECON_PIPE_HDOME ? RECON_OP_HDOME : RECON_OP_FILL_HOLES;
        t.conn = r.cfg.conn;
        t.image = dev_image(r, r.slots[slots[k]], PA);
        t.h = op == RECON_PIPE_HDOME ? r.cfg.h : 0;
    }
    const int rc = recon_batch(r.ctx, tasks.data(), (int32_t)tasks.size(), s);
    if (rc) return set_err(r, rc, "GPU batch of operation %d failed: %s", op, recon_last_error());
    return RECON_OK;
}

int cpu_compute(Run &r, Slot &sl, int op, hostops::Scratch *scr) {
    const recon_pipe_config &c = r.cfg;
    const recon_pipe_tile &t = r.tiles[sl.tile];
    hostops::Plane a{sl.h[PA], t.height, t.width, r.pitch};
    try {
        switch (op) {
            case RECON_PIPE_HDOME: hostops::hdome(scr, a, c.h, c.conn); break;
            case RECON_PIPE_FILL: hostops::fill_holes(scr, a, c.conn); break;
            case RECON_PIPE_AREA: hostops::area_threshold(scr, a, c.conn, c.area_min, c.area_max); break;
            case RECON_PIPE_MARKERS: {
                hostops::Plane b{sl.h[PB], t.height, t.width, r.pitch};
                for (int y = 0; y < t.height; ++y) std::memcpy(b.row(y), a.row(y), t.width);
                hostops::pre_watershed(scr, b, c.conn);
                break;
            }
            case RECON_PIPE_LABEL:
                sl.h_count = hostops::label(scr, a, (int32_t *)sl.h[PL], r.lpitch, c.conn);
                break;
        }
    } catch (const std::exception &e) {
        return set_err(r, RECON_ENOMEM, "CPU operation %d failed: %s", op, e.what());
    }
    return RECON_OK;
}

// ---- admission and the ready list

// Reserve free slots for the next tiles (under r.mu); returns the slots whose
// image the caller copies in (outside the lock) before calling release_loaded.
std::vector<int> reserve(Run &r) {
    std::vector<int> got;
    for (int k = 0; k < r.nslots && r.next_tile < r.n; ++k) {
        Slot &sl = r.slots[k];
        if (sl.tile >= 0) continue;
        sl.tile = r.next_tile++;
        got.push_back(k);
    }
    return got;
}

// Copy `rows` rows of `row_bytes` between pitched planes: one copy when both
// are contiguous (a large copy streams past the caches; row by row it would
// read every destination line first).
void copy_rows(void *dst, int64_t dst_pitch, const void *src, int64_t src_pitch, size_t row_bytes, int rows) {
    if (dst_pitch == (int64_t)row_bytes && src_pitch == (int64_t)row_bytes) {
        std::memcpy(dst, src, row_bytes * (size_t)rows);
        return;
    }
    for (int y = 0; y < rows; ++y)
        std::memcpy((uint8_t *)dst + (int64_t)y * dst_pitch, (const uint8_t *)src + (int64_t)y * src_pitch, row_bytes);
}

// Copy the tile's image into the slot's pinned plane and reset its counters.
void load(Run &r, int k) {
    Slot &sl = r.slots[k];
    const recon_pipe_tile &t = r.tiles[sl.tile];
    copy_rows(sl.h[PA], r.pitch, t.image, t.pitch, (size_t)t.width, t.height);
    sl.where[PA].store(ON_HOST);
    sl.where[PB].store(0);
    sl.where[PL].store(0);
    sl.left = RECON_PIPE_NOPS;
    for (int o = 0; o < RECON_PIPE_NOPS; ++o) sl.waiting[o] = kOps[o].deps;
}

// Admit the next tiles into free slots.  With prefetching (and a GPU) the
// admitting thread also uploads each image to the slot's device plane on its
// stream `s` before the tile's first operation is queued, so that the GPU
// finds it resident (the paper's prefetching of inputs, Sec. IV-D).
int load_slot(Run &r, int k, hipStream_t s) {
    load(r, k);
    return r.cfg.prefetch && r.cfg.use_gpu ? stage(r, r.slots[k], 1u << PA, true, s) : RECON_OK;
}

// Queue the first operation of the loaded slots, in order (under r.mu).
void queue_first(Run &r, const std::vector<int> &got) {
    for (int k : got) r.ready.push_back({k, RECON_PIPE_HDOME, r.seq++, r.cfg.speedup[RECON_PIPE_HDOME]});
    if (!got.empty()) {
        r.ready_gen.fetch_add(1);
        r.cv.notify_all();
    }
}

int admit(Run &r, hipStream_t s) {
    std::vector<int> got;
    {
        std::lock_guard<std::mutex> g(r.mu);
        got = reserve(r);
    }
    for (int k : got) {
        int rc = load_slot(r, k, s);
        if (rc) return rc;
    }
    std::lock_guard<std::mutex> g(r.mu);
    queue_first(r, got);
    return RECON_OK;
}

// The first window of tiles: loaded (and prefetched) on the I/O threads'
// streams side by side, then queued together in tile order, before any device
// starts (so the order in which the devices see them does not depend on
// which load ends first).
int admit_first(Run &r, const std::vector<hipStream_t> &streams) {
    std::vector<int> got;
    {
        std::lock_guard<std::mutex> g(r.mu);
        got = reserve(r);
    }
    std::atomic<size_t> next{0};
    std::atomic<int> rc{RECON_OK};
    auto body = [&](hipStream_t s) {
        if (r.cfg.use_gpu && hipSetDevice(r.device) != hipSuccess) {
            rc = set_err(r, RECON_EDEVICE, "hipSetDevice failed in a pipeline thread");
            return;
        }
        for (size_t i; rc == RECON_OK && (i = next++) < got.size();) {
            const int e = load_slot(r, got[i], s);
            if (e) rc = e;
        }
    };
    std::vector<std::thread> th;
    for (size_t k = 1; k < streams.size() && k < got.size(); ++k) th.emplace_back(body, streams[k]);
    body(streams[0]);
    for (auto &t : th) t.join();
    if (rc != RECON_OK) return rc;
    std::lock_guard<std::mutex> g(r.mu);
    queue_first(r, got);
    return RECON_OK;
}

bool resident(const Run &r, const Ready &x) {
    const Slot &sl = r.slots[x.slot];
    for (int p = 0; p < NPLANES; ++p)
        if ((kOps[x.op].in_mask & (1u << p)) && !(sl.where[p].load() & ON_DEV)) return false;
    return true;
}

// Index (in r.ready) of the instance the device takes next, or -1 (under r.mu).
int pick(const Run &r, bool gpu) {
    const auto &q = r.ready;
    if (q.empty()) return -1;
    const bool pats = r.cfg.policy == RECON_SCHED_PATS;
    auto before = [&](const Ready &a, const Ready &b) {
        if (pats && a.speedup != b.speedup) return gpu ? a.speedup > b.speedup : a.speedup < b.speedup;
        return a.seq < b.seq;
    };
    // a CPU worker may be kept off the instances a core would take too long on:
    // above a speedup limit, or (guard) longer than the GPU's remaining work
    const float limit = gpu ? 0.0f : r.cfg.cpu_max_speedup;
    const bool guard = !gpu && r.cfg.cpu_guard && r.cfg.use_gpu;
    auto allowed = [&](const Ready &x) {
        if (limit > 0.0f && x.speedup > limit) return false;
        if (guard && (double)x.speedup * r.cfg.gpu_ms[x.op] > r.gpu_left_ms - r.cfg.gpu_ms[x.op]) return false;
        return true;
    };
    int best = -1;
    for (int i = 0; i < (int)q.size(); ++i)
        if (allowed(q[i]) && (best < 0 || before(q[i], q[best]))) best = i;
    if (!gpu || !r.cfg.data_locality || best < 0) return best;
    // data locality: the preferred instance among those whose inputs are in
    // device memory already
    int local = -1;
    for (int i = 0; i < (int)q.size(); ++i)
        if (resident(r, q[i]) && (local < 0 || before(q[i], q[local]))) local = i;
    if (local < 0 || local == best) return best;
    if (!pats) return local;   // without speedup estimates, reuse the data
    const float impact = r.cfg.transfer_impact[q[best].op];
    return q[local].speedup >= q[best].speedup * (1.0f - impact) ? local : best;
}

// Mark op of the slot done and queue the operations it releases (under r.mu);
// true if it was the tile's last.
bool complete(Run &r, int slot, int op) {
    Slot &sl = r.slots[slot];
    for (int k = 0; k < 2; ++k) {
        const int nx = kOps[op].next[k];
        if (nx >= 0 && --sl.waiting[nx] == 0) {
            r.ready.push_back({slot, nx, r.seq++, r.cfg.speedup[nx]});
            r.ready_gen.fetch_add(1);
        }
    }
    return --sl.left == 0;
}

// The tile's last operation finished: bring its results to the host, copy them
// out, free the slot and admit the next tile (whose image is copied into the
// slot's pinned plane here, ahead of its first operation).
int finish_tile(Run &r, int slot, hipStream_t s) {
    const auto t0 = Clock::now();
    Slot &sl = r.slots[slot];
    int rc = stage(r, sl, (1u << PA) | (1u << PB) | (1u << PL), false, s);
    if (rc) return rc;
    const recon_pipe_tile &t = r.tiles[sl.tile];
    if (t.objects) copy_rows(t.objects, t.pitch, sl.h[PA], r.pitch, (size_t)t.width, t.height);
    if (t.markers) copy_rows(t.markers, t.pitch, sl.h[PB], r.pitch, (size_t)t.width, t.height);
    if (t.labels) copy_rows(t.labels, t.label_pitch * 4, sl.h[PL], r.lpitch * 4, (size_t)t.width * 4, t.height);
    if (t.count) *t.count = sl.h_count;
    {
        std::lock_guard<std::mutex> g(r.mu);
        sl.tile = -1;
        ++r.done_tiles;
        r.cv.notify_all();
    }
    rc = admit(r, s);
    std::lock_guard<std::mutex> g(r.mu);
    r.st.io_ms += ms_since(t0);
    return rc;
}

// Tile completion and admission run on their own threads (the paper's
// asynchronous download and prefetch of Sec. IV-D), so that neither the GPU
// manager nor a CPU worker spends its time copying whole tiles.
void io_thread(Run &r, hipStream_t s) {
    if (r.cfg.use_gpu && hipSetDevice(r.device) != hipSuccess) {
        set_err(r, RECON_EDEVICE, "hipSetDevice failed in a pipeline thread");
        return;
    }
    while (true) {
        int slot;
        {
            std::unique_lock<std::mutex> lk(r.mu);
            r.cv.wait(lk, [&] { return r.err || r.done_tiles == r.n || !r.finished.empty(); });
            if (r.err || r.done_tiles == r.n) return;
            slot = r.finished.back();
            r.finished.pop_back();
        }
        if (finish_tile(r, slot, s)) return;
    }
}

// Take ready instance i for device `dev` (under r.mu): remove it from the
// ready list, count its estimated GPU time out of the remaining work and open
// its trace entry (returned, or -1).
int64_t take(Run &r, int i, const Device &dev, int &slot, int &op) {
    slot = r.ready[i].slot;
    op = r.ready[i].op;
    r.ready.erase(r.ready.begin() + i);
    r.gpu_left_ms -= r.cfg.gpu_ms[op];
    int64_t ev = -1;
    if (r.cfg.trace && r.st.trace_n < r.cfg.trace_cap) {
        ev = r.st.trace_n++;
        recon_pipe_event &e = r.cfg.trace[ev];
        e.tile = r.slots[slot].tile;
        e.op = op;
        e.device = dev.id;
        e.reserved = 0;
        e.start_ms = ms_since(r.t0);
        e.end_ms = -1.0;
    }
    return ev;
}

// An instance's outputs were written on `dev`: an in-place write leaves the
// only valid copy where it was made.
void outputs_written(Slot &sl, int op, const Device &dev) {
    std::lock_guard<std::mutex> xg(sl.xfer_mu);
    for (int p = 0; p < NPLANES; ++p)
        if (kOps[op].out_mask & (1u << p)) sl.where[p].store(dev.gpu ? ON_DEV : ON_HOST);
}

// The instance of op on the slot has finished on `dev` (computation time ms)
// and its outputs' location is recorded: mark it done (releasing its
// successors; the tile's last instance hands the tile to the I/O threads).
void finish_instance(Run &r, const Device &dev, int slot, int op, int64_t ev, double ms) {
    bool last;
    {
        std::lock_guard<std::mutex> g(r.mu);
        if (ev >= 0) r.cfg.trace[ev].end_ms = ms_since(r.t0);
        if (dev.gpu) {
            r.st.ops_gpu[op]++;
            r.st.busy_gpu_ms[op] += ms;
        } else {
            r.st.ops_cpu[op]++;
            r.st.busy_cpu_ms[op] += ms;
        }
        last = complete(r, slot, op);
        if (last) r.finished.push_back(slot);
        r.cv.notify_all();
    }
}

void worker(Run &r, Device dev) {
    if (r.cfg.use_gpu && hipSetDevice(r.device) != hipSuccess) {
        set_err(r, RECON_EDEVICE, "hipSetDevice failed in a pipeline thread");
        return;
    }
    while (true) {
        int slot, op;
        int64_t ev;
        {
            std::unique_lock<std::mutex> lk(r.mu);
            int i = -1;
            r.cv.wait(lk, [&] { return r.err || r.done_tiles == r.n || (i = pick(r, false)) >= 0; });
            if (r.err || r.done_tiles == r.n) return;
            ev = take(r, i, dev, slot, op);
        }
        Slot &sl = r.slots[slot];
        if (stage(r, sl, kOps[op].in_mask, false, dev.stream)) return;
        const auto t0 = Clock::now();
        if (cpu_compute(r, sl, op, dev.scratch)) return;
        const double ms = ms_since(t0);
        outputs_written(sl, op, dev);
        finish_instance(r, dev, slot, op, ev, ms);
    }
}

// The GPU manager.  Instances are enqueued on the manager's stream, at most
// cfg.gpu_inflight at once, each followed by a write of its launch's outcome
// into pinned memory and an event; the oldest is retired once its event has
// completed.  Inputs are staged on a separate transfer stream (waited for
// before the instance is enqueued), so a transfer never waits behind the
// instances already enqueued.  Its time per instance runs from the later of
// its enqueue and the previous instance's completion to its own completion.
void gpu_manager(Run &r, Device dev) {
    if (hipSetDevice(r.device) != hipSuccess) {
        set_err(r, RECON_EDEVICE, "hipSetDevice failed in a pipeline thread");
        return;
    }
    const int depth = std::max(1, (int)r.cfg.gpu_inflight);
    const bool basic = !r.cfg.data_locality;
    const int batch = std::max(1, (int)r.cfg.gpu_batch);
    struct Inst {
        int slot;
        int64_t ev;
    };
    struct Issued {   // one launch: instances of one operation
        std::vector<Inst> insts;
        int op, k;
        Clock::time_point t_enq;
    };
    std::vector<hipEvent_t> done(depth, nullptr);
    uint32_t *outcome = nullptr;   // pinned, one word per in-flight position
    bool ok = hipHostMalloc((void **)&outcome, (size_t)depth * sizeof(uint32_t), hipHostMallocDefault) == hipSuccess;
    for (int k = 0; ok && k < depth; ++k)
        ok = hipEventCreateWithFlags(&done[k], hipEventDisableTiming) == hipSuccess;
    std::deque<Issued> q;
    std::vector<int> free_k;
    for (int k = depth - 1; k >= 0; --k) free_k.push_back(k);
    Clock::time_point last_done = Clock::now();
    if (!ok) set_err(r, RECON_EDEVICE, "GPU manager: event or pinned allocation failed");

    // retire the oldest instance (its event has completed); false on an error
    auto retire = [&]() -> bool {
        const Issued x = q.front();
        q.pop_front();
        free_k.push_back(x.k);
        const auto now = Clock::now();
        const double ms =
            std::chrono::duration<double, std::milli>(now - std::max(x.t_enq, last_done)).count();
        last_done = now;
        if (((volatile uint32_t *)outcome)[x.k] != 0) {
            set_err(r, RECON_EDEVICE, "GPU operation %d: the scheduler watchdog gave the launch up", x.op);
            return false;
        }
        for (const Inst &in_x : x.insts) {
            Slot &sl = r.slots[in_x.slot];
            outputs_written(sl, x.op, dev);
            if (basic) {
                // the basic mode brings every GPU assignment's outputs back to the
                // host (and its inputs in again next time): no data stays on the device
                const uint8_t in = kOps[x.op].in_mask;
                if (stage(r, sl, kOps[x.op].out_mask, false, dev.xfer, true)) return false;
                std::lock_guard<std::mutex> xg(sl.xfer_mu);
                for (int p = 0; p < NPLANES; ++p)
                    if (in & (1u << p)) sl.where[p].store(sl.where[p].load() & (uint8_t)~ON_DEV);
            }
            // a launch's time is shared by its instances
            finish_instance(r, dev, in_x.slot, x.op, in_x.ev, ms / (double)x.insts.size());
        }
        return true;
    };

    while (ok) {
        if (!q.empty()) {
            const hipError_t e = hipEventQuery(done[q.front().k]);
            if (e == hipSuccess) {
                if (!retire()) break;
                continue;
            }
            if (e != hipErrorNotReady) {
                set_err(r, RECON_EDEVICE, "GPU manager stream failed: %s", hipGetErrorString(e));
                break;
            }
        }
        // take another instance while there is room (blocking only when none is
        // in flight); a reconstruction takes the other ready instances of its
        // operation along, up to the batch size, oldest first
        int slot = -1, op = -1;
        std::vector<Inst> group;
        const uint64_t gen = r.ready_gen.load();
        if ((int)q.size() < depth) {
            std::unique_lock<std::mutex> lk(r.mu);
            int i = -1;
            if (q.empty())
                r.cv.wait(lk, [&] { return r.err || r.done_tiles == r.n || (i = pick(r, true)) >= 0; });
            else if (!r.err)
                i = pick(r, true);
            if (r.err || (q.empty() && r.done_tiles == r.n)) break;
            if (i >= 0) {
                int64_t ev = take(r, i, dev, slot, op);
                group.push_back({slot, ev});
                if (batch > 1 && (op == RECON_PIPE_HDOME || op == RECON_PIPE_FILL)) {
                    std::vector<int> more;   // indices into r.ready, oldest first
                    for (int j = 0; j < (int)r.ready.size(); ++j)
                        if (r.ready[j].op == op) more.push_back(j);
                    std::sort(more.begin(), more.end(),
                              [&](int a, int b) { return r.ready[a].seq < r.ready[b].seq; });
                    if ((int)more.size() > batch - 1) more.resize(batch - 1);
                    // take from the back so that the remaining indices stay valid
                    std::sort(more.begin(), more.end(), [](int a, int b) { return a > b; });
                    for (int j : more) {
                        int s2, o2;
                        const int64_t e2 = take(r, j, dev, s2, o2);
                        group.push_back({s2, e2});
                    }
                }
            }
        }
        if (slot >= 0) {
            const int k = free_k.back();
            free_k.pop_back();
            bool staged = true;
            for (const Inst &g : group)
                if (stage(r, r.slots[g.slot], kOps[op].in_mask, true, dev.xfer)) {
                    staged = false;
                    break;
                }
            if (!staged) break;
            const auto t_enq = Clock::now();
            if (group.size() == 1) {
                if (gpu_enqueue(r, r.slots[slot], op, dev.stream)) break;
            } else {
                std::vector<int> slots;
                for (const Inst &g : group) slots.push_back(g.slot);
                if (gpu_enqueue_batch(r, slots, op, dev.stream)) break;
            }
            // the reconstructions (h-dome, fill-holes, the markers' regional
            // maxima) report a launch their scheduler gave up through its outcome
            if (op == RECON_PIPE_HDOME || op == RECON_PIPE_FILL || op == RECON_PIPE_MARKERS) {
                if (recon_enqueue_status(r.ctx, outcome + k, dev.stream) != RECON_OK) {
                    set_err(r, RECON_EDEVICE, "GPU operation %d: %s", op, recon_last_error());
                    break;
                }
            } else {
                outcome[k] = 0;
            }
            if (hipEventRecord(done[k], dev.stream) != hipSuccess) {
                set_err(r, RECON_EDEVICE, "GPU manager: event record failed");
                break;
            }
            q.push_back({std::move(group), op, k, t_enq});
            continue;
        }
        // wait for the oldest instance, or (with room) for newly ready ones:
        // polled without sleeping for 2 ms, then with short sleeps, 60 s at most
        const auto t_wait = Clock::now();
        while (true) {
            const hipError_t e = hipEventQuery(done[q.front().k]);
            if (e != hipErrorNotReady) break;
            if ((int)q.size() < depth && r.ready_gen.load() != gen) break;
            const double w = ms_since(t_wait);
            if (w > 60000.0) {
                set_err(r, RECON_ETIMEDOUT, "GPU manager: an instance did not finish within 60 s");
                ok = false;
                break;
            }
            if (w > 2.0) std::this_thread::sleep_for(std::chrono::microseconds(20));
        }
    }
    // leave nothing in flight behind: the slots' planes are freed after the run
    for (const Issued &x : q) (void)hipEventSynchronize(done[x.k]);
    for (hipEvent_t e : done)
        if (e) (void)hipEventDestroy(e);
    if (outcome) (void)hipHostFree(outcome);
}

int check_config(const recon_pipe_config *c, recon_ctx *ctx) {
    if (c->policy != RECON_SCHED_FCFS && c->policy != RECON_SCHED_PATS) return 1;
    if (c->cpu_workers < 0 || c->cpu_workers > 256 || c->window < 1 || c->window > 1024) return 1;
    if (c->io_threads < 0 || c->io_threads > 64) return 1;
    if (c->trace_cap < 0 || (c->trace_cap > 0 && !c->trace)) return 1;
    if (c->prefetch < 0 || c->prefetch > 1) return 1;
    if (c->gpu_inflight < 0 || c->gpu_inflight > 4 || c->gpu_batch < 0 || c->gpu_batch > 8) return 1;
    if (c->use_gpu && !ctx) return 1;
    if (!c->use_gpu && c->cpu_workers == 0) return 1;
    if (c->conn != 4 && c->conn != 8) return 1;
    if (c->h < 1 || c->h > 255 || c->area_min < 0 || c->area_max < c->area_min) return 1;
    if (!(c->cpu_max_speedup >= 0.0f) || c->cpu_guard < 0 || c->cpu_guard > 1) return 1;
    for (int o = 0; o < RECON_PIPE_NOPS; ++o)
        if (!(c->gpu_ms[o] >= 0.0f) || !(c->speedup[o] >= 0.0f)) return 1;
    // without a GPU the CPU workers must be able to take every operation
    if (!c->use_gpu && c->cpu_max_speedup > 0.0f)
        for (int o = 0; o < RECON_PIPE_NOPS; ++o)
            if (c->speedup[o] > c->cpu_max_speedup) return 1;
    return 0;
}

int invalid(const char *what) {
    g_pipe_err = what;
    return RECON_EINVAL;
}

}  // namespace

extern "C" const char *recon_pipeline_error(void) { return g_pipe_err.c_str(); }

extern "C" int recon_pipeline_run(recon_ctx *ctx, const recon_pipe_tile *tiles, int32_t n,
                                  const recon_pipe_config *cfg, recon_pipe_stats *stats) {
    if (!tiles || n < 0 || !cfg) return invalid("null tiles or configuration, or n < 0");
    if (check_config(cfg, ctx)) return invalid("bad pipeline configuration");
    Run r;
    r.ctx = ctx;
    r.tiles = tiles;
    r.n = n;
    r.cfg = *cfg;
    for (int i = 0; i < n; ++i) {
        const recon_pipe_tile &t = tiles[i];
        if (!t.image || t.height < 1 || t.width < 1 || t.pitch < t.width || t.height > 16384 || t.width > 16384 ||
            (t.labels && t.label_pitch < t.width))
            return invalid("bad tile shape, pitch or label pitch");
        r.H = std::max(r.H, t.height);
        r.W = std::max(r.W, t.width);
    }
    if (n == 0) {
        if (stats) *stats = recon_pipe_stats{};
        return RECON_OK;
    }
    r.pitch = (r.W + 255) / 256 * 256;
    r.lpitch = r.pitch;
    if (cfg->use_gpu && hipGetDevice(&r.device) != hipSuccess) {
        g_pipe_err = "hipGetDevice failed";
        return RECON_EDEVICE;
    }

    r.nslots = std::min(cfg->window, n);
    r.slots.reset(new Slot[r.nslots]);
    int rc = RECON_OK;
    for (int k = 0; k < r.nslots; ++k) {
        Slot &sl = r.slots[k];
        for (int p = 0; p < NPLANES && rc == RECON_OK; ++p) {
            if (cfg->use_gpu) {
                if (hipHostMalloc((void **)&sl.h[p], r.plane_bytes(p), hipHostMallocDefault) != hipSuccess ||
                    hipMalloc((void **)&sl.d[p], r.plane_bytes(p)) != hipSuccess)
                    rc = RECON_ENOMEM;
            } else {
                sl.h[p] = (uint8_t *)malloc(r.plane_bytes(p));
                if (!sl.h[p]) rc = RECON_ENOMEM;
            }
        }
        if (rc == RECON_OK && cfg->use_gpu && hipMalloc((void **)&sl.d_count, 4) != hipSuccess) rc = RECON_ENOMEM;
    }
    if (rc) r.err_msg = "allocation of the tile slots failed";
    std::vector<Device> devs;
    if (rc == RECON_OK && cfg->use_gpu) {
        Device g;
        g.gpu = true;
        if (hipStreamCreateWithFlags(&g.stream, hipStreamNonBlocking) != hipSuccess ||
            hipStreamCreateWithFlags(&g.xfer, hipStreamNonBlocking) != hipSuccess)
            rc = RECON_EDEVICE;
        devs.push_back(g);
    }
    for (int k = 0; rc == RECON_OK && k < cfg->cpu_workers; ++k) {
        Device c;
        c.gpu = false;
        c.id = 1 + k;
        c.scratch = hostops::scratch_new();
        if (cfg->use_gpu && hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking) != hipSuccess)
            rc = RECON_EDEVICE;
        devs.push_back(c);
    }
    const int n_io = cfg->io_threads > 0 ? cfg->io_threads : 2;
    std::vector<hipStream_t> io_streams(n_io, nullptr);
    for (int k = 0; rc == RECON_OK && cfg->use_gpu && k < n_io; ++k)
        if (hipStreamCreateWithFlags(&io_streams[k], hipStreamNonBlocking) != hipSuccess) rc = RECON_EDEVICE;
    if (rc && r.err_msg.empty()) r.err_msg = "stream creation failed";
    for (int o = 0; o < RECON_PIPE_NOPS; ++o) r.gpu_left_ms += (double)n * cfg->gpu_ms[o];
    if (rc == RECON_OK) {
        const auto t0 = Clock::now();
        r.t0 = t0;
        // the first tiles are admitted here, before the devices and the I/O threads start
        if (admit_first(r, io_streams) != RECON_OK) r.cv.notify_all();
        std::vector<std::thread> th;
        for (auto &d : devs) th.emplace_back(d.gpu ? gpu_manager : worker, std::ref(r), d);
        for (int k = 0; k < n_io; ++k) th.emplace_back(io_thread, std::ref(r), io_streams[k]);
        for (auto &t : th) t.join();
        r.st.makespan_ms = ms_since(t0);
        rc = r.err;
    }
    for (hipStream_t st : io_streams)
        if (st) (void)hipStreamDestroy(st);
    for (auto &d : devs) {
        if (d.stream) (void)hipStreamDestroy(d.stream);
        if (d.xfer) (void)hipStreamDestroy(d.xfer);
        if (d.scratch) hostops::scratch_free(d.scratch);
    }
    for (int k = 0; k < r.nslots; ++k) {
        Slot &sl = r.slots[k];
        for (int p = 0; p < NPLANES; ++p) {
            if (cfg->use_gpu) {
                if (sl.h[p]) (void)hipHostFree(sl.h[p]);
                if (sl.d[p]) (void)hipFree(sl.d[p]);
            } else {
                free(sl.h[p]);
            }
        }
        if (sl.d_count) (void)hipFree(sl.d_count);
    }
    g_pipe_err = rc == RECON_OK ? std::string() : r.err_msg;
    if (stats) *stats = r.st;
    return rc;
}

extern "C" int recon_pipeline_host_op(int op, recon_image *img, const recon_pipe_config *cfg, int32_t *labels,
                                      int64_t label_pitch, int32_t *count) {
    if (!img || !img->data || !cfg || img->height < 1 || img->width < 1 || img->pitch < img->width)
        return invalid("null image or configuration, or bad shape or pitch");
    if (cfg->conn != 4 && cfg->conn != 8) return invalid("conn must be 4 or 8");
    if (op == RECON_PIPE_HDOME && (cfg->h < 1 || cfg->h > 255)) return invalid("h must be in 1..255");
    if (op == RECON_PIPE_AREA && (cfg->area_min < 0 || cfg->area_max < cfg->area_min))
        return invalid("bad area bounds");
    if (op == RECON_PIPE_LABEL && (!labels || label_pitch < img->width)) return invalid("bad labels plane");
    if (op < 0 || op >= RECON_PIPE_NOPS) return invalid("unknown pipeline operation");
    hostops::Scratch *s = hostops::scratch_new();
    hostops::Plane a{img->data, img->height, img->width, img->pitch};
    int rc = RECON_OK;
    try {
        switch (op) {
            case RECON_PIPE_HDOME: hostops::hdome(s, a, cfg->h, cfg->conn); break;
            case RECON_PIPE_FILL: hostops::fill_holes(s, a, cfg->conn); break;
            case RECON_PIPE_AREA: hostops::area_threshold(s, a, cfg->conn, cfg->area_min, cfg->area_max); break;
            case RECON_PIPE_MARKERS: hostops::pre_watershed(s, a, cfg->conn); break;
            case RECON_PIPE_LABEL: {
                const int32_t c = hostops::label(s, a, labels, label_pitch, cfg->conn);
                if (count) *count = c;
                break;
            }
        }
    } catch (const std::exception &e) {
        g_pipe_err = e.what();
        rc = RECON_ENOMEM;
    }
    hostops::scratch_free(s);
    if (rc == RECON_OK) g_pipe_err.clear();
    return rc;
}
