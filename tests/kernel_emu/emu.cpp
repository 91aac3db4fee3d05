// Host emulation of the librecon kernels (test infrastructure, CPU only).
//
// Compiles paper_1209_3332_amd/csrc/kernels.hpp against the stand-in
// hip/hip_runtime.h next to this file and runs the same launch sequence as the
// library (reset -> fill init -> persistent kernel -> fill finish) on host
// memory.  Each workgroup (one 64-lane wave) runs on its own OS thread, its
// lanes as fibers switched at every cross-lane operation, so inter-wave
// atomics and the block scheduler run with real concurrency.  Every LDS
// buffer and every image copy is an exact-size heap allocation, so a build
// with -fsanitize=address bounds-checks all of the kernels' memory accesses.
#include "hip/hip_runtime.h"


#include <cstdio>
#include <cstdlib>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

#include "../../paper_1209_3332_amd/csrc/kernels.hpp"
#include "../../paper_1209_3332_amd/csrc/label.hpp"
#include "../../paper_1209_3332_amd/csrc/component.hpp"
#include "../../paper_1209_3332_amd/csrc/distance.hpp"

#if defined(__has_feature)
#if __has_feature(address_sanitizer)
#define KEMU_ASAN 1
#include <sanitizer/common_interface_defs.h>
#endif
#endif

namespace kemu {

thread_local Dim3 blockIdx_, threadIdx_, blockDim_, gridDim_;

// Minimal fiber switch for x86-64 SysV: push the callee-saved registers on
// the current stack, store the stack pointer in *from, load *to, pop, return.
// (glibc's swapcontext also saves the signal mask with a system call on every
// switch, which made emulation two orders of magnitude slower.)
extern "C" void kemu_switch(void **from, void *to);
asm(R"(
.text
.globl kemu_switch
.type kemu_switch,@function
kemu_switch:
    pushq %rbp
    pushq %rbx
    pushq %r12
    pushq %r13
    pushq %r14
    pushq %r15
    movq %rsp, (%rdi)
    movq %rsi, %rsp
    popq %r15
    popq %r14
    popq %r13
    popq %r12
    popq %rbx
    popq %rbp
    ret
.size kemu_switch,.-kemu_switch
)");

constexpr int kLanes = 64;
constexpr size_t kStack = 512 * 1024;

struct Wave {
    void *sched_sp = nullptr;
    void *sp[kLanes] = {};
    std::vector<char *> stacks;
    int cur = 0;
    bool finished[kLanes] = {};
    int parity[kLanes] = {};
    uint64_t xch[2][kLanes] = {};
    uint8_t *lds = nullptr;
    size_t lds_size = 0;
    std::function<void()> body;
    const void *sched_bottom = nullptr;
    size_t sched_size = 0;
    void *fake[kLanes + 1] = {};
    bool error = false;
};

thread_local Wave *tw = nullptr;

int lane() { return tw->cur; }
// The lanes of an emulated wave share one OS thread, so a thread_local index
// cannot tell them apart: inside a wave the thread index is the lane.
Dim3 thread_idx() {
    if (tw) return Dim3{(uint32_t)tw->cur, 0, 0};
    return threadIdx_;
}
uint8_t *wave_lds() { return tw->lds; }

uint64_t wall_ticks() {
    using namespace std::chrono;
    return (uint64_t)duration_cast<nanoseconds>(steady_clock::now().time_since_epoch()).count() / 10;
}

void check_lds(const void *p, size_t n) {
    const uint8_t *q = (const uint8_t *)p;
    if (q < tw->lds || q + n > tw->lds + tw->lds_size) {
        std::fprintf(stderr, "kemu: LDS atomic out of bounds (offset %ld)\n", (long)(q - tw->lds));
        std::abort();
    }
}

// lane -> scheduler switch
static void yield_to_sched() {
    Wave *w = tw;
    const int l = w->cur;
#ifdef KEMU_ASAN
    __sanitizer_start_switch_fiber(&w->fake[l], w->sched_bottom, w->sched_size);
#endif
    kemu_switch(&w->sp[l], w->sched_sp);
#ifdef KEMU_ASAN
    __sanitizer_finish_switch_fiber(w->fake[l], nullptr, nullptr);
#endif
}

void wave_sync() { yield_to_sched(); }

uint64_t exchange(uint64_t v, int src) {
    Wave *w = tw;
    const int l = w->cur;
    const int p = w->parity[l];
    w->xch[p][l] = v;
    w->parity[l] = p ^ 1;
    yield_to_sched();
    if (src < 0 || src >= kLanes) {
        std::fprintf(stderr, "kemu: shuffle from lane %d\n", src);
        std::abort();
    }
    return w->xch[p][src];
}

uint64_t ballot(bool pred) {
    Wave *w = tw;
    const int l = w->cur;
    const int p = w->parity[l];
    w->xch[p][l] = pred ? 1u : 0u;
    w->parity[l] = p ^ 1;
    yield_to_sched();
    uint64_t m = 0;
    for (int k = 0; k < kLanes; ++k)
        if (w->xch[p][k]) m |= 1ull << k;
    return m;
}

[[noreturn]] static void lane_entry() {
    Wave *w = tw;
#ifdef KEMU_ASAN
    __sanitizer_finish_switch_fiber(nullptr, &w->sched_bottom, &w->sched_size);
#endif
    w->body();
    w->finished[w->cur] = true;
    void *dead = nullptr;
#ifdef KEMU_ASAN
    __sanitizer_start_switch_fiber(nullptr, w->sched_bottom, w->sched_size);
#endif
    kemu_switch(&dead, w->sched_sp);
    __builtin_unreachable();
}

// Run `body` as one 64-lane wave on the calling thread.
static bool run_wave(const std::function<void()> &body, size_t lds_size) {
    Wave w;
    w.body = body;
    w.lds_size = lds_size;
    w.lds = (uint8_t *)std::malloc(lds_size);
    std::memset(w.lds, 0xcd, lds_size);   // garbage, like fresh LDS
    tw = &w;
    for (int l = 0; l < kLanes; ++l) {
        char *st = (char *)std::malloc(kStack);
        w.stacks.push_back(st);
        // initial frame: six callee-saved registers (zero) and the entry point as return address
        uintptr_t top = ((uintptr_t)(st + kStack) & ~(uintptr_t)15) - 8;   // entry sees rsp % 16 == 8
        void **sp = (void **)top;
        *--sp = (void *)&lane_entry;
        for (int k = 0; k < 6; ++k) *--sp = nullptr;
        w.sp[l] = sp;
    }
    bool ok = true;
    while (true) {
        int alive = 0, done = 0;
        for (int l = 0; l < kLanes; ++l) {
            if (w.finished[l]) { ++done; continue; }
            w.cur = l;
#ifdef KEMU_ASAN
            __sanitizer_start_switch_fiber(&w.fake[kLanes], w.stacks[l], kStack);
#endif
            kemu_switch(&w.sched_sp, w.sp[l]);
#ifdef KEMU_ASAN
            __sanitizer_finish_switch_fiber(w.fake[kLanes], nullptr, nullptr);
#endif
            if (!w.finished[l]) ++alive;
        }
        if (alive == 0) break;
        if (done > 0 && alive > 0) {   // some lanes returned while others wait at a collective
            std::fprintf(stderr, "kemu: non-uniform exit of a wave\n");
            ok = false;
            break;
        }
    }
    for (char *st : w.stacks) std::free(st);
    std::free(w.lds);
    tw = nullptr;
    return ok;
}

}  // namespace kemu

// ---------------------------------------------------------------------------
// labelling driver: the phases of recon_label / recon_area_threshold in
// order, each as a grid of emulated waves on concurrent threads.

static int emu_label(const uint8_t *img_in, int h, int w, int conn, int n_waves, int32_t *labels_out,
                     int32_t *count_out, int64_t min_area, int64_t max_area, uint8_t *area_out) {
    using namespace rk;
    // exact-size copies (the sanitizer bounds-checks every access); the label
    // plane has a padded pitch so that pitched node ids are exercised
    const int64_t pitch_img = w + 3, pitch_lab = (w + 3) / 4 * 4 + 4;   // 16-byte rows: vector path
    std::vector<uint8_t> img((size_t)h * pitch_img, 0);
    for (int y = 0; y < h; ++y) std::memcpy(&img[(size_t)y * pitch_img], img_in + (size_t)y * w, w);
    int32_t *lab = (int32_t *)std::malloc((size_t)((h - 1) * pitch_lab + w) * sizeof(int32_t));
    LabelArgs a{};
    a.img = img.data() + 0;
    a.pitch_img = pitch_img;
    a.lab = lab;
    a.pitch_lab = pitch_lab;
    a.h = h;
    a.w = w;
    a.conn = conn;
    a.tiles_x = (w + LT_W - 1) / LT_W;
    const uint64_t nbits = (uint64_t)(h - 1) * pitch_lab + w;
    a.n_words = (uint32_t)((nbits + 31) / 32);
    a.n_segs = (a.n_words + RANK_SEG - 1) / RANK_SEG;
    a.bits = (uint32_t *)std::malloc(a.n_words * 4);
    a.word_off = (uint32_t *)std::malloc(a.n_words * 4);
    a.seg_sum = (uint32_t *)std::malloc(a.n_segs * 4);
    int32_t count = -1;
    a.count = &count;
    a.lab_vec = (((uintptr_t)lab | (uintptr_t)(pitch_lab * 4)) & 15u) == 0 ? 1 : 0;
    auto serial = [&](auto fn, uint32_t blocks, uint32_t threads) {
        kemu::gridDim_.x = blocks;
        kemu::blockDim_.x = threads;
        for (uint32_t b = 0; b < blocks; ++b)
            for (uint32_t t = 0; t < threads; ++t) {
                kemu::blockIdx_.x = b;
                kemu::threadIdx_.x = t;
                fn();
            }
    };
    std::atomic<int> bad{0};
    auto waves = [&](int nw, size_t lds, const std::function<void()> &body) {
        std::vector<std::thread> th;
        for (int g = 0; g < nw; ++g)
            th.emplace_back([&, g] {
                kemu::blockIdx_.x = (uint32_t)g;
                kemu::gridDim_.x = (uint32_t)nw;
                kemu::blockDim_.x = 64;
                if (!kemu::run_wave(body, lds)) bad++;
            });
        for (auto &t : th) t.join();
    };
    serial([&] { clear_words(a.bits, a.n_words); }, 2, 64);
    waves(n_waves, (size_t)LT_H * LT_W * 4, [&] { label_local(a); });
    waves(n_waves, 0, [&] { label_merge(a); });
    waves(n_waves, 0, [&] { label_flatten(a); });
    std::vector<int32_t> roots((size_t)((h - 1) * pitch_lab + w));   // the flattened plane (root ids)
    std::memcpy(roots.data(), lab, roots.size() * 4);
    waves(n_waves, 0, [&] { rank_segments(a); });
    waves(1, 0, [&] { rank_scan(a); });
    waves(n_waves, 0, [&] { rank_words(a); });
    waves(n_waves, 0, [&] { label_final(a); });
    for (int y = 0; y < h; ++y) std::memcpy(labels_out + (size_t)y * w, lab + (size_t)y * pitch_lab, w * 4);
    *count_out = count;
    if (area_out) {
        // as the library does: counts per root id on the flattened plane
        std::memcpy(lab, roots.data(), roots.size() * 4);
        const size_t n_area = (size_t)h * pitch_lab + 1;
        uint32_t *area = (uint32_t *)std::malloc(n_area * 4);
        AreaArgs b{};
        b.lab = lab;
        b.pitch_lab = pitch_lab;
        b.lab_vec = a.lab_vec;
        b.out_aligned = (((uintptr_t)img.data() | (uintptr_t)pitch_img) & 3u) == 0 ? 1 : 0;
        b.area = area;
        b.out = img.data();
        b.pitch_out = pitch_img;
        b.h = h;
        b.w = w;
        b.min_area = min_area;
        b.max_area = max_area;
        serial([&] { clear_words(area, (uint32_t)n_area); }, 2, 64);
        waves(n_waves, 0, [&] { area_count(b); });
        waves(n_waves, 0, [&] { area_apply(b); });
        for (int y = 0; y < h; ++y) std::memcpy(area_out + (size_t)y * w, &img[(size_t)y * pitch_img], w);
        std::free(area);
    }
    std::free(lab);
    std::free(a.bits);
    std::free(a.word_off);
    std::free(a.seg_sum);
    return bad ? -2 : 0;
}

// ---------------------------------------------------------------------------
// distance-transform driver: mode 0 writes dist2 (int32), mode 1 D8 (uint8)

static int emu_edt(const uint8_t *img_in, int h, int w, int mode, int n_waves, int32_t *d2_out, uint8_t *d8_out) {
    using namespace rk;
    // padded pitches, exact-size allocations; widths divisible by 4 take the dword path
    const int64_t pitch_img = w % 4 == 0 ? w + 4 : w + 1, pitch_g = w % 4 == 0 ? w + 4 : w + 2;
    std::vector<uint8_t> img((size_t)(h - 1) * pitch_img + w);
    for (int y = 0; y < h; ++y) std::memcpy(&img[(size_t)y * pitch_img], img_in + (size_t)y * w, w);
    std::vector<int32_t> g((size_t)(h - 1) * pitch_g + w, -5);
    EdtArgs a{};
    a.img = img.data();
    a.pitch_img = pitch_img;
    a.g = g.data();
    a.pitch_g = pitch_g;
    a.d8 = img.data();   // in place over the input, as the library does
    a.pitch_d8 = pitch_img;
    a.h = h;
    a.w = w;
    a.mode = mode;
    const size_t n_sum = (size_t)((h + EDT_SEG - 1) / EDT_SEG) * w;
    std::vector<int32_t> zf(n_sum, -9), zl(n_sum, -9);
    a.zfirst = zf.data();
    a.zlast = zl.data();
    kemu::gridDim_.x = 3;
    kemu::blockDim_.x = 64;
    for (int kern = 0; kern < 2; ++kern)
        for (uint32_t b = 0; b < 3; ++b)
            for (uint32_t t = 0; t < 64; ++t) {
                kemu::blockIdx_.x = b;
                kemu::threadIdx_.x = t;
                if (kern == 0) edt_zeros(a);
                else edt_cols(a);
            }
    std::atomic<int> bad{0};
    std::vector<std::thread> th;
    for (int gi = 0; gi < n_waves; ++gi)
        th.emplace_back([&, gi] {
            kemu::blockIdx_.x = (uint32_t)gi;
            kemu::gridDim_.x = (uint32_t)n_waves;
            kemu::blockDim_.x = 64;
            if (!kemu::run_wave([&] { edt_rows(a); }, (size_t)w * 4))
                bad++;
        });
    for (auto &t : th) t.join();
    for (int y = 0; y < h; ++y) {
        if (mode == 0) std::memcpy(d2_out + (size_t)y * w, &g[(size_t)y * pitch_g], (size_t)w * 4);
        else std::memcpy(d8_out + (size_t)y * w, &img[(size_t)y * pitch_img], (size_t)w);
    }
    return bad ? -2 : 0;
}

// ---------------------------------------------------------------------------
// driver (called through ctypes)

extern "C" {

struct EmuTask {
    int32_t op;        // 0 dilate, 1 fill-holes, 2 erode, 3 h-dome, 4 regional maxima
    int32_t conn;
    int32_t hval;      // h-dome height
    int32_t h, w;
    uint8_t *image;    // dilate / erode: marker (in/out); the others: image (in/out); dense h x w
    const uint8_t *mask;
};

struct EmuStats {
    int64_t dense, revisit, rerun, overflow, aborted, route, spill;
};

int emu_run(const EmuTask *tasks, int n, int bh, int qcap, int scan_rounds, int n_waves,
            double watchdog_s, int stop_after, EmuStats *stats) {
    using namespace rk;
    if (bh != 16 && bh != 32 && bh != 64) return -1;
    // exact-size copies so that the sanitizer bounds-checks global accesses
    std::vector<uint8_t *> jplanes(n), iplanes(n, nullptr), scratch(n, nullptr);
    // the component route (KEMU_COMPONENT=1): an exact-size int32 label plane per task
    const char *ce = std::getenv("KEMU_COMPONENT");
    // 1: every two-valued mask takes the route; 2: where it pays (the library's default)
    const int component_mode = ce ? std::atoi(ce) : 0;
    const bool component = (component_mode == 1 || component_mode == 2) && stop_after == 0;
    std::vector<int32_t *> labs(n, nullptr);
    std::vector<TaskDev> table(n);
    uint32_t total = 0;
    bool any_mapped = false;
    for (int k = 0; k < n; ++k) {
        const EmuTask &e = tasks[k];
        const size_t px = (size_t)e.h * e.w;
        TaskDev d{};
        d.h = e.h;
        d.w = e.w;
        d.conn = e.conn;
        d.nby = (e.h + bh - 1) / bh;
        d.nbx = (e.w + BW - 1) / BW;
        d.block0 = total;
        total += (uint32_t)(d.nby * d.nbx);
        d.scan_rounds = scan_rounds;
        d.qcap = qcap;
        jplanes[k] = (uint8_t *)std::malloc(px);
        std::memcpy(jplanes[k], e.image, px);
        d.minv = (e.op == 1 || e.op == 2) ? 1 : 0;
        d.hval = e.op == 3 ? e.hval : (e.op == 4 ? 1 : 0);
        if (e.op == 0 || e.op == 2) {
            iplanes[k] = (uint8_t *)std::malloc(px);
            std::memcpy(iplanes[k], e.mask, px);
            d.op = e.op == 0 ? OP_DILATE : OP_ERODE;
            d.j = jplanes[k];
            d.pitch_j = e.w;
            d.i = iplanes[k];
            d.pitch_i = e.w;
            d.img = e.op == 0 ? nullptr : jplanes[k];
            d.pitch_img = e.w;
            d.aligned = (e.w % 4 == 0);
        } else {
            const int64_t pj = (e.w + 3) / 4 * 4;
            scratch[k] = (uint8_t *)std::malloc((size_t)pj * e.h);
            std::memset(scratch[k], 0xee, (size_t)pj * e.h);   // garbage: init_marker overwrites it
            d.op = e.op == 1 ? OP_FILL : (e.op == 3 ? OP_HDOME : OP_RMAX);
            d.i = jplanes[k];
            d.pitch_i = e.w;
            d.img = jplanes[k];
            d.pitch_img = e.w;
            d.j = scratch[k];
            d.pitch_j = pj;
            d.aligned = (e.w % 4 == 0);
        }
        if (e.op != 0) any_mapped = true;
        d.lab = nullptr;
        d.pitch_lab = (e.w + 3) / 4 * 4 + 4;   // padded: pitched node ids are exercised
        if (component) {
            labs[k] = (int32_t *)std::malloc(((size_t)(e.h - 1) * d.pitch_lab + e.w) * sizeof(int32_t));
            d.lab = labs[k];
        }
        table[k] = d;
    }
    // task table: inline in the "kernel arguments" when small, else in memory
    std::vector<uint8_t> ext_mem;
    TaskTable tt{};
    if (n <= MAX_INLINE_TASKS) {
        tt.n_inline = (uint32_t)n;
        tt.total_inline = total;
        tt.ring_cap_inline = total + (uint32_t)n_waves + 1;
        tt.seq_inline = 1;   // the launch's number (Work starts zeroed)
        for (int k = 0; k < n; ++k) tt.inl[k] = table[k];
    } else {
        ext_mem.resize(sizeof(BatchHdr) + n * sizeof(TaskDev));
        BatchHdr hdr{};
        hdr.n_tasks = (uint32_t)n;
        hdr.total_blocks = total;
        hdr.ring_cap = total + (uint32_t)n_waves + 1;
        hdr.any_mapped = any_mapped ? 1u : 0u;
        hdr.launch_seq = 1;
        std::memcpy(ext_mem.data(), &hdr, sizeof(hdr));
        std::memcpy(ext_mem.data() + sizeof(hdr), table.data(), n * sizeof(TaskDev));
        tt.hdr = (const BatchHdr *)ext_mem.data();
        tt.ext = (const TaskDev *)(ext_mem.data() + sizeof(BatchHdr));
    }
    Work *work = (Work *)std::calloc(1, sizeof(Work));
    uint32_t *state = (uint32_t *)std::malloc((size_t)total * STATE_STRIDE * sizeof(uint32_t));
    uint32_t *ring = (uint32_t *)std::malloc((size_t)(total + n_waves + 1) * RING_STRIDE * sizeof(uint32_t));
    uint32_t *tpend = (uint32_t *)std::malloc(n * sizeof(uint32_t));
    uint32_t *tdone = (uint32_t *)std::malloc(n * sizeof(uint32_t));
    uint32_t *route = component ? (uint32_t *)std::malloc(ROUTE_WORDS * n * sizeof(uint32_t)) : nullptr;

    auto grid_run = [&](auto fn, uint32_t blocks, uint32_t threads) {
        kemu::gridDim_.x = blocks;
        kemu::blockDim_.x = threads;
        for (uint32_t b = 0; b < blocks; ++b)
            for (uint32_t t = 0; t < threads; ++t) {
                kemu::blockIdx_.x = b;
                kemu::threadIdx_.x = t;
                fn();
            }
    };
    // stop_after 0: the persistent pipeline; 1..3: the staged one, stopped after that stage
    const bool merged = stop_after == 0;
    KArgs ka;
    ka.work = work;
    ka.state = state;
    ka.ring = ring;
    ka.tile_pending = tpend;
    ka.tile_done = tdone;
    ka.qcap = qcap;
    ka.scan_rounds = scan_rounds;
    ka.watchdog_ticks = (uint64_t)(watchdog_s * 1e8);
    ka.drain_budget = 128;
    ka.binary_drain_budget = 4;
    ka.route = route;
    ka.route_policy = component_mode == 1 ? 1 : 0;
    ka.launch_seq = 1;
    ka.host_done = nullptr;
    // global spill queues (KEMU_SPILL = entries per wave; unset or 0: none), exact size
    const char *se = std::getenv("KEMU_SPILL");
    const uint32_t spill_cap = se ? (uint32_t)std::atoi(se) : 0u;
    std::vector<uint16_t> spill_mem((size_t)n_waves * spill_cap + 1);
    ka.spill = spill_cap ? spill_mem.data() : nullptr;
    ka.spill_cap = spill_cap;
    {   // test hook of the block claims (see KArgs::test_fault)
        const char *f = std::getenv("KEMU_TEST_FAULT");
        ka.test_fault = f ? std::atoi(f) : 0;
    }
    {   // reset_work samples the tasks' masks with cross-lane operations: run it as emulated waves
        const int mode = !merged ? RESET_STAGED : (component ? RESET_ROUTE : RESET_QUEUE_ALL);
        std::atomic<int> rbad{0};
        std::vector<std::thread> th;
        for (int g = 0; g < 4; ++g)
            th.emplace_back([&, g] {
                kemu::blockIdx_.x = (uint32_t)g;
                kemu::gridDim_.x = 4;
                kemu::blockDim_.x = 64;
                if (!kemu::run_wave([&] { reset_work(tt, ka, mode); }, 16))
                    rbad++;
            });
        for (auto &t : th) t.join();
        if (rbad) return -2;
    }

    const size_t lds = bh == 16 ? lds_bytes<16>(qcap) : bh == 32 ? lds_bytes<32>(qcap) : lds_bytes<64>(qcap);
    std::atomic<int> bad{0};
    auto run_grid = [&](int stage, int waves) {
        std::vector<std::thread> th;
        for (int g = 0; g < waves; ++g) {
            th.emplace_back([&, g, stage] {
                kemu::blockIdx_.x = (uint32_t)g;
                kemu::gridDim_.x = (uint32_t)waves;
                kemu::blockDim_.x = 64;
                std::function<void()> body;
#define KEMU_PICK(K)                                            \
    switch (bh) {                                               \
        case 16: body = [&] { K<16>(tt, ka); }; break;          \
        case 32: body = [&] { K<32>(tt, ka); }; break;          \
        default: body = [&] { K<64>(tt, ka); }; break;          \
    }
                if (stage == 1) { KEMU_PICK(dense_pass) }
                else if (stage == 2) { KEMU_PICK(border_seed) }
                else { KEMU_PICK(revisit_drain) }
#undef KEMU_PICK
                if (!kemu::run_wave(body, lds)) bad++;
            });
        }
        for (auto &t : th) t.join();
    };
    if (component) {   // classification, labelling and the per-component maxima, as the library runs them
        auto comp_grid = [&](int which, size_t lds_sz) {
            std::vector<std::thread> th;
            for (int g = 0; g < n_waves; ++g) {
                th.emplace_back([&, g, which, lds_sz] {
                    kemu::blockIdx_.x = (uint32_t)g;
                    kemu::gridDim_.x = (uint32_t)n_waves;
                    kemu::blockDim_.x = 64;
                    std::function<void()> body;
#define KEMU_PICK(K)                                            \
    switch (bh) {                                               \
        case 16: body = [&] { K<16>(tt, ka); }; break;          \
        case 32: body = [&] { K<32>(tt, ka); }; break;          \
        default: body = [&] { K<64>(tt, ka); }; break;          \
    }
                    if (which == 0) { KEMU_PICK(comp_classify) }
                    else if (which == 1) { KEMU_PICK(comp_label_local) }
                    else if (which == 2) { KEMU_PICK(comp_label_merge) }
                    else if (which == 3) { KEMU_PICK(comp_flatten_max) }
                    else { KEMU_PICK(comp_write) }
#undef KEMU_PICK
                    if (!kemu::run_wave(body, lds_sz)) bad++;
                });
            }
            for (auto &t : th) t.join();
        };
        comp_grid(0, 0);   // the classification; its last workgroup decides the routes
        grid_run([&] { prepare(tt, ka, any_mapped ? 1 : 0); }, 8, 64);
        comp_grid(1, (size_t)LT_H * LT_W * 4);
        comp_grid(2, 0);
        comp_grid(3, 0);
        comp_grid(4, 0);
    } else if (any_mapped) {
        grid_run([&] { init_marker(tt, nullptr); }, 8, 64);
    }
    if (!merged) run_grid(1, n_waves);
    if (stop_after >= 2) run_grid(2, n_waves);
    if (merged || stop_after >= 3) run_grid(3, n_waves);
    if (any_mapped) grid_run([&] { finish_result(tt, route); }, 4, 64);

    for (int k = 0; k < n; ++k) {
        const EmuTask &e = tasks[k];
        std::memcpy(e.image, jplanes[k], (size_t)e.h * e.w);
        std::free(jplanes[k]);
        if (iplanes[k]) std::free(iplanes[k]);
        if (scratch[k]) std::free(scratch[k]);
        if (labs[k]) std::free(labs[k]);
    }
    if (stats) {
        stats->dense = (int64_t)work->stat_dense;
        stats->revisit = (int64_t)work->stat_revisit;
        stats->rerun = (int64_t)work->stat_rerun;
        stats->overflow = (int64_t)work->stat_overflow;
        stats->aborted = (int64_t)work->abort;
        stats->route = (int64_t)work->stat_route;
        stats->spill = (int64_t)work->stat_spill;
    }
    const bool full = stop_after == 0 || stop_after >= 3;
    const int rc = bad ? -2 : (work->abort ? -3 : (full && work->pending != 0 ? -4 : 0));
    std::free(work);
    std::free(state);
    std::free(ring);
    std::free(tpend);
    std::free(tdone);
    std::free(route);
    return rc;
}

}  // extern "C"

#ifdef KEMU_MAIN
// Stand-alone driver (lets the sanitizer runtime link into the executable):
//   kemu <bh> <qcap> <scan_rounds> <waves> <watchdog_s> <n> then n lines of
//   "op conn hval h w image_path mask_path_or_- out_path" on stdin.
#include <string>
int main(int argc, char **argv) {
    //   kemu label <conn> <h> <w> <waves> <min_area> <max_area> <image_path> <labels_out> <area_out>
    if (argc == 11 && std::string(argv[1]) == "label") {
        const int conn = std::atoi(argv[2]), h = std::atoi(argv[3]), w = std::atoi(argv[4]);
        const int nw = std::atoi(argv[5]);
        const int64_t lo = std::atoll(argv[6]), hi = std::atoll(argv[7]);
        std::vector<uint8_t> img((size_t)h * w), area((size_t)h * w);
        std::vector<int32_t> lab((size_t)h * w);
        FILE *f = std::fopen(argv[8], "rb");
        if (!f || std::fread(img.data(), 1, img.size(), f) != img.size()) return 4;
        std::fclose(f);
        int32_t count = -1;
        const int rc = emu_label(img.data(), h, w, conn, nw, lab.data(), &count, lo, hi, area.data());
        f = std::fopen(argv[9], "wb");
        std::fwrite(lab.data(), 4, lab.size(), f);
        std::fclose(f);
        f = std::fopen(argv[10], "wb");
        std::fwrite(area.data(), 1, area.size(), f);
        std::fclose(f);
        std::printf("rc %d count %d\n", rc, count);
        return rc == 0 ? 0 : 1;
    }
    //   kemu edt <h> <w> <waves> <image_path> <dist2_out> <d8_out>
    if (argc == 8 && std::string(argv[1]) == "edt") {
        const int h = std::atoi(argv[2]), w = std::atoi(argv[3]), nw = std::atoi(argv[4]);
        std::vector<uint8_t> img((size_t)h * w), d8((size_t)h * w);
        std::vector<int32_t> d2((size_t)h * w);
        FILE *f = std::fopen(argv[5], "rb");
        if (!f || std::fread(img.data(), 1, img.size(), f) != img.size()) return 4;
        std::fclose(f);
        int rc = emu_edt(img.data(), h, w, 0, nw, d2.data(), nullptr);
        if (rc == 0) rc = emu_edt(img.data(), h, w, 1, nw, nullptr, d8.data());
        f = std::fopen(argv[6], "wb");
        std::fwrite(d2.data(), 4, d2.size(), f);
        std::fclose(f);
        f = std::fopen(argv[7], "wb");
        std::fwrite(d8.data(), 1, d8.size(), f);
        std::fclose(f);
        std::printf("rc %d\n", rc);
        return rc == 0 ? 0 : 1;
    }
    if (argc < 7) return 2;
    const int bh = std::atoi(argv[1]), qcap = std::atoi(argv[2]), rounds = std::atoi(argv[3]);
    const int waves = std::atoi(argv[4]);
    const double wd = std::atof(argv[5]);
    const int n = std::atoi(argv[6]);
    const int stop_after = argc > 7 ? std::atoi(argv[7]) : 0;
    std::vector<EmuTask> tasks(n);
    std::vector<std::vector<uint8_t>> imgs(n), masks(n);
    std::vector<std::string> outs(n);
    for (int k = 0; k < n; ++k) {
        int op, conn, hval, h, w;
        char ip[1024], mp[1024], op_[1024];
        if (std::scanf("%d %d %d %d %d %1023s %1023s %1023s", &op, &conn, &hval, &h, &w, ip, mp, op_) != 8)
            return 3;
        const bool two = op == 0 || op == 2;
        imgs[k].resize((size_t)h * w);
        FILE *f = std::fopen(ip, "rb");
        if (!f || std::fread(imgs[k].data(), 1, imgs[k].size(), f) != imgs[k].size()) return 4;
        std::fclose(f);
        if (two) {
            masks[k].resize((size_t)h * w);
            f = std::fopen(mp, "rb");
            if (!f || std::fread(masks[k].data(), 1, masks[k].size(), f) != masks[k].size()) return 5;
            std::fclose(f);
        }
        tasks[k] = EmuTask{op, conn, hval, h, w, imgs[k].data(), two ? masks[k].data() : nullptr};
        outs[k] = op_;
    }
    EmuStats st{};
    const int rc = emu_run(tasks.data(), n, bh, qcap, rounds, waves, wd, stop_after, &st);
    for (int k = 0; k < n; ++k) {
        FILE *f = std::fopen(outs[k].c_str(), "wb");
        std::fwrite(imgs[k].data(), 1, imgs[k].size(), f);
        std::fclose(f);
    }
    std::printf("rc %d dense %lld revisit %lld rerun %lld overflow %lld aborted %lld route %lld spill %lld\n", rc,
                (long long)st.dense, (long long)st.revisit, (long long)st.rerun, (long long)st.overflow,
                (long long)st.aborted, (long long)st.route, (long long)st.spill);
    return rc == 0 ? 0 : 1;
}
#endif
