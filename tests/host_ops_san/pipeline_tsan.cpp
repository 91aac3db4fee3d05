// The co-scheduling runtime (paper_1209_3332_amd/csrc/pipeline.cpp) with CPU
// workers only, built with ThreadSanitizer (g++, host code only): several CPU
// workers and I/O threads, both policies, several windows, then every tile's
// outputs against the CPU variants run one after another on one thread.
// The GPU entry points are never called without a GPU; the stubs below only
// satisfy the linker (they fail if they ever are).
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../../include/recon.h"
#include "../../paper_1209_3332_amd/csrc/host_ops.hpp"

extern "C" {
int recon_hdome(recon_ctx *, recon_image *, int, int, void *) { abort(); }
int recon_fill_holes(recon_ctx *, recon_image *, int, void *) { abort(); }
int recon_area_threshold(recon_ctx *, recon_image *, int, int64_t, int64_t, void *) { abort(); }
int recon_pre_watershed(recon_ctx *, recon_image *, int, void *) { abort(); }
int recon_label(recon_ctx *, const recon_image *, int32_t *, int64_t, int, int32_t *, void *) { abort(); }
int recon_enqueue_status(recon_ctx *, uint32_t *, void *) { abort(); }
int recon_batch(recon_ctx *, const recon_task *, int32_t, void *) { abort(); }
const char *recon_last_error(void) { return ""; }
}

static uint32_t lcg(uint32_t &s) { return s = s * 1664525u + 1013904223u; }

int main() {
    const int n = 7;
    std::vector<std::vector<uint8_t>> img(n);
    std::vector<int> H(n), W(n);
    uint32_t seed = 12345u;
    for (int i = 0; i < n; ++i) {
        H[i] = 20 + (int)(lcg(seed) % 90);
        W[i] = 20 + (int)(lcg(seed) % 140);
        img[i].resize((size_t)H[i] * W[i]);
        // smooth blobs plus noise: domes, holes and small objects for every operation
        for (int y = 0; y < H[i]; ++y)
            for (int x = 0; x < W[i]; ++x) {
                const int v = ((x / 9 + y / 7) % 3) * 70 + (int)(lcg(seed) % 40);
                img[i][(size_t)y * W[i] + x] = (uint8_t)(v > 255 ? 255 : v);
            }
    }
    // the reference: the CPU variants in order, on this thread
    std::vector<std::vector<uint8_t>> ref_obj(n), ref_mk(n);
    std::vector<std::vector<int32_t>> ref_lab(n);
    std::vector<int32_t> ref_cnt(n);
    hostops::Scratch *s = hostops::scratch_new();
    for (int i = 0; i < n; ++i) {
        std::vector<uint8_t> a = img[i];
        hostops::Plane p{a.data(), H[i], W[i], W[i]};
        hostops::hdome(s, p, 20, 8);
        hostops::fill_holes(s, p, 8);
        hostops::area_threshold(s, p, 8, 20, 1000);
        ref_obj[i] = a;
        std::vector<uint8_t> m = a;
        hostops::pre_watershed(s, hostops::Plane{m.data(), H[i], W[i], W[i]}, 8);
        ref_mk[i] = m;
        ref_lab[i].resize(a.size());
        ref_cnt[i] = hostops::label(s, p, ref_lab[i].data(), W[i], 8);
    }
    hostops::scratch_free(s);
    int bad = 0;
    for (int policy = 0; policy < 2; ++policy)
        for (int window : {1, 3, 7}) {
            std::vector<std::vector<uint8_t>> obj(n), mk(n);
            std::vector<std::vector<int32_t>> lab(n);
            std::vector<int32_t> cnt(n, -1);
            std::vector<recon_pipe_tile> t(n);
            for (int i = 0; i < n; ++i) {
                obj[i].assign(img[i].size(), 7);
                mk[i].assign(img[i].size(), 7);
                lab[i].assign(img[i].size(), -7);
                t[i] = recon_pipe_tile{img[i].data(), H[i], W[i], W[i], obj[i].data(), mk[i].data(),
                                       lab[i].data(), W[i], &cnt[i]};
            }
            recon_pipe_config c{};
            c.policy = policy;
            c.cpu_workers = 4;
            c.use_gpu = 0;
            c.window = window;
            c.data_locality = 1;
            c.conn = 8;
            c.h = 20;
            c.area_min = 20;
            c.area_max = 1000;
            c.io_threads = 3;
            const float sp[5] = {30, 20, 5, 10, 2};
            for (int o = 0; o < 5; ++o) c.speedup[o] = sp[o];
            std::vector<recon_pipe_event> ev(5 * n);
            c.trace = ev.data();
            c.trace_cap = 5 * n;
            recon_pipe_stats st{};
            const int rc = recon_pipeline_run(nullptr, t.data(), n, &c, &st);
            if (rc != 0 || st.trace_n != 5 * n) {
                fprintf(stderr, "policy %d window %d: rc %d (%s), %lld events\n", policy, window, rc,
                        recon_pipeline_error(), (long long)st.trace_n);
                ++bad;
                continue;
            }
            for (int i = 0; i < n; ++i)
                if (obj[i] != ref_obj[i] || mk[i] != ref_mk[i] || lab[i] != ref_lab[i] || cnt[i] != ref_cnt[i]) {
                    fprintf(stderr, "policy %d window %d: tile %d differs\n", policy, window, i);
                    ++bad;
                }
        }
    printf("%s\n", bad ? "MISMATCH" : "ok");
    return bad ? 1 : 0;
}
