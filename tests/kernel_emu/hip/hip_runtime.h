// Host stand-in for <hip/hip_runtime.h> used ONLY to compile the device code of
// paper_1209_3332_amd/csrc/kernels.hpp for the CPU, so that its scheduling and
// pixel logic can be run and bounds-checked on the host (tests/kernel_emu).
// A wave is emulated as 64 fibers run round-robin on one OS thread; every
// cross-lane operation (shuffle, ballot, barrier) is a switch point.
#pragma once
#include <atomic>
#include <chrono>
#include <cstdint>
#include <cstring>
#include <thread>

#define __device__ inline
#define __host__
#define __global__
#define __forceinline__
#define __launch_bounds__(x)
#define __align__(x) __attribute__((aligned(x)))

#define __HIP_MEMORY_SCOPE_WAVEFRONT 2
#define __HIP_MEMORY_SCOPE_WORKGROUP 3
#define __HIP_MEMORY_SCOPE_AGENT 4
#define __HIP_MEMORY_SCOPE_SYSTEM 5

#define __hip_atomic_load(p, o, s) __atomic_load_n((p), (o))
#define __hip_atomic_store(p, v, o, s) __atomic_store_n((p), (v), (o))
#define __hip_atomic_fetch_add(p, v, o, s) __atomic_fetch_add((p), (v), (o))
#define __hip_atomic_fetch_sub(p, v, o, s) __atomic_fetch_sub((p), (v), (o))
#define __hip_atomic_fetch_or(p, v, o, s) __atomic_fetch_or((p), (v), (o))
#define __hip_atomic_exchange(p, v, o, s) __atomic_exchange_n((p), (v), (o))
#define __hip_atomic_compare_exchange_strong(p, e, d, o1, o2, s) \
    __atomic_compare_exchange_n((p), (e), (d), false, (o1), (o2))
#define __hip_atomic_compare_exchange_weak(p, e, d, o1, o2, s) \
    __atomic_compare_exchange_n((p), (e), (d), true, (o1), (o2))

namespace kemu {

struct Dim3 { uint32_t x = 0, y = 0, z = 0; };
extern thread_local Dim3 blockIdx_, threadIdx_, blockDim_, gridDim_;

int lane();                           // current lane of the running wave
void wave_sync();                     // all 64 lanes reach this point
uint64_t exchange(uint64_t v, int src_lane);   // value of `v` in lane src_lane
uint64_t ballot(bool p);
uint8_t *wave_lds();
uint64_t wall_ticks();
void check_lds(const void *p, size_t n);       // bounds check of an LDS access

}  // namespace kemu

#define blockIdx kemu::blockIdx_
#define threadIdx kemu::threadIdx_
#define blockDim kemu::blockDim_
#define gridDim kemu::gridDim_

inline int __lane_id() { return kemu::lane(); }
inline void __syncthreads() { kemu::wave_sync(); }
// The wave barrier orders memory accesses across the lanes of one wave (the
// hardware runs them in lockstep); here it is a switch point like a barrier.
inline void __builtin_amdgcn_wave_barrier() { kemu::wave_sync(); }
inline void __threadfence() { std::atomic_thread_fence(std::memory_order_seq_cst); }
inline unsigned long long __ballot(int p) { return kemu::ballot(p != 0); }
inline int __popcll(unsigned long long v) { return __builtin_popcountll(v); }
inline uint64_t wall_clock64() { return kemu::wall_ticks(); }

inline uint32_t __shfl(uint32_t v, int src) { return (uint32_t)kemu::exchange(v, src); }
inline int __shfl(int v, int src) { return (int)kemu::exchange((uint32_t)v, src); }
inline uint32_t __shfl_up(uint32_t v, unsigned d) {
    const int l = kemu::lane();
    const uint32_t r = (uint32_t)kemu::exchange(v, l - (int)d >= 0 ? l - (int)d : l);
    return r;
}
inline uint32_t __shfl_down(uint32_t v, unsigned d) {
    const int l = kemu::lane();
    return (uint32_t)kemu::exchange(v, l + (int)d < 64 ? l + (int)d : l);
}

inline uint32_t __builtin_amdgcn_mbcnt_lo(uint32_t m, uint32_t acc) {
    const int l = kemu::lane();
    const uint32_t below = l >= 32 ? m : (l == 0 ? 0u : (m & ((1u << l) - 1u)));
    return acc + (uint32_t)__builtin_popcount(below);
}
inline uint32_t __builtin_amdgcn_mbcnt_hi(uint32_t m, uint32_t acc) {
    const int l = kemu::lane();
    const uint32_t below = l < 32 ? 0u : (l == 32 ? 0u : (m & ((1u << (l - 32)) - 1u)));
    return acc + (uint32_t)__builtin_popcount(below);
}
inline void __builtin_amdgcn_s_sleep(int) { std::this_thread::yield(); }
inline int __builtin_amdgcn_readfirstlane(int v) { return (int)(uint32_t)kemu::exchange((uint32_t)v, 0); }
// DPP: only the whole-wave shifts by one lane are emulated (bound_ctrl: 0 where no source lane)
inline int __builtin_amdgcn_update_dpp(int old, int src, int ctrl, int row_mask, int bank_mask, bool bound_ctrl) {
    (void)old; (void)row_mask; (void)bank_mask; (void)bound_ctrl;
    const int l = kemu::lane();
    const int from = ctrl == 0x138 ? l - 1 : (ctrl == 0x130 ? l + 1 : -100);
    if (from == -100) { __builtin_trap(); }
    const uint32_t v = (uint32_t)kemu::exchange((uint32_t)src, from >= 0 && from < 64 ? from : l);
    return (from >= 0 && from < 64) ? (int)v : 0;
}

inline uint32_t atomicCAS(uint32_t *p, uint32_t expected, uint32_t desired) {
    kemu::check_lds(p, 4);
    __atomic_compare_exchange_n(p, &expected, desired, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST);
    return expected;
}

inline int min(int a, int b) { return a < b ? a : b; }
inline int max(int a, int b) { return a > b ? a : b; }
inline uint32_t min(uint32_t a, uint32_t b) { return a < b ? a : b; }
inline uint32_t max(uint32_t a, uint32_t b) { return a > b ? a : b; }

#define RK_DYN_LDS_PROVIDED 1
namespace rk {
inline uint8_t *dyn_lds() { return kemu::wave_lds(); }
}
