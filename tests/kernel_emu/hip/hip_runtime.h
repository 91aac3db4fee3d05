// Host stand-in for <hip/hip_runtime.h> used ONLY to compile the device code of
// paper_1209_3332_amd/csrc/kernels.hpp for the CPU, so that its scheduling and
// pixel logic can be run and bounds-checked on the host (tests/kernel_emu).
// A wave is emulated as 64 fibers run round-robin on one OS thread; every
// cross-lane operation (shuffle, ballot, barrier) is a switch point.
#pragma once
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>

#define __device__ inline
#define __host__
#define __global__
// a kernel's __shared__ variable: one per emulated workgroup (a workgroup is
// one wave, whose lanes are fibers of one OS thread)
#define __shared__ static thread_local
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
// fetch-min: a compare-exchange loop on the host
template <typename T>
inline T kemu_fetch_min(T *p, T v) {
    T cur = __atomic_load_n(p, __ATOMIC_SEQ_CST);
    while (v < cur && !__atomic_compare_exchange_n(p, &cur, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) {
    }
    return cur;
}
#define __hip_atomic_fetch_min(p, v, o, s) kemu_fetch_min((p), (v))
template <typename T>
inline T kemu_fetch_max(T *p, T v) {
    T cur = __atomic_load_n(p, __ATOMIC_SEQ_CST);
    while (v > cur && !__atomic_compare_exchange_n(p, &cur, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) {
    }
    return cur;
}
#define __hip_atomic_fetch_max(p, v, o, s) kemu_fetch_max((p), (v))
#define __hip_atomic_fetch_and(p, v, o, s) __atomic_fetch_and((p), (v), (o))
#define __hip_atomic_exchange(p, v, o, s) __atomic_exchange_n((p), (v), (o))
#define __hip_atomic_compare_exchange_strong(p, e, d, o1, o2, s) \
    __atomic_compare_exchange_n((p), (e), (d), false, (o1), (o2))
#define __hip_atomic_compare_exchange_weak(p, e, d, o1, o2, s) \
    __atomic_compare_exchange_n((p), (e), (d), true, (o1), (o2))

namespace kemu {

struct Dim3 { uint32_t x = 0, y = 0, z = 0; };
extern thread_local Dim3 blockIdx_, threadIdx_, blockDim_, gridDim_;

int lane();                           // current lane of the running wave
Dim3 thread_idx();                    // inside a wave: (lane, 0, 0); else threadIdx_
void wave_sync();                     // all 64 lanes reach this point
uint64_t exchange(uint64_t v, int src_lane);   // value of `v` in lane src_lane
uint64_t ballot(bool p);
uint8_t *wave_lds();
uint64_t wall_ticks();
void check_lds(const void *p, size_t n);       // bounds check of an LDS access

}  // namespace kemu

#define blockIdx kemu::blockIdx_
#define threadIdx kemu::thread_idx()
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
inline int __popc(unsigned int v) { return __builtin_popcount(v); }
inline uint64_t wall_clock64() { return kemu::wall_ticks(); }

inline uint32_t __shfl(uint32_t v, int src) { return (uint32_t)kemu::exchange(v, src); }
inline int __shfl(int v, int src) { return (int)kemu::exchange((uint32_t)v, src); }
inline uint32_t __shfl_up(uint32_t v, unsigned d) {
    const int l = kemu::lane();
    const uint32_t r = (uint32_t)kemu::exchange(v, l - (int)d >= 0 ? l - (int)d : l);
    return r;
}
inline int __shfl_xor(int v, int m) {
    const int l = kemu::lane();
    return (int)kemu::exchange((uint32_t)v, l ^ m);
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
// an instruction-scheduling hint for the compiler: no effect on what a wave computes
inline void __builtin_amdgcn_sched_barrier(int) {}
inline int __builtin_amdgcn_readfirstlane(int v) { return (int)(uint32_t)kemu::exchange((uint32_t)v, 0); }
// DPP data movement as used by the kernels: row shifts (within 16-lane rows),
// whole-wave shifts by one lane, and the row broadcasts.  A lane whose source
// is invalid reads 0 with bound_ctrl, else keeps `old`; rows outside row_mask
// keep `old`.
inline int __builtin_amdgcn_update_dpp(int old, int src, int ctrl, int row_mask, int bank_mask, bool bound_ctrl) {
    if (bank_mask != 0xf) __builtin_trap();
    const int l = kemu::lane();
    const int row = l >> 4, pos = l & 15;
    int from = -1;
    if (ctrl >= 0x101 && ctrl <= 0x10f) from = pos + (ctrl - 0x100) <= 15 ? l + (ctrl - 0x100) : -1;   // row_shl
    else if (ctrl >= 0x111 && ctrl <= 0x11f) from = pos - (ctrl - 0x110) >= 0 ? l - (ctrl - 0x110) : -1;  // row_shr
    else if (ctrl == 0x130) from = l + 1 < 64 ? l + 1 : -1;   // wave_shl:1
    else if (ctrl == 0x138) from = l - 1;                       // wave_shr:1
    else if (ctrl == 0x142) from = row > 0 ? 16 * row - 1 : -1;  // row_bcast:15
    else if (ctrl == 0x143) from = row > 1 ? 31 : -1;            // row_bcast:31
    else __builtin_trap();
    const uint32_t v = (uint32_t)kemu::exchange((uint32_t)src, from >= 0 ? from : l);
    if (!((row_mask >> row) & 1)) return old;
    if (from < 0) return bound_ctrl ? 0 : old;
    return (int)v;
}
inline int __builtin_amdgcn_readlane(int v, int lane) { return (int)(uint32_t)kemu::exchange((uint32_t)v, lane); }
// Memory fence of a given order at a named scope: a full fence on the host.
inline void __builtin_amdgcn_fence(int, const char *) { std::atomic_thread_fence(std::memory_order_seq_cst); }
// Waiting for this wave's memory operations: a full fence on the host.
inline void __builtin_amdgcn_s_waitcnt(int) { std::atomic_thread_fence(std::memory_order_seq_cst); }

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
#define RK_LDS
#define RK_GLOBAL
#define RK_LANE_SYNC() kemu::wave_sync()
namespace rk {
inline uint8_t *dyn_lds() { return kemu::wave_lds(); }
}
