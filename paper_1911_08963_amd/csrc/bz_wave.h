// Wave-level atomics shared by the persistent and schedule kernels. Included
// by the HIP sources only.
#pragma once

#include <hip/hip_runtime.h>

#include "bz_tile.h"

namespace bz {

// Wave-level atomics: one memory operation per wave, by construction. The
// asm block (skipped when no lane is active) narrows exec to the wave's
// first active lane, issues a single
// global atomic and waits for it before restoring exec; readfirstlane then
// hands the old value to the whole wave. (Left to the compiler, a wave-wide
// atomic is folded into one operation only when the optimizer can prove its
// address uniform; when it cannot, all 64 lanes hit the word and a tile
// claim costs 64 atomics on the hottest cache line.) The fences give the
// acquire/release ordering of the operation at agent scope.
__device__ __forceinline__ unsigned long long wave_fetch_add64(unsigned long long *p, unsigned long long v,
                                                               uint32_t lane) {
    (void)lane;
    unsigned long long old;
    uint64_t save;
    uint32_t first;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    asm volatile(
        "s_cmp_eq_u64 exec, 0\n\t"
        "s_cbranch_scc1 1f\n\t"
        "s_mov_b64 %1, exec\n\t"
        "s_ff1_i32_b64 %2, exec\n\t"
        "s_lshl_b64 exec, 1, %2\n\t"
        "global_atomic_add_x2 %0, %3, %4, off sc0\n\t"
        "s_waitcnt vmcnt(0)\n\t"
        "s_mov_b64 exec, %1\n"
        "1:"
        : "=&v"(old), "=&s"(save), "=&s"(first)
        : "v"(p), "v"(v)
        : "memory", "scc");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return uni64(old);
}

// The same without the fences: for counters whose value carries no data the
// wave then reads (claims validated by a later acquire, tickets, log slots).
__device__ __forceinline__ unsigned long long wave_fetch_add64_relaxed(unsigned long long *p, unsigned long long v) {
    unsigned long long old;
    uint64_t save;
    uint32_t first;
    asm volatile(
        "s_cmp_eq_u64 exec, 0\n\t"
        "s_cbranch_scc1 1f\n\t"
        "s_mov_b64 %1, exec\n\t"
        "s_ff1_i32_b64 %2, exec\n\t"
        "s_lshl_b64 exec, 1, %2\n\t"
        "global_atomic_add_x2 %0, %3, %4, off sc0\n\t"
        "s_waitcnt vmcnt(0)\n\t"
        "s_mov_b64 exec, %1\n"
        "1:"
        : "=&v"(old), "=&s"(save), "=&s"(first)
        : "v"(p), "v"(v)
        : "memory", "scc");
    return uni64(old);
}

__device__ __forceinline__ void wave_fetch_max64(unsigned long long *p, unsigned long long v) {
    uint64_t save;
    uint32_t first;
    asm volatile(
        "s_cmp_eq_u64 exec, 0\n\t"
        "s_cbranch_scc1 1f\n\t"
        "s_mov_b64 %0, exec\n\t"
        "s_ff1_i32_b64 %1, exec\n\t"
        "s_lshl_b64 exec, 1, %1\n\t"
        "global_atomic_umax_x2 %2, %3, off\n\t"
        "s_waitcnt vmcnt(0)\n\t"
        "s_mov_b64 exec, %0\n"
        "1:"
        : "=&s"(save), "=&s"(first)
        : "v"(p), "v"(v)
        : "memory", "scc");
}

// The same, returning the old value (relaxed).
__device__ __forceinline__ unsigned long long wave_fetch_max64_old(unsigned long long *p, unsigned long long v) {
    unsigned long long old;
    uint64_t save;
    uint32_t first;
    asm volatile(
        "s_cmp_eq_u64 exec, 0\n\t"
        "s_cbranch_scc1 1f\n\t"
        "s_mov_b64 %1, exec\n\t"
        "s_ff1_i32_b64 %2, exec\n\t"
        "s_lshl_b64 exec, 1, %2\n\t"
        "global_atomic_umax_x2 %0, %3, %4, off sc0\n\t"
        "s_waitcnt vmcnt(0)\n\t"
        "s_mov_b64 exec, %1\n"
        "1:"
        : "=&v"(old), "=&s"(save), "=&s"(first)
        : "v"(p), "v"(v)
        : "memory", "scc");
    return uni64(old);
}

}  // namespace bz
