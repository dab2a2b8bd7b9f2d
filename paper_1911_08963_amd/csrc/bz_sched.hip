// The paper's distributed schedules on one GPU (Sec. 3 of arXiv:1911.08963),
// with the device's waves as the workers: one (Gamma_j, g) task is cut into
// prefix tasks and dealt statically (cyclic or snake cyclic) or through a
// shared counter (one task or a front/back pair per claim), in lexicographic
// or left-lexicographic order (bz_sched.h). A wave processes a prefix the way
// Process_prefix does: the prefix rows are added once (their XOR joins every
// lane sum) and then every completion, the (g - p)-subsets of the rows after
// the prefix's last element, runs through the tile code of the enumeration
// kernel (bz_tile.h) over a tiling of that suffix range prepared on the host.
// A wave keeps its combination count and statistics in registers and adds
// them to the task's words once, when it leaves (prefix tasks can be tiny).
// The search's results do not depend on the schedule; its time does, which is
// what the paper compares.
#include <hip/hip_runtime.h>

#include "bz_internal.h"
#include "bz_kernels.h"
#include "bz_sched.h"
#include "bz_tile.h"
#include "bz_wave.h"

namespace bz {

typedef const __attribute__((address_space(4))) PlanEntry *cptr_plan;

template <int W, bool PARTIAL, bool STATS>
__global__ __launch_bounds__(kBlock) void bz_sched_kernel(SchedArgs s) {
    constexpr int SLOTS = (int)slots_for_w(W);
    extern __shared__ uint64_t smem[];
    const TaskArgs &a0 = s.t;
    const uint32_t bt = a0.g + 1;                          // binomial row stride in LDS
    uint64_t *sbin = smem;                                 // (k+1) x (g+1)
    uint32_t *srow = (uint32_t *)(smem + (size_t)(a0.k + 1) * bt);   // k x W
    for (uint32_t i = threadIdx.x; i < (a0.k + 1) * bt; i += blockDim.x) {
        uint32_t x = i / bt, y = i - x * bt;
        sbin[i] = a0.binom[x * (kBinomT + 1) + y];
    }
    for (uint32_t i = threadIdx.x; i < a0.k * W; i += blockDim.x) srow[i] = a0.rows[i];
    uint32_t *spx = srow + a0.k * W;                     // (k+1) x W prefix XORs
    __syncthreads();
    build_prefix_xor<W>(srow, spx, a0.k);
    __syncthreads();

    const uint32_t lane = threadIdx.x & (kWaveSize - 1);
    cptr32 rows = (cptr32)a0.rows;
    cptr64 binom_c = (cptr64)a0.binom;
    cptr_rect rects = (cptr_rect)s.rects;
    cptr_plan plans = (cptr_plan)s.plans;
    const uint32_t waves_per_block = blockDim.x / kWaveSize;
    const uint64_t worker = (uint64_t)blockIdx.x * waves_per_block + uni(threadIdx.x / kWaveSize);
    const uint64_t nworkers = (uint64_t)gridDim.x * waves_per_block;
    const uint32_t K = a0.k - (a0.g - s.pre);             // prefixes: the pre-subsets of [0, K)

    // The enumeration kernel's stop rule, checked before every tile; the
    // caller's cancel word (host memory, a bus round trip) before every
    // kCancelEvery-th tile of the wave only, as prefix tasks can be tiny.
    constexpr uint32_t kCancelEvery = 32;
    uint32_t polls = 0;
    auto stop_now = [&]() -> bool {
        bool stop = false;
        if (a0.exit_at) {
            unsigned long long kv = __hip_atomic_load(a0.key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            uint32_t cur = min((uint32_t)(kv >> kTileBits), a0.u_prev);
            stop = uni(cur) <= a0.exit_at;
        }
        if (a0.cancel && polls++ % kCancelEvery == 0) {
            uint32_t cv = __hip_atomic_load(a0.cancel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            stop = stop || uni(cv) != 0u;
        }
        return stop;
    };

    TileSum sum;                                           // this wave's count and statistics

    // Process_prefix for one task; true when the wave must stop
    auto run_task = [&](uint64_t task) -> bool {
        uint32_t pre[W];
#pragma unroll
        for (int w = 0; w < W; ++w) pre[w] = 0;
        uint32_t pre_low = 0, last = 0;
        prefix_unrank(s.order, task, s.pre, K,
                      [&](uint32_t x, uint32_t y) -> uint64_t { return binom_c[x * (kBinomT + 1) + y]; },
                      [&](uint32_t, uint32_t c) {
                          const uint32_t row = uni(c);
                          cptr32 rp = rows + row * W;
#pragma unroll
                          for (int w = 0; w < W; ++w) pre[w] ^= rp[w];
                          pre_low += row < a0.k_low ? 1u : 0u;
                          last = max(last, row + 1);
                      });
        const uint32_t lo = s.pre ? uni(last) : 0u;       // completions: rows [lo, k)
        TaskArgs a = a0;
        a.nrects = plans[lo].nrects;
        a.heads_per_tile = plans[lo].heads_per_tile;
        const uint64_t ntiles = plans[lo].total_tiles;
        cptr_rect rp = rects + plans[lo].rect_off;
        for (uint64_t tile = 0; tile < ntiles; ++tile) {
            if (stop_now()) return true;
            run_tile_pre<W, SLOTS, PARTIAL, STATS, true>(a, rows, binom_c, srow, spx, sbin, bt, rp, tile, lane, pre,
                                                         pre_low, task * s.stride + tile, &sum);
        }
        return false;
    };

    if (s.dist == kDistCyclic || s.dist == kDistSnake) {
        for (uint64_t turn = 0; turn * nworkers < s.ntasks; ++turn) {
            const uint64_t task = static_task(s.dist, worker, nworkers, turn, s.ntasks);
            if (task == ~0ull) continue;
            if (run_task(uni64(task))) break;
        }
    } else {
        for (;;) {
            const uint64_t c = wave_fetch_add64_relaxed(a0.tile_ctr, 1ull);   // the task needs no data from the claim
            uint64_t t0 = 0, t1 = 0;
            const uint32_t nt = claim_tasks(s.dist, c, s.ntasks, t0, t1);
            if (nt == 0) break;
            if (run_task(uni64(t0))) break;
            if (nt == 2 && run_task(uni64(t1))) break;
        }
    }
    if (lane == 0 && sum.comb) {
        atomicAdd(a0.ncomb, (unsigned long long)sum.comb);
        if (STATS) stats_merge(a0.stats, sum.min, sum.cnt);
    }
}

// ---------------------------------------------------------------- dispatch

static size_t sched_lds(const SchedArgs &a, uint32_t W) { return enum_lds_bytes(a.t.k, a.t.g, W); }

template <int W>
static const void *sched_fn(bool partial, bool stats) {
    if (stats) return partial ? (const void *)bz_sched_kernel<W, true, true> : (const void *)bz_sched_kernel<W, false, true>;
    return partial ? (const void *)bz_sched_kernel<W, true, false> : (const void *)bz_sched_kernel<W, false, false>;
}

static const void *sched_kernel_for(uint32_t W, bool partial, bool stats) {
    switch (W) {
    case 1: return sched_fn<1>(partial, stats);
    case 2: return sched_fn<2>(partial, stats);
    case 3: return sched_fn<3>(partial, stats);
    case 4: return sched_fn<4>(partial, stats);
    case 5: return sched_fn<5>(partial, stats);
    case 6: return sched_fn<6>(partial, stats);
    case 7: return sched_fn<7>(partial, stats);
    case 8: return sched_fn<8>(partial, stats);
    default: return nullptr;
    }
}

hipError_t launch_sched(const SchedArgs &a, uint32_t W, bool partial, bool stats, uint32_t grid, hipStream_t st) {
    const void *fn = sched_kernel_for(W, partial, stats);
    if (!fn) return hipErrorInvalidValue;
    void *args[] = {(void *)&a};
    return hipLaunchKernel(fn, dim3(grid), dim3(kBlock), args, sched_lds(a, W), st);
}

int sched_blocks_per_cu(uint32_t W, bool partial, bool stats, size_t lds) {
    const void *fn = sched_kernel_for(W, partial, stats);
    int n = 0;
    if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, kBlock, lds) != hipSuccess || n < 1) return 1;
    return n;
}

}  // namespace bz
