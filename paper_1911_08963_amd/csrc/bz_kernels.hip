// HIP kernels for gfx950 behind bz_min_distance: the enumeration of row sums
// of one Gamma matrix at one level (the inner loop of Alg. 1 of
// arXiv:1911.08963), the task reset, and witness recovery. The tile itself
// (decomposition, registers, instruction mix) is described in bz_tile.h.
//
// bz_enum_kernel stages the Gamma_j rows and the binomials C(x, y), x <= k,
// y <= g, in LDS once per work-group, then deals tiles round-robin to its waves
// by uniform arithmetic (tiles of a level cost the same, so no work queue is
// needed inside one task). Before each tile a wave reads the task key and
// stops when the upper bound has reached the certified lower bound (fast mode
// only) or when the caller's cancel word is set. A wave keeps its combination
// count and statistics word in LDS; the work-group adds them to the task's
// words once, when it leaves, and the last work-group to leave applies Alg. 1's
// bookkeeping for the task to the window's state (no launch of its own).
#include <hip/hip_runtime.h>

#include "bz_internal.h"
#include "bz_kernels.h"
#include "bz_tile.h"

namespace bz {

// Alg. 1's bookkeeping after one task of a window, on the device: lower U by
// the task's minimum, and, when the task is complete, raise the certified
// bound (and at the level's end Alg. 1's L) and stop once L reaches U. A task
// that is not complete ended early (certified bound reached, or canceled): the
// search stops. The host replays the same steps on the read-back records.
__device__ void chain_step_apply(const ChainStep &s, unsigned long long key, unsigned long long ncomb) {
    ChainState c = *s.state;
    if (c.done) return;
    const uint32_t tmin = key == ~0ull ? 0xffffffffu : (uint32_t)(key >> kTileBits);
    c.U = min(c.U, tmin);
    if (ncomb != s.total) {
        c.done = 1;
    } else {
        c.Lcert = max(c.Lcert, s.cert_task);
        c.exit_at = s.stats ? 0u : c.Lcert;
        if (!s.level_stop) c.L = max(c.L, c.Lcert);
        if (s.last_of_level) c.L = max(c.L, s.cert_level);
        if ((!s.level_stop || s.last_of_level) && c.L >= c.U) c.done = 1;
    }
    *s.state = c;
}

template <int W, int SLOTS, bool PARTIAL, bool STATS>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu((STATS || PARTIAL) ? 1 : 5))) void bz_enum_kernel(TaskArgs a) {
    // In a window the bounds come from the previous task's step; once the
    // search has stopped the task is empty (the whole work-group leaves).
    uint32_t u_prev = a.u_prev, exit_at = a.exit_at;
    if (a.chain) {
        if (a.chain->done) return;
        u_prev = a.chain->U;
        exit_at = a.chain->exit_at;
    }
    extern __shared__ uint64_t smem[];
    const uint32_t G = a.group > 1 ? a.group : 1u;       // tasks of this launch
    const uint32_t bt = a.g + 1;                          // binomial row stride in LDS
    uint64_t *sbin = smem;                                // (k+1) x (g+1)
    uint32_t *srows = (uint32_t *)(smem + (size_t)(a.k + 1) * bt);   // G x k x W
    uint32_t *spxs = srows + (size_t)G * a.k * W;         // G x (k+1) x W prefix XORs
    for (uint32_t i = threadIdx.x; i < (a.k + 1) * bt; i += blockDim.x) {
        uint32_t x = i / bt, y = i - x * bt;
        sbin[i] = a.binom[x * (kBinomT + 1) + y];
    }
    for (uint32_t i = threadIdx.x; i < G * a.k * W; i += blockDim.x) {
        const uint32_t ti = i / (a.k * W), r = i - ti * (a.k * W);
        srows[i] = a.rows[(size_t)ti * a.rows_stride + r];
    }
    __syncthreads();
    for (uint32_t ti = 0; ti < G; ++ti) build_prefix_xor<W>(srows + ti * a.k * W, spxs + ti * (a.k + 1) * W, a.k);
    __syncthreads();

    const uint32_t lane = threadIdx.x & (kWaveSize - 1);
    cptr_rect rect_p = (cptr_rect)a.rects;
    cptr64 binom_c = (cptr64)a.binom;
    // Static round-robin of tiles over waves: the tile index is uniform
    // arithmetic only (tiles of a level cost the same, so no work queue is
    // needed inside one task).
    const uint32_t waves_per_block = blockDim.x / kWaveSize;
    const uint64_t first = (uint64_t)blockIdx.x * waves_per_block + uni(threadIdx.x / kWaveSize);
    const uint64_t stride = (uint64_t)gridDim.x * waves_per_block;
    // The wave's combination count and statistics word live in LDS until it
    // leaves: one global atomic per wave instead of one per tile on the same
    // word (on a level of many short tiles those serialise the whole launch).
    __shared__ unsigned long long wave_words[kBlock / kWaveSize][kMaxGroup][2];
    const uint32_t wv = uni(threadIdx.x / kWaveSize);
    if (lane == 0)
        for (uint32_t ti = 0; ti < kMaxGroup; ++ti) {
            wave_words[wv][ti][0] = 0;
            wave_words[wv][ti][1] = ~0ull;               // "none", as the task's own word starts
        }
    TaskArgs t = a;
    for (uint64_t it = first; it < G * a.total_tiles; it += stride) {
        // tile of task ti (all tasks of a group share the tiling)
        const uint32_t ti = uni((uint32_t)(it / a.total_tiles));
        const uint64_t tile = uni64(it - (uint64_t)ti * a.total_tiles);
        if (a.cancel) {
            uint32_t cv = __hip_atomic_load(a.cancel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            if (uni(cv) != 0u) break;
        }
        t.rows = a.rows + (size_t)ti * a.rows_stride;
        t.key = a.key + (size_t)ti * kRecWords;
        t.ncomb = &wave_words[wv][ti][0];
        t.stats = &wave_words[wv][ti][1];
        if (exit_at) {
            // the task's own minimum and the bound from before the launch: a
            // later task of the group may not cut an earlier one short
            unsigned long long kv = __hip_atomic_load(t.key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            uint32_t cur = min((uint32_t)(kv >> kTileBits), u_prev);
            if (uni(cur) <= exit_at) continue;
        }
        cptr32 rows = (cptr32)uni64((uint64_t)t.rows);
        run_tile<W, SLOTS, PARTIAL, STATS>(t, rows, binom_c, srows + ti * a.k * W, spxs + ti * (a.k + 1) * W, sbin,
                                           bt, rect_p, tile, lane);
    }
    // One global atomic per work-group, not per wave: when the waves of a
    // short level end together, atomics on the same word queue up at the
    // memory side (measured: the last of 2,441 waves of a C(64,6) level waited
    // 12-19 us there).
    __syncthreads();
    if (threadIdx.x == 0) {
        for (uint32_t ti = 0; ti < G; ++ti) {
            unsigned long long nc = 0;
            uint32_t smin = 0xffffffffu;
            uint64_t scnt = 0;
            for (uint32_t w = 0; w < kBlock / kWaveSize; ++w) {
                nc += wave_words[w][ti][0];
                const unsigned long long sw = wave_words[w][ti][1];
                if (STATS && wave_words[w][ti][0] && sw != ~0ull) {
                    const uint32_t m = (uint32_t)(sw >> kCountBits);
                    if (m < smin) { smin = m; scnt = sw & kCountMask; }
                    else if (m == smin) scnt += sw & kCountMask;
                }
            }
            if (nc) {
                atomicAdd(a.ncomb + (size_t)ti * kRecWords, nc);
                if (STATS && smin != 0xffffffffu) stats_merge(a.stats + (size_t)ti * kRecWords, smin, scnt);
            }
        }
        if (a.step.state) {
            // the last work-group to leave applies the tasks' bookkeeping
            // steps, in Alg. 1's order, in place of launches of their own:
            // every other work-group's atomics are ordered before its count
            // (release), and read after the last count (acquire)
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            const unsigned long long left = atomicAdd(a.tile_ctr, 1ull);
            if (left + 1 == gridDim.x) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                for (uint32_t ti = 0; ti < G; ++ti) {
                    ChainStep s = a.step;
                    s.key = a.key + (size_t)ti * kRecWords;
                    s.ncomb = a.ncomb + (size_t)ti * kRecWords;
                    if (G > 1) {
                        s.cert_task = a.cert_tasks[ti];
                        s.last_of_level = (a.last_mask >> ti) & 1u;
                    }
                    chain_step_apply(s, __hip_atomic_load(s.key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                                     __hip_atomic_load(s.ncomb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                }
            }
        }
    }
}

// Consecutive tasks of several small levels in one launch (a group spanning
// level ends, LevelsArgs): the same staging, tiles and bookkeeping as
// bz_enum_kernel, with each task's tiling, level and step read from a table in
// LDS once per tile. Tasks of a later level run before the earlier ones'
// steps have been applied: with the bounds from before the launch, so they
// may enumerate more than Alg. 1 would, never less, and their steps are
// applied in order by the last work-group (a step after the stop does
// nothing).
template <int W, int SLOTS, bool STATS>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(STATS ? 1 : 5))) void bz_enum_levels_kernel(LevelsArgs la) {
    const TaskArgs &a = la.t;
    if (a.chain->done) return;
    const uint32_t u_prev = a.chain->U, exit_at = a.chain->exit_at;
    extern __shared__ uint64_t smem[];
    const uint32_t G = la.ntasks;
    const uint32_t bt = a.g + 1;                          // largest level: binomial row stride in LDS
    uint64_t *sbin = smem;                                // (k+1) x (g+1)
    uint32_t *srows = (uint32_t *)(smem + (size_t)(a.k + 1) * bt);   // G x k x W
    uint32_t *spxs = srows + (size_t)G * a.k * W;         // G x (k+1) x W prefix XORs
    __shared__ uint64_t s_tile_end[kMaxLevelTasks];
    __shared__ uint32_t s_task[kMaxLevelTasks][5];        // rectangles, level, rectangle count, heads, rows
    for (uint32_t i = threadIdx.x; i < (a.k + 1) * bt; i += blockDim.x) {
        uint32_t x = i / bt, y = i - x * bt;
        sbin[i] = a.binom[x * (kBinomT + 1) + y];
    }
    for (uint32_t i = threadIdx.x; i < G * a.k * W; i += blockDim.x) {
        const uint32_t ti = i / (a.k * W), r = i - ti * (a.k * W);
        srows[i] = a.rows[la.row_off[ti] + r];
    }
    if (threadIdx.x < G) {
        const uint32_t q = threadIdx.x;
        s_tile_end[q] = la.tile_end[q];
        s_task[q][0] = la.rect_off[q];
        s_task[q][1] = la.g[q];
        s_task[q][2] = la.nrects[q];
        s_task[q][3] = la.heads[q];
        s_task[q][4] = la.row_off[q];
    }
    __syncthreads();
    for (uint32_t ti = 0; ti < G; ++ti) build_prefix_xor<W>(srows + ti * a.k * W, spxs + ti * (a.k + 1) * W, a.k);
    __syncthreads();

    const uint32_t lane = threadIdx.x & (kWaveSize - 1);
    cptr64 binom_c = (cptr64)a.binom;
    const uint32_t waves_per_block = blockDim.x / kWaveSize;
    const uint64_t first = (uint64_t)blockIdx.x * waves_per_block + uni(threadIdx.x / kWaveSize);
    const uint64_t stride = (uint64_t)gridDim.x * waves_per_block;
    __shared__ unsigned long long wave_words[kBlock / kWaveSize][kMaxLevelTasks][2];
    const uint32_t wv = uni(threadIdx.x / kWaveSize);
    if (lane == 0)
        for (uint32_t ti = 0; ti < kMaxLevelTasks; ++ti) {
            wave_words[wv][ti][0] = 0;
            wave_words[wv][ti][1] = ~0ull;
        }
    TaskArgs t = a;
    for (uint64_t it = first; it < a.total_tiles; it += stride) {
        // the group's tasks take consecutive ranges of the launch's tiles
        uint32_t ti = 0;
        while (ti + 1 < G && it >= uni64(s_tile_end[ti])) ++ti;
        const uint64_t tile = it - (ti ? uni64(s_tile_end[ti - 1]) : 0ull);
        const cptr_rect rp = (cptr_rect)a.rects + uni(s_task[ti][0]);
        t.g = uni(s_task[ti][1]);
        t.nrects = uni(s_task[ti][2]);
        t.heads_per_tile = uni(s_task[ti][3]);
        t.rows = a.rows + uni(s_task[ti][4]);
        if (a.cancel) {
            uint32_t cv = __hip_atomic_load(a.cancel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            if (uni(cv) != 0u) break;
        }
        t.key = a.key + (size_t)ti * kRecWords;
        t.ncomb = &wave_words[wv][ti][0];
        t.stats = &wave_words[wv][ti][1];
        if (exit_at) {
            unsigned long long kv = __hip_atomic_load(t.key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            uint32_t cur = min((uint32_t)(kv >> kTileBits), u_prev);
            if (uni(cur) <= exit_at) continue;
        }
        cptr32 rows = (cptr32)uni64((uint64_t)t.rows);
        run_tile<W, SLOTS, false, STATS>(t, rows, binom_c, srows + ti * a.k * W, spxs + ti * (a.k + 1) * W, sbin,
                                         bt, rp, tile, lane);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (uint32_t ti = 0; ti < G; ++ti) {
            unsigned long long nc = 0;
            uint32_t smin = 0xffffffffu;
            uint64_t scnt = 0;
            for (uint32_t w = 0; w < kBlock / kWaveSize; ++w) {
                nc += wave_words[w][ti][0];
                const unsigned long long sw = wave_words[w][ti][1];
                if (STATS && wave_words[w][ti][0] && sw != ~0ull) {
                    const uint32_t m = (uint32_t)(sw >> kCountBits);
                    if (m < smin) { smin = m; scnt = sw & kCountMask; }
                    else if (m == smin) scnt += sw & kCountMask;
                }
            }
            if (nc) {
                atomicAdd(a.ncomb + (size_t)ti * kRecWords, nc);
                if (STATS && smin != 0xffffffffu) stats_merge(a.stats + (size_t)ti * kRecWords, smin, scnt);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned long long left = atomicAdd(a.tile_ctr, 1ull);
        if (left + 1 == gridDim.x) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            for (uint32_t ti = 0; ti < G; ++ti) {
                ChainStep s = a.step;
                s.key = a.key + (size_t)ti * kRecWords;
                s.ncomb = a.ncomb + (size_t)ti * kRecWords;
                s.total = la.totals[ti];
                s.cert_task = la.cert_task[ti];
                s.cert_level = la.cert_level[ti];
                s.last_of_level = (la.last_mask >> ti) & 1u;
                chain_step_apply(s, __hip_atomic_load(s.key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                                 __hip_atomic_load(s.ncomb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            }
        }
    }
}

// Resets a task's device words: key and statistics to "none", counters to 0.
__global__ void bz_task_init_kernel(unsigned long long *key, unsigned long long *stats,
                                    unsigned long long *ncomb, unsigned long long *ctr) {
    if (threadIdx.x == 0) {
        *key = ~0ull;
        *stats = ~0ull;
        *ncomb = 0;
        *ctr = 0;
    }
}

// Resets the records of a window's tasks (key and statistics to "none",
// counts to 0), writes the bounds the window starts from, and clears the
// witness flag when given.
__global__ void bz_chain_init_kernel(unsigned long long *records, uint32_t n, ChainState *state, ChainState init,
                                     unsigned int *clear) {
    const uint32_t i = threadIdx.x;
    if (i < n) {
        unsigned long long *r = records + (size_t)i * kRecWords;
        r[kRecKey] = ~0ull;
        r[kRecStats] = ~0ull;
        r[kRecNcomb] = 0;
        r[kRecCtr] = 0;
    }
    if (i == 0) *state = init;
    if (i == 1 && clear) *clear = 0u;
}

// Witness recovery: one thread per combination of the winning tile, each
// computed from scratch (no shared state with the enumeration kernel), joined
// to the rows of the tile's prefix task when it has one. The first thread
// whose combination has the target weight writes its row indices and the
// codeword (XOR of the full rows, original coordinates).
// bn, bstride: the binomials C(x, y) at bn[x * bstride + y] (the device table,
// or a work-group's copy in LDS).
__device__ void recover_tile(const RecoverArgs &a, uint64_t id, const uint64_t *bn, uint32_t bstride) {
    const Rect R = a.rect;
    // the tile's lane subsets: lane_mult blocks of 64 * slots
    const uint64_t lane_items = (uint64_t)kWaveSize * a.slots * (R.lane_mult ? R.lane_mult : 1u);
    const uint64_t local = a.tile - R.tile_begin;
    const uint64_t lb = local / R.head_blocks, hb = local - lb * R.head_blocks;
    const uint64_t li = id % lane_items, hs = id / lane_items;
    const uint64_t q = (uint64_t)lb * lane_items + li;
    const uint64_t h = (uint64_t)hb * a.heads_per_tile + hs;
    if (hs >= a.heads_per_tile || q >= R.lane_count || h >= R.head_count) return;
    uint32_t idx[kBinomT];
    uint32_t cnt = 0;
    uint32_t word[kMaxW];
    for (int w = 0; w < kMaxW; ++w) word[w] = 0;
    uint32_t ident = 0;
    auto add_subset = [&](uint64_t r, uint32_t t, uint32_t off, uint32_t nside) {
        uint32_t hi = nside - 1;
        for (uint32_t i = t; i >= 1; --i) {
            uint32_t lo = i - 1, c = hi;
            while (lo < c) {
                uint32_t mid = (lo + c + 1) >> 1;
                if (bn[mid * bstride + i] <= r) lo = mid; else c = mid - 1;
            }
            r -= bn[lo * bstride + i];
            const uint32_t row = off + lo;
            idx[cnt++] = row;
            for (uint32_t w = 0; w < a.W; ++w) word[w] ^= a.rows[row * a.W + w];
            ident += row < a.k_low ? 1u : 0u;
            hi = lo - 1;
        }
    };
    for (uint32_t i = 0; i < a.pre_n; ++i) {          // a prefix task's rows
        const uint32_t row = a.pre_rows[i];
        idx[cnt++] = row;
        for (uint32_t w = 0; w < a.W; ++w) word[w] ^= a.rows[row * a.W + w];
        ident += row < a.k_low ? 1u : 0u;
    }
    add_subset(q, R.lane_t, R.lane_off, R.lane_n);
    if (R.head_t) add_subset(h, R.head_t, R.head_off, R.head_n);
    uint32_t wgt = ident;
    for (uint32_t w = 0; w < a.W; ++w) wgt += __builtin_popcount(word[w]);
    if (wgt != a.target) return;
    if (atomicCAS(a.flag, 0u, 1u) != 0u) return;
    uint64_t cw[kHostWords];
    for (int w = 0; w < kHostWords; ++w) cw[w] = 0;
    for (uint32_t i = 0; i < cnt; ++i)
        for (int w = 0; w < kHostWords; ++w) cw[w] ^= a.full_rows[(size_t)idx[i] * kHostWords + w];
    for (int w = 0; w < kHostWords; ++w) a.codeword[w] = cw[w];
    for (uint32_t i = 0; i < cnt; ++i) a.indices[i] = idx[i];
    a.indices_len[0] = cnt;
}

__global__ void bz_recover_kernel(RecoverArgs a) {
    recover_tile(a, (uint64_t)blockIdx.x * blockDim.x + threadIdx.x, a.binom, kBinomT + 1);
}

// The window's winning task, by the host's rule (the first task whose minimum
// reaches the final upper bound), then the same per-thread recovery over its
// tile. Nothing happens unless the window stopped the search and the winner
// is one of its tasks: then the host recovers the witness itself.
__global__ void bz_recover_window_kernel(RecoverWindowArgs a) {
    if (!a.state->done) return;
    // the binomials C(x, y), x <= k, y <= lds_g, in LDS when the launch has room
    extern __shared__ uint64_t rbin[];
    const uint64_t *bn = a.binom;
    uint32_t bstride = kBinomT + 1;
    if (a.lds_g) {
        bstride = a.lds_g + 1;
        for (uint32_t i = threadIdx.x; i < (a.k + 1) * bstride; i += blockDim.x) {
            const uint32_t x = i / bstride, y = i - x * bstride;
            rbin[i] = a.binom[x * (kBinomT + 1) + y];
        }
        __syncthreads();
        bn = rbin;
    }
    uint32_t U = a.U0;
    bool have = a.have0 != 0;
    int best = -1;
    uint64_t tile = 0;
    for (uint32_t i = 0; i < a.ntasks; ++i) {
        const unsigned long long key = a.records[(size_t)i * kRecWords + kRecKey];
        const uint32_t tmin = key == ~0ull ? 0xffffffffu : (uint32_t)(key >> kTileBits);
        if (tmin < U || (tmin == U && !have)) {
            U = tmin;
            have = true;
            best = (int)i;
            tile = key & kTileMask;
        }
    }
    if (best < 0) return;
    const RecoverTask T = a.tasks[best];
    uint32_t lo = 0, hi = T.nrects - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (T.rects[mid].tile_begin <= tile) lo = mid; else hi = mid - 1;
    }
    RecoverArgs r{};
    r.rows = T.rows;
    r.full_rows = T.full_rows;
    r.binom = a.binom;
    r.rect = T.rects[lo];
    r.flag = a.flag;
    r.indices = a.indices;
    r.indices_len = a.indices_len;
    r.codeword = a.codeword;
    r.tile = tile;
    r.slots = T.slots;
    r.heads_per_tile = T.heads_per_tile;
    r.W = T.W;
    r.k_low = T.k_low;
    r.target = U;
    r.pre_n = 0;
    // a grid-stride walk over the tile's combinations, left once one is found
    const uint64_t n = (uint64_t)kWaveSize * T.slots * (r.rect.lane_mult ? r.rect.lane_mult : 1u) * T.heads_per_tile;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t id = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; id < n; id += stride) {
        recover_tile(r, id, bn, bstride);
        if (__hip_atomic_load(a.flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
    }
}

// ---------------------------------------------------------------- dispatch

template <int W, int SLOTS, bool PARTIAL, bool STATS>
static hipError_t launch_one(const TaskArgs &a, uint32_t grid, size_t lds, hipStream_t st) {
    hipLaunchKernelGGL((bz_enum_kernel<W, SLOTS, PARTIAL, STATS>), dim3(grid), dim3(kBlock), lds, st, a);
    return hipGetLastError();
}

template <int W, int SLOTS>
static hipError_t launch_ws(const TaskArgs &a, bool partial, bool stats, uint32_t grid, size_t lds,
                            hipStream_t st) {
    if (stats) {
        return partial ? launch_one<W, SLOTS, true, true>(a, grid, lds, st)
                       : launch_one<W, SLOTS, false, true>(a, grid, lds, st);
    }
    return partial ? launch_one<W, SLOTS, true, false>(a, grid, lds, st)
                   : launch_one<W, SLOTS, false, false>(a, grid, lds, st);
}

template <int W>
static hipError_t launch_w(const TaskArgs &a, uint32_t slots, bool partial, bool stats, uint32_t grid,
                           size_t lds, hipStream_t st) {
    switch (slots) {
    case 2: return launch_ws<W, 2>(a, partial, stats, grid, lds, st);
    case 4: return launch_ws<W, 4>(a, partial, stats, grid, lds, st);
    case 8: return launch_ws<W, 8>(a, partial, stats, grid, lds, st);
    case 16:
        if constexpr (W <= 4) return launch_ws<W, 16>(a, partial, stats, grid, lds, st);
        return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_enum(const TaskArgs &a, uint32_t W, uint32_t slots, bool partial, bool stats,
                       uint32_t grid, hipStream_t st) {
    const size_t lds = enum_lds_bytes(a.k, a.g, W, a.group);
    switch (W) {
    case 1: return launch_w<1>(a, slots, partial, stats, grid, lds, st);
    case 2: return launch_w<2>(a, slots, partial, stats, grid, lds, st);
    case 3: return launch_w<3>(a, slots, partial, stats, grid, lds, st);
    case 4: return launch_w<4>(a, slots, partial, stats, grid, lds, st);
    case 5: return launch_w<5>(a, slots, partial, stats, grid, lds, st);
    case 6: return launch_w<6>(a, slots, partial, stats, grid, lds, st);
    case 7: return launch_w<7>(a, slots, partial, stats, grid, lds, st);
    case 8: return launch_w<8>(a, slots, partial, stats, grid, lds, st);
    default: return hipErrorInvalidValue;
    }
}

template <int W>
static hipError_t launch_levels_w(const LevelsArgs &a, uint32_t slots, bool stats, uint32_t grid, size_t lds,
                                  hipStream_t st) {
#define BZ_LEVELS(S)                                                                                         \
    do {                                                                                                     \
        if (stats) hipLaunchKernelGGL((bz_enum_levels_kernel<W, S, true>), dim3(grid), dim3(kBlock), lds, st, a);  \
        else hipLaunchKernelGGL((bz_enum_levels_kernel<W, S, false>), dim3(grid), dim3(kBlock), lds, st, a);        \
        return hipGetLastError();                                                                            \
    } while (0)
    switch (slots) {
    case 2: BZ_LEVELS(2);
    case 4: BZ_LEVELS(4);
    case 8: BZ_LEVELS(8);
    case 16:
        if constexpr (W <= 4) BZ_LEVELS(16);
        return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
#undef BZ_LEVELS
}

hipError_t launch_enum_levels(const LevelsArgs &a, uint32_t W, uint32_t slots, bool stats, uint32_t grid,
                              hipStream_t st) {
    if (a.ntasks < 2 || a.ntasks > kMaxLevelTasks || !a.t.chain || !a.t.step.state) return hipErrorInvalidValue;
    const size_t lds = enum_lds_bytes(a.t.k, a.t.g, W, a.ntasks);
    switch (W) {
    case 1: return launch_levels_w<1>(a, slots, stats, grid, lds, st);
    case 2: return launch_levels_w<2>(a, slots, stats, grid, lds, st);
    case 3: return launch_levels_w<3>(a, slots, stats, grid, lds, st);
    case 4: return launch_levels_w<4>(a, slots, stats, grid, lds, st);
    case 5: return launch_levels_w<5>(a, slots, stats, grid, lds, st);
    case 6: return launch_levels_w<6>(a, slots, stats, grid, lds, st);
    case 7: return launch_levels_w<7>(a, slots, stats, grid, lds, st);
    case 8: return launch_levels_w<8>(a, slots, stats, grid, lds, st);
    default: return hipErrorInvalidValue;
    }
}

size_t enum_lds_bytes(uint32_t k, uint32_t g, uint32_t W, uint32_t group) {
    // binomials, then per task of the group its rows and their prefix XORs
    return (size_t)(k + 1) * (g + 1) * sizeof(uint64_t) +
           (size_t)(group > 1 ? group : 1) * (2 * k + 1) * W * sizeof(uint32_t);
}

hipError_t launch_task_init(unsigned long long *key, unsigned long long *stats, unsigned long long *ncomb,
                            unsigned long long *ctr, hipStream_t st) {
    hipLaunchKernelGGL(bz_task_init_kernel, dim3(1), dim3(64), 0, st, key, stats, ncomb, ctr);
    return hipGetLastError();
}

hipError_t launch_chain_init(unsigned long long *records, uint32_t n, ChainState *state, const ChainState &init,
                             unsigned int *clear, hipStream_t st) {
    if (n > 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(bz_chain_init_kernel, dim3(1), dim3(64), 0, st, records, n, state, init, clear);
    return hipGetLastError();
}

hipError_t launch_recover_window(const RecoverWindowArgs &a, uint64_t threads, hipStream_t st) {
    const uint32_t grid = (uint32_t)std::min<uint64_t>((threads + 255) / 256, 2048);
    const size_t lds = a.lds_g ? (size_t)(a.k + 1) * (a.lds_g + 1) * sizeof(uint64_t) : 0;
    hipLaunchKernelGGL(bz_recover_window_kernel, dim3(grid), dim3(256), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_recover(const RecoverArgs &a, hipStream_t st) {
    const uint64_t total =
        (uint64_t)kWaveSize * a.slots * (a.rect.lane_mult ? a.rect.lane_mult : 1u) * a.heads_per_tile;
    const uint32_t grid = (uint32_t)((total + 255) / 256);
    hipLaunchKernelGGL(bz_recover_kernel, dim3(grid), dim3(256), 0, st, a);
    return hipGetLastError();
}

// Issue-rate probe: 8 independent XOR+popcount chains per lane, the same
// instruction pair as the enumeration (v_xor with an SGPR operand, then
// v_bcnt_u32_b32 accumulating). One store per lane keeps the chains alive.
__global__ __launch_bounds__(kBlock) void bz_valu_probe_kernel(uint32_t iters, uint32_t s0, uint32_t s1,
                                                               uint32_t *sink) {
    uint32_t a[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) a[c] = threadIdx.x * 2654435761u + (uint32_t)c * 40503u + blockIdx.x;
    const uint32_t u0 = uni(s0), u1 = uni(s1);
    for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < 8; ++c) a[c] = bcnt_acc(a[c] ^ ((c & 1) ? u1 : u0), a[c]);
    }
    uint32_t x = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c) x ^= a[c];
    sink[blockIdx.x * kBlock + threadIdx.x] = x;
}

hipError_t launch_valu_probe(uint32_t iters, uint32_t blocks, uint32_t *sink, hipStream_t st) {
    hipLaunchKernelGGL(bz_valu_probe_kernel, dim3(blocks), dim3(kBlock), 0, st, iters, 0x9e3779b9u, 0x7f4a7c15u,
                       sink);
    return hipGetLastError();
}

int valu_probe_blocks_per_cu() {
    int n = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, bz_valu_probe_kernel, kBlock, 0);
    return (e == hipSuccess && n > 0) ? n : 1;
}

}  // namespace bz
