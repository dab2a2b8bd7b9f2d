// Codewords of a given weight w: the collect kernel behind
// bz_count_codewords. It enumerates one task (Gamma_j, g) with the same tiles
// as the search (bz_tile.h) and, for every combination whose codeword has
// weight exactly w, appends the combination's coordinates (tile, lane-subset
// rank, head rank) to an output list. Such combinations are rare, so the
// check after each head step is one ballot over the wave and the appends are
// per-lane atomics taken only when a lane has a hit.
#include <hip/hip_runtime.h>

#include "bz_internal.h"
#include "bz_kernels.h"
#include "bz_tile.h"

namespace bz {

template <int W, int SLOTS>
__global__ __launch_bounds__(kBlock) void bz_collect_kernel(CollectArgs a) {
    extern __shared__ uint64_t smem[];
    const uint32_t bt = a.g + 1;                          // binomial row stride in LDS
    uint64_t *sbin = smem;                                // (k+1) x (g+1)
    uint32_t *srow = (uint32_t *)(smem + (size_t)(a.k + 1) * bt);   // k x W
    for (uint32_t i = threadIdx.x; i < (a.k + 1) * bt; i += blockDim.x) {
        uint32_t x = i / bt, y = i - x * bt;
        sbin[i] = a.binom[x * (kBinomT + 1) + y];
    }
    for (uint32_t i = threadIdx.x; i < a.k * W; i += blockDim.x) srow[i] = a.rows[i];
    uint32_t *spx = srow + a.k * W;                      // (k+1) x W prefix XORs
    __syncthreads();
    build_prefix_xor<W>(srow, spx, a.k);
    __syncthreads();

    const uint32_t lane = threadIdx.x & (kWaveSize - 1);
    cptr32 rows = (cptr32)a.rows;
    cptr_rect rect_p = (cptr_rect)a.rects;
    cptr64 binom_c = (cptr64)a.binom;
    const uint32_t waves_per_block = blockDim.x / kWaveSize;
    const uint64_t first = (uint64_t)blockIdx.x * waves_per_block + uni(threadIdx.x / kWaveSize);
    const uint64_t stride = (uint64_t)gridDim.x * waves_per_block;
    for (uint64_t it = first; it < a.total_tiles; it += stride) {
        const uint64_t tile = uni64(it);
        const TileGeom t = locate_tile(a.nrects, rect_p, tile);
        const uint64_t h0 = t.hb * a.heads_per_tile;
        const uint64_t count = umin64(h0 + a.heads_per_tile, t.head_count) - h0;
        uint64_t nvalid = 0;
        for (uint32_t sb = 0; sb < t.lane_mult; ++sb) {
            const uint64_t base = (t.lb * t.lane_mult + sb) * (uint64_t)(kWaveSize * SLOTS);
            if (base >= t.lane_count) break;
            uint32_t P[SLOTS][W], low[SLOTS], pen[SLOTS], none[W];
#pragma unroll
            for (int w = 0; w < W; ++w) none[w] = 0;
            nvalid += lane_setup<W, SLOTS>(t, base, a.k_low, srow, spx, sbin, bt, lane, none, 0u, P, low, pen);
            head_walk<W, true>(t, rows, binom_c, a.k_low, h0, count,
                               [&](const uint32_t (&H)[W], uint32_t hl, uint32_t step) {
                uint32_t hit = 0;
#pragma unroll
                for (int s = 0; s < SLOTS; ++s) {
                    uint32_t v = bcnt_acc_s(H[0] ^ P[s][0], hl);
#pragma unroll
                    for (int w = 1; w < W; ++w) v = bcnt_acc(H[w] ^ P[s][w], v);
                    hit |= (v + low[s] + pen[s] == a.target) ? (1u << s) : 0u;
                }
                if (__builtin_amdgcn_ballot_w64(hit != 0) == 0) return false;
                for (int s = 0; s < SLOTS; ++s) {
                    if (!((hit >> s) & 1u)) continue;
                    const unsigned long long idx = atomicAdd(a.nhits, 1ull);
                    if (idx < a.cap) {
                        CollectHit &o = a.hits[idx];
                        o.tile = tile;
                        o.q = base + (uint64_t)lane * SLOTS + s;
                        o.h = h0 + step;
                    }
                }
                return false;
            });
        }
        if (lane == 0) atomicAdd(a.ncomb, (unsigned long long)nvalid * count);
    }
}

template <int W, int SLOTS>
static hipError_t launch_collect_w(const CollectArgs &a, uint32_t grid, size_t lds, hipStream_t st) {
    hipLaunchKernelGGL((bz_collect_kernel<W, SLOTS>), dim3(grid), dim3(kBlock), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_collect(const CollectArgs &a, uint32_t W, uint32_t grid, hipStream_t st) {
    const size_t lds = (size_t)(a.k + 1) * (a.g + 1) * sizeof(uint64_t) + (size_t)(2 * a.k + 1) * W * sizeof(uint32_t);
    switch (W) {
#define BZ_COLLECT(WW) \
    case WW: return launch_collect_w<WW, slots_for_w(WW)>(a, grid, lds, st);
        BZ_COLLECT(1) BZ_COLLECT(2) BZ_COLLECT(3) BZ_COLLECT(4)
        BZ_COLLECT(5) BZ_COLLECT(6) BZ_COLLECT(7) BZ_COLLECT(8)
#undef BZ_COLLECT
    default: return hipErrorInvalidValue;
    }
}

}  // namespace bz
