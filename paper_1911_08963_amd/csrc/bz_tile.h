// Device code shared by the enumeration kernels: one wave tile of one
// (Gamma_j, g) task, plus the small helpers it needs. Included by the HIP
// sources only.
//
// A level of Gamma_j is a list of rectangles (bz_plan.cpp), each the product
// of a lane factor (lane_t-subsets of one row range) and a head factor
// (head_t-subsets of another, at most 64 rows). A wave tile is 64 * SLOTS
// lane subsets by up to heads_per_tile consecutive head subsets in colex
// order.
//  - Lanes: each lane unranks its SLOTS lane subsets (combinatorial number
//    system) and keeps their XOR sums P[s] in VGPRs.
//  - Head: the whole wave steps the head subset as a 64-bit mask in SGPRs. The
//    smallest element runs fastest: H = S2 ^ row[e], where S2 is the XOR of
//    the other head rows and changes only when the smallest element wraps
//    (a Gosper step on the mask). Rows come through scalar loads, one row ahead.
//  - Per combination, per 32-bit word: one v_xor (SGPR ^ VGPR) and one
//    v_bcnt (popcount plus accumulate); one v_min3 folds two combinations
//    into the running minimum: 2W + 1/2 VALU operations per combination. The
//    identity part of a full-rank Gamma_j weighs exactly g, added per tile.
//  - The partial Gamma_m weighs |c & [0, k_m)| on its identity part: the head's
//    share enters through the bcnt accumulator (an SGPR operand), the lane's
//    share is added per slot when the tile ends.
//  - End of a tile: a wave-wide minimum, then one 64-bit atomicMin of
//    (weight << 55 | tile) into the task key; in statistics mode also the
//    number of combinations reaching the tile minimum, merged by a CAS loop.
#pragma once

#include <hip/hip_runtime.h>

#include "bz_internal.h"
#include "bz_kernels.h"

namespace bz {

typedef const __attribute__((address_space(4))) uint32_t *cptr32;
typedef const __attribute__((address_space(4))) uint64_t *cptr64;
typedef const __attribute__((address_space(4))) Rect *cptr_rect;

__device__ __forceinline__ uint32_t uni(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint64_t uni64(uint64_t x) {
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t umin64(uint64_t a, uint64_t b) { return a < b ? a : b; }

__device__ __forceinline__ uint32_t wave_min(uint32_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, off, 64));
    return v;
}
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += (uint32_t)__shfl_xor((int)v, off, 64);
    return v;
}

// Popcount-accumulate and three-way minimum as single VALU instructions.
// Written as ALU-only inline assembly so that the compiler keeps the
// accumulate chain (it would otherwise split it into separate counts joined
// by v_add3, and fold pairwise minima into a deeper tree).
__device__ __forceinline__ uint32_t bcnt_acc(uint32_t x, uint32_t acc) {
    uint32_t r;
    asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(r) : "v"(x), "v"(acc));
    return r;
}
__device__ __forceinline__ uint32_t bcnt_acc_s(uint32_t x, uint32_t acc_uniform) {
    uint32_t r;
    asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(r) : "v"(x), "s"(acc_uniform));
    return r;
}
__device__ __forceinline__ uint32_t min3u(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t r;
    asm("v_min3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// Statistics word: minimum in the top 9 bits, count in the low 55.
constexpr int kCountBits = 55;
constexpr unsigned long long kCountMask = (1ull << kCountBits) - 1;

__device__ void stats_merge(unsigned long long *p, uint32_t w, uint64_t cnt) {
    unsigned long long mine = ((unsigned long long)w << kCountBits) | (cnt & kCountMask);
    unsigned long long old = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (;;) {
        uint32_t ow = (uint32_t)(old >> kCountBits);
        unsigned long long nv;
        if (w < ow) nv = mine;
        else if (w > ow) return;
        else nv = old + (cnt & kCountMask);
        if (__hip_atomic_compare_exchange_strong(p, &old, nv, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT))
            return;
    }
}

// Largest c in [lo, hi] with C(c, i) <= r; binomials from LDS (row stride bt).
__device__ __forceinline__ uint32_t colex_digit(const uint64_t *sb, uint32_t bt, uint32_t i,
                                                 uint32_t lo, uint32_t hi, uint64_t r) {
    while (lo < hi) {
        uint32_t mid = (lo + hi + 1) >> 1;
        if (sb[mid * bt + i] <= r) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// The same digit and its binomial C(c, i), with few dependent look-ups: the
// start is the root of C(c, i) ~ (c - (i - 1)/2)^i / i! (lf = log2(i!)), and
// steps up or down correct it, so the result is exact whatever the estimate
// (C(i - 1, i) = 0 <= r ends the way down, c <= hi the way up). Two
// independent look-ups usually settle a digit, where a bisection costs one
// dependent look-up per halving of [i - 1, hi].
__device__ __forceinline__ uint32_t colex_digit_est(const uint64_t *sb, uint32_t bt, uint32_t i, uint32_t hi,
                                                    uint64_t r, float lf, uint64_t &bc) {
    const float fi = (float)i;
    const float root =
        __builtin_amdgcn_exp2f((__builtin_amdgcn_logf((float)r) + lf) * __builtin_amdgcn_rcpf(fi));
    uint32_t c = (uint32_t)fminf(fmaxf(root + 0.5f * (fi - 1.0f), fi - 1.0f), (float)hi);
    uint64_t b0 = sb[c * bt + i];
    uint64_t b1 = c < hi ? sb[(c + 1) * bt + i] : ~0ull;
    if (b0 > r) {
        do {
            --c;
            b0 = sb[c * bt + i];
        } while (b0 > r);
    } else {
        while (b1 <= r) {
            ++c;
            b0 = b1;
            b1 = c < hi ? sb[(c + 1) * bt + i] : ~0ull;
        }
    }
    bc = b0;
    return c;
}

// The same for uniform values, with binomials through the scalar cache.
__device__ __forceinline__ uint32_t colex_digit_s(cptr64 gb, uint32_t i, uint32_t lo, uint32_t hi,
                                                   uint64_t r) {
    while (lo < hi) {
        uint32_t mid = (lo + hi + 1) >> 1;
        if (gb[mid * (kBinomT + 1) + i] <= r) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Where a tile sits: its rectangle's two factors and the tile's block
// coordinates along them (all uniform).
struct TileGeom {
    uint32_t lane_off, lane_n, lane_t, head_off, head_n, head_t, lane_mult;
    uint64_t lane_count, head_count, lb, hb;   // lb: the tile's first lane block / lane_mult
};

__device__ __forceinline__ TileGeom locate_tile(uint32_t nrects, cptr_rect rect_p, uint64_t tile) {
    uint32_t lo = 0, hi = nrects - 1;
    while (lo < hi) {
        uint32_t mid = (lo + hi + 1) >> 1;
        if (rect_p[mid].tile_begin <= tile) lo = mid; else hi = mid - 1;
    }
    const uint32_t ri = uni(lo);
    TileGeom t;
    t.lane_off = rect_p[ri].lane_off; t.lane_n = rect_p[ri].lane_n; t.lane_t = rect_p[ri].lane_t;
    t.head_off = rect_p[ri].head_off; t.head_n = rect_p[ri].head_n; t.head_t = rect_p[ri].head_t;
    t.lane_count = rect_p[ri].lane_count;
    t.head_count = rect_p[ri].head_count;
    t.lane_mult = rect_p[ri].lane_mult ? rect_p[ri].lane_mult : 1u;
    const uint64_t head_blocks = rect_p[ri].head_blocks;
    const uint64_t local = tile - rect_p[ri].tile_begin;
    t.lb = local / head_blocks;
    t.hb = local - t.lb * head_blocks;
    return t;
}

// The prefix XORs of k rows in LDS: spx[i * W + w] = XOR of srow[r * W + w]
// over r < i, for i = 0..k, by an XOR scan across each wave (a wave per word).
// The caller synchronises the work-group before and after.
template <int W>
__device__ void build_prefix_xor(const uint32_t *srow, uint32_t *spx, uint32_t k) {
    const uint32_t lane = threadIdx.x & (kWaveSize - 1);
    const uint32_t nw = blockDim.x / kWaveSize;
    for (uint32_t w = threadIdx.x / kWaveSize; w < (uint32_t)W; w += nw) {
        uint32_t carry = 0;
        for (uint32_t c = 0; c < k; c += kWaveSize) {
            uint32_t v = (c + lane < k) ? srow[(c + lane) * W + w] : 0u;
            for (uint32_t d = 1; d < kWaveSize; d <<= 1) {
                const uint32_t o = __shfl_up(v, d, kWaveSize);
                v ^= (lane >= d) ? o : 0u;
            }
            v ^= carry;
            if (c + lane < k) spx[(c + lane + 1) * W + w] = v;
            carry = __shfl(v, kWaveSize - 1, kWaveSize);
        }
        if (lane == 0) spx[w] = 0;
    }
}

// The lane subsets of one lane block of a tile: lane l, slot s holds the lane
// subset of colex rank base + l * SLOTS + s, so that a lane's slots are consecutive
// ranks. P[s] is the XOR of its rows, low[s] the number of its rows below
// k_low, pen[s] = 0x10000 when the rank is past the factor's end. Returns the
// number of valid lane subsets (uniform).
// A lane unranks its first subset (colex digits, binomials from sbin) and
// reaches the next ones by colex successor steps on a 64-bit mask of the lane
// range (Gosper's step). The rows a step changes form two intervals of the
// range, so with the prefix XORs of the rows (spx: spx[i * W + w] is the XOR of
// rows 0..i-1) a step costs four look-ups; without them (spx null) the lane
// XORs the changed rows one by one, a loop whose length depends on the lane.
// A lane range wider than 64 rows unranks every slot instead.
// No other branch depends on the lane. A slot past the end holds a combination
// of the same tile (a lane past the end unranks the block's first rank; a
// successor step past the range keeps the last subset) and is masked by pen.
// (Seeding the fast path's first count with 0 instead of pen, which such a
// repeat would allow, measured 1.4 % slower on the [192,64] search.) (With an "if (valid)"
// per lane around the unranking the optimizer once specialised the tile's
// uniform combination count per divergent path and the wave took the wrong
// path's value.)
// pre / pre_low: the XOR and the count below k_low of rows joined to every
// combination of the tile (a prefix task's prefix; zero otherwise).
// Unranks colex rank r of the lane range (lane_n <= 64) into P (XOR of its rows)
// and returns its rows as a mask of the range.
template <int W>
__device__ __forceinline__ uint64_t unrank_lane(const TileGeom &t, uint64_t r, const uint32_t *srow,
                                                const uint64_t *sbin, uint32_t bt, float lf_top,
                                                uint32_t (&P)[W]) {
    uint64_t x = 0;
    uint32_t hi = t.lane_n - 1;
    float lf = lf_top;
    for (uint32_t i = t.lane_t; i >= 1; --i) {
        uint64_t bc;
        const uint32_t c = colex_digit_est(sbin, bt, i, hi, r, lf, bc);
        r -= bc;
        const uint32_t row = t.lane_off + c;
#pragma unroll
        for (int w = 0; w < W; ++w) P[w] ^= srow[row * W + w];
        x |= 1ull << c;                            // c < lane_n <= 64
        lf -= __builtin_amdgcn_logf((float)i);
        hi = c - 1;
    }
    return x;
}

template <int W, int SLOTS>
__device__ __forceinline__ uint32_t lane_setup(const TileGeom &t, uint64_t base, uint32_t k_low,
                                               const uint32_t *srow, const uint32_t *spx,
                                               const uint64_t *sbin, uint32_t bt,
                                               uint32_t lane, const uint32_t (&pre)[W], uint32_t pre_low,
                                               uint32_t (&P)[SLOTS][W], uint32_t (&low)[SLOTS],
                                               uint32_t (&pen)[SLOTS]) {
    const uint32_t nvalid =
        uni(t.lane_count > base ? (uint32_t)umin64(t.lane_count - base, (uint64_t)kWaveSize * SLOTS) : 0u);
    float lf_top = 0.f;                            // log2(lane_t!)
    for (uint32_t j = 2; j <= t.lane_t; ++j) lf_top += __builtin_amdgcn_logf((float)j);
    const uint64_t q0 = base + (uint64_t)lane * SLOTS;
    // rows of the lane range below k_low, as a mask of the range
    uint64_t low_mask = 0;
    if (k_low > t.lane_off) {
        const uint32_t nl = k_low - t.lane_off;
        low_mask = nl >= 64 ? ~0ull : ((1ull << nl) - 1);
    }
    if (t.lane_n <= 64) {
        uint32_t cur[W];
#pragma unroll
        for (int w = 0; w < W; ++w) cur[w] = pre[w];
        uint64_t x = unrank_lane<W>(t, q0 < t.lane_count ? q0 : base, srow, sbin, bt, lf_top, cur);
        const uint64_t range = t.lane_n >= 64 ? ~0ull : ((1ull << t.lane_n) - 1);
        uint32_t px0[W];                           // prefix XOR below the range
#pragma unroll
        for (int w = 0; w < W; ++w) px0[w] = spx ? spx[t.lane_off * W + w] : 0u;
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
#pragma unroll
            for (int w = 0; w < W; ++w) P[s][w] = cur[w];
            low[s] = pre_low + (uint32_t)__builtin_popcountll(x & low_mask);
            pen[s] = (q0 + (uint64_t)s < t.lane_count) ? 0u : 0x10000u;
            if (s + 1 < SLOTS) {
                // colex successor: the lowest run of ones, bits p..top-1, moves its
                // top bit to top and the rest of it to the bottom
                const uint64_t u = x & (~x + 1);
                const uint64_t v = x + u;
                const uint32_t p = (uint32_t)__builtin_ctzll(x | (1ull << 63));
                const uint64_t nx = v | (((v ^ x) >> 2) >> p);
                // past the last subset of the range the slots are masked: keep the sum
                const bool ok = v != 0 && (nx & ~range) == 0;
                if (spx) {
                    // the rows that change are the intervals [p, top] and [0, top - p - 2]
                    // of the range: four prefix XORs, no lane-dependent loop
                    const uint32_t top = 63u - (uint32_t)__builtin_clzll((v ^ x) | 1ull);
                    const uint32_t i1 = ok ? t.lane_off + top + 1 : t.lane_off;
                    const uint32_t i2 = ok ? t.lane_off + p : t.lane_off;
                    const uint32_t i3 = ok ? t.lane_off + top - p - 1 : t.lane_off;
#pragma unroll
                    for (int w = 0; w < W; ++w)
                        cur[w] ^= spx[i1 * W + w] ^ spx[i2 * W + w] ^ spx[i3 * W + w] ^ px0[w];
                } else {
                    uint64_t diff = ok ? (x ^ nx) : 0ull;
                    while (diff) {
                        const uint32_t b = (uint32_t)__builtin_ctzll(diff);
                        diff &= diff - 1;
                        const uint32_t row = t.lane_off + b;
#pragma unroll
                        for (int w = 0; w < W; ++w) cur[w] ^= srow[row * W + w];
                    }
                }
                x = ok ? nx : x;
            }
        }
    } else {
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
            const uint64_t q = q0 + (uint64_t)s;
            const bool valid = q < t.lane_count;
#pragma unroll
            for (int w = 0; w < W; ++w) P[s][w] = pre[w];
            pen[s] = valid ? 0u : 0x10000u;
            low[s] = pre_low;
            if (base + (uint64_t)s >= t.lane_count) continue;      // uniform: a slot with no valid lane
            uint64_t r = valid ? q : base;
            uint32_t hi = t.lane_n - 1;
            float lf = lf_top;
            for (uint32_t i = t.lane_t; i >= 1; --i) {
                uint64_t bc;
                const uint32_t c = colex_digit_est(sbin, bt, i, hi, r, lf, bc);
                r -= bc;
                const uint32_t row = t.lane_off + c;
#pragma unroll
                for (int w = 0; w < W; ++w) P[s][w] ^= srow[row * W + w];
                low[s] += (row < k_low) ? 1u : 0u;
                lf -= __builtin_amdgcn_logf((float)i);
                hi = c - 1;
            }
        }
    }
    return nvalid;
}

// Visits the head subsets of colex ranks [h0, h0 + count) of the tile's head
// factor, in order. visit(H, hl, step) gets the XOR H of the head rows
// (uniform, in SGPRs), the number hl of head rows below k_low (only when
// COUNT_LOW) and the step index; it returns true to stop the walk early.
// The smallest head element runs fastest (H = S2 ^ row[e]); S2, the XOR of
// the other head rows, changes at a Gosper step of the 64-bit mask. Returns
// whether the walk was stopped.
template <int W, bool COUNT_LOW, typename Visit>
__device__ __forceinline__ bool head_walk(const TileGeom &t, cptr32 rows, cptr64 binom_c, uint32_t k_low,
                                          uint64_t h0, uint64_t count, Visit &&visit) {
    if (t.head_t == 0) {
        uint32_t H[W];
#pragma unroll
        for (int w = 0; w < W; ++w) H[w] = 0;
        return visit(H, 0u, 0u);
    }
    const uint32_t head_off = t.head_off, head_n = t.head_n;
    uint64_t head_low_mask = 0;
    if (COUNT_LOW && k_low > head_off) {
        const uint32_t nl = k_low - head_off;
        head_low_mask = nl >= 64 ? ~0ull : ((1ull << nl) - 1);
    }
    // unrank h0 into the head mask (uniform; binomials through the scalar cache)
    uint64_t x = 0;
    {
        uint64_t r = h0;
        uint32_t hi = head_n - 1;
        for (uint32_t i = t.head_t; i >= 1; --i) {
            uint32_t c = uni(colex_digit_s(binom_c, i, i - 1, hi, r));
            r -= binom_c[c * (kBinomT + 1) + i];
            x |= 1ull << c;
            hi = c - 1;
        }
        x = uni64(x);
    }
    uint32_t S2[W];
#pragma unroll
    for (int w = 0; w < W; ++w) S2[w] = 0;
    {
        uint64_t rest = x & (x - 1);
        while (rest) {
            uint32_t b = (uint32_t)__builtin_ctzll(rest);
            rest &= rest - 1;
            cptr32 rp = rows + (head_off + b) * W;
#pragma unroll
            for (int w = 0; w < W; ++w) S2[w] ^= rp[w];
        }
    }
    uint64_t remaining = count;
    uint32_t step = 0;
    for (;;) {
        const uint32_t e1 = (uint32_t)__builtin_ctzll(x);
        const uint64_t xhi = x & (x - 1);
        const uint32_t e2 = xhi ? (uint32_t)__builtin_ctzll(xhi) : head_n;
        const uint32_t len = (uint32_t)umin64((uint64_t)(e2 - e1), remaining);
        uint32_t hl_base = 0;
        if (COUNT_LOW) hl_base = (uint32_t)__builtin_popcountll(xhi & head_low_mask);
        // one row ahead: the device rows carry a zero row after row k-1,
        // so reading row head_off + e + 1 stays inside the buffer
        cptr32 rp = rows + (head_off + e1) * W;
        uint32_t nxt[W];
#pragma unroll
        for (int w = 0; w < W; ++w) nxt[w] = rp[w];
        for (uint32_t e = e1; e < e1 + len; ++e) {
            uint32_t H[W];
#pragma unroll
            for (int w = 0; w < W; ++w) H[w] = S2[w] ^ nxt[w];
            rp += W;
#pragma unroll
            for (int w = 0; w < W; ++w) nxt[w] = rp[w];
            uint32_t hl = 0;
            if (COUNT_LOW) hl = hl_base + (((head_low_mask >> e) & 1ull) ? 1u : 0u);
            if (visit(H, hl, step)) return true;
            ++step;
        }
        remaining -= len;
        if (remaining == 0) break;
        // colex successor of the last subset visited, xhi | bit(e2 - 1) (Gosper's step)
        const uint64_t xl = xhi | (1ull << (e2 - 1));
        const uint64_t lowbit = xl & (~xl + 1);
        const uint64_t rr = xl + lowbit;
        const uint64_t nx = (((rr ^ xl) >> 2) >> __builtin_ctzll(xl)) | rr;
        uint64_t diff = xhi ^ (nx & (nx - 1));
        while (diff) {
            uint32_t b = (uint32_t)__builtin_ctzll(diff);
            diff &= diff - 1;
            cptr32 rp2 = rows + (head_off + b) * W;
#pragma unroll
            for (int w = 0; w < W; ++w) S2[w] ^= rp2[w];
        }
        x = nx;
    }
    return false;
}

// A wave's running totals of tiles whose counter updates it defers: combinations,
// and the minimum weight with the number of combinations reaching it (all uniform).
struct TileSum {
    uint64_t comb = 0;
    uint32_t min = 0xffffffffu, cnt = 0;
    __device__ void add(uint64_t c, uint32_t m, uint32_t n) {
        comb += c;
        if (m < min) { min = m; cnt = n; }
        else if (m == min) cnt += n;
    }
};

// One tile whose combinations all contain the rows of pre (XOR pre, pre_low of
// them below k_low); the task key records key_tile for it. With DEFER the
// combination count and statistics go to *sum instead of the task's counters
// (a wave running many small tiles flushes them once: every tile's atomic on
// the same word would serialise the waves).
template <int W, int SLOTS, bool PARTIAL, bool STATS, bool DEFER = false>
__device__ __forceinline__ void run_tile_pre(const TaskArgs &a, cptr32 rows, cptr64 binom_c,
                                             const uint32_t *srow, const uint32_t *spx,
                                             const uint64_t *sbin, uint32_t bt,
                                             cptr_rect rect_p, uint64_t tile, uint32_t lane,
                                             const uint32_t (&pre)[W], uint32_t pre_low, uint64_t key_tile,
                                             TileSum *sum = nullptr) {
    const TileGeom t = locate_tile(a.nrects, rect_p, tile);
    const uint64_t h0 = t.hb * a.heads_per_tile;
    const uint64_t count = umin64(h0 + a.heads_per_tile, t.head_count) - h0;
    uint64_t nvalid = 0;                         // lane subsets of the tile (uniform)
    uint32_t m = 0xffffffffu;                    // full: running minimum of all slots
    uint32_t lane_best = 0xffffffffu;            // partial or statistics: the lane's best weight
    uint32_t lane_cnt = 0;
    // the tile's lane blocks, each against the same walk over the heads
    for (uint32_t sb = 0; sb < t.lane_mult; ++sb) {
        const uint64_t base = (t.lb * t.lane_mult + sb) * (uint64_t)(kWaveSize * SLOTS);
        if (base >= t.lane_count) break;         // uniform: the rectangle's last lane block is done
        uint32_t P[SLOTS][W], low[SLOTS], pen[SLOTS];
        nvalid += lane_setup<W, SLOTS>(t, base, a.k_low, srow, spx, sbin, bt, lane, pre, pre_low, P, low, pen);

        uint32_t ms[SLOTS], cs[SLOTS];           // partial or statistics: per slot
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) { ms[s] = 0xffffffffu; cs[s] = 0; }

        head_walk<W, PARTIAL>(t, rows, binom_c, a.k_low, h0, count,
                              [&](const uint32_t (&H)[W], uint32_t hl, uint32_t) {
            if (!PARTIAL && !STATS) {
                uint32_t acc[SLOTS];
#pragma unroll
                for (int s = 0; s < SLOTS; ++s) {
                    uint32_t v = bcnt_acc(H[0] ^ P[s][0], pen[s]);
#pragma unroll
                    for (int w = 1; w < W; ++w) v = bcnt_acc(H[w] ^ P[s][w], v);
                    acc[s] = v;
                }
#pragma unroll
                for (int s = 0; s < SLOTS; s += 2) m = min3u(m, acc[s], acc[s + 1]);
            } else {
#pragma unroll
                for (int s = 0; s < SLOTS; ++s) {
                    uint32_t v = bcnt_acc_s(H[0] ^ P[s][0], hl);
#pragma unroll
                    for (int w = 1; w < W; ++w) v = bcnt_acc(H[w] ^ P[s][w], v);
                    if (STATS) {
                        cs[s] = (v < ms[s]) ? 0u : cs[s];
                        ms[s] = min(ms[s], v);
                        cs[s] += (v == ms[s]) ? 1u : 0u;
                    } else {
                        ms[s] = min(ms[s], v);
                    }
                }
            }
            return false;
        });

        if (PARTIAL || STATS) {
#pragma unroll
            for (int s = 0; s < SLOTS; ++s) {
                if (pen[s]) continue;
                // full-rank statistics: head weight hl was 0, add the whole identity part g
                const uint32_t wgt = PARTIAL ? ms[s] + low[s] : ms[s] + a.g;
                if (wgt < lane_best) { lane_best = wgt; lane_cnt = STATS ? cs[s] : 0; }
                else if (STATS && wgt == lane_best) lane_cnt += cs[s];
            }
        }
    }
    const uint64_t tile_comb = nvalid * count;

    // ---- end of tile: weights, wave reduction, atomics
    if (!PARTIAL && !STATS) {
        lane_best = m + a.g;                     // identity part of a full-rank Gamma_j
        if (m >= 0x10000u) lane_best = 0xffffffffu;
    }
    const uint32_t tmin = uni(wave_min(lane_best));
    uint32_t tcnt = 0;
    if (STATS) tcnt = uni(wave_sum(lane_best == tmin ? lane_cnt : 0u));
    if (DEFER) sum->add(tile_comb, tmin, tcnt);
    if (lane == 0) {
        // most tiles do not lower the key: read it first, update only when needed
        const unsigned long long mine = ((unsigned long long)tmin << kTileBits) | key_tile;
        if (mine < __hip_atomic_load(a.key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMin(a.key, mine);
        if (!DEFER) {
            atomicAdd(a.ncomb, (unsigned long long)tile_comb);
            if (STATS) stats_merge(a.stats, tmin, tcnt);
        }
    }
}

// A tile of the task's own tiling (no prefix).
template <int W, int SLOTS, bool PARTIAL, bool STATS>
__device__ __forceinline__ void run_tile(const TaskArgs &a, cptr32 rows, cptr64 binom_c,
                                         const uint32_t *srow, const uint32_t *spx, const uint64_t *sbin,
                                         uint32_t bt, cptr_rect rect_p, uint64_t tile, uint32_t lane) {
    uint32_t none[W];
#pragma unroll
    for (int w = 0; w < W; ++w) none[w] = 0;
    run_tile_pre<W, SLOTS, PARTIAL, STATS>(a, rows, binom_c, srow, spx, sbin, bt, rect_p, tile, lane, none, 0u,
                                           tile);
}

// Finds one combination of the tile whose weight is target (the tile is
// known to hold one). The lane subsets are taken one slot at a time (slot s of
// lane block b: ranks b * 64 * SLOTS + lane * SLOTS + s; slots s_first,
// s_first + s_step, ... when several waves share the search, each leaving once
// the work-group's stop word is set), each against a walk over the tile's
// heads; after each head step a ballot tells whether any lane hit. Returns
// (uniform) true and, in every lane, the lane-subset rank and head rank of the
// first hit. Few registers: this runs inside the resident serving kernel.
template <int W, int SLOTS>
__device__ __forceinline__ bool find_in_tile(const TaskArgs &a, cptr32 rows, cptr64 binom_c,
                                             const uint32_t *srow, const uint64_t *sbin, uint32_t bt,
                                             cptr_rect rect_p, uint64_t tile, uint32_t lane, uint32_t target,
                                             TileGeom &t, uint64_t &q_hit, uint64_t &h_hit, uint32_t s_first = 0,
                                             uint32_t s_step = 1, const uint32_t *stop = nullptr) {
    t = locate_tile(a.nrects, rect_p, tile);
    const uint64_t h0 = t.hb * a.heads_per_tile;
    const uint64_t count = umin64(h0 + a.heads_per_tile, t.head_count) - h0;
    bool found = false;
    const uint64_t nslots = (uint64_t)t.lane_mult * SLOTS;
    float lf_top = 0.f;                            // log2(lane_t!)
    for (uint32_t j = 2; j <= t.lane_t; ++j) lf_top += __builtin_amdgcn_logf((float)j);
    for (uint64_t s = s_first; s < nslots && !found; s += s_step) {
        // another wave of the work-group has found one (stop: an LDS word)
        if (stop && uni(__hip_atomic_load(stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))) break;
        // slot s % SLOTS of lane block s / SLOTS of the tile
        const uint64_t base = (t.lb * t.lane_mult + s / SLOTS) * (kWaveSize * SLOTS) + s % SLOTS;
        if (base >= t.lane_count) break;                // lane 0 past the end: every lane is
        const uint64_t q = base + (uint64_t)lane * SLOTS;
        const bool valid = q < t.lane_count;      // no lane-dependent branch (see lane_setup)
        uint32_t P[W], low = 0;
        const uint32_t pen = valid ? 0u : 0x10000u;
#pragma unroll
        for (int w = 0; w < W; ++w) P[w] = 0;
        {
            uint64_t r = valid ? q : 0ull;
            uint32_t hi = t.lane_n - 1;
            float lf = lf_top;
            for (uint32_t i = t.lane_t; i >= 1; --i) {
                uint64_t bc;
                const uint32_t c = colex_digit_est(sbin, bt, i, hi, r, lf, bc);   // two look-ups, not a bisection
                r -= bc;
                const uint32_t row = t.lane_off + c;
#pragma unroll
                for (int w = 0; w < W; ++w) P[w] ^= srow[row * W + w];
                low += (row < a.k_low) ? 1u : 0u;
                lf -= __builtin_amdgcn_logf((float)i);
                hi = c - 1;
            }
        }
        head_walk<W, true>(t, rows, binom_c, a.k_low, h0, count,
                           [&](const uint32_t (&H)[W], uint32_t hl, uint32_t step) {
            uint32_t v = low + hl + pen;
#pragma unroll
            for (int w = 0; w < W; ++w) v += __builtin_popcount(H[w] ^ P[w]);
            const uint64_t ballot = __builtin_amdgcn_ballot_w64(v == target);
            if (ballot == 0) return false;
            q_hit = base + (uint64_t)__builtin_ctzll(ballot) * SLOTS;
            h_hit = h0 + step;
            found = true;
            return true;
        });
    }
    return found;
}

}  // namespace bz
