// bz_count_codewords (include/bz.h): the number of codewords of a given
// weight w, and the codewords themselves.
//
// The tasks (Gamma_j, g) run in the order of Alg. 1, every sum of weight w is
// collected on the device (bz_count.hip), and the loop stops once the bound
// certified by the completed tasks exceeds w: from then on every codeword not
// enumerated weighs more than w. A codeword is met once in every Gamma_j in
// which it is light enough, so the host rebuilds each hit's codeword (the XOR
// of the full rows its combination picks) and keeps the distinct ones.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstring>
#include <unordered_set>
#include <vector>

#include "bz_host.h"
#include "bz_internal.h"
#include "bz_kernels.h"

namespace {

using bz::fail;

constexpr uint64_t kMaxHits = 1ull << 21;          // weight-w sums one task may hold (48 MiB)

using Word4 = std::array<uint64_t, bz::kHostWords>;

struct Word4Hash {
    size_t operator()(const Word4 &x) const {
        uint64_t h = 0x9e3779b97f4a7c15ull;
        for (uint64_t v : x) h = (h ^ v) * 0xff51afd7ed558ccdull + (h >> 29);
        return (size_t)h;
    }
};

// Colex unranking: the t-subset of [off, off + nside) of rank r; XORs the
// chosen rows of `full` into x.
void xor_subset(uint64_t r, uint32_t t, uint32_t off, uint32_t nside, const bz::HostRow *full, Word4 &x) {
    uint32_t hi = nside - 1;
    for (uint32_t i = t; i >= 1; --i) {
        uint32_t lo = i - 1, c = hi;
        while (lo < c) {
            uint32_t mid = (lo + c + 1) >> 1;
            if (bz::binom_sat(mid, i) <= r) lo = mid; else c = mid - 1;
        }
        r -= bz::binom_sat(lo, i);
        for (int w = 0; w < bz::kHostWords; ++w) x[w] ^= full[off + lo][w];
        hi = lo - 1;
    }
}

bool row_less(const Word4 &a, const Word4 &b) {
    for (int w = bz::kHostWords - 1; w >= 0; --w)
        if (a[w] != b[w]) return a[w] < b[w];
    return false;
}

// The lower bound certified once Gamma_0..Gamma_j are done at level g and the
// later matrices at level g - 1 (j = m_f is the partial matrix: Alg. 1's L).
uint32_t certified(uint32_t j, uint32_t g, uint32_t m_f, uint32_t k_m, uint32_t k) {
    if (j >= m_f) {
        int64_t e = k_m ? (int64_t)g + 1 - k + k_m : 0;
        return m_f * (g + 1) + (uint32_t)std::max<int64_t>(0, e);
    }
    int64_t e = k_m ? (int64_t)g - k + k_m : 0;
    return (j + 1) * (g + 1) + (m_f - j - 1) * g + (uint32_t)std::max<int64_t>(0, e);
}

}  // namespace

extern "C" {

bz_status bz_count_codewords(bz_code *c, const bz_opts *o, bz_weight_count *res) {
    if (!c || !res) return fail(BZ_EINVAL, "null argument");
    if (!c->dev) return fail(BZ_EINVAL, "code prepared host-only (BZ_PREPARE_HOST_ONLY)");
    bz_opts opt{};
    if (o) opt = *o;
    const double t0 = bz::now_s();
    const uint32_t n = c->n, k = c->k, m_f = c->num_full, k_m = c->partial_rank;
    res->count = 0; res->hits = 0; res->combinations = 0; res->last_level = 0; res->codewords_len = 0;
    uint32_t w = res->weight;
    if (w == 0) {
        // the minimum distance first
        bz_opts fo{};
        fo.hip_stream = opt.hip_stream;
        fo.flags = BZ_F_NO_WITNESS;
        bz_result r{};
        bz_status st = bz_min_distance(c, &fo, &r);
        if (st != BZ_OK) return st;
        w = r.d;
        res->weight = w;
    }
    const uint32_t nw = (n + 63) / 64;
    if (w > n) { res->search_s = bz::now_s() - t0; return BZ_OK; }
    if (k == n) {
        // the whole space: every weight-w vector, the first ones in colex order
        res->count = bz::binom_sat(n, w);
        if (res->count >= bz::kBinomSat) return fail(BZ_ELIMIT, "C(n, w) >= 2^63");
        if (res->codewords && res->codewords_cap) {
            std::vector<bz::HostRow> unit(n);
            for (uint32_t i = 0; i < n; ++i) { unit[i].fill(0); unit[i][i >> 6] = 1ull << (i & 63); }
            const uint64_t m = std::min<uint64_t>(res->count, res->codewords_cap);
            for (uint64_t r = 0; r < m; ++r) {
                Word4 x{};
                xor_subset(r, w, 0, n, unit.data(), x);
                for (uint32_t q = 0; q < nw; ++q) res->codewords[r * nw + q] = x[q];
            }
            res->codewords_len = m;
        }
        res->search_s = bz::now_s() - t0;
        return BZ_OK;
    }

    if (hipSetDevice(c->device) != hipSuccess) return fail(BZ_EDEVICE, "hipSetDevice");
    bz::DeviceConst dc;
    bz_status s0 = bz::device_const(c->device, dc);
    if (s0 != BZ_OK) return s0;
    hipStream_t st = (hipStream_t)opt.hip_stream;
    const size_t max_rects = 16384;
    const size_t off_words = 0, off_rects = 256, off_hits = off_rects + max_rects * sizeof(bz::Rect);
    char *mem = nullptr;
    BZ_HIP(hipMalloc((void **)&mem, off_hits + kMaxHits * sizeof(bz::CollectHit)));
    struct Guard {
        char *p;
        ~Guard() { (void)hipFree(p); }
    } guard{mem};
    auto *words = (unsigned long long *)(mem + off_words);
    auto *d_rects = (bz::Rect *)(mem + off_rects);
    auto *d_hits = (bz::CollectHit *)(mem + off_hits);

    std::unordered_set<Word4, Word4Hash> seen;
    std::vector<bz::CollectHit> hits;
    const uint64_t resident_waves = (uint64_t)dc.cus * 32;
    bool done = false;
    for (uint32_t g = 1; g <= k && !done; ++g) {
        if (opt.max_level && g > opt.max_level)
            return fail(BZ_ELIMIT, "max_level reached before the count was complete");
        res->last_level = g;
        for (uint32_t j = 0; j < c->nsets && !done; ++j) {
            const uint32_t W = c->W(j);
            bz::LevelPlan plan;
            std::string err;
            if (!bz::plan_level(k, g, bz::slots_for_w(W), 0, bz::kFixedTilesPerWave * resident_waves, plan, err))
                return fail(BZ_ELIMIT, err);
            if (plan.rects.size() > max_rects) return fail(BZ_ELIMIT, "too many rectangles in one level");
            BZ_HIP(hipMemcpyAsync(d_rects, plan.rects.data(), plan.rects.size() * sizeof(bz::Rect),
                                  hipMemcpyHostToDevice, st));
            BZ_HIP(hipMemsetAsync(words, 0, 2 * sizeof(unsigned long long), st));
            bz::CollectArgs a{};
            a.rows = (const uint32_t *)c->dev + c->packed_off[j];
            a.binom = dc.binom;
            a.rects = d_rects;
            a.ncomb = words; a.nhits = words + 1;
            a.hits = d_hits; a.cap = kMaxHits;
            a.total_tiles = plan.total_tiles;
            a.nrects = (uint32_t)plan.rects.size();
            a.k = k; a.k_low = c->k_low(j); a.g = g;
            a.heads_per_tile = plan.heads_per_tile;
            a.target = w;
            const uint64_t blocks = (plan.total_tiles + 3) / 4;
            const uint32_t grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(blocks, (uint64_t)dc.cus * 8));
            BZ_HIP(bz::launch_collect(a, W, grid, st));
            unsigned long long back[2];
            BZ_HIP(hipMemcpyAsync(back, words, sizeof(back), hipMemcpyDeviceToHost, st));
            BZ_HIP(hipStreamSynchronize(st));
            if (back[0] != plan.combinations) return fail(BZ_EDEVICE, "internal: the counting pass missed combinations");
            if (back[1] > kMaxHits) return fail(BZ_ELIMIT, "more weight-w sums in one task than the pass can hold");
            res->combinations += back[0];
            res->hits += back[1];
            hits.resize(back[1]);
            if (back[1])
                BZ_HIP(hipMemcpy(hits.data(), d_hits, back[1] * sizeof(bz::CollectHit), hipMemcpyDeviceToHost));
            const bz::HostRow *full = c->full_rows.data() + (size_t)j * k;
            for (const bz::CollectHit &h : hits) {
                size_t lo = 0, hi = plan.rects.size() - 1;
                while (lo < hi) {
                    size_t mid = (lo + hi + 1) / 2;
                    if (plan.rects[mid].tile_begin <= h.tile) lo = mid; else hi = mid - 1;
                }
                const bz::Rect &R = plan.rects[lo];
                Word4 x{};
                xor_subset(h.q, R.lane_t, R.lane_off, R.lane_n, full, x);
                if (R.head_t) xor_subset(h.h, R.head_t, R.head_off, R.head_n, full, x);
                uint32_t wt = 0;
                for (uint64_t v : x) wt += (uint32_t)__builtin_popcountll(v);
                if (wt != w) return fail(BZ_EDEVICE, "internal: a collected sum has the wrong weight");
                seen.insert(x);
            }
            // every codeword not met yet weighs at least the certified bound
            if (certified(j, g, m_f, k_m, k) > w) done = true;
        }
    }
    res->count = seen.size();
    if (res->codewords && res->codewords_cap) {
        std::vector<Word4> all(seen.begin(), seen.end());
        std::sort(all.begin(), all.end(), row_less);
        const uint64_t m = std::min<uint64_t>(all.size(), res->codewords_cap);
        for (uint64_t i = 0; i < m; ++i)
            for (uint32_t q = 0; q < nw; ++q) res->codewords[i * nw + q] = all[i][q];
        res->codewords_len = m;
    }
    res->search_s = bz::now_s() - t0;
    return BZ_OK;
}

}  // extern "C"
