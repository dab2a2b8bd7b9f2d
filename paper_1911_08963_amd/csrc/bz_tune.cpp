// Autotuning of the enumeration's two free parameters (include/bz.h,
// bz_autotune*): the lane sums kept per lane ("slots", the words a thread
// holds: SLOTS x W registers, the paper's unrolling of several left
// combinations per fetched right one, Sec. 2.2.1) and the chunk size of a
// task (Sec. 3.1), expressed as tiles per resident wave so that every level
// gets tiles of a size that suits it. Both change only speed, never a result:
// every tiling covers each combination once.
//
// bz_autotune times the plain kernel on a synthetic full-rank task of the
// given shape for every candidate and installs the fastest as the choice for
// that row width W; bz_min_distance uses it when the caller leaves both
// parameters at 0. bz_autotune_batch times one batch at several tile counts
// per task and installs the fastest for later batches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "bz_host.h"
#include "bz_internal.h"
#include "bz_kernels.h"

namespace {

using bz::fail;

std::mutex g_tune_mu;
std::map<uint32_t, bz_tune_entry> g_tuned;    // W -> chosen (slots, tiles per wave)
uint32_t g_batch_tiles = 0;                   // tiles per task for batches (0 = not tuned)

constexpr double kTuneCombinations = bz::kLargeLevelComb;    // size of the timed task (several milliseconds)
constexpr uint32_t kTilesPerWave[] = {1, 2, 4, 8, 16, 64};    // kFixedTilesPerWave: the fixed rule

uint64_t splitmix(uint64_t &s) {
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

}  // namespace

namespace bz {

bool tuned_choice(uint32_t W, uint32_t &slots, uint32_t &tiles_per_wave) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(W);
    if (it == g_tuned.end()) return false;
    slots = it->second.slots_per_lane;
    tiles_per_wave = it->second.tiles_per_wave;
    return true;
}

uint32_t tuned_batch_tiles() {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    return g_batch_tiles;
}

}  // namespace bz

extern "C" {

bz_status bz_autotune(uint32_t W, uint32_t k, bz_tune_entry *out) {
    if (!out) return fail(BZ_EINVAL, "out is null");
    if (W < 1 || W > (uint32_t)bz::kMaxW) return fail(BZ_EINVAL, "W must be 1..8");
    if (k < 2 || k > (uint32_t)bz::kMaxN) return fail(BZ_EINVAL, "k must be 2..256");
    int dev = 0;
    BZ_HIP(hipGetDevice(&dev));
    bz::DeviceConst dc;
    bz_status s0 = bz::device_const(dev, dc);
    if (s0 != BZ_OK) return s0;

    // the timed task: level g of a full-rank matrix, the first with at least
    // kTuneCombinations sums (for small k, the level with the most)
    uint32_t g = 1;
    uint64_t gc = 0;
    for (uint32_t t = 1; t <= std::min<uint32_t>(k, bz::kBinomT); ++t) {
        const uint64_t c = bz::binom_sat(k, t);
        if (c >= (1ull << 40)) break;
        if ((double)c >= kTuneCombinations) { g = t; break; }
        if (c > gc) { g = t; gc = c; }                     // small k: the largest level
    }
    const uint64_t comb = bz::binom_sat(k, g);

    // synthetic rows (the enumeration's cost does not depend on their bits),
    // with the zero row the head walk's prefetch reads past the end
    std::vector<uint32_t> rows((size_t)(k + 1) * W, 0u);
    uint64_t seed = 0x5eedull * W + k;
    for (size_t i = 0; i < (size_t)k * W; ++i) rows[i] = (uint32_t)splitmix(seed);

    std::vector<std::pair<uint32_t, uint32_t>> cands;      // (slots, tiles per resident wave)
    for (uint32_t slots : {2u, 4u, 8u, 16u}) {
        if (slots == 16 && W > 4) continue;
        for (uint32_t t : kTilesPerWave) cands.push_back({slots, t});
    }
    const uint64_t resident_waves = (uint64_t)dc.cus * 32;
    std::vector<bz::LevelPlan> plans(cands.size());
    size_t max_rects = 0;
    for (size_t i = 0; i < cands.size(); ++i) {
        std::string err;
        if (!bz::plan_level(k, g, cands[i].first, 0, cands[i].second * resident_waves, plans[i], err))
            return fail(BZ_ELIMIT, err);
        max_rects = std::max(max_rects, plans[i].rects.size());
    }

    char *mem = nullptr;
    const size_t off_rows = 0, off_words = 4096 * ((rows.size() * 4 + 4095) / 4096);
    const size_t off_rects = off_words + 256;
    BZ_HIP(hipMalloc((void **)&mem, off_rects + max_rects * sizeof(bz::Rect)));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    struct Guard {
        char *p; hipEvent_t &a, &b;
        ~Guard() { (void)hipFree(p); if (a) (void)hipEventDestroy(a); if (b) (void)hipEventDestroy(b); }
    } guard{mem, e0, e1};
    BZ_HIP(hipEventCreate(&e0));
    BZ_HIP(hipEventCreate(&e1));
    BZ_HIP(hipMemcpy(mem + off_rows, rows.data(), rows.size() * 4, hipMemcpyHostToDevice));
    auto *words = (unsigned long long *)(mem + off_words);

    double best = 0.0, dflt = 0.0;
    size_t best_i = 0;
    for (size_t i = 0; i < cands.size(); ++i) {
        const bz::LevelPlan &p = plans[i];
        BZ_HIP(hipMemcpy(mem + off_rects, p.rects.data(), p.rects.size() * sizeof(bz::Rect), hipMemcpyHostToDevice));
        bz::TaskArgs a{};
        a.rows = (const uint32_t *)(mem + off_rows);
        a.binom = dc.binom;
        a.rects = (const bz::Rect *)(mem + off_rects);
        a.key = words; a.stats = words + 1; a.ncomb = words + 2; a.tile_ctr = words + 3;
        a.nrects = (uint32_t)p.rects.size();
        a.k = k; a.k_low = k; a.g = g;
        a.heads_per_tile = p.heads_per_tile;
        a.total_tiles = p.total_tiles;
        a.u_prev = 0xffffffffu;
        a.exit_at = 0;                                       // every tile runs
        const uint64_t blocks = (p.total_tiles + 3) / 4;
        const uint32_t grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(blocks, (uint64_t)dc.cus * 8));
        float tmin = 0.f;
        for (int rep = 0; rep < 4; ++rep) {                  // one warm-up, the fastest of three
            BZ_HIP(bz::launch_task_init(a.key, a.stats, a.ncomb, a.tile_ctr, nullptr));
            BZ_HIP(hipEventRecord(e0, nullptr));
            BZ_HIP(bz::launch_enum(a, W, cands[i].first, false, false, grid, nullptr));
            BZ_HIP(hipEventRecord(e1, nullptr));
            BZ_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            BZ_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (rep == 1 || (rep > 1 && ms < tmin)) tmin = ms;
        }
        unsigned long long back[3];
        BZ_HIP(hipMemcpy(back, words, sizeof(back), hipMemcpyDeviceToHost));
        if (back[2] != comb) return fail(BZ_EDEVICE, "autotune: a timed launch did not enumerate its task");
        const double rate = (double)comb / (tmin * 1e-3);
        if (cands[i].first == bz::slots_for_w(W) && cands[i].second == bz::kFixedTilesPerWave) dflt = rate;
        if (rate > best) { best = rate; best_i = i; }
    }
    bz_tune_entry e{};
    e.W = W; e.k = k; e.g = g;
    e.slots_per_lane = cands[best_i].first;
    e.tiles_per_wave = cands[best_i].second;
    e.heads_per_tile = plans[best_i].heads_per_tile;
    e.combinations = comb;
    e.comb_per_s = best;
    e.default_comb_per_s = dflt;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned[W] = e;
    }
    *out = e;
    return BZ_OK;
}

bz_status bz_autotune_set(const bz_tune_entry *e) {
    if (!e) return fail(BZ_EINVAL, "null entry");
    if (e->W < 1 || e->W > (uint32_t)bz::kMaxW) return fail(BZ_EINVAL, "W must be 1..8");
    const uint32_t sl = e->slots_per_lane;
    if (sl != 2 && sl != 4 && sl != 8 && sl != 16) return fail(BZ_EINVAL, "slots per lane must be 2, 4, 8 or 16");
    if (sl == 16 && e->W > 4) return fail(BZ_EINVAL, "16 slots per lane need W <= 4");
    if (e->tiles_per_wave < 1 || e->tiles_per_wave > 4096) return fail(BZ_EINVAL, "tiles per wave must be 1..4096");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[e->W] = *e;
    return BZ_OK;
}

bz_status bz_autotune_get(uint32_t W, bz_tune_entry *out) {
    if (!out) return fail(BZ_EINVAL, "out is null");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(W);
    if (it == g_tuned.end()) return fail(BZ_EINVAL, "no tuned entry for this W");
    *out = it->second;
    return BZ_OK;
}

void bz_autotune_clear(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned.clear();
    g_batch_tiles = 0;
}

bz_status bz_autotune_batch(bz_code *const *codes, uint32_t count, const bz_opts *o, uint32_t *tiles_per_task,
                            double *seconds) {
    if (!codes || !count || !tiles_per_task || !seconds) return fail(BZ_EINVAL, "null argument");
    bz_opts opt{};
    if (o) opt = *o;
    opt.flags |= BZ_F_NO_WITNESS;
    std::vector<bz_result> res(count);
    std::vector<bz_status> per(count);
    double best = 0.0;
    uint32_t best_t = 0;
    for (uint32_t t : {16u, 64u, 256u, 1024u}) {
        opt.tiles_per_task = t;
        double tmin = 0.0;
        for (int rep = 0; rep < 2; ++rep) {
            for (auto &r : res) std::memset(&r, 0, sizeof(r));
            const double t0 = bz::now_s();
            bz_status st = bz_min_distance_batch(codes, count, &opt, res.data(), per.data());
            const double dt = bz::now_s() - t0;
            if (st != BZ_OK) return st;
            if (rep == 0 || dt < tmin) tmin = dt;
        }
        if (best_t == 0 || tmin < best) { best = tmin; best_t = t; }
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_batch_tiles = best_t;
    }
    *tiles_per_task = best_t;
    *seconds = best;
    return BZ_OK;
}

}  // extern "C"
