// Host half of the paper's schedules (Sec. 3 of arXiv:1911.08963; the device
// half is bz_sched.hip, the shared mapping bz_sched.h): the tilings of the
// completion spaces of a level's prefix tasks, the prefix of a task (for
// witness recovery), and bz_debug_schedule, which lists the prefixes each
// worker or claim receives without a device.
#include <algorithm>
#include <string>
#include <vector>

#include "../../include/bz_debug.h"
#include "bz_host.h"
#include "bz_internal.h"
#include "bz_sched.h"

namespace bz {

// Completion tiles are made large (one task is one wave's work, and a tile is
// the unit of the stop check): the planner is asked for one tile per plan and
// caps heads per tile at its maximum.
constexpr uint64_t kSchedTargetTiles = 1;

bool build_sched_plan(uint32_t k, uint32_t g, bool dynamic, uint32_t prefix, uint32_t slots, SchedPlan &out,
                      std::string &err) {
    out = SchedPlan{};
    if (g == 0 || g > k) { err = "level out of range"; return false; }
    out.pre = prefix_elems(dynamic, prefix, g);
    const uint32_t t = g - out.pre;                          // completion size, >= 1
    out.entries.assign(k + 1, PlanEntry{});
    const uint32_t lo_first = out.pre, lo_last = out.pre ? k - t : 0;
    for (uint32_t lo = lo_first; lo <= lo_last; ++lo) {
        LevelPlan p;
        if (!plan_range(lo, k - lo, t, slots, 0, kSchedTargetTiles, p, err)) return false;
        PlanEntry &e = out.entries[lo];
        e.total_tiles = p.total_tiles;
        e.rect_off = (uint32_t)out.rects.size();
        e.nrects = (uint32_t)p.rects.size();
        e.heads_per_tile = p.heads_per_tile;
        out.rects.insert(out.rects.end(), p.rects.begin(), p.rects.end());
        out.stride = std::max<uint64_t>(out.stride, p.total_tiles);
    }
    out.ntasks = out.pre ? binom_sat(k - t, out.pre) : 1;
    if (out.ntasks == kBinomSat) { err = "too many prefix tasks"; return false; }
    if (out.ntasks > kTileMask / std::max<uint64_t>(1, out.stride)) {
        err = "prefix tasks x completion tiles exceed the task key's tile field";
        return false;
    }
    return true;
}

void sched_prefix(const SchedPlan &sp, uint32_t k, uint32_t g, uint32_t order, uint64_t task,
                  std::vector<uint32_t> &rows, uint32_t &lo) {
    rows.assign(sp.pre, 0);
    const uint32_t K = k - (g - sp.pre);
    prefix_unrank(order, task, sp.pre, K, [](uint32_t a, uint32_t b) { return binom_sat(a, b); },
                  [&](uint32_t i, uint32_t c) { rows[i] = c; });
    lo = sp.pre ? rows[sp.pre - 1] + 1 : 0;
}

}  // namespace bz

extern "C" {

bz_status bz_debug_schedule(uint32_t schedule, uint32_t k, uint32_t g, uint32_t p, uint32_t workers,
                            uint32_t turns, int32_t *out, uint64_t cap, uint32_t *pre_elems, uint64_t *ntasks) {
    uint32_t dist = 0, order = 0;
    bool dynamic = false;
    if (!bz::sched_parts(schedule, dist, order, dynamic)) return bz::fail(BZ_EINVAL, "schedule must be 1..8");
    if (k == 0 || k > (uint32_t)bz::kMaxN || g == 0 || g > k || g > (uint32_t)bz::kBinomT)
        return bz::fail(BZ_EINVAL, "bad k or g");
    if (p == 0) return bz::fail(BZ_EINVAL, "prefix size must be >= 1");
    if (workers == 0) return bz::fail(BZ_EINVAL, "workers must be >= 1");
    const uint32_t pre = bz::prefix_elems(dynamic, p, g);
    const uint32_t K = k - (g - pre);
    const uint64_t n = pre ? bz::binom_sat(K, pre) : 1;
    if (n == bz::kBinomSat) return bz::fail(BZ_ELIMIT, "too many prefix tasks");
    if (pre_elems) *pre_elems = pre;
    if (ntasks) *ntasks = n;
    if (!out) return BZ_OK;
    const uint32_t per = dynamic ? 2u : turns;            // entries per worker (claims: up to 2 prefixes)
    const uint64_t need = (uint64_t)workers * per * std::max<uint32_t>(pre, 1);
    if (need > cap) return bz::fail(BZ_ELIMIT, "output buffer too small");
    std::fill(out, out + need, -1);
    auto put = [&](uint64_t slot, uint64_t task) {
        if (!pre) { out[slot] = (int32_t)task; return; }   // the single task: index 0
        bz::prefix_unrank(order, task, pre, K, [](uint32_t a, uint32_t b) { return bz::binom_sat(a, b); },
                          [&](uint32_t i, uint32_t c) { out[slot * pre + i] = (int32_t)c; });
    };
    for (uint32_t w = 0; w < workers; ++w) {
        if (dynamic) {
            uint64_t t0 = 0, t1 = 0;
            const uint32_t m = bz::claim_tasks(dist, w, n, t0, t1);
            if (m >= 1) put((uint64_t)w * 2, t0);
            if (m == 2) put((uint64_t)w * 2 + 1, t1);
        } else {
            for (uint32_t s = 0; s < turns; ++s) {
                const uint64_t task = bz::static_task(dist, w, workers, s, n);
                if (task != ~0ull) put((uint64_t)w * turns + s, task);
            }
        }
    }
    return BZ_OK;
}

}  // extern "C"
