// Tiling of one level: the g-subsets of the k rows of a Gamma matrix, cut
// into products of two colex subset spaces.
//
// The g-subsets of a range R = A u B (A below B) split by how many elements
// fall in A. For each i the part is the product of the i-subsets of A and the
// (g-i)-subsets of B (Vandermonde's identity). The parts with i = 0 or i = g
// are again "all t-subsets of one range", and recurse. A range whose subset
// count is small becomes a lanes-only rectangle.
//
// In a product, one factor goes to the lanes of a wave (each lane holds the
// XOR of a few fixed subsets in VGPRs). The other factor, the "head", is
// stepped in colex order identically by the whole wave, its XOR held in
// SGPRs. The head must be a range of at most 64 rows (a 64-bit mask), and
// gets the smaller of the two counts. A tile is a block of 64 * slots lane
// subsets by heads_per_tile head steps, so tiles of one level cost the same
// except at the edges (the paper's point about unequal prefix costs, Sec. 3.1,
// is why the work is cut by rank ranges and not by prefixes).
#include <algorithm>

#include "bz_internal.h"
#include "bz_kernels.h"

namespace bz {
namespace {

struct Builder {
    uint64_t threshold;
    std::vector<Rect> *out;
    bool overflow = false;

    void terminal(uint32_t lo, uint32_t n, uint32_t t) {
        Rect r{};
        r.lane_off = lo; r.lane_n = n; r.lane_t = t;
        r.head_off = lo; r.head_n = 0; r.head_t = 0;
        r.lane_count = binom_sat(n, t);
        r.head_count = 1;
        out->push_back(r);
    }

    void product(uint32_t lane_off, uint32_t lane_n, uint32_t lane_t,
                 uint32_t head_off, uint32_t head_n, uint32_t head_t) {
        Rect r{};
        r.lane_off = lane_off; r.lane_n = lane_n; r.lane_t = lane_t;
        r.head_off = head_off; r.head_n = head_n; r.head_t = head_t;
        r.lane_count = binom_sat(lane_n, lane_t);
        r.head_count = binom_sat(head_n, head_t);
        if (r.lane_count == kBinomSat || r.head_count == kBinomSat) overflow = true;
        out->push_back(r);
    }

    // every t-subset of [lo, lo + n), t >= 1
    void all(uint32_t lo, uint32_t n, uint32_t t) {
        if (t > n) return;
        uint64_t total = binom_sat(n, t);
        if (total == kBinomSat) { overflow = true; return; }
        if (total <= threshold || n <= 2 || t == n) { terminal(lo, n, t); return; }
        uint32_t nA = (n > 2 * (uint32_t)kMaxHeadSide) ? (uint32_t)kMaxHeadSide : n / 2;
        uint32_t nB = n - nA, mid = lo + nA;
        for (uint32_t i = 0; i <= t; ++i) {
            if (i > nA || t - i > nB) continue;
            if (i == 0) { all(mid, nB, t); continue; }
            if (i == t) { all(lo, nA, t); continue; }
            uint64_t cA = binom_sat(nA, i), cB = binom_sat(nB, t - i);
            bool headA_ok = nA <= (uint32_t)kMaxHeadSide, headB_ok = nB <= (uint32_t)kMaxHeadSide;
            bool head_is_A = headA_ok && (!headB_ok || cA < cB);
            if (head_is_A) product(mid, nB, t - i, lo, nA, i);
            else product(lo, nA, i, mid, nB, t - i);
        }
    }
};

}  // namespace

// The lane setup of one lane block (first subset unranked, successor steps
// for the other slots) in units of one head step of the tile loop: about 850
// instructions against 80 per head step for k = 64, W = 2, 16 slots.
constexpr uint64_t kSetupHeads = 12;

bool plan_level(uint32_t k, uint32_t g, uint32_t slots, uint32_t heads_per_tile,
                uint64_t target_tiles, LevelPlan &out, std::string &err, bool widen) {
    return plan_range(0, k, g, slots, heads_per_tile, target_tiles, out, err, widen);
}

bool plan_range(uint32_t lo, uint32_t n, uint32_t g, uint32_t slots, uint32_t heads_per_tile,
                uint64_t target_tiles, LevelPlan &out, std::string &err, bool widen) {
    out = LevelPlan{};
    out.k = lo + n; out.g = g; out.slots = slots;
    if (g == 0 || g > n) { err = "level out of range"; return false; }
    uint64_t total = binom_sat(n, g);
    if (total == kBinomSat) { err = "C(k, g) >= 2^63"; return false; }
    if (g > (uint32_t)kBinomT) { err = "level above the device binomial table"; return false; }
    Builder b;
    b.threshold = 4ull * kWaveSize * slots;
    b.out = &out.rects;
    b.all(lo, n, g);
    if (b.overflow) { err = "a factor count overflows 2^63"; return false; }
    uint64_t lane_items = (uint64_t)kWaveSize * slots;
    uint32_t ht = heads_per_tile;
    if (ht == 0) {
        // aim at target_tiles tiles of equal cost, within [32, 4096] heads
        uint64_t want = total / std::max<uint64_t>(1, target_tiles) / lane_items;
        ht = 32;
        while (ht < 4096 && ht < want) ht <<= 1;
    }
    for (;;) {
        uint64_t tiles = 0, comb = 0;
        for (Rect &r : out.rects) {
            uint64_t lb = (r.lane_count + lane_items - 1) / lane_items;
            uint64_t hb = (r.head_count + ht - 1) / ht;
            if (lb >= kMaxTiles) { err = "level too large for the tile index"; return false; }
            // a rectangle of few heads (a factor of one or two rows) would
            // otherwise give tiles a fraction of the others' cost: on a level
            // of about one tile per wave the waves holding full tiles then
            // decide the launch's length. A lane block costs its setup (about
            // kSetupHeads head steps) plus its heads.
            uint64_t m = 1;
            if (widen && r.head_count < ht)
                m = std::max<uint64_t>(1, std::min<uint64_t>(lb, (ht + kSetupHeads) / (r.head_count + kSetupHeads)));
            r.lane_mult = (uint32_t)m;
            lb = (lb + m - 1) / m;
            r.lane_blocks = lb;
            r.head_blocks = hb;
            r.tile_begin = tiles;
            tiles += lb * hb;
            comb += r.lane_count * r.head_count;
        }
        if (comb != total) { err = "internal: tiling does not cover C(k, g)"; return false; }
        if (tiles < kMaxTiles) {
            out.total_tiles = tiles;
            out.combinations = comb;
            out.heads_per_tile = ht;
            return true;
        }
        if (ht >= (1u << 24)) { err = "level too large for the tile index"; return false; }
        ht <<= 1;
    }
}

uint32_t build_level_plans(uint32_t k, uint32_t slots, uint32_t heads_per_tile, uint64_t target_tiles,
                           uint64_t max_comb, uint32_t rect_base, std::vector<PlanEntry> &plans,
                           std::vector<Rect> &rects, uint32_t max_heads) {
    uint32_t gmax = 0;
    for (uint32_t g = 1; g <= std::min<uint32_t>(k, kBinomT); ++g) {
        if (binom_sat(k, g) >= max_comb) break;
        uint32_t ht = heads_per_tile;
        if (ht == 0 && max_heads) {
            // the planner's rule (about target_tiles tiles) with a smaller cap
            const uint64_t want = binom_sat(k, g) / std::max<uint64_t>(1, target_tiles) / ((uint64_t)kWaveSize * slots);
            ht = 32;
            while (ht < max_heads && ht < want) ht <<= 1;
        }
        LevelPlan p;
        std::string err;
        if (!plan_level(k, g, slots, ht, target_tiles, p, err)) break;
        PlanEntry e{};
        e.total_tiles = p.total_tiles;
        e.rect_off = rect_base + (uint32_t)rects.size();
        e.nrects = (uint32_t)p.rects.size();
        e.heads_per_tile = p.heads_per_tile;
        rects.insert(rects.end(), p.rects.begin(), p.rects.end());
        plans.push_back(e);
        gmax = g;
    }
    return gmax;
}

}  // namespace bz
