// Internal declarations shared by the host side of libbz and its HIP kernels.
#pragma once

#include <array>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/bz.h"

namespace bz {

constexpr int kMaxN = BZ_MAX_N;
constexpr int kHostWords = kMaxN / 64;   // 64-bit words of a host row
constexpr int kMaxW = kMaxN / 32;        // 32-bit words of a device row
constexpr int kBinomT = 64;              // columns 0..kBinomT of the device binomial table
constexpr int kBinomRows = kMaxN + 1;    // rows 0..kMaxN
constexpr uint64_t kBinomSat = ~0ull;    // stored for values >= 2^63
constexpr int kMaxHeadSide = 64;         // the head side is a 64-bit mask
constexpr int kWaveSize = 64;
constexpr int kBlock = 256;              // threads per work-group (4 waves)

// Bytes of the device array that bz_min_distance_noalloc works in (one per
// device): the binomial table, then a single search's workspace.
constexpr size_t kNoAllocScratchBytes = BZ_NOALLOC_SCRATCH_BYTES;

using HostRow = std::array<uint64_t, kHostWords>;

// Combinations each lane keeps per head step, by 32-bit words per row: one
// head step carries 70-140 VALU operations, so the scalar head stepping (and
// its colex carries) stays well below the vector work. Measured on the MI355X
// against 8/4 (W <= 4 / above): the batched workload 1.5 s instead of 2.3 s.
constexpr uint32_t slots_for_w(uint32_t W) { return W <= 4 ? 16u : 8u; }

// Tiles per resident wave the planner aims at for one task of a single-code
// search: enough for the static round-robin to balance, few enough that a
// tile's setup (unranking its lane subsets) stays small against its work.
constexpr uint32_t kFixedTilesPerWave = 4;
// Levels of fewer sums than this (the size the autotuner times) get one tile
// per resident wave: there a tile's setup weighs more than the balance that
// smaller tiles buy.
constexpr double kLargeLevelComb = 2e10;
// Lane sums per lane on the smallest levels of a single-code search: there a
// wave runs one short tile whose time is mostly the setup that unranks its
// lane subsets (a chain of binomial look-ups per slot), so fewer slots finish
// sooner. Measured per level on k = 64, W = 2: level 2 (2016 sums) 6.5 us with
// 2 slots against 19 us with 16; level 5 (7.6e6 sums) 22 us with 8 against 37.
constexpr double kTinyLevelComb = 2097152.0;      // 2^21: 2 slots
constexpr double kSmallLevelComb = 16777216.0;    // 2^24: at most 8 slots

// One product of two colex subset spaces inside the g-subsets of [0, k):
// every union of a lane_t-subset of [lane_off, lane_off + lane_n) and a
// head_t-subset of [head_off, head_off + head_n). The two ranges are disjoint.
// A tile is lane_mult consecutive blocks of 64 * slots lane subsets by
// heads_per_tile head steps: a rectangle with fewer heads than that takes
// several lane blocks per tile, so that the tiles of a level cost about the same.
struct Rect {
    uint32_t lane_off, lane_n, lane_t, head_off;
    uint32_t head_n, head_t, lane_mult, _r1;
    uint64_t lane_count, head_count;   // C(lane_n, lane_t), C(head_n, head_t)
    uint64_t tile_begin;               // first tile index of this rectangle
    uint64_t lane_blocks, head_blocks; // tiles along each factor (lane: blocks of lane_mult)
    uint64_t _r2;
};
static_assert(sizeof(Rect) == 80, "Rect is 80 bytes");

// Task key: minimum weight in the top 9 bits, tile index in the low 55.
constexpr int kTileBits = 55;
constexpr uint64_t kTileMask = (1ull << kTileBits) - 1;
constexpr uint64_t kMaxTiles = 1ull << 40;

// The tiling of one level g (shared by every Gamma_j of the code: all have k rows).
struct LevelPlan {
    uint32_t k = 0, g = 0, slots = 0, heads_per_tile = 0;
    uint64_t total_tiles = 0, combinations = 0;
    std::vector<Rect> rects;
};

// widen: rectangles with fewer heads than a tile holds take several lane
// blocks per tile (lane_mult); otherwise lane_mult is 1.
bool plan_level(uint32_t k, uint32_t g, uint32_t slots, uint32_t heads_per_tile,
                uint64_t target_tiles, LevelPlan &out, std::string &err, bool widen = false);

// A code's smallest levels run in one launch of a single work-group
// (bz_one_kernel): the levels of at most kOneLaunchComb sums, tasks small
// enough that one compute unit finishes them sooner than a launch of their own
// would start. Their task list and tilings are fixed by the code, so
// bz_prepare builds and uploads them with Gamma_j.
constexpr double kOneLaunchComb = 4096.0;
constexpr uint64_t kOneTargetTiles = 8;            // tiles per task: two per wave of the work-group
constexpr uint32_t kOneMaxTasks = 128;
constexpr uint32_t kOneMaxRects = 64;

// Task (Gamma_j, g) of that launch, in Alg. 1's order.
struct OneTask {
    uint64_t total_tiles;         // tiles of the task's tiling
    uint64_t comb;                // C(k, g): what a complete task enumerates
    uint32_t j, g, rect_off, nrects;
    uint32_t heads_per_tile, W, row_off;   // row width of Gamma_j; dword offset of its packed rows
    uint32_t cert_task;           // bound certified once this task is complete
    uint32_t cert_level;          // Alg. 1's L once the level is complete
    uint32_t last_of_level;       // the level's last matrix
    uint32_t _pad[2];
};
static_assert(sizeof(OneTask) == 64, "OneTask is 64 bytes");
// The same for the g-subsets of rows [lo, lo + n) (plan_level is lo = 0, n = k).
bool plan_range(uint32_t lo, uint32_t n, uint32_t g, uint32_t slots, uint32_t heads_per_tile,
                uint64_t target_tiles, LevelPlan &out, std::string &err, bool widen = false);

// C(a, b) with saturation at kBinomSat for values >= 2^63.
uint64_t binom_sat(uint32_t a, uint32_t b);

}  // namespace bz

// A prepared code: Gamma_j on the host and on one device.
struct bz_code {
    uint32_t n = 0, k = 0, num_full = 0, partial_rank = 0;
    uint32_t nsets = 0;                 // num_full + (partial_rank > 0)
    uint32_t W_full = 0, W_partial = 0;
    int device = 0;
    std::vector<int32_t> set_of_column; // n entries
    std::vector<bz::HostRow> full_rows; // nsets * k rows, original coordinates
    std::vector<uint32_t> packed;       // per matrix: k * W(j) dwords, non-set columns
    std::vector<size_t> packed_off;     // dword offset of matrix j in packed
    void *dev = nullptr;                // device copy: packed rows, then full rows
    size_t dev_bytes = 0;
    size_t dev_full_off = 0;            // byte offset of the full rows in dev
    uint32_t px_delta = 0;              // dwords from packed rows to their prefix XORs in packed
    // the smallest levels' one launch: task list, the tiling of each task's
    // level (one_plan_of), and where its arguments, tasks and rectangles sit in dev
    std::vector<bz::OneTask> one_tasks;
    std::vector<bz::LevelPlan> one_plans;
    std::vector<uint32_t> one_plan_of;
    size_t dev_one_off = 0;
    size_t one_lds = 0;                 // LDS bytes of the launch
    bool one_lds_binom = false;         // binomials staged in LDS
    bool one_likely = false;            // the one launch's levels may well end the search
    double prepare_s = 0.0;
    uint32_t W(uint32_t j) const { return j < num_full ? W_full : W_partial; }
    uint32_t k_low(uint32_t j) const { return j < num_full ? k : partial_rank; }
};

namespace bz {
bz_status prepare_host(const uint64_t *G, uint32_t k, uint32_t n, uint32_t ld,
                       const bz_prepare_opts *opts, bz_code &c, std::string &err);
}
