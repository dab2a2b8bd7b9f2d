// Host-side helpers shared by the C ABI's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include <vector>

#include "bz_internal.h"
#include "bz_kernels.h"

namespace bz {

extern thread_local std::string g_err;       // the message bz_last_error returns

bz_status fail(bz_status s, const std::string &msg);
double now_s();                               // steady clock, seconds

// Per-device constants: the binomial table and the compute-unit count.
struct DeviceConst {
    uint64_t *binom = nullptr;
    int cus = 0;
};
bz_status device_const(int dev, DeviceConst &out);
// The binomial table as the kernels read it: kBinomRows x (kBinomT + 1) values.
std::vector<uint64_t> binom_table();

// Device address of the no-allocation search's scratch array on the current
// device (bz_noalloc.hip).
hipError_t noalloc_scratch_address(void **ptr);

// Plans of levels 1, 2, ... for one (k, slots): appends one PlanEntry per level
// (rect_off counted from rect_base + the rects already in `rects`) while
// C(k, g) < max_comb. Returns the last level planned. With heads_per_tile 0
// each level gets about target_tiles tiles; max_heads (0 = the planner's own
// cap) bounds their head steps.
uint32_t build_level_plans(uint32_t k, uint32_t slots, uint32_t heads_per_tile, uint64_t target_tiles,
                           uint64_t max_comb, uint32_t rect_base, std::vector<PlanEntry> &plans,
                           std::vector<Rect> &rects, uint32_t max_heads = 0);

// A (Gamma_j, g) task cut into the prefix tasks of one of the paper's
// schedules (bz_sched.h): entries[lo] tiles the completions of a prefix whose
// last element is lo - 1 (entries[0]: the empty prefix), rect_off counted in
// rects; the other entries are zero.
struct SchedPlan {
    uint32_t pre = 0;                 // prefix elements (0: the level is one task)
    uint64_t ntasks = 0;              // C(k - (g - pre), pre)
    uint64_t stride = 0;              // tiles of the largest completion plan
    std::vector<PlanEntry> entries;   // k + 1
    std::vector<Rect> rects;
};
bool build_sched_plan(uint32_t k, uint32_t g, bool dynamic, uint32_t prefix, uint32_t slots, SchedPlan &out,
                      std::string &err);
// The rows of prefix task `task` (ascending) and its completion plan's index.
void sched_prefix(const SchedPlan &sp, uint32_t k, uint32_t g, uint32_t order, uint64_t task,
                  std::vector<uint32_t> &rows, uint32_t &lo);

// The autotuned (slots per lane, tiles per resident wave) for row width W, if any.
bool tuned_choice(uint32_t W, uint32_t &slots, uint32_t &tiles_per_wave);
// The autotuned tiles per task of batches (0 = none).
uint32_t tuned_batch_tiles();

}  // namespace bz

#define BZ_HIP(call)                                                                                        \
    do {                                                                                                    \
        hipError_t e_ = (call);                                                                             \
        if (e_ != hipSuccess) return bz::fail(BZ_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)
