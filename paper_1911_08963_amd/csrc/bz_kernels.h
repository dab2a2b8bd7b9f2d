// Launch interface of the HIP kernels (host <-> device argument blocks).
#pragma once

#include <hip/hip_runtime.h>

#include "bz_internal.h"

namespace bz {

// One (Gamma_j, g) task: arguments of the enumeration kernel.
struct TaskArgs {
    const uint32_t *rows;        // k x W packed rows of Gamma_j (device)
    const uint64_t *binom;       // kBinomRows x (kBinomT + 1) binomials (device)
    const Rect *rects;           // the level's rectangles (device)
    unsigned long long *key;     // (min weight << 55) | tile, atomicMin
    unsigned long long *stats;   // (min << 55) | count, statistics mode
    unsigned long long *ncomb;   // combinations enumerated
    unsigned long long *tile_ctr;   // reserved (tiles are assigned statically)
    const uint32_t *cancel;      // host-visible cancel word, or null
    uint32_t nrects, k, k_low, g;
    uint32_t heads_per_tile;
    uint64_t total_tiles;
    uint32_t u_prev;             // upper bound from completed tasks
    uint32_t exit_at;            // stop when the upper bound is <= this (0 = never)
};

struct RecoverArgs {
    const uint32_t *rows;        // packed rows of Gamma_j
    const uint64_t *full_rows;   // k x kHostWords full rows of Gamma_j
    const uint64_t *binom;
    const Rect *rect;            // the winning tile's rectangle (device)
    unsigned int *flag;          // 0 before the launch
    uint32_t *indices;           // up to g row indices
    uint32_t *indices_len;
    unsigned long long *codeword;   // kHostWords words
    uint64_t tile;
    uint32_t slots, heads_per_tile, W, k_low, target;
};

hipError_t launch_enum(const TaskArgs &a, uint32_t W, uint32_t slots, bool partial, bool stats,
                       uint32_t grid, hipStream_t st);
size_t enum_lds_bytes(uint32_t k, uint32_t g, uint32_t W);
hipError_t launch_task_init(unsigned long long *key, unsigned long long *stats,
                            unsigned long long *ncomb, unsigned long long *ctr, hipStream_t st);
hipError_t launch_recover(const RecoverArgs &a, hipStream_t st);

}  // namespace bz
