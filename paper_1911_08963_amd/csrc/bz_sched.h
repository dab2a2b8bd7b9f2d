// The prefix tasks of the paper's distributed algorithms (Sec. 3 of
// arXiv:1911.08963) and the eight ways they are dealt to workers, as plain
// functions that the schedule kernel (bz_sched.hip, workers = waves) and the
// host's inspection entry point (bz_debug_schedule) share.
//
// A task at level g is a prefix: a p-subset c_1 < ... < c_p of the k rows whose
// last element leaves room for the other g - p, so the prefixes are the
// p-subsets of [0, k - (g - p)), C(k - (g - p), p) of them (Sec. 3.1.1).
// Processing a prefix enumerates every (g - p)-subset of (c_p, k) joined to it
// (Process_prefix, Sec. 3.1); its cost is C(k - 1 - c_p, g - p) (Sec. 3.1.2).
//
// Orders (Sec. 3.1.3): lexicographic, or left-lexicographic, where the
// left-most element changes fastest (colex order: the last element never
// decreases, so the costly prefixes come first).
// Distributions (Secs. 3.2 and 3.3):
//  - cyclic: turn s of worker w is task s * P + w (P workers);
//  - snake cyclic: the same on even turns, reversed (s * P + P - 1 - w) on odd;
//  - queue: each claim of a shared counter hands out the next task;
//  - queue by pairs ("2cm"): claim c hands out task c from the front of the
//    order and task N - 1 - c from its end.
// Static schedules (S-*) take the prefix size relative to g (the prefix has
// g - p elements); dynamic ones (D-*) take it as given. When the prefix would
// have g or more elements, or none, the level is one task: the empty prefix,
// whose completions are all g-subsets (the paper replicates the level on every
// worker instead of splitting it; one worker's time is the same).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bz {

enum : uint32_t { kDistCyclic = 0, kDistSnake = 1, kDistQueue = 2, kDistQueuePairs = 3 };
enum : uint32_t { kOrderLex = 0, kOrderLeftLex = 1 };

// The public schedule number (include/bz.h, BZ_SCHED_*) split into its
// distribution and order; false for 0 (equal-cost tiles) and unknown values.
__host__ __device__ inline bool sched_parts(uint32_t schedule, uint32_t &dist, uint32_t &order, bool &dynamic) {
    switch (schedule) {
    case 1: dist = kDistQueue;      order = kOrderLex;     dynamic = true;  return true;   // D-Lex
    case 2: dist = kDistQueuePairs; order = kOrderLex;     dynamic = true;  return true;   // D-Lex-2cm
    case 3: dist = kDistQueue;      order = kOrderLeftLex; dynamic = true;  return true;   // D-Lle
    case 4: dist = kDistQueuePairs; order = kOrderLeftLex; dynamic = true;  return true;   // D-Lle-2cm
    case 5: dist = kDistCyclic;     order = kOrderLex;     dynamic = false; return true;   // S-Lex
    case 6: dist = kDistSnake;      order = kOrderLex;     dynamic = false; return true;   // S-Lex-Snc
    case 7: dist = kDistCyclic;     order = kOrderLeftLex; dynamic = false; return true;   // S-Lle
    case 8: dist = kDistSnake;      order = kOrderLeftLex; dynamic = false; return true;   // S-Lle-Snc
    default: return false;
    }
}

// The prefix's number of elements at level g for the given prefix size
// (relative for static schedules); 0 means the whole level is one task.
__host__ __device__ inline uint32_t prefix_elems(bool dynamic, uint32_t p, uint32_t g) {
    const uint32_t e = dynamic ? p : (g > p ? g - p : 0u);
    return e >= g ? 0u : e;
}

// Static distributions: the task of worker w at its turn s (turns run while
// s * P < ntasks), or ~0 when that turn has none (only on a last, partial row).
__host__ __device__ inline uint64_t static_task(uint32_t dist, uint64_t w, uint64_t P, uint64_t s, uint64_t ntasks) {
    const uint64_t col = (dist == kDistSnake && (s & 1)) ? P - 1 - w : w;
    const uint64_t t = s * P + col;
    return t < ntasks ? t : ~0ull;
}

// Dynamic distributions: the tasks of claim c; returns how many (0 = none left).
__host__ __device__ inline uint32_t claim_tasks(uint32_t dist, uint64_t c, uint64_t ntasks, uint64_t &t0,
                                                uint64_t &t1) {
    if (dist == kDistQueuePairs) {
        if (c >= ntasks || c >= ntasks - c) return 0;   // past the end, or front passed back
        t0 = c;
        t1 = ntasks - 1 - c;
        return t1 == c ? 1u : 2u;
    }
    if (c >= ntasks) return 0;
    t0 = c;
    return 1;
}

// The prefix of the given rank among the p-subsets of [0, K), in the given
// order: emit(i, c) for each element, i its 0-based position in ascending
// order (the elements come largest first for left-lexicographic ranks,
// smallest first for lexicographic ones). binom(a, b) gives C(a, b) for
// a <= K, b <= p. Left-lexicographic is colex: the largest element is the
// largest c with C(c, p) <= rank, and so on down. A lexicographic rank i is
// the colex rank C(K, p) - 1 - i of the mirrored subset {K - 1 - c}.
template <class Binom, class Emit>
__host__ __device__ inline void prefix_unrank(uint32_t order, uint64_t rank, uint32_t p, uint32_t K, Binom binom,
                                              Emit emit) {
    uint64_t r = order == kOrderLex ? binom(K, p) - 1 - rank : rank;
    uint32_t hi = K - 1;
    for (uint32_t i = p; i >= 1; --i) {
        uint32_t lo = i - 1, top = hi;
        while (lo < top) {
            const uint32_t mid = (lo + top + 1) >> 1;
            if (binom(mid, i) <= r) lo = mid; else top = mid - 1;
        }
        r -= binom(lo, i);
        // colex digit i is the i-th smallest element; mirrored for lex
        if (order == kOrderLex) emit(p - i, K - 1 - lo);
        else emit(i - 1, lo);
        hi = lo - 1;
    }
}

}  // namespace bz
