/*
 * bz_debug.h -- inspection and measurement entry points of libbz.
 *
 * The first three run without a GPU: they expose the host halves of
 * bz_prepare, of the level planner and of the prefix schedules so that tests
 * (and curious users) can check them on a CPU. The last measures the device's
 * sustained integer issue rate.
 * Same conventions as bz.h (status codes, LSB-first uint64 rows, no retained
 * pointers, bz_last_error for details).
 */
#ifndef BZ_DEBUG_H
#define BZ_DEBUG_H

#include "bz.h"

#ifdef __cplusplus
extern "C" {
#endif

/* The host part of bz_prepare (Sec. 2.1 of arXiv:1911.08963): information sets
 * and Gamma_j, without touching a device.
 * gamma_rows: (num_full + [partial_rank > 0]) * k rows of ld_words words, or NULL;
 * gamma_cap_rows is its capacity in rows. packed: the device form, per matrix
 * k rows of W(j) 32-bit words over the columns outside S_j in ascending order,
 * matrices back to back; packed_cap in words (NULL allowed).
 * Errors: as bz_prepare, plus BZ_ELIMIT when a buffer is too small. */
bz_status bz_debug_prepare_host(const uint64_t *G, uint32_t k, uint32_t n, uint32_t ld_words,
                                uint32_t *num_full, uint32_t *partial_rank, int32_t *set_of_column,
                                uint64_t *gamma_rows, uint32_t gamma_cap_rows,
                                uint32_t *packed, size_t packed_cap);

/* One rectangle of a level's tiling: every union of a lane_t-subset of
 * [lane_off, lane_off + lane_n) and a head_t-subset of [head_off, head_off + head_n). */
typedef struct {
    uint32_t lane_off, lane_n, lane_t, head_off;
    uint32_t head_n, head_t;
    uint32_t lane_mult;                /* blocks of 64 * slots lane subsets per tile */
    uint32_t _reserved1;
    uint64_t lane_count, head_count;   /* C(lane_n, lane_t), C(head_n, head_t)   */
    uint64_t tile_begin;               /* first tile of this rectangle           */
    uint64_t lane_blocks, head_blocks; /* tiles along each factor               */
    uint64_t _reserved2;
} bz_debug_rect;

/* The tiling the search uses for level g of a Gamma matrix with k rows
 * (slots per lane 2, 4, 8 or 16; heads_per_tile 0 = chosen from target_tiles;
 * widen != 0: rectangles with fewer heads than a tile take several lane blocks
 * per tile, as in bz_min_distance's own tilings). */
bz_status bz_debug_plan_level(uint32_t k, uint32_t g, uint32_t slots, uint32_t heads_per_tile,
                              uint64_t target_tiles, uint32_t widen, bz_debug_rect *rects, uint32_t cap,
                              uint32_t *nrects, uint64_t *total_tiles, uint32_t *heads_used);

/* The prefixes a schedule BZ_SCHED_1..8 hands out at level g of a Gamma
 * matrix with k rows and prefix size p (relative for the static schedules),
 * computed on the host with the device kernel's own mapping. Static: out[(w *
 * turns + s) * e + i] is element i of the prefix worker w of `workers` takes
 * at turn s. Dynamic: out[(c * 2 + s) * e + i] is element i of the s-th prefix
 * (s < 2) of claim c, for claims c < workers. e = *pre_elems, the prefix's
 * element count (0: the level is one task; then one entry per prefix, 0 for
 * the task). -1 marks no prefix. *ntasks gets the number of prefixes.
 * out may be NULL (counts only); cap is its length in entries. Errors: EINVAL
 * (schedule not 1..8, k not 1..256, g not 1..min(k, 64), p or workers 0),
 * ELIMIT (cap too small, too many prefixes). */
bz_status bz_debug_schedule(uint32_t schedule, uint32_t k, uint32_t g, uint32_t p, uint32_t workers,
                            uint32_t turns, int32_t *out, uint64_t cap, uint32_t *pre_elems, uint64_t *ntasks);

/* Sustained int32 VALU rate of the current device on the enumeration's own
 * instruction pair (an XOR with a wave-uniform operand, then a popcount that
 * accumulates), over 8 independent chains per lane in every wave the device
 * holds. iters: loop trips per lane (0 = 200000). Writes lane operations per
 * second (2 per XOR+popcount step) and the kernel's device seconds. It is the
 * measured peak beside the specification's (256 CUs x 4 SIMDs x 16 lanes x
 * clock). Errors: EINVAL (null output), EDEVICE. */
bz_status bz_debug_valu_rate(uint32_t iters, double *lane_ops_per_s, double *seconds);

#ifdef __cplusplus
}
#endif
#endif /* BZ_DEBUG_H */
