/*
 * bz_debug.h -- inspection and measurement entry points of libbz.
 *
 * The first two run without a GPU: they expose the host halves of bz_prepare
 * and of the level planner so that tests (and curious users) can check them
 * on a CPU. The last measures the device's sustained integer issue rate.
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
    uint32_t head_n, head_t, _reserved0, _reserved1;
    uint64_t lane_count, head_count;   /* C(lane_n, lane_t), C(head_n, head_t)   */
    uint64_t tile_begin;               /* first tile of this rectangle           */
    uint64_t lane_blocks, head_blocks; /* tiles along each factor               */
    uint64_t _reserved2;
} bz_debug_rect;

/* The tiling the search uses for level g of a Gamma matrix with k rows
 * (slots per lane 2, 4, 8 or 16; heads_per_tile 0 = chosen from target_tiles). */
bz_status bz_debug_plan_level(uint32_t k, uint32_t g, uint32_t slots, uint32_t heads_per_tile,
                              uint64_t target_tiles, bz_debug_rect *rects, uint32_t cap,
                              uint32_t *nrects, uint64_t *total_tiles, uint32_t *heads_used);

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
