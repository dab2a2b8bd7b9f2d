/*
 * bz.h -- C ABI of libbz: the Brouwer-Zimmermann minimum distance of a binary
 * linear code on one AMD Instinct MI355X (gfx950).
 *
 * Method: arXiv:1911.08963, Sec. 2.1 and Alg. 1. For an [n, k] code with
 * generator matrix G, find disjoint information sets S_1..S_{m_f} (plus a
 * leftover set S_m of rank k_m < k), put G in systematic form Gamma_j on each,
 * and for g = 1, 2, ... enumerate every sum of g rows of every Gamma_j. The
 * smallest weight seen is an upper bound U on d; after each completed
 * (Gamma_j, g) the enumerated sums certify a lower bound L. The search stops
 * once L >= U, and then d = U.
 *
 * Conventions for every call:
 *  - All functions return a bz_status: 0 = success, negative = error.
 *  - On error, no output is marked valid (d = 0).
 *  - bz_last_error() holds a thread-local message describing the last error.
 *  - Bit layout: matrices are row-major uint64 words, LSB first. Coordinate c
 *    of row i is bit (c % 64) of word [i * ld_words + c / 64]. Bits at
 *    positions >= n are ignored on input and zero on output.
 *  - Host pointers are read or written only during the call. The library keeps
 *    no caller pointer after it returns.
 *  - Device work runs on the caller's HIP stream (bz_opts.hip_stream, NULL = the
 *    null stream). Calls are synchronous: the results are in caller memory when
 *    they return. A prepared bz_code is immutable: any number of threads may
 *    search it concurrently, each on its own stream with its own workspace.
 *  - Limits: n <= BZ_MAX_N. Every level searched must have C(k, g) < 2^63
 *    (BZ_ELIMIT otherwise).
 */
#ifndef BZ_H
#define BZ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BZ_MAX_N 256

typedef enum {
    BZ_OK = 0,
    BZ_EINVAL = -1,     /* a null pointer, a size out of range, an unknown flag   */
    BZ_ERANK = -2,      /* the k rows of G are linearly dependent                  */
    BZ_ENOMEM = -3,     /* host or device allocation failed, or workspace too small */
    BZ_EDEVICE = -4,    /* a HIP call failed (bz_last_error names it)              */
    BZ_ELIMIT = -5,     /* C(k,g) >= 2^63, max_level reached, or stats buffer full */
    BZ_ECANCELED = -6,  /* the caller's cancel word became nonzero                 */
    BZ_EBUSY = -7       /* the server has no free slot                             */
} bz_status;

typedef struct bz_code bz_code;   /* opaque; immutable after bz_prepare */

/* Column-permutation search for the information sets (Sec. 2.2 tries random
 * permutations of the columns). perm_trials = 0 or 1 scans the columns in
 * their natural order. With perm_trials = T > 1 the greedy scan runs for
 * trials t = 0..T-1 over the column order p_t and keeps the trial with the
 * most full-rank sets, then the largest leftover rank (the first on ties).
 * p_0 is the natural order; for t >= 1, p_t is the Fisher-Yates shuffle of
 * (0..n-1) that, for i = n-1 down to 1, swaps positions i and x mod (i+1),
 * x the next output of SplitMix64 (Steele, Lea, Flood 2014) started from
 * state perm_seed + t. The sets are sorted ascending, so Gamma_j depends only
 * on its set. d never depends on the sets; the per-level statistics do.
 * perm_trials above 100000 is EINVAL. */
typedef struct {
    uint32_t perm_trials;
    uint32_t flags;             /* BZ_PREPARE_HOST_ONLY: keep Gamma_j on the host only */
    uint64_t perm_seed;
} bz_prepare_opts;

/* A host-only code makes no device allocation and no device copy; only a
 * server (bz_server_submit) can search it, which copies Gamma_j itself. */
#define BZ_PREPARE_HOST_ONLY 1u

/* Sec. 2.1, information sets and the systematic matrices Gamma_j.
 * Copies G (k rows of ld_words uint64, layout above); the caller keeps G.
 * Finds the information sets greedily: S_1 is the first basis in column order,
 * S_2 the first basis of the remaining columns, and so on, while the remaining
 * columns still have rank k. The last columns have rank k_m < k. Gamma_j is
 * the reduced echelon form of G with S_j's columns first. Gamma_j's
 * non-identity columns are uploaded to the current HIP device (not for
 * BZ_PREPARE_HOST_ONLY). bz_min_distance and bz_min_distance_batch refuse a
 * host-only code (EINVAL).
 * Errors: EINVAL (G or out null, k == 0, k > n, n > BZ_MAX_N,
 * ld_words < ceil(n/64)); ERANK (rank(G) < k); ENOMEM; EDEVICE. */
bz_status bz_prepare(const uint64_t *G, uint32_t k, uint32_t n, uint32_t ld_words,
                     const bz_prepare_opts *opts /* nullable */, bz_code **out);

typedef struct {
    uint32_t n, k;
    uint32_t num_full;      /* m_f: number of full-rank disjoint information sets   */
    uint32_t partial_rank;  /* k_m: rank of the leftover columns (0 = no Gamma_m)   */
    uint32_t W_full;        /* 32-bit words per device row of a full-rank Gamma_j   */
    uint32_t W_partial;     /* the same for Gamma_m (0 if absent)                    */
} bz_code_info;

/* The shape of a prepared code: m_f and k_m of Sec. 2.1 (the number of
 * disjoint full-rank information sets and the rank of the leftover columns),
 * and the 32-bit words per device row. set_of_column (nullable, n entries):
 * index j of the set holding column c, or -1. */
bz_status bz_code_get_info(const bz_code *c, bz_code_info *out, int32_t *set_of_column);

/* Host copy of Gamma_j (k rows of ld_words uint64, original column order). */
bz_status bz_code_get_gamma(const bz_code *c, uint32_t matrix, uint64_t *rows, uint32_t ld_words);

void bz_free(bz_code *c);

/* Search flags. */
enum {
    BZ_F_STATS = 1u,        /* record per-(Gamma_j, g) minimum and count; no exit inside a task */
    BZ_F_LEVEL_STOP = 2u,   /* check L >= U once per level (Alg. 1 as printed)                 */
    BZ_F_NO_WITNESS = 4u,   /* skip witness recovery                                           */
    BZ_F_TASK_LAUNCHES = 8u /* bz_min_distance: one launch per task on every level (by default the
                               levels of at most 4096 sums run in one launch of one work-group,
                               and consecutive full-rank tasks of levels below 2^27 sums that
                               use the same kernel variant share launches); EINVAL elsewhere */
};

typedef struct {
    uint32_t flags;
    uint32_t max_level;         /* 0 = no limit; otherwise stop (BZ_ELIMIT) after this level */
    void *hip_stream;           /* hipStream_t, or NULL for the null stream                  */
    void *workspace;            /* caller device memory, or NULL: the library allocates     */
    size_t workspace_bytes;
    volatile const uint32_t *cancel;   /* host-visible word; nonzero cancels (nullable)      */
    uint32_t slots_per_lane;    /* combinations kept per lane (2, 4, 8, 16); 0 = autotuned or by row width */
    uint32_t heads_per_tile;    /* head steps per wave tile; 0 = autotuned or the planner's choice      */
    uint32_t tiles_per_task;    /* batch: tiles a task is cut into (about); 0 = autotuned or 64         */
    uint32_t schedule;          /* bz_min_distance: BZ_SCHED_* (0 = equal-cost tiles, the default)       */
    uint32_t prefix;            /* prefix size p of BZ_SCHED_1..8: absolute (D_*) or relative (S_*)     */
    uint32_t _reserved;
} bz_opts;

/* How bz_min_distance cuts a (Gamma_j, g) task and deals it to the device's
 * waves. The default cuts the level's combinations into tiles of equal cost
 * and deals them round-robin. The other eight are the distributed algorithms
 * of Sec. 3 of arXiv:1911.08963 with one wave per worker: a task is a prefix,
 * a p-subset c_1 < ... < c_p of the rows, that stands for every g-subset
 * starting with it (C(k - 1 - c_p, g - p) of them; C(k - (g - p), p)
 * prefixes); a wave adds the prefix rows once and enumerates the completions.
 * Prefixes come in lexicographic order (Lex) or left-lexicographic order
 * (Lle: the left-most element changes fastest). Dynamic schedules (D_*) hand
 * them out from a shared counter, one per claim, or with 2CM two per claim,
 * one from each end of the order. Static ones (S_*) deal them cyclically, or
 * snake cyclically (SNC: every second round in reverse). D_* take p as the
 * prefix size; S_* take it relative to g (the prefix has g - p elements).
 * A prefix of g or more elements, or of none, makes the level one task. The
 * result (d, bounds, statistics) is the same under every schedule; only the
 * time changes. Schedules 1..8 need prefix >= 1, use the fixed lane sums per
 * lane (16 up to W = 4, else 8) and tilings of their own (slots_per_lane and
 * heads_per_tile are ignored), allocate those tilings on the device per
 * search, and apply to bz_min_distance only (the batch call returns
 * BZ_EINVAL; the server ignores the field). */
enum {
    BZ_SCHED_TILES = 0,
    BZ_SCHED_D_LEX = 1, BZ_SCHED_D_LEX_2CM = 2, BZ_SCHED_D_LLE = 3, BZ_SCHED_D_LLE_2CM = 4,
    BZ_SCHED_S_LEX = 5, BZ_SCHED_S_LEX_SNC = 6, BZ_SCHED_S_LLE = 7, BZ_SCHED_S_LLE_SNC = 8
};

typedef struct {
    uint16_t matrix, level;     /* j (0-based; the partial Gamma_m is j = m_f) and g        */
    uint32_t min_weight;        /* min wt(c Gamma_j) over wt(c) = g                          */
    uint64_t count_at_min;      /* number of c reaching it (BZ_F_STATS only, else 0)         */
    uint64_t combinations;      /* C(k, g) for a completed task                              */
} bz_level_stat;

typedef struct {
    uint32_t d;                 /* minimum distance (0 unless status is BZ_OK)               */
    uint32_t lower_bound;       /* last certified L                                          */
    uint32_t upper_bound;       /* U at the end                                              */
    uint32_t last_level;        /* last level g entered                                      */
    uint64_t combinations;      /* row combinations enumerated                               */
    uint64_t *witness;          /* caller buffer of ceil(n/64) words, or NULL                */
    bz_level_stat *stats;       /* caller buffer of stats_cap entries, or NULL               */
    uint32_t stats_cap;
    uint32_t stats_len;         /* tasks completed (may exceed stats_cap: then BZ_ELIMIT)    */
    uint32_t launches;          /* enumeration kernel launches                               */
    uint32_t _pad;
    double prepare_s;           /* host seconds in bz_prepare (filled by the batch call)     */
    double search_s;            /* host wall seconds of the search                           */
    double kernel_s;            /* summed device time of the enumeration launches            */
} bz_result;

/* Device bytes the library needs for these codes under these options (the
 * workspace of bz_min_distance with count 0 or 1, of bz_min_distance_batch
 * otherwise). A property of this library's layout; the paper has no
 * counterpart. Errors: EINVAL, EDEVICE. */
bz_status bz_workspace_bytes(bz_code *const *codes, uint32_t count, const bz_opts *o, size_t *bytes);

/* Alg. 1 on one code, the check after every Gamma_j by default.
 * Level g of Gamma_j is one launch of the enumeration kernel. Each wave takes
 * equal-sized tiles of the combination space (Sec. 3.1 explains why tasks
 * should cost the same), keeps the running minimum in registers, and ends each
 * tile with one atomic. The witness is the codeword of weight d that the
 * recovery kernel re-finds in the winning tile. */
bz_status bz_min_distance(bz_code *code, const bz_opts *o, bz_result *res);

/* A search that allocates nothing, for callers that cannot allocate device
 * or pinned memory while they run: code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation.
 *
 * Gives exactly what bz_min_distance gives for the same code and options, but
 * works in a device array inside the library instead of a workspace:
 *  - The array holds BZ_NOALLOC_SCRATCH_BYTES per device (the binomial table
 *    and one search's workspace); each device the library runs on keeps its
 *    own copy until the process ends. o->workspace must be NULL.
 *  - The first call on a device looks up the array's address there and copies
 *    the binomial table into it (a copy, no allocation), and sets aside the
 *    host memory for the read-backs. Later calls only use them.
 *  - Calls on one device share its array, so they would race if they
 *    overlapped: the library serialises them with a lock per device (calls on
 *    different devices run concurrently). Each call initialises every part of
 *    the array it reads; nothing carries over from the previous call.
 *  - Read-backs go through ordinary host memory, and kernel_s stays 0 (no
 *    timing events).
 * Limits and errors: as bz_min_distance; EINVAL for a workspace or for
 * schedules 1..8 (their tilings need device memory of their own); ELIMIT for a
 * level whose tiling needs more than the 16384 rectangles the array holds. */
#define BZ_NOALLOC_SCRATCH_BYTES 1572864u
bz_status bz_min_distance_noalloc(bz_code *code, const bz_opts *o, bz_result *res);

/* Many codes at once: Alg. 1 (with the per-Gamma check of Sec. 2.2) for each
 * code, all in one persistent launch that drains a device queue of
 * (code, Gamma_j, g, tile) work; the wave that completes a task does that
 * code's bookkeeping and publishes its next task (the dynamic coordinator and
 * workers of Sec. 3.2, on the waves of one GPU; the paper runs one code at a
 * time). Each code's result equals bz_min_distance's for it. res[i] and
 * per_code[i] belong to codes[i]. Returns the first per-code error, or BZ_OK.
 * o->workspace, when given, must hold bz_workspace_bytes for these codes
 * (ENOMEM otherwise). */
bz_status bz_min_distance_batch(bz_code *const *codes, uint32_t count, const bz_opts *o,
                                bz_result *res, bz_status *per_code);

/* ---- Codewords of a given weight (the exact count A_w; not in the paper,
 * which returns d only).
 *
 * Runs the tasks (Gamma_j, g) in the order of Alg. 1, collects every sum of
 * weight w, and stops once the bound certified by the completed tasks (the
 * per-Gamma bound of Sec. 2.2 / Alg. 1) exceeds w: then every codeword not
 * enumerated weighs more than w. A codeword is met in every Gamma_j in which
 * it is light, so the library keeps the distinct codewords. */
typedef struct {
    uint32_t weight;            /* in: w; 0 = the minimum distance (found first). out: w     */
    uint32_t last_level;        /* last level g enumerated                                   */
    uint64_t count;             /* codewords of weight w                                     */
    uint64_t hits;              /* weight-w sums met (with repeats across the Gamma_j)        */
    uint64_t combinations;      /* sums enumerated by the counting pass                      */
    uint64_t *codewords;        /* caller buffer of codewords_cap x ceil(n/64) words, or NULL */
    uint64_t codewords_cap;
    uint64_t codewords_len;     /* codewords written: the smallest as integers (last word most significant) */
    double search_s;
} bz_weight_count;

/* o: hip_stream; max_level (0 = none; ELIMIT if reached before the count is
 * complete). Errors: EINVAL (null, host-only code), ELIMIT (C(k,g) >= 2^63,
 * max_level, or more than 2^21 weight-w sums in one task), EDEVICE. */
bz_status bz_count_codewords(bz_code *code, const bz_opts *o, bz_weight_count *res);

/* ---- Autotuning of the enumeration's free parameters.
 *
 * Two parameters change only speed, never a result: the lane sums a lane keeps
 * (slots per lane: SLOTS x W registers, the unrolling of several left
 * combinations per fetched right one, Sec. 2.2.1) and the chunk size of a task
 * (Sec. 3.1), set as tiles per resident wave: the planner sizes each level's
 * tiles so the level has about that many per wave the device holds.
 * bz_autotune times the enumeration kernel on a synthetic full-rank task of k
 * rows and row width W (the first level g with 2e10 sums or more, else the
 * largest) for slots 2/4/8/16 x tiles per wave 1/2/4/8/16/64, each the fastest
 * of three launches, and installs the fastest for W: later bz_min_distance
 * calls use it when slots_per_lane and heads_per_tile are both 0 (the fixed
 * rule otherwise: 16 slots up to W = 4, then 8; 4 tiles per wave). The table
 * is per process and shared by all threads. Errors: EINVAL (W not 1..8, k not
 * 2..256), ELIMIT, EDEVICE. */
typedef struct {
    uint32_t W, k, g;           /* the shape timed                                       */
    uint32_t slots_per_lane;    /* chosen                                                */
    uint32_t tiles_per_wave;    /* chosen                                                */
    uint32_t heads_per_tile;    /* what that gave at the timed level                     */
    uint64_t combinations;      /* sums per timed launch (C(k, g))                        */
    double comb_per_s;          /* with the chosen pair                                  */
    double default_comb_per_s;  /* with the fixed rule                                   */
} bz_tune_entry;

bz_status bz_autotune(uint32_t W, uint32_t k, bz_tune_entry *out);
/* The installed entry for W (EINVAL if none). */
bz_status bz_autotune_get(uint32_t W, bz_tune_entry *out);
/* Installs a choice without timing (for example one saved from an earlier
 * bz_autotune): only W, slots_per_lane and tiles_per_wave are read. Errors:
 * EINVAL (W not 1..8, slots not 2/4/8/16 or 16 with W > 4, tiles per wave not
 * 1..4096). */
bz_status bz_autotune_set(const bz_tune_entry *e);
/* Forget every installed choice (plain and batch). */
void bz_autotune_clear(void);
/* Times bz_min_distance_batch on these codes (fast mode, no witness) with
 * 16, 64, 256 and 1024 tiles per task, twice each, and installs the fastest
 * for later batch calls that leave tiles_per_task at 0. Writes it and its
 * best wall time. Errors: as bz_min_distance_batch. */
bz_status bz_autotune_batch(bz_code *const *codes, uint32_t count, const bz_opts *o, uint32_t *tiles_per_task,
                            double *seconds);

/* ---- Serving: a resident search that admits requests while it runs.
 *
 * Continuous batching of many searches on one device (the dynamic
 * coordinator/worker scheme of Sec. 3.2, with the GPU's waves as workers).
 * bz_server_create launches one persistent kernel that stays on the device
 * until bz_server_destroy. Each bz_server_submit stages one code's Gamma_j in
 * pinned host memory and publishes it at once: a wave of the running kernel
 * copies it onto the device and starts its level loop beside the requests
 * already there, and idle waves help with the largest task of any request.
 * Every request runs the same Alg. 1 bookkeeping as bz_min_distance_batch,
 * so its result does not depend on what else runs.
 *
 * Admission: a request takes one of `slots` request slots and dev_bytes of
 * the HBM budget until it is polled. Without a free slot or budget, submit
 * returns BZ_EBUSY and the caller retries after bz_server_poll. Device data of
 * finished requests is recycled by draining the server and relaunching the
 * kernel (submit returns BZ_EBUSY until the requests in flight are done).
 *
 * While a server runs it holds every compute unit of its device: other
 * libbz searches on that device wait until it is destroyed.
 * A server is used by one thread at a time (calls are serialized inside).
 */
typedef struct bz_server bz_server;

typedef struct {
    uint32_t slots;             /* requests in flight at most (1..65536; 0 = 1024)                 */
    uint32_t flags;             /* BZ_F_STATS: statistics mode for every request                   */
    size_t hbm_budget;          /* device bytes in-flight requests may hold (0 = no limit)         */
    uint32_t stats_cap;         /* task records kept per request (0 = 512)                         */
    uint32_t target_tiles;      /* tiles per task aimed at by the planner (0 = 4 per resident wave) */
    size_t arena_bytes;         /* device bytes for Gamma_j of one kernel launch (0 = 1 GiB)       */
    uint32_t codes_per_launch;  /* requests per kernel launch before a relaunch (0 = 1 << 18)      */
    uint32_t _reserved;
} bz_server_opts;

/* Creates a server on the current HIP device and launches its kernel on a
 * stream of its own. Errors: EINVAL, ENOMEM, EDEVICE. */
bz_status bz_server_create(const bz_server_opts *o /* nullable */, bz_server **out);

/* Submits one search. o: flags BZ_F_LEVEL_STOP / BZ_F_NO_WITNESS, and BZ_F_STATS
 * exactly as the server was created; max_level. The other bz_opts fields are
 * ignored. The code may be freed after the call. res (with its witness and
 * stats buffers) must stay valid until bz_server_poll returns its ticket; then
 * it holds what bz_min_distance would give, search_s being the time from
 * submission to completion. Errors: EINVAL, EBUSY (no slot, budget or ring
 * entry free: poll, then retry), ENOMEM (plan tables full), EDEVICE. */
bz_status bz_server_submit(bz_server *s, const bz_code *code, const bz_opts *o, bz_result *res,
                           uint64_t *ticket);

/* Collects finished requests: fills their bz_result and writes up to cap
 * (ticket, status) pairs, in completion order; *n_done is their number. */
bz_status bz_server_poll(bz_server *s, uint64_t *tickets, bz_status *statuses, uint32_t cap,
                         uint32_t *n_done);

/* Requests submitted and not yet polled. */
bz_status bz_server_pending(bz_server *s, uint32_t *pending);

/* Lets the published requests finish, stops the kernel and frees everything.
 * Results not polled are dropped. Returns EDEVICE if the kernel had to be
 * stopped (after timeout_s seconds; 0 = 60) before the requests finished. */
bz_status bz_server_destroy(bz_server *s, double timeout_s);

const char *bz_status_str(bz_status s);
const char *bz_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BZ_H */
