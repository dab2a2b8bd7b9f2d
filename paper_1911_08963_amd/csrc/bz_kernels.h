// Launch interface of the HIP kernels (host <-> device argument blocks).
#pragma once

#include <hip/hip_runtime.h>

#include "bz_internal.h"

namespace bz {

// Bounds of a single search held on the device while a window of its tasks
// runs without the host: the enumeration kernel takes U and its exit bound
// from here, and a one-thread step after each task applies Alg. 1's
// bookkeeping to it (lower U, raise the certified bound, stop).
struct ChainState {
    uint32_t U;                  // upper bound from completed tasks
    uint32_t exit_at;            // the next task stops once U <= this (0 = never)
    uint32_t done;               // nonzero: the search has stopped, later tasks do nothing
    uint32_t L;                  // Alg. 1's lower bound
    uint32_t Lcert;              // bound certified by the completed tasks
    uint32_t _pad[3];
};

// Per-task words of a window, one record each: the key, the statistics and
// combination count, the schedules' claim counter, each on a 128-byte line.
constexpr uint32_t kRecWords = 48;       // 384 bytes
constexpr uint32_t kRecKey = 0, kRecStats = 16, kRecNcomb = 17, kRecCtr = 32;

// Tasks of one level that may share a launch (TaskArgs::group).
constexpr uint32_t kMaxGroup = 4;

// One task's step of the device-side bookkeeping (run after the task).
struct ChainStep {
    ChainState *state;
    const unsigned long long *key;     // the task's key and combination count
    const unsigned long long *ncomb;
    uint64_t total;                    // C(k, g): what a complete task enumerates
    uint32_t cert_task;                // bound certified once this task is complete
    uint32_t last_of_level;            // the level's last matrix: Alg. 1's L and stop check
    uint32_t cert_level;               // Alg. 1's L once the level is complete
    uint32_t level_stop;               // stop only at level ends (Alg. 1 as printed)
    uint32_t stats;                    // statistics mode: no exit inside a task
    uint32_t _pad;
};

// One (Gamma_j, g) task: arguments of the enumeration kernel.
struct TaskArgs {
    const uint32_t *rows;        // k x W packed rows of Gamma_j (device)
    const uint64_t *binom;       // kBinomRows x (kBinomT + 1) binomials (device)
    const Rect *rects;           // the level's rectangles (device)
    unsigned long long *key;     // (min weight << 55) | tile, atomicMin
    unsigned long long *stats;   // (min << 55) | count, statistics mode
    unsigned long long *ncomb;   // combinations enumerated
    unsigned long long *tile_ctr;   // schedules: claim counter; enumeration with a step: work-groups done
    const uint32_t *cancel;      // host-visible cancel word, or null
    uint32_t nrects, k, k_low, g;
    uint32_t heads_per_tile;
    uint64_t total_tiles;
    uint32_t u_prev;             // upper bound from completed tasks
    uint32_t exit_at;            // stop when the upper bound is <= this (0 = never)
    const ChainState *chain;     // when set: u_prev and exit_at come from here, and a stopped search skips the task
    ChainStep step;              // when step.state is set: the last work-group to leave applies the task's
                                 // bookkeeping step (counting the work-groups in tile_ctr, zero at the start)
    // A group of consecutive tasks of one level in one launch (enumeration
    // kernel only): Gamma_j .. Gamma_j+group-1, all full rank, same tiling.
    // Task i's rows are at rows + i * rows_stride, its record kRecWords words
    // after task i-1's (key, stats, ncomb, tile_ctr), its step is step with
    // cert_task = cert_tasks[i] and last_of_level = bit i of last_mask.
    uint32_t group;              // 0 or 1: one task
    uint32_t rows_stride;
    uint32_t cert_tasks[kMaxGroup];
    uint32_t last_mask;
};

// Consecutive tasks of several levels in one launch (bz_enum_levels_kernel).
constexpr uint32_t kMaxLevelTasks = 8;

// A group of consecutive tasks in Alg. 1's order, spanning level ends: all
// full rank, all of one kernel variant. t carries what they share (binomials,
// k, bounds, cancel word, the step's state and flags), with t.rows the packed
// rows' base, t.rects the tilings' base, t.key the first task's record (task i's
// is kRecWords words further), t.g the largest level and t.total_tiles the sum.
// Task i: rows at t.rows + row_off[i], rectangles at t.rects + rect_off[i]
// (nrects[i] of them, heads[i] heads per tile), level g[i], tiles
// [tile_end[i-1], tile_end[i]) of the launch; its step has total = totals[i],
// cert_task = cert_task[i], cert_level = cert_level[i] and last_of_level =
// bit i of last_mask.
struct LevelsArgs {
    TaskArgs t;
    uint32_t ntasks, last_mask;
    uint32_t row_off[kMaxLevelTasks], rect_off[kMaxLevelTasks];
    uint32_t g[kMaxLevelTasks], nrects[kMaxLevelTasks], heads[kMaxLevelTasks];
    uint32_t cert_task[kMaxLevelTasks], cert_level[kMaxLevelTasks];
    uint64_t tile_end[kMaxLevelTasks], totals[kMaxLevelTasks];
};

struct RecoverArgs {
    const uint32_t *rows;        // packed rows of Gamma_j
    const uint64_t *full_rows;   // k x kHostWords full rows of Gamma_j
    const uint64_t *binom;
    Rect rect;                   // the winning tile's rectangle
    unsigned int *flag;          // 0 before the launch
    uint32_t *indices;           // up to g row indices
    uint32_t *indices_len;
    unsigned long long *codeword;   // kHostWords words
    uint64_t tile;
    uint32_t slots, heads_per_tile, W, k_low, target;
    uint32_t pre_n;              // rows of a prefix task joined to every combination (0 = none)
    const uint32_t *pre_rows;    // their indices (device)
};

// One task of a window, as the window's witness recovery needs it.
struct RecoverTask {
    const uint32_t *rows;        // packed rows of the task's Gamma_j
    const uint64_t *full_rows;   // k x kHostWords full rows of Gamma_j
    const Rect *rects;           // the task's tiling (device)
    uint32_t nrects, slots, heads_per_tile, W;
    uint32_t k_low, _pad;
};
static_assert(sizeof(RecoverTask) == 48, "RecoverTask is 48 bytes");

// Witness recovery at the end of a window, before the host has read it back:
// when the window stopped the search and the winning tile is one of its
// tasks', the window's last launch recovers the witness on the device.
struct RecoverWindowArgs {
    const ChainState *state;             // the window's bounds after its last step
    const unsigned long long *records;   // the window's records, kRecWords words apart
    const RecoverTask *tasks;            // ntasks entries
    const uint64_t *binom;
    unsigned int *flag;                  // 0 before the launch
    uint32_t *indices;
    uint32_t *indices_len;
    unsigned long long *codeword;        // kHostWords words
    uint32_t ntasks;
    uint32_t U0;                         // the upper bound when the window started
    uint32_t have0;                      // a winning tile was known when the window started
    uint32_t k;
    uint32_t lds_g;                      // binomials with y <= lds_g staged in LDS (0: read from binom)
    uint32_t _pad;
};

// ---- batched persistent search (bz_min_distance_batch)

// Tiling of level g for one k: rects[rect_off .. rect_off + nrects).
struct PlanEntry {
    uint64_t total_tiles;
    uint32_t rect_off, nrects, heads_per_tile, _pad[3];
};
static_assert(sizeof(PlanEntry) == 32, "PlanEntry is 32 bytes");

// Immutable description of one code of a batch. Whole scalar-cache lines:
// a server writes the entry of a new code while its neighbours are read.
struct alignas(64) BatchCode {
    const uint32_t *rows;        // packed rows: Gamma_j at j * (k + 1) * W_full, Gamma_m after them
    const uint64_t *full_rows;   // Gamma_j full rows at j * k * kHostWords
    uint32_t n, k, m_f, k_m;
    uint32_t nsets, W_full, W_partial, g_max;   // plans exist for levels 1..g_max
    uint32_t plan_full;          // plan of level g for a full-rank Gamma_j: plans[plan_full + g - 1]
    uint32_t plan_partial;       // the same for the partial Gamma_m (its slot count may differ)
    uint32_t stats_off, stats_cap;
    uint32_t flags, max_level;   // BZ_F_LEVEL_STOP; stop after this level (0 = no limit)
    uint64_t tag;                // serving: the request's ticket
    uint32_t slot;               // serving: the completion record and statistics slot
    uint32_t px_delta;           // dwords from rows to the rows' prefix XORs (same layout per matrix)
};
static_assert(sizeof(BatchCode) % 64 == 0, "BatchCode fills whole cache lines");

// One task of one code; two per code, selected by the parity of the epoch.
// The words of a task that many waves touch each sit on a 128-byte line of
// their own (the L2 serialises atomics per line): the completion count, the
// counts added once per claim, the key every tile polls, and the read-mostly
// description of the task.
struct alignas(128) TaskSlot {
    unsigned long long completed; // tiles finished
    unsigned long long _line0[15];
    unsigned long long ncomb;     // combinations enumerated
    unsigned long long stats;     // (min << 55) | count
    unsigned long long _line1[14];
    unsigned long long key;       // (min weight << 55) | tile
    unsigned long long _line2[15];
    unsigned long long tiles;     // (epoch << 40) | tile count: which task this slot holds
    uint32_t j, g, rect_off, nrects, heads_per_tile, exit_at;
    uint32_t u_prev, _pad[3];
};
static_assert(sizeof(TaskSlot) == 512, "TaskSlot is four 128-byte lines");

// The task log's control words (head, tail, the next unstarted code or
// ticket), each on a 128-byte line of its own, then the entries; offsets in
// 64-bit words from the log's base.
constexpr size_t kLogHead = 0, kLogTail = 16, kLogNext = 32, kLogEntries = 48;

constexpr uint64_t kEpochShift = 40;
constexpr uint64_t kCursorMask = (1ull << kEpochShift) - 1;
constexpr uint64_t kDoneEpoch = (1ull << 24) - 1;

struct alignas(128) CodeState {
    unsigned long long cursor;    // (epoch << 40) | next tile to hand out; epoch kDoneEpoch = finished
    unsigned long long _line0[15];   // the claim cursor has its line to itself
    uint32_t U, L, Lcert, status;
    uint32_t last_level, nstats, have_best, best_j;
    uint32_t best_g, _pad0;
    uint64_t best_tile, combinations;
    TaskSlot slot[2];
};
static_assert(sizeof(CodeState) == 1280, "CodeState is ten 128-byte lines");

struct BatchStat {                // one completed task
    uint16_t matrix, level;
    uint32_t min_weight;
    uint64_t count_at_min, combinations;
};

struct BatchRecover {             // witness of one code
    uint32_t flag, len, _pad[2];
    uint64_t codeword[kHostWords];
    uint32_t indices[kBinomT];
};

struct BatchArgs {
    const BatchCode *codes;
    CodeState *state;
    const PlanEntry *plans;
    const Rect *rects;
    const uint64_t *binom;
    BatchStat *stats;
    BatchRecover *recover;
    unsigned long long *log;      // published tasks, (code << 24 | epoch) + 1, append-only
    unsigned long long *log_head; // entries before it are exhausted
    unsigned long long *log_tail; // next free entry
    unsigned long long *next_code;// codes not yet started: next index to hand out
    unsigned int *done_count;
    const uint32_t *cancel;
    uint64_t log_cap;             // ring size of the log, a power of two (entry q at q & (log_cap - 1))
    uint32_t ncodes;
    // binomials C(x, y), x <= lds_k, y <= lds_g, staged in each work-group's
    // LDS when the launch gives it room for them (0 = read from binom)
    uint32_t lds_k, lds_g, _pad;
};

// ---- one code's smallest levels in one work-group (bz_min_distance)
//
// bz_prepare lists the tasks (Gamma_j, g) of the code's smallest levels in
// Alg. 1's order (OneTask) and uploads them with their tilings and the launch's
// arguments; a search launches one work-group over them and gets a record per
// task and the final state.

// Status of a launch (OneState::status).
enum : uint32_t { kOneRunning = 0, kOneStopped = 1, kOneContinue = 2, kOneCanceled = 3 };

// The result, written by the work-group.
struct alignas(128) OneState {
    uint32_t U, L, Lcert, status;
    uint32_t ntasks, have_best, best_task, wit_flag;   // tasks run; witness: 0 not sought, 1 found, 2 not found
    uint64_t best_tile, combinations;
    uint64_t witness[kHostWords];
};
static_assert(sizeof(OneState) == 128, "OneState is one 128-byte line");

// Arguments fixed by the code (built by bz_prepare, in device memory).
struct OneArgs {
    const OneTask *tasks;
    const uint32_t *rows;         // packed rows of every Gamma_j ((k + 1) x W per matrix)
    const uint64_t *full_rows;    // full rows (witness), k x kHostWords per matrix
    const Rect *rects;
    const uint64_t *binom;        // kBinomRows x (kBinomT + 1)
    uint32_t ntasks, k, k_m, m_f;
    uint32_t U0;                  // n - k + 1
    uint32_t lds_g;               // binomials C(x, y), y <= lds_g, staged in LDS (0: read from binom)
    uint32_t row_words;           // packed-row and prefix-XOR dwords of all matrices, staged in LDS
    uint32_t px_delta;            // dwords from a matrix's rows to its prefix XORs
};

// Arguments of one search (by value).
struct OneRun {
    OneState *state;              // the result: host-visible pinned memory, or device memory
    BatchStat *stats;             // one record per task run
    const uint32_t *cancel;       // host-visible cancel word, or null
    uint32_t ntasks;              // run the first ntasks tasks of the list
    uint32_t level_stop, want_witness, _pad;
};

// One work-group of kBlock threads. args: in device memory. lds: the packed
// rows, then the binomial table (batch_lds_bytes(k, lds_g)) when lds_binom.
hipError_t launch_one(const OneArgs *args, const OneRun &run, bool stats, bool lds_binom, size_t lds,
                      hipStream_t st);

// ---- serving: a resident search that admits codes while it runs
//
// The host stages each request in pinned host memory and publishes it by
// raising a ticket count; the wave that holds the ticket copies the request
// onto the device itself, so nothing but the resident kernel writes the device
// memory it reads while it runs. Within one launch the code index of a request
// is its ticket and its device data sits at addresses no earlier request
// used: Gamma_j rows are read through the scalar cache, which a running kernel
// never invalidates. The host relaunches the kernel to recycle them.

constexpr uint32_t kNoPlan = 0xffffffffu;

struct ServeReq {                 // one published request (ring entry ticket % ring)
    BatchCode code;               // pointers already into the request's device region
    const uint64_t *src;          // payload in pinned host memory: packed rows, then full rows
    uint64_t *dst;                // the request's device region
    uint64_t words;               // payload length in 64-bit words
    uint32_t plan_copy[2];        // plans whose tables this request copies in (kNoPlan = none)
    uint32_t plan_wait[2];        // plans copied in by an earlier request (kNoPlan = none)
};

struct ServePlanDesc {            // where plan p lives in the plan and rectangle tables
    uint32_t entry_off, levels, rect_off, nrects;
};

// Completion record of one request slot, in pinned host memory; the device writes it
// with system-scope stores and sets flag last.
struct ServeRecord {
    uint32_t flag;                // 1 once every other field is final
    int32_t status;
    uint32_t d, lower_bound, upper_bound, last_level, nstats, _pad;
    uint64_t ticket;
    uint64_t combinations;
    uint64_t t_done;              // device wall clock at completion
    uint64_t witness[kHostWords];
};

struct ServeArgs {
    BatchArgs b;                  // codes / state: one entry per ticket of this launch; ncodes = capacity
    const ServeReq *reqs;         // pinned ring of staged requests
    const ServePlanDesc *plan_desc;   // pinned
    const PlanEntry *host_plans;  // pinned mirror of the plan table
    const Rect *host_rects;       // pinned mirror of the rectangle table
    unsigned int *plan_ready;     // device: nonzero once plan p's tables are copied in
    const unsigned long long *published;   // pinned: tickets below it are staged
    const uint32_t *shutdown;     // pinned: 1 = finish the published requests and leave, 2 = leave now
    ServeRecord *records;         // pinned, one per slot
    BatchStat *host_stats;        // pinned, stats_cap per slot
    unsigned long long *view;     // device: [last poll time, published seen, shutdown seen]
    uint64_t ring;                // entries of reqs, a power of two
    uint32_t stats_cap, _pad;
};

// sv: device memory holding the arguments, unchanged while the kernel runs
hipError_t launch_serve(const ServeArgs *sv, uint32_t grid, bool stats, hipStream_t st);
int serve_blocks_per_cu(bool stats);

// b: the arguments in device memory (read while the kernel runs).
// lds_bytes: the binomial table's LDS (batch_lds_bytes of the args' lds_k, lds_g; 0 = none).
hipError_t launch_batch(const BatchArgs *b, uint32_t grid, bool stats, size_t lds_bytes, hipStream_t st);
hipError_t launch_batch_recover(const BatchArgs &b, hipStream_t st);
int batch_blocks_per_cu(bool stats, size_t lds_bytes);
// LDS bytes of the binomial table C(x, y), x <= k, y <= g.
constexpr size_t batch_lds_bytes(uint32_t k, uint32_t g) { return (size_t)(k + 1) * (g + 1) * sizeof(uint64_t); }
// Largest table staged in LDS: with more the work-groups a CU holds would drop.
constexpr size_t kBatchLdsMax = 24 * 1024;

hipError_t launch_enum(const TaskArgs &a, uint32_t W, uint32_t slots, bool partial, bool stats,
                       uint32_t grid, hipStream_t st);
size_t enum_lds_bytes(uint32_t k, uint32_t g, uint32_t W, uint32_t group = 1);
// A group of tasks spanning levels (full rank, W <= 8, the variant's slots);
// the shared memory is enum_lds_bytes(k, largest g, W, ntasks).
hipError_t launch_enum_levels(const LevelsArgs &a, uint32_t W, uint32_t slots, bool stats, uint32_t grid,
                              hipStream_t st);
hipError_t launch_task_init(unsigned long long *key, unsigned long long *stats,
                            unsigned long long *ncomb, unsigned long long *ctr, hipStream_t st);
// Resets n task records (kRecWords each), writes the window's starting bounds
// and zeroes *clear (the witness flag) when it is set.
hipError_t launch_chain_init(unsigned long long *records, uint32_t n, ChainState *state, const ChainState &init,
                             unsigned int *clear, hipStream_t st);
hipError_t launch_recover(const RecoverArgs &a, hipStream_t st);
// threads: the largest tile (combinations) of the window's tasks; the launch
// takes at most 2048 work-groups of 256 and walks larger tiles in strides.
hipError_t launch_recover_window(const RecoverWindowArgs &a, uint64_t threads, hipStream_t st);

// ---- the paper's prefix-task schedules (bz_sched.hip, bz_sched.h)

// One (Gamma_j, g) task run as prefix tasks dealt to waves. plans[lo] tiles
// the (g - pre)-subsets of rows [lo, k) (unused entries zero); a prefix whose
// last element is c uses plans[c + 1], the empty prefix plans[0]. The task
// key's tile field is task * stride + tile within the prefix's plan.
struct SchedArgs {
    TaskArgs t;                  // rows, binom, key, stats, ncomb, tile_ctr (claims), cancel, k, k_low, g, u_prev, exit_at
    const PlanEntry *plans;      // k + 1 entries
    const Rect *rects;           // every plan's rectangles
    uint64_t ntasks;             // C(k - (g - pre), pre)
    uint64_t stride;             // tiles of the largest suffix plan
    uint32_t pre;                // prefix elements (0: the level is one task)
    uint32_t dist, order;        // kDist*, kOrder* (bz_sched.h)
    uint32_t _pad;
};

hipError_t launch_sched(const SchedArgs &a, uint32_t W, bool partial, bool stats, uint32_t grid, hipStream_t st);
// Work-groups of the schedule kernel one CU holds (its waves are the workers).
int sched_blocks_per_cu(uint32_t W, bool partial, bool stats, size_t lds);

// ---- codewords of a given weight (bz_count_codewords)

struct CollectHit {                // one combination of the target weight
    uint64_t tile, q, h;           // its tile, lane-subset rank and head rank in the tile's rectangle
};

struct CollectArgs {
    const uint32_t *rows;          // (k + 1) x W packed rows of Gamma_j (the last row zero)
    const uint64_t *binom;
    const Rect *rects;
    unsigned long long *ncomb;     // combinations enumerated
    unsigned long long *nhits;     // hits met (may exceed cap)
    CollectHit *hits;
    uint64_t cap, total_tiles;
    uint32_t nrects, k, k_low, g, heads_per_tile, target;
};

// Slots per lane follow slots_for_w(W).
hipError_t launch_collect(const CollectArgs &a, uint32_t W, uint32_t grid, hipStream_t st);

// Issue-rate probe: 16 int32 lane operations per lane per trip.
hipError_t launch_valu_probe(uint32_t iters, uint32_t blocks, uint32_t *sink, hipStream_t st);
int valu_probe_blocks_per_cu();

}  // namespace bz
