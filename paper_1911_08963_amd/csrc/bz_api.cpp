// The C ABI of libbz (include/bz.h): preparation, the level driver of Alg. 1
// (arXiv:1911.08963) for one code, witness recovery, and errors.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <optional>
#include <string>
#include <tuple>
#include <vector>

#include "bz_host.h"
#include "bz_internal.h"
#include "bz_kernels.h"
#include "bz_sched.h"

namespace bz {

thread_local std::string g_err;

bz_status fail(bz_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

static std::mutex g_mu;
static std::map<int, DeviceConst> g_devconst;

std::vector<uint64_t> binom_table() {
    std::vector<uint64_t> tab((size_t)kBinomRows * (kBinomT + 1));
    for (uint32_t x = 0; x < (uint32_t)kBinomRows; ++x)
        for (uint32_t y = 0; y <= (uint32_t)kBinomT; ++y)
            tab[(size_t)x * (kBinomT + 1) + y] = binom_sat(x, y);
    return tab;
}

bz_status device_const(int dev, DeviceConst &out) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_devconst.find(dev);
    if (it != g_devconst.end()) { out = it->second; return BZ_OK; }
    DeviceConst dc;
    BZ_HIP(hipDeviceGetAttribute(&dc.cus, hipDeviceAttributeMultiprocessorCount, dev));
    const std::vector<uint64_t> tab = binom_table();
    BZ_HIP(hipMalloc(&dc.binom, tab.size() * sizeof(uint64_t)));
    BZ_HIP(hipMemcpy(dc.binom, tab.data(), tab.size() * sizeof(uint64_t), hipMemcpyHostToDevice));
    g_devconst[dev] = dc;
    out = dc;
    return BZ_OK;
}

}  // namespace bz

namespace {

using bz::DeviceConst;
using bz::device_const;
using bz::fail;
using bz::g_err;
using bz::now_s;

// Workspace layout of one search (bytes). A window of up to kChainMax tasks
// runs between two host synchronisations; each task has a record of
// kRecWords words (key, counts and claim counter on separate 128-byte lines),
// after the window's bounds (bz::ChainState).
constexpr size_t kWsIndices = 512;     // the witness's row indices: up to 384 u32 before kWsPreRows
constexpr size_t kWsPreRows = 2048;    // a prefix task's rows, up to 64 u32
constexpr size_t kWsRecTasks = 2304;   // a window's tasks for its witness recovery (bz::RecoverTask)
constexpr size_t kWsRects = 4096;
constexpr size_t kMaxRects = 16384;
constexpr uint32_t kChainMax = 32;
constexpr size_t kRecBytes = bz::kRecWords * 8;
constexpr size_t kWsChain = kWsRects + kMaxRects * sizeof(bz::Rect);   // ChainState, then the records
constexpr size_t kChainBytes = 128 + kChainMax * kRecBytes;
// the witness recovery's flag, length (u32) and codeword (4 x u64), in the
// window state's line: a window's one read-back returns them with its records
constexpr size_t kWsRecover = kWsChain + 64;
// Where a one launch of the code's smallest levels writes its state and
// records when they cannot go straight to pinned host memory.
constexpr size_t kWsOne = kWsChain + kChainBytes;
constexpr size_t kOneStatsOff = sizeof(bz::OneState);
constexpr size_t kOneBytes = kOneStatsOff + bz::kOneMaxTasks * sizeof(bz::BatchStat);
constexpr size_t kWsBytes = kWsOne + ((kOneBytes + 255) & ~(size_t)255);
static_assert(sizeof(bz::ChainState) <= 128, "bounds fit their line");
static_assert(sizeof(bz::ChainState) <= 64 && 64 + 8 + bz::kHostWords * sizeof(uint64_t) <= 128,
              "the window state, then the recovery's flag, length and codeword, fit one line");
static_assert(kWsPreRows - kWsIndices >= (size_t)bz::kBinomT * sizeof(uint32_t),
              "the recovered combination's row indices (g <= kBinomT) fit below the prefix rows");
static_assert(kWsRecTasks - kWsPreRows >= 64 * sizeof(uint32_t), "a prefix task's rows fit below the window's tasks");
static_assert(kWsRects - kWsRecTasks >= kChainMax * sizeof(bz::RecoverTask), "a window's tasks fit below the tilings");


// A level's tiling depends on (k, g, lane sums, heads per tile, target tile
// count) only: a process-wide cache keeps it for every later search of the
// same shape (up to kPlanCacheBytes of rectangles; past that, tilings are
// built per search).
constexpr size_t kPlanCacheBytes = 64u << 20;
std::shared_ptr<const bz::LevelPlan> cached_plan(uint32_t k, uint32_t g, uint32_t slots, uint32_t heads,
                                                 uint64_t target, std::string &err) {
    using Key = std::tuple<uint32_t, uint32_t, uint32_t, uint32_t, uint64_t>;
    static std::mutex mu;
    static std::map<Key, std::shared_ptr<const bz::LevelPlan>> cache;
    static size_t bytes = 0;
    const Key key{k, g, slots, heads, target};
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        if (it != cache.end()) return it->second;
    }
    auto p = std::make_shared<bz::LevelPlan>();
    if (!bz::plan_level(k, g, slots, heads, target, *p, err, true)) return nullptr;
    std::lock_guard<std::mutex> lk(mu);
    const size_t b = p->rects.size() * sizeof(bz::Rect);
    if (bytes + b <= kPlanCacheBytes && cache.emplace(key, p).second) bytes += b;
    return p;
}

// Levels of fewer sums than this run their full-rank Gamma_j in one launch
// (up to bz::kMaxGroup of them): their launches are mostly fixed cost, and the
// work a task past the stop still does there is small.
constexpr double kGroupMaxComb = 134217728.0;   // 2^27
// A launch of tasks spanning level ends runs the later levels' tasks with the
// bounds from before the launch, even when an earlier task ends the search:
// their sums together stay below this (about half a millisecond).
constexpr double kSpanMaxComb = 16777216.0;     // 2^24

// Lower bound certified once Gamma_0..Gamma_j are done at level g and the
// later matrices at level g-1 (j == m_f is the partial matrix).
uint32_t certified(uint32_t j, uint32_t g, uint32_t m_f, uint32_t k_m, uint32_t k) {
    if (j >= m_f) {
        int64_t extra = k_m ? (int64_t)g + 1 - k + k_m : 0;
        return m_f * (g + 1) + (uint32_t)std::max<int64_t>(0, extra);
    }
    int64_t extra = k_m ? (int64_t)g - k + k_m : 0;
    return (j + 1) * (g + 1) + (m_f - j - 1) * g + (uint32_t)std::max<int64_t>(0, extra);
}

// Pinned host memory for the read-back of a window and for staging the
// tilings and prefix rows a window uploads (a copy from or into pageable memory
// goes through a staging buffer of the runtime and waits for the stream).
// Buffers are taken from and returned to a process-wide pool and kept until
// the process ends.
constexpr size_t kStageBytes = 64 * 1024;
constexpr size_t kPinnedBytes = kChainBytes + kStageBytes;
// the staging area's tail: a window's tasks for the recovery
constexpr size_t kStageTasksOff = kStageBytes - kChainMax * sizeof(bz::RecoverTask);
static_assert(kOneBytes <= kChainBytes, "a one launch's state and records fit the read-back buffer");
class PinnedWords {
  public:
    PinnedWords() {
        std::lock_guard<std::mutex> lk(mu());
        if (!pool().empty()) {
            p_ = pool().back();
            pool().pop_back();
        } else if (hipHostMalloc((void **)&p_, kPinnedBytes, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            p_ = nullptr;
        }
        if (!p_) fallback_.resize(kPinnedBytes / 8);
    }
    ~PinnedWords() {
        if (!p_) return;
        std::lock_guard<std::mutex> lk(mu());
        pool().push_back(p_);
    }
    unsigned long long *get() { return p_ ? p_ : fallback_.data(); }
    bool pinned() const { return p_ != nullptr; }          // device-accessible (hipHostMalloc)

  private:
    static std::mutex &mu() { static std::mutex m; return m; }
    static std::vector<unsigned long long *> &pool() { static std::vector<unsigned long long *> v; return v; }
    unsigned long long *p_ = nullptr;
    std::vector<unsigned long long> fallback_;
};

struct Best {
    bool have = false;
    uint32_t j = 0, g = 0, slots = 0, ht = 0;
    uint64_t tile = 0;
    bz::Rect rect{};
    std::vector<uint32_t> pre;       // rows of the winning prefix task (schedules 1..8)
};


// ---------------------------------------------------------------- batched search

constexpr uint64_t kBatchMaxComb = 1ull << 50;   // levels with C(k, g) beyond this get no plan
static_assert(kBatchMaxComb <= (1ull << 55), "a task's count at the minimum fits the statistics word's 55 bits");
constexpr uint64_t kBatchTargetTiles = 64;        // tiles per task aimed at by the planner
// Head steps per tile at most. Finer caps cut a large task into more tiles
// and cost more than they balance (4096-code batch kernel, measured: 0.78 s
// at 4096, 0.83 s at 1024, 0.91 s at 512, 1.08 s at 256).
constexpr uint32_t kBatchMaxHeads = 4096;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct BatchLayout {
    std::vector<bz::BatchCode> codes;
    std::vector<bz::CodeState> states;
    std::vector<bz::PlanEntry> plans;
    std::vector<bz::Rect> rects;
    std::vector<unsigned long long> log_init;   // initial task-log entries
    unsigned long long log_tail = 0;             // initial log tail (head and next code start at 0)
    uint32_t done_init = 0, grid = 0, stats_total = 0;
    uint32_t lds_k = 0, lds_g = 0;               // binomial table staged in LDS (0: none)
    size_t lds_bytes = 0;
    uint64_t log_cap = 0;
    size_t off_codes = 0, off_states = 0, off_plans = 0, off_rects = 0, off_stats = 0,
           off_recover = 0, off_log = 0, off_done = 0, off_args = 0, total = 0;
};

bz_status batch_layout(bz_code *const *codes, uint32_t count, const bz_opts &opt, int cus, bool stats,
                       BatchLayout &Lo) {
    Lo = BatchLayout{};
    // plans per (k, slots): (first entry, levels with a plan)
    std::map<std::pair<uint32_t, uint32_t>, std::pair<uint32_t, uint32_t>> plan_of;
    auto plans_for = [&](uint32_t k, uint32_t slots) -> std::pair<uint32_t, uint32_t> {
        auto key = std::make_pair(k, slots);
        auto it = plan_of.find(key);
        if (it != plan_of.end()) return it->second;
        const uint32_t base = (uint32_t)Lo.plans.size();
        const uint32_t tiles = opt.tiles_per_task ? opt.tiles_per_task
                               : (bz::tuned_batch_tiles() ? bz::tuned_batch_tiles() : kBatchTargetTiles);
        const uint32_t gmax = bz::build_level_plans(k, slots, opt.heads_per_tile, tiles, kBatchMaxComb,
                                                    0, Lo.plans, Lo.rects, kBatchMaxHeads);
        return plan_of[key] = {base, gmax};
    };
    for (uint32_t i = 0; i < count; ++i)
        if (!codes[i]) return fail(BZ_EINVAL, "null code in batch");
    for (uint32_t i = 0; i < count; ++i) {
        const bz_code *c = codes[i];
        bz::BatchCode d{};
        d.rows = (const uint32_t *)c->dev;
        d.px_delta = c->px_delta;
        d.full_rows = (const uint64_t *)((const char *)c->dev + c->dev_full_off);
        d.n = c->n; d.k = c->k; d.m_f = c->num_full; d.k_m = c->partial_rank;
        d.nsets = c->nsets; d.W_full = c->W_full; d.W_partial = c->W_partial;
        const auto pf = plans_for(c->k, bz::slots_for_w(c->W_full));
        const auto pp = c->W_partial ? plans_for(c->k, bz::slots_for_w(c->W_partial)) : pf;
        d.plan_full = pf.first;
        d.plan_partial = pp.first;
        d.g_max = std::min(pf.second, pp.second);
        d.stats_off = Lo.stats_total;
        d.stats_cap = c->nsets * std::max<uint32_t>(1, d.g_max);
        d.flags = opt.flags;
        d.max_level = opt.max_level;
        Lo.stats_total += d.stats_cap;
        Lo.codes.push_back(d);
        bz::CodeState S{};
        S.U = c->n - c->k + 1;
        S.L = 1; S.Lcert = 1; S.last_level = 1;
        if (c->k == c->n) {
            S.cursor = (unsigned long long)(bz::kDoneEpoch << bz::kEpochShift);
            S.L = 1; S.U = 1;
            Lo.done_init++;
        } else {
            const bz::PlanEntry &P = Lo.plans[d.plan_full];
            S.cursor = 0;
            bz::TaskSlot &t = S.slot[0];
            t.key = ~0ull; t.stats = ~0ull; t.ncomb = 0; t.completed = 0;
            t.tiles = P.total_tiles;                          // epoch 0
            if (P.total_tiles >= 8) Lo.log_init.push_back(((unsigned long long)i << 24) + 1ull);
            t.j = 0; t.g = 1; t.rect_off = P.rect_off; t.nrects = P.nrects;
            t.heads_per_tile = P.heads_per_tile;
            t.exit_at = stats ? 0u : 1u;
            t.u_prev = S.U;
        }
        Lo.states.push_back(S);
        Lo.log_cap += (uint64_t)d.nsets * std::max<uint32_t>(1, d.g_max) + 1;
    }
    // the lane setup's binomials C(x, y), x < k, y <= g, in each work-group's
    // LDS when the batch's largest table is small enough
    uint32_t kmax = 0, gmax = 0;
    for (const bz::BatchCode &d : Lo.codes) {
        kmax = std::max(kmax, d.k);
        gmax = std::max(gmax, d.g_max);
    }
    if (kmax && gmax && bz::batch_lds_bytes(kmax, gmax) <= bz::kBatchLdsMax) {
        Lo.lds_k = kmax;
        Lo.lds_g = gmax;
        Lo.lds_bytes = bz::batch_lds_bytes(kmax, gmax);
    }
    Lo.grid = (uint32_t)std::max(1, cus * bz::batch_blocks_per_cu(stats, Lo.lds_bytes));
    size_t off = 0;
    Lo.off_codes = off; off = align256(off + count * sizeof(bz::BatchCode));
    Lo.off_states = off; off = align256(off + count * sizeof(bz::CodeState));
    Lo.off_plans = off; off = align256(off + Lo.plans.size() * sizeof(bz::PlanEntry));
    Lo.off_rects = off; off = align256(off + Lo.rects.size() * sizeof(bz::Rect));
    Lo.off_stats = off; off = align256(off + (size_t)Lo.stats_total * sizeof(bz::BatchStat));
    Lo.off_recover = off; off = align256(off + count * sizeof(bz::BatchRecover));
    // the log is a ring indexed with a mask: a power of two at least the entries possible
    uint64_t cap2 = 1;
    while (cap2 < Lo.log_cap) cap2 <<= 1;
    Lo.log_cap = cap2;
    Lo.off_log = off; off = align256(off + (Lo.log_cap + bz::kLogEntries) * sizeof(unsigned long long));
    Lo.off_done = off; off = align256(off + sizeof(uint32_t));
    Lo.off_args = off; off = align256(off + sizeof(bz::BatchArgs));
    Lo.total = std::max(off, kWsBytes);
    return BZ_OK;
}

bz_status batch_run(bz_code *const *codes, uint32_t count, const bz_opts *o, bz_result *res,
                    bz_status *per_code) {
    if (count && (!codes || !res || !per_code)) return fail(BZ_EINVAL, "null argument");
    if (count == 0) return BZ_OK;
    bz_opts opt{};
    if (o) opt = *o;
    if (opt.flags & ~(uint32_t)(BZ_F_STATS | BZ_F_LEVEL_STOP | BZ_F_NO_WITNESS)) return fail(BZ_EINVAL, "unknown flag");
    if (opt.slots_per_lane)
        return fail(BZ_EINVAL, "the batched search chooses slots per lane itself (pass 0)");
    if (opt.schedule != BZ_SCHED_TILES) return fail(BZ_EINVAL, "schedules 1..8 apply to bz_min_distance only");
    const bool stats = opt.flags & BZ_F_STATS;
    const double t0 = now_s();
    for (uint32_t i = 0; i < count; ++i) {
        per_code[i] = BZ_EDEVICE;
        res[i].d = 0; res[i].lower_bound = 0; res[i].upper_bound = 0; res[i].last_level = 0;
        res[i].combinations = 0; res[i].stats_len = 0; res[i].launches = 0;
        res[i].search_s = 0; res[i].kernel_s = 0;
        if (!codes[i]) return fail(BZ_EINVAL, "null code in batch");
        if (!codes[i]->dev) return fail(BZ_EINVAL, "host-only code in batch (BZ_PREPARE_HOST_ONLY)");
        res[i].prepare_s = codes[i]->prepare_s;
        if (codes[i]->device != codes[0]->device) return fail(BZ_EINVAL, "codes of a batch must be on one device");
    }
    const int dev = codes[0]->device;
    if (hipSetDevice(dev) != hipSuccess) return fail(BZ_EDEVICE, "hipSetDevice");
    if (opt.cancel) {
        hipPointerAttribute_t pa;
        if (hipPointerGetAttributes(&pa, (const void *)opt.cancel) != hipSuccess || pa.type != hipMemoryTypeHost) {
            (void)hipGetLastError();
            return fail(BZ_EINVAL, "cancel must point to pinned host memory (hipHostMalloc)");
        }
    }
    DeviceConst dc;
    bz_status s0 = device_const(dev, dc);
    if (s0 != BZ_OK) return s0;
    BatchLayout Lo;
    s0 = batch_layout(codes, count, opt, dc.cus, stats, Lo);
    if (s0 != BZ_OK) return s0;

    char *ws = (char *)opt.workspace;
    bool own_ws = false;
    if (ws) {
        if (opt.workspace_bytes < Lo.total) return fail(BZ_ENOMEM, "workspace smaller than bz_workspace_bytes");
    } else {
        if (hipMalloc((void **)&ws, Lo.total) != hipSuccess) return fail(BZ_ENOMEM, "workspace allocation");
        own_ws = true;
    }
    struct WsGuard {
        char *p; bool own;
        ~WsGuard() { if (own) (void)hipFree(p); }
    } guard{ws, own_ws};

    hipStream_t st = (hipStream_t)opt.hip_stream;
    // uploads (not part of the captured graph)
    const uint32_t done_init = Lo.done_init;
    BZ_HIP(hipMemcpyAsync(ws + Lo.off_codes, Lo.codes.data(), count * sizeof(bz::BatchCode), hipMemcpyHostToDevice, st));
    BZ_HIP(hipMemcpyAsync(ws + Lo.off_states, Lo.states.data(), count * sizeof(bz::CodeState), hipMemcpyHostToDevice, st));
    BZ_HIP(hipMemcpyAsync(ws + Lo.off_plans, Lo.plans.data(), Lo.plans.size() * sizeof(bz::PlanEntry), hipMemcpyHostToDevice, st));
    BZ_HIP(hipMemcpyAsync(ws + Lo.off_rects, Lo.rects.data(), Lo.rects.size() * sizeof(bz::Rect), hipMemcpyHostToDevice, st));
    BZ_HIP(hipMemcpyAsync(ws + Lo.off_done, &done_init, sizeof(uint32_t), hipMemcpyHostToDevice, st));
    BZ_HIP(hipMemsetAsync(ws + Lo.off_recover, 0, count * sizeof(bz::BatchRecover), st));
    // task log: control words (head 0, tail = the initial entries, next code 0), then entries
    BZ_HIP(hipMemsetAsync(ws + Lo.off_log, 0, (Lo.log_cap + bz::kLogEntries) * sizeof(unsigned long long), st));
    Lo.log_tail = Lo.log_init.size();
    BZ_HIP(hipMemcpyAsync(ws + Lo.off_log + bz::kLogTail * sizeof(unsigned long long), &Lo.log_tail,
                          sizeof(Lo.log_tail), hipMemcpyHostToDevice, st));
    if (!Lo.log_init.empty())
        BZ_HIP(hipMemcpyAsync(ws + Lo.off_log + bz::kLogEntries * sizeof(unsigned long long), Lo.log_init.data(),
                              Lo.log_init.size() * sizeof(unsigned long long), hipMemcpyHostToDevice, st));

    bz::BatchArgs b{};
    b.codes = (const bz::BatchCode *)(ws + Lo.off_codes);
    b.state = (bz::CodeState *)(ws + Lo.off_states);
    b.plans = (const bz::PlanEntry *)(ws + Lo.off_plans);
    b.rects = (const bz::Rect *)(ws + Lo.off_rects);
    b.binom = dc.binom;
    b.stats = (bz::BatchStat *)(ws + Lo.off_stats);
    b.recover = (bz::BatchRecover *)(ws + Lo.off_recover);
    unsigned long long *log_base = (unsigned long long *)(ws + Lo.off_log);
    b.log_head = log_base + bz::kLogHead;
    b.log_tail = log_base + bz::kLogTail;
    b.next_code = log_base + bz::kLogNext;
    b.log = log_base + bz::kLogEntries;
    b.log_cap = Lo.log_cap;
    b.done_count = (unsigned int *)(ws + Lo.off_done);
    b.cancel = (const uint32_t *)opt.cancel;
    b.ncodes = count;
    b.lds_k = Lo.lds_k;
    b.lds_g = Lo.lds_g;
    BZ_HIP(hipMemcpyAsync(ws + Lo.off_args, &b, sizeof(b), hipMemcpyHostToDevice, st));

    // one captured graph: the persistent search, then witness recovery
    hipStream_t cs = nullptr;
    hipEvent_t e_ready = nullptr, e_done = nullptr, ev0 = nullptr, ev1 = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    struct GraphGuard {
        hipStream_t &cs; hipEvent_t &a, &b2, &c, &d; hipGraph_t &g; hipGraphExec_t &x;
        ~GraphGuard() {
            if (x) (void)hipGraphExecDestroy(x);
            if (g) (void)hipGraphDestroy(g);
            for (hipEvent_t e : {a, b2, c, d}) if (e) (void)hipEventDestroy(e);
            if (cs) (void)hipStreamDestroy(cs);
        }
    } gg{cs, e_ready, e_done, ev0, ev1, graph, exec};
    BZ_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    BZ_HIP(hipEventCreate(&e_ready));
    BZ_HIP(hipEventCreate(&e_done));
    BZ_HIP(hipEventCreate(&ev0));
    BZ_HIP(hipEventCreate(&ev1));
    BZ_HIP(hipEventRecord(e_ready, st));
    BZ_HIP(hipStreamWaitEvent(cs, e_ready, 0));
    BZ_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    hipError_t le = bz::launch_batch((const bz::BatchArgs *)(ws + Lo.off_args), Lo.grid, stats, Lo.lds_bytes, cs);
    hipError_t lr = (le == hipSuccess && !(opt.flags & BZ_F_NO_WITNESS)) ? bz::launch_batch_recover(b, cs) : hipSuccess;
    hipError_t ec = hipStreamEndCapture(cs, &graph);
    if (le != hipSuccess || lr != hipSuccess || ec != hipSuccess)
        return fail(BZ_EDEVICE, std::string("graph capture: ") + hipGetErrorString(le != hipSuccess ? le : (lr != hipSuccess ? lr : ec)));
    BZ_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    BZ_HIP(hipEventRecord(ev0, cs));
    BZ_HIP(hipGraphLaunch(exec, cs));
    BZ_HIP(hipEventRecord(ev1, cs));
    BZ_HIP(hipEventRecord(e_done, cs));
    BZ_HIP(hipStreamWaitEvent(st, e_done, 0));

    std::vector<bz::CodeState> states(count);
    std::vector<bz::BatchStat> bstats(Lo.stats_total);
    std::vector<bz::BatchRecover> rec(count);
    BZ_HIP(hipMemcpyAsync(states.data(), ws + Lo.off_states, count * sizeof(bz::CodeState), hipMemcpyDeviceToHost, st));
    if (Lo.stats_total)
        BZ_HIP(hipMemcpyAsync(bstats.data(), ws + Lo.off_stats, Lo.stats_total * sizeof(bz::BatchStat), hipMemcpyDeviceToHost, st));
    BZ_HIP(hipMemcpyAsync(rec.data(), ws + Lo.off_recover, count * sizeof(bz::BatchRecover), hipMemcpyDeviceToHost, st));
    BZ_HIP(hipStreamSynchronize(st));
    float ms = 0.f;
    BZ_HIP(hipEventElapsedTime(&ms, ev0, ev1));
    const double wall = now_s() - t0;
    const bool canceled = opt.cancel && *opt.cancel;
    bz_status first = BZ_OK;
    for (uint32_t i = 0; i < count; ++i) {
        const bz::CodeState &S = states[i];
        const bz_code *c = codes[i];
        bz_result &r = res[i];
        r.launches = 1;
        r.kernel_s = ms * 1e-3;
        r.search_s = wall;
        r.lower_bound = S.L; r.upper_bound = S.U; r.last_level = c->k == c->n ? 0 : S.last_level;
        r.combinations = S.combinations;
        r.stats_len = S.nstats;
        bz_status st_i = (bz_status)(int32_t)S.status;
        const bool finished = (S.cursor >> bz::kEpochShift) == bz::kDoneEpoch;
        if (!finished) st_i = canceled ? BZ_ECANCELED : BZ_EDEVICE;
        if (r.stats) {
            const uint32_t n = std::min(S.nstats, std::min(r.stats_cap, Lo.codes[i].stats_cap));
            for (uint32_t t = 0; t < n; ++t) {
                const bz::BatchStat &bs = bstats[Lo.codes[i].stats_off + t];
                r.stats[t].matrix = bs.matrix; r.stats[t].level = bs.level;
                r.stats[t].min_weight = bs.min_weight; r.stats[t].count_at_min = bs.count_at_min;
                r.stats[t].combinations = bs.combinations;
            }
            if (st_i == BZ_OK && S.nstats > std::min(r.stats_cap, Lo.codes[i].stats_cap)) st_i = BZ_ELIMIT;
        }
        if (st_i == BZ_OK && !(opt.flags & BZ_F_NO_WITNESS) && r.witness) {
            if (c->k == c->n) {
                for (uint32_t w = 0; w < (c->n + 63) / 64; ++w) r.witness[w] = c->full_rows[0][w];
            } else if (rec[i].flag == 1) {
                for (uint32_t w = 0; w < (c->n + 63) / 64; ++w) r.witness[w] = rec[i].codeword[w];
            } else {
                st_i = BZ_EDEVICE;
            }
        }
        if (st_i == BZ_OK) r.d = S.U;
        per_code[i] = st_i;
        if (st_i != BZ_OK && first == BZ_OK) {
            first = st_i;
            g_err = std::string("code ") + std::to_string(i) + ": " + bz_status_str(st_i);
        }
    }
    return first;
}

// The task list of a code's smallest levels (C(k, g) <= kOneLaunchComb, at
// most kOneMaxTasks tasks and kOneMaxRects rectangles), in Alg. 1's order,
// with one tiling per (level, lane sums per lane).
bool build_one_launch(bz_code &c, std::vector<bz::Rect> &rects, std::string &err) {
    c.one_tasks.clear();
    c.one_plans.clear();
    c.one_plan_of.clear();
    const uint32_t k = c.k, last_j = c.nsets - 1;
    if (k == c.n) return true;                       // d = 1 without any enumeration
    // The one launch pays off when its levels end the search; otherwise the
    // search waits for it before its first window. It can end the search only if
    // d is at most the bound its last level certifies. Against the weight where a
    // random [n, k] code expects its first nonzero codeword (sum over w' <= w of
    // C(n, w') 2^(k - n) reaches 1), allowing two below: a speed choice only,
    // the result is the same either way. When it does not pay off, no one
    // launch is prepared at all.
    {
        uint32_t g_last = 0;
        for (uint32_t g = 1; g <= k && g <= (uint32_t)bz::kBinomT; ++g) {
            if ((double)bz::binom_sat(k, g) > bz::kOneLaunchComb) break;
            if ((g - 1) * c.nsets + c.nsets > bz::kOneMaxTasks) break;
            g_last = g;
        }
        if (g_last == 0) return true;
        double acc = 0.0;
        uint32_t w_est = 0;
        while (w_est < c.n && acc < 1.0) {
            ++w_est;
            acc += std::exp(std::lgamma((double)c.n + 1) - std::lgamma((double)w_est + 1) -
                            std::lgamma((double)(c.n - w_est) + 1) + ((double)k - (double)c.n) * std::log(2.0));
        }
        c.one_likely = certified(last_j, g_last, c.num_full, c.partial_rank, k) + 2 >= w_est;
        if (!c.one_likely) return true;
    }
    std::map<std::pair<uint32_t, uint32_t>, uint32_t> plan_index;   // (g, slots) -> index in one_plans
    for (uint32_t g = 1; g <= k && g <= (uint32_t)bz::kBinomT; ++g) {
        if ((double)bz::binom_sat(k, g) > bz::kOneLaunchComb) break;
        if (c.one_tasks.size() + c.nsets > bz::kOneMaxTasks) break;
        const size_t tasks_before = c.one_tasks.size(), plans_before = c.one_plans.size(),
                     rects_before = rects.size();
        std::vector<uint32_t> rect_of_plan;
        for (uint32_t j = 0; j < c.nsets; ++j) {
            const uint32_t W = c.W(j), slots = bz::slots_for_w(W);
            const auto key = std::make_pair(g, slots);
            if (!plan_index.count(key)) {
                bz::LevelPlan p;
                if (!bz::plan_level(k, g, slots, 0, bz::kOneTargetTiles, p, err)) return false;
                plan_index[key] = (uint32_t)c.one_plans.size();
                c.one_plans.push_back(std::move(p));
            }
            const uint32_t pi = plan_index[key];
            const bz::LevelPlan &p = c.one_plans[pi];
            bz::OneTask T{};
            T.total_tiles = p.total_tiles;
            T.comb = bz::binom_sat(k, g);
            T.j = j; T.g = g;
            T.nrects = (uint32_t)p.rects.size();
            T.heads_per_tile = p.heads_per_tile;
            T.W = W;
            T.row_off = (uint32_t)c.packed_off[j];
            T.cert_task = certified(j, g, c.num_full, c.partial_rank, k);
            T.cert_level = certified(last_j, g, c.num_full, c.partial_rank, k);
            T.last_of_level = j == last_j;
            c.one_tasks.push_back(T);
            c.one_plan_of.push_back(pi);
        }
        // rectangles of the plans this level added (earlier plans are already placed)
        for (size_t pi = plans_before; pi < c.one_plans.size(); ++pi)
            rects.insert(rects.end(), c.one_plans[pi].rects.begin(), c.one_plans[pi].rects.end());
        if (rects.size() > bz::kOneMaxRects) {
            // this level's tilings do not fit: it goes to the per-task launches
            c.one_tasks.resize(tasks_before);
            c.one_plan_of.resize(tasks_before);
            for (auto it = plan_index.begin(); it != plan_index.end();)
                it = it->second >= plans_before ? plan_index.erase(it) : std::next(it);
            c.one_plans.resize(plans_before);
            rects.resize(rects_before);
            break;
        }
    }
    // each task's first rectangle: the plans' rectangles are concatenated in order
    std::vector<uint32_t> first(c.one_plans.size(), 0);
    for (size_t pi = 1; pi < c.one_plans.size(); ++pi) first[pi] = first[pi - 1] + (uint32_t)c.one_plans[pi - 1].rects.size();
    for (size_t t = 0; t < c.one_tasks.size(); ++t) c.one_tasks[t].rect_off = first[c.one_plan_of[t]];
    return true;
}

}  // namespace

extern "C" {

const char *bz_status_str(bz_status s) {
    switch (s) {
    case BZ_OK: return "ok";
    case BZ_EINVAL: return "invalid argument";
    case BZ_ERANK: return "generator matrix rank < k";
    case BZ_ENOMEM: return "out of memory";
    case BZ_EDEVICE: return "device error";
    case BZ_ELIMIT: return "limit reached";
    case BZ_ECANCELED: return "canceled";
    case BZ_EBUSY: return "busy";
    }
    return "unknown status";
}

const char *bz_last_error(void) { return g_err.c_str(); }

bz_status bz_prepare(const uint64_t *G, uint32_t k, uint32_t n, uint32_t ld_words,
                     const bz_prepare_opts *opts, bz_code **out) {
    if (!out) return fail(BZ_EINVAL, "out is null");
    *out = nullptr;
    double t0 = now_s();
    std::unique_ptr<bz_code> c(new (std::nothrow) bz_code());
    if (!c) return fail(BZ_ENOMEM, "host allocation");
    std::string err;
    bz_status st = bz::prepare_host(G, k, n, ld_words, opts, *c, err);
    if (st != BZ_OK) return fail(st, err);
    const bool host_only = opts && (opts->flags & BZ_PREPARE_HOST_ONLY);
    if (host_only) {
        // no device needed: a server copies Gamma_j from the host copy
        if (hipGetDevice(&c->device) != hipSuccess) {
            (void)hipGetLastError();
            c->device = -1;
        }
    } else {
        BZ_HIP(hipGetDevice(&c->device));
    }
    // device layout: per matrix (k + 1) x W dwords (the last row zero); then
    // the same again holding prefix XORs (entry i of matrix j: the XOR of its
    // rows 0..i-1, for the lane setup's successor steps); then the full rows
    // at a 256-byte boundary
    std::vector<uint32_t> dev_packed;
    std::vector<size_t> dev_off;
    for (uint32_t j = 0; j < c->nsets; ++j) {
        dev_off.push_back(dev_packed.size());
        const uint32_t W = c->W(j);
        dev_packed.insert(dev_packed.end(), c->packed.begin() + c->packed_off[j],
                          c->packed.begin() + c->packed_off[j] + (size_t)k * W);
        dev_packed.insert(dev_packed.end(), W, 0u);
    }
    c->px_delta = (uint32_t)dev_packed.size();
    for (uint32_t j = 0; j < c->nsets; ++j) {
        const uint32_t W = c->W(j);
        const size_t base = dev_packed.size();
        dev_packed.insert(dev_packed.end(), (size_t)(k + 1) * W, 0u);
        for (uint32_t i = 0; i < k; ++i)
            for (uint32_t w = 0; w < W; ++w)
                dev_packed[base + (size_t)(i + 1) * W + w] =
                    dev_packed[base + (size_t)i * W + w] ^ dev_packed[dev_off[j] + (size_t)i * W + w];
    }
    c->packed_off = dev_off;
    c->packed = dev_packed;
    size_t pbytes = (dev_packed.size() * sizeof(uint32_t) + 255) & ~(size_t)255;
    c->dev_full_off = pbytes;
    c->dev_bytes = pbytes + c->full_rows.size() * sizeof(bz::HostRow);
    if (host_only) {
        c->prepare_s = now_s() - t0;
        *out = c.release();
        return BZ_OK;
    }
    // the smallest levels' one launch: arguments, task list and tilings after the rows
    DeviceConst dc;
    st = device_const(c->device, dc);
    if (st != BZ_OK) return st;
    std::vector<bz::Rect> one_rects;
    {
        std::string err;
        if (!build_one_launch(*c, one_rects, err)) return fail(BZ_ELIMIT, err);
    }
    size_t one_bytes = 0;
    if (!c->one_tasks.empty()) {
        c->dev_one_off = (c->dev_bytes + 255) & ~(size_t)255;
        one_bytes = 256 + c->one_tasks.size() * sizeof(bz::OneTask) + one_rects.size() * sizeof(bz::Rect);
        c->dev_bytes = c->dev_one_off + one_bytes;
    }
    if (hipMalloc(&c->dev, c->dev_bytes) != hipSuccess) return fail(BZ_ENOMEM, "device allocation for Gamma_j");
    // one upload of the whole layout, from pinned memory when it fits (a copy
    // from pageable memory goes through the runtime's staging buffer)
    PinnedWords pinned;
    std::vector<char> pageable;
    char *img = (char *)pinned.get();
    if (c->dev_bytes > kPinnedBytes) {
        pageable.resize(c->dev_bytes);
        img = pageable.data();
    }
    std::memset(img, 0, pbytes);
    std::memcpy(img, dev_packed.data(), dev_packed.size() * sizeof(uint32_t));
    std::memcpy(img + pbytes, c->full_rows.data(), c->full_rows.size() * sizeof(bz::HostRow));
    if (one_bytes) {
        char *o = img + c->dev_one_off;
        char *dbase = (char *)c->dev + c->dev_one_off;
        std::memset(o, 0, 256);
        bz::OneArgs oa{};
        oa.tasks = (const bz::OneTask *)(dbase + 256);
        oa.rows = (const uint32_t *)c->dev;
        oa.full_rows = (const uint64_t *)((const char *)c->dev + c->dev_full_off);
        oa.rects = (const bz::Rect *)(dbase + 256 + c->one_tasks.size() * sizeof(bz::OneTask));
        oa.binom = dc.binom;
        oa.ntasks = (uint32_t)c->one_tasks.size();
        oa.k = k; oa.k_m = c->partial_rank; oa.m_f = c->num_full;
        oa.U0 = n - k + 1;
        oa.row_words = (uint32_t)dev_packed.size();
        oa.px_delta = c->px_delta;
        const uint32_t glast = c->one_tasks.back().g;
        c->one_lds = ((size_t)oa.row_words * 4 + 7) & ~(size_t)7;
        if (bz::batch_lds_bytes(k, glast) <= 32 * 1024) {
            oa.lds_g = glast;
            c->one_lds += bz::batch_lds_bytes(k, glast);
            c->one_lds_binom = true;
        }
        static_assert(sizeof(bz::OneArgs) <= 256, "the one launch's arguments fit their slot");
        std::memcpy(o, &oa, sizeof(oa));
        std::memcpy(o + 256, c->one_tasks.data(), c->one_tasks.size() * sizeof(bz::OneTask));
        std::memcpy(o + 256 + c->one_tasks.size() * sizeof(bz::OneTask), one_rects.data(),
                    one_rects.size() * sizeof(bz::Rect));
    }
    if (hipMemcpy(c->dev, img, c->dev_bytes, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(c->dev);
        return fail(BZ_EDEVICE, "upload of Gamma_j");
    }
    c->prepare_s = now_s() - t0;
    *out = c.release();
    return BZ_OK;
}

bz_status bz_code_get_info(const bz_code *c, bz_code_info *out, int32_t *set_of_column) {
    if (!c || !out) return fail(BZ_EINVAL, "null argument");
    out->n = c->n; out->k = c->k; out->num_full = c->num_full; out->partial_rank = c->partial_rank;
    out->W_full = c->W_full; out->W_partial = c->W_partial;
    if (set_of_column) std::memcpy(set_of_column, c->set_of_column.data(), c->n * sizeof(int32_t));
    return BZ_OK;
}

bz_status bz_code_get_gamma(const bz_code *c, uint32_t matrix, uint64_t *rows, uint32_t ld_words) {
    if (!c || !rows || matrix >= c->nsets || ld_words < (c->n + 63) / 64) return fail(BZ_EINVAL, "bad argument");
    for (uint32_t i = 0; i < c->k; ++i)
        for (uint32_t w = 0; w < ld_words; ++w)
            rows[(size_t)i * ld_words + w] = w < (uint32_t)bz::kHostWords ? c->full_rows[(size_t)matrix * c->k + i][w] : 0;
    return BZ_OK;
}

void bz_free(bz_code *c) {
    if (!c) return;
    if (c->dev) (void)hipFree(c->dev);
    delete c;
}

bz_status bz_workspace_bytes(bz_code *const *codes, uint32_t count, const bz_opts *o, size_t *bytes) {
    if (!bytes || (count && !codes)) return fail(BZ_EINVAL, "null argument");
    *bytes = kWsBytes;
    if (count == 0) return BZ_OK;
    bz_opts opt{};
    if (o) opt = *o;
    if (!codes[0]) return fail(BZ_EINVAL, "null code");
    if (hipSetDevice(codes[0]->device) != hipSuccess) return fail(BZ_EDEVICE, "hipSetDevice");
    DeviceConst dc;
    bz_status s0 = device_const(codes[0]->device, dc);
    if (s0 != BZ_OK) return s0;
    BatchLayout Lo;
    s0 = batch_layout(codes, count, opt, dc.cus, (opt.flags & BZ_F_STATS) != 0, Lo);
    if (s0 != BZ_OK) return s0;
    *bytes = Lo.total;
    return BZ_OK;
}

}  // extern "C"

namespace {

// What a search that allocates nothing works with instead of the library's
// allocations: the binomial table and the workspace inside the device scratch
// array, host memory set aside for the read-backs, and no timing events.
struct NoAllocEnv {
    DeviceConst dc;
    char *ws = nullptr;
    unsigned long long *host = nullptr;   // kPinnedBytes of host memory
};

bz_status min_distance_impl(bz_code *c, const bz_opts *o, bz_result *res, const NoAllocEnv *na) {
    if (!c || !res) return fail(BZ_EINVAL, "null argument");
    if (!c->dev) return fail(BZ_EINVAL, "code prepared host-only (BZ_PREPARE_HOST_ONLY): submit it to a server");
    bz_opts opt{};
    if (o) opt = *o;
    res->d = 0; res->lower_bound = 0; res->upper_bound = 0; res->last_level = 0;
    res->combinations = 0; res->stats_len = 0; res->launches = 0;
    res->prepare_s = c->prepare_s; res->search_s = 0; res->kernel_s = 0;
    if (opt.flags & ~(uint32_t)(BZ_F_STATS | BZ_F_LEVEL_STOP | BZ_F_NO_WITNESS | BZ_F_TASK_LAUNCHES))
        return fail(BZ_EINVAL, "unknown flag");
    if (opt.slots_per_lane && opt.slots_per_lane != 2 && opt.slots_per_lane != 4 && opt.slots_per_lane != 8 &&
        opt.slots_per_lane != 16)
        return fail(BZ_EINVAL, "slots_per_lane must be 0, 2, 4, 8 or 16");
    const bool use_sched = opt.schedule != BZ_SCHED_TILES;
    uint32_t sched_dist = 0, sched_order = 0;
    bool sched_dynamic = false;
    if (use_sched) {
        if (!bz::sched_parts(opt.schedule, sched_dist, sched_order, sched_dynamic))
            return fail(BZ_EINVAL, "schedule must be 0..8");
        if (opt.prefix == 0) return fail(BZ_EINVAL, "schedules 1..8 need a prefix size >= 1");
    }
    const bool stats = opt.flags & BZ_F_STATS, level_stop = opt.flags & BZ_F_LEVEL_STOP;
    const bool want_witness = !(opt.flags & BZ_F_NO_WITNESS) && res->witness;
    const uint32_t n = c->n, k = c->k, m_f = c->num_full, k_m = c->partial_rank;
    const double t0 = now_s();

    if (hipSetDevice(c->device) != hipSuccess) return fail(BZ_EDEVICE, "hipSetDevice");
    if (opt.cancel) {
        // the kernels read the cancel word: it must be host memory the device can map
        hipPointerAttribute_t pa;
        if (hipPointerGetAttributes(&pa, (const void *)opt.cancel) != hipSuccess ||
            pa.type != hipMemoryTypeHost) {
            (void)hipGetLastError();
            return fail(BZ_EINVAL, "cancel must point to pinned host memory (hipHostMalloc)");
        }
    }
    hipStream_t st = (hipStream_t)opt.hip_stream;
    DeviceConst dc;
    if (na) {
        dc = na->dc;
    } else {
        bz_status s0 = device_const(c->device, dc);
        if (s0 != BZ_OK) return s0;
    }

    char *ws = na ? na->ws : (char *)opt.workspace;
    bool own_ws = false;
    if (na) {
        // the scratch array holds the workspace (checked when the library is built)
    } else if (ws) {
        if (opt.workspace_bytes < kWsBytes) return fail(BZ_ENOMEM, "workspace smaller than bz_workspace_bytes");
    } else {
        if (hipMalloc((void **)&ws, kWsBytes) != hipSuccess) return fail(BZ_ENOMEM, "workspace allocation");
        own_ws = true;
    }
    struct WsGuard {
        char *p; bool own;
        ~WsGuard() { if (own) (void)hipFree(p); }
    } guard{ws, own_ws};

    auto *d_state = (bz::ChainState *)(ws + kWsChain);
    auto *d_records = (unsigned long long *)(ws + kWsChain + 128);
    auto *d_rects = (bz::Rect *)(ws + kWsRects);

    // Timing events, created once per thread and device (a search on one
    // thread runs at a time) and kept until the process ends. A search that
    // allocates nothing is not timed.
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (!na) {
        thread_local std::map<int, std::pair<hipEvent_t, hipEvent_t>> t_events;
        auto evit = t_events.find(c->device);
        if (evit == t_events.end()) {
            hipEvent_t e0 = nullptr, e1 = nullptr;
            BZ_HIP(hipEventCreate(&e0));
            if (hipEventCreate(&e1) != hipSuccess) {
                (void)hipEventDestroy(e0);
                return fail(BZ_EDEVICE, "hipEventCreate");
            }
            evit = t_events.emplace(c->device, std::make_pair(e0, e1)).first;
        }
        ev0 = evit->second.first;
        ev1 = evit->second.second;
    }

    uint32_t U = n - k + 1, L = 1, Lcert = 1;
    Best best;
    bz_status status = BZ_OK;
    if (k == n) {
        // the loop of Alg. 1 never runs; any row of Gamma_1 has weight 1
        res->d = 1; res->lower_bound = 1; res->upper_bound = 1;
        if (want_witness)
            for (uint32_t w = 0; w < (n + 63) / 64; ++w) res->witness[w] = c->full_rows[0][w];
        res->search_s = now_s() - t0;
        return BZ_OK;
    }

    using PlanKey = std::tuple<uint32_t, uint32_t, uint32_t>;                  // (g, slots, tiles/wave)
    std::map<PlanKey, std::shared_ptr<const bz::LevelPlan>> plans;
    // Tilings already on the device (rect offset in the workspace): a level's
    // tiling is uploaded once for all its Gamma_j. When the region is full it
    // starts over at a window's start; every earlier launch has finished by then.
    std::map<PlanKey, size_t> on_device;
    size_t rects_used = 0;
    std::optional<PinnedWords> pinned;
    if (!na) pinned.emplace();
    unsigned long long *words = na ? na->host : pinned->get();   // read-back of a window
    char *stage = (char *)words + kChainBytes;             // uploads of a window
    std::map<std::pair<uint32_t, uint32_t>, bz::SchedPlan> splans;            // (g, slots) -> prefix tasks
    struct DevBuf {
        char *p = nullptr;
        size_t cap = 0;
        ~DevBuf() { if (p) (void)hipFree(p); }
    } sbuf;                                                                    // schedule tilings
    const uint64_t resident_waves = (uint64_t)dc.cus * 32;
    const uint32_t last_j = c->nsets - 1;
    // Alg. 1's L once every matrix is done at level g
    auto level_bound = [&](uint32_t g) { return certified(last_j, g, m_f, k_m, k); };

    struct Task {
        uint32_t j, g, W, slots;
        const bz::LevelPlan *plan;       // equal-cost tiles, or
        const bz::SchedPlan *sp;         // the paper's prefix tasks
        PlanKey key;
    };
    auto make_task = [&](uint32_t j, uint32_t g, Task &t) -> bz_status {
        t = Task{};
        t.j = j; t.g = g; t.W = c->W(j);
        uint32_t slots = opt.slots_per_lane ? opt.slots_per_lane : bz::slots_for_w(t.W);
        uint32_t per_wave = bz::kFixedTilesPerWave;     // tiles per resident wave
        if (!opt.slots_per_lane && !opt.heads_per_tile) {
            (void)bz::tuned_choice(t.W, slots, per_wave);
            const double comb = (double)bz::binom_sat(k, g);
            if (comb < bz::kLargeLevelComb) per_wave = 1;
            if (comb < bz::kTinyLevelComb) slots = 2;
            else if (comb < bz::kSmallLevelComb) slots = std::min(slots, 8u);
        }
        if (slots == 16 && t.W > 4) return fail(BZ_EINVAL, "16 slots per lane need W <= 4");
        if (stats && bz::binom_sat(k, g) >= (1ull << 55))
            return fail(BZ_ELIMIT, "statistics mode keeps a task's count in 55 bits: C(k, g) >= 2^55");
        if (use_sched) {
            slots = bz::slots_for_w(t.W);               // the schedule kernel's fixed lane sums
            auto skey = std::make_pair(g, slots);
            if (!splans.count(skey)) {
                std::string err;
                bz::SchedPlan p;
                if (!bz::build_sched_plan(k, g, sched_dynamic, opt.prefix, slots, p, err)) return fail(BZ_ELIMIT, err);
                splans[skey] = std::move(p);
            }
            t.sp = &splans[skey];
        } else {
            t.key = std::make_tuple(g, slots, per_wave);
            if (!plans.count(t.key)) {
                std::string err;
                auto p = cached_plan(k, g, slots, opt.heads_per_tile, per_wave * resident_waves, err);
                if (!p) return fail(BZ_ELIMIT, err);
                if (p->rects.size() > kMaxRects) return fail(BZ_ELIMIT, "a level's tiling needs more than the workspace's 16384 rectangles");
                plans[t.key] = std::move(p);
            }
            t.plan = plans[t.key].get();
        }
        t.slots = slots;
        return BZ_OK;
    };

    // Tasks run in windows: the host enqueues several (Gamma_j, g) tasks with a
    // one-thread bookkeeping step after each (bz::ChainState), synchronises
    // once, then replays Alg. 1's bookkeeping on the read-back records. A
    // window ends at the task after which the bounds known when it starts
    // would already stop the search; tasks enqueued past the point where the
    // device stops (U fell within the window) leave at once. Such a task costs
    // a launch that returns at its first instruction (a few microseconds); a
    // window's synchronisation, read-back and replay cost several times more,
    // so windows start at 16 tasks and double up to kChainMax. Schedule tasks
    // run one per window.
    uint32_t next_g = 1, next_j = 0;         // the next task in Alg. 1's order
    uint32_t window = 16;
    bool done = false;
    bool finished_in_one = false;            // the one launch ended the search (witness included)
    bool witness_done = false;               // a window recovered the witness on the device
    std::vector<Task> win;
    std::vector<bz::Rect> staged;
    // ---- the smallest levels in one work-group (bz_one_kernel)
    // bz_prepare listed the tasks of the levels of at most kOneLaunchComb sums
    // and uploaded them with their tilings: one launch of a single work-group
    // runs them (it goes from task to task itself) and writes a record per task
    // and its final state straight into pinned host memory; the host replays the
    // same bookkeeping on the records. A search that is not over by then goes on
    // with windows of per-task launches below.
    uint32_t one_run = 0;
    if (!use_sched && !(opt.flags & BZ_F_TASK_LAUNCHES) && c->one_likely)
        for (const bz::OneTask &T : c->one_tasks)
            if (!opt.max_level || T.g <= opt.max_level) one_run++;
    if (one_run) {
        bz::OneRun run{};
        // pinned read-back memory takes the device's stores directly; the
        // search that allocates nothing reads back from its scratch instead
        const bool direct = !na && pinned->pinned();
        char *out = direct ? (char *)words : ws + kWsOne;
        run.state = (bz::OneState *)out;
        run.stats = (bz::BatchStat *)(out + kOneStatsOff);
        run.cancel = (const uint32_t *)opt.cancel;
        run.ntasks = one_run;
        run.level_stop = level_stop;
        run.want_witness = want_witness;
        if (ev0) BZ_HIP(hipEventRecord(ev0, st));
        BZ_HIP(bz::launch_one((const bz::OneArgs *)((const char *)c->dev + c->dev_one_off), run, stats,
                              c->one_lds_binom, c->one_lds, st));
        if (ev1) BZ_HIP(hipEventRecord(ev1, st));
        if (!direct)
            BZ_HIP(hipMemcpyAsync(words, out, kOneStatsOff + one_run * sizeof(bz::BatchStat), hipMemcpyDeviceToHost,
                                  st));
        BZ_HIP(hipStreamSynchronize(st));
        if (ev0) {
            float ms = 0.f;
            BZ_HIP(hipEventElapsedTime(&ms, ev0, ev1));
            res->kernel_s += ms * 1e-3;
        }
        const auto *sd = (const bz::OneState *)words;
        const auto *rec = (const bz::BatchStat *)((const char *)words + kOneStatsOff);
        const uint32_t nrun = sd->ntasks;
        if (nrun > one_run) return fail(BZ_EDEVICE, "internal: one launch ran more tasks than listed");
        // Alg. 1's bookkeeping replayed on the records (the host is the authority)
        bool stop = false;
        int64_t best_i = -1;                                       // the winning task, if in this launch
        for (uint32_t i = 0; i < nrun && !stop; ++i) {
            const bz::OneTask &T = c->one_tasks[i];
            const bz::BatchStat &r = rec[i];
            if (r.matrix != T.j || r.level != T.g) return fail(BZ_EDEVICE, "internal: one launch's record order");
            const uint32_t j = T.j, g = T.g, tmin = r.min_weight;
            res->last_level = g;
            res->launches++;
            res->combinations += r.combinations;
            if (res->stats && res->stats_len < res->stats_cap) {
                bz_level_stat &s = res->stats[res->stats_len];
                s.matrix = (uint16_t)j; s.level = (uint16_t)g; s.min_weight = tmin;
                s.count_at_min = r.count_at_min;
                s.combinations = r.combinations;
            }
            res->stats_len++;
            if (tmin < U || (tmin == U && !best.have)) {
                U = tmin;
                best.have = true;
                best_i = i;
            }
            next_j = j == last_j ? 0 : j + 1;
            next_g = j == last_j ? g + 1 : g;
            if (r.combinations != T.comb) {
                if (U > Lcert) return fail(BZ_EDEVICE, "internal: task ended early without a certificate");
                L = std::max(L, Lcert);
                stop = true;
                break;
            }
            Lcert = std::max(Lcert, T.cert_task);
            if (!level_stop) {
                L = std::max(L, Lcert);
                if (L >= U) stop = true;
            }
            if (!stop && T.last_of_level) {
                L = std::max(L, T.cert_level);
                if (L >= U || g == k) stop = true;
            }
        }
        if (best_i >= 0) {
            // the winning tile as the device recorded it, and its rectangle
            if ((uint32_t)best_i != sd->best_task) return fail(BZ_EDEVICE, "internal: one launch's winning task");
            const bz::OneTask &T = c->one_tasks[best_i];
            const bz::LevelPlan &p = c->one_plans[c->one_plan_of[best_i]];
            best.j = T.j; best.g = T.g; best.tile = sd->best_tile;
            best.slots = bz::slots_for_w(T.W);
            best.ht = p.heads_per_tile;
            best.pre.clear();
            size_t lo = 0, hi = p.rects.size() - 1;
            while (lo < hi) {
                size_t mid = (lo + hi + 1) / 2;
                if (p.rects[mid].tile_begin <= best.tile) lo = mid; else hi = mid - 1;
            }
            best.rect = p.rects[lo];
        }
        const uint32_t dev_status = sd->status;
        if (dev_status == bz::kOneCanceled || dev_status == bz::kOneRunning) {
            // the work-group left before its end: only the cancel word does that
            if (dev_status == bz::kOneRunning || !(opt.cancel && *opt.cancel))
                return fail(BZ_EDEVICE, "internal: one launch left early");
            status = BZ_ECANCELED;
            g_err = "canceled";
            done = true;
        } else {
            const bool dev_stop = dev_status == bz::kOneStopped;
            if (dev_stop != stop || sd->U != U || sd->L != L || sd->Lcert != Lcert)
                return fail(BZ_EDEVICE, "internal: device and host bookkeeping disagree (one launch)");
            if (stop) {
                done = true;
                finished_in_one = true;
                if (want_witness) {
                    if (sd->wit_flag != 1) return fail(BZ_EDEVICE, "internal: witness not found in its tile");
                    for (uint32_t w = 0; w < (n + 63) / 64; ++w) res->witness[w] = sd->witness[w];
                }
            }
        }
    }
    while (!done) {
        if (next_j == 0) {
            if (next_g > k || L >= U) break;
            if (opt.max_level && next_g > opt.max_level) { status = BZ_ELIMIT; g_err = "max_level reached"; break; }
        }
        if (opt.cancel && *opt.cancel) { status = BZ_ECANCELED; g_err = "canceled"; break; }
        win.clear();
        staged.clear();
        std::vector<std::pair<PlanKey, size_t>> placed;                         // tilings staged for this window
        {
            uint32_t g = next_g, j = next_j, Lw = L, Lc = Lcert;
            const uint32_t cap = use_sched ? 1u : window;
            // a level small enough for its tasks to share a launch is not split
            // across windows (up to the records' kChainMax)
            auto more = [&]() {
                if (win.size() < cap) return true;
                return !use_sched && j != 0 && win.size() < kChainMax &&
                       (double)bz::binom_sat(k, g) < kGroupMaxComb;
            };
            while (more() && g <= k && !(opt.max_level && g > opt.max_level)) {
                Task t;
                const bz_status e = make_task(j, g, t);
                if (e != BZ_OK) return e;
                if (t.plan && !on_device.count(t.key)) {
                    bool staged_now = false;
                    for (auto &pl : placed) staged_now = staged_now || pl.first == t.key;
                    if (!staged_now) {
                        if (rects_used + t.plan->rects.size() > kMaxRects) {
                            if (!win.empty()) break;                             // next window
                            on_device.clear();
                            rects_used = 0;
                        }
                        placed.emplace_back(t.key, rects_used);
                        staged.insert(staged.end(), t.plan->rects.begin(), t.plan->rects.end());
                        rects_used += t.plan->rects.size();
                    }
                }
                win.push_back(t);
                Lc = std::max(Lc, certified(j, g, m_f, k_m, k));
                bool stop = false;
                if (!level_stop) {
                    Lw = std::max(Lw, Lc);
                    stop = Lw >= U;
                }
                if (j == last_j) {
                    Lw = std::max(Lw, level_bound(g));
                    stop = stop || Lw >= U;
                    j = 0;
                    ++g;
                } else {
                    ++j;
                }
                if (stop) break;
            }
            window = std::min(window * 2, kChainMax);
        }
        if (win.empty()) return fail(BZ_EDEVICE, "internal: empty window");
        if (!staged.empty()) {
            const size_t off = placed.front().second, bytes = staged.size() * sizeof(bz::Rect);
            const void *src = staged.data();
            if (bytes <= kStageTasksOff) {              // the previous window's copies have finished
                std::memcpy(stage, staged.data(), bytes);
                src = stage;
            }
            BZ_HIP(hipMemcpyAsync(d_rects + off, src, bytes, hipMemcpyHostToDevice, st));
            for (auto &pl : placed) on_device[pl.first] = pl.second;
        }
        bz::ChainState init{};
        init.U = U;
        init.exit_at = stats ? 0u : Lcert;
        init.L = L;
        init.Lcert = Lcert;
        // an enumeration window recovers its witness on the device when it
        // ends the search: no further synchronisation after the read-back
        const bool dev_recover = want_witness && !use_sched;
        uint64_t rec_threads = 0;
        if (dev_recover) {
            auto *rtasks = (bz::RecoverTask *)(stage + kStageTasksOff);
            for (size_t i = 0; i < win.size(); ++i) {
                const Task &t = win[i];
                bz::RecoverTask &rt = rtasks[i];
                rt = bz::RecoverTask{};
                rt.rows = (const uint32_t *)c->dev + c->packed_off[t.j];
                rt.full_rows = (const uint64_t *)((char *)c->dev + c->dev_full_off) + (size_t)t.j * k * bz::kHostWords;
                rt.rects = d_rects + on_device.at(t.key);
                rt.nrects = (uint32_t)t.plan->rects.size();
                rt.slots = t.slots;
                rt.heads_per_tile = t.plan->heads_per_tile;
                rt.W = t.W;
                rt.k_low = c->k_low(t.j);
                uint32_t mult = 1;
                for (const bz::Rect &r : t.plan->rects) mult = std::max(mult, r.lane_mult);
                rec_threads = std::max<uint64_t>(rec_threads,
                                                 (uint64_t)bz::kWaveSize * t.slots * mult * t.plan->heads_per_tile);
            }
            BZ_HIP(hipMemcpyAsync(ws + kWsRecTasks, rtasks, win.size() * sizeof(bz::RecoverTask),
                                  hipMemcpyHostToDevice, st));
        }
        BZ_HIP(bz::launch_chain_init(d_records, (uint32_t)win.size(), d_state, init,
                                     want_witness ? (unsigned int *)(ws + kWsRecover) : nullptr, st));
        const uint32_t U_start = U;
        const bool have_start = best.have;
        for (size_t i = 0; i < win.size(); ++i) {
            const Task &t = win[i];
            unsigned long long *rec = d_records + i * bz::kRecWords;
            // consecutive full-rank tasks of small levels that run the same
            // kernel variant share one launch: up to kMaxLevelTasks when they
            // span a level's end, else up to kMaxGroup of the one level
            const bool grouping = !(opt.flags & BZ_F_TASK_LAUNCHES);
            auto groupable = [&](const Task &u) {
                return !u.sp && u.j < m_f && (double)bz::binom_sat(k, u.g) < kGroupMaxComb && u.W == t.W &&
                       u.slots == t.slots;
            };
            uint32_t span = 1, gmax = t.g;
            double later = 0;                    // sums of the tasks past the first task's level
            if (grouping && groupable(t))
                while (span < bz::kMaxLevelTasks && i + span < win.size() && groupable(win[i + span]) &&
                       bz::enum_lds_bytes(k, std::max(gmax, win[i + span].g), t.W, span + 1) <= 65536) {
                    const Task &u = win[i + span];
                    if (u.g != t.g) {
                        later += (double)bz::binom_sat(k, u.g);
                        if (later > kSpanMaxComb) break;
                    }
                    gmax = std::max(gmax, u.g);
                    ++span;
                }
            if (span > 1 && win[i + span - 1].g != t.g) {
                bz::LevelsArgs la{};
                bz::TaskArgs &a = la.t;
                a.rows = (const uint32_t *)c->dev;
                a.binom = dc.binom;
                a.rects = d_rects;
                a.key = rec + bz::kRecKey; a.stats = rec + bz::kRecStats; a.ncomb = rec + bz::kRecNcomb;
                a.tile_ctr = rec + bz::kRecCtr;
                a.cancel = (const uint32_t *)opt.cancel;
                a.k = k; a.k_low = c->k_low(t.j); a.g = gmax;
                a.chain = d_state;
                la.ntasks = span;
                uint64_t tiles = 0;
                for (uint32_t q = 0; q < span; ++q) {
                    const Task &u = win[i + q];
                    la.row_off[q] = (uint32_t)c->packed_off[u.j];
                    la.rect_off[q] = (uint32_t)on_device.at(u.key);
                    la.g[q] = u.g;
                    la.nrects[q] = (uint32_t)u.plan->rects.size();
                    la.heads[q] = u.plan->heads_per_tile;
                    tiles += u.plan->total_tiles;
                    la.tile_end[q] = tiles;
                    la.totals[q] = bz::binom_sat(k, u.g);
                    la.cert_task[q] = certified(u.j, u.g, m_f, k_m, k);
                    la.cert_level[q] = level_bound(u.g);
                    if (u.j == last_j) la.last_mask |= 1u << q;
                }
                a.total_tiles = tiles;
                bz::ChainStep &cs = a.step;
                cs.state = d_state;
                cs.level_stop = level_stop;
                cs.stats = stats;
                const uint32_t grid = (uint32_t)std::max<uint64_t>(
                    1, std::min<uint64_t>((tiles + 3) / 4, (uint64_t)dc.cus * 8));
                if (i == 0 && ev0) BZ_HIP(hipEventRecord(ev0, st));
                BZ_HIP(bz::launch_enum_levels(la, t.W, t.slots, stats, grid, st));
                i += span - 1;
                continue;
            }
            uint32_t group = 1;
            if (grouping && groupable(t))
                while (group < bz::kMaxGroup && i + group < win.size() && !win[i + group].sp &&
                       win[i + group].g == t.g && win[i + group].j == t.j + group && win[i + group].j < m_f &&
                       win[i + group].key == t.key && bz::enum_lds_bytes(k, t.g, t.W, group + 1) <= 65536)
                    ++group;
            bz::TaskArgs a{};
            a.rows = (const uint32_t *)c->dev + c->packed_off[t.j];
            a.binom = dc.binom;
            a.key = rec + bz::kRecKey; a.stats = rec + bz::kRecStats; a.ncomb = rec + bz::kRecNcomb;
            a.tile_ctr = rec + bz::kRecCtr;
            a.cancel = (const uint32_t *)opt.cancel;
            a.k = k; a.k_low = c->k_low(t.j); a.g = t.g;
            a.u_prev = U;
            a.exit_at = stats ? 0u : Lcert;
            if (t.sp) {
                const bz::SchedPlan *sp = t.sp;
                const size_t eb = align256(sp->entries.size() * sizeof(bz::PlanEntry));
                const size_t need = eb + sp->rects.size() * sizeof(bz::Rect);
                if (need > sbuf.cap) {
                    if (sbuf.p) (void)hipFree(sbuf.p);
                    sbuf.p = nullptr;
                    sbuf.cap = 0;
                    if (hipMalloc((void **)&sbuf.p, need) != hipSuccess) return fail(BZ_ENOMEM, "schedule tilings");
                    sbuf.cap = need;
                }
                BZ_HIP(hipMemcpyAsync(sbuf.p, sp->entries.data(), sp->entries.size() * sizeof(bz::PlanEntry),
                                      hipMemcpyHostToDevice, st));
                BZ_HIP(hipMemcpyAsync(sbuf.p + eb, sp->rects.data(), sp->rects.size() * sizeof(bz::Rect),
                                      hipMemcpyHostToDevice, st));
                bz::SchedArgs sa{};
                sa.t = a;
                sa.plans = (const bz::PlanEntry *)sbuf.p;
                sa.rects = (const bz::Rect *)(sbuf.p + eb);
                sa.ntasks = sp->ntasks;
                sa.stride = sp->stride;
                sa.pre = sp->pre;
                sa.dist = sched_dist;
                sa.order = sched_order;
                const size_t lds = bz::enum_lds_bytes(k, t.g, t.W);
                const uint32_t grid =
                    (uint32_t)dc.cus * (uint32_t)bz::sched_blocks_per_cu(t.W, t.j >= m_f, stats, lds);
                if (i == 0 && ev0) BZ_HIP(hipEventRecord(ev0, st));
                BZ_HIP(bz::launch_sched(sa, t.W, t.j >= m_f, stats, grid, st));
            } else {
                a.chain = d_state;
                a.rects = d_rects + on_device.at(t.key);
                a.nrects = (uint32_t)t.plan->rects.size();
                a.heads_per_tile = t.plan->heads_per_tile;
                a.total_tiles = t.plan->total_tiles;
                a.group = group;
                a.rows_stride = group > 1 ? (uint32_t)(c->packed_off[t.j + 1] - c->packed_off[t.j]) : 0u;
                for (uint32_t q = 0; q < group; ++q) {
                    a.cert_tasks[q] = certified(t.j + q, t.g, m_f, k_m, k);
                    if (t.j + q == last_j) a.last_mask |= 1u << q;
                }
                const uint64_t blocks = (group * t.plan->total_tiles + 3) / 4;
                const uint32_t grid =
                    (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(blocks, (uint64_t)dc.cus * 8));
                // the task's bookkeeping step runs in its last work-group
                bz::ChainStep &cs = a.step;
                cs.state = d_state;
                cs.key = a.key;
                cs.ncomb = a.ncomb;
                cs.total = bz::binom_sat(k, t.g);
                cs.cert_task = certified(t.j, t.g, m_f, k_m, k);
                cs.last_of_level = t.j == last_j;
                cs.cert_level = level_bound(t.g);
                cs.level_stop = level_stop;
                cs.stats = stats;
                if (i == 0 && ev0) BZ_HIP(hipEventRecord(ev0, st));
                BZ_HIP(bz::launch_enum(a, t.W, t.slots, t.j >= m_f, stats, grid, st));
                i += group - 1;
            }
        }
        if (ev1) BZ_HIP(hipEventRecord(ev1, st));
        if (dev_recover) {
            bz::RecoverWindowArgs ra{};
            ra.state = d_state;
            ra.records = d_records;
            ra.tasks = (const bz::RecoverTask *)(ws + kWsRecTasks);
            ra.binom = dc.binom;
            ra.flag = (unsigned int *)(ws + kWsRecover);
            ra.indices_len = (uint32_t *)(ws + kWsRecover + 4);
            ra.codeword = (unsigned long long *)(ws + kWsRecover + 8);
            ra.indices = (uint32_t *)(ws + kWsIndices);
            ra.ntasks = (uint32_t)win.size();
            ra.U0 = U_start;
            ra.have0 = have_start ? 1u : 0u;
            ra.k = k;
            uint32_t gmax = 0;
            for (const Task &t : win) gmax = std::max(gmax, t.g);
            if ((size_t)(k + 1) * (gmax + 1) * sizeof(uint64_t) <= 32 * 1024) ra.lds_g = gmax;
            BZ_HIP(bz::launch_recover_window(ra, rec_threads, st));
        }
        BZ_HIP(hipMemcpyAsync(words, ws + kWsChain, 128 + win.size() * kRecBytes, hipMemcpyDeviceToHost, st));
        BZ_HIP(hipStreamSynchronize(st));
        if (ev0) {
            float ms = 0.f;
            BZ_HIP(hipEventElapsedTime(&ms, ev0, ev1));
            res->kernel_s += ms * 1e-3;
        }

        bool stopped = false;                  // L reached U at a level start inside the window
        bool best_here = false;                // the winning tile is one of this window's
        for (size_t i = 0; i < win.size() && !done; ++i) {
            const Task &t = win[i];
            if (i > 0 && t.j == 0 && L >= U) { stopped = true; break; }
            const unsigned long long *r = words + 16 + i * bz::kRecWords;
            const uint32_t j = t.j, g = t.g, slots = t.slots;
            res->last_level = g;
            res->launches++;
            const uint32_t tmin = r[bz::kRecKey] == ~0ull ? 0xffffffffu : (uint32_t)(r[bz::kRecKey] >> bz::kTileBits);
            const uint64_t ncomb = r[bz::kRecNcomb];
            const bool complete = ncomb == bz::binom_sat(k, g);
            res->combinations += ncomb;
            if (res->stats && res->stats_len < res->stats_cap) {
                bz_level_stat &s = res->stats[res->stats_len];
                s.matrix = (uint16_t)j; s.level = (uint16_t)g; s.min_weight = tmin;
                s.count_at_min = stats ? (r[bz::kRecStats] & ((1ull << 55) - 1)) : 0;
                s.combinations = ncomb;
            }
            res->stats_len++;
            if (tmin < U || (tmin == U && !best.have)) {
                U = tmin;
                best_here = true;
                best.have = true; best.j = j; best.g = g; best.tile = r[bz::kRecKey] & bz::kTileMask;
                best.slots = slots;
                const bz::Rect *rr = nullptr;
                size_t nr = 0;
                if (t.sp) {
                    // key tile = prefix task * stride + tile of that task's completion plan
                    const uint64_t task = best.tile / t.sp->stride;
                    best.tile -= task * t.sp->stride;
                    uint32_t lo = 0;
                    bz::sched_prefix(*t.sp, k, g, sched_order, task, best.pre, lo);
                    const bz::PlanEntry &e = t.sp->entries[lo];
                    rr = t.sp->rects.data() + e.rect_off;
                    nr = e.nrects;
                    best.ht = e.heads_per_tile;
                } else {
                    best.pre.clear();
                    rr = t.plan->rects.data();
                    nr = t.plan->rects.size();
                    best.ht = t.plan->heads_per_tile;
                }
                size_t lo = 0, hi = nr - 1;
                while (lo < hi) {
                    size_t mid = (lo + hi + 1) / 2;
                    if (rr[mid].tile_begin <= best.tile) lo = mid; else hi = mid - 1;
                }
                best.rect = rr[lo];
            }
            next_j = j == last_j ? 0 : j + 1;
            next_g = j == last_j ? g + 1 : g;
            if (opt.cancel && *opt.cancel && !complete) { status = BZ_ECANCELED; g_err = "canceled"; done = true; break; }
            if (!complete) {
                // a wave only leaves a task early once U <= the certified bound
                if (U > Lcert) return fail(BZ_EDEVICE, "internal: task ended early without a certificate");
                L = std::max(L, Lcert);
                done = true;
                break;
            }
            Lcert = std::max(Lcert, certified(j, g, m_f, k_m, k));
            if (!level_stop) {
                L = std::max(L, Lcert);
                if (L >= U) done = true;
            }
            if (!done && j == last_j) L = std::max(L, level_bound(g));
        }
        if (!use_sched) {
            // the device took the same decisions: it stopped exactly where the host does
            const bool host_stop = done || stopped || (next_j == 0 && L >= U);
            const bool dev_stop = ((const bz::ChainState *)words)->done != 0;
            if (host_stop != dev_stop) return fail(BZ_EDEVICE, "internal: device and host bookkeeping disagree");
            if (dev_recover && dev_stop && best_here && status == BZ_OK) {
                // the window recovered the witness of the same winning tile
                const unsigned long long *back = words + (kWsRecover - kWsChain) / 8;
                if ((uint32_t)back[0] != 1u) return fail(BZ_EDEVICE, "internal: witness not found in its tile");
                for (uint32_t w = 0; w < (n + 63) / 64; ++w) res->witness[w] = back[1 + w];
                witness_done = true;
            }
        }
    }
    res->lower_bound = L;
    res->upper_bound = U;
    if (status == BZ_OK && res->stats && res->stats_len > res->stats_cap) {
        status = BZ_ELIMIT;
        g_err = "stats buffer too small";
    }
    if (status == BZ_OK && want_witness && !finished_in_one && !witness_done) {
        if (!best.have) return fail(BZ_EDEVICE, "internal: no witness tile");
        bz::RecoverArgs ra{};
        const uint32_t j = best.j;
        ra.rows = (const uint32_t *)c->dev + c->packed_off[j];
        ra.full_rows = (const uint64_t *)((char *)c->dev + c->dev_full_off) + (size_t)j * k * bz::kHostWords;
        ra.binom = dc.binom;
        ra.rect = best.rect;
        ra.flag = (unsigned int *)(ws + kWsRecover);        // cleared by the last window's init
        ra.indices_len = (uint32_t *)(ws + kWsRecover + 4);
        ra.codeword = (unsigned long long *)(ws + kWsRecover + 8);
        ra.indices = (uint32_t *)(ws + kWsIndices);
        ra.tile = best.tile; ra.slots = best.slots; ra.heads_per_tile = best.ht;
        ra.W = c->W(j); ra.k_low = c->k_low(j); ra.target = U;
        ra.pre_n = (uint32_t)best.pre.size();
        ra.pre_rows = (const uint32_t *)(ws + kWsPreRows);
        if (ra.pre_n) {
            if (ra.pre_n > 64) return fail(BZ_EDEVICE, "internal: prefix longer than its buffer");
            std::memcpy(stage, best.pre.data(), ra.pre_n * sizeof(uint32_t));
            BZ_HIP(hipMemcpyAsync(ws + kWsPreRows, stage, ra.pre_n * sizeof(uint32_t), hipMemcpyHostToDevice, st));
        }
        BZ_HIP(bz::launch_recover(ra, st));
        unsigned long long *back = words;
        BZ_HIP(hipMemcpyAsync(back, ws + kWsRecover, 5 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
        BZ_HIP(hipStreamSynchronize(st));
        if ((uint32_t)back[0] != 1u) return fail(BZ_EDEVICE, "internal: witness not found in its tile");
        for (uint32_t w = 0; w < (n + 63) / 64; ++w) res->witness[w] = back[1 + w];
    }
    if (status == BZ_OK) res->d = U;
    res->search_s = now_s() - t0;
    return status;
}

// The no-allocation search's per-device state: found once per device, then
// shared (under its lock) by every call on that device.
struct NoAllocDevice {
    std::mutex mu;
    bool ready = false;
    NoAllocEnv env;
    std::vector<unsigned long long> host;
};

constexpr size_t kBinomBytes = (size_t)bz::kBinomRows * (bz::kBinomT + 1) * sizeof(uint64_t);
constexpr size_t kNoAllocWsOff = (kBinomBytes + 255) & ~(size_t)255;
static_assert(kNoAllocWsOff + kWsBytes <= bz::kNoAllocScratchBytes,
              "the scratch array holds the binomial table and one search's workspace");

NoAllocDevice &noalloc_device(int dev) {
    static std::mutex mu;
    static std::map<int, std::unique_ptr<NoAllocDevice>> devs;
    std::lock_guard<std::mutex> lk(mu);
    auto &p = devs[dev];
    if (!p) p.reset(new NoAllocDevice());
    return *p;
}

// Set-up on the first call on a device, with that device current: the scratch
// array's address on this device, the binomial table copied into it, and the
// host read-back memory.
bz_status noalloc_setup(int dev, NoAllocDevice &D) {
    void *base = nullptr;
    const hipError_t e = bz::noalloc_scratch_address(&base);
    if (e != hipSuccess || !base)
        return fail(BZ_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    BZ_HIP(hipDeviceGetAttribute(&D.env.dc.cus, hipDeviceAttributeMultiprocessorCount, dev));
    const std::vector<uint64_t> tab = bz::binom_table();
    BZ_HIP(hipMemcpy(base, tab.data(), kBinomBytes, hipMemcpyHostToDevice));
    D.env.dc.binom = (uint64_t *)base;
    D.env.ws = (char *)base + kNoAllocWsOff;
    D.host.assign(kPinnedBytes / 8, 0ull);
    D.env.host = D.host.data();
    D.ready = true;
    return BZ_OK;
}

}  // namespace

extern "C" {

bz_status bz_min_distance(bz_code *c, const bz_opts *o, bz_result *res) {
    return min_distance_impl(c, o, res, nullptr);
}

bz_status bz_min_distance_noalloc(bz_code *c, const bz_opts *o, bz_result *res) {
    if (!c || !res) return fail(BZ_EINVAL, "null argument");
    if (!c->dev) return fail(BZ_EINVAL, "code prepared host-only (BZ_PREPARE_HOST_ONLY): submit it to a server");
    if (o && o->workspace)
        return fail(BZ_EINVAL, "the no-allocation search works in the library's scratch array: pass no workspace");
    if (o && o->schedule != BZ_SCHED_TILES)
        return fail(BZ_EINVAL, "schedules 1..8 need device memory for their tilings: use bz_min_distance");
    if (hipSetDevice(c->device) != hipSuccess) return fail(BZ_EDEVICE, "hipSetDevice");
    NoAllocDevice &D = noalloc_device(c->device);
    std::lock_guard<std::mutex> lk(D.mu);          // calls on one device share its array
    if (!D.ready) {
        const bz_status s = noalloc_setup(c->device, D);
        if (s != BZ_OK) return s;
    }
    return min_distance_impl(c, o, res, &D.env);
}

bz_status bz_min_distance_batch(bz_code *const *codes, uint32_t count, const bz_opts *o,
                                bz_result *res, bz_status *per_code) {
    return batch_run(codes, count, o, res, per_code);
}

}  // extern "C"

// ---------------------------------------------------------------- host-only inspection

#include "../../include/bz_debug.h"

extern "C" {

bz_status bz_debug_prepare_host(const uint64_t *G, uint32_t k, uint32_t n, uint32_t ld_words,
                                uint32_t *num_full, uint32_t *partial_rank, int32_t *set_of_column,
                                uint64_t *gamma_rows, uint32_t gamma_cap_rows,
                                uint32_t *packed, size_t packed_cap) {
    bz_code c;
    std::string err;
    bz_status st = bz::prepare_host(G, k, n, ld_words, nullptr, c, err);
    if (st != BZ_OK) return fail(st, err);
    if (num_full) *num_full = c.num_full;
    if (partial_rank) *partial_rank = c.partial_rank;
    if (set_of_column) std::memcpy(set_of_column, c.set_of_column.data(), n * sizeof(int32_t));
    if (gamma_rows) {
        if ((uint64_t)c.nsets * k > gamma_cap_rows) return fail(BZ_ELIMIT, "gamma buffer too small");
        for (size_t r = 0; r < c.full_rows.size(); ++r)
            for (uint32_t w = 0; w < ld_words; ++w)
                gamma_rows[r * ld_words + w] = w < (uint32_t)bz::kHostWords ? c.full_rows[r][w] : 0;
    }
    if (packed) {
        if (c.packed.size() > packed_cap) return fail(BZ_ELIMIT, "packed buffer too small");
        std::memcpy(packed, c.packed.data(), c.packed.size() * sizeof(uint32_t));
    }
    return BZ_OK;
}

bz_status bz_debug_plan_level(uint32_t k, uint32_t g, uint32_t slots, uint32_t heads_per_tile,
                              uint64_t target_tiles, uint32_t widen, bz_debug_rect *rects, uint32_t cap,
                              uint32_t *nrects, uint64_t *total_tiles, uint32_t *heads_used) {
    if (k == 0 || k > (uint32_t)bz::kMaxN || (slots != 2 && slots != 4 && slots != 8 && slots != 16))
        return fail(BZ_EINVAL, "bad k or slots");
    bz::LevelPlan p;
    std::string err;
    if (!bz::plan_level(k, g, slots, heads_per_tile, target_tiles, p, err, widen != 0)) return fail(BZ_ELIMIT, err);
    if (nrects) *nrects = (uint32_t)p.rects.size();
    if (total_tiles) *total_tiles = p.total_tiles;
    if (heads_used) *heads_used = p.heads_per_tile;
    if (rects) {
        if (p.rects.size() > cap) return fail(BZ_ELIMIT, "rect buffer too small");
        static_assert(sizeof(bz_debug_rect) == sizeof(bz::Rect), "layouts agree");
        std::memcpy(rects, p.rects.data(), p.rects.size() * sizeof(bz::Rect));
    }
    return BZ_OK;
}

bz_status bz_debug_valu_rate(uint32_t iters, double *lane_ops_per_s, double *seconds) {
    if (!lane_ops_per_s || !seconds) return fail(BZ_EINVAL, "null output");
    if (iters == 0) iters = 200000;
    int dev = 0;
    BZ_HIP(hipGetDevice(&dev));
    DeviceConst dc;
    bz_status s0 = device_const(dev, dc);
    if (s0 != BZ_OK) return s0;
    const uint32_t blocks = (uint32_t)(dc.cus * bz::valu_probe_blocks_per_cu());
    uint32_t *sink = nullptr;
    BZ_HIP(hipMalloc((void **)&sink, (size_t)blocks * bz::kBlock * sizeof(uint32_t)));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    struct Guard {
        uint32_t *p; hipEvent_t &a, &b;
        ~Guard() { (void)hipFree(p); if (a) (void)hipEventDestroy(a); if (b) (void)hipEventDestroy(b); }
    } g{sink, e0, e1};
    BZ_HIP(hipEventCreate(&e0));
    BZ_HIP(hipEventCreate(&e1));
    BZ_HIP(bz::launch_valu_probe(iters / 10 + 1, blocks, sink, nullptr));       // warm-up: clocks up
    BZ_HIP(hipEventRecord(e0, nullptr));
    BZ_HIP(bz::launch_valu_probe(iters, blocks, sink, nullptr));
    BZ_HIP(hipEventRecord(e1, nullptr));
    BZ_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    BZ_HIP(hipEventElapsedTime(&ms, e0, e1));
    *seconds = ms * 1e-3;
    *lane_ops_per_s = (double)blocks * bz::kBlock * (double)iters * 16.0 / (*seconds);
    return BZ_OK;
}

}  // extern "C"
