// Serving (bz_server_* in include/bz.h): continuous batching of
// Brouwer-Zimmermann searches (Alg. 1 of arXiv:1911.08963) on one device.
//
// One persistent kernel (bz_serve_kernel) stays resident. The host stages
// each request in pinned host memory (its Gamma_j payload, its code
// description, new plan tables) and raises the published ticket count; the
// wave holding that ticket copies the request onto the device and starts it
// while the others go on. A finished request's statistics, bounds and
// witness come back in a pinned completion record whose flag a watcher
// thread timestamps. This is the paper's dynamic coordinator/worker scheme
// (Sec. 3.2) with requests arriving over time instead of a fixed code.
//
// Within one kernel launch every request gets a fresh code index (its
// ticket) and fresh device addresses, because the kernel reads Gamma_j rows
// through the scalar cache, which nothing invalidates while it runs. When
// the indices or the arena run out, the server drains, stops the kernel and
// launches it again.
#include <hip/hip_runtime.h>
#include <sys/prctl.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <set>
#include <thread>
#include <vector>

#include "bz_host.h"
#include "bz_internal.h"
#include "bz_kernels.h"

namespace {

using bz::fail;
using bz::now_s;

constexpr uint64_t kServeMaxComb = 1ull << 50;  // levels with C(k, g) beyond this get no plan
static_assert(kServeMaxComb <= (1ull << 55), "a task's count at the minimum fits the statistics word's 55 bits");
constexpr uint32_t kMaxPlans = 4096;            // distinct (k, slots) plans per server
constexpr uint32_t kPlanEntries = 1u << 17;     // PlanEntry table (4 MiB)
constexpr uint32_t kPlanRects = 1u << 19;       // Rect table (40 MiB)
constexpr uint64_t kLogCap = 1ull << 20;        // shared task log ring
constexpr size_t kSlotBytes = 48 * 1024;        // staged payload of one request (n <= 256 needs <= 40 KiB)
constexpr uint32_t kEntryAlign = 8;             // plans start on 256-byte boundaries ...
constexpr uint32_t kRectAlign = 16;             // ... in both tables (16 x 80 B = 5 x 256 B)
// Tiles of a served request: each level is cut into about target_tiles tiles
// (by default 4 per wave the device holds, as for bz_min_distance), with at
// most kServeMaxHeads head steps each: a large task splits into few claims.
// (The waves that will start new requests hold no tiles meanwhile, so tile
// length does not delay a request's start.)
constexpr uint32_t kServeMaxHeads = 4096;

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

struct SlotInfo {
    bool busy = false, finished = false;
    uint64_t ticket = 0;        // global ticket
    uint64_t ring_entry = 0;
    bz_result *res = nullptr;
    uint32_t flags = 0, n = 0, dev_stats_cap = 0;
    double t_submit = 0, t_done = 0, prepare_s = 0;
    size_t bytes = 0;
};

struct PlanInfo {
    uint32_t pid = 0, gmax = 0, entry_off = 0;
};

}  // namespace

struct bz_server {
    int device = 0;
    bool stats = false;
    uint32_t slots = 0, stats_cap = 0, target_tiles = 0, codes_per_launch = 0, grid = 0;
    size_t hbm_budget = 0, arena_bytes = 0;
    uint64_t ring = 0;
    hipStream_t stream = nullptr;
    bz::DeviceConst dc;
    // device memory
    char *dmem = nullptr;
    size_t off_codes = 0, off_state = 0, off_plans = 0, off_rects = 0, off_stats = 0, off_log = 0, off_done = 0,
           off_view = 0, off_ready = 0, off_args = 0, off_arena = 0, dbytes = 0;
    // pinned host memory
    char *hmem = nullptr;
    bz::ServeReq *reqs = nullptr;
    bz::ServePlanDesc *plan_desc = nullptr;
    bz::PlanEntry *host_plans = nullptr;
    bz::Rect *host_rects = nullptr;
    unsigned long long *published = nullptr;
    uint32_t *shutdown = nullptr;
    bz::ServeRecord *records = nullptr;
    bz::BatchStat *host_stats = nullptr;
    char *staging = nullptr;
    // host state, under mu
    std::mutex mu;
    bool running = false;
    uint64_t next_ticket = 0, gen_base = 0;
    size_t arena_used = 0, inflight_bytes = 0;
    uint32_t unfinished = 0, pending = 0, launches = 0;
    std::vector<SlotInfo> slot;
    std::vector<uint32_t> free_slots, active;
    std::vector<uint8_t> ring_busy;
    std::map<std::pair<uint32_t, uint32_t>, PlanInfo> plans;
    uint32_t nplans = 0, entries_used = 0, rects_used = 0;
    std::deque<uint32_t> finished;
    std::thread watcher;
    std::atomic<bool> stop_watch{false};
};

namespace {

std::mutex g_live_mu;
std::set<bz_server *> g_live;
bool g_atexit = false;

// Marks finished requests (records flagged by the device). Caller holds mu.
void observe_locked(bz_server *s) {
    const double t = now_s();
    for (size_t i = 0; i < s->active.size();) {
        const uint32_t sl = s->active[i];
        if (__atomic_load_n(&s->records[sl].flag, __ATOMIC_ACQUIRE)) {
            SlotInfo &si = s->slot[sl];
            si.finished = true;
            si.t_done = t;
            s->finished.push_back(sl);
            s->unfinished--;
            s->active[i] = s->active.back();
            s->active.pop_back();
        } else {
            ++i;
        }
    }
}

void watch(bz_server *s) {
    prctl(PR_SET_TIMERSLACK, 1000UL);        // 1 us: sleeps of a few tens of us stay short
    while (!s->stop_watch.load(std::memory_order_acquire)) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            observe_locked(s);
        }
        std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}

bz::ServeArgs serve_args(bz_server *s) {
    bz::ServeArgs a{};
    bz::BatchArgs &b = a.b;
    b.codes = (const bz::BatchCode *)(s->dmem + s->off_codes);
    b.state = (bz::CodeState *)(s->dmem + s->off_state);
    b.plans = (const bz::PlanEntry *)(s->dmem + s->off_plans);
    b.rects = (const bz::Rect *)(s->dmem + s->off_rects);
    b.binom = s->dc.binom;
    b.stats = (bz::BatchStat *)(s->dmem + s->off_stats);
    b.recover = nullptr;
    unsigned long long *log_base = (unsigned long long *)(s->dmem + s->off_log);
    b.log_head = log_base + bz::kLogHead;
    b.log_tail = log_base + bz::kLogTail;
    b.next_code = log_base + bz::kLogNext;
    b.log = log_base + bz::kLogEntries;
    b.log_cap = kLogCap;
    b.done_count = (unsigned int *)(s->dmem + s->off_done);
    b.cancel = nullptr;
    b.ncodes = s->codes_per_launch;
    a.reqs = s->reqs;
    a.plan_desc = s->plan_desc;
    a.host_plans = s->host_plans;
    a.host_rects = s->host_rects;
    a.plan_ready = (unsigned int *)(s->dmem + s->off_ready);
    a.published = s->published;
    a.shutdown = s->shutdown;
    a.records = s->records;
    a.host_stats = s->host_stats;
    a.view = (unsigned long long *)(s->dmem + s->off_view);
    a.ring = s->ring;
    a.stats_cap = s->stats_cap;
    return a;
}

// Starts a kernel launch with empty counters. Caller holds mu; no kernel runs.
bz_status launch_locked(bz_server *s) {
    BZ_HIP(hipMemsetAsync(s->dmem + s->off_log, 0, (kLogCap + bz::kLogEntries) * sizeof(unsigned long long),
                          s->stream));
    BZ_HIP(hipMemsetAsync(s->dmem + s->off_done, 0, 256, s->stream));
    BZ_HIP(hipMemsetAsync(s->dmem + s->off_view, 0, 256, s->stream));
    BZ_HIP(hipStreamSynchronize(s->stream));
    __atomic_store_n(s->published, 0ull, __ATOMIC_RELEASE);
    __atomic_store_n(s->shutdown, 0u, __ATOMIC_RELEASE);
    const bz::ServeArgs a = serve_args(s);
    bz::ServeArgs *da = (bz::ServeArgs *)(s->dmem + s->off_args);
    BZ_HIP(hipMemcpyAsync(da, &a, sizeof(a), hipMemcpyHostToDevice, s->stream));
    BZ_HIP(hipStreamSynchronize(s->stream));
    hipError_t e = bz::launch_serve(da, s->grid, s->stats, s->stream);
    if (e != hipSuccess) return fail(BZ_EDEVICE, std::string("serving kernel launch: ") + hipGetErrorString(e));
    s->running = true;
    s->launches++;
    s->gen_base = s->next_ticket;
    s->arena_used = 0;
    std::fill(s->ring_busy.begin(), s->ring_busy.end(), 0);
    return BZ_OK;
}

// Waits for the kernel to leave; after timeout_s it is told to leave at once.
// Returns BZ_EDEVICE if it had to be stopped that way or did not stop.
bz_status stop_locked(bz_server *s, double timeout_s) {
    if (!s->running) return BZ_OK;
    __atomic_store_n(s->shutdown, 1u, __ATOMIC_RELEASE);
    bz_status result = BZ_OK;
    const double t0 = now_s();
    bool forced = false;
    for (;;) {
        hipError_t q = hipStreamQuery(s->stream);
        if (q == hipSuccess) break;
        if (q != hipErrorNotReady) {
            s->running = false;
            return fail(BZ_EDEVICE, std::string("serving kernel: ") + hipGetErrorString(q));
        }
        const double el = now_s() - t0;
        if (!forced && el > timeout_s) {
            __atomic_store_n(s->shutdown, 2u, __ATOMIC_RELEASE);
            forced = true;
            result = fail(BZ_EDEVICE, "serving kernel stopped before its requests finished");
        }
        if (el > timeout_s + 30.0) {
            s->running = false;
            return fail(BZ_EDEVICE, "serving kernel did not stop");
        }
        std::this_thread::sleep_for(std::chrono::microseconds(200));
    }
    s->running = false;
    return result;
}

// The plans of one (k, slots), built and placed in the host mirror on first
// use; copy = the request that brings them onto the device.
bz_status plan_for(bz_server *s, uint32_t k, uint32_t slots, PlanInfo &out, bool &copy) {
    auto key = std::make_pair(k, slots);
    auto it = s->plans.find(key);
    if (it != s->plans.end()) {
        out = it->second;
        copy = false;
        return BZ_OK;
    }
    if (s->nplans >= kMaxPlans) return fail(BZ_ENOMEM, "server plan table full (distinct k)");
    const uint32_t eo = (s->entries_used + kEntryAlign - 1) / kEntryAlign * kEntryAlign;
    const uint32_t ro = (s->rects_used + kRectAlign - 1) / kRectAlign * kRectAlign;
    std::vector<bz::PlanEntry> pe;
    std::vector<bz::Rect> rc;
    const uint32_t gmax =
        bz::build_level_plans(k, slots, 0, s->target_tiles, kServeMaxComb, ro, pe, rc, kServeMaxHeads);
    if ((uint64_t)eo + pe.size() > kPlanEntries || (uint64_t)ro + rc.size() > kPlanRects)
        return fail(BZ_ENOMEM, "server plan tables full");
    std::memcpy(s->host_plans + eo, pe.data(), pe.size() * sizeof(bz::PlanEntry));
    std::memcpy(s->host_rects + ro, rc.data(), rc.size() * sizeof(bz::Rect));
    PlanInfo p;
    p.pid = s->nplans++;
    p.gmax = gmax;
    p.entry_off = eo;
    bz::ServePlanDesc &d = s->plan_desc[p.pid];
    d.entry_off = eo;
    d.levels = (uint32_t)pe.size();
    d.rect_off = ro;
    d.nrects = (uint32_t)rc.size();
    s->entries_used = eo + (uint32_t)pe.size();
    s->rects_used = ro + (uint32_t)rc.size();
    s->plans[key] = p;
    out = p;
    copy = true;
    return BZ_OK;
}

void free_server(bz_server *s) {
    if (s->watcher.joinable()) {
        s->stop_watch.store(true, std::memory_order_release);
        s->watcher.join();
    }
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    if (s->dmem) (void)hipFree(s->dmem);
    if (s->hmem) (void)hipHostFree(s->hmem);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

// A process that exits with a server still running must not leave its
// kernel behind: tell every live kernel to leave and wait for it.
void stop_all_at_exit() {
    std::lock_guard<std::mutex> lk(g_live_mu);
    for (bz_server *s : g_live) {
        std::lock_guard<std::mutex> l2(s->mu);
        (void)stop_locked(s, 5.0);
    }
}

}  // namespace

extern "C" {

bz_status bz_server_create(const bz_server_opts *o, bz_server **out) {
    if (!out) return fail(BZ_EINVAL, "out is null");
    *out = nullptr;
    bz_server_opts opt{};
    if (o) opt = *o;
    if (opt.flags & ~(uint32_t)BZ_F_STATS) return fail(BZ_EINVAL, "server flags: only BZ_F_STATS");
    if (opt.slots > 65536) return fail(BZ_EINVAL, "slots must be at most 65536");
    std::unique_ptr<bz_server> s(new (std::nothrow) bz_server());
    if (!s) return fail(BZ_ENOMEM, "host allocation");
    s->stats = opt.flags & BZ_F_STATS;
    s->slots = opt.slots ? opt.slots : 1024;
    s->stats_cap = opt.stats_cap ? opt.stats_cap : 512;
    s->target_tiles = opt.target_tiles;     // 0: set from the device below
    s->arena_bytes = opt.arena_bytes ? opt.arena_bytes : ((size_t)1 << 30);
    s->codes_per_launch = opt.codes_per_launch ? opt.codes_per_launch : (1u << 18);
    s->hbm_budget = opt.hbm_budget;
    s->ring = 1024;                          // a power of two, at least 4 x slots
    while (s->ring < 4ull * s->slots) s->ring <<= 1;
    if (s->arena_bytes < kSlotBytes) return fail(BZ_EINVAL, "arena_bytes below one request");
    BZ_HIP(hipGetDevice(&s->device));
    bz_status st0 = bz::device_const(s->device, s->dc);
    if (st0 != BZ_OK) return st0;
    if (!s->target_tiles) s->target_tiles = (uint32_t)s->dc.cus * 32 * bz::kFixedTilesPerWave;

    // device memory
    size_t off = 0;
    s->off_codes = off; off = a256(off + (size_t)s->codes_per_launch * sizeof(bz::BatchCode));
    s->off_state = off; off = a256(off + (size_t)s->codes_per_launch * sizeof(bz::CodeState));
    s->off_plans = off; off = a256(off + (size_t)kPlanEntries * sizeof(bz::PlanEntry));
    s->off_rects = off; off = a256(off + (size_t)kPlanRects * sizeof(bz::Rect));
    s->off_stats = off; off = a256(off + (size_t)s->slots * s->stats_cap * sizeof(bz::BatchStat));
    s->off_log = off; off = a256(off + (kLogCap + bz::kLogEntries) * sizeof(unsigned long long));
    s->off_done = off; off = a256(off + 256);
    s->off_view = off; off = a256(off + 256);
    s->off_ready = off; off = a256(off + kMaxPlans * sizeof(unsigned int));
    s->off_args = off; off = a256(off + sizeof(bz::ServeArgs));
    s->off_arena = off; off = a256(off + s->arena_bytes);
    s->dbytes = off;
    if (hipMalloc((void **)&s->dmem, s->dbytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(BZ_ENOMEM, "server device memory");
    }
    // pinned host memory, coherent: the running kernel polls and writes it
    size_t h = 0;
    const size_t h_reqs = h; h = a256(h + s->ring * sizeof(bz::ServeReq));
    const size_t h_desc = h; h = a256(h + kMaxPlans * sizeof(bz::ServePlanDesc));
    const size_t h_plans = h; h = a256(h + (size_t)kPlanEntries * sizeof(bz::PlanEntry));
    const size_t h_rects = h; h = a256(h + (size_t)kPlanRects * sizeof(bz::Rect));
    const size_t h_pub = h; h = a256(h + 256);
    const size_t h_rec = h; h = a256(h + (size_t)s->slots * sizeof(bz::ServeRecord));
    const size_t h_stats = h; h = a256(h + (size_t)s->slots * s->stats_cap * sizeof(bz::BatchStat));
    const size_t h_stage = h; h = a256(h + (size_t)s->slots * kSlotBytes);
    if (hipHostMalloc((void **)&s->hmem, h, hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(s->dmem);
        return fail(BZ_ENOMEM, "server pinned host memory");
    }
    std::memset(s->hmem, 0, h_stage);        // everything but the staging area
    s->reqs = (bz::ServeReq *)(s->hmem + h_reqs);
    s->plan_desc = (bz::ServePlanDesc *)(s->hmem + h_desc);
    s->host_plans = (bz::PlanEntry *)(s->hmem + h_plans);
    s->host_rects = (bz::Rect *)(s->hmem + h_rects);
    s->published = (unsigned long long *)(s->hmem + h_pub);
    s->shutdown = (uint32_t *)(s->hmem + h_pub + 64);
    s->records = (bz::ServeRecord *)(s->hmem + h_rec);
    s->host_stats = (bz::BatchStat *)(s->hmem + h_stats);
    s->staging = s->hmem + h_stage;

    auto undo = [&](bz_status st) {
        if (s->stream) (void)hipStreamDestroy(s->stream);
        (void)hipFree(s->dmem);
        (void)hipHostFree(s->hmem);
        return st;
    };
    if (hipMemset(s->dmem + s->off_ready, 0, kMaxPlans * sizeof(unsigned int)) != hipSuccess ||
        hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        return undo(fail(BZ_EDEVICE, "server stream"));
    }
    s->grid = (uint32_t)std::max(1, s->dc.cus * bz::serve_blocks_per_cu(s->stats));
    s->slot.resize(s->slots);
    for (uint32_t i = s->slots; i-- > 0;) s->free_slots.push_back(i);
    s->ring_busy.assign(s->ring, 0);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        bz_status st = launch_locked(s.get());
        if (st != BZ_OK) return undo(st);
    }
    s->watcher = std::thread(watch, s.get());
    {
        std::lock_guard<std::mutex> lk(g_live_mu);
        g_live.insert(s.get());
        if (!g_atexit) {
            std::atexit(stop_all_at_exit);
            g_atexit = true;
        }
    }
    *out = s.release();
    return BZ_OK;
}

bz_status bz_server_submit(bz_server *s, const bz_code *c, const bz_opts *o, bz_result *res, uint64_t *ticket) {
    if (!s || !c || !res || !ticket) return fail(BZ_EINVAL, "null argument");
    bz_opts opt{};
    if (o) opt = *o;
    if (opt.flags & ~(uint32_t)(BZ_F_STATS | BZ_F_LEVEL_STOP | BZ_F_NO_WITNESS)) return fail(BZ_EINVAL, "unknown flag");
    if (((opt.flags & BZ_F_STATS) != 0) != s->stats)
        return fail(BZ_EINVAL, "BZ_F_STATS must match the server's mode");
    if (c->dev && c->device != s->device) return fail(BZ_EINVAL, "code prepared on another device");
    const size_t payload = c->dev_bytes;
    if (payload > kSlotBytes) return fail(BZ_EINVAL, "code too large for a request slot");
    res->d = 0; res->lower_bound = 0; res->upper_bound = 0; res->last_level = 0;
    res->combinations = 0; res->stats_len = 0; res->launches = 0;
    res->prepare_s = c->prepare_s; res->search_s = 0; res->kernel_s = 0;

    std::lock_guard<std::mutex> lk(s->mu);
    if (!s->running) return fail(BZ_EDEVICE, "serving kernel is not running");
    hipError_t q = hipStreamQuery(s->stream);
    if (q != hipErrorNotReady) {
        s->running = false;
        return fail(BZ_EDEVICE, std::string("serving kernel ended: ") + hipGetErrorString(q));
    }
    observe_locked(s);
    if (s->free_slots.empty()) return fail(BZ_EBUSY, "no free request slot");
    const uint32_t k = c->k, n = c->n;
    const bool whole = (k == n);
    uint32_t dev_stats_cap = std::min<uint32_t>(s->stats_cap, c->nsets * std::max<uint32_t>(1, k));
    const size_t req_bytes = a256(payload) + sizeof(bz::BatchCode) + sizeof(bz::CodeState) +
                             (size_t)dev_stats_cap * sizeof(bz::BatchStat);
    if (s->hbm_budget && s->inflight_bytes + req_bytes > s->hbm_budget)
        return fail(BZ_EBUSY, "HBM budget of the requests in flight reached");

    // a new launch when the code indices or the arena are used up
    uint64_t dt = s->next_ticket - s->gen_base;
    if (dt >= s->codes_per_launch || s->arena_used + a256(payload) > s->arena_bytes) {
        if (s->unfinished > 0) return fail(BZ_EBUSY, "draining before the serving kernel is relaunched");
        bz_status st = stop_locked(s, 60.0);
        if (st != BZ_OK) return st;
        st = launch_locked(s);
        if (st != BZ_OK) return st;
        dt = 0;
    }
    const uint64_t e = dt & (s->ring - 1);
    if (s->ring_busy[e]) return fail(BZ_EBUSY, "request ring entry still in use");

    bz::ServeReq R{};
    R.plan_copy[0] = R.plan_copy[1] = R.plan_wait[0] = R.plan_wait[1] = bz::kNoPlan;
    uint32_t gmax = 0, plan_full = 0, plan_partial = 0;
    if (!whole) {
        PlanInfo pf, pp;
        bool cf = false, cp = false;
        bz_status st = plan_for(s, k, bz::slots_for_w(c->W_full), pf, cf);
        if (st != BZ_OK) return st;
        pp = pf;
        if (c->W_partial) {
            st = plan_for(s, k, bz::slots_for_w(c->W_partial), pp, cp);
            if (st != BZ_OK) return st;
        }
        (cf ? R.plan_copy[0] : R.plan_wait[0]) = pf.pid;
        if (pp.pid != pf.pid) (cp ? R.plan_copy[1] : R.plan_wait[1]) = pp.pid;
        gmax = std::min(pf.gmax, pp.gmax);
        plan_full = pf.entry_off;
        plan_partial = pp.entry_off;
        dev_stats_cap = std::min<uint32_t>(s->stats_cap, c->nsets * std::max<uint32_t>(1, gmax));
    }
    const uint32_t sl = s->free_slots.back();
    s->free_slots.pop_back();
    // payload: packed rows (with their zero rows), then the full rows at dev_full_off
    char *stage = s->staging + (size_t)sl * kSlotBytes;
    const size_t packed_bytes = c->packed.size() * sizeof(uint32_t);
    std::memcpy(stage, c->packed.data(), packed_bytes);
    std::memset(stage + packed_bytes, 0, c->dev_full_off - packed_bytes);
    std::memcpy(stage + c->dev_full_off, c->full_rows.data(), c->full_rows.size() * sizeof(bz::HostRow));
    char *dst = s->dmem + s->off_arena + s->arena_used;

    bz::BatchCode &D = R.code;
    D.rows = (const uint32_t *)dst;
    D.px_delta = c->px_delta;
    D.full_rows = (const uint64_t *)(dst + c->dev_full_off);
    D.n = n; D.k = k; D.m_f = c->num_full; D.k_m = c->partial_rank;
    D.nsets = c->nsets; D.W_full = c->W_full; D.W_partial = c->W_partial; D.g_max = gmax;
    D.plan_full = plan_full; D.plan_partial = plan_partial;
    D.stats_off = sl * s->stats_cap; D.stats_cap = dev_stats_cap;
    D.flags = opt.flags; D.max_level = opt.max_level;
    D.tag = s->next_ticket; D.slot = sl;
    R.src = (const uint64_t *)stage;
    R.dst = (uint64_t *)dst;
    R.words = (payload + 7) / 8;
    std::memcpy((void *)&s->reqs[e], &R, sizeof(R));
    __atomic_store_n(&s->records[sl].flag, 0u, __ATOMIC_RELAXED);

    SlotInfo &si = s->slot[sl];
    si = SlotInfo{};
    si.busy = true;
    si.ticket = s->next_ticket;
    si.ring_entry = e;
    si.res = res;
    si.flags = opt.flags;
    si.n = n;
    si.dev_stats_cap = dev_stats_cap;
    si.prepare_s = c->prepare_s;
    si.bytes = req_bytes;
    s->ring_busy[e] = 1;
    s->arena_used += a256(payload);
    s->inflight_bytes += req_bytes;
    s->unfinished++;
    s->pending++;
    s->active.push_back(sl);
    *ticket = s->next_ticket++;
    si.t_submit = now_s();
    // publish: every staged byte before the count the kernel polls
    __atomic_store_n(s->published, (unsigned long long)(dt + 1), __ATOMIC_RELEASE);
    return BZ_OK;
}

bz_status bz_server_poll(bz_server *s, uint64_t *tickets, bz_status *statuses, uint32_t cap, uint32_t *n_done) {
    if (!s || !n_done || (cap && (!tickets || !statuses))) return fail(BZ_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    observe_locked(s);
    uint32_t nd = 0;
    while (nd < cap && !s->finished.empty()) {
        const uint32_t sl = s->finished.front();
        s->finished.pop_front();
        SlotInfo &si = s->slot[sl];
        const bz::ServeRecord &rec = s->records[sl];
        bz_result &r = *si.res;
        bz_status st = (bz_status)rec.status;
        if (rec.ticket != si.ticket) st = BZ_EDEVICE;
        r.lower_bound = rec.lower_bound;
        r.upper_bound = rec.upper_bound;
        r.last_level = rec.last_level;
        r.combinations = rec.combinations;
        r.stats_len = rec.nstats;
        r.launches = 0;
        r.prepare_s = si.prepare_s;
        r.search_s = si.t_done - si.t_submit;
        r.kernel_s = 0;
        if (r.stats) {
            const uint32_t lim = std::min(r.stats_cap, si.dev_stats_cap);
            const uint32_t cnt = std::min(rec.nstats, lim);
            const bz::BatchStat *from = s->host_stats + (size_t)sl * s->stats_cap;
            for (uint32_t t = 0; t < cnt; ++t) {
                r.stats[t].matrix = from[t].matrix; r.stats[t].level = from[t].level;
                r.stats[t].min_weight = from[t].min_weight; r.stats[t].count_at_min = from[t].count_at_min;
                r.stats[t].combinations = from[t].combinations;
            }
            if (st == BZ_OK && rec.nstats > lim) st = BZ_ELIMIT;
        }
        if (st == BZ_OK && !(si.flags & BZ_F_NO_WITNESS) && r.witness)
            for (uint32_t w = 0; w < (si.n + 63) / 64; ++w) r.witness[w] = rec.witness[w];
        r.d = st == BZ_OK ? rec.d : 0;
        tickets[nd] = si.ticket;
        statuses[nd] = st;
        ++nd;
        __atomic_store_n(&s->records[sl].flag, 0u, __ATOMIC_RELAXED);
        s->ring_busy[si.ring_entry] = 0;
        s->inflight_bytes -= si.bytes;
        s->pending--;
        si = SlotInfo{};
        s->free_slots.push_back(sl);
    }
    *n_done = nd;
    return BZ_OK;
}

bz_status bz_server_pending(bz_server *s, uint32_t *pending) {
    if (!s || !pending) return fail(BZ_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    *pending = s->pending;
    return BZ_OK;
}

bz_status bz_server_destroy(bz_server *s, double timeout_s) {
    if (!s) return BZ_OK;
    {
        std::lock_guard<std::mutex> lk(g_live_mu);
        g_live.erase(s);
    }
    bz_status st;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        st = stop_locked(s, timeout_s > 0 ? timeout_s : 60.0);
    }
    free_server(s);
    return st;
}

}  // extern "C"
