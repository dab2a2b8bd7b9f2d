// Batched persistent search behind bz_min_distance_batch: one launch drains
// the Brouwer-Zimmermann level loop (Alg. 1 of arXiv:1911.08963) of many
// codes at once.
//
// Every code has one current task, (Gamma_j, g), at a time. Its tiles are
// handed out by a cursor word (epoch << 40 | next tile): a wave claims one tile
// with a fetch-add on that word and keeps it if the slot of that epoch says the
// tile exists. It runs the same tile code as the single-code kernel
// (bz_tile.h) and then counts the tile as finished. The wave that finishes a
// task's last tile advances the code on the device: it records the task's
// statistics, moves U, applies the certified lower bound, and either
// publishes the next task (the other of the code's two task slots, then a
// release store of the new epoch, then an entry at the end of the task log)
// or marks the code finished. This is the coordinator/worker scheme of the
// paper's dynamic algorithms (Sec. 3.2) collapsed into one GPU: the
// coordinator is whichever wave finishes last.
//
// Finding work: every code being searched has an owner, the wave that
// finished its last task, which goes straight on with the next task. A wave
// without a code first takes an unstarted one (a counter over the batch);
// when none is left it helps: tasks with at least kShareTiles tiles are also
// appended to a shared task log, which helpers walk, moving the head past
// exhausted entries. In a batch every helper starts at the head, so helpers
// converge on the oldest large task, and small tasks never leave their owner;
// the server spreads helpers over the newest entries instead. Idle waves back off
// exponentially. Waves leave when every code is finished or the cancel word is
// set.
//
// Atomics whose result the wave needs are issued once per wave: the helpers of
// bz_wave.h narrow exec to the wave's first active lane around a single global
// atomic, restore it, and readfirstlane hands the old value to every lane, so
// no lane-dependent branch surrounds that readfirstlane.
#include <hip/hip_runtime.h>

#include "bz_internal.h"
#include "bz_kernels.h"
#include "bz_tile.h"
#include "bz_wave.h"

namespace bz {

// Tasks with this many tiles are offered to helpers: the batch shares only
// large tasks (small ones stay with their owner, throughput first); the server
// shares almost every task (a request's latency is its tasks' latency).
template <bool SERVE>
constexpr uint64_t kShareTiles = SERVE ? 2 : 8;

// Log entries a server helper samples from: the newest this many.
constexpr uint64_t kServeWindow = 256;
// Tickets held ahead of the published count: a holder takes no tiles (it only
// waits for its request), so a published request starts within a poll, and
// every other wave is free to help with tiles of any length.
constexpr uint64_t kTicketsAhead = 64;

// Lower bound certified once Gamma_0..Gamma_j are done at level g and the
// later matrices at level g - 1 (j == m_f is the partial matrix).
__device__ __forceinline__ uint32_t certified_bound(uint32_t j, uint32_t g, uint32_t m_f, uint32_t k_m,
                                                    uint32_t k) {
    if (j >= m_f) {
        int e = k_m ? (int)g + 1 - (int)k + (int)k_m : 0;
        return m_f * (g + 1) + (uint32_t)(e > 0 ? e : 0);
    }
    int e = k_m ? (int)g - (int)k + (int)k_m : 0;
    return (j + 1) * (g + 1) + (m_f - j - 1) * g + (uint32_t)(e > 0 ? e : 0);
}

// A device-scope (relaxed) load: coherent across the XCDs' L2 caches.
template <typename T>
__device__ __forceinline__ T ld_agent(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One tile of a code's current task. The tile's combination count and
// statistics go to the wave's own words (LDS), which the caller adds to the
// task's once per claim. The lane setup steps with the rows' prefix XORs.
template <bool STATS>
__device__ __forceinline__ void batch_tile(const BatchArgs &b, uint32_t code, uint64_t epoch, uint64_t tile,
                                           uint32_t lane, cptr64 binom_c, const uint64_t *sb, uint32_t bt,
                                           unsigned long long *wave_words) {
    const BatchCode &D = b.codes[code];
    TaskSlot *s = &b.state[code].slot[epoch & 1];
    // The slot's fields change with every task a code runs: device-scope
    // loads read them where every XCD sees the publisher's stores, with no
    // cache invalidation per claim (the release that published the epoch
    // wrote them back first).
    const uint32_t j = uni(ld_agent(&s->j)), g = uni(ld_agent(&s->g));
    const uint32_t k = uni(D.k), m_f = uni(D.m_f);
    const bool partial = j >= m_f;
    const uint32_t W = uni(partial ? D.W_partial : D.W_full);
    const uint32_t W_full = uni(D.W_full);
    // uniform (readfirstlane): the head rows are then read with scalar loads
    // into SGPRs, as in the single-code kernel, not with vector loads
    const uint32_t *rows =
        (const uint32_t *)uni64((uint64_t)(D.rows + (size_t)(partial ? m_f : j) * (k + 1) * W_full));
    const uint32_t *px = rows + uni(D.px_delta);       // the rows' prefix XORs
    TaskArgs a{};
    a.rows = rows;
    a.binom = b.binom;
    a.rects = b.rects + uni(ld_agent(&s->rect_off));
    a.key = &s->key;
    a.ncomb = wave_words;
    a.stats = wave_words + 1;
    a.nrects = uni(ld_agent(&s->nrects));
    a.k = k;
    a.k_low = partial ? uni(D.k_m) : k;
    a.g = g;
    a.heads_per_tile = uni(ld_agent(&s->heads_per_tile));
    a.total_tiles = uni64(ld_agent(&s->tiles)) & kCursorMask;
    a.u_prev = uni(ld_agent(&s->u_prev));
    a.exit_at = uni(ld_agent(&s->exit_at));
    if (a.exit_at) {
        unsigned long long kv = __hip_atomic_load(a.key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t cur = min((uint32_t)(kv >> kTileBits), a.u_prev);
        if (uni(cur) <= a.exit_at) return;        // the bound is met: skip, still counted as done
    }
    cptr32 rc = (cptr32)rows;
    cptr_rect rp = (cptr_rect)a.rects;
    switch (W * 2 + (partial ? 1u : 0u)) {
#define BZ_CASE(WW)                                                                                   \
    case WW * 2:                                                                                      \
        run_tile<WW, slots_for_w(WW), false, STATS>(a, rc, binom_c, rows, px, sb, bt, rp, tile, lane);      \
        break;                                                                                        \
    case WW * 2 + 1:                                                                                  \
        run_tile<WW, slots_for_w(WW), true, STATS>(a, rc, binom_c, rows, px, sb, bt, rp, tile, lane);       \
        break;
        BZ_CASE(1) BZ_CASE(2) BZ_CASE(3) BZ_CASE(4) BZ_CASE(5) BZ_CASE(6) BZ_CASE(7) BZ_CASE(8)
#undef BZ_CASE
    default: break;
    }
}

template <bool STATS>
__device__ void serve_finish(const ServeArgs &sv, uint32_t code, uint32_t lane, uint32_t status, uint32_t U,
                             uint32_t L, uint32_t last_level, uint32_t nstats, uint64_t combos, uint32_t best_j,
                             uint32_t best_g, uint64_t best_tile, bool have_best);

// Appends (code, epoch) to the shared task log unless the ring is full.
__device__ __forceinline__ void log_append(const BatchArgs &b, uint32_t code, uint64_t epoch, uint32_t lane) {
    const uint64_t head = uni64(__hip_atomic_load(b.log_head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    const uint64_t tail = uni64(__hip_atomic_load(b.log_tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    if (tail - head >= b.log_cap) return;          // full: the owner runs the task alone
    const unsigned long long pos = wave_fetch_add64_relaxed(b.log_tail, 1ull);
    if (lane == 0)
        __hip_atomic_store(b.log + (pos & (b.log_cap - 1)), (unsigned long long)((((uint64_t)code) << 24) | epoch) + 1ull,
                           __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// The last wave of a task: bookkeeping of Alg. 1 for one code, then the next
// task or the end. All values are uniform; lane 0 does the stores.
template <bool STATS, bool SERVE>
__device__ void batch_advance(const BatchArgs &b, const ServeArgs *sv, uint32_t code, uint64_t epoch,
                              uint32_t lane) {
    CodeState *S = &b.state[code];
    const BatchCode &D = b.codes[code];
    TaskSlot *s = &S->slot[epoch & 1];
    const uint32_t j = uni(s->j), g = uni(s->g);
    const uint32_t k = uni(D.k), m_f = uni(D.m_f), k_m = uni(D.k_m), nsets = uni(D.nsets);
    const uint32_t flags = uni(D.flags), max_level = uni(D.max_level);
    const unsigned long long key = uni64(__hip_atomic_load(&s->key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    const unsigned long long sw = uni64(__hip_atomic_load(&s->stats, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    const unsigned long long nc = uni64(__hip_atomic_load(&s->ncomb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    const uint32_t tmin = key == ~0ull ? 0xffffffffu : (uint32_t)(key >> kTileBits);
    const uint64_t total = uni64(b.binom[(size_t)k * (kBinomT + 1) + g]);
    const bool complete = nc == total;

    uint32_t U = uni(S->U), L = uni(S->L), Lcert = uni(S->Lcert), nstats = uni(S->nstats);
    uint32_t have_best = uni(S->have_best), best_j = uni(S->best_j), best_g = uni(S->best_g);
    uint64_t best_tile = uni64(S->best_tile), combos = uni64(S->combinations) + nc;
    uint32_t last_level = uni(S->last_level), status = uni(S->status);
    if (lane == 0 && nstats < D.stats_cap) {
        BatchStat st;
        st.matrix = (uint16_t)j;
        st.level = (uint16_t)g;
        st.min_weight = tmin;
        st.count_at_min = STATS ? (sw & ((1ull << kTileBits) - 1)) : 0ull;
        st.combinations = nc;
        b.stats[D.stats_off + nstats] = st;
    }
    nstats++;
    if (tmin < U || (tmin == U && !have_best)) {
        U = tmin;
        have_best = 1; best_j = j; best_g = g; best_tile = key & kTileMask;
    }
    bool done = false;
    uint32_t nj = 0, ng = 0;
    if (!complete) {
        // a wave skips tiles only once U <= the bound certified before this task
        L = max(L, Lcert);
        done = true;
    } else {
        const uint32_t Lc = certified_bound(j, g, m_f, k_m, k);
        Lcert = max(Lcert, Lc);
        // per-Gamma stop: check after every matrix; Alg. 1 as printed: only once a level is done
        const bool check = !(flags & BZ_F_LEVEL_STOP) || j + 1 == nsets;
        if (check) L = max(L, Lc);
        if (check && L >= U) {
            done = true;
        } else {
            nj = j + 1; ng = g;
            if (nj == nsets) { nj = 0; ng = g + 1; }
            if (ng > k) {
                done = true;                                  // everything enumerated: d = U
            } else if (ng > uni(D.g_max) || (max_level && ng > max_level)) {
                done = true;
                status = (uint32_t)(int32_t)BZ_ELIMIT;
            }
        }
    }
    if (!done && ng > last_level) last_level = ng;
    if (lane == 0) {
        S->U = U; S->L = L; S->Lcert = Lcert; S->nstats = nstats;
        S->have_best = have_best; S->best_j = best_j; S->best_g = best_g; S->best_tile = best_tile;
        S->combinations = combos; S->last_level = last_level; S->status = status;
        if (!done) {
            const PlanEntry P = b.plans[(nj < m_f ? D.plan_full : D.plan_partial) + ng - 1];
            TaskSlot *n = &S->slot[(epoch + 1) & 1];
            n->key = ~0ull;
            n->stats = ~0ull;
            n->ncomb = 0;
            n->completed = 0;
            n->j = nj; n->g = ng;
            n->rect_off = P.rect_off; n->nrects = P.nrects; n->heads_per_tile = P.heads_per_tile;
            n->exit_at = STATS ? 0u : Lcert;
            n->u_prev = U;
            __hip_atomic_store(&n->tiles, (unsigned long long)(((epoch + 1) << kEpochShift) | P.total_tiles),
                               __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&S->cursor, (unsigned long long)((epoch + 1) << kEpochShift), __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_AGENT);
        } else {
            __hip_atomic_store(&S->cursor, (unsigned long long)(kDoneEpoch << kEpochShift), __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_AGENT);
            if (!SERVE) __hip_atomic_fetch_add(b.done_count, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    if (SERVE && done) {
        serve_finish<STATS>(*sv, code, lane, status, U, L, last_level, nstats, combos, best_j, best_g, best_tile,
                            have_best != 0);
        if (lane == 0) __hip_atomic_fetch_add(b.done_count, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (!done &&
        uni64(b.plans[(nj < m_f ? D.plan_full : D.plan_partial) + ng - 1].total_tiles) >= kShareTiles<SERVE>)
        log_append(b, code, epoch + 1, lane);
}

// Claims tiles [tile, tile + count) of the code's current task: one, or for a
// task of many tiles a few consecutive ones, so that the waves of one large
// task queue fewer atomics on its cursor and completion words.
constexpr uint64_t kClaim2 = 4096, kClaim4 = 16384, kClaim8 = 65536;   // tiles per task from which 2, 4, 8 per claim
__device__ __forceinline__ bool try_claim(const BatchArgs &b, uint32_t code, uint32_t lane, uint64_t &epoch,
                                          uint64_t &tile, uint64_t &count) {
    (void)lane;
    CodeState *S = b.state + code;
    const unsigned long long w0 = uni64(__hip_atomic_load(&S->cursor, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    const uint64_t e0 = w0 >> kEpochShift;
    if (e0 == kDoneEpoch) return false;
    const unsigned long long tw0 =
        uni64(__hip_atomic_load(&S->slot[e0 & 1].tiles, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    if ((tw0 >> kEpochShift) != e0 || (w0 & kCursorMask) >= (tw0 & kCursorMask)) return false;
    const uint64_t T0 = tw0 & kCursorMask;
    const uint64_t K = T0 >= kClaim8 ? 8 : (T0 >= kClaim4 ? 4 : (T0 >= kClaim2 ? 2 : 1));
    // relaxed: the claimer reads the task's slot with device-scope loads
    // (batch_tile), published before this epoch by a release store, and
    // publishes nothing by claiming
    const unsigned long long w = wave_fetch_add64_relaxed(&S->cursor, K);
    const uint64_t e = w >> kEpochShift, t = w & kCursorMask;
    if (e == kDoneEpoch) return false;
    const unsigned long long tw =
        uni64(__hip_atomic_load(&S->slot[e & 1].tiles, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    const uint64_t T = tw & kCursorMask;
    if ((tw >> kEpochShift) != e || t >= T) return false;
    epoch = e;
    tile = t;
    count = umin64(K, T - t);
    return true;
}

__device__ __forceinline__ bool entry_exhausted(const BatchArgs &b, uint32_t code, uint64_t ep) {
    CodeState *S = b.state + code;
    const unsigned long long w = uni64(__hip_atomic_load(&S->cursor, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    const uint64_t e = w >> kEpochShift;
    if (e == kDoneEpoch || e != ep) return true;
    const unsigned long long tw =
        uni64(__hip_atomic_load(&S->slot[e & 1].tiles, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    return (tw >> kEpochShift) == e && (w & kCursorMask) >= (tw & kCursorMask);
}

// XORs into cw the full rows of the t elements of the colex rank r (t-subsets
// of [off, off + nside)).
__device__ void unrank_xor(const uint64_t *binom, uint64_t r, uint32_t t, uint32_t off, uint32_t nside,
                           const uint64_t *full, uint64_t (&cw)[kHostWords]) {
    uint32_t hi = nside - 1;
    for (uint32_t i = t; i >= 1; --i) {
        uint32_t lo = i - 1, c = hi;
        while (lo < c) {
            uint32_t mid = (lo + c + 1) >> 1;
            if (binom[mid * (kBinomT + 1) + i] <= r) lo = mid; else c = mid - 1;
        }
        r -= binom[lo * (kBinomT + 1) + i];
        for (int w = 0; w < kHostWords; ++w) cw[w] ^= full[(size_t)(off + lo) * kHostWords + w];
        hi = lo - 1;
    }
}

// Writes the t elements of the colex rank r (t-subsets of [off, off + nside)) into idx.
__device__ uint32_t unrank_into(const uint64_t *binom, uint64_t r, uint32_t t, uint32_t off, uint32_t nside,
                                uint32_t *idx) {
    uint32_t hi = nside - 1;
    for (uint32_t i = t; i >= 1; --i) {
        uint32_t lo = i - 1, c = hi;
        while (lo < c) {
            uint32_t mid = (lo + c + 1) >> 1;
            if (binom[mid * (kBinomT + 1) + i] <= r) lo = mid; else c = mid - 1;
        }
        r -= binom[lo * (kBinomT + 1) + i];
        idx[t - i] = off + lo;
        hi = lo - 1;
    }
    return t;
}

// ---- one code's smallest levels in one work-group
//
// The single-code search hands its first levels, while their tasks are tiny,
// to one launch of bz_one_kernel: a single work-group, whose four waves are
// always resident together, runs the tasks (Gamma_j, g) in Alg. 1's order
// (OneTask list, fixed by the host). Each task's tiles are dealt to the waves
// round-robin; every wave keeps its key, combination count and statistics word
// in LDS; after a barrier wave 0 merges them and applies Alg. 1's bookkeeping
// (the rules of the enumeration kernel's step), and after a second barrier the
// waves go on with the next task or leave. When the search is over the four
// waves find the witness in the winning tile. Nothing but LDS and the final
// records is written, and no device-scope atomic is needed. Larger levels go
// on as launches of the enumeration kernel.

template <bool STATS>
__device__ __forceinline__ void one_tile(const OneArgs &a, const OneTask &T, uint64_t tile, uint32_t lane,
                                         cptr64 binom_c, const uint64_t *sb, uint32_t bt, const uint32_t *lrows,
                                         uint32_t u_prev, uint32_t exit_at, unsigned long long *words) {
    const bool partial = T.j >= a.m_f;
    const uint32_t *rows = (const uint32_t *)uni64((uint64_t)(a.rows + T.row_off));
    TaskArgs t{};
    t.rows = rows;
    t.binom = a.binom;
    t.rects = a.rects + T.rect_off;
    t.key = words;
    t.ncomb = words + 1;
    t.stats = words + 2;
    t.nrects = T.nrects;
    t.k = a.k;
    t.k_low = partial ? a.k_m : a.k;
    t.g = T.g;
    t.heads_per_tile = T.heads_per_tile;
    t.total_tiles = T.total_tiles;
    t.u_prev = u_prev;
    t.exit_at = exit_at;
    cptr32 rc = (cptr32)rows;
    cptr_rect rp = (cptr_rect)t.rects;
    const uint32_t *srow = lrows + T.row_off;
    const uint32_t *spx = srow + a.px_delta;
    switch (T.W * 2 + (partial ? 1u : 0u)) {
#define BZ_CASE(WW)                                                                                   \
    case WW * 2:                                                                                      \
        run_tile<WW, slots_for_w(WW), false, STATS>(t, rc, binom_c, srow, spx, sb, bt, rp, tile, lane);     \
        break;                                                                                        \
    case WW * 2 + 1:                                                                                  \
        run_tile<WW, slots_for_w(WW), true, STATS>(t, rc, binom_c, srow, spx, sb, bt, rp, tile, lane);      \
        break;
        BZ_CASE(1) BZ_CASE(2) BZ_CASE(3) BZ_CASE(4) BZ_CASE(5) BZ_CASE(6) BZ_CASE(7) BZ_CASE(8)
#undef BZ_CASE
    default: break;
    }
}

// The witness of a finished search: a combination of weight U in the winning
// tile (one wave), then the XOR of its full rows.
__device__ bool one_witness(const OneArgs &a, const OneTask &T, uint64_t tile, uint32_t U, uint32_t lane,
                            cptr64 binom_c, const uint64_t *sb, uint32_t bt, const uint32_t *lrows,
                            uint64_t (&cw)[kHostWords], uint32_t s_first, uint32_t s_step, const uint32_t *stop) {
    const bool partial = T.j >= a.m_f;
    const uint32_t *rows = (const uint32_t *)uni64((uint64_t)(a.rows + T.row_off));
    TaskArgs t{};
    t.rows = rows;
    t.rects = a.rects + T.rect_off;
    t.nrects = T.nrects;
    t.k = a.k;
    t.k_low = partial ? a.k_m : a.k;
    t.g = T.g;
    t.heads_per_tile = T.heads_per_tile;
    cptr32 rc = (cptr32)rows;
    cptr_rect rp = (cptr_rect)t.rects;
    const uint32_t *srow = lrows + T.row_off;
    TileGeom g{};
    uint64_t q = 0, h = 0;
    bool found = false;
    switch (T.W) {
#define BZ_FIND(WW)                                                                                          \
    case WW:                                                                                                 \
        found = find_in_tile<WW, slots_for_w(WW)>(t, rc, binom_c, srow, sb, bt, rp, tile, lane, U, g, q, h, \
                                                  s_first, s_step, stop);                                   \
        break;
        BZ_FIND(1) BZ_FIND(2) BZ_FIND(3) BZ_FIND(4) BZ_FIND(5) BZ_FIND(6) BZ_FIND(7) BZ_FIND(8)
#undef BZ_FIND
    default: break;
    }
    if (!found) return false;
    // the digits from the binomials in LDS (row stride bt), the rows from memory
    const uint64_t *full = a.full_rows + (size_t)T.j * a.k * kHostWords;
    auto xor_subset = [&](uint64_t r, uint32_t t, uint32_t off, uint32_t nside) {
        uint32_t hi = nside - 1;
        for (uint32_t i = t; i >= 1; --i) {
            const uint32_t c = colex_digit(sb, bt, i, i - 1, hi, r);
            r -= sb[c * bt + i];
            for (int w = 0; w < kHostWords; ++w) cw[w] ^= full[(size_t)(off + c) * kHostWords + w];
            hi = c - 1;
        }
    };
    xor_subset(q, g.lane_t, g.lane_off, g.lane_n);
    if (g.head_t) xor_subset(h, g.head_t, g.head_off, g.head_n);
    return true;
}

// Task t's fields, known to be uniform (readfirstlane): the loops they bound
// are then left by the whole wave at once.
__device__ __forceinline__ OneTask one_task(const OneTask *p) {
    OneTask T;
    T.total_tiles = uni64(p->total_tiles);
    T.comb = uni64(p->comb);
    T.j = uni(p->j); T.g = uni(p->g); T.rect_off = uni(p->rect_off); T.nrects = uni(p->nrects);
    T.heads_per_tile = uni(p->heads_per_tile); T.W = uni(p->W); T.row_off = uni(p->row_off);
    T.cert_task = uni(p->cert_task); T.cert_level = uni(p->cert_level); T.last_of_level = uni(p->last_of_level);
    T._pad[0] = T._pad[1] = 0;
    return T;
}

// Launched as a single work-group of kBlock threads. The arguments live in
// device memory (a by-value struct whose address the device functions take
// would be copied to per-lane scratch, and its fields would no longer be known
// to be uniform).
template <bool STATS, bool LDS_BINOM>
__global__ __launch_bounds__(kBlock) void bz_one_kernel(const OneArgs *__restrict__ ap, OneRun run) {
    const OneArgs &a = *ap;
    constexpr uint32_t kWaves = kBlock / kWaveSize;
    const uint32_t lane = threadIdx.x & (kWaveSize - 1);
    const uint32_t wv = uni(threadIdx.x / kWaveSize);
    extern __shared__ uint64_t one_lds[];
    uint32_t *lrows = (uint32_t *)one_lds;
    for (uint32_t i = threadIdx.x; i < a.row_words; i += blockDim.x) lrows[i] = a.rows[i];
    const uint64_t *sb = a.binom;
    uint32_t bt = kBinomT + 1;
    if (LDS_BINOM) {
        uint64_t *lb = one_lds + (a.row_words + 1) / 2;
        bt = a.lds_g + 1;
        for (uint32_t i = threadIdx.x; i < (a.k + 1) * bt; i += blockDim.x) {
            const uint32_t x = i / bt, y = i - x * bt;
            lb[i] = a.binom[x * (kBinomT + 1) + y];
        }
        sb = lb;
    }
    cptr64 binom_c = (cptr64)a.binom;
    // per wave: key, combinations, statistics word of the current task
    __shared__ unsigned long long words[kWaves][3];
    // the bounds, written by wave 0 between the barriers: U, exit_at, go on (1) or leave (0)
    __shared__ uint32_t shared_bounds[3];
    OneState *S = run.state;
    uint32_t U = a.U0, L = 1, Lcert = 1, have_best = 0, best_task = 0;
    uint64_t best_tile = 0, combos = 0;
    uint32_t status = kOneRunning, ntasks = 0;
    if (threadIdx.x == 0) {
        shared_bounds[0] = U;
        shared_bounds[1] = STATS ? 0u : Lcert;
        shared_bounds[2] = 1;
    }
    for (uint32_t t = 0; t < run.ntasks; ++t) {
        // wave 0 has read every wave's words of the previous task before this barrier
        __syncthreads();
        if (!uni(shared_bounds[2])) break;              // the search stopped (uniform for the group)
        if (lane == 0) {
            words[wv][0] = ~0ull;
            words[wv][1] = 0;
            words[wv][2] = ~0ull;
        }
        const OneTask T = one_task(a.tasks + t);
        const uint32_t u_prev = uni(shared_bounds[0]), exit_at = uni(shared_bounds[1]);
        bool canceled = false;
        if (run.cancel) canceled = uni(__hip_atomic_load(run.cancel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)) != 0;
        if (!canceled) {
            for (uint64_t tile = wv; tile < T.total_tiles; tile += kWaves) {
                if (exit_at) {
                    const uint32_t cur = min((uint32_t)(words[wv][0] >> kTileBits), u_prev);
                    if (uni(cur) <= exit_at) break;     // the bound is met
                }
                one_tile<STATS>(a, T, tile, lane, binom_c, sb, bt, lrows, u_prev, exit_at, words[wv]);
            }
        }
        __syncthreads();
        if (wv == 0) {
            // merge the waves' words, then Alg. 1's bookkeeping for task t
            unsigned long long key = ~0ull, nc = 0;
            uint32_t smin = 0xffffffffu;
            uint64_t scnt = 0;
            for (uint32_t w = 0; w < kWaves; ++w) {
                key = key < words[w][0] ? key : words[w][0];
                nc += words[w][1];
                if (STATS && words[w][2] != ~0ull) {
                    const uint32_t m = (uint32_t)(words[w][2] >> kCountBits);
                    const uint64_t c = words[w][2] & kCountMask;
                    if (m < smin) { smin = m; scnt = c; } else if (m == smin) scnt += c;
                }
            }
            const uint32_t tmin = key == ~0ull ? 0xffffffffu : (uint32_t)(key >> kTileBits);
            if (canceled) {
                // the task did not run: no record, leave
                status = kOneCanceled;
                if (lane == 0) shared_bounds[2] = 0;
                continue;
            }
            ntasks = t + 1;
            combos += nc;
            if (lane == 0) {
                BatchStat st;
                st.matrix = (uint16_t)T.j;
                st.level = (uint16_t)T.g;
                st.min_weight = tmin;
                st.count_at_min = STATS ? scnt : 0ull;
                st.combinations = nc;
                run.stats[t] = st;
            }
            if (tmin < U || (tmin == U && !have_best)) {
                U = tmin;
                have_best = 1; best_task = t; best_tile = key & kTileMask;
            }
            if (nc != T.comb) {
                // waves skip tiles only once U <= the bound certified before this task
                L = max(L, Lcert);
                status = kOneStopped;
            } else {
                Lcert = max(Lcert, T.cert_task);
                if (!run.level_stop) {
                    L = max(L, Lcert);
                    if (L >= U) status = kOneStopped;
                }
                if (status == kOneRunning && T.last_of_level) {
                    L = max(L, T.cert_level);
                    if (L >= U || T.g == a.k) status = kOneStopped;   // g == k: every combination enumerated
                }
                if (status == kOneRunning && t + 1 >= run.ntasks) status = kOneContinue;
            }
            if (lane == 0) {
                shared_bounds[0] = U;
                shared_bounds[1] = STATS ? 0u : Lcert;
                shared_bounds[2] = status == kOneRunning ? 1u : 0u;
            }
        }
    }
    // The witness: the four waves share the winning tile's slots (wave w takes
    // slots w, w + 4, ...); the first to find a combination of weight U writes
    // it, and the others leave their search at their next slot.
    __shared__ uint32_t wit_share[5];                  // status, U, have_best, best_task, found
    __shared__ unsigned long long wit_tile;
    if (wv == 0 && lane == 0) {
        wit_share[0] = status; wit_share[1] = U; wit_share[2] = have_best; wit_share[3] = best_task;
        wit_share[4] = 0;
        wit_tile = best_tile;
    }
    __syncthreads();
    if (uni(wit_share[0]) == kOneStopped && run.want_witness && uni(wit_share[2])) {
        uint64_t cw[kHostWords] = {0, 0, 0, 0};
        const bool ok = one_witness(a, one_task(a.tasks + uni(wit_share[3])), uni64(wit_tile), uni(wit_share[1]),
                                    lane, binom_c, sb, bt, lrows, cw, wv, kWaves, &wit_share[4]);
        if (ok) {
            uint32_t won = 0;
            if (lane == 0) won = atomicCAS(&wit_share[4], 0u, 1u) == 0u ? 1u : 0u;
            if (uni(won) && lane == 0)
                for (int w = 0; w < kHostWords; ++w) S->witness[w] = cw[w];
        }
    }
    __syncthreads();
    if (wv == 0 && lane == 0) {
        uint32_t wit = 0;
        if (status == kOneStopped && run.want_witness && have_best) wit = wit_share[4] ? 1u : 2u;
        S->wit_flag = wit;
        S->U = U; S->L = L; S->Lcert = Lcert; S->status = status; S->ntasks = ntasks;
        S->have_best = have_best; S->best_task = best_task; S->best_tile = best_tile;
        S->combinations = combos;
    }
}

hipError_t launch_one(const OneArgs *args, const OneRun &run, bool stats, bool lds_binom, size_t lds,
                      hipStream_t st) {
    if (stats && lds_binom)
        hipLaunchKernelGGL((bz_one_kernel<true, true>), dim3(1), dim3(kBlock), lds, st, args, run);
    else if (stats)
        hipLaunchKernelGGL((bz_one_kernel<true, false>), dim3(1), dim3(kBlock), lds, st, args, run);
    else if (lds_binom)
        hipLaunchKernelGGL((bz_one_kernel<false, true>), dim3(1), dim3(kBlock), lds, st, args, run);
    else
        hipLaunchKernelGGL((bz_one_kernel<false, false>), dim3(1), dim3(kBlock), lds, st, args, run);
    return hipGetLastError();
}

// ---- serving

__device__ __forceinline__ uint64_t sys_load64(const void *p) {
    return __hip_atomic_load((const unsigned long long *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ uint32_t sys_load32(const void *p) {
    return __hip_atomic_load((const uint32_t *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void sys_store64(void *p, uint64_t v) {
    __hip_atomic_store((unsigned long long *)p, (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void sys_store32(void *p, uint32_t v) {
    __hip_atomic_store((uint32_t *)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Copies `words` 64-bit words from pinned host memory to device memory, all lanes.
__device__ __forceinline__ void wave_copy_in(uint64_t *dst, const uint64_t *src, uint64_t words, uint32_t lane) {
    constexpr uint32_t kUnroll = 4;
    uint64_t i = lane;
    for (; i + (kUnroll - 1) * kWaveSize < words; i += kUnroll * kWaveSize) {
        uint64_t v[kUnroll];
#pragma unroll
        for (uint32_t u = 0; u < kUnroll; ++u) v[u] = sys_load64(src + i + u * kWaveSize);
#pragma unroll
        for (uint32_t u = 0; u < kUnroll; ++u) dst[i + u * kWaveSize] = v[u];
    }
    for (; i < words; i += kWaveSize) dst[i] = sys_load64(src + i);
}

constexpr uint64_t kPollTicks = 500;          // wall-clock ticks between polls of the host words (5 us at 100 MHz)

// The wave's view of the host's published count and shutdown word. Device
// copies are read every time, relaxed (every wave reads them every round; an
// acquire would invalidate the caches the working waves read from): a wave
// that acts on a new ticket takes an acquire fence first. At most one wave per
// kPollTicks reads the host words (pinned memory across the bus) and
// refreshes them.
__device__ __forceinline__ void serve_view(const ServeArgs &sv, uint32_t lane, uint64_t &pub, uint32_t &stop) {
    unsigned long long *v = sv.view;
    stop = uni((uint32_t)__hip_atomic_load(v + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    pub = uni64(__hip_atomic_load(v + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    const uint64_t now = uni64(wall_clock64());
    const uint64_t last = uni64(__hip_atomic_load(v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    if (now - last <= kPollTicks || now < last) return;
    const uint64_t old = wave_fetch_max64_old(v, now);
    if (now - old <= kPollTicks || now < old) return;     // another wave polls
    // the host raises published before it sets shutdown: read them in the other order
    const uint32_t s = uni(__hip_atomic_load(sv.shutdown, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM));
    const uint64_t p = uni64(__hip_atomic_load(sv.published, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM));
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    wave_fetch_max64(v + 1, p);
    if (s && lane == 0) __hip_atomic_store(v + 2, (unsigned long long)s, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    if (p > pub) pub = p;
    if (s > stop) stop = s;
}

// The wave holding ticket t brings request t onto the device: payload, new
// plan tables, the code's description and its first task. The request's code
// index is its ticket. Returns false (nothing started) only when told to stop
// at once while waiting for another request's plan tables.
template <bool STATS>
__device__ bool serve_start(const ServeArgs &sv, uint64_t ticket, uint32_t lane) {
    const BatchArgs &b = sv.b;
    const ServeReq *R = sv.reqs + (ticket & (sv.ring - 1));
    const uint32_t slot = (uint32_t)ticket;
    const uint64_t *src = (const uint64_t *)uni64(sys_load64(&R->src));
    uint64_t *dst = (uint64_t *)uni64(sys_load64(&R->dst));
    const uint64_t words = uni64(sys_load64(&R->words));
    wave_copy_in(dst, src, words, lane);
    // the code description (BatchCode is a whole number of 64-bit words)
    static_assert(sizeof(BatchCode) % 8 == 0, "BatchCode is copied as 64-bit words");
    wave_copy_in((uint64_t *)(b.codes + slot), (const uint64_t *)&R->code, sizeof(BatchCode) / 8, lane);
    for (int p = 0; p < 2; ++p) {
        const uint32_t pid = uni(sys_load32(&R->plan_copy[p]));
        if (pid == kNoPlan) continue;
        const ServePlanDesc *pd = sv.plan_desc + pid;
        const uint32_t eo = uni(sys_load32(&pd->entry_off)), lv = uni(sys_load32(&pd->levels));
        const uint32_t ro = uni(sys_load32(&pd->rect_off)), nr = uni(sys_load32(&pd->nrects));
        static_assert(sizeof(PlanEntry) % 8 == 0 && sizeof(Rect) % 8 == 0, "plan tables copy as words");
        wave_copy_in((uint64_t *)(b.plans + eo), (const uint64_t *)(sv.host_plans + eo),
                     (uint64_t)lv * sizeof(PlanEntry) / 8, lane);
        wave_copy_in((uint64_t *)(b.rects + ro), (const uint64_t *)(sv.host_rects + ro),
                     (uint64_t)nr * sizeof(Rect) / 8, lane);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (lane == 0) __hip_atomic_store(sv.plan_ready + pid, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    for (int p = 0; p < 2; ++p) {
        const uint32_t pid = uni(sys_load32(&R->plan_wait[p]));
        if (pid == kNoPlan) continue;
        // copied in by the wave of an earlier ticket, which never waits on a later one
        while (!uni(__hip_atomic_load(sv.plan_ready + pid, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT))) {
            if (uni(__hip_atomic_load(sv.shutdown, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)) >= 2) return false;
            __builtin_amdgcn_s_sleep(8);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
    const BatchCode &D = b.codes[slot];
    const uint32_t n = uni(D.n), k = uni(D.k);
    CodeState *S = b.state + slot;
    const uint32_t U0 = n - k + 1;
    if (k == n) {
        // the whole space: d = 1, no enumeration
        if (lane == 0) {
            S->U = 1; S->L = 1; S->Lcert = 1; S->status = 0; S->last_level = 0; S->nstats = 0;
            S->have_best = 0; S->best_j = 0; S->best_g = 0; S->best_tile = 0; S->combinations = 0;
            __hip_atomic_store(&S->cursor, (unsigned long long)(kDoneEpoch << kEpochShift), __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        serve_finish<STATS>(sv, slot, lane, 0u, 1u, 1u, 0u, 0u, 0ull, 0u, 0u, 0ull, false);
        if (lane == 0) __hip_atomic_fetch_add(b.done_count, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        return true;
    }
    const PlanEntry P = b.plans[uni(D.plan_full)];
    if (lane == 0) {
        S->U = U0; S->L = 1; S->Lcert = 1; S->status = 0; S->last_level = 1; S->nstats = 0;
        S->have_best = 0; S->best_j = 0; S->best_g = 0; S->best_tile = 0; S->combinations = 0;
        TaskSlot *t = &S->slot[0];
        t->key = ~0ull; t->stats = ~0ull; t->ncomb = 0; t->completed = 0;
        t->j = 0; t->g = 1; t->rect_off = P.rect_off; t->nrects = P.nrects; t->heads_per_tile = P.heads_per_tile;
        t->exit_at = STATS ? 0u : 1u;
        t->u_prev = U0;
        __hip_atomic_store(&t->tiles, (unsigned long long)P.total_tiles, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&S->cursor, 0ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (uni64(P.total_tiles) >= kShareTiles<true>) log_append(b, slot, 0, lane);
    return true;
}

// The persistent loop shared by the batch (a fixed set of codes, started
// through a counter) and the server (requests published while it runs,
// started by the wave holding their ticket).
template <bool STATS, bool SERVE, bool LDS_BINOM>
__device__ __forceinline__ void queue_loop(const BatchArgs &b, const ServeArgs *sv) {
    const uint32_t lane = threadIdx.x & (kWaveSize - 1);
    cptr64 binom_c = (cptr64)b.binom;
    // The lane setup's binomials: from the work-group's LDS when the launch
    // staged them there (they do not depend on the code), else from memory.
    const uint64_t *sb = b.binom;
    uint32_t bt = kBinomT + 1;
    if (LDS_BINOM) {
        extern __shared__ uint64_t sbin_lds[];
        const uint32_t bk = b.lds_k, bg = b.lds_g;
        bt = bg + 1;
        for (uint32_t i = threadIdx.x; i < (bk + 1) * bt; i += blockDim.x) {
            const uint32_t x = i / bt, y = i - x * bt;
            sbin_lds[i] = b.binom[x * (kBinomT + 1) + y];
        }
        __syncthreads();
        sb = sbin_lds;
    }
    constexpr uint32_t kNone = 0xffffffffu;
    constexpr uint64_t kNoTicket = ~0ull;
    uint32_t cur = kNone;                              // the code this wave owns or helps
    uint32_t fenced = kNone;                           // serving: the last request this wave acquired
    uint32_t idle = 0;                                 // consecutive rounds without work
    uint64_t ticket = kNoTicket;                       // serving: the request this wave will start
    uint64_t spread = uni64(((uint64_t)blockIdx.x << 8) ^ (threadIdx.x >> 6) ^ 0x9e3779b97f4a7c15ull);
    __shared__ unsigned long long wave_words[kBlock / kWaveSize][2];   // per wave: combinations, statistics
    const uint32_t wv = uni(threadIdx.x / kWaveSize);
    for (;;) {
        uint64_t pub = 0;
        if (SERVE) {
            uint32_t stop = 0;
            serve_view(*sv, lane, pub, stop);
            if (stop >= 2) break;
            if (stop == 1 &&
                uni(__hip_atomic_load(b.done_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) >= pub)
                break;
        } else {
            // relaxed: leaving needs no data (the launch's end orders the results)
            const uint32_t dc = uni(__hip_atomic_load(b.done_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            if (dc >= b.ncodes) break;
            if (b.cancel) {
                uint32_t cv = __hip_atomic_load(b.cancel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                if (uni(cv)) break;
            }
        }
        bool got = false;
        uint32_t code = 0;
        uint64_t epoch = 0, tile = 0, count = 1;
        if (SERVE && ticket != kNoTicket && ticket < pub) {
            // a new request first: its latency starts at publication (the
            // acquire pairs with the release that published the view's count)
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            const bool started = serve_start<STATS>(*sv, ticket, lane);
            const uint32_t c = (uint32_t)ticket;
            ticket = kNoTicket;
            if (!started) continue;                    // stopping: the loop's top leaves
            if (try_claim(b, c, lane, epoch, tile, count)) {
                got = true;
                code = cur = c;
            }
        }
        if (!got && cur != kNone) {
            got = try_claim(b, cur, lane, epoch, tile, count);
            if (got) code = cur; else cur = kNone;
        }
        if (SERVE) {
            if (!got && ticket == kNoTicket &&
                uni64(__hip_atomic_load(b.next_code, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) <
                    pub + kTicketsAhead) {
                // tickets past the launch's capacity are never published
                ticket = wave_fetch_add64_relaxed(b.next_code, 1ull);
                if (ticket < pub) continue;
            }
        } else {
            // an unstarted code
            while (!got &&
                   uni64(__hip_atomic_load(b.next_code, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) < b.ncodes) {
                const unsigned long long nc = wave_fetch_add64_relaxed(b.next_code, 1ull);
                if (nc >= b.ncodes) break;
                if (try_claim(b, (uint32_t)nc, lane, epoch, tile, count)) {
                    got = true;
                    code = cur = (uint32_t)nc;
                }
            }
        }
        if (!got && !(SERVE && ticket != kNoTicket)) {
            // Help with a task in the log. Batch: walk from the oldest entry
            // (throughput). Server: in 7 rounds of 8, start at a pseudo-random
            // entry among the newest kServeWindow and walk forward, wrapping
            // inside them: every live task re-enters the log when it starts, so
            // live entries are recent, while the head can sit behind one long
            // task with thousands of finished entries after it. Helpers spread
            // over the active tasks (close to processor sharing). In the other
            // round a server wave walks from the head, which moves the head past
            // finished entries.
            const uint64_t head = uni64(__hip_atomic_load(b.log_head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            const uint64_t end =
                uni64(__hip_atomic_load(b.log_tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            uint64_t lo = head, off = 0;                          // walk [lo, end) from lo + off
            if (SERVE && end > head + 1) {
                spread = spread * 6364136223846793005ull + 1442695040888963407ull;   // per-wave LCG
                if ((spread >> 61) != 0) {
                    lo = end - umin64(end - head, kServeWindow);
                    off = (((spread >> 16) & 0xffffffffull) * (end - lo)) >> 32;    // in [0, end - lo)
                }
            }
            const uint64_t range = end > lo ? end - lo : 0;
            const uint32_t nsteps = (uint32_t)umin64(64, range);
            for (uint32_t steps = 0; steps < nsteps && !got; ++steps) {
                const uint64_t q = lo + off;
                off = (off + 1 == range) ? 0 : off + 1;
                // relaxed: an entry only names a (code, epoch); try_claim validates it
                const unsigned long long ent = uni64(
                    __hip_atomic_load(b.log + (q & (b.log_cap - 1)), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                if (ent == 0) break;                              // being written
                const uint32_t cc = (uint32_t)((ent - 1) >> 24);
                const uint64_t ep = (ent - 1) & ((1ull << 24) - 1);
                if (cc >= b.ncodes || entry_exhausted(b, cc, ep)) {
                    // move the shared head past it (it only ever moves forward)
                    if (q == uni64(__hip_atomic_load(b.log_head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)))
                        wave_fetch_max64(b.log_head, q + 1);
                    continue;
                }
                if (try_claim(b, cc, lane, epoch, tile, count)) {
                    got = true;
                    code = cur = cc;
                }
            }
        }
        if (!got) {
            // exponential back-off (batch: up to ~110 us, serving: ~27 us, a
            // ticket holder ~3.4 us): idle waves must not crowd the few cache
            // lines the working waves claim and complete tiles on
            constexpr uint32_t kMaxShift = SERVE ? 3 : 5;
            if (SERVE && ticket != kNoTicket) {
                __builtin_amdgcn_s_sleep(127);
                continue;
            }
            const uint32_t rounds = 1u << (idle < kMaxShift ? idle : kMaxShift);
            for (uint32_t r = 0; r < rounds; ++r) __builtin_amdgcn_s_sleep(127);
            ++idle;
            continue;
        }
        idle = 0;
        if (SERVE && code != fenced) {
            // a request's code description, rows and plan tables are written
            // while the server runs: a wave acquires once before its first
            // tile of each request (the acquire pairs with the release that
            // published the request's first task)
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            fenced = code;
        }
        // the claim's count and statistics: the wave's LDS words, then one
        // atomic each on the task's words before the completion count
        if (lane == 0) {
            wave_words[wv][0] = 0;
            wave_words[wv][1] = ~0ull;
        }
        for (uint64_t i = 0; i < count; ++i)
            batch_tile<STATS>(b, code, epoch, tile + i, lane, binom_c, sb, bt, wave_words[wv]);
        TaskSlot *s = &b.state[code].slot[epoch & 1];
        if (lane == 0 && wave_words[wv][0]) {
            atomicAdd(&s->ncomb, wave_words[wv][0]);
            if (STATS) {
                const unsigned long long sw = wave_words[wv][1];
                stats_merge(&s->stats, (uint32_t)(sw >> kCountBits), sw & kCountMask);
            }
        }
        const uint64_t T = uni64(ld_agent(&s->tiles)) & kCursorMask;
        // The claim's count and statistics (atomics) are performed before the
        // completion count; the wave has no plain stores to publish (its
        // words are in LDS), so no cache write-back is needed.
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        const unsigned long long prev = wave_fetch_add64_relaxed(&s->completed, count);
        if (prev + count == T) {
            // the last wave reads the code's state the previous advance wrote
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            batch_advance<STATS, SERVE>(b, sv, code, epoch, lane);
        }
    }
}

// The arguments of both persistent kernels live in device memory: passed by
// value, their address (taken by the rare paths) would force a copy into
// per-lane scratch.
// The batch kernel's register budget: at least 3 waves per SIMD. Forcing 4
// or 5 made the 4096-code batch slower (0.78 s kernel at 3, 0.81 s at 4,
// 0.84 s at 5: spilled registers in the wider row variants).
template <bool STATS, bool LDS_BINOM>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3))) void bz_batch_kernel(
    const BatchArgs *__restrict__ b) {
    queue_loop<STATS, false, LDS_BINOM>(*b, nullptr);
}

// Three waves per SIMD: left to itself the compiler gives the fast variant 222
// VGPRs (two waves) once the lane setup steps with prefix XORs; capped it fits
// in 167 with no more spill than before.
template <bool STATS>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3))) void bz_serve_kernel(
    const ServeArgs *__restrict__ sv) {
    queue_loop<STATS, true, false>(sv->b, sv);
}

// A finished request: its statistics and witness (found by this wave in the
// winning tile) go to its completion record in host memory, flag last.
template <bool STATS>
__device__ void serve_finish(const ServeArgs &sv, uint32_t code, uint32_t lane, uint32_t status, uint32_t U,
                             uint32_t L, uint32_t last_level, uint32_t nstats, uint64_t combos, uint32_t best_j,
                             uint32_t best_g, uint64_t best_tile, bool have_best) {
    const BatchArgs &b = sv.b;
    const BatchCode &D = b.codes[code];
    const uint32_t hs = uni(D.slot);
    ServeRecord *rec = sv.records + hs;
    // task statistics: device copy -> host, three words per entry
    {
        static_assert(sizeof(BatchStat) == 24, "BatchStat is three words");
        const uint32_t ns = min(nstats, uni(D.stats_cap));
        const uint64_t *from = (const uint64_t *)(b.stats + uni(D.stats_off));
        uint64_t *to = (uint64_t *)(sv.host_stats + (size_t)hs * sv.stats_cap);
        for (uint32_t i = lane; i < ns * 3; i += kWaveSize) sys_store64(to + i, from[i]);
    }
    uint64_t cw[kHostWords] = {0, 0, 0, 0};
    uint32_t st = status;
    const uint32_t k = uni(D.k), n = uni(D.n);
    if (st == 0 && k == n) {
        // d = 1: any row of Gamma_1
        for (int w = 0; w < kHostWords; ++w) cw[w] = D.full_rows[w];
    } else if (st == 0 && have_best && !(uni(D.flags) & BZ_F_NO_WITNESS)) {
        const uint32_t m_f = uni(D.m_f);
        const bool partial = best_j >= m_f;
        const uint32_t W = uni(partial ? D.W_partial : D.W_full);
        const uint32_t *rows = D.rows + (size_t)(partial ? m_f : best_j) * (k + 1) * uni(D.W_full);
        const PlanEntry P = b.plans[(partial ? D.plan_partial : D.plan_full) + best_g - 1];
        TaskArgs a{};
        a.rows = rows;
        a.rects = b.rects + P.rect_off;
        a.nrects = P.nrects;
        a.k = k;
        a.k_low = partial ? uni(D.k_m) : k;
        a.g = best_g;
        a.heads_per_tile = P.heads_per_tile;
        cptr32 rc = (cptr32)rows;
        cptr64 binom_c = (cptr64)b.binom;
        cptr_rect rp = (cptr_rect)a.rects;
        TileGeom t{};
        uint64_t q = 0, h = 0;
        bool found = false;
        switch (W) {
#define BZ_FIND(WW)                                                                                            \
    case WW:                                                                                                   \
        found = find_in_tile<WW, slots_for_w(WW)>(a, rc, binom_c, rows, b.binom, kBinomT + 1, rp, best_tile,   \
                                                  lane, U, t, q, h);                                           \
        break;
            BZ_FIND(1) BZ_FIND(2) BZ_FIND(3) BZ_FIND(4) BZ_FIND(5) BZ_FIND(6) BZ_FIND(7) BZ_FIND(8)
#undef BZ_FIND
        default: break;
        }
        if (found) {
            const uint64_t *full = D.full_rows + (size_t)best_j * k * kHostWords;
            unrank_xor(b.binom, q, t.lane_t, t.lane_off, t.lane_n, full, cw);
            if (t.head_t) unrank_xor(b.binom, h, t.head_t, t.head_off, t.head_n, full, cw);
        } else {
            st = (uint32_t)(int32_t)BZ_EDEVICE;
        }
    }
    if (lane == 0) {
        sys_store32(&rec->status, st);
        sys_store32(&rec->d, st == 0 ? U : 0u);
        sys_store32(&rec->lower_bound, L);
        sys_store32(&rec->upper_bound, U);
        sys_store32(&rec->last_level, last_level);
        sys_store32(&rec->nstats, nstats);
        sys_store64(&rec->ticket, D.tag);
        sys_store64(&rec->combinations, combos);
        sys_store64(&rec->t_done, wall_clock64());
        for (int w = 0; w < kHostWords; ++w) sys_store64(&rec->witness[w], cw[w]);
    }
    // every lane's stores (the statistics) before the flag
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
    if (lane == 0) __hip_atomic_store(&rec->flag, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Witness of each finished code: one work-group per code re-scans the winning
// tile. Its lane subsets' sums go to LDS first; then every thread takes head
// steps, builds the head sum from scratch, and compares every lane sum
// against the target weight. The first match writes the row indices and the
// codeword (XOR of the full rows).
constexpr int kRecoverLanes = kWaveSize * 16;


__global__ __launch_bounds__(kBlock) void bz_batch_recover_kernel(BatchArgs b) {
    __shared__ uint32_t sP[kRecoverLanes * kMaxW];
    __shared__ uint32_t sLow[kRecoverLanes];
    __shared__ uint32_t sFound;
    const uint32_t code = blockIdx.x;
    const CodeState *S = b.state + code;
    const BatchCode &D = b.codes[code];
    BatchRecover *out = b.recover + code;
    if (S->status != 0 || !S->have_best || D.k == D.n) return;   // uniform per block
    const uint32_t j = S->best_j, g = S->best_g, k = D.k;
    (void)g;
    const bool partial = j >= D.m_f;
    const uint32_t W = partial ? D.W_partial : D.W_full;
    const uint32_t k_low = partial ? D.k_m : k;
    const uint32_t *rows = D.rows + (size_t)(partial ? D.m_f : j) * (k + 1) * D.W_full;
    const uint64_t *full = D.full_rows + (size_t)j * k * kHostWords;
    const PlanEntry P = b.plans[(partial ? D.plan_partial : D.plan_full) + g - 1];
    const Rect *rects = b.rects + P.rect_off;
    const uint64_t tile = S->best_tile;
    uint32_t lo = 0, hi = P.nrects - 1;
    while (lo < hi) {
        uint32_t mid = (lo + hi + 1) >> 1;
        if (rects[mid].tile_begin <= tile) lo = mid; else hi = mid - 1;
    }
    const Rect R = rects[lo];
    const uint64_t local = tile - R.tile_begin;
    const uint64_t lb = local / R.head_blocks, hb = local - lb * R.head_blocks;
    // batch and serving tilings keep one lane block per tile (lane_mult 1)
    const uint32_t lane_items = kWaveSize * slots_for_w(W);
    const uint64_t q0 = lb * lane_items;
    const uint32_t nl = (uint32_t)((R.lane_count - q0) < lane_items ? (R.lane_count - q0) : lane_items);
    const uint64_t h0 = hb * P.heads_per_tile;
    const uint32_t nh = (uint32_t)((R.head_count - h0) < P.heads_per_tile ? (R.head_count - h0) : P.heads_per_tile);
    uint32_t idx[kBinomT];
    for (uint32_t q = threadIdx.x; q < nl; q += blockDim.x) {
        unrank_into(b.binom, q0 + q, R.lane_t, R.lane_off, R.lane_n, idx);
        uint32_t low = 0;
        for (uint32_t w = 0; w < W; ++w) sP[q * kMaxW + w] = 0;
        for (uint32_t i = 0; i < R.lane_t; ++i) {
            for (uint32_t w = 0; w < W; ++w) sP[q * kMaxW + w] ^= rows[idx[i] * W + w];
            low += idx[i] < k_low ? 1u : 0u;
        }
        sLow[q] = low;
    }
    if (threadIdx.x == 0) sFound = 0;
    __syncthreads();
    const uint32_t target = S->U;
    for (uint32_t h = threadIdx.x; h < nh; h += blockDim.x) {
        if (__hip_atomic_load(&sFound, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) break;
        uint32_t H[kMaxW];
        for (uint32_t w = 0; w < kMaxW; ++w) H[w] = 0;
        uint32_t hl = 0;
        if (R.head_t) {
            unrank_into(b.binom, h0 + h, R.head_t, R.head_off, R.head_n, idx);
            for (uint32_t i = 0; i < R.head_t; ++i) {
                for (uint32_t w = 0; w < W; ++w) H[w] ^= rows[idx[i] * W + w];
                hl += idx[i] < k_low ? 1u : 0u;
            }
        }
        for (uint32_t q = 0; q < nl; ++q) {
            // identity part: rows below k_low (every row of a full-rank Gamma_j)
            uint32_t wt = sLow[q] + hl;
            for (uint32_t w = 0; w < W; ++w) wt += __builtin_popcount(sP[q * kMaxW + w] ^ H[w]);
            if (wt != target) continue;
            if (atomicCAS(&sFound, 0u, 1u) != 0u) break;
            // rebuild the combination's row indices and the codeword
            uint32_t n_idx = 0;
            uint32_t all[kBinomT];
            n_idx += unrank_into(b.binom, q0 + q, R.lane_t, R.lane_off, R.lane_n, all);
            if (R.head_t) n_idx += unrank_into(b.binom, h0 + h, R.head_t, R.head_off, R.head_n, all + n_idx);
            uint64_t cw[kHostWords];
            for (int w = 0; w < kHostWords; ++w) cw[w] = 0;
            for (uint32_t i = 0; i < n_idx; ++i)
                for (int w = 0; w < kHostWords; ++w) cw[w] ^= full[(size_t)all[i] * kHostWords + w];
            for (int w = 0; w < kHostWords; ++w) out->codeword[w] = cw[w];
            for (uint32_t i = 0; i < n_idx; ++i) out->indices[i] = all[i];
            out->len = n_idx;
            __hip_atomic_store(&out->flag, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            break;
        }
    }
}

template <bool STATS>
static hipError_t launch_batch_t(const BatchArgs *b, uint32_t grid, size_t lds, hipStream_t st) {
    if (lds)
        hipLaunchKernelGGL((bz_batch_kernel<STATS, true>), dim3(grid), dim3(kBlock), lds, st, b);
    else
        hipLaunchKernelGGL((bz_batch_kernel<STATS, false>), dim3(grid), dim3(kBlock), 0, st, b);
    return hipGetLastError();
}

hipError_t launch_batch(const BatchArgs *b, uint32_t grid, bool stats, size_t lds_bytes, hipStream_t st) {
    return stats ? launch_batch_t<true>(b, grid, lds_bytes, st) : launch_batch_t<false>(b, grid, lds_bytes, st);
}

template <bool STATS>
static hipError_t launch_serve_t(const ServeArgs *sv, uint32_t grid, hipStream_t st) {
    hipLaunchKernelGGL((bz_serve_kernel<STATS>), dim3(grid), dim3(kBlock), 0, st, sv);
    return hipGetLastError();
}

hipError_t launch_serve(const ServeArgs *sv, uint32_t grid, bool stats, hipStream_t st) {
    return stats ? launch_serve_t<true>(sv, grid, st) : launch_serve_t<false>(sv, grid, st);
}

int serve_blocks_per_cu(bool stats) {
    int n = 0;
    hipError_t e = stats ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, bz_serve_kernel<true>, kBlock, 0)
                         : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, bz_serve_kernel<false>, kBlock, 0);
    return (e == hipSuccess && n > 0) ? n : 1;
}

int batch_blocks_per_cu(bool stats, size_t lds) {
    int n = 0;
    hipError_t e;
    if (lds)
        e = stats ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, bz_batch_kernel<true, true>, kBlock, lds)
                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, bz_batch_kernel<false, true>, kBlock, lds);
    else
        e = stats ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, bz_batch_kernel<true, false>, kBlock, 0)
                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, bz_batch_kernel<false, false>, kBlock, 0);
    return (e == hipSuccess && n > 0) ? n : 1;
}

hipError_t launch_batch_recover(const BatchArgs &b, hipStream_t st) {
    hipLaunchKernelGGL(bz_batch_recover_kernel, dim3(b.ncodes), dim3(kBlock), 0, st, b);
    return hipGetLastError();
}

}  // namespace bz
