// Host preparation of a code (Sec. 2.1 of arXiv:1911.08963): disjoint
// information sets and the systematic matrices Gamma_j, then the bit-packed
// device form of each Gamma_j.
//
// Information sets are found column by column: a column joins the current set
// when it is independent of the columns already in it. Independence is
// tested by reducing the column (a k-bit vector) against a GF(2) basis indexed
// by leading bit. Scanning the available columns in ascending order gives the
// greedy (first) basis. This is repeated on the remaining columns while they
// still have rank k.
//
// Sec. 2.2 tries random column permutations to find better sets. With
// perm_trials > 1 the scan above runs once per trial t, over the columns in
// the order p_t: p_0 is the identity, and for t >= 1 p_t is a Fisher-Yates
// shuffle (for i = n-1 down to 1, swap positions i and x mod (i+1)) driven by
// SplitMix64 (Steele, Lea, Flood 2014) from state perm_seed + t. The trial
// with the most full-rank sets, then the largest leftover rank, wins (the
// first on ties); each set is then sorted ascending.
//
// Gamma_j is G brought to reduced echelon form with S_j's columns taken as
// pivots first (in ascending order), then the other columns ascending. For a
// full-rank S_j this puts I_k on S_j. For the leftover set it gives the block
// form [[I_{k_m}, A], [0, B]] of Sec. 2.1. The reduced echelon form for a
// given column order is unique, so Gamma_j is well defined.
#include <algorithm>
#include <chrono>
#include <cstring>

#include "bz_internal.h"

namespace bz {
namespace {

using ColVec = std::array<uint64_t, kHostWords>;   // a k-bit column, k <= 256

inline bool bit(const HostRow &r, uint32_t c) { return (r[c >> 6] >> (c & 63)) & 1u; }

// The highest set bit of the first kw words of v, or -1.
int leading_bit(const ColVec &v, int kw) {
    for (int w = kw - 1; w >= 0; --w)
        if (v[w]) return w * 64 + 63 - __builtin_clzll(v[w]);
    return -1;
}

// A GF(2) basis of k-bit vectors, one slot per leading bit (vectors of
// kw = ceil(k / 64) words; the words above are zero).
struct XorBasis {
    std::vector<ColVec> slot;
    std::vector<char> used;
    int kw;
    explicit XorBasis(uint32_t k) : slot(k), used(k, 0), kw((int)((k + 63) / 64)) {}
    // Inserts v; returns true iff v was independent of the basis.
    bool insert(ColVec v) {
        for (;;) {
            int lb = leading_bit(v, kw);
            if (lb < 0) return false;
            if (!used[lb]) { slot[lb] = v; used[lb] = 1; return true; }
            for (int w = 0; w < kw; ++w) v[w] ^= slot[lb][w];
        }
    }
};

// In-place transpose of a 64 x 64 bit matrix (bit c of a[r] <-> bit r of
// a[c]): off-diagonal blocks of 32, then 16, ... 1 bits are swapped.
void transpose64(uint64_t (&a)[64]) {
    uint64_t m = 0x00000000FFFFFFFFull;
    for (uint32_t j = 32; j != 0; j >>= 1, m ^= m << j)
        for (uint32_t r = 0; r < 64; r = (r + j + 1) & ~j) {
            const uint64_t t = ((a[r] >> j) ^ a[r + j]) & m;
            a[r + j] ^= t;
            a[r] ^= t << j;
        }
}

// Reduced echelon form of rows under a column order (rows of nw words).
// Returns the rank.
uint32_t reduce(std::vector<HostRow> &rows, const std::vector<uint32_t> &order, uint32_t nw) {
    uint32_t k = (uint32_t)rows.size(), r = 0;
    for (uint32_t c : order) {
        if (r == k) break;
        uint32_t p = r;
        while (p < k && !bit(rows[p], c)) ++p;
        if (p == k) continue;
        std::swap(rows[p], rows[r]);
        // without branches on the data (random bits would mispredict half the time)
        for (uint32_t i = 0; i < k; ++i) {
            const uint64_t m = (uint64_t)0 - (uint64_t)(bit(rows[i], c) && i != r);
            for (uint32_t w = 0; w < nw; ++w) rows[i][w] ^= rows[r][w] & m;
        }
        ++r;
    }
    return r;
}

// SplitMix64: advance the state by the golden gamma, then mix.
uint64_t splitmix64(uint64_t &state) {
    uint64_t z = (state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

std::vector<uint32_t> scan_order(uint32_t n, uint32_t trial, uint64_t seed) {
    std::vector<uint32_t> p(n);
    for (uint32_t c = 0; c < n; ++c) p[c] = c;
    if (trial == 0) return p;
    uint64_t st = seed + trial;
    for (uint32_t i = n - 1; i >= 1; --i) std::swap(p[i], p[splitmix64(st) % (uint64_t)(i + 1)]);
    return p;
}

// Greedy disjoint information sets, scanning the columns in `scan`.
struct SetChoice {
    std::vector<std::vector<uint32_t>> sets;
    uint32_t num_full = 0, partial = 0;
};

SetChoice find_sets(const std::vector<ColVec> &col, uint32_t k, const std::vector<uint32_t> &scan) {
    const uint32_t n = (uint32_t)col.size();
    SetChoice r;
    std::vector<char> taken(n, 0);
    for (;;) {
        XorBasis basis(k);
        std::vector<uint32_t> S;
        for (uint32_t t = 0; t < n && S.size() < k; ++t) {
            const uint32_t cc = scan[t];
            if (!taken[cc] && basis.insert(col[cc])) S.push_back(cc);
        }
        std::sort(S.begin(), S.end());
        if (S.size() == k) {
            for (uint32_t cc : S) taken[cc] = 1;
            r.sets.push_back(S);
            ++r.num_full;
            continue;
        }
        r.partial = (uint32_t)S.size();
        if (r.partial) r.sets.push_back(S);
        break;
    }
    return r;
}

}  // namespace

uint64_t binom_sat(uint32_t a, uint32_t b) {
    if (b > a) return 0;
    if (b > a - b) b = a - b;
    unsigned __int128 r = 1;
    for (uint32_t i = 1; i <= b; ++i) {
        r = r * (a - b + i) / i;
        if (r >= ((unsigned __int128)1 << 63)) return kBinomSat;
    }
    return (uint64_t)r;
}

bz_status prepare_host(const uint64_t *G, uint32_t k, uint32_t n, uint32_t ld,
                       const bz_prepare_opts *opts, bz_code &c, std::string &err) {
    if (!G) { err = "G is null"; return BZ_EINVAL; }
    if (k == 0 || k > n || n > (uint32_t)kMaxN) { err = "need 0 < k <= n <= BZ_MAX_N"; return BZ_EINVAL; }
    if (ld < (n + 63) / 64) { err = "ld_words < ceil(n/64)"; return BZ_EINVAL; }
    if (opts && opts->perm_trials > 100000) { err = "perm_trials above 100000"; return BZ_EINVAL; }
    if (opts && (opts->flags & ~(uint32_t)BZ_PREPARE_HOST_ONLY)) { err = "unknown prepare flag"; return BZ_EINVAL; }

    const uint32_t nw = (n + 63) / 64;
    std::vector<HostRow> rows(k);
    for (uint32_t i = 0; i < k; ++i) {
        rows[i].fill(0);
        for (uint32_t w = 0; w < nw; ++w) rows[i][w] = G[(size_t)i * ld + w];
        if (n & 63) rows[i][nw - 1] &= (1ull << (n & 63)) - 1;      // bits past column n - 1
    }
    // columns as k-bit vectors
    std::vector<ColVec> col(n);
    for (uint32_t cc = 0; cc < n; ++cc) col[cc].fill(0);
    for (uint32_t ib = 0; ib * 64 < k; ++ib)
        for (uint32_t w = 0; w < nw; ++w) {
            uint64_t a[64];
            for (uint32_t r = 0; r < 64; ++r) a[r] = ib * 64 + r < k ? rows[ib * 64 + r][w] : 0;
            transpose64(a);
            for (uint32_t r = 0; r < 64 && w * 64 + r < n; ++r) col[w * 64 + r][ib] = a[r];
        }
    const uint32_t trials = (opts && opts->perm_trials > 1) ? opts->perm_trials : 1;
    const uint64_t seed = opts ? opts->perm_seed : 0;
    SetChoice best = find_sets(col, k, scan_order(n, 0, seed));
    if (best.num_full == 0) { err = "rank(G) < k"; return BZ_ERANK; }
    for (uint32_t t = 1; t < trials; ++t) {
        SetChoice s2 = find_sets(col, k, scan_order(n, t, seed));
        if (s2.num_full > best.num_full || (s2.num_full == best.num_full && s2.partial > best.partial))
            best = std::move(s2);
    }
    const std::vector<std::vector<uint32_t>> &sets = best.sets;
    const uint32_t num_full = best.num_full, partial = best.partial;

    c.n = n; c.k = k; c.num_full = num_full; c.partial_rank = partial;
    c.nsets = (uint32_t)sets.size();
    c.set_of_column.assign(n, -1);
    c.W_full = (n - k + 31) / 32;
    c.W_partial = partial ? (n - partial + 31) / 32 : 0;
    c.full_rows.clear();
    c.packed.clear();
    c.packed_off.clear();
    for (uint32_t j = 0; j < c.nsets; ++j) {
        const std::vector<uint32_t> &S = sets[j];
        std::vector<char> in(n, 0);
        for (uint32_t cc : S) { in[cc] = 1; c.set_of_column[cc] = (int32_t)j; }
        std::vector<uint32_t> order(S.begin(), S.end());
        for (uint32_t cc = 0; cc < n; ++cc) if (!in[cc]) order.push_back(cc);
        std::vector<HostRow> gam = rows;
        uint32_t rk = reduce(gam, order, nw);
        if (rk != k) { err = "internal: Gamma_j lost rank"; return BZ_ERANK; }
        // the identity part on S (rows 0..|S|-1) is implied by the pivot order
        for (uint32_t i = 0; i < (uint32_t)S.size(); ++i)
            if (!bit(gam[i], S[i])) { err = "internal: pivot order"; return BZ_ERANK; }
        const uint32_t W = (j < num_full) ? c.W_full : c.W_partial;
        c.packed_off.push_back(c.packed.size());
        // the columns outside S_j, in ascending order
        std::vector<uint32_t> rest;
        for (uint32_t cc = 0; cc < n; ++cc) if (!in[cc]) rest.push_back(cc);
        for (uint32_t i = 0; i < k; ++i) {
            c.full_rows.push_back(gam[i]);
            const size_t at = c.packed.size();
            c.packed.resize(at + W, 0u);
            for (uint32_t pos = 0; pos < (uint32_t)rest.size(); ++pos)
                c.packed[at + (pos >> 5)] |= (uint32_t)bit(gam[i], rest[pos]) << (pos & 31);
        }
    }
    return BZ_OK;
}

}  // namespace bz
