/*
 * bz_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded CPU implementation of the Brouwer-Zimmermann
 * minimum-weight algorithm over F2, written from the paper "Parallel
 * Implementations for Computing the Minimum Distance of a Random Linear Code
 * on Multicomputers" (Quintana-Orti, Hernando, Igual; arXiv:1911.08963).
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may load
 * it. It shares no code, header, table or helper with the GPU library.
 *
 * Everything here is exact integer arithmetic. Rows are n-bit vectors held in
 * OR_NW 64-bit words, coordinate c at bit c%64 of word c/64.
 *
 * What it computes, step by step:
 *   1. Information sets (Sec. 2.1, the paragraph introducing information sets
 *      and Gamma_m): scanning the available columns in ascending order, the
 *      pivot columns of the reduced echelon form are a greedy basis. S_1 is the
 *      basis of all columns; S_2 the basis of the columns left after removing
 *      S_1, and so on while the remaining columns still have rank k. The last
 *      remaining columns have rank k_m < k; if k_m > 0, S_m is their greedy basis.
 *   2. Gamma_j (Sec. 2.1, systematic form (I_k | A) and the block form of
 *      Gamma_m): the reduced echelon form of G when columns are scanned in the
 *      order (S_j ascending, then all other columns ascending). Rows stay in
 *      original coordinates. For a full-rank S_j this is I_k on S_j; for the
 *      partial S_m the first k_m rows carry I_{k_m} on S_m and the other rows
 *      are zero there.
 *   3. Bounds and levels (Alg. 1): L = 1, U = n - k + 1; for g = 1, 2, ... while
 *      g <= k and L < U, every Gamma_j contributes the minimum weight of c*Gamma_j
 *      over all c with wt(c) = g; after the level L = m_f (g+1) + max{0, g+1-k+k_m}.
 *      By default the bound is also checked after every Gamma_j (the prose of
 *      Sec. 2.2 says the bounds are checked after processing each Gamma matrix),
 *      using the bound certified by the matrices completed so far:
 *          after Gamma_j (j <= m_f) at level g:
 *              j (g+1) + (m_f - j) g + [k_m > 0] max{0, g - k + k_m}
 *          after the partial Gamma_m at level g: Alg. 1's L.
 *      Flag OR_LEVEL_STOP applies Alg. 1 literally (check once per level).
 *   4. Enumeration inside one (Gamma_j, g) (Alg. 2 with the stack-based variant
 *      of Sec. 2.2.1): every g-subset of the k rows in lexicographic order,
 *      starting at (0, 1, ..., g-1); a stack holds the running sums of the
 *      first 1, 2, ..., g chosen rows and is rebuilt from the left-most changed
 *      position. The weight of each sum is the popcount of the full n-bit row.
 *   5. Per (Gamma_j, g) statistics: minimum weight, number of combinations
 *      reaching it, number of combinations (= C(k, g)).
 *   6. Witness: U starts at the Singleton value n-k+1, which need not be the
 *      weight of any codeword; the first codeword met with weight < U, or = U
 *      while no witness is held yet, becomes the witness.
 *
 *   8. Codewords of a given weight w (not in the paper, which returns d only):
 *      the tasks (Gamma_j, g) run in the order of step 3 and every sum of
 *      weight w is collected, until the bound certified by the completed tasks
 *      exceeds w. From then on every codeword not enumerated has weight > w,
 *      so the distinct collected codewords are all codewords of weight w (a
 *      codeword is met once in every Gamma_j where it is light enough, so
 *      duplicates are removed by sorting).
 *   7. Random column permutations (Sec. 2.2: the implementation tries random
 *      permutations of the columns to find good information sets): with
 *      or_set_permutation_search(T, seed), step 1 is run T times, trial t
 *      scanning the columns in the order p_t instead of ascending order, and
 *      the trial with the most full sets, then the largest k_m, is kept (the
 *      first such trial on ties). p_0 is the identity; for t >= 1, p_t is a
 *      Fisher-Yates shuffle of (0..n-1): for i = n-1 down to 1, swap entries i
 *      and (x mod (i+1)), x the next output of SplitMix64 (Steele, Lea, Flood,
 *      OOPSLA 2014) started from state seed + t. The sets are sorted ascending
 *      before step 2, so each Gamma_j depends only on its set.
 *
 * Readings of the paper that this file takes (the paper is silent on them):
 * the canonical greedy choice of information sets (trial 0 above; the
 * permutation search only when asked, with the generator above);
 * the reduced echelon basis for every Gamma_j; the per-Gamma bound above; the
 * partial Gamma_m enumerated at every level; k = n returns d = 1 at once (the
 * loop condition fails before any level, since U = n - k + 1 = 1).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXN 256
#define OR_NW (OR_MAXN / 64)
#define OR_MAXK OR_MAXN
#define OR_MAXM OR_MAXN

enum { OR_OK = 0, OR_EINVAL = -1, OR_ERANK = -2, OR_ENOMEM = -3, OR_ELIMIT = -5 };
enum { OR_LEVEL_STOP = 2u };

typedef struct {
    uint32_t matrix, level, min_weight, _pad;
    uint64_t count_at_min, combinations;
} or_stat;

typedef struct {
    int32_t status;
    uint32_t d;            /* 0 unless the search converged                     */
    uint32_t lower_bound;  /* last certified lower bound L                       */
    uint32_t upper_bound;  /* U when the search ended                            */
    uint32_t last_level;   /* last level g entered                               */
    uint32_t num_full;     /* m_f                                                */
    uint32_t partial_rank; /* k_m                                                */
    uint32_t stats_len;
    uint64_t combinations; /* all combinations enumerated                        */
    uint64_t witness[OR_NW];
} or_result;

typedef uint64_t row_t[OR_NW];

static int getbit(const uint64_t *r, int c) { return (int)((r[c >> 6] >> (c & 63)) & 1u); }

static void row_xor(uint64_t *dst, const uint64_t *a, const uint64_t *b)
{
    for (int w = 0; w < OR_NW; ++w) dst[w] = a[w] ^ b[w];
}

static int row_weight(const uint64_t *r)
{
    int s = 0;
    for (int w = 0; w < OR_NW; ++w) s += __builtin_popcountll(r[w]);
    return s;
}

static void load_rows(row_t *M, const uint64_t *G, int k, int n, int ldw)
{
    memset(M, 0, sizeof(row_t) * (size_t)k);
    for (int i = 0; i < k; ++i)
        for (int w = 0; w < (n + 63) / 64; ++w) M[i][w] = G[(size_t)i * ldw + w];
    /* clear any bit at or beyond n */
    for (int i = 0; i < k; ++i)
        for (int c = n; c < OR_MAXN; ++c) M[i][c >> 6] &= ~(1ull << (c & 63));
}

/* Gauss-Jordan elimination of the k rows of M, scanning the columns in the
 * given order. Returns the rank; piv[r] is the pivot column of row r. On
 * return rows 0..rank-1 form the reduced echelon form (each pivot column has a
 * single 1) and rows rank..k-1 are zero. */
static int gauss_jordan(row_t *M, int k, const int *order, int ncols, int *piv)
{
    int r = 0;
    for (int t = 0; t < ncols && r < k; ++t) {
        int c = order[t], p = -1;
        for (int i = r; i < k; ++i)
            if (getbit(M[i], c)) { p = i; break; }
        if (p < 0) continue;
        if (p != r) {
            row_t tmp;
            memcpy(tmp, M[p], sizeof(row_t));
            memcpy(M[p], M[r], sizeof(row_t));
            memcpy(M[r], tmp, sizeof(row_t));
        }
        for (int i = 0; i < k; ++i)
            if (i != r && getbit(M[i], c)) row_xor(M[i], M[i], M[r]);
        piv[r++] = c;
    }
    return r;
}

typedef struct {
    int n, k, m_f, k_m;
    int set_of_column[OR_MAXN];   /* index of the information set, or -1       */
    int nsets;                     /* m_f + (k_m > 0)                           */
    row_t *gamma;                  /* nsets * k rows                            */
} or_code;

static void free_code(or_code *oc) { free(oc->gamma); oc->gamma = NULL; }

/* Step 7 of the header: the permutation search's parameters (0 = natural order). */
static uint32_t g_perm_trials = 0;
static uint64_t g_perm_seed = 0;

void or_set_permutation_search(uint32_t trials, uint64_t seed)
{
    g_perm_trials = trials;
    g_perm_seed = seed;
}

/* SplitMix64: the state advances by the golden gamma; the output mixes it. */
static uint64_t splitmix64_next(uint64_t *state)
{
    uint64_t z = (*state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

uint64_t or_splitmix64(uint64_t *state) { return splitmix64_next(state); }

/* p_t of step 7. */
static void trial_order(int n, uint32_t t, uint64_t seed, int *order)
{
    for (int c = 0; c < n; ++c) order[c] = c;
    if (t == 0) return;
    uint64_t st = seed + t;
    for (int i = n - 1; i >= 1; --i) {
        int j = (int)(splitmix64_next(&st) % (uint64_t)(i + 1));
        int tmp = order[i]; order[i] = order[j]; order[j] = tmp;
    }
}

void or_trial_order(uint32_t n, uint32_t t, uint64_t seed, int32_t *order)
{
    int buf[OR_MAXN];
    if (n > OR_MAXN) return;
    trial_order((int)n, t, seed, buf);
    for (uint32_t c = 0; c < n; ++c) order[c] = buf[c];
}

static int cmp_int(const void *a, const void *b) { return *(const int *)a - *(const int *)b; }

/* Step 1 with the columns scanned in the given order: fills sets (each sorted
 * ascending), their sizes, m_f and k_m; returns the number of sets or an error. */
static int find_sets(const uint64_t *G, int k, int n, int ldw, const int *scan, row_t *M, int *piv,
                     int sets[][OR_MAXK], int *setsize, int *m_f, int *k_m)
{
    int avail[OR_MAXN];
    for (int c = 0; c < n; ++c) avail[c] = scan[c];
    int navail = n, nsets = 0;
    *m_f = 0; *k_m = 0;
    for (;;) {
        load_rows(M, G, k, n, ldw);
        int rank = gauss_jordan(M, k, avail, navail, piv);
        if (nsets == 0 && rank < k) return OR_ERANK;
        if (rank < k) {                       /* the leftover columns          */
            *k_m = rank;
            if (rank > 0) {
                memcpy(sets[nsets], piv, sizeof(int) * (size_t)rank);
                qsort(sets[nsets], (size_t)rank, sizeof(int), cmp_int);
                setsize[nsets] = rank;
                nsets++;
            }
            break;
        }
        memcpy(sets[nsets], piv, sizeof(int) * (size_t)k);
        qsort(sets[nsets], (size_t)k, sizeof(int), cmp_int);
        setsize[nsets] = k;
        nsets++;
        (*m_f)++;
        /* remove the chosen columns from the available list, keeping its order */
        int w = 0;
        for (int t = 0; t < navail; ++t) {
            int used = 0;
            for (int i = 0; i < k; ++i) if (piv[i] == avail[t]) { used = 1; break; }
            if (!used) avail[w++] = avail[t];
        }
        navail = w;
        if (navail == 0) { *k_m = 0; break; }
    }
    return nsets;
}

/* Steps 1, 2 and 7 of the header. */
static int prepare(const uint64_t *G, int k, int n, int ldw, or_code *oc)
{
    if (!G || k <= 0 || n <= 0 || k > n || n > OR_MAXN || ldw < (n + 63) / 64) return OR_EINVAL;
    memset(oc, 0, sizeof(*oc));
    oc->n = n; oc->k = k;
    row_t *M = (row_t *)malloc(sizeof(row_t) * (size_t)k);
    int *piv = (int *)malloc(sizeof(int) * (size_t)n);
    static int sets[OR_MAXM][OR_MAXK], trial_sets[OR_MAXM][OR_MAXK];
    int setsize[OR_MAXM], trial_size[OR_MAXM];
    int scan[OR_MAXN];
    if (!M || !piv) { free(M); free(piv); return OR_ENOMEM; }
    for (int c = 0; c < n; ++c) oc->set_of_column[c] = -1;
    int status = OR_OK, nsets = -1;
    const uint32_t trials = g_perm_trials > 1 ? g_perm_trials : 1;
    for (uint32_t t = 0; t < trials; ++t) {
        trial_order(n, t, g_perm_seed, scan);
        int mf = 0, km = 0;
        int ns = find_sets(G, k, n, ldw, scan, M, piv, trial_sets, trial_size, &mf, &km);
        if (ns < 0) { status = ns; break; }   /* rank(G) < k in every order   */
        if (nsets < 0 || mf > oc->m_f || (mf == oc->m_f && km > oc->k_m)) {
            nsets = ns; oc->m_f = mf; oc->k_m = km;
            for (int j = 0; j < ns; ++j) {
                setsize[j] = trial_size[j];
                memcpy(sets[j], trial_sets[j], sizeof(int) * (size_t)trial_size[j]);
            }
        }
    }
    if (status == OR_OK) {
        oc->nsets = nsets;
        oc->gamma = (row_t *)malloc(sizeof(row_t) * (size_t)k * (size_t)nsets);
        if (!oc->gamma) status = OR_ENOMEM;
    }
    if (status == OR_OK) {
        int *order = (int *)malloc(sizeof(int) * (size_t)n);
        for (int j = 0; j < nsets; ++j) {
            int t = 0;
            char inset[OR_MAXN];
            memset(inset, 0, sizeof(inset));
            for (int i = 0; i < setsize[j]; ++i) { order[t++] = sets[j][i]; inset[sets[j][i]] = 1; }
            for (int c = 0; c < n; ++c) if (!inset[c]) order[t++] = c;
            row_t *Gam = oc->gamma + (size_t)j * k;
            load_rows(Gam, G, k, n, ldw);
            gauss_jordan(Gam, k, order, n, piv);
            for (int i = 0; i < setsize[j]; ++i) oc->set_of_column[sets[j][i]] = j;
        }
        free(order);
    }
    free(M); free(piv);
    if (status != OR_OK) free_code(oc);
    return status;
}

static uint64_t binom(int a, int b)
{
    if (b < 0 || b > a) return 0;
    if (b > a - b) b = a - b;
    /* exact for every value below 2^63 that the enumeration can reach */
    unsigned __int128 r = 1;
    for (int i = 1; i <= b; ++i) r = r * (unsigned)(a - b + i) / (unsigned)i;
    return (uint64_t)r;
}

/* Lexicographic successor of the g-subset c of {0..k-1} (Alg. 2's
 * Get_next_combination). Returns the left-most changed position, or -1 when c
 * was the last subset. */
static int lex_next(int *c, int g, int k)
{
    int i = g - 1;
    while (i >= 0 && c[i] == k - g + i) --i;
    if (i < 0) return -1;
    c[i]++;
    for (int t = i + 1; t < g; ++t) c[t] = c[t - 1] + 1;
    return i;
}

/* Lower bound certified after Gamma_j (0-based; j == m_f means the partial)
 * is finished at level g and every later matrix at level g-1. */
static int certified_bound(int j, int g, int m_f, int k_m, int k)
{
    if (j >= m_f) {                              /* partial done at level g     */
        int extra = (k_m > 0) ? (g + 1 - k + k_m) : 0;
        return m_f * (g + 1) + (extra > 0 ? extra : 0);
    }
    int extra = (k_m > 0) ? (g - k + k_m) : 0;   /* partial done at level g-1   */
    return (j + 1) * (g + 1) + (m_f - j - 1) * g + (extra > 0 ? extra : 0);
}

/* Alg. 1's L after level g is complete. */
static int level_bound(int g, int m_f, int k_m, int k)
{
    int extra = (k_m > 0) ? (g + 1 - k + k_m) : 0;
    return m_f * (g + 1) + (extra > 0 ? extra : 0);
}

int or_min_distance(const uint64_t *G, uint32_t k, uint32_t n, uint32_t ldw,
                    uint32_t flags, uint32_t max_level,
                    or_result *res, or_stat *stats, uint32_t stats_cap)
{
    if (!res) return OR_EINVAL;
    memset(res, 0, sizeof(*res));
    or_code oc;
    int st = prepare(G, (int)k, (int)n, (int)ldw, &oc);
    if (st != OR_OK) { res->status = st; return st; }
    res->num_full = (uint32_t)oc.m_f;
    res->partial_rank = (uint32_t)oc.k_m;

    int K = (int)k, N = (int)n;
    int L = 1, U = N - K + 1, have_witness = 0, done = 0;
    if (K == N) {                      /* the level loop never runs: d = 1    */
        memcpy(res->witness, oc.gamma[0], sizeof(row_t));
        res->d = 1; res->lower_bound = 1; res->upper_bound = 1;
        free_code(&oc);
        return OR_OK;
    }
    row_t *stack = (row_t *)malloc(sizeof(row_t) * (size_t)(K + 1));
    int *c = (int *)malloc(sizeof(int) * (size_t)(K + 1));
    int g = 1;
    st = OR_OK;
    while (g <= K && L < U && !done) {
        if (max_level && (uint32_t)g > max_level) { st = OR_ELIMIT; break; }
        res->last_level = (uint32_t)g;
        for (int j = 0; j < oc.nsets && !done; ++j) {
            row_t *Gam = oc.gamma + (size_t)j * K;
            uint32_t minw = 0xffffffffu;
            uint64_t cnt = 0, ncomb = 0;
            for (int i = 0; i < g; ++i) c[i] = i;
            int from = 0;
            for (;;) {
                /* rebuild the running sums from the left-most changed index */
                for (int i = from; i < g; ++i) {
                    if (i == 0) memcpy(stack[0], Gam[c[0]], sizeof(row_t));
                    else row_xor(stack[i], stack[i - 1], Gam[c[i]]);
                }
                uint32_t w = (uint32_t)row_weight(stack[g - 1]);
                ncomb++;
                if (w < minw) { minw = w; cnt = 1; } else if (w == minw) cnt++;
                if ((int)w < U || ((int)w == U && !have_witness)) {
                    U = (int)w;
                    memcpy(res->witness, stack[g - 1], sizeof(row_t));
                    have_witness = 1;
                }
                from = lex_next(c, g, K);
                if (from < 0) break;
            }
            res->combinations += ncomb;
            if (stats && res->stats_len < stats_cap) {
                or_stat *s = &stats[res->stats_len];
                s->matrix = (uint32_t)j; s->level = (uint32_t)g; s->min_weight = minw;
                s->count_at_min = cnt; s->combinations = ncomb;
            }
            res->stats_len++;
            if (!(flags & OR_LEVEL_STOP)) {
                int Lj = certified_bound(j, g, oc.m_f, oc.k_m, K);
                if (Lj > L) L = Lj;
                if (L >= U) done = 1;
            }
        }
        if (!done) {
            int Lg = level_bound(g, oc.m_f, oc.k_m, K);
            if (Lg > L) L = Lg;
        }
        ++g;
    }
    res->lower_bound = (uint32_t)L;
    res->upper_bound = (uint32_t)U;
    if (st == OR_OK && res->stats_len > stats_cap && stats) st = OR_ELIMIT;
    if (st == OR_OK) res->d = (uint32_t)U;
    res->status = st;
    free(stack); free(c); free_code(&oc);
    return st;
}

/* Information sets and Gamma matrices, for structural tests.
 * gamma_out: (m_f + [k_m > 0]) * k rows of out_ld words, or NULL. */
int or_prepare(const uint64_t *G, uint32_t k, uint32_t n, uint32_t ldw,
               int32_t *set_of_column, uint32_t *num_full, uint32_t *partial_rank,
               uint64_t *gamma_out, uint32_t out_ld, uint32_t gamma_cap_rows)
{
    or_code oc;
    int st = prepare(G, (int)k, (int)n, (int)ldw, &oc);
    if (st != OR_OK) return st;
    if (set_of_column) for (uint32_t c = 0; c < n; ++c) set_of_column[c] = oc.set_of_column[c];
    if (num_full) *num_full = (uint32_t)oc.m_f;
    if (partial_rank) *partial_rank = (uint32_t)oc.k_m;
    if (gamma_out) {
        uint32_t rows = (uint32_t)oc.nsets * k;
        if (rows > gamma_cap_rows || out_ld < (n + 63) / 64) { free_code(&oc); return OR_EINVAL; }
        for (uint32_t r = 0; r < rows; ++r)
            for (uint32_t w = 0; w < out_ld; ++w)
                gamma_out[(size_t)r * out_ld + w] = (w < OR_NW) ? oc.gamma[r][w] : 0;
    }
    free_code(&oc);
    return OR_OK;
}

/* The lexicographic sequence of g-subsets of {0..k-1} that the enumeration
 * visits, written as consecutive g-tuples. Returns the number of subsets. */
int64_t or_lex_sequence(uint32_t k, uint32_t g, int32_t *out, uint64_t cap_subsets)
{
    if (g == 0 || g > k || k > OR_MAXN) return -1;
    int c[OR_MAXN];
    for (uint32_t i = 0; i < g; ++i) c[i] = (int)i;
    uint64_t cnt = 0;
    do {
        if (cnt < cap_subsets) for (uint32_t i = 0; i < g; ++i) out[cnt * g + i] = c[i];
        cnt++;
    } while (lex_next(c, (int)g, (int)k) >= 0);
    return (int64_t)cnt;
}

uint64_t or_binomial(uint32_t a, uint32_t b) { return binom((int)a, (int)b); }

/* ---- The prefix split of Sec. 3 (Alg. 3), used by the multi-process oracle ----
 *
 * A prefix is a p-subset (in lexicographic order) whose right-most element is
 * at most k-1-(g-p) (Sec. 3.1); Process_prefix adds the prefix rows once and
 * then every (g-p)-subset of the indices after the prefix's last element.
 * Prefixes are dealt to nparts workers cyclically by their lexicographic index
 * (the static S-Lex distribution of Sec. 3.3). When p >= g there is no split:
 * worker 0 takes the whole level (prefix replication). */

typedef struct {
    uint32_t min_weight;
    uint32_t _pad;
    uint64_t count_at_min, combinations;
    uint64_t witness[OR_NW];
} or_task_result;

/* Enumerate the completions of one prefix. If seq is non-NULL the visited
 * g-tuples are written there (for order tests) instead of being weighed. */
static void expand_prefix(const row_t *Gam, int k, int g, const int *prefix, int p,
                          or_task_result *tr, int32_t *seq, uint64_t seq_cap, uint64_t *seq_len)
{
    int c[OR_MAXN];
    row_t stack[OR_MAXN + 1];
    row_t base;
    memset(base, 0, sizeof(base));
    for (int i = 0; i < p; ++i) { c[i] = prefix[i]; row_xor(base, base, Gam[prefix[i]]); }
    int s = g - p;                           /* suffix length                 */
    int lo = (p > 0) ? prefix[p - 1] + 1 : 0;
    if (s > k - lo) return;
    for (int i = 0; i < s; ++i) c[p + i] = lo + i;
    int from = 0;
    for (;;) {
        for (int i = from; i < s; ++i) {
            if (i == 0) row_xor(stack[0], base, Gam[c[p]]);
            else row_xor(stack[i], stack[i - 1], Gam[c[p + i]]);
        }
        const uint64_t *sum = (s > 0) ? stack[s - 1] : base;
        if (seq) {
            if (*seq_len < seq_cap) for (int i = 0; i < g; ++i) seq[*seq_len * g + i] = c[i];
            (*seq_len)++;
        } else {
            uint32_t w = (uint32_t)row_weight(sum);
            tr->combinations++;
            if (w < tr->min_weight) {
                tr->min_weight = w; tr->count_at_min = 1;
                memcpy(tr->witness, sum, sizeof(row_t));
            } else if (w == tr->min_weight) tr->count_at_min++;
        }
        if (s == 0) break;
        /* lexicographic successor of the suffix inside [lo, k) */
        int i = s - 1;
        while (i >= 0 && c[p + i] == k - s + i) --i;
        if (i < 0) break;
        c[p + i]++;
        for (int t = i + 1; t < s; ++t) c[p + t] = c[p + t - 1] + 1;
        from = i;
    }
}

int or_task(const uint64_t *G, uint32_t k, uint32_t n, uint32_t ldw,
            uint32_t matrix, uint32_t g, uint32_t p, uint32_t part, uint32_t nparts,
            or_task_result *out)
{
    if (!out || nparts == 0 || part >= nparts || g == 0 || g > k) return OR_EINVAL;
    memset(out, 0, sizeof(*out));
    out->min_weight = 0xffffffffu;
    or_code oc;
    int st = prepare(G, (int)k, (int)n, (int)ldw, &oc);
    if (st != OR_OK) return st;
    if ((int)matrix >= oc.nsets) { free_code(&oc); return OR_EINVAL; }
    const row_t *Gam = oc.gamma + (size_t)matrix * k;
    int K = (int)k, Gl = (int)g;
    if ((int)p >= Gl || p == 0) {            /* prefix replication            */
        if (part == 0) {
            int none[1] = {0};
            expand_prefix(Gam, K, Gl, none, 0, out, NULL, 0, NULL);
        }
    } else {
        int P = (int)p, pre[OR_MAXN];
        int maxlast = K - 1 - (Gl - P);      /* valid-prefix bound            */
        for (int i = 0; i < P; ++i) pre[i] = i;
        uint64_t idx = 0;
        if (pre[P - 1] <= maxlast) {
            for (;;) {
                if (idx % nparts == part) expand_prefix(Gam, K, Gl, pre, P, out, NULL, 0, NULL);
                idx++;
                /* lexicographic successor among p-subsets of {0..maxlast} */
                int i = P - 1;
                while (i >= 0 && pre[i] == maxlast - (P - 1 - i)) --i;
                if (i < 0) break;
                pre[i]++;
                for (int t = i + 1; t < P; ++t) pre[t] = pre[t - 1] + 1;
            }
        }
    }
    free_code(&oc);
    return OR_OK;
}

static int cmp_row(const void *a, const void *b)
{
    const uint64_t *x = (const uint64_t *)a, *y = (const uint64_t *)b;
    for (int w = OR_NW - 1; w >= 0; --w)
        if (x[w] != y[w]) return x[w] < y[w] ? -1 : 1;
    return 0;
}

/* Step 8 of the header: the number of codewords of weight w; up to cap of them
 * (sorted as integers, most significant word last) go to out. Returns OR_OK,
 * or OR_ELIMIT when more than max_hits weighted sums would have to be held. */
int or_count_weight(const uint64_t *G, uint32_t k, uint32_t n, uint32_t ldw, uint32_t w,
                    uint64_t max_hits, uint64_t *count, uint64_t *out, uint64_t cap,
                    uint32_t *last_level)
{
    if (!count || w == 0) return OR_EINVAL;
    *count = 0;
    or_code oc;
    int st = prepare(G, (int)k, (int)n, (int)ldw, &oc);
    if (st != OR_OK) return st;
    int K = (int)k;
    row_t *hits = (row_t *)malloc(sizeof(row_t) * (size_t)(max_hits ? max_hits : 1));
    row_t *stack = (row_t *)malloc(sizeof(row_t) * (size_t)(K + 1));
    int *c = (int *)malloc(sizeof(int) * (size_t)(K + 1));
    uint64_t nh = 0;
    int done = 0;
    st = OR_OK;
    for (int g = 1; g <= K && !done && st == OR_OK; ++g) {
        if (last_level) *last_level = (uint32_t)g;
        for (int j = 0; j < oc.nsets && !done && st == OR_OK; ++j) {
            row_t *Gam = oc.gamma + (size_t)j * K;
            for (int i = 0; i < g; ++i) c[i] = i;
            int from = 0;
            for (;;) {
                for (int i = from; i < g; ++i) {
                    if (i == 0) memcpy(stack[0], Gam[c[0]], sizeof(row_t));
                    else row_xor(stack[i], stack[i - 1], Gam[c[i]]);
                }
                if ((uint32_t)row_weight(stack[g - 1]) == w) {
                    if (nh >= max_hits) { st = OR_ELIMIT; break; }
                    memcpy(hits[nh++], stack[g - 1], sizeof(row_t));
                }
                from = lex_next(c, g, K);
                if (from < 0) break;
            }
            /* every codeword not met yet weighs at least the certified bound */
            if (certified_bound(j, g, oc.m_f, oc.k_m, K) > (int)w) done = 1;
        }
    }
    if (st == OR_OK) {
        qsort(hits, (size_t)nh, sizeof(row_t), cmp_row);
        uint64_t distinct = 0;
        for (uint64_t i = 0; i < nh; ++i) {
            if (i > 0 && cmp_row(hits[i], hits[i - 1]) == 0) continue;
            if (out && distinct < cap) memcpy(out + distinct * OR_NW, hits[i], sizeof(row_t));
            distinct++;
        }
        *count = distinct;
    }
    free(hits); free(stack); free(c); free_code(&oc);
    return st;
}

/* The g-tuples Process_prefix visits for one prefix, in order. */
int64_t or_prefix_sequence(uint32_t k, uint32_t g, const int32_t *prefix, uint32_t p,
                           int32_t *out, uint64_t cap)
{
    if (g == 0 || g > k || p > g || k > OR_MAXN) return -1;
    static row_t zero[OR_MAXN];
    int pre[OR_MAXN];
    for (uint32_t i = 0; i < p; ++i) pre[i] = prefix[i];
    uint64_t len = 0;
    expand_prefix(zero, (int)k, (int)g, pre, (int)p, NULL, out, cap, &len);
    return (int64_t)len;
}

/* Number of valid prefixes at (k, g, p), counted by walking them. */
int64_t or_prefix_count(uint32_t k, uint32_t g, uint32_t p)
{
    if (p == 0 || p >= g || g > k) return -1;
    int P = (int)p, pre[OR_MAXN], maxlast = (int)k - 1 - ((int)g - P);
    for (int i = 0; i < P; ++i) pre[i] = i;
    if (pre[P - 1] > maxlast) return 0;
    int64_t cnt = 0;
    for (;;) {
        cnt++;
        int i = P - 1;
        while (i >= 0 && pre[i] == maxlast - (P - 1 - i)) --i;
        if (i < 0) break;
        pre[i]++;
        for (int t = i + 1; t < P; ++t) pre[t] = pre[t - 1] + 1;
    }
    return cnt;
}

/* The lower bounds used by the stop rule, exported so tests can check them
 * against brute force. */
int or_certified_bound(int j, int g, int m_f, int k_m, int k) { return certified_bound(j, g, m_f, k_m, k); }
int or_level_bound(int g, int m_f, int k_m, int k) { return level_bound(g, m_f, k_m, k); }
