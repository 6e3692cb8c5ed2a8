/*
 * MinJoin oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct CPU implementation of MinJoin (Zhang & Zhang,
 * "MinJoin: Efficient Edit Similarity Joins via Local Hash Minima", arXiv:1810.08833).
 * It exists to check the GPU library against the paper.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it; the product path never
 * does.  It shares no code with the HIP library: every definition below is written
 * out again here from the paper and the fixed readings of it.
 *
 * Conventions (0-based; the paper is 1-based):
 *   - a string is an array of symbol codes in [0, sigma);
 *   - b = ceil(log2 sigma) bits per symbol; q*b <= 64.
 *
 * Parity pinned by: tests/test_oracle_*.py (worked example of Tables 2-4, published
 * SplitMix64 outputs, closed forms, brute force, full Wagner-Fischer, Lemma 1).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

/* ------------------------------------------------------------------------- */
/* Random hash Pi over q-grams (Sec. 2.1: Pi maps Sigma^q into (0,1); Thm 1 proof:
 * rolling hash).  Reading: the q-gram is packed injectively into G (first symbol most
 * significant), then passed through the SplitMix64 output function (a bijection on
 * 64-bit words, Steele, Lea & Flood 2014) after XOR with a seed-derived salt.  Pi is
 * therefore collision-free on distinct q-grams; u64 order stands for order in (0,1). */

#define ORC_GAMMA 0x9E3779B97F4A7C15ULL  /* SplitMix64 increment (odd) */
#define ORC_GAMMA_B 0x632BE59BD9B4E019ULL /* separates the partition-key base */
#define ORC_P61 ((1ULL << 61) - 1)

uint64_t orc_mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

int orc_symbol_bits(int sigma) {
    int b = 1;
    while ((1 << b) < sigma) b++;
    return b;
}

/* salt S = M(seed + gamma): seed 0 must not give S = 0, since M(0) = 0 */
uint64_t orc_pi_salt(uint64_t seed) { return orc_mix64(seed + ORC_GAMMA); }

/* Pi of the q-gram starting at s[p], computed directly from its symbols */
static uint64_t pi_direct(const uint8_t *s, int64_t p, int q, int b, uint64_t salt,
                          const uint64_t *table) {
    uint64_t g = 0;
    for (int k = 0; k < q; k++) g = (g << b) | (uint64_t)s[p + k];
    if (table) return table[g];
    return orc_mix64(g ^ salt);
}

void orc_qgram_hashes(const uint8_t *s, int64_t m, int q, int b, uint64_t seed,
                      const uint64_t *table, uint64_t *out) {
    uint64_t salt = orc_pi_salt(seed);
    for (int64_t p = 0; p + q <= m; p++) out[p] = pi_direct(s, p, q, b, salt, table);
}

/* ------------------------------------------------------------------------- */
/* Number of targeted partitions T (Remark 1: T in [K/5, K]).  Reading: T = t_fixed
 * when given, else max(1, ceil(K / t_div)). */
int64_t orc_target_partitions(int64_t K, int t_div, int t_fixed) {
    if (t_fixed > 0) return t_fixed;
    int64_t T = (K + t_div - 1) / t_div;
    return T < 1 ? 1 : T;
}

/* Neighbourhood radius (Alg. 2, the line defining r): floor((|s|-q+1-T)/(2T+2)).
 * Reading: clamped to >= 1 (the paper assumes long strings). */
int64_t orc_radius(int64_t m, int q, int64_t T) {
    int64_t num = m - q + 1 - T;
    if (num <= 0) return 1;
    int64_t r = num / (2 * T + 2);
    return r < 1 ? 1 : r;
}

/* Find-Anchor (Alg. 2), from the definition of an anchor: a q-gram start p is an
 * anchor when its hash is strictly smaller than each of the other 2r hashes within
 * distance r (Sec. 2.1: the strict local minimum; equal q-grams suppress each other),
 * among the p whose window [p-r, p+r] lies inside the hash array.  The first position
 * and the end sentinel m are anchors too, so that the partitions tile the string
 * (Table 4).  Writes the anchors in increasing order; returns their count. */
static uint64_t min_hash(const uint64_t *h, int64_t lo, int64_t hi) {
    uint64_t v = UINT64_MAX;
    for (int64_t j = lo; j <= hi; j++) v = h[j] < v ? h[j] : v;
    return v;
}

int64_t orc_find_anchors(const uint8_t *s, int64_t m, int q, int b, int64_t T,
                         uint64_t seed, const uint64_t *table, int64_t *out) {
    int64_t na = 0;
    if (m == 0) return 0;
    out[na++] = 0;
    int64_t npos = m - q + 1;
    if (npos > 0) {
        uint64_t *h = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)npos);
        orc_qgram_hashes(s, m, q, b, seed, table, h);
        int64_t r = orc_radius(m, q, T);
        for (int64_t p = r; p + r < npos; p++) {
            /* strictly below the smallest hash on each side of p */
            if (h[p] < min_hash(h, p - r, p - 1) && h[p] < min_hash(h, p + 1, p + r))
                out[na++] = p;
        }
        free(h);
    }
    out[na++] = m;
    return na;
}

/* ------------------------------------------------------------------------- */
/* Bucket function f of Alg. 3 (a hash of the partition's content).  Reading: the
 * Karp-Rabin polynomial over GF(2^61-1) with the length folded in as the leading
 * coefficient, Phi = L*B^L + sum_k (x_k+1) B^(L-1-k), then f = M(Phi xor S). */

static uint64_t mulmod61(uint64_t a, uint64_t b) {
    unsigned __int128 p = (unsigned __int128)a * b;
    uint64_t lo = (uint64_t)p & ORC_P61;
    uint64_t hi = (uint64_t)(p >> 61);
    uint64_t r = lo + hi;
    if (r >= ORC_P61) r -= ORC_P61;
    return r;
}

uint64_t orc_phi_base(uint64_t seed) {
    return 2 + orc_mix64(seed ^ ORC_GAMMA_B) % (ORC_P61 - 3);
}

uint64_t orc_partition_phi(const uint8_t *x, int64_t L, uint64_t seed) {
    uint64_t B = orc_phi_base(seed);
    uint64_t h = (uint64_t)L % ORC_P61;
    for (int64_t k = 0; k < L; k++) {
        h = mulmod61(h, B) + (uint64_t)x[k] + 1;
        if (h >= ORC_P61) h -= ORC_P61;
    }
    return h;
}

uint64_t orc_partition_key(const uint8_t *x, int64_t L, uint64_t seed) {
    return orc_mix64(orc_partition_phi(x, L, seed) ^ orc_pi_salt(seed));
}

/* ------------------------------------------------------------------------- */
/* Parameters shared by partition / join / search. */
typedef struct {
    int32_t q;
    int32_t sigma;
    uint64_t seed;
    int32_t t_div;
    int32_t t_fixed;
    int32_t reps;               /* parallel repetitions (Sec. 2.2, before Thm 1) */
    int32_t threads;
    int64_t k;                  /* uniform K, or -1 to use k_per_string */
    const int32_t *k_per_string;
    const uint64_t *pi_table;   /* optional injected Pi (indexed by packed q-gram) */
} orc_params;

typedef struct {
    uint64_t key;
    int32_t sid;
    int32_t pos;
    int32_t len;
    int32_t rep;
} orc_record;

static int64_t string_k(const orc_params *p, int32_t i) {
    return p->k >= 0 ? p->k : (int64_t)p->k_per_string[i];
}

/* Partition-String (Alg. 1) for one string and one repetition: consecutive anchors
 * a_k < a_(k+1) give the partition (a_k, a_(k+1) - a_k). */
static int64_t partition_one(const uint8_t *s, int64_t m, const orc_params *p, int64_t K,
                             int rep, int32_t sid, orc_record *out, int64_t *anch) {
    int b = orc_symbol_bits(p->sigma);
    int64_t T = orc_target_partitions(K, p->t_div, p->t_fixed);
    uint64_t seed = p->seed + (uint64_t)rep;
    int64_t na = orc_find_anchors(s, m, p->q, b, T, seed, p->pi_table, anch);
    int64_t np = 0;
    for (int64_t k = 0; k + 1 < na; k++) {
        int64_t pos = anch[k], len = anch[k + 1] - anch[k];
        out[np].key = orc_partition_key(s + pos, len, p->seed);
        out[np].sid = sid;
        out[np].pos = (int32_t)pos;
        out[np].len = (int32_t)len;
        out[np].rep = rep;
        np++;
    }
    return np;
}

/* All partitions of all strings, in string order, repetition-major within a string.
 * *out is malloc'ed (free with orc_free). Returns the record count. */
int64_t orc_partition_all(const uint8_t *chars, const int64_t *offsets, int32_t n,
                          const orc_params *p, orc_record **out) {
    int reps = p->reps > 0 ? p->reps : 1;
    int64_t *start = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    /* Room per string and repetition: two interior strict minima of radius r are more
     * than r apart (each lies in the other's window), so there are at most
     * (m-q+1)/(r+1) + 1 interior anchors and one partition more. */
    start[0] = 0;
    for (int32_t i = 0; i < n; i++) {
        int64_t m = offsets[i + 1] - offsets[i];
        int64_t T = orc_target_partitions(string_k(p, i), p->t_div, p->t_fixed);
        int64_t npos = m - p->q + 1 > 0 ? m - p->q + 1 : 0;
        int64_t bound = npos / (orc_radius(m, p->q, T) + 1) + 2;
        start[i + 1] = start[i] + bound * reps;
    }
    orc_record *tmp = (orc_record *)malloc(sizeof(orc_record) * ((size_t)start[n] + 1));
    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int nt = p->threads > 0 ? p->threads : 1;
#pragma omp parallel num_threads(nt)
    {
        int64_t cap = 0;
        int64_t *anch = NULL;
#pragma omp for schedule(dynamic, 16)
        for (int32_t i = 0; i < n; i++) {
            int64_t m = offsets[i + 1] - offsets[i];
            if (m + 2 > cap) { cap = m + 2; anch = (int64_t *)realloc(anch, sizeof(int64_t) * (size_t)cap); }
            int64_t c = 0;
            for (int rep = 0; rep < reps; rep++)
                c += partition_one(chars + offsets[i], m, p, string_k(p, i), rep, i,
                                   tmp + start[i] + c, anch);
            cnt[i] = c;
        }
        free(anch);
    }
    /* compact in place (the write position never passes the read position) */
    int64_t w = 0;
    for (int32_t i = 0; i < n; i++) {
        if (cnt[i]) memmove(tmp + w, tmp + start[i], sizeof(orc_record) * (size_t)cnt[i]);
        w += cnt[i];
    }
    orc_record *res = (orc_record *)realloc(tmp, sizeof(orc_record) * ((size_t)w + 1));
    free(cnt); free(start);
    *out = res ? res : tmp;
    return w;
}

/* ------------------------------------------------------------------------- */
/* Edit distance (unit-cost insertions, deletions, substitutions; Sec. 1). */

/* Textbook Wagner-Fischer over the full matrix (two rows). */
int64_t orc_edit_distance(const uint8_t *x, int64_t m, const uint8_t *y, int64_t n) {
    int64_t *prev = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    for (int64_t j = 0; j <= n; j++) prev[j] = j;
    for (int64_t i = 1; i <= m; i++) {
        cur[0] = i;
        for (int64_t j = 1; j <= n; j++) {
            int64_t d = prev[j - 1] + (x[i - 1] != y[j - 1]);
            int64_t u = prev[j] + 1, l = cur[j - 1] + 1;
            cur[j] = d < u ? (d < l ? d : l) : (u < l ? u : l);
        }
        int64_t *t = prev; prev = cur; cur = t;
    }
    int64_t r = prev[n];
    free(prev); free(cur);
    return r;
}

/* Ukkonen's banded test ED(x,y) <= K (Alg. 3 verification; Sec. 3): only cells with
 * |i-j| <= K are evaluated; any cell outside the band counts as K+1 and values are
 * saturated at K+1.  Row by row; a row whose minimum exceeds K rejects early.
 * Returns 1 if ED <= K, else 0. */
int orc_ed_within(const uint8_t *x, int64_t m, const uint8_t *y, int64_t n, int64_t K) {
    if (K < 0) return 0;
    if (m - n > K || n - m > K) return 0;
    int64_t W = 2 * K + 1, CAP = K + 1;
    /* row[d] holds D[i][i - K + d] */
    int64_t *prev = (int64_t *)malloc(sizeof(int64_t) * (size_t)W);
    int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)W);
    for (int64_t d = 0; d < W; d++) {
        int64_t j = d - K;
        prev[d] = (j >= 0 && j <= n) ? (j < CAP ? j : CAP) : CAP;
    }
    int ok = 1;
    for (int64_t i = 1; i <= m && ok; i++) {
        int64_t rowmin = CAP;
        for (int64_t d = 0; d < W; d++) {
            int64_t j = i - K + d;
            int64_t v = CAP;
            if (j >= 0 && j <= n) {
                if (j == 0) {
                    v = i;
                } else {
                    /* D[i-1][j-1] is prev[d]; D[i-1][j] is prev[d+1]; D[i][j-1] is cur[d-1] */
                    int64_t diag = prev[d] + (x[i - 1] != y[j - 1]);
                    int64_t up = (d + 1 < W ? prev[d + 1] : CAP) + 1;
                    int64_t left = (d > 0 ? cur[d - 1] : CAP) + 1;
                    v = diag;
                    if (up < v) v = up;
                    if (left < v) v = left;
                }
                if (v > CAP) v = CAP;
            }
            cur[d] = v;
            if (v < rowmin) rowmin = v;
        }
        if (rowmin > K) ok = 0;
        int64_t *t = prev; prev = cur; cur = t;
    }
    int res = 0;
    if (ok) res = prev[n - m + K] <= K;
    free(prev); free(cur);
    return res;
}

/* ------------------------------------------------------------------------- */
/* MinJoin (Alg. 3) from the definition of its candidate set: two strings are a
 * candidate when they hold partitions in the same bucket (equal key f: a common
 * partition, Sec. 2.1) whose pair passes the length filter and the position filter
 * (Alg. 3; Sec. 3) under the pair's threshold.  Alg. 3 walks the strings by length and
 * evicts bucket entries failing the length filter; eviction drops only entries that
 * the filter would reject for every later string, so testing every pair of records of
 * a bucket gives the same set.  The candidates are deduplicated and each is verified
 * with the banded test. */

static int cmp_u64(const void *a, const void *b) {
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return x < y ? -1 : (x > y);
}

static int64_t abs64(int64_t v) { return v < 0 ? -v : v; }

/* The length filter and the position filter of Alg. 3 with threshold K. */
static int pass_length(int64_t mi, int64_t mj, int64_t K) { return abs64(mi - mj) <= K; }
static int pass_position(int64_t pi, int64_t mi, int64_t pj, int64_t mj, int64_t K) {
    return abs64(pi - pj) + abs64((mi - pi) - (mj - pj)) <= K;
}

typedef struct {
    int64_t records, candidates, output, pair_tests;
    /* wall-clock seconds of the stages (the split of the paper's Fig. 5) */
    double partition_s, join_s, dedup_s, verify_s;
} orc_stats;

static int64_t dedup_sorted(uint64_t *a, int64_t n) {
    if (n == 0) return 0;
    qsort(a, (size_t)n, sizeof(uint64_t), cmp_u64);
    int64_t w = 1;
    for (int64_t i = 1; i < n; i++) if (a[i] != a[w - 1]) a[w++] = a[i];
    return w;
}

/* Records ordered by bucket key (ties by string, position, repetition). */
static int cmp_record_key(const void *a, const void *b) {
    const orc_record *x = (const orc_record *)a, *y = (const orc_record *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->sid != y->sid) return x->sid < y->sid ? -1 : 1;
    if (x->pos != y->pos) return x->pos < y->pos ? -1 : 1;
    return x->rep < y->rep ? -1 : (x->rep > y->rep);
}

/* Verification of a deduplicated, sorted candidate list with pair threshold
 * max(K_i, K_j); keeps accepted pairs in order.  Returns their count. */
static int64_t verify_pairs(const uint8_t *chars, const int64_t *off, const int64_t *kq,
                            uint64_t *pairs, int64_t np, int nt) {
    uint8_t *ok = (uint8_t *)malloc((size_t)np + 1);
#pragma omp parallel for schedule(dynamic, 4) num_threads(nt)
    for (int64_t c = 0; c < np; c++) {
        int32_t i = (int32_t)(pairs[c] >> 32), j = (int32_t)(pairs[c] & 0xffffffffu);
        int64_t K = kq[i] > kq[j] ? kq[i] : kq[j];
        ok[c] = (uint8_t)orc_ed_within(chars + off[i], off[i + 1] - off[i],
                                       chars + off[j], off[j + 1] - off[j], K);
    }
    int64_t w = 0;
    for (int64_t c = 0; c < np; c++) if (ok[c]) pairs[w++] = pairs[c];
    free(ok);
    return w;
}

/* Join.  Outputs (malloc'ed, free with orc_free): the deduplicated candidate pairs
 * and the accepted pairs, both as sorted u64 (min id << 32 | max id). */
static int join_impl(const uint8_t *chars, const int64_t *offsets, int32_t n, const orc_params *p,
                     uint64_t **cand_out, int64_t *ncand, uint64_t **pairs_out, int64_t *npairs,
                     orc_stats *stats, int do_verify) {
    int nt = p->threads > 0 ? p->threads : 1;
    int64_t *K = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    for (int32_t i = 0; i < n; i++) K[i] = string_k(p, i);
    /* the partitions of every string (and repetition), grouped into buckets by key */
    double t0 = omp_get_wtime();
    orc_record *rec = NULL;
    int64_t R = orc_partition_all(chars, offsets, n, p, &rec);
    double t1 = omp_get_wtime();
    qsort(rec, (size_t)R, sizeof(orc_record), cmp_record_key);
    /* every pair of records of a bucket: distinct strings passing both filters */
    int64_t cc = 0, ccap = 1024, tests = 0;
    uint64_t *cand = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)ccap);
    for (int64_t g0 = 0, g1; g0 < R; g0 = g1) {
        for (g1 = g0 + 1; g1 < R && rec[g1].key == rec[g0].key; g1++) {}
        for (int64_t a = g0; a < g1; a++) {
            for (int64_t b = a + 1; b < g1; b++) {
                int32_t i = rec[a].sid, j = rec[b].sid;
                int64_t mi = offsets[i + 1] - offsets[i], mj = offsets[j + 1] - offsets[j];
                int64_t Kij = K[i] > K[j] ? K[i] : K[j];
                tests++;
                if (i == j) continue;  /* a string repeating a partition meets itself */
                if (!pass_length(mi, mj, Kij)) continue;
                if (!pass_position(rec[a].pos, mi, rec[b].pos, mj, Kij)) continue;
                if (cc == ccap) { ccap *= 2; cand = (uint64_t *)realloc(cand, sizeof(uint64_t) * (size_t)ccap); }
                uint64_t lo = (uint64_t)(i < j ? i : j), hi = (uint64_t)(i < j ? j : i);
                cand[cc++] = (lo << 32) | hi;
            }
        }
    }
    double t2 = omp_get_wtime();
    /* dedup (Alg. 3 removes duplicate pairs) */
    cc = dedup_sorted(cand, cc);
    uint64_t *c2 = (uint64_t *)malloc(sizeof(uint64_t) * ((size_t)cc + 1));
    memcpy(c2, cand, sizeof(uint64_t) * (size_t)cc);
    double t3 = omp_get_wtime();
    /* verification */
    int64_t no = do_verify ? verify_pairs(chars, offsets, K, cand, cc, nt) : 0;
    double t4 = omp_get_wtime();
    if (stats) {
        stats->records = R; stats->candidates = cc; stats->output = no; stats->pair_tests = tests;
        stats->partition_s = t1 - t0; stats->join_s = t2 - t1; stats->dedup_s = t3 - t2;
        stats->verify_s = t4 - t3;
    }
    *cand_out = c2; *ncand = cc;
    *pairs_out = cand; *npairs = no;
    free(rec); free(K);
    return 0;
}

int orc_join(const uint8_t *chars, const int64_t *offsets, int32_t n, const orc_params *p,
             uint64_t **cand_out, int64_t *ncand, uint64_t **pairs_out, int64_t *npairs,
             orc_stats *stats) {
    return join_impl(chars, offsets, n, p, cand_out, ncand, pairs_out, npairs, stats, 1);
}

/* The join without its verification stage: candidates only (*npairs = 0). */
int orc_join_candidates(const uint8_t *chars, const int64_t *offsets, int32_t n,
                        const orc_params *p, uint64_t **cand_out, int64_t *ncand,
                        uint64_t **pairs_out, int64_t *npairs, orc_stats *stats) {
    return join_impl(chars, offsets, n, p, cand_out, ncand, pairs_out, npairs, stats, 0);
}

/* Search: the index holds every partition of the index strings (no eviction); each
 * query is partitioned with the same q, seed and T rule, probes the index, applies the
 * filters with its own K, dedups and verifies with its own K.  Output: sorted
 * (query id << 32 | string id). */

/* Search (the query side of Alg. 3 against a dictionary holding every index record):
 * the dictionary is the index records sorted by key, probed by binary search. */
int orc_search(const uint8_t *ichars, const int64_t *ioff, int32_t ni, const orc_params *ip,
               const uint8_t *qchars, const int64_t *qoff, int32_t nq, const orc_params *qp,
               uint64_t **cand_out, int64_t *ncand, uint64_t **pairs_out, int64_t *npairs) {
    int nt = qp->threads > 0 ? qp->threads : 1;
    orc_record *irec = NULL, *qrec = NULL;
    int64_t RI = orc_partition_all(ichars, ioff, ni, ip, &irec);
    int64_t RQ = orc_partition_all(qchars, qoff, nq, qp, &qrec);
    qsort(irec, (size_t)RI, sizeof(orc_record), cmp_record_key);
    int64_t cc = 0, ccap = 1024;
    uint64_t *cand = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)ccap);
    for (int64_t r = 0; r < RQ; r++) {
        int32_t qi = qrec[r].sid;
        int64_t mq = qoff[qi + 1] - qoff[qi];
        int64_t Kq = string_k(qp, qi);
        int64_t lo = 0, hi = RI;  /* first index record with key >= the query key */
        while (lo < hi) {
            int64_t mid = lo + (hi - lo) / 2;
            if (irec[mid].key < qrec[r].key) lo = mid + 1; else hi = mid;
        }
        for (int64_t e = lo; e < RI && irec[e].key == qrec[r].key; e++) {
            int64_t ms = ioff[irec[e].sid + 1] - ioff[irec[e].sid];
            if (pass_length(mq, ms, Kq) && pass_position(qrec[r].pos, mq, irec[e].pos, ms, Kq)) {
                if (cc == ccap) { ccap *= 2; cand = (uint64_t *)realloc(cand, sizeof(uint64_t) * (size_t)ccap); }
                cand[cc++] = ((uint64_t)qi << 32) | (uint64_t)(uint32_t)irec[e].sid;
            }
        }
    }
    cc = dedup_sorted(cand, cc);
    uint64_t *c2 = (uint64_t *)malloc(sizeof(uint64_t) * ((size_t)cc + 1));
    memcpy(c2, cand, sizeof(uint64_t) * (size_t)cc);
    uint8_t *ok = (uint8_t *)malloc((size_t)cc + 1);
#pragma omp parallel for schedule(dynamic, 4) num_threads(nt)
    for (int64_t c = 0; c < cc; c++) {
        int32_t qi = (int32_t)(cand[c] >> 32), sj = (int32_t)(cand[c] & 0xffffffffu);
        ok[c] = (uint8_t)orc_ed_within(qchars + qoff[qi], qoff[qi + 1] - qoff[qi],
                                       ichars + ioff[sj], ioff[sj + 1] - ioff[sj],
                                       string_k(qp, qi));
    }
    int64_t w = 0;
    for (int64_t c = 0; c < cc; c++) if (ok[c]) cand[w++] = cand[c];
    free(ok);
    *cand_out = c2; *ncand = cc;
    *pairs_out = cand; *npairs = w;
    free(irec); free(qrec);
    return 0;
}

/* Verify a given list of pairs (i << 32 | j) with pair threshold max(K_i, K_j);
 * writes one flag per pair.  Used to sample-check large runs. */
void orc_verify_list(const uint8_t *chars, const int64_t *offsets, const orc_params *p,
                     const uint64_t *pairs, int64_t np, uint8_t *flags) {
    int nt = p->threads > 0 ? p->threads : 1;
#pragma omp parallel for schedule(dynamic, 4) num_threads(nt)
    for (int64_t c = 0; c < np; c++) {
        int32_t i = (int32_t)(pairs[c] >> 32), j = (int32_t)(pairs[c] & 0xffffffffu);
        int64_t Ki = string_k(p, i), Kj = string_k(p, j);
        flags[c] = (uint8_t)orc_ed_within(chars + offsets[i], offsets[i + 1] - offsets[i],
                                          chars + offsets[j], offsets[j + 1] - offsets[j],
                                          Ki > Kj ? Ki : Kj);
    }
}

int orc_max_threads(void) { return omp_get_max_threads(); }

void orc_free(void *ptr) { free(ptr); }
