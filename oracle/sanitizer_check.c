/*
 * Sanitizer run of the MinJoin oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Compiled together with minjoin_oracle.c under AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_oracle_sanitizers.py, it drives every entry
 * point of the oracle over small seeded collections (empty strings, strings shorter than
 * q, homopolymers, clustered near-copies; 4, 25 and 37 symbols; uniform and per-string K;
 * repetitions; fixed and K-derived T) and checks two invariants on the way: the output is
 * a subset of the candidates, and every output pair is within its threshold by the full
 * edit distance.  A sanitizer report or a failed check ends the run with a nonzero status.
 */
#include <stdio.h>

#include "minjoin_oracle.c"

/* SplitMix64 as a seeded source of test inputs (Steele, Lea & Flood 2014) */
static uint64_t g_state;
static uint64_t next_u64(void) {
    g_state += ORC_GAMMA;
    return orc_mix64(g_state);
}
static int64_t below(int64_t n) { return n > 0 ? (int64_t)(next_u64() % (uint64_t)n) : 0; }

typedef struct {
    uint8_t *chars;
    int64_t *off;
    int32_t n;
} coll;

/* clusters of near-copies of random bases plus degenerate strings */
static coll make_collection(int sigma, int clusters, int copies, int64_t minlen, int64_t maxlen) {
    int32_t n = clusters * copies + 4;
    coll c;
    c.n = n;
    c.off = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    int64_t cap = (int64_t)n * (maxlen + maxlen / 4 + 8) + 16;
    c.chars = (uint8_t *)malloc((size_t)cap);
    uint8_t *base = (uint8_t *)malloc((size_t)maxlen + 1);
    int64_t w = 0;
    int32_t id = 0;
    for (int k = 0; k < clusters; k++) {
        int64_t L = minlen + below(maxlen - minlen + 1);
        for (int64_t i = 0; i < L; i++) base[i] = (uint8_t)below(sigma);
        for (int t = 0; t < copies; t++) {
            c.off[id++] = w;
            for (int64_t i = 0; i < L; i++) {
                int64_t r = below(100);
                if (r < 2) continue;                                        /* deletion */
                if (r < 4) c.chars[w++] = (uint8_t)below(sigma);            /* insertion */
                c.chars[w++] = r < 6 ? (uint8_t)below(sigma) : base[i];     /* substitution */
            }
        }
    }
    c.off[id++] = w;                                  /* empty string */
    c.off[id++] = w; c.chars[w++] = (uint8_t)below(sigma);  /* one symbol */
    c.off[id++] = w;                                  /* homopolymer */
    for (int i = 0; i < 300; i++) c.chars[w++] = (uint8_t)(sigma - 1);
    c.off[id++] = w;                                  /* duplicate of string 0 */
    for (int64_t i = c.off[0]; i < c.off[1]; i++) c.chars[w++] = c.chars[i];
    c.off[id] = w;
    free(base);
    return c;
}

static int check_join(const coll *c, const orc_params *p, const int64_t *kq) {
    uint64_t *cand = NULL, *out = NULL;
    int64_t nc = 0, no = 0;
    orc_stats st;
    orc_join(c->chars, c->off, c->n, p, &cand, &nc, &out, &no, &st);
    int bad = 0;
    for (int64_t t = 0, u = 0; t < no; t++) {
        while (u < nc && cand[u] < out[t]) u++;
        if (u == nc || cand[u] != out[t]) bad = 1;
        int32_t i = (int32_t)(out[t] >> 32), j = (int32_t)(out[t] & 0xffffffffu);
        int64_t K = kq[i] > kq[j] ? kq[i] : kq[j];
        if (orc_edit_distance(c->chars + c->off[i], c->off[i + 1] - c->off[i], c->chars + c->off[j],
                              c->off[j + 1] - c->off[j]) > K)
            bad = 1;
    }
    uint64_t *cand2 = NULL, *out2 = NULL;
    int64_t nc2 = 0, no2 = 0;
    orc_join_candidates(c->chars, c->off, c->n, p, &cand2, &nc2, &out2, &no2, &st);
    if (nc2 != nc || (nc && memcmp(cand2, cand, sizeof(uint64_t) * (size_t)nc))) bad = 1;
    uint8_t *flags = (uint8_t *)malloc((size_t)nc + 1);
    orc_verify_list(c->chars, c->off, p, cand, nc, flags);
    int64_t acc = 0;
    for (int64_t t = 0; t < nc; t++) acc += flags[t];
    if (acc != no) bad = 1;
    orc_record *rec = NULL;
    int64_t R = orc_partition_all(c->chars, c->off, c->n, p, &rec);
    if (R != st.records) bad = 1;
    free(flags); orc_free(rec); orc_free(cand); orc_free(out); orc_free(cand2); orc_free(out2);
    return bad;
}

int main(void) {
    int bad = 0, runs = 0;
    const int sigmas[3] = {4, 25, 37}, qs[3] = {4, 4, 6};
    for (int a = 0; a < 3; a++) {
        for (int v = 0; v < 4; v++) {
            g_state = 1000u * (uint64_t)a + (uint64_t)v;
            coll c = make_collection(sigmas[a], 6, 4, 40 + 60 * v, 400 + 300 * v);
            int64_t *kq = (int64_t *)malloc(sizeof(int64_t) * (size_t)c.n);
            int32_t *k32 = (int32_t *)malloc(sizeof(int32_t) * (size_t)c.n);
            for (int32_t i = 0; i < c.n; i++) {
                int64_t m = c.off[i + 1] - c.off[i];
                k32[i] = (int32_t)((8 * m + 99) / 100);
            }
            orc_params p;
            memset(&p, 0, sizeof(p));
            p.q = qs[a];
            p.sigma = sigmas[a];
            p.seed = (uint64_t)v;
            p.t_div = 1 + v % 3;
            p.t_fixed = v == 3 ? 2 : 0;
            p.reps = 1 + v % 2;
            p.threads = 2;
            if (v % 2) {
                p.k = -1;
                p.k_per_string = k32;
                for (int32_t i = 0; i < c.n; i++) kq[i] = k32[i];
            } else {
                p.k = 30 + 20 * v;
                for (int32_t i = 0; i < c.n; i++) kq[i] = p.k;
            }
            bad |= check_join(&c, &p, kq);
            /* search: the first half as queries with per-query K against the rest */
            int32_t nq = c.n / 2;
            uint64_t *sc = NULL, *so = NULL;
            int64_t nsc = 0, nso = 0;
            orc_params qp = p;
            qp.k = -1;
            qp.k_per_string = k32;
            orc_search(c.chars, c.off + nq, c.n - nq, &p, c.chars, c.off, nq, &qp, &sc, &nsc, &so,
                       &nso);
            if (nso > nsc) bad = 1;
            orc_free(sc); orc_free(so);
            free(kq); free(k32); free(c.chars); free(c.off);
            runs++;
        }
    }
    printf("oracle sanitizer check: %d runs, %s\n", runs, bad ? "FAILED" : "ok");
    return bad;
}
