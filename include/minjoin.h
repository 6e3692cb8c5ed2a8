/*
 * minjoin.h -- C-ABI of the MI355X MinJoin library (libminjoin.so).
 *
 * MinJoin (Zhang & Zhang, "MinJoin: Efficient Edit Similarity Joins via Local Hash
 * Minima", arXiv:1810.08833) finds all pairs of strings with edit distance at most K
 * (Sec. 1, problem statement; Alg. 3 `Ensure`).  Each string is cut at anchors --
 * positions whose q-gram hash is a strict minimum within radius r (Alg. 2) -- into
 * partitions (Alg. 1); strings sharing a partition that pass the length and position
 * filters become candidates (Alg. 3); every candidate is verified with Ukkonen's banded
 * dynamic program (Alg. 3, Sec. 3).  Every step runs in HIP kernels for gfx950.
 *
 * Conventions
 *   - Device pointers are HIP device addresses on the context's device.  "Borrowed"
 *     inputs must stay valid until the stream work of the call has completed (every
 *     call below returns only after its results are complete on `stream`).
 *   - Strings: `chars[offsets[i] .. offsets[i+1])` holds string i as symbol codes
 *     in [0, sigma), one byte per symbol.  Positions are 0-based.
 *   - Pairs are packed as uint64 `(a << 32) | b`; join pairs have a < b (input ids),
 *     search pairs are (query id, string id).  Pair lists are sorted ascending.
 *   - Every call returns an mj_status; on error the outputs are left untouched and
 *     mj_last_error() returns a thread-local message.  No C++ exception crosses the
 *     ABI.  Calls on one context must not overlap (the context owns one workspace).
 */
#ifndef MINJOIN_H
#define MINJOIN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MJ_OK = 0,
    MJ_EINVAL = 1,    /* invalid argument */
    MJ_ENOMEM = 2,    /* device allocation failed */
    MJ_EDEVICE = 3,   /* HIP runtime error */
    MJ_ECAPACITY = 4, /* a documented size limit was exceeded */
} mj_status;

typedef struct mj_ctx mj_ctx;
typedef struct mj_pairs mj_pairs;
typedef struct mj_records mj_records;
typedef struct mj_index mj_index;

/* Borrowed description of a string collection (all pointers device). */
typedef struct {
    const uint8_t *chars;    /* symbol codes, one byte each, in [0, sigma) */
    const int64_t *offsets;  /* n + 1 non-decreasing offsets, offsets[0] = 0 */
    int32_t n;               /* number of strings, >= 0 */
    int32_t sigma;           /* alphabet size, 2 .. 256 */
} mj_strings;

/* Method parameters (Alg. 2, Alg. 3, Remark 1).
 *   q        q-gram length; q * ceil(log2 sigma) <= 64.
 *   seed     randomness of the hash Pi and the bucket function f.  Pi of a q-gram is
 *            SplitMix64's output function applied to the injectively packed q-gram
 *            xor a salt derived from seed; f hashes a partition's content with a
 *            Karp-Rabin polynomial over GF(2^61-1) (length folded in), then mixes it.
 *   t_div, t_fixed
 *            number of targeted partitions T = t_fixed if t_fixed > 0, else
 *            max(1, ceil(K_i / t_div)) for string i (Remark 1 recommends T in [K/5, K]).
 *            The radius is r = max(1, floor((m - q + 1 - T) / (2T + 2))) (Alg. 2).
 *   reps     parallel repetitions (Sec. 2.2, boosting before Thm 1): repetition rho
 *            hashes q-grams with seed + rho; the union of all partitions is joined.
 *   k        uniform threshold K >= 0, or -1 to read k_per_string.
 *   k_per_string  device int32[n], per-string K_i >= 0 (used when k == -1).  A join
 *            pair uses max(K_i, K_j); a search pair uses the query's K.
 *   pi_table optional device uint64[2^(q*b)] replacing Pi (indexed by the packed
 *            q-gram, first symbol most significant, b = ceil(log2 sigma) bits each);
 *            NULL for the seeded hash.  Needs q * b <= 24. */
typedef struct {
    int32_t q;
    int32_t t_div;
    int32_t t_fixed;
    int32_t reps;
    uint64_t seed;
    int64_t k;
    const int32_t *k_per_string;
    const uint64_t *pi_table;
} mj_params;

/* Per-call counters and stage times (milliseconds between HIP events recorded on the
 * call's stream, so they include the host read-backs between stages).  Stage order:
 * 0 setup (per-string parameters, bit-plane packing), 1 partition (anchors and
 * records), 2 sort, 3 group and filter (probe and filter for search), 4 dedup,
 * 5 verify, 6 output; 7 is unused. */
typedef struct {
    int64_t records;     /* partitions over all strings and repetitions */
    int64_t groups;      /* buckets holding >= 2 records */
    int64_t pair_tests;  /* record pairs tested by the filters */
    int64_t candidates;  /* distinct candidate pairs */
    int64_t output;      /* pairs with ED <= K */
    int64_t band_cells;  /* (columns processed) x (band width) summed over candidates */
    float stage_ms[8];
    /* Device time of the hot kernels, summed over their launches in the call (HIP events
     * recorded on the call's stream immediately around each launch), and the launch
     * counts: 0 anchors, 1 partition records, 2 candidate emission, 3 verification. */
    float kernel_ms[4];
    int32_t kernel_launches[4];
    int64_t positions;   /* symbols scanned by the anchor kernel, over all repetitions */
} mj_stats;

/* ---- context ---------------------------------------------------------------- */

/* Create a context on HIP device `device` (made current for the calls).  The context
 * owns a growable device workspace.  EINVAL for a bad device, EDEVICE on HIP errors. */
mj_status mj_ctx_create(int device, mj_ctx **out);
void mj_ctx_destroy(mj_ctx *ctx);

/* Thread-local description of the last error (never NULL). */
const char *mj_last_error(void);

/* Library version string. */
const char *mj_version(void);

/* ---- join (Alg. 3): all pairs i < j with ED(s_i, s_j) <= K that share a partition
 * passing the filters ---------------------------------------------------------- */

/* Stream-ordered; returns once the pair count is known.  *out is library-owned until
 * mj_pairs_free.  stats may be NULL.  EINVAL on bad arguments (q < 1, q*b > 64,
 * t_div < 1, K < -1, sigma outside 2..256, offsets decreasing); ECAPACITY when a
 * documented limit is exceeded: record-pair tests of one call above 2^31, a radius r
 * above 1920 on a string long enough to have interior positions, or a candidate whose
 * threshold K is above 2047; ENOMEM when device memory runs out. */
mj_status mj_join(mj_ctx *ctx, const mj_strings *strings, const mj_params *params,
                  void *stream, mj_pairs **out, mj_stats *stats);

/* Stages of the join, for inspection and timing:
 *   mj_partition   Alg. 1-2 for every string and repetition: one record per partition
 *                  (key f, string id, start position, length), ordered by
 *                  (repetition, string, position).
 *   mj_candidates  Alg. 3 up to the dedup: the distinct candidate pairs, sorted.
 *   mj_verify      Alg. 3 verification of a caller-given device list of n pairs
 *                  (a << 32 | b, any order) with threshold max(K_a, K_b): writes
 *                  flags[i] = 1 if ED <= K else 0 (device uint8[n]). */
mj_status mj_partition(mj_ctx *ctx, const mj_strings *strings, const mj_params *params,
                       void *stream, mj_records **out);
mj_status mj_candidates(mj_ctx *ctx, const mj_strings *strings, const mj_params *params,
                        void *stream, mj_pairs **out, mj_stats *stats);
mj_status mj_verify(mj_ctx *ctx, const mj_strings *strings, const mj_params *params,
                    const uint64_t *pairs, int64_t n, uint8_t *flags, void *stream);

/* ---- search: index the strings once, then find (query, string) pairs with
 * ED <= K_query.  Queries use the index's q, seed, t_div/t_fixed and reps. ------- */

/* Builds partitions of `strings` (Alg. 1-2) and keeps them sorted by key in device
 * memory together with a packed copy of the strings; inputs are borrowed only during
 * the call.  *out is library-owned until mj_index_free. */
mj_status mj_index_build(mj_ctx *ctx, const mj_strings *strings, const mj_params *params,
                         void *stream, mj_index **out);
void mj_index_free(mj_index *index);
int64_t mj_index_records(const mj_index *index);

/* queries: borrowed; qparams->k / k_per_string give each query's K (q, seed, T rule
 * and reps are taken from the index). */
mj_status mj_search(mj_ctx *ctx, const mj_index *index, const mj_strings *queries,
                    const mj_params *qparams, void *stream, mj_pairs **out,
                    mj_stats *stats);

/* ---- results ----------------------------------------------------------------- */

int64_t mj_pairs_count(const mj_pairs *p);
const uint64_t *mj_pairs_device(const mj_pairs *p);     /* count entries, sorted */
/* Copies count packed pairs to host memory; EINVAL if cap < count. */
mj_status mj_pairs_copy_to_host(const mj_pairs *p, uint64_t *dst, int64_t cap);
void mj_pairs_free(mj_pairs *p);

int64_t mj_records_count(const mj_records *r);
/* Copies the records to host arrays of `cap` entries each (any pointer may be NULL);
 * EINVAL if cap < count. */
mj_status mj_records_copy_to_host(const mj_records *r, uint64_t *key, int32_t *sid,
                                  int32_t *pos, int32_t *len, int64_t cap);
void mj_records_free(mj_records *r);

#ifdef __cplusplus
}
#endif
#endif /* MINJOIN_H */
