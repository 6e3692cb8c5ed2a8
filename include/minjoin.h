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

/* Borrowed description of a string collection (all pointers device).
 *   packing MJ_PACK_U8: chars holds one byte per symbol, symbol g of the collection at
 *           chars[g].
 *   packing MJ_PACK_2BIT (sigma <= 4; the packed storage of DNA-shaped inputs): four
 *           symbols per byte, symbol g in bits 2(g mod 4) .. 2(g mod 4)+1 of byte g/4
 *           (the first symbol in the low bits).  The buffer holds whole 32-bit words,
 *           ceil(offsets[n] / 16) of them, 4-byte aligned; bits past the last symbol are
 *           ignored.  Positions and offsets still count symbols. */
enum { MJ_PACK_U8 = 0, MJ_PACK_2BIT = 1 };
typedef struct {
    const uint8_t *chars;    /* symbol codes in [0, sigma), stored as `packing` says */
    const int64_t *offsets;  /* n + 1 non-decreasing offsets, offsets[0] = 0 */
    int32_t n;               /* number of strings, >= 0 */
    int32_t sigma;           /* alphabet size, 2 .. 256 */
    int32_t packing;         /* MJ_PACK_U8 or MJ_PACK_2BIT */
    int32_t reserved;        /* 0 */
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
 *            NULL for the seeded hash.  Needs q * b <= 24.
 *   verifier MJ_VERIFY_BATCHED (0): all candidates in one persistent launch, a pair per
 *            lane group, longest pairs first, group width timed once per context;
 *            MJ_VERIFY_PLAIN (1): a pair per lane, one launch per band size.  Both give
 *            the same decisions.
 *   verify_lanes  batched verifier only: 0 lets the context time the choices (the
 *            default); 1, 2, 4 or 8 fixes the lanes per pair that split the band words;
 *            -2 fixes two lanes per pair that split the text columns (one runs forward
 *            over the first half, the other over the reversed second half); -3 sizes each
 *            pair's window by its own band class (2, 4, 8, 16 or 32 words on 1, 1, 2, 4
 *            or 8 lanes; widest classes first), for per-pair K (bands up to K = 992).  A
 *            fixed choice whose lanes cannot hold the band fails with MJ_ECAPACITY. */
typedef struct {
    int32_t q;
    int32_t t_div;
    int32_t t_fixed;
    int32_t reps;
    uint64_t seed;
    int64_t k;
    const int32_t *k_per_string;
    const uint64_t *pi_table;
    int32_t verifier;
    int32_t verify_lanes;
} mj_params;

enum { MJ_VERIFY_BATCHED = 0, MJ_VERIFY_PLAIN = 1 };

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
    int64_t band_cells;  /* (columns processed) x (K + 1 band diagonals), summed over candidates */
    float stage_ms[8];
    /* Device time of the hot kernels, summed over their launches in the call (HIP events
     * recorded on the call's stream around the launches), and the launch counts: 0 anchors,
     * 1 partition records (each one launch, or one pair of launches, covering every
     * repetition), 2 candidate emission, 3 verification. */
    float kernel_ms[4];
    int32_t kernel_launches[4];
    int64_t positions;   /* symbols scanned by the anchor kernel, over all repetitions */
    int32_t verify_group;  /* lanes per pair of the batched verifier (0: plain; -2: two
                              lanes splitting the text columns, forward and reversed; -3:
                              per-pair band classes) */
    int32_t verify_words;  /* band words per lane of the batched verifier */
    int32_t verify_blocks; /* most workgroups the batched verifier's persistent launch may
                              have (fewer when the pairs need fewer) */
    int32_t streamed;      /* 1: the join sized its stages on the device (see mj_join);
                              2: the same, replayed from captured graphs */
    int32_t host_reads;    /* reads of device values the host waited for: 2 when
                              streamed, 0 (not counted) stage by stage */
    int32_t member_filter; /* 1: only the records that may share their key went through
                              the record sort (see mj_ctx_set_member_filter) */
    int64_t members;       /* records sorted and grouped (records when member_filter is 0) */
} mj_stats;

/* ---- context ---------------------------------------------------------------- */

/* Device memory from the caller's pool (e.g. a framework's caching allocator).  alloc
 * returns `bytes` of device memory on the context's device, 256-byte aligned, or NULL;
 * free returns a block alloc gave.  The library calls them from the
 * thread of the entry point that needs the memory (a server's worker threads use their
 * own contexts, without an allocator), only after the stream work using a block has
 * completed when freeing it. */
typedef struct {
    void *(*alloc)(size_t bytes, void *user);
    void (*free)(void *ptr, void *user);
    void *user;
} mj_allocator;

/* Create a context on HIP device `device` (made current for the calls).  The context
 * owns a growable device workspace.  alloc (nullable, copied) backs every device buffer
 * the context's calls obtain -- the workspace, result pair lists, record lists and
 * indexes built with it (each result keeps the allocator to free itself); with NULL the
 * library uses hipMalloc.  EINVAL for a bad device or an allocator without alloc/free,
 * EDEVICE on HIP errors. */
mj_status mj_ctx_create(int device, const mj_allocator *alloc, mj_ctx **out);
void mj_ctx_destroy(mj_ctx *ctx);
/* Record-pair tests per candidate-emission pass (default 2^28, at least 1024): a join
 * whose groups hold more tests emits and deduplicates them in passes of this many, then
 * deduplicates the union, which bounds the candidate buffer (8 bytes per test of a pass)
 * however skewed the groups are.  EINVAL for a NULL context or a smaller value. */
mj_status mj_ctx_set_pair_test_pass(mj_ctx *ctx, int64_t tests);
/* Joins with at least min_records records (default 2^23; 0: every join; -1: none) first
 * keep only the records that may share their key with another one -- those whose key's top
 * 32 bits occur twice, found with two radix passes over 8-byte elements (ordering them by
 * the key's top 16 bits into buckets) and a per-bucket LDS bitmap -- and sort and group
 * those alone.  A bucket of more than bucket_limit records (0: the default, 65,536) is
 * kept whole.  Results are the same either way (a record whose key occurs once forms no
 * group); the filter saves time when most records are unique.  EINVAL for a NULL context,
 * min_records < -1 or bucket_limit < 0. */
mj_status mj_ctx_set_member_filter(mj_ctx *ctx, int64_t min_records, int32_t bucket_limit);
/* Candidate emission by tile pairs (Alg. 3's pair tests within a bucket of D): in a join
 * whose groups of 64 records or more hold at least min_tile_pairs tile pairs of 64 x 64
 * records (default 32,768; 0: every join with such groups; -1: none), those groups' record
 * pairs are tested a tile pair per wavefront and the smaller groups' test by test; else
 * every group's test by test.  Results are the same either way (the same pairs are tested
 * with the same filter); tile pairs save time when there are many of them.  A streamed
 * join follows the choice of the last join of its shape.  EINVAL for a NULL context or
 * min_tile_pairs < -1. */
mj_status mj_ctx_set_tile_emission(mj_ctx *ctx, int64_t min_tile_pairs);

/* How joins after the first (see mj_join) run: 0 stage by stage, each stage sized exactly
 * from a read-back (the least memory); 1 streamed (the default: stages sized on the device
 * from capacities, two host reads); 2 streamed and captured into two HIP graphs (the
 * set-up and everything after it), replayed while the strings' pointers and sizes, the
 * parameters and the set-up's results stay the same.  Captured joins give no kernel times
 * in mj_stats (stage_ms[0] is the set-up graph, stage_ms[7] the main graph).  EINVAL for a
 * NULL context or another mode. */
mj_status mj_ctx_set_streaming(mj_ctx *ctx, int mode);

/* Thread-local description of the last error (never NULL). */
const char *mj_last_error(void);

/* Library version string. */
const char *mj_version(void);

/* ---- join (Alg. 3): all pairs i < j with ED(s_i, s_j) <= K that share a partition
 * passing the filters ---------------------------------------------------------- */

/* Stream-ordered; returns once the pair count is known.  *out is library-owned until
 * mj_pairs_free.  stats may be NULL.
 * With the batched verifier, a join that follows one with the same parameters on the same
 * context runs streamed: every stage after the per-string set-up is sized on the device
 * (records by a bound from the set-up, candidates by the last join's rate, the verifier in
 * the configuration the context timed), so the host waits twice -- for the set-up and for
 * the result.  When a capacity turns out too small, the join runs again stage by stage
 * (which sizes every stage from read-backs) and the result is the same.  EINVAL on bad arguments (q < 1, q*b > 64,
 * t_div < 1, K < -1, sigma outside 2..256, offsets decreasing, a symbol code >= sigma,
 * verifier or verify_lanes not one of the listed values); ECAPACITY when a
 * documented limit is exceeded: a candidate whose threshold K is above 2047; ENOMEM when
 * device memory runs out.  Any radius r is taken: strings with r above 1920 are anchored
 * by a separate pass over their hashes in device memory (24 bytes per q-gram start). */
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

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): mj_verify's batched verification with
 * no context and no allocation of any kind.  Every scratch buffer comes from one fixed
 * array of 64 MiB in device memory that each GPU holds from the library's first such call
 * until the process ends (the call's device is the current HIP device).  Arguments, layout
 * and result are mj_verify's (params->verifier must be MJ_VERIFY_BATCHED; the lanes per
 * pair are the fixed small-call choice unless verify_lanes fixes them).  A call whose
 * strings, planes and pairs need more scratch than the array holds fails with
 * MJ_ECAPACITY before writing flags (about 12 bytes per string, 2-8 bits per symbol
 * (2 for 4 letters, 6 for 37), 8 bytes per pair, plus ~70 KB).  Calls on one GPU share
 * its array, which keeps the last call's contents: the library serialises them with a
 * lock and each returns only after its work on `stream` is complete, so calls from this
 * process never overlap on the device; calls that overlapped would race. */
mj_status mj_verify_noalloc(const mj_strings *strings, const mj_params *params,
                            const uint64_t *pairs, int64_t n, uint8_t *flags, void *stream);

/* ---- search: index the strings once, then find (query, string) pairs with
 * ED <= K_query.  Queries use the index's q, seed, t_div/t_fixed and reps. ------- */

/* Builds partitions of `strings` (Alg. 1-2) and keeps them sorted by key in device
 * memory, with the strings' bit planes for verification (2 bits per symbol for 4
 * letters) and their lengths and thresholds -- not the input symbols; inputs are
 * borrowed only during the call.  *out is library-owned until mj_index_free. */
mj_status mj_index_build(mj_ctx *ctx, const mj_strings *strings, const mj_params *params,
                         void *stream, mj_index **out);
void mj_index_free(mj_index *index);
int64_t mj_index_records(const mj_index *index);
/* Device memory the index holds, in bytes (records, planes, lengths, thresholds, offsets). */
int64_t mj_index_bytes(const mj_index *index);

/* queries: borrowed; qparams->k / k_per_string give each query's K, qparams->verifier and
 * verify_lanes choose the verifier as for mj_join (EINVAL on other values); q, seed, the
 * T rule and reps are taken from the index, which keeps its own copy of an injected Pi
 * table. */
mj_status mj_search(mj_ctx *ctx, const mj_index *index, const mj_strings *queries,
                    const mj_params *qparams, void *stream, mj_pairs **out,
                    mj_stats *stats);

/* ---- serving: continuous batching over a resident index ------------------------
 * Callers that submit queries one at a time (a request stream).  Worker threads each own
 * a HIP stream and a workspace on the index's device; a free worker admits every queued
 * request that fits (up to max_batch queries, and while the estimated device memory of
 * all batches in flight stays within memory_budget), so requests that arrive while other
 * batches run on the GPU join the next batch and the batches of different workers
 * overlap on the device.  A query's answer is the same as mj_search gives it alone:
 * queries of one batch do not interact. */

typedef struct mj_server mj_server;

typedef struct {
    int32_t workers;        /* batches in flight at once, 1..16 */
    int32_t max_batch;      /* queries per batch, 1..65536 */
    int64_t memory_budget;  /* bytes; a batch's estimate is 8 MiB plus 96 bytes per query
                               symbol and 4 KiB per query */
} mj_server_config;

typedef struct {
    uint64_t tag;           /* caller's tag from mj_server_submit */
    int32_t status;         /* mj_status of the batch that answered the request */
    int32_t count;          /* matching string ids written at ids[offset .. offset+count) */
    int64_t offset;
    int32_t batch_size;     /* queries in the batch that answered it */
    int32_t worker;
    double submit_ms;       /* times in ms since the server started */
    double start_ms;        /* its batch was admitted */
    double done_ms;         /* its batch completed */
    int64_t batch_estimate; /* the admission estimate of its batch (bytes) */
    int64_t batch_device;   /* device memory its batch used: the search's workspace blocks
                               and the batch's query buffers (bytes) */
} mj_reply;

/* The index must outlive the server.  EINVAL on bad config. */
mj_status mj_server_create(int device, const mj_index *index, const mj_server_config *cfg,
                           mj_server **out);
/* Copies the query (host symbol codes, length len >= 0) and queues it with threshold k
 * (0 <= k <= 2047).  EINVAL if a code is not below the index's sigma or if the request
 * alone exceeds the memory budget. */
mj_status mj_server_submit(mj_server *srv, const uint8_t *codes, int32_t len, int32_t k,
                           uint64_t tag);
/* Waits up to timeout_ms (0: no wait; < 0: until one reply) for completed requests and
 * moves up to max_replies of them to replies[], their matching ids (ascending) to
 * ids[0 .. ids_cap); stops early when ids_cap would be exceeded.  *n_replies and *n_ids
 * give what was written. */
mj_status mj_server_poll(mj_server *srv, mj_reply *replies, int32_t max_replies, uint32_t *ids,
                         int64_t ids_cap, int32_t timeout_ms, int32_t *n_replies,
                         int64_t *n_ids);
/* Requests queued or in flight (not yet polled). */
int64_t mj_server_pending(const mj_server *srv);
/* Finishes the batches in flight, drops queued requests, joins the workers. */
void mj_server_destroy(mj_server *srv);

/* ---- results ----------------------------------------------------------------- */

int64_t mj_pairs_count(const mj_pairs *p);
const uint64_t *mj_pairs_device(const mj_pairs *p);     /* count entries, sorted */
/* Copies count packed pairs to host memory; EINVAL if cap < count. */
mj_status mj_pairs_copy_to_host(const mj_pairs *p, uint64_t *dst, int64_t cap);
/* Returns the pairs' device memory: to the context's allocator when it has one, else to a
 * per-device stream-ordered pool (hipFreeAsync on the stream the pairs were made on, which
 * must still exist; work on other streams that reads the pairs must be complete).  Neither
 * the join's allocation of the result nor this free waits for the device. */
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
