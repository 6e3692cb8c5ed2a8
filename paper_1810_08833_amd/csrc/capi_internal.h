// Objects behind the opaque handles of the C-ABI (shared by capi.hip and server.hip).
#pragma once

#include "mj_common.h"

using namespace mj;

// What a join of the batched path learned for the next join with the same parameters:
// how many candidates (before the dedup) per record it emitted, the emission layout, and
// the verifier configuration it used.  With it, the next join sizes its stages from the
// set-up read-back alone (the streamed join: one more read, at the end).
struct StreamHints {
    bool valid = false;
    // parameters the hints belong to
    int32_t q = 0, t_div = 0, t_fixed = 0, reps = 0, sigma = 0, packing = 0, verify_lanes = 0;
    uint64_t seed = 0;
    int64_t k = 0;
    double cand_per_record = 0;  // emitted candidates (before the dedup) per record bound
    double rec_per_bound = 1;    // records per record bound
    double mem_per_bound = 1;    // records kept by the member filter per record bound
    EmitHints emit;
    int verify_g = 0, verify_blocks = 0;
};

// Sizes of a streamed join, fixed by the set-up read-back and the hints of the last join,
// and the device buffer the host copies the result from after the final read.
struct StreamedPlan {
    SetupInfo si;
    int cmax = 0;
    int64_t rcap = 0, scap = 0, ccap = 0;
    bool members = false;  // the member filter runs; mcap: room for its records
    int64_t mcap = 0;
    EmitHints emit;
};
struct StreamedDev {
    uint64_t *outbuf = nullptr;
};

// A captured join (see run_join_graph in capi.hip): the strings and parameters it was
// captured for, its two executable graphs, and what the host needs around them.
struct JoinGraph {
    const void *chars = nullptr;
    const int64_t *offsets = nullptr;
    int32_t n = 0, sigma = 0, packing = 0;
    mj_params params{};
    hipGraphExec_t setup = nullptr, main = nullptr;
    DevStrings d, md;      // after the set-up graph; with the planes of the main graph
    PartitionParams pp{};
    SetupInfo si;          // the set-up results the main graph was captured for
    int64_t total = -1;
    StreamedPlan plan;     // sizes and buffers of the main graph
    StreamedDev dv;
};

struct mj_ctx {
    int device = 0;
    Workspace ws;
    uint64_t *pinned = nullptr;  // host scratch for read-backs (HOST_SCRATCH_BYTES)
    hipEvent_t ev[9] = {};
    KTimer kt;
    VerifyTuning tune;
    // latency first (server workers): the batched verifier takes its fixed small-call
    // configuration instead of timing the choices on a live call
    bool no_tuning = false;
    int64_t pair_test_pass = (int64_t)1 << 28;  // record-pair tests per emission pass
    int64_t tile_min = EMIT_SPLIT_UNITS;          // tile pairs for the tile emission (-1: never)
    int64_t member_min = (int64_t)1 << 23;      // records from which the member filter runs
    uint32_t member_big = 1u << 16;             // its buckets above this are kept whole
    int streaming = 1;  // 0 stage by stage, 1 streamed, 2 streamed and captured (mj_ctx_set_streaming)
    StreamHints stream;
    JoinGraph graph;
    hipStream_t cap_stream = nullptr;  // the stream graphs are captured on
    int streamed_joins = 0, stream_fallbacks = 0;
    // the last stage-by-stage join's emitted candidates, records and record bound, and its
    // pair tests of the small groups and tile pairs of the large ones
    int64_t last_c0 = 0, last_R = 0, last_rcap = 0, last_M = 0;
    uint64_t last_small_tests = 0, last_units = 0;
};

struct mj_pairs {
    uint64_t *d = nullptr;
    int64_t n = 0;
    mj_allocator alloc{};  // the allocator that made d
    hipStream_t stream = nullptr;  // d is complete once this stream's work is
};

struct mj_records {
    RecBuf rb;
};

struct mj_index {
    int device = 0;
    PartitionParams pp{};
    int32_t n = 0, sigma = 0, bits = 0;
    int64_t total = 0;
    int64_t *offsets = nullptr;
    int32_t *len = nullptr, *kk = nullptr;
    uint32_t *planes = nullptr;
    int64_t plane_words = 0;
    int np = 0;
    uint64_t *pi_table = nullptr;  // the index's own copy of an injected Pi table
    RecBuf rec;  // sorted by key
    mj_allocator alloc{};  // the allocator that made the index's arrays
};

// Sets the thread-local error message and returns the status.
mj_status mj_fail(mj_status st, const std::string &m);
