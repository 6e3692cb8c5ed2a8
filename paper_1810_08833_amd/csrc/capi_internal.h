// Objects behind the opaque handles of the C-ABI (shared by capi.hip and server.hip).
#pragma once

#include "mj_common.h"

using namespace mj;

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
};

struct mj_pairs {
    uint64_t *d = nullptr;
    int64_t n = 0;
    mj_allocator alloc{};  // the allocator that made d
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
