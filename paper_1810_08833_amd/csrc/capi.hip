// C-ABI of libminjoin: argument checks, stage sequencing on the caller's stream, count
// read-backs between stages, per-stage HIP-event timers and result ownership.
#include <string.h>

#include <algorithm>
#include <string>

#include "capi_internal.h"

using namespace mj;

static thread_local std::string g_err = "no error";

static mj_status fail(mj_status st, const std::string &m) {
    g_err = m;
    return st;
}

mj_status mj_fail(mj_status st, const std::string &m) { return fail(st, m); }

#define MJ_API_BEGIN try {
#define MJ_API_END                                            \
    }                                                         \
    catch (const mj::Error &e) {                              \
        return fail(e.status, e.what());                      \
    }                                                         \
    catch (const std::exception &e) {                         \
        return fail(MJ_EDEVICE, e.what());                    \
    }                                                         \
    catch (...) {                                             \
        return fail(MJ_EDEVICE, "unknown error");             \
    }

extern "C" const char *mj_last_error(void) { return g_err.c_str(); }

extern "C" const char *mj_version(void) { return "minjoin-mi355x 0.1 (gfx950)"; }

extern "C" mj_status mj_ctx_create(int device, const mj_allocator *alloc, mj_ctx **out) {
    if (!out) return fail(MJ_EINVAL, "out is NULL");
    if (alloc && (!alloc->alloc || !alloc->free)) return fail(MJ_EINVAL, "allocator needs alloc and free");
    MJ_API_BEGIN
    int count = 0;
    MJ_HIP(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) return fail(MJ_EINVAL, "bad device index");
    MJ_HIP(hipSetDevice(device));
    mj_ctx *c = new mj_ctx();
    c->device = device;
    if (alloc) c->ws.alloc = *alloc;
    if (hipHostMalloc((void **)&c->pinned, HOST_SCRATCH_BYTES, hipHostMallocDefault) != hipSuccess) {
        delete c;
        return fail(MJ_ENOMEM, "pinned host allocation failed");
    }
    for (auto &e : c->ev) MJ_HIP(hipEventCreate(&e));
    c->kt.create();
    *out = c;
    return MJ_OK;
    MJ_API_END
}

extern "C" void mj_ctx_destroy(mj_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    AllocScope as(ctx->ws.alloc);
    if (ctx->graph.setup) (void)hipGraphExecDestroy(ctx->graph.setup);
    if (ctx->graph.main) (void)hipGraphExecDestroy(ctx->graph.main);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    for (auto &e : ctx->ev)
        if (e) (void)hipEventDestroy(e);
    ctx->kt.destroy();
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    delete ctx;
}

static void graph_drop(mj_ctx *ctx);

extern "C" mj_status mj_ctx_set_pair_test_pass(mj_ctx *ctx, int64_t tests) {
    if (!ctx) return fail(MJ_EINVAL, "ctx is NULL");
    if (tests < 1024) return fail(MJ_EINVAL, "a pass must hold at least 1024 pair tests");
    ctx->pair_test_pass = tests;
    return MJ_OK;
}

extern "C" mj_status mj_ctx_set_tile_emission(mj_ctx *ctx, int64_t min_tile_pairs) {
    if (!ctx) return fail(MJ_EINVAL, "ctx is NULL");
    if (min_tile_pairs < -1) return fail(MJ_EINVAL, "min_tile_pairs must be >= -1");
    ctx->tile_min = min_tile_pairs;
    return MJ_OK;
}

extern "C" mj_status mj_ctx_set_member_filter(mj_ctx *ctx, int64_t min_records,
                                              int32_t bucket_limit) {
    if (!ctx) return fail(MJ_EINVAL, "ctx is NULL");
    if (min_records < -1) return fail(MJ_EINVAL, "min_records must be >= -1");
    if (bucket_limit < 0) return fail(MJ_EINVAL, "bucket_limit must be >= 0");
    ctx->member_min = min_records;
    ctx->member_big = bucket_limit ? (uint32_t)bucket_limit : 1u << 16;
    return MJ_OK;
}

static bool use_members(const mj_ctx *ctx, int64_t records) {
    return ctx->member_min >= 0 && records >= std::max<int64_t>(ctx->member_min, 2);
}

extern "C" mj_status mj_ctx_set_streaming(mj_ctx *ctx, int mode) {
    if (!ctx) return fail(MJ_EINVAL, "ctx is NULL");
    if (mode < 0 || mode > 2) return fail(MJ_EINVAL, "streaming mode must be 0, 1 or 2");
    MJ_API_BEGIN
    MJ_HIP(hipSetDevice(ctx->device));
    if (mode != 2) graph_drop(ctx);
    ctx->streaming = mode;
    return MJ_OK;
    MJ_API_END
}

// ---------------------------------------------------------------- helpers
// The verify_lanes / verify_group code of a batched configuration: lanes per pair, -2 for
// the column split, -3 for the band classes.
static int lanes_code(int g) {
    return g == VERIFY_BIDIR ? -2 : g == VERIFY_CLASSES ? -3 : g;
}

// Band words per lane of configuration g for a band of cmax words (the window holds
// cmax + 1), 0 when it cannot hold it; the band classes give their widest class's 4.
static int window_words_per_lane(int g, int cmax) {
    if (g == VERIFY_CLASSES) return cmax + 1 <= 32 ? 4 : 0;
    for (int v : {1, 2, 3, 4, 5, 6, 7, 8, 9, 11})
        if (v * (g == VERIFY_BIDIR ? 1 : g) >= cmax + 1) return v;
    return 0;
}

static void check_verifier(const mj_params *p) {
    if (p->verifier != MJ_VERIFY_BATCHED && p->verifier != MJ_VERIFY_PLAIN)
        throw Error(MJ_EINVAL, "verifier must be MJ_VERIFY_BATCHED or MJ_VERIFY_PLAIN");
    if (p->verify_lanes != 0 && p->verify_lanes != 1 && p->verify_lanes != 2 &&
        p->verify_lanes != 4 && p->verify_lanes != 8 && p->verify_lanes != -2 &&
        p->verify_lanes != -3)
        throw Error(MJ_EINVAL, "verify_lanes must be 0, 1, 2, 4, 8, -2 or -3");
}

static void check_params(const mj_params *p, int sigma, bool need_k) {
    if (!p) throw Error(MJ_EINVAL, "params is NULL");
    if (sigma < 2 || sigma > 256) throw Error(MJ_EINVAL, "sigma must be in 2..256");
    int b = symbol_bits(sigma);
    if (p->q < 1 || (int64_t)p->q * b > 64) throw Error(MJ_EINVAL, "q must satisfy 1 <= q*ceil(log2 sigma) <= 64");
    if (p->t_fixed <= 0 && p->t_div < 1) throw Error(MJ_EINVAL, "t_div must be >= 1");
    if (p->reps < 0 || p->reps > 64) throw Error(MJ_EINVAL, "reps must be in 0..64");
    if (need_k) {
        if (p->k > 2047) throw Error(MJ_ECAPACITY, "threshold K exceeds the verifier's band limit (K <= 2047)");
        if (p->k < -1) throw Error(MJ_EINVAL, "k must be >= 0 or -1");
        if (p->k == -1 && !p->k_per_string) throw Error(MJ_EINVAL, "k == -1 needs k_per_string");
        if (p->k > 0x3FFFFFFF) throw Error(MJ_EINVAL, "k too large");
    }
    if (p->pi_table && (int64_t)p->q * b > 24) throw Error(MJ_EINVAL, "pi_table needs q*b <= 24");
    check_verifier(p);
}

static void check_strings(const mj_strings *s) {
    if (!s) throw Error(MJ_EINVAL, "strings is NULL");
    if (s->n < 0) throw Error(MJ_EINVAL, "n must be >= 0");
    if (s->n > 0 && (!s->offsets)) throw Error(MJ_EINVAL, "offsets is NULL");
    if (s->packing != MJ_PACK_U8 && s->packing != MJ_PACK_2BIT)
        throw Error(MJ_EINVAL, "packing must be MJ_PACK_U8 or MJ_PACK_2BIT");
    if (s->packing == MJ_PACK_2BIT && (s->sigma > 4 || ((uintptr_t)s->chars & 3)))
        throw Error(MJ_EINVAL, "2-bit packing needs sigma <= 4 and 4-byte aligned words");
}

static PartitionParams to_pp(const mj_params *p, int bits) {
    PartitionParams pp;
    pp.q = p->q;
    pp.bits = bits;
    pp.t_div = std::max(1, p->t_div);
    pp.t_fixed = p->t_fixed;
    pp.reps = p->reps > 0 ? p->reps : 1;
    pp.seed = p->seed;
    pp.k = p->k;
    pp.k_per_string = p->k_per_string;
    pp.pi_table = p->pi_table;
    return pp;
}

// With read_total false the symbol count stays unknown (-1) until prepare_strings reads it
// back together with its own results.
static DevStrings view(const mj_strings *s, hipStream_t st, uint64_t *pinned,
                       bool read_total = true) {
    DevStrings d;
    d.chars = s->chars;
    d.packing = s->packing;
    d.offsets = s->offsets;
    d.n = s->n;
    d.sigma = s->sigma;
    d.bits = symbol_bits(s->sigma);
    if (!read_total && s->n > 0) {
        d.total = -1;
        return d;
    }
    d.total = s->n > 0 ? read_back<int64_t>(s->offsets + s->n, st, pinned) : 0;
    check_total(d);
    return d;
}

// All partitions of all repetitions, sorted by key (stable: equal keys keep partition order).
static void sorted_records(const DevStrings &d, const PartitionParams &pp, int32_t halo, RecBuf &rb,
                           Workspace &ws, hipStream_t s, uint64_t *pinned) {
    partition_records(d, pp, halo, rb, ws, s, pinned);
    int64_t R = rb.count;
    if (R > 1) {
        sort_records(rb.key, rb.val, R, ws, s, pinned);
    }
}

static mj_pairs *compact_pairs(const uint64_t *pairs, const uint8_t *flags, int64_t n, Workspace &ws,
                               hipStream_t s, uint64_t *pinned) {
    mj_pairs *out = new mj_pairs();
    out->alloc = t_dev_alloc;
    out->stream = s;
    if (n == 0) {
        out->d = (uint64_t *)result_alloc(16, out->alloc, s);
        out->n = 0;
        return out;
    }
    // flags are 0/1 here (2 would mean an unhandled band, rejected earlier)
    int64_t *idx = ws.get_n<int64_t>(n + 1);
    int64_t c = compact_flags(flags, n, idx, ws, s, pinned);
    out->d = (uint64_t *)result_alloc((size_t)(c + 1) * 8, out->alloc, s);
    gather_u64(pairs, idx, out->d, c, s);
    out->n = c;
    return out;
}

__global__ void k_check_flags(const uint8_t *f, int64_t n, uint32_t *bad) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride)
        if (f[i] > 1) atomicOr(bad, 1u);
}

static void check_flags(const uint8_t *f, int64_t n, Workspace &ws, hipStream_t s, uint64_t *pinned) {
    if (n <= 0) return;
    uint32_t *bad = ws.get_n<uint32_t>(2);
    fill_u32(bad, 0, 1, s);
    unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, 16384);
    hipLaunchKernelGGL(k_check_flags, dim3(g), dim3(256), 0, s, f, n, bad);
    MJ_LAUNCH_CHECK();
    if (read_back<uint32_t>(bad, s, pinned)) throw Error(MJ_ECAPACITY, "threshold K exceeds the verifier's band limit (K <= 2047)");
}

// Verification of library-produced pairs with the chosen verifier.
// The band-cell count lands in *cells_h (pinned), valid after the stream's next
// synchronisation.
static void run_verify(mj_ctx *ctx, const uint64_t *pairs, int64_t n, const DevStrings &A,
                       const DevStrings &B, int kmode, int64_t uniform_k, const mj_params *p,
                       uint8_t *flags, hipStream_t s, mj_stats *stats, uint64_t *cells_h) {
    cells_h[0] = cells_h[1] = 0;
    if (p->verifier == MJ_VERIFY_BATCHED) {
        verify_pairs_batched(pairs, n, A, B, kmode, flags, ctx->ws, s, ctx->pinned, &ctx->kt,
                             ctx->no_tuning ? nullptr : &ctx->tune, uniform_k, cells_h,
                             p->verify_lanes);
        if (stats) {
            stats->verify_group = lanes_code(ctx->tune.last_g);
            stats->verify_words = ctx->tune.last_nwl;
            stats->verify_blocks = ctx->tune.last_blocks;
        }
        return;
    }
    *cells_h = (uint64_t)verify_pairs(pairs, n, A, B, kmode, flags, ctx->ws, s, ctx->pinned,
                                      &ctx->kt, uniform_k);
    if (uniform_k < 0) check_flags(flags, n, ctx->ws, s, ctx->pinned);
}

// last two words of the pinned scratch: the deferred band-cell count and the batched
// verifier's undersized-window error word
static uint64_t *cells_slot(mj_ctx *ctx) { return ctx->pinned + HOST_SCRATCH_BYTES / 8 - 2; }

// After the stream has synchronised: the deferred band-cell count; fails (freeing `out`)
// when some pair's band did not fit the verifier's window.
static int64_t take_cells(mj_ctx *ctx, mj_pairs *out) {
    const uint64_t *c = cells_slot(ctx);
    if (c[1]) {
        mj_pairs_free(out);
        throw Error(MJ_ECAPACITY, "a pair's band exceeds the verifier window");
    }
    return (int64_t)c[0];
}

struct StageTimer {
    mj_ctx *ctx;
    hipStream_t s;
    int next = 0;
    StageTimer(mj_ctx *c, hipStream_t st) : ctx(c), s(st) {
        ctx->kt.reset();
        mark();
    }
    void mark() {
        if (next < 9) MJ_HIP(hipEventRecord(ctx->ev[next++], s));
    }
    void fill(mj_stats *st) {
        if (!st) return;
        MJ_HIP(hipStreamSynchronize(s));
        for (int i = 0; i < 8; i++) {
            float ms = 0.f;
            if (i + 1 < next) MJ_HIP(hipEventElapsedTime(&ms, ctx->ev[i], ctx->ev[i + 1]));
            st->stage_ms[i] = ms;
        }
        ctx->kt.collect(st->kernel_ms, st->kernel_launches);
    }
};

struct Released {
    Workspace &ws;
    ~Released() { ws.release_all(); }
};

// ---------------------------------------------------------------- join pipeline
// Runs the join up to `upto`: 1 = candidates, 2 = output.  Fills stats.
static mj_pairs *run_join(mj_ctx *ctx, const mj_strings *strings, const mj_params *params,
                          hipStream_t s, int upto, mj_stats *stats) {
    Workspace &ws = ctx->ws;
    Released rel{ws};
    StageTimer tm(ctx, s);
    DevStrings d = view(strings, s, ctx->pinned, false);
    PartitionParams pp = to_pp(params, d.bits);
    SetupInfo si;
    int32_t halo = prepare_strings(d, pp, ws, s, ctx->pinned, &si);
    pack_planes(d, verify_planes(d.bits), ws, s);  // also checks the symbol codes
    tm.mark();  // 0 setup
    RecBuf rb;
    rb.ws = &ws;  // workspace memory: cached across calls, returned when the call ends
    partition_records(d, pp, halo, rb, ws, s, ctx->pinned, &ctx->kt);
    tm.mark();  // 1 partition: anchors and records
    int64_t R = rb.count;
    // the records that are sorted and grouped: all of them, or those the member filter keeps
    uint64_t *gkey = rb.key, *gval = rb.val;
    int64_t M = R;
    const bool members = use_members(ctx, R);
    if (members) {
        gkey = ws.get_n<uint64_t>(R + 1);
        gval = ws.get_n<uint64_t>(R + 1);
        int64_t *m_dev = ws.get_n<int64_t>(2);
        group_members(rb.key, rb.val, R, nullptr, gkey, gval, R, m_dev, ctx->member_big, ws, s);
        M = read_back<int64_t>(m_dev, s, ctx->pinned);
    }
    if (M > 1) {
        sort_records(gkey, gval, M, ws, s, ctx->pinned);
    }
    tm.mark();  // 2 sort
    GroupInfo g = find_groups(gkey, M, ws, s, ctx->pinned);
    uint64_t *uniq = nullptr;
    int64_t C = 0;
    const uint64_t pass_tests = (uint64_t)ctx->pair_test_pass;
    if (g.tests <= pass_tests) {
        int64_t cap = (int64_t)g.tests;
        uint64_t *cand = ws.get_n<uint64_t>(cap + 1);
        int64_t c0 = emit_candidates(gval, M, g, d, cand, cap, ws, s, ctx->pinned, ctx->tile_min,
                                     &ctx->kt);
        ctx->last_c0 = c0;
        tm.mark();  // 3 group + filter
        C = dedup_pairs(cand, c0, d.n, d.n, ws, s, ctx->pinned, &uniq, upto != 1);
    } else {
        // more record-pair tests than one pass holds (huge groups): emit and dedup them in
        // passes, then dedup the union of the passes' distinct pairs
        std::vector<std::pair<uint64_t *, int64_t>> parts;  // workspace blocks
        int64_t total_u = 0;
        uint64_t *cand = ws.get_n<uint64_t>(pass_tests + 1);
        for (uint64_t t0 = 0; t0 < g.tests; t0 += pass_tests) {
            const uint64_t t1 = std::min(g.tests, t0 + pass_tests);
            int64_t c0 = emit_candidates(gval, M, g, d, cand, (int64_t)pass_tests, ws, s,
                                         ctx->pinned, ctx->tile_min, &ctx->kt, t0, t1);
            uint64_t *u = nullptr;
            const int64_t nu = dedup_pairs(cand, c0, d.n, d.n, ws, s, ctx->pinned, &u, true);
            parts.push_back({u, nu});
            total_u += nu;
        }
        uint64_t *all = ws.get_n<uint64_t>(total_u + 1);
        int64_t at = 0;
        for (auto &pr : parts) {
            if (pr.second)
                MJ_HIP(hipMemcpyAsync(all + at, pr.first, (size_t)pr.second * 8,
                                      hipMemcpyDeviceToDevice, s));
            at += pr.second;
        }
        ctx->last_c0 = total_u;
        tm.mark();  // 3 group + filter
        C = dedup_pairs(all, total_u, d.n, d.n, ws, s, ctx->pinned, &uniq, upto != 1);
    }
    ctx->last_R = R;
    ctx->last_M = M;
    ctx->last_small_tests = g.small_tests;
    ctx->last_units = g.units;
    ctx->last_rcap = std::max<int64_t>(si.rec_bound * pp.reps, 2);
    tm.mark();  // 4 dedup
    if (stats) {
        memset(stats, 0, sizeof(*stats));
        stats->records = R;
        stats->groups = g.groups;
        stats->pair_tests = (int64_t)g.tests;
        stats->candidates = C;
        stats->positions = d.total * pp.reps;
        stats->member_filter = members ? 1 : 0;
        stats->members = M;
    }
    if (upto == 1) {
        mj_pairs *out = new mj_pairs();
        out->alloc = t_dev_alloc;
        out->stream = s;
        out->d = uniq;
        out->n = C;
        tm.fill(stats);
        return out;
    }
    uint8_t *flags = ws.get_n<uint8_t>(C + 1);
    run_verify(ctx, uniq, C, d, d, 0, params->k, params, flags, s, stats, cells_slot(ctx));
    tm.mark();  // 5 verify
    mj_pairs *out = compact_pairs(uniq, flags, C, ws, s, ctx->pinned);  // synchronises when C > 0
    const int64_t cells = take_cells(ctx, out);
    tm.mark();  // 6 output
    if (stats) {
        stats->output = out->n;
        stats->band_cells = cells;
    }
    tm.fill(stats);
    return out;
}

// ---------------------------------------------------------------- streamed join
// The batched join with every size after the set-up on the device: records by the set-up's
// bound, candidates by the last join's candidates-per-record (with room to spare), the
// verifier in the configuration the context timed.  Between the set-up read-back and the
// final one, no stage waits for the host.  Returns nullptr when a capacity was exceeded
// (the caller then runs the join stage by stage, which sizes everything exactly).

__global__ void k_collect(const int64_t *R, const uint64_t *slot, const unsigned long long *c0,
                          const uint32_t *u, const uint32_t *outn, const unsigned long long *cells,
                          const uint32_t *symbol_err, const int64_t *M, uint64_t *dst) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    dst[10] = (uint64_t)*M;
    dst[9] = symbol_err ? *symbol_err : 0;
    dst[0] = (uint64_t)*R;
    dst[1] = slot ? slot[0] : 0;
    dst[2] = slot ? slot[1] : 0;
    dst[3] = slot ? slot[2] : 0;
    dst[4] = *c0;
    dst[5] = *u;
    dst[6] = *outn;
    dst[7] = cells[0];
    dst[8] = cells[1];
    dst[11] = slot ? slot[3] : 0;
    dst[12] = slot ? slot[4] : 0;
}

static bool hints_match(const StreamHints &h, const mj_strings *st, const mj_params *p) {
    return h.valid && h.q == p->q && h.t_div == p->t_div && h.t_fixed == p->t_fixed &&
           h.reps == p->reps && h.seed == p->seed && h.k == p->k && h.sigma == st->sigma &&
           h.packing == st->packing && h.verify_lanes == p->verify_lanes;
}

static bool plan_streamed(mj_ctx *ctx, const mj_params *params, const DevStrings &d,
                          const PartitionParams &pp, const SetupInfo &si, StreamedPlan &pl) {
    const StreamHints &h = ctx->stream;
    pl.si = si;
    pl.cmax = (int)((std::min<int64_t>(params->k >= 0 ? params->k : si.kmax, 0x3FFFFFFF) + 31) >> 5);
    if (pl.cmax > persist_max_c()) return false;
    const int np = verify_planes(d.bits);
    // the configuration the last join used (the small-call one if it verified nothing)
    const int g = params->verify_lanes == -2 ? VERIFY_BIDIR
                : params->verify_lanes == -3 ? VERIFY_CLASSES
                : params->verify_lanes ? params->verify_lanes
                : h.verify_g ? h.verify_g : verify_small_call_lanes(pl.cmax);
    const int nwl = window_words_per_lane(g, pl.cmax);
    if (g == 0 || nwl == 0) return false;  // no configuration for this band: stage by stage
    const int ci = std::min(pl.cmax, 63);
    ctx->tune.best_g[ci][np / 2 - 1] = g;
    if (!ctx->tune.best_blocks[ci][np / 2 - 1])
        ctx->tune.best_blocks[ci][np / 2 - 1] = h.verify_blocks ? h.verify_blocks : 512;
    pl.rcap = std::max<int64_t>(si.rec_bound * pp.reps, 2);
    // the stages after the partition are sized by the last join's records per bound, with
    // room (more records than that: the join runs again stage by stage)
    pl.scap = std::max<int64_t>(
        2, std::min<int64_t>(pl.rcap, (int64_t)(1.02 * h.rec_per_bound * (double)pl.rcap) + 4096));
    // candidates before the dedup: the last join's rate per record bound, with room
    const double ccap = 1.1 * h.cand_per_record * (double)pl.rcap + 65536.0;
    if (ccap > (double)std::min<int64_t>(ctx->pair_test_pass, 0x7FFFFFF0LL))
        return false;  // candidates beyond one emission pass: stage by stage, in passes
    pl.ccap = (int64_t)ccap;
    // the member filter's records: the last join's rate per record bound, with room
    pl.members = use_members(ctx, pl.scap);
    pl.mcap = pl.members ? std::max<int64_t>(2, std::min<int64_t>(
                               pl.scap, (int64_t)(1.1 * h.mem_per_bound * (double)pl.rcap) + 65536))
                         : pl.scap;
    pl.emit = h.emit;
    return true;
}

// Everything from the plane packing to the copy of the result counts into ctx->pinned,
// with no host read.  tm and kt are null while the launches are captured into a graph.
static StreamedDev launch_streamed_main(mj_ctx *ctx, DevStrings &d, const PartitionParams &pp,
                                        const StreamedPlan &pl, const mj_params *params,
                                        hipStream_t s, StageTimer *tm, KTimer *kt) {
    Workspace &ws = ctx->ws;
    StreamedDev dv;
    pack_planes(d, verify_planes(d.bits), ws, s);
    if (tm) tm->mark();  // 0 setup
    uint64_t *key = ws.get_n<uint64_t>(pl.rcap + 1);
    uint64_t *val = ws.get_n<uint64_t>(pl.rcap + 1);
    int64_t *R_dev = ws.get_n<int64_t>(2);
    partition_records_streamed(d, pp, pl.si, key, val, R_dev, ws, s, kt);
    if (tm) tm->mark();  // 1 partition
    uint64_t *gkey = key, *gval = val;
    int64_t *M_dev = R_dev;
    if (pl.members) {
        gkey = ws.get_n<uint64_t>(pl.mcap + 1);
        gval = ws.get_n<uint64_t>(pl.mcap + 1);
        M_dev = ws.get_n<int64_t>(2);
        group_members(key, val, pl.scap, R_dev, gkey, gval, pl.mcap, M_dev, ctx->member_big, ws, s);
    }
    sort_records(gkey, gval, pl.mcap, ws, s, ctx->pinned, M_dev);
    if (tm) tm->mark();  // 2 sort
    GroupInfo g = find_groups_streamed(gkey, pl.mcap, M_dev, ws, s);
    uint64_t *cand = ws.get_n<uint64_t>(pl.ccap + 1);
    unsigned long long *c0 = (unsigned long long *)ws.get_n<uint64_t>(2);
    emit_candidates_streamed(gval, pl.mcap, M_dev, g, d, cand, pl.ccap, c0, pl.emit, ws, s, kt);
    if (tm) tm->mark();  // 3 group + filter
    uint64_t *uniq = nullptr;
    const uint32_t *u = dedup_pairs_streamed(cand, pl.ccap, c0, d.n, d.n, ws, s, &uniq);
    if (tm) tm->mark();  // 4 dedup
    uint8_t *flags = ws.get_n<uint8_t>(pl.ccap + 4);
    unsigned long long *cells = nullptr;
    verify_pairs_batched_streamed(uniq, pl.ccap, u, d, d, 0, pl.cmax, flags, ws, s, kt, ctx->tune,
                                  params->verify_lanes, &cells);
    if (tm) tm->mark();  // 5 verify
    int64_t *idx = ws.get_n<int64_t>(pl.ccap + 1);
    const uint32_t *on = compact_flags_async(flags, pl.ccap, idx, ws, s);
    dv.outbuf = ws.get_n<uint64_t>(pl.ccap + 1);
    gather_u64(uniq, idx, dv.outbuf, pl.ccap, s, on);
    uint64_t *res = ws.get_n<uint64_t>(16);
    hipLaunchKernelGGL(k_collect, dim3(1), dim3(64), 0, s, R_dev, g.slot, c0, u, on, cells,
                       (const uint32_t *)d.symbol_err, M_dev, res);
    MJ_LAUNCH_CHECK();
    MJ_HIP(hipMemcpyAsync(ctx->pinned, res, 13 * 8, hipMemcpyDeviceToHost, s));
    return dv;
}

// After the final synchronisation: the counts, the result pairs, the stats and the hints
// of the next join.  nullptr when a capacity was exceeded.
static mj_pairs *finish_streamed(mj_ctx *ctx, const StreamedPlan &pl, const StreamedDev &dv,
                                 const DevStrings &d, const PartitionParams &pp, hipStream_t s,
                                 mj_stats *stats) {
    uint64_t hv[13];
    memcpy(hv, ctx->pinned, sizeof(hv));
    const int64_t R = (int64_t)hv[0], c0h = (int64_t)hv[4], C = (int64_t)hv[5], nout = (int64_t)hv[6];
    const int64_t M = (int64_t)hv[10];
    if (hv[9]) throw Error(MJ_EINVAL, "a symbol code is not below sigma");
    // more than the room left: stage by stage
    if (c0h > pl.ccap || R > pl.scap || M > pl.mcap) return nullptr;
    if (M > 1 && (hv[1] & 0xFFFFFFFFu) != (hv[1] >> 32)) throw Error(MJ_EDEVICE, "group boundary mismatch");
    if (hv[8]) throw Error(MJ_ECAPACITY, "a pair's band exceeds the verifier window");
    mj_pairs *out = new mj_pairs();
    out->alloc = t_dev_alloc;
    out->stream = s;
    out->n = nout;
    out->d = (uint64_t *)result_alloc((size_t)(nout + 1) * 8, out->alloc, s);
    if (nout) MJ_HIP(hipMemcpyAsync(out->d, dv.outbuf, (size_t)nout * 8, hipMemcpyDeviceToDevice, s));
    if (stats) {
        memset(stats, 0, sizeof(*stats));
        stats->records = R;
        stats->groups = (int64_t)hv[2];
        stats->pair_tests = (int64_t)hv[3];
        stats->candidates = C;
        stats->output = nout;
        stats->band_cells = (int64_t)hv[7];
        stats->positions = d.total * pp.reps;
        const int ci = std::min(pl.cmax, 63), npi = verify_planes(d.bits) / 2 - 1;
        const int gg = ctx->tune.best_g[ci][npi];
        stats->verify_group = lanes_code(gg);
        stats->verify_words = window_words_per_lane(gg, pl.cmax);
        stats->verify_blocks = ctx->tune.best_blocks[ci][npi];
        stats->streamed = 1;
        stats->host_reads = 2;
        stats->member_filter = pl.members ? 1 : 0;
        stats->members = M;
    }
    // keep the rates current (capacities of the next join)
    ctx->stream.cand_per_record = (double)c0h / (double)pl.rcap;
    ctx->stream.rec_per_bound = (double)R / (double)pl.rcap;
    ctx->stream.mem_per_bound = (double)M / (double)pl.rcap;
    ctx->stream.emit = emit_hints((uint64_t)hv[3], (uint64_t)hv[11], (uint64_t)hv[12], M, d.n,
                                  ctx->tile_min);
    return out;
}

static mj_pairs *run_join_streamed(mj_ctx *ctx, const mj_strings *strings, const mj_params *params,
                                   hipStream_t s, mj_stats *stats) {
    Workspace &ws = ctx->ws;
    Released rel{ws};
    StageTimer tm(ctx, s);
    DevStrings d = view(strings, s, ctx->pinned, false);
    PartitionParams pp = to_pp(params, d.bits);
    SetupInfo si;
    (void)prepare_strings(d, pp, ws, s, ctx->pinned, &si);  // the one read before the end
    StreamedPlan pl;
    if (!plan_streamed(ctx, params, d, pp, si, pl)) return nullptr;
    StreamedDev dv = launch_streamed_main(ctx, d, pp, pl, params, s, &tm, &ctx->kt);
    MJ_HIP(hipStreamSynchronize(s));  // the one read at the end
    mj_pairs *out = finish_streamed(ctx, pl, dv, d, pp, s, stats);
    if (out) {
        tm.mark();  // 6 output
        tm.fill(stats);
    }
    return out;
}

// ---------------------------------------------------------------- captured join
// The streamed join captured into two HIP graphs and replayed while the strings, the
// parameters and the set-up results stay the same: the set-up graph (per-string
// parameters and their read-back), then, once the host has checked those, the main graph
// (planes to the result counts).  Workspace blocks used by the graphs are held for them;
// scans take their multi-pass form (no state carried between calls).  Kernel timers cannot
// sit inside a graph: the stats give the two graphs' times only (stage 0 and stage 7).

static void graph_drop(mj_ctx *ctx) {
    JoinGraph &gr = ctx->graph;
    if (gr.setup) (void)hipGraphExecDestroy(gr.setup);
    if (gr.main) (void)hipGraphExecDestroy(gr.main);
    gr = JoinGraph();
    ctx->ws.drop_holds();
}

static bool graph_key_matches(const JoinGraph &gr, const mj_strings *st, const mj_params *p) {
    return gr.setup && gr.chars == st->chars && gr.offsets == st->offsets && gr.n == st->n &&
           gr.sigma == st->sigma && gr.packing == st->packing &&
           memcmp(&gr.params, p, sizeof(mj_params)) == 0;
}

// Captures fn's launches on the context's capture stream into an executable graph.
template <class F>
static hipGraphExec_t capture(mj_ctx *ctx, F fn) {
    if (!ctx->cap_stream) MJ_HIP(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    hipStream_t cs = ctx->cap_stream;
    MJ_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));  // workspace blocks may be allocated
    ctx->ws.hold(true);
    ctx->ws.no_lookback = true;
    try {
        fn(cs);
    } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(cs, &g);
        if (g) (void)hipGraphDestroy(g);
        ctx->ws.hold(false);
        ctx->ws.no_lookback = false;
        throw;
    }
    ctx->ws.hold(false);
    ctx->ws.no_lookback = false;
    hipGraph_t g = nullptr;
    MJ_HIP(hipStreamEndCapture(cs, &g));
    hipGraphExec_t ex = nullptr;
    const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    MJ_HIP(e);
    return ex;
}

static mj_pairs *run_join_graph(mj_ctx *ctx, const mj_strings *strings, const mj_params *params,
                                hipStream_t s, mj_stats *stats) {
    JoinGraph &gr = ctx->graph;
    Workspace &ws = ctx->ws;
    Released rel{ws};
    if (!graph_key_matches(gr, strings, params)) {
        graph_drop(ctx);
        gr.chars = strings->chars;
        gr.offsets = strings->offsets;
        gr.n = strings->n;
        gr.sigma = strings->sigma;
        gr.packing = strings->packing;
        gr.params = *params;
        gr.d = view(strings, s, ctx->pinned, false);
        gr.pp = to_pp(params, gr.d.bits);
        gr.setup = capture(ctx, [&](hipStream_t cs) { prepare_launch(gr.d, gr.pp, ws, cs, ctx->pinned); });
    }
    MJ_HIP(hipEventRecord(ctx->ev[0], s));
    MJ_HIP(hipGraphLaunch(gr.setup, s));
    MJ_HIP(hipStreamSynchronize(s));  // the one read before the end
    DevStrings d = gr.d;  // the set-up graph's arrays; total comes with its read-back
    SetupInfo si;
    (void)prepare_finish(d, ctx->pinned, &si);
    if (!gr.main || si.halo != gr.si.halo || si.rec_bound != gr.si.rec_bound ||
        si.kmax != gr.si.kmax || d.total != gr.total || d.wide_count != gr.md.wide_count ||
        d.wide_pos != gr.md.wide_pos) {
        if (gr.main) (void)hipGraphExecDestroy(gr.main);
        gr.main = nullptr;
        StreamedPlan pl;
        if (!plan_streamed(ctx, params, d, gr.pp, si, pl)) return nullptr;
        gr.plan = pl;
        gr.si = si;
        gr.total = d.total;
        gr.md = d;
        gr.main = capture(ctx, [&](hipStream_t cs) {
            gr.dv = launch_streamed_main(ctx, gr.md, gr.pp, gr.plan, params, cs, nullptr, nullptr);
        });
    }
    MJ_HIP(hipEventRecord(ctx->ev[1], s));
    MJ_HIP(hipGraphLaunch(gr.main, s));
    MJ_HIP(hipEventRecord(ctx->ev[2], s));
    MJ_HIP(hipStreamSynchronize(s));  // the one read at the end
    mj_pairs *out = finish_streamed(ctx, gr.plan, gr.dv, gr.md, gr.pp, s, stats);
    if (!out) {
        graph_drop(ctx);  // recaptured with the new capacities next time
        return nullptr;
    }
    if (stats) {
        MJ_HIP(hipStreamSynchronize(s));
        float a = 0.f, b = 0.f;
        MJ_HIP(hipEventElapsedTime(&a, ctx->ev[0], ctx->ev[1]));
        MJ_HIP(hipEventElapsedTime(&b, ctx->ev[1], ctx->ev[2]));
        stats->stage_ms[0] = a;
        stats->stage_ms[7] = b;
        stats->streamed = 2;
    }
    return out;
}

extern "C" mj_status mj_join(mj_ctx *ctx, const mj_strings *strings, const mj_params *params,
                             void *stream, mj_pairs **out, mj_stats *stats) {
    if (!ctx || !out) return fail(MJ_EINVAL, "ctx/out is NULL");
    MJ_API_BEGIN
    check_strings(strings);
    check_params(params, strings->sigma, true);
    MJ_HIP(hipSetDevice(ctx->device));
    AllocScope as(ctx->ws.alloc);
    hipStream_t s = (hipStream_t)stream;
    const bool batched = params->verifier == MJ_VERIFY_BATCHED;
    if (batched && ctx->streaming && !ctx->no_tuning && hints_match(ctx->stream, strings, params)) {
        mj_pairs *r = ctx->streaming == 2 ? run_join_graph(ctx, strings, params, s, stats)
                                          : run_join_streamed(ctx, strings, params, s, stats);
        if (r) {
            ctx->streamed_joins++;
            *out = r;
            return MJ_OK;
        }
        ctx->stream_fallbacks++;
    }
    *out = run_join(ctx, strings, params, s, 2, stats);
    if (batched && !ctx->no_tuning && stats) {
        // what the streamed join of the next call with these parameters needs
        StreamHints &h = ctx->stream;
        h.valid = true;
        h.q = params->q; h.t_div = params->t_div; h.t_fixed = params->t_fixed; h.reps = params->reps;
        h.seed = params->seed; h.k = params->k; h.sigma = strings->sigma; h.packing = strings->packing;
        h.verify_lanes = params->verify_lanes;
        h.cand_per_record = (double)ctx->last_c0 / (double)std::max<int64_t>(ctx->last_rcap, 1);
        h.rec_per_bound = (double)ctx->last_R / (double)std::max<int64_t>(ctx->last_rcap, 1);
        h.mem_per_bound = (double)ctx->last_M / (double)std::max<int64_t>(ctx->last_rcap, 1);
        h.emit = emit_hints((uint64_t)stats->pair_tests, ctx->last_small_tests, ctx->last_units,
                            stats->members, strings->n, ctx->tile_min);
        h.verify_g = ctx->tune.last_g;
        h.verify_blocks = ctx->tune.last_blocks;
    }
    return MJ_OK;
    MJ_API_END
}

extern "C" mj_status mj_candidates(mj_ctx *ctx, const mj_strings *strings, const mj_params *params,
                                   void *stream, mj_pairs **out, mj_stats *stats) {
    if (!ctx || !out) return fail(MJ_EINVAL, "ctx/out is NULL");
    MJ_API_BEGIN
    check_strings(strings);
    check_params(params, strings->sigma, true);
    MJ_HIP(hipSetDevice(ctx->device));
    AllocScope as(ctx->ws.alloc);
    *out = run_join(ctx, strings, params, (hipStream_t)stream, 1, stats);
    return MJ_OK;
    MJ_API_END
}

extern "C" mj_status mj_partition(mj_ctx *ctx, const mj_strings *strings, const mj_params *params,
                                  void *stream, mj_records **out) {
    if (!ctx || !out) return fail(MJ_EINVAL, "ctx/out is NULL");
    MJ_API_BEGIN
    check_strings(strings);
    check_params(params, strings->sigma, true);
    MJ_HIP(hipSetDevice(ctx->device));
    AllocScope as(ctx->ws.alloc);
    hipStream_t s = (hipStream_t)stream;
    Workspace &ws = ctx->ws;
    Released rel{ws};
    DevStrings d = view(strings, s, ctx->pinned);
    PartitionParams pp = to_pp(params, d.bits);
    int32_t halo = prepare_strings(d, pp, ws, s, ctx->pinned);
    pack_planes(d, verify_planes(d.bits), ws, s);  // checks the symbol codes
    mj_records *r = new mj_records();
    r->rb.with_len = true;
    r->rb.alloc = ctx->ws.alloc;
    try {
        partition_records(d, pp, halo, r->rb, ws, s, ctx->pinned);
        MJ_HIP(hipStreamSynchronize(s));
    } catch (...) {
        r->rb.release();
        delete r;
        throw;
    }
    *out = r;
    return MJ_OK;
    MJ_API_END
}

extern "C" mj_status mj_verify(mj_ctx *ctx, const mj_strings *strings, const mj_params *params,
                               const uint64_t *pairs, int64_t n, uint8_t *flags, void *stream) {
    if (!ctx) return fail(MJ_EINVAL, "ctx is NULL");
    if (n < 0 || (n > 0 && (!pairs || !flags))) return fail(MJ_EINVAL, "bad pair list");
    MJ_API_BEGIN
    check_strings(strings);
    check_params(params, strings->sigma, true);
    MJ_HIP(hipSetDevice(ctx->device));
    AllocScope as(ctx->ws.alloc);
    hipStream_t s = (hipStream_t)stream;
    Workspace &ws = ctx->ws;
    Released rel{ws};
    DevStrings d = view(strings, s, ctx->pinned);
    PartitionParams pp = to_pp(params, d.bits);
    (void)prepare_strings(d, pp, ws, s, ctx->pinned);
    pack_planes(d, verify_planes(d.bits), ws, s);
    check_symbols(d, s, ctx->pinned);
    if (params->verifier == MJ_VERIFY_BATCHED) {
        verify_pairs_batched(pairs, n, d, d, 0, flags, ws, s, ctx->pinned, nullptr, &ctx->tune, -1,
                             nullptr, params->verify_lanes);
    } else {
        verify_pairs(pairs, n, d, d, 0, flags, ws, s, ctx->pinned);
        check_flags(flags, n, ws, s, ctx->pinned);
    }
    MJ_HIP(hipStreamSynchronize(s));
    return MJ_OK;
    MJ_API_END
}

// ---------------------------------------------------------------- search
extern "C" mj_status mj_index_build(mj_ctx *ctx, const mj_strings *strings, const mj_params *params,
                                    void *stream, mj_index **out) {
    if (!ctx || !out) return fail(MJ_EINVAL, "ctx/out is NULL");
    MJ_API_BEGIN
    check_strings(strings);
    check_params(params, strings->sigma, true);
    MJ_HIP(hipSetDevice(ctx->device));
    AllocScope as(ctx->ws.alloc);
    hipStream_t s = (hipStream_t)stream;
    Workspace &ws = ctx->ws;
    Released rel{ws};
    DevStrings d = view(strings, s, ctx->pinned);
    PartitionParams pp = to_pp(params, d.bits);
    pp.k_per_string = nullptr;  // not kept: the index stores per-string K below
    mj_index *ix = new mj_index();
    ix->alloc = ctx->ws.alloc;
    ix->rec.alloc = ctx->ws.alloc;
    try {
        ix->device = ctx->device;
        ix->n = d.n;
        ix->sigma = d.sigma;
        ix->bits = d.bits;
        ix->total = d.total;
        ix->np = verify_planes(d.bits);
        ix->offsets = (int64_t *)dev_alloc(((size_t)d.n + 1) * 8);
        ix->len = (int32_t *)dev_alloc(((size_t)d.n + 1) * 4);
        ix->kk = (int32_t *)dev_alloc(((size_t)d.n + 1) * 4);
        MJ_HIP(hipMemcpyAsync(ix->offsets, d.offsets, ((size_t)d.n + 1) * 8, hipMemcpyDeviceToDevice, s));
        // the symbols are read from the caller's buffer during the build only: the index
        // keeps the verifier's bit planes, not the input
        DevStrings di = d;
        di.offsets = ix->offsets;
        PartitionParams pk = to_pp(params, d.bits);
        int32_t halo = prepare_strings(di, pk, ws, s, ctx->pinned);
        if (d.n) {
            MJ_HIP(hipMemcpyAsync(ix->len, di.len, (size_t)d.n * 4, hipMemcpyDeviceToDevice, s));
            MJ_HIP(hipMemcpyAsync(ix->kk, di.kk, (size_t)d.n * 4, hipMemcpyDeviceToDevice, s));
        }
        ix->plane_words = plane_words_for(di.total);
        ix->planes = (uint32_t *)dev_alloc((size_t)ix->np * ix->plane_words * 4);
        pack_planes(di, ix->np, ws, s, ix->planes);
        sorted_records(di, pk, halo, ix->rec, ws, s, ctx->pinned);
        if (pp.pi_table) {
            // searches partition their queries with this table long after the caller's
            // copy may be gone: the index keeps its own
            const size_t tb = (size_t)8 << (pp.q * d.bits);
            ix->pi_table = (uint64_t *)dev_alloc(tb);
            MJ_HIP(hipMemcpyAsync(ix->pi_table, pp.pi_table, tb, hipMemcpyDeviceToDevice, s));
            pp.pi_table = ix->pi_table;
        }
        MJ_HIP(hipStreamSynchronize(s));
        ix->pp = pp;
    } catch (...) {
        mj_index_free(ix);
        throw;
    }
    *out = ix;
    return MJ_OK;
    MJ_API_END
}

extern "C" void mj_index_free(mj_index *ix) {
    if (!ix) return;
    (void)hipSetDevice(ix->device);
    dev_free(ix->offsets, ix->alloc);
    dev_free(ix->len, ix->alloc);
    dev_free(ix->kk, ix->alloc);
    dev_free(ix->planes, ix->alloc);
    dev_free(ix->pi_table, ix->alloc);
    ix->rec.release();
    delete ix;
}

extern "C" int64_t mj_index_records(const mj_index *ix) { return ix ? ix->rec.count : 0; }

extern "C" int64_t mj_index_bytes(const mj_index *ix) {
    if (!ix) return 0;
    int64_t b = ((int64_t)ix->n + 1) * (8 + 4 + 4);  // offsets, lengths, thresholds
    b += (int64_t)ix->np * ix->plane_words * 4;
    b += ix->rec.cap * (8 + 8 + (ix->rec.with_len ? 4 : 0));
    if (ix->pi_table) b += (int64_t)8 << (ix->pp.q * ix->bits);
    return b;
}

extern "C" mj_status mj_search(mj_ctx *ctx, const mj_index *ix, const mj_strings *queries,
                               const mj_params *qparams, void *stream, mj_pairs **out,
                               mj_stats *stats) {
    if (!ctx || !ix || !out) return fail(MJ_EINVAL, "ctx/index/out is NULL");
    MJ_API_BEGIN
    check_strings(queries);
    if (!qparams) throw Error(MJ_EINVAL, "qparams is NULL");
    if (queries->sigma > ix->sigma || queries->sigma < 2)
        throw Error(MJ_EINVAL, "query alphabet must not exceed the index alphabet");
    if (queries->packing == MJ_PACK_2BIT && ix->bits > 2)
        throw Error(MJ_EINVAL, "2-bit packed queries need an index over at most 4 symbols");
    if (qparams->k < -1 || (qparams->k == -1 && !qparams->k_per_string))
        throw Error(MJ_EINVAL, "bad query threshold");
    if (qparams->k > 2047) throw Error(MJ_ECAPACITY, "threshold K exceeds the verifier's band limit (K <= 2047)");
    check_verifier(qparams);
    MJ_HIP(hipSetDevice(ctx->device));
    AllocScope as(ctx->ws.alloc);
    hipStream_t s = (hipStream_t)stream;
    Workspace &ws = ctx->ws;
    Released rel{ws};
    StageTimer tm(ctx, s);
    if (stats) memset(stats, 0, sizeof(*stats));
    DevStrings qd = view(queries, s, ctx->pinned, false);
    qd.sigma = ix->sigma;
    qd.bits = ix->bits;
    PartitionParams qp = ix->pp;  // q, seed, T rule, reps of the index
    qp.k = qparams->k;
    qp.k_per_string = qparams->k_per_string;
    int32_t halo = prepare_strings(qd, qp, ws, s, ctx->pinned);
    pack_planes(qd, ix->np, ws, s);
    tm.mark();  // 0 setup
    RecBuf rb;
    rb.ws = &ws;
    partition_records(qd, qp, halo, rb, ws, s, ctx->pinned, &ctx->kt);
    tm.mark();  // 1 partition
    if (rb.count > 1) {
        sort_records(rb.key, rb.val, rb.count, ws, s, ctx->pinned);
    }
    tm.mark();  // 2 sort
    DevStrings id;  // the index keeps no symbols: planes, lengths and thresholds only
    id.chars = nullptr;
    id.offsets = ix->offsets;
    id.n = ix->n;
    id.sigma = ix->sigma;
    id.bits = ix->bits;
    id.total = ix->total;
    id.len = ix->len;
    id.kk = ix->kk;
    id.planes = ix->planes;
    id.plane_words = ix->plane_words;
    uint64_t tests = 0;
    int64_t need = probe_candidates(rb.key, rb.val, rb.count, ix->rec.key, ix->rec.val, ix->rec.count,
                                    qd, id, nullptr, -1, &tests, ws, s, ctx->pinned);
    (void)need;
    if (tests > (uint64_t)0x7FFFFFFF)
        throw Error(MJ_ECAPACITY, "record-pair tests exceed 2^31");
    uint64_t *cand = ws.get_n<uint64_t>(tests + 1);
    int64_t c0 = tests ? probe_candidates(rb.key, rb.val, rb.count, ix->rec.key, ix->rec.val,
                                          ix->rec.count, qd, id, cand, (int64_t)tests, &tests, ws, s,
                                          ctx->pinned)
                       : 0;
    tm.mark();  // 3 probe + filter
    uint64_t *uniq = nullptr;
    int64_t C = dedup_pairs(cand, c0, qd.n, ix->n, ws, s, ctx->pinned, &uniq, true);
    tm.mark();  // 4 dedup
    uint8_t *flags = ws.get_n<uint8_t>(C + 1);
    run_verify(ctx, uniq, C, qd, id, 1, qparams->k, qparams, flags, s, stats, cells_slot(ctx));
    tm.mark();  // 5 verify
    mj_pairs *res = compact_pairs(uniq, flags, C, ws, s, ctx->pinned);  // synchronises when C > 0
    const int64_t cells = take_cells(ctx, res);
    tm.mark();  // 6 output
    if (stats) {
        stats->records = rb.count;
        stats->pair_tests = (int64_t)tests;
        stats->candidates = C;
        stats->output = res->n;
        stats->band_cells = cells;
        stats->positions = qd.total * qp.reps;
    }
    tm.fill(stats);
    *out = res;
    return MJ_OK;
    MJ_API_END
}

// ---------------------------------------------------------------- results
extern "C" int64_t mj_pairs_count(const mj_pairs *p) { return p ? p->n : 0; }
extern "C" const uint64_t *mj_pairs_device(const mj_pairs *p) { return p ? p->d : nullptr; }

extern "C" mj_status mj_pairs_copy_to_host(const mj_pairs *p, uint64_t *dst, int64_t cap) {
    if (!p) return fail(MJ_EINVAL, "pairs is NULL");
    if (cap < p->n || (p->n > 0 && !dst)) return fail(MJ_EINVAL, "destination too small");
    MJ_API_BEGIN
    if (p->n) {
        MJ_HIP(hipMemcpyAsync(dst, p->d, (size_t)p->n * 8, hipMemcpyDeviceToHost, p->stream));
        MJ_HIP(hipStreamSynchronize(p->stream));
    }
    return MJ_OK;
    MJ_API_END
}

extern "C" void mj_pairs_free(mj_pairs *p) {
    if (!p) return;
    result_free(p->d, p->alloc, p->stream);
    delete p;
}

extern "C" int64_t mj_records_count(const mj_records *r) { return r ? r->rb.count : 0; }

__global__ void k_split_records(const uint64_t *val, int64_t n, int32_t *sid, int32_t *pos) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) {
        sid[i] = (int32_t)(val[i] >> 32);
        pos[i] = (int32_t)(uint32_t)val[i];
    }
}

extern "C" mj_status mj_records_copy_to_host(const mj_records *r, uint64_t *key, int32_t *sid,
                                             int32_t *pos, int32_t *len, int64_t cap) {
    if (!r) return fail(MJ_EINVAL, "records is NULL");
    int64_t n = r->rb.count;
    if (cap < n) return fail(MJ_EINVAL, "destination too small");
    MJ_API_BEGIN
    if (n == 0) return MJ_OK;
    if (key) MJ_HIP(hipMemcpy(key, r->rb.key, (size_t)n * 8, hipMemcpyDeviceToHost));
    if (len && r->rb.len) MJ_HIP(hipMemcpy(len, r->rb.len, (size_t)n * 4, hipMemcpyDeviceToHost));
    if (sid || pos) {
        AllocScope as(r->rb.alloc);
        int32_t *ds = (int32_t *)dev_alloc((size_t)n * 4), *dp = (int32_t *)dev_alloc((size_t)n * 4);
        unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, 16384);
        hipLaunchKernelGGL(k_split_records, dim3(g), dim3(256), 0, 0, r->rb.val, n, ds, dp);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess && sid) e = hipMemcpy(sid, ds, (size_t)n * 4, hipMemcpyDeviceToHost);
        if (e == hipSuccess && pos) e = hipMemcpy(pos, dp, (size_t)n * 4, hipMemcpyDeviceToHost);
        dev_free(ds);
        dev_free(dp);
        MJ_HIP(e);
    }
    return MJ_OK;
    MJ_API_END
}

extern "C" void mj_records_free(mj_records *r) {
    if (!r) return;
    r->rb.release();
    delete r;
}
