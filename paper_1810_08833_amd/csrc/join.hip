// Join stage: groups of records with equal bucket key (the hash table D of Alg. 3),
// candidate emission through the length and position filters (Alg. 3; Sec. 3),
// candidate dedup, and the probe of a resident index for search.
#include <string.h>

#include <algorithm>
#include <type_traits>
#include <cmath>

#include "mj_common.h"

namespace mj {

static unsigned grid_for(int64_t n, int block, unsigned cap = 65535u) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    return (unsigned)std::min<int64_t>(g, cap);
}

static int ceil_log2(uint64_t v) {
    int b = 0;
    while (b < 63 && (1ull << b) < v) b++;
    return b;
}

// ---------------------------------------------------------------- groups
// A group is a maximal run of equal keys in the sorted records; only runs of length
// >= 2 can produce pairs.  start flag: first of a run of >= 2; end flag: last of one.
// R_dev (nullable): the record count on the device; flags up to the capacity R are
// written (0 past the count), so that compactions over the capacity see only records.
__global__ void k_group_flags(const uint64_t *key, int64_t R, uint8_t *fs, uint8_t *fe,
                              const int64_t *R_dev) {
    const int64_t cap = R;
    if (R_dev) R = min(R, *R_dev);
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < cap; i += stride) {
        bool s1 = false, e1 = false;
        if (i < R) {
            uint64_t k = key[i];
            bool same_prev = i > 0 && key[i - 1] == k;
            bool same_next = i + 1 < R && key[i + 1] == k;
            s1 = !same_prev && same_next;
            e1 = same_prev && !same_next;
        }
        fs[i] = s1 ? 1 : 0;
        fe[i] = e1 ? 1 : 0;
    }
}

// Per group: its pair tests (all), the same for the groups below EMIT_TILE records and 0
// for the others (small), and the tile pairs I <= J of the groups of EMIT_TILE records or
// more, 0 for the others (units; nt tiles of EMIT_TILE records give nt (nt + 1) / 2).
struct GroupCounts {
    uint64_t all, small, units;
    __device__ GroupCounts &operator+=(const GroupCounts &o) {
        all += o.all;
        small += o.small;
        units += o.units;
        return *this;
    }
};

__device__ __forceinline__ GroupCounts group_counts(const int64_t *gs, const int64_t *ge, int64_t g) {
    const uint64_t sz = (uint64_t)(ge[g] - gs[g] + 1);
    const uint64_t nt = (sz + EMIT_TILE - 1) / EMIT_TILE;
    const bool big = sz >= (uint64_t)EMIT_TILE;
    GroupCounts c;
    c.all = sz * (sz - 1) / 2;
    c.small = big ? 0 : c.all;
    c.units = big ? nt * (nt + 1) / 2 : 0;
    return c;
}

__device__ __forceinline__ uint64_t shfl_up_u64(uint64_t v, int d) {
    const uint32_t lo = (uint32_t)__shfl_up((int)(uint32_t)v, d, 64);
    const uint32_t hi = (uint32_t)__shfl_up((int)(uint32_t)(v >> 32), d, 64);
    return ((uint64_t)hi << 32) | lo;
}

// Exclusive scan of one GroupCounts per thread over the block (GS_THREADS threads); the
// block total goes to *total.
constexpr int GS_THREADS = 256, GS_ITEMS = 8, GS_TILE = GS_THREADS * GS_ITEMS;
__device__ GroupCounts block_scan_counts(GroupCounts v, GroupCounts *smem /* [4] */,
                                         GroupCounts *total) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    GroupCounts inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        GroupCounts o;
        o.all = shfl_up_u64(inc.all, d);
        o.small = shfl_up_u64(inc.small, d);
        o.units = shfl_up_u64(inc.units, d);
        if (lane >= d) inc += o;
    }
    if (lane == 63) smem[wv] = inc;
    __syncthreads();
    GroupCounts pre = {0, 0, 0}, tot = {0, 0, 0};
    for (int w = 0; w < GS_THREADS / 64; w++) {
        if (w < wv) pre += smem[w];
        tot += smem[w];
    }
    __syncthreads();
    *total = tot;
    pre += inc;
    pre.all -= v.all;
    pre.small -= v.small;
    pre.units -= v.units;
    return pre;
}

// The three exclusive prefixes over the groups, with the group counts c1 (starts) and c2
// (ends) on the device, in three launches: per-tile sums of GS_TILE groups, a scan of
// those (one workgroup; totals to slot[2..4] and to the prefixes' entry G), and the
// prefixes (each group's counts computed again).  slot[0] = c1 | c2 << 32, slot[1] =
// G = min(c1, c2).
__global__ __launch_bounds__(GS_THREADS) void k_gscan_reduce(const int64_t *__restrict__ gs,
                                                            const int64_t *__restrict__ ge,
                                                            const uint32_t *c1, const uint32_t *c2,
                                                            GroupCounts *part, uint64_t *slot) {
    __shared__ GroupCounts smem[GS_THREADS / 64];
    const int64_t G = min(*c1, *c2);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        slot[0] = (uint64_t)*c1 | ((uint64_t)*c2 << 32);
        slot[1] = (uint64_t)G;
    }
    const int64_t base = (int64_t)blockIdx.x * GS_TILE;
    if (base >= G) return;  // block-uniform
    GroupCounts v = {0, 0, 0};
    for (int k = 0; k < GS_ITEMS; k++) {
        const int64_t g = base + (int64_t)k * GS_THREADS + threadIdx.x;
        if (g < G) v += group_counts(gs, ge, g);
    }
    GroupCounts tot;
    block_scan_counts(v, smem, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(GS_THREADS) void k_gscan_top(GroupCounts *part, const uint32_t *c1,
                                                         const uint32_t *c2, uint64_t *slot,
                                                         uint64_t *tstart, uint64_t *tsmall,
                                                         uint64_t *ustart) {
    __shared__ GroupCounts smem[GS_THREADS / 64];
    const int64_t G = min(*c1, *c2);
    const int64_t nb = (G + GS_TILE - 1) / GS_TILE;
    const int64_t per = (nb + GS_THREADS - 1) / GS_THREADS;  // consecutive tiles per thread
    const int64_t b0 = (int64_t)threadIdx.x * per, b1 = min(nb, b0 + per);
    GroupCounts v = {0, 0, 0};
    for (int64_t b = b0; b < b1; b++) v += part[b];
    GroupCounts tot;
    GroupCounts run = block_scan_counts(v, smem, &tot);
    for (int64_t b = b0; b < b1; b++) {
        const GroupCounts x = part[b];
        part[b] = run;
        run += x;
    }
    if (threadIdx.x == 0) {
        slot[2] = tot.all;
        slot[3] = tot.small;
        slot[4] = tot.units;
        tstart[G] = tot.all;
        tsmall[G] = tot.small;
        ustart[G] = tot.units;
    }
}

__global__ __launch_bounds__(GS_THREADS) void k_gscan_apply(const int64_t *__restrict__ gs,
                                                           const int64_t *__restrict__ ge,
                                                           const uint32_t *c1, const uint32_t *c2,
                                                           const GroupCounts *__restrict__ part,
                                                           uint64_t *tstart, uint64_t *tsmall,
                                                           uint64_t *ustart) {
    __shared__ GroupCounts smem[GS_THREADS / 64];
    __shared__ uint64_t zs[GS_TILE];  // group sizes of the tile, read coalesced
    const int64_t G = min(*c1, *c2);
    const int64_t base = (int64_t)blockIdx.x * GS_TILE;
    if (base >= G) return;  // block-uniform
    for (int k = 0; k < GS_ITEMS; k++) {
        const int i = k * GS_THREADS + threadIdx.x;
        zs[i] = base + i < G ? (uint64_t)(ge[base + i] - gs[base + i] + 1) : 0;
    }
    __syncthreads();
    // the thread's GS_ITEMS consecutive groups
    const int i0 = threadIdx.x * GS_ITEMS;
    GroupCounts c[GS_ITEMS], v = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < GS_ITEMS; k++) {
        const uint64_t sz = zs[i0 + k];
        const uint64_t nt = (sz + EMIT_TILE - 1) / EMIT_TILE;
        const bool big = sz >= (uint64_t)EMIT_TILE;
        c[k].all = sz ? sz * (sz - 1) / 2 : 0;
        c[k].small = big ? 0 : c[k].all;
        c[k].units = big ? nt * (nt + 1) / 2 : 0;
        v += c[k];
    }
    GroupCounts tot;
    GroupCounts run = block_scan_counts(v, smem, &tot);
    run += part[blockIdx.x];
    GroupCounts pre[GS_ITEMS];
#pragma unroll
    for (int k = 0; k < GS_ITEMS; k++) {
        pre[k] = run;
        run += c[k];
    }
    // each prefix through the LDS tile, then stored coalesced
    uint64_t *const dst[3] = {tstart, tsmall, ustart};
#pragma unroll
    for (int f = 0; f < 3; f++) {
        __syncthreads();  // the tile's previous contents are read
#pragma unroll
        for (int k = 0; k < GS_ITEMS; k++)
            zs[i0 + k] = f == 0 ? pre[k].all : f == 1 ? pre[k].small : pre[k].units;
        __syncthreads();
        for (int k = 0; k < GS_ITEMS; k++) {
            const int i = k * GS_THREADS + threadIdx.x;
            if (base + i < G) dst[f][base + i] = zs[i];
        }
    }
}

// Group boundaries and the three prefixes over the groups, with the group counts on the
// device: the arrays are sized by the bound R / 2 (a group holds >= 2 records) and the
// totals land in slot[2..4].
static GroupInfo group_tests(const uint64_t *key, int64_t R, const int64_t *R_dev, Workspace &ws,
                             hipStream_t s) {
    GroupInfo gi;
    uint8_t *fs = ws.get_n<uint8_t>(R);
    uint8_t *fe = ws.get_n<uint8_t>(R);
    hipLaunchKernelGGL(k_group_flags, dim3(grid_for(R, 256, 16384)), dim3(256), 0, s, key, R, fs, fe,
                       R_dev);
    MJ_LAUNCH_CHECK();
    int64_t *gs = ws.get_n<int64_t>(R / 2 + 2);
    int64_t *ge = ws.get_n<int64_t>(R / 2 + 2);
    const uint32_t *c1 = compact_flags_async(fs, R, gs, ws, s);
    const uint32_t *c2 = compact_flags_async(fe, R, ge, ws, s);
    const int64_t gmax = R / 2;
    const int64_t nb = std::max<int64_t>(1, (gmax + GS_TILE - 1) / GS_TILE);
    GroupCounts *part = reinterpret_cast<GroupCounts *>(ws.get_n<uint64_t>(3 * (nb + 1)));
    gi.tstart = ws.get_n<uint64_t>(gmax + 1);
    gi.tsmall = ws.get_n<uint64_t>(gmax + 1);
    gi.ustart = ws.get_n<uint64_t>(gmax + 1);
    uint64_t *slot = ws.get_n<uint64_t>(5);
    hipLaunchKernelGGL(k_gscan_reduce, dim3((unsigned)nb), dim3(GS_THREADS), 0, s, gs, ge, c1, c2, part,
                       slot);
    MJ_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_gscan_top, dim3(1), dim3(GS_THREADS), 0, s, part, c1, c2, slot, gi.tstart,
                       gi.tsmall, gi.ustart);
    MJ_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_gscan_apply, dim3((unsigned)nb), dim3(GS_THREADS), 0, s, gs, ge, c1, c2,
                       (const GroupCounts *)part, gi.tstart, gi.tsmall, gi.ustart);
    MJ_LAUNCH_CHECK();
    gi.gstart = gs;
    gi.gend = ge;
    gi.slot = slot;
    gi.gmax = gmax;
    return gi;
}

GroupInfo find_groups(const uint64_t *key, int64_t R, Workspace &ws, hipStream_t s,
                      uint64_t *host_scratch) {
    if (R < 2) return GroupInfo();
    GroupInfo gi = group_tests(key, R, nullptr, ws, s);
    // one read brings back both group counts and the totals
    MJ_HIP(hipMemcpyAsync(host_scratch, gi.slot, 40, hipMemcpyDeviceToHost, s));
    MJ_HIP(hipStreamSynchronize(s));
    uint64_t hs[5];
    memcpy(hs, host_scratch, 40);
    const int64_t G1 = (int64_t)(hs[0] & 0xFFFFFFFFu), G2 = (int64_t)(hs[0] >> 32);
    if (G1 != G2) throw Error(MJ_EDEVICE, "group boundary mismatch");
    gi.groups = G1;
    gi.tests = G1 > 0 ? hs[2] : 0;
    gi.small_tests = G1 > 0 ? hs[3] : 0;
    gi.units = G1 > 0 ? hs[4] : 0;
    gi.slot = nullptr;
    return gi;
}

GroupInfo find_groups_streamed(const uint64_t *key, int64_t R_cap, const int64_t *R_dev,
                               Workspace &ws, hipStream_t s) {
    GroupInfo gi = group_tests(key, std::max<int64_t>(R_cap, 2), R_dev, ws, s);
    gi.groups = -1;  // on the device, in slot
    return gi;
}

// ---------------------------------------------------------------- candidate emission
// Pair tests are numbered consecutively across groups; each thread takes a run of
// consecutive tests (EMIT_CHUNK, or a multiple of it in k_emit), so a huge group is
// spread over many threads.  Inside a group of
// size z, test u is the pair (a, b), a < b, with u = b(b-1)/2 + a.  In a join emitted in
// one pass, the groups of EMIT_TILE records or more have no tests in this numbering (their
// prefix does not grow): k_emit_big takes them by tile pairs.
// Filter (Alg. 3): |m_i - m_j| <= K and |pos_i - pos_j| + |(m_i-pos_i) - (m_j-pos_j)| <= K,
// evaluated as max(|m_i - m_j|, |(2pos_i - m_i) - (2pos_j - m_j)|) <= K (the same test,
// since |u| + |v| = max(|u + v|, |u - v|)).
constexpr int EMIT_CHUNK = 16;
constexpr int EMIT_BATCH = 4;  // tests whose loads k_emit issues together (divides EMIT_CHUNK)

__device__ __forceinline__ int64_t iabs64(int64_t v) { return v < 0 ? -v : v; }

__device__ __forceinline__ bool pass_filter(int64_t mi, int64_t pi, int64_t mj, int64_t pj,
                                            int64_t K) {
    int64_t d1 = iabs64(mi - mj);
    int64_t d2 = iabs64((2 * pi - mi) - (2 * pj - mj));
    return (d1 > d2 ? d1 : d2) <= K;
}

// The same test in 32-bit arithmetic, for inputs of fewer than 2^29 symbols: then
// m, pos < 2^29, 2 pos - m lies in (-2^29, 2^30), and both differences fit an int32.
__device__ __forceinline__ bool pass_filter32(int32_t mi, int32_t pi, int32_t mj, int32_t pj,
                                              uint32_t K) {
    const int32_t d1 = abs(mi - mj);
    const int32_t d2 = abs((2 * pi - mi) - (2 * pj - mj));
    return (uint32_t)max(d1, d2) <= K;
}

// Passing tests of one block's sweep are staged in LDS and written out with one
// device-wide atomic per block and sweep: a single counter bumped by every wave of all
// XCDs serialises (device-scope atomics are not served by an XCD's own L2).
constexpr int EMIT_BLOCK = 256;
struct EmitStage {
    uint64_t buf[EMIT_BLOCK * EMIT_CHUNK];
    uint32_t n;
    unsigned long long base;
};

__device__ __forceinline__ void stage(bool pass, uint64_t v, EmitStage &st) {
    const uint64_t mask = __ballot(pass);
    if (mask == 0) return;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((unsigned long long)mask) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(&st.n, (uint32_t)__popcll(mask));
    base = __shfl(base, leader, 64);
    if (pass) st.buf[base + __popcll(mask & ((1ull << lane) - 1))] = v;
}

// Block-uniform: every thread of the block calls it after the same sweep.
__device__ __forceinline__ void flush(EmitStage &st, unsigned long long *counter, uint64_t *out,
                                      int64_t cap) {
    __syncthreads();
    const uint32_t n = st.n;
    if (threadIdx.x == 0 && n) st.base = atomicAdd(counter, (unsigned long long)n);
    __syncthreads();
    if (n) {
        const unsigned long long base = st.base;
        if (threadIdx.x == 0) st.n = 0;  // every thread has read n before the barrier above
        for (uint32_t i = threadIdx.x; i < n; i += EMIT_BLOCK)
            if ((int64_t)(base + i) < cap) out[base + i] = st.buf[i];
        __syncthreads();  // buf and n are free for the next sweep
    }
}

// lk[s] = m << 32 | K of string s: one gather where a record's string is looked up
__global__ void k_string_meta(const int32_t *__restrict__ len, const int32_t *__restrict__ kk,
                              int32_t n, uint64_t *__restrict__ lk) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        lk[i] = ((uint64_t)(uint32_t)len[i] << 32) | (uint32_t)kk[i];
}

// meta[i] = the (m, K) word of the string owning sorted record i, so that a pair test
// reads four record-aligned words (two payloads, two metas) with no dependent gathers.
__global__ void k_record_meta(const uint64_t *__restrict__ val, int64_t R,
                              const uint64_t *__restrict__ lk, uint64_t *__restrict__ meta,
                              const int64_t *__restrict__ R_dev) {
    if (R_dev) R = min(R, *R_dev);
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < R; i += stride) meta[i] = lk[(int32_t)(val[i] >> 32)];
}

// Largest g in [lo, hi) with us[g] <= w, given us[lo] <= w (us non-decreasing): a 64-way
// search by the whole wave (one probe of 64 entries per level; every lane of the wave
// takes part).  lo, hi and w are wave-uniform, and so is the result.
__device__ __forceinline__ int64_t last_le_wave(const uint64_t *__restrict__ us, int64_t lo,
                                                int64_t hi, uint64_t w) {
    const int lane = threadIdx.x & 63;
    while (hi - lo > 1) {
        const int64_t step = (hi - lo + 63) / 64;
        const int64_t idx = lo + (int64_t)lane * step;
        const bool le = idx < hi && us[idx] <= w;
        const int c = __popcll(__ballot(le));  // a prefix of the lanes: lane 0 always
        const int64_t nlo = lo + (int64_t)(c - 1) * step;
        hi = min(hi, nlo + step);
        lo = nlo;
    }
    return lo;
}

// Largest g in [lo, hi) with a[g] <= w, given a[lo] <= w (a non-decreasing), for
// wave-uniform arguments: a binary search whose loads are the same for every lane.
__device__ __forceinline__ int64_t last_le_uniform(const uint64_t *__restrict__ a, int64_t lo,
                                                   int64_t hi, uint64_t w) {
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (a[mid] <= w) lo = mid; else hi = mid;
    }
    return lo;
}

// The same, galloping up from lo (for a w close above a[lo]).
__device__ __forceinline__ int64_t last_le_gallop(const uint64_t *__restrict__ a, int64_t lo,
                                                  int64_t hi, uint64_t w) {
    int64_t step = 1;
    while (lo + step < hi && a[lo + step] <= w) {
        lo += step;
        step <<= 1;
    }
    return last_le_uniform(a, lo, min(hi, lo + step), w);
}

// LAZY: no meta array; a record's (m, K) word is gathered by its string id at each use
// (fewer pair tests than records, as on text and DNA), from lk if given, else from the
// length and K arrays.  SMALL: the input holds fewer than 2^29 symbols (32-bit filter).
template <bool LAZY, bool SMALL>
__global__ __launch_bounds__(EMIT_BLOCK) void k_emit(const uint64_t *__restrict__ val,
                                              const uint64_t *__restrict__ meta,
                                              const uint64_t *__restrict__ lk,
                                              const int32_t *__restrict__ len,
                                              const int32_t *__restrict__ kk,
                                              const int64_t *__restrict__ gs,
                                              const uint64_t *__restrict__ ts, int64_t G,
                                              uint64_t P, uint64_t *out, int64_t cap,
                                              unsigned long long *counter, int chunk,
                                              const uint64_t *__restrict__ slot, int pslot,
                                              uint64_t tb) {
    // group and test counts on the device (the streamed join): slot[1], and the tests of
    // all groups (pslot 2) or of the groups below EMIT_TILE records (pslot 3)
    if (slot) {
        G = (int64_t)slot[1];
        P = G > 0 ? slot[pslot] : 0;
    }
    // tests [tb, P): the whole range, or one pass of a join emitted in passes
    __shared__ EmitStage st;
    if (threadIdx.x == 0) st.n = 0;
    __syncthreads();
    const uint64_t nthreads = (uint64_t)gridDim.x * EMIT_BLOCK;
    for (uint64_t t0 = tb + ((uint64_t)blockIdx.x * EMIT_BLOCK + threadIdx.x) * chunk; ;
         t0 += nthreads * chunk) {
        // block-uniform loop exit (the flush has barriers)
        if (t0 - (uint64_t)threadIdx.x * chunk >= P) break;
        bool active = t0 < P;
        int64_t g = 0;
        uint64_t a = 0, b = 1;
        // The groups of the wave's first and last runs (lane 0's t0 and lane 63's, at most
        // P - 1), by one search with the same loads for every lane (a binary search, then a
        // gallop); each lane then searches that short range.  Searches of 64 far-apart
        // groups per wave missed the caches at their deeper levels.
        int64_t gA = 0, gB = G;
        const uint64_t tw0 = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)t0)) |
                             ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(t0 >> 32)) << 32);
        if (tw0 < P) {  // wave-uniform
            const uint64_t twl = min(P - 1, tw0 + (uint64_t)63 * chunk);
            gA = last_le_uniform(ts, 0, G, tw0);
            gB = last_le_gallop(ts, gA, G, twl) + 1;
        }
        if (active) {
            int64_t lo = gA, hi = gB;  // largest g with ts[g] <= t0
            while (hi - lo > 1) {
                int64_t mid = (lo + hi) >> 1;
                if (ts[mid] <= t0) lo = mid; else hi = mid;
            }
            g = lo;
            uint64_t u = t0 - ts[g];
            b = (uint64_t)((1.0 + sqrt(1.0 + 8.0 * (double)u)) * 0.5);
            while (b > 1 && b * (b - 1) / 2 > u) b--;
            while ((b + 1) * b / 2 <= u) b++;
            a = u - b * (b - 1) / 2;
        }
        // The run is taken EMIT_BATCH tests at a time: first the walk over the tests (the
        // records a and b of each; the group bounds, with the next group's preloaded),
        // then every load of the batch at once, then the filter and the stage.  A lane's
        // loads thus overlap instead of waiting one test at a time.
        int64_t s0 = 0, s0n = 0;
        uint64_t gend = 0, gendn = 0;
        if (active) {
            s0 = gs[g];
            gend = ts[g + 1];
            if (g + 1 < G) {
                s0n = gs[g + 1];
                gendn = ts[g + 2];
            }
        }
        auto meta_of = [&](int64_t i, uint64_t v) -> uint64_t {
            if constexpr (LAZY) {
                const int32_t sid = (int32_t)(v >> 32);
                if (lk) return lk[sid];
                return ((uint64_t)(uint32_t)len[sid] << 32) | (uint32_t)kk[sid];
            } else {
                return meta[i];
            }
        };
        for (int cb = 0; cb < chunk; cb += EMIT_BATCH) {
            int64_t ra[EMIT_BATCH], rb[EMIT_BATCH];
            bool lv[EMIT_BATCH];
#pragma unroll
            for (int k = 0; k < EMIT_BATCH; k++) {
                const uint64_t t = t0 + cb + k;
                lv[k] = active && t < P;
                ra[k] = s0 + (int64_t)a;
                rb[k] = s0 + (int64_t)b;
                if (lv[k]) {
                    // next test: (a+1, b); else (0, b+1); the group ends where the next
                    // group's tests start, and groups with no tests in this numbering are
                    // passed over
                    a++;
                    if (a == b) {
                        a = 0;
                        b++;
                    }
                    if (t + 1 == gend && g + 1 < G) {
                        g++;
                        s0 = s0n;
                        gend = gendn;
                        while (gend == t + 1 && g + 1 < G) {
                            g++;
                            s0 = gs[g];
                            gend = ts[g + 1];
                        }
                        if (g + 1 < G) {
                            s0n = gs[g + 1];
                            gendn = ts[g + 2];
                        }
                        a = 0;
                        b = 1;
                    }
                }
            }
            uint64_t va[EMIT_BATCH], vb[EMIT_BATCH], xa[EMIT_BATCH], xb[EMIT_BATCH];
#pragma unroll
            for (int k = 0; k < EMIT_BATCH; k++) {
                va[k] = lv[k] ? val[ra[k]] : 0ull;
                vb[k] = lv[k] ? val[rb[k]] : 0ull;
                if constexpr (!LAZY) {
                    xa[k] = lv[k] ? meta[ra[k]] : 0ull;
                    xb[k] = lv[k] ? meta[rb[k]] : 0ull;
                }
            }
            if constexpr (LAZY) {
#pragma unroll
                for (int k = 0; k < EMIT_BATCH; k++) {
                    xa[k] = lv[k] ? meta_of(ra[k], va[k]) : 0ull;
                    xb[k] = lv[k] ? meta_of(rb[k], vb[k]) : 0ull;
                }
            }
#pragma unroll
            for (int k = 0; k < EMIT_BATCH; k++) {
                bool pass = false;
                uint64_t pairkey = 0;
                const int32_t ia = (int32_t)(va[k] >> 32), ib = (int32_t)(vb[k] >> 32);
                if (lv[k] && ia != ib) {
                    if constexpr (SMALL) {
                        pass = pass_filter32((int32_t)(xa[k] >> 32), (int32_t)(uint32_t)va[k],
                                             (int32_t)(xb[k] >> 32), (int32_t)(uint32_t)vb[k],
                                             max((uint32_t)xa[k], (uint32_t)xb[k]));
                    } else {
                        const int64_t ma = (int64_t)(xa[k] >> 32), mb = (int64_t)(xb[k] >> 32);
                        const int64_t K = max((int64_t)(uint32_t)xa[k], (int64_t)(uint32_t)xb[k]);
                        pass = pass_filter(ma, (int64_t)(uint32_t)va[k], mb, (int64_t)(uint32_t)vb[k], K);
                    }
                    const uint64_t lo = (uint64_t)min(ia, ib), hi = (uint64_t)max(ia, ib);
                    pairkey = (lo << 32) | hi;
                }
                stage(pass, pairkey, st);
                // the stage holds EMIT_CHUNK tests per thread (chunk is a multiple of it)
                if (((cb + k) & (EMIT_CHUNK - 1)) == EMIT_CHUNK - 1) flush(st, counter, out, cap);
            }
        }
    }
}

// Pair tests of the groups of EMIT_TILE records or more, by tile pairs.  A group of z
// records is cut into nt = ceil(z / 64) tiles; tile pair u = J (J + 1) / 2 + I, I <= J,
// tests records a = 64 I + l against b = 64 J + j (a < b: l < j when I = J), the same
// pairs as the group's tests in k_emit, each once.  A wave takes a tile pair: lane l holds
// record a, tile J's records are staged in LDS and read by the whole wave at one address
// per column, so the inner loop reads no global memory.  Wave k takes the tile pairs
// [k per, (k + 1) per) in order (one group search, then a walk).  The kernel runs twice
// with the same grid: COUNT writes the number of each wave's passing pairs to wcnt[k];
// after an exclusive scan of those (wpre) WRITE stores the pairs at out[*wbase + wpre[k]
// ..), staged per wave in LDS: no shared counter (a device atomic on one address, taken
// by every wave, serialises).
constexpr int EB_WAVES = 4;   // waves per workgroup
constexpr int EB_BUF = 512;   // staged pairs per wave

__device__ __forceinline__ void wave_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The next group with tiles after g (the first g' > g with us[g'] <= w < us[g' + 1], where
// w = us[g + 1]): a forward scan by the whole wave, 64 entries per probe, the common case
// being a short gap of groups without tiles.
__device__ __forceinline__ int64_t next_group_of_unit(const uint64_t *__restrict__ us, int64_t g,
                                                      int64_t G, uint64_t w) {
    const int lane = threadIdx.x & 63;
    int64_t lo = g + 1;  // us[lo] <= w
    for (;;) {
        const int64_t idx = lo + 1 + lane;
        const bool le = idx < G && us[idx] <= w;
        const int c = __popcll(__ballot(le));
        if (c < 64) return lo + c;
        lo += 64;
    }
}

template <bool LAZY, bool SMALL, bool WRITE>
__global__ __launch_bounds__(64 * EB_WAVES) void k_emit_big(const uint64_t *__restrict__ val,
                                                           const uint64_t *__restrict__ meta,
                                                           const uint64_t *__restrict__ lk,
                                                           const int32_t *__restrict__ len,
                                                           const int32_t *__restrict__ kk,
                                                           const int64_t *__restrict__ gs,
                                                           const int64_t *__restrict__ ge,
                                                           const uint64_t *__restrict__ us,
                                                           int64_t G, uint64_t U, uint64_t *wcnt,
                                                           const uint64_t *__restrict__ wbase,
                                                           uint64_t *out, int64_t cap,
                                                           const uint64_t *__restrict__ slot) {
    // group and tile-pair counts on the device (the streamed join): slot[1], slot[4]
    if (slot) {
        G = (int64_t)slot[1];
        U = G > 0 ? slot[4] : 0;
    }
    __shared__ uint64_t buf[WRITE ? EB_WAVES : 1][WRITE ? EB_BUF : 1];
    // tile J's records, one 16-byte entry each, read by the whole wave at one address:
    // SMALL {string id, -m, -(2 pos - m), K'}, else {string id, m, pos, K}, where
    // K' = min(K, 2^31 - 1) as an unsigned word (the same test: |x| < 2^31 below)
    __shared__ int4 tileJ[EB_WAVES][64];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // wave-uniform
    const uint64_t wid = (uint64_t)blockIdx.x * EB_WAVES + wave;
    const uint64_t nwaves = (uint64_t)gridDim.x * EB_WAVES;
    const uint64_t per = (U + nwaves - 1) / nwaves;
    uint64_t w = wid * per;
    const uint64_t wend = min(U, w + per);
    uint64_t *wb = buf[WRITE ? wave : 0];
    int4 *tj = tileJ[wave];
    uint64_t pos = 0;  // WRITE: where the next flushed pair goes
    if constexpr (WRITE) pos = *wbase + wcnt[wid];
    uint64_t npass = 0;  // passing pairs so far (COUNT) or staged (WRITE); wave-uniform
    auto meta_of = [&](int64_t i, uint64_t v) -> uint64_t {
        if constexpr (LAZY) {
            const int32_t sid = (int32_t)(v >> 32);
            if (lk) return lk[sid];
            return ((uint64_t)(uint32_t)len[sid] << 32) | (uint32_t)kk[sid];
        } else {
            return meta[i];
        }
    };
    if (w < wend) {
        int64_t g = last_le_wave(us, 0, G, w);
        const uint64_t u = w - us[g];
        uint64_t J = (uint64_t)((sqrt(8.0 * (double)u + 1.0) - 1.0) * 0.5);
        while (J > 0 && J * (J + 1) / 2 > u) J--;
        while ((J + 1) * (J + 2) / 2 <= u) J++;
        uint64_t I = u - J * (J + 1) / 2;
        int64_t s0 = gs[g], z = ge[g] - s0 + 1;
        uint64_t nt = (uint64_t)(z + 63) / 64;
        int64_t loadedJ = -1;
        for (;;) {
            const int64_t ra = (int64_t)I * 64 + lane;
            const bool ha = ra < z;
            uint64_t va = 0, xa = 0;
            if (ha) {
                va = val[s0 + ra];
                xa = meta_of(s0 + ra, va);
            }
            if ((int64_t)J != loadedJ) {
                const int64_t rb = (int64_t)J * 64 + lane;
                uint64_t vb = 0, xb = 0;
                if (rb < z) {
                    vb = val[s0 + rb];
                    xb = meta_of(s0 + rb, vb);
                }
                const int32_t mb = (int32_t)(xb >> 32), pb = (int32_t)(uint32_t)vb;
                wave_fence();  // the previous tile's reads are done
                if constexpr (SMALL)
                    tj[lane] = make_int4((int32_t)(vb >> 32), -mb, mb - 2 * pb,
                                         (int32_t)min((uint32_t)xb, 0x7FFFFFFFu));
                else
                    tj[lane] = make_int4((int32_t)(vb >> 32), mb, pb, (int32_t)(uint32_t)xb);
                wave_fence();  // the tile is in place for every lane
                loadedJ = (int64_t)J;
            }
            const int nb = (int)min<int64_t>(64, z - (int64_t)J * 64);
            const bool diag = I == J;
            const uint64_t hmask = __ballot(ha);  // lanes holding a record
            const int32_t ia = (int32_t)(va >> 32);
            const int32_t ma = (int32_t)(xa >> 32), pa = (int32_t)(uint32_t)va;
            const int32_t qa = 2 * pa - ma;
            const uint32_t ka = SMALL ? min((uint32_t)xa, 0x7FFFFFFFu) : (uint32_t)xa;
            // the columns j of tile J against every lane's record a; DIAG (I = J): only lanes
            // l < j (records a < b, which exist as b does)
            auto columns = [&](auto diag_tag) {
                constexpr bool DIAG = decltype(diag_tag)::value;
                uint64_t ok = DIAG ? 0ull : hmask;  // lanes that pair with the column
                uint32_t cnt = 0;                   // COUNT: passing pairs of the tile pair
                auto step = [&](int j, const int4 e) {
                    uint64_t fm;
                    if constexpr (SMALL) {
                        // |x| <= K  <=>  x + K <= 2K in 32-bit unsigned arithmetic, exact for
                        // |x| < 2^31 and K < 2^31: with fewer than 2^29 symbols |m_a - m_b| <
                        // 2^29 and |(2 pos_a - m_a) - (2 pos_b - m_b)| < 1.5 * 2^30 (the test
                        // of pass_filter32; a clamped K' passes every such x, as K >= 2^31 does)
                        const uint32_t K = max(ka, (uint32_t)e.w);
                        const uint32_t t1 = (uint32_t)(ma + e.y) + K, t2 = (uint32_t)(qa + e.z) + K;
                        fm = __ballot(max(t1, t2) <= 2 * K);
                    } else {
                        fm = __ballot(pass_filter((int64_t)(uint32_t)ma, (int64_t)(uint32_t)pa,
                                                  (int64_t)(uint32_t)e.y, (int64_t)(uint32_t)e.z,
                                                  (int64_t)max(ka, (uint32_t)e.w)));
                    }
                    const uint64_t mask = fm & __ballot(ia != e.x) & ok;  // the strings differ
                    if constexpr (DIAG) ok = (ok << 1) | 1ull;            // lanes < j + 1
                    if constexpr (WRITE) {
                        if (mask) {
                            if ((mask >> lane) & 1) {
                                const uint64_t plo = (uint64_t)min(ia, e.x), phi = (uint64_t)max(ia, e.x);
                                wb[npass + __popcll(mask & ((1ull << lane) - 1))] = (plo << 32) | phi;
                            }
                            npass += (uint64_t)__popcll(mask);
                            if (npass > EB_BUF - 64) {
                                wave_fence();  // the lanes' staged writes are in place
                                for (uint32_t i = lane; i < (uint32_t)npass; i += 64)
                                    if ((int64_t)(pos + i) < cap) out[pos + i] = wb[i];
                                pos += npass;
                                npass = 0;
                                wave_fence();  // read before the buffer is refilled
                            }
                        }
                    } else {
                        cnt += (uint32_t)__popcll(mask);
                    }
                };
                // every lane reads the same entries; four at a time, then the rest
                int j = 0;
                for (; j + 4 <= nb; j += 4) {
                    const int4 e0 = tj[j], e1 = tj[j + 1], e2 = tj[j + 2], e3 = tj[j + 3];
                    step(j, e0);
                    step(j + 1, e1);
                    step(j + 2, e2);
                    step(j + 3, e3);
                }
                for (; j < nb; j++) step(j, tj[j]);
                if constexpr (!WRITE) npass += cnt;
            };
            if (diag) columns(std::true_type{});
            else columns(std::false_type{});
            // the next tile pair: (I + 1, J), else (0, J + 1), else the next group with tiles
            if (++w >= wend) break;
            if (++I > J) {
                I = 0;
                if (++J >= nt) {
                    g = next_group_of_unit(us, g, G, w);
                    J = 0;
                    s0 = gs[g];
                    z = ge[g] - s0 + 1;
                    nt = (uint64_t)(z + 63) / 64;
                    loadedJ = -1;
                }
            }
        }
    }
    if constexpr (WRITE) {
        if (npass) {
            wave_fence();
            for (uint32_t i = lane; i < (uint32_t)npass; i += 64)
                if ((int64_t)(pos + i) < cap) out[pos + i] = wb[i];
        }
    } else {
        if (lane == 0) wcnt[wid] = npass;
    }
}

// base[0] = the pairs emitted so far (*counter), then *counter += the tile pairs' total
__global__ void k_emit_big_base(unsigned long long *counter, const uint64_t *total, uint64_t *base) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        base[0] = *counter;
        *counter += *total;
    }
}

// Whether the large groups go by tile pairs (tile_min: -1 never, else at least
// max(tile_min, 1) tile pairs).
static bool split_pays(uint64_t units, int64_t tile_min) {
    return tile_min >= 0 && units >= (uint64_t)std::max<int64_t>(tile_min, 1);
}

// The tile-pair emission: count, scan, base, write (see k_emit_big).  U and G are host
// values, or taken from slot on the device when slot is given.
using EmitBigFn = void (*)(const uint64_t *, const uint64_t *, const uint64_t *, const int32_t *,
                           const int32_t *, const int64_t *, const int64_t *, const uint64_t *,
                           int64_t, uint64_t, uint64_t *, const uint64_t *, uint64_t *, int64_t,
                           const uint64_t *);
template <bool WRITE>
static EmitBigFn emit_big_fn(bool lazy, bool small) {
    return lazy ? (small ? k_emit_big<true, true, WRITE> : k_emit_big<true, false, WRITE>)
                : (small ? k_emit_big<false, true, WRITE> : k_emit_big<false, false, WRITE>);
}
// workgroups for U tile pairs: about 2 per wave, at most EB_MAX_BLOCKS (8 waves per SIMD)
constexpr int64_t EB_MAX_BLOCKS = 2048;
static int64_t tile_blocks_for(uint64_t units) {
    return (int64_t)std::max<uint64_t>(
        1, std::min<uint64_t>((units + 2 * EB_WAVES - 1) / (2 * EB_WAVES), EB_MAX_BLOCKS));
}
static void emit_big(const uint64_t *val, const uint64_t *meta, const uint64_t *lk, const DevStrings &d,
                     const GroupInfo &g, int64_t G, uint64_t U, const uint64_t *slot, bool lazy,
                     bool small, int64_t blocks, uint64_t *out, int64_t cap,
                     unsigned long long *counter, Workspace &ws, hipStream_t s) {
    const int64_t nw = blocks * EB_WAVES;
    uint64_t *wcnt = ws.get_n<uint64_t>(nw + 1);
    uint64_t *wpre = ws.get_n<uint64_t>(nw + 1);
    uint64_t *tot = ws.get_n<uint64_t>(2);
    hipLaunchKernelGGL(emit_big_fn<false>(lazy, small), dim3((unsigned)blocks), dim3(64 * EB_WAVES), 0,
                       s, val, meta, lk, d.len, d.kk, g.gstart, g.gend, g.ustart, G, U, wcnt,
                       (const uint64_t *)nullptr, out, cap, slot);
    MJ_LAUNCH_CHECK();
    exclusive_scan_u64_dev(wcnt, wpre, nw, nullptr, tot, ws, s);
    hipLaunchKernelGGL(k_emit_big_base, dim3(1), dim3(64), 0, s, counter, (const uint64_t *)tot, tot + 1);
    MJ_LAUNCH_CHECK();
    hipLaunchKernelGGL(emit_big_fn<true>(lazy, small), dim3((unsigned)blocks), dim3(64 * EB_WAVES), 0,
                       s, val, meta, lk, d.len, d.kk, g.gstart, g.gend, g.ustart, G, U, wpre,
                       (const uint64_t *)(tot + 1), out, cap, slot);
    MJ_LAUNCH_CHECK();
}

int64_t emit_candidates(const uint64_t *val, int64_t R, const GroupInfo &g, const DevStrings &d,
                        uint64_t *out, int64_t cap, Workspace &ws, hipStream_t s,
                        uint64_t *host_scratch, int64_t tile_min, KTimer *kt, uint64_t t_begin,
                        uint64_t t_end) {
    if (g.groups == 0 || g.tests == 0) return 0;
    if (t_end == 0 || t_end > g.tests) t_end = g.tests;
    if (t_begin >= t_end) return 0;
    // the whole join in one pass: the small groups test by test and the large ones by
    // tile pairs, when those are many enough; else (and for a pass of a join emitted in
    // passes) the range of all groups' tests, test by test
    const bool split = t_begin == 0 && t_end == g.tests && split_pays(g.units, tile_min);
    const uint64_t tb = split ? 0 : t_begin, te = split ? g.small_tests : t_end;
    const uint64_t tests = te - tb;  // test by test
    unsigned long long *counter = (unsigned long long *)ws.get_n<uint64_t>(2);
    fill_u64((uint64_t *)counter, 0, 1, s);
    // the (m, K) words of all records in one pass when the pair tests outnumber the
    // records; gathered at each use otherwise (measured: text with 0.46 tests per record
    // gains 0.7 ms, protein with 3.7 loses 0.2 ms gathering)
    const bool lazy = g.tests < (uint64_t)R;
    uint64_t *meta = lazy ? nullptr : ws.get_n<uint64_t>(R + 1);
    // one (m, K) word per string, one gather per look-up, when look-ups are many enough
    // (16 per string) to repay its pass
    const bool packed = !lazy || g.tests >= 16 * (uint64_t)std::max(d.n, 1);
    uint64_t *lk = packed ? ws.get_n<uint64_t>((size_t)d.n + 1) : nullptr;
    int th = kt ? kt->begin(KTimer::EMIT, s) : -1;
    if (packed) {
        hipLaunchKernelGGL(k_string_meta, dim3(grid_for(d.n, 256, 65535)), dim3(256), 0, s, d.len,
                           d.kk, d.n, lk);
        MJ_LAUNCH_CHECK();
    }
    if (!lazy) {
        hipLaunchKernelGGL(k_record_meta, dim3(grid_for(R, 256, 16384)), dim3(256), 0, s, val, R,
                           lk, meta, (const int64_t *)nullptr);
        MJ_LAUNCH_CHECK();
    }
    const bool small = d.total < (1ll << 29);
    if (tests > 0) {
        // a thread locates its first test by a binary search over the groups; with tests
        // enough for 2^20 threads it takes longer runs (up to 4 x EMIT_CHUNK) per search,
        // but not when only the groups below EMIT_TILE records are left (split): there
        // every lane of a wave walks other groups' records, and longer runs put more
        // records in flight than an XCD's L2 holds
        int chunk = EMIT_CHUNK;
        while (!split && chunk < 4 * EMIT_CHUNK && tests / (uint64_t)(2 * chunk) >= (1ull << 20))
            chunk *= 2;
        uint64_t threads = (tests + chunk - 1) / chunk;
        unsigned grid = (unsigned)std::min<uint64_t>((threads + EMIT_BLOCK - 1) / EMIT_BLOCK, 1u << 16);
        hipLaunchKernelGGL(lazy ? (small ? k_emit<true, true> : k_emit<true, false>)
                                : (small ? k_emit<false, true> : k_emit<false, false>),
                           dim3(grid), dim3(EMIT_BLOCK), 0, s, val, meta, lk, d.len, d.kk, g.gstart,
                           split ? g.tsmall : g.tstart, g.groups, te, out, cap, counter, chunk,
                           (const uint64_t *)nullptr, 0, tb);
        MJ_LAUNCH_CHECK();
    }
    if (split && g.units > 0)
        emit_big(val, meta, lk, d, g, g.groups, g.units, nullptr, lazy, small,
                 tile_blocks_for(g.units), out, cap, counter, ws, s);
    if (kt) kt->end(th, s);
    uint64_t c = read_back<uint64_t>((const uint64_t *)counter, s, host_scratch);
    if ((int64_t)c > cap) throw Error(MJ_ECAPACITY, "candidate buffer overflow");
    return (int64_t)c;
}

// ---------------------------------------------------------------- dedup
__global__ void k_unique_flags(const uint64_t *p, int64_t n, uint8_t *f) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) f[i] = (i == 0 || p[i] != p[i - 1]) ? 1 : 0;
}

// (first << 32 | second) <-> (first << b | second), second < 2^b: the same order
__global__ void k_pack_pairs(uint64_t *p, int64_t n, int b) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = ((p[i] >> 32) << b) | (p[i] & 0xFFFFFFFFull);
}

__global__ void k_unpack_pairs(uint64_t *p, int64_t n, int b) {
    const uint64_t lo = b >= 64 ? ~0ull : ((1ull << b) - 1);
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = ((p[i] >> b) << 32) | (p[i] & lo);
}

int64_t dedup_pairs(uint64_t *pairs, int64_t n, int32_t n_first, int32_t n_second, Workspace &ws,
                    hipStream_t s, uint64_t *host_scratch, uint64_t **result, bool to_ws) {
    auto out_buf = [&](int64_t count) {
        return to_ws ? ws.get_n<uint64_t>(count + 1)
                     : (uint64_t *)result_alloc((size_t)(count + 1) * 8, t_dev_alloc, s);
    };
    if (n == 0) {
        *result = out_buf(0);
        return 0;
    }
    // pair = first << 32 | second with first < 2^bf and second < 2^bs.  The radix sort
    // takes 8-bit digits; when the two fields waste digit bits (19 + 19 bits: 3 + 3
    // passes) they are packed next to each other first (38 bits: 5 passes).
    auto field_bits = [](int32_t count) {
        return std::min(32, ceil_log2((uint64_t)std::max(count, 1)));
    };
    const int bf = field_bits(n_first), bs = field_bits(n_second);
    const bool pack = (bf + bs + 7) / 8 < (bf + 7) / 8 + (bs + 7) / 8;
    const unsigned pgrid = grid_for(n, 256, 16384);
    if (pack) {
        hipLaunchKernelGGL(k_pack_pairs, dim3(pgrid), dim3(256), 0, s, pairs, n, bs);
        MJ_LAUNCH_CHECK();
    }
    auto ones = [](int b) { return b >= 64 ? ~0ull : ((1ull << b) - 1); };
    uint64_t *sorted = pairs;  // where the sorted keys end up (no copy back)
    radix_sort(pairs, nullptr, n, pack ? ones(bf + bs) : (ones(bf) << 32) | ones(bs), ws, s,
               nullptr, nullptr, nullptr, &sorted);
    uint8_t *f = ws.get_n<uint8_t>(n);
    hipLaunchKernelGGL(k_unique_flags, dim3(pgrid), dim3(256), 0, s, sorted, n, f);
    MJ_LAUNCH_CHECK();
    int64_t *idx = ws.get_n<int64_t>(n + 1);
    int64_t u = compact_flags(f, n, idx, ws, s, host_scratch);
    uint64_t *res = out_buf(u);
    gather_u64(sorted, idx, res, u, s);
    if (pack && u > 0) {
        hipLaunchKernelGGL(k_unpack_pairs, dim3(grid_for(u, 256, 16384)), dim3(256), 0, s, res, u, bs);
        MJ_LAUNCH_CHECK();
    }
    *result = res;
    return u;
}

// Emission with the record, group and test counts on the device; the candidates go to
// out[0 .. cap), their count (which may exceed cap: the caller checks) to *count.  The
// layout choices (record-aligned (m, K) words, string words, tests per search) come from
// the caller's hints (the last call of the same shape), as they only affect speed.
void emit_candidates_streamed(const uint64_t *val, int64_t R_cap, const int64_t *R_dev,
                              const GroupInfo &g, const DevStrings &d, uint64_t *out, int64_t cap,
                              unsigned long long *count, const EmitHints &h, Workspace &ws,
                              hipStream_t s, KTimer *kt) {
    fill_u64((uint64_t *)count, 0, 1, s);
    uint64_t *meta = h.lazy ? nullptr : ws.get_n<uint64_t>(R_cap + 1);
    const bool packed = !h.lazy || h.string_words;
    uint64_t *lk = packed ? ws.get_n<uint64_t>((size_t)d.n + 1) : nullptr;
    int th = kt ? kt->begin(KTimer::EMIT, s) : -1;
    if (packed) {
        hipLaunchKernelGGL(k_string_meta, dim3(grid_for(d.n, 256, 65535)), dim3(256), 0, s, d.len,
                           d.kk, d.n, lk);
        MJ_LAUNCH_CHECK();
    }
    if (!h.lazy) {
        hipLaunchKernelGGL(k_record_meta, dim3(grid_for(R_cap, 256, 16384)), dim3(256), 0, s, val,
                           R_cap, lk, meta, R_dev);
        MJ_LAUNCH_CHECK();
    }
    const int chunk = std::max(EMIT_CHUNK, h.chunk);
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(h.blocks, 1 << 16));
    const bool small = d.total < (1ll << 29);
    // split (as the last join of this shape chose): the small groups test by test, the
    // large ones by tile pairs; else every group test by test (counts in g.slot)
    hipLaunchKernelGGL(h.lazy ? (small ? k_emit<true, true> : k_emit<true, false>)
                              : (small ? k_emit<false, true> : k_emit<false, false>),
                       dim3(grid), dim3(EMIT_BLOCK), 0, s,
                       val, meta, lk, d.len, d.kk, g.gstart, h.split ? g.tsmall : g.tstart, (int64_t)0,
                       (uint64_t)0, out, cap, count, chunk, (const uint64_t *)g.slot, h.split ? 3 : 2,
                       (uint64_t)0);
    MJ_LAUNCH_CHECK();
    if (h.split)
        emit_big(val, meta, lk, d, g, 0, 0, g.slot, h.lazy, small,
                 std::max<int64_t>(1, std::min<int64_t>(h.tile_blocks, EB_MAX_BLOCKS)), out, cap, count,
                 ws, s);
    if (kt) kt->end(th, s);
}

EmitHints emit_hints(uint64_t tests, uint64_t small_tests, uint64_t units, int64_t R, int32_t n,
                     int64_t tile_min) {
    EmitHints h;
    h.lazy = tests < (uint64_t)R;
    h.string_words = tests >= 16 * (uint64_t)std::max(n, 1);
    h.split = split_pays(units, tile_min);
    const uint64_t tt = h.split ? small_tests : tests;  // test by test
    int chunk = EMIT_CHUNK;  // as in emit_candidates
    while (!h.split && chunk < 4 * EMIT_CHUNK && tt / (uint64_t)(2 * chunk) >= (1ull << 20)) chunk *= 2;
    h.chunk = chunk;
    const uint64_t threads = (tt + chunk - 1) / chunk;
    h.blocks = (int64_t)std::max<uint64_t>(1, std::min<uint64_t>((threads + EMIT_BLOCK - 1) / EMIT_BLOCK,
                                                                  1u << 16));
    h.tile_blocks = tile_blocks_for(units);
    return h;
}

__global__ void k_clamp_count(const unsigned long long *c, int64_t cap, int64_t *out) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *out = min((int64_t)*c, cap);
}

__global__ void k_unique_flags_dev(const uint64_t *p, int64_t cap, const int64_t *n_dev, uint8_t *f) {
    const int64_t n = *n_dev;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < cap; i += stride) f[i] = (i < n && (i == 0 || p[i] != p[i - 1])) ? 1 : 0;
}

__global__ void k_pack_pairs_dev(uint64_t *p, const int64_t *n_dev, int64_t cap, int b, int unpack,
                                 const uint32_t *u_dev) {
    const int64_t n = u_dev ? (int64_t)*u_dev : min(cap, *n_dev);
    const uint64_t lo = b >= 64 ? ~0ull : ((1ull << b) - 1);
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride)
        p[i] = unpack ? ((p[i] >> b) << 32) | (p[i] & lo) : ((p[i] >> 32) << b) | (p[i] & 0xFFFFFFFFull);
}

// Dedup with the candidate count on the device (*count, at most cap of them kept); the
// distinct pairs go to a workspace array of cap entries, their number to the returned
// device word.
const uint32_t *dedup_pairs_streamed(uint64_t *pairs, int64_t cap, const unsigned long long *count,
                                     int32_t n_first, int32_t n_second, Workspace &ws, hipStream_t s,
                                     uint64_t **result) {
    cap = std::max<int64_t>(cap, 1);
    int64_t *n_dev = ws.get_n<int64_t>(2);
    hipLaunchKernelGGL(k_clamp_count, dim3(1), dim3(64), 0, s, count, cap, n_dev);
    MJ_LAUNCH_CHECK();
    auto field_bits = [](int32_t c) { return std::min(32, ceil_log2((uint64_t)std::max(c, 1))); };
    const int bf = field_bits(n_first), bs = field_bits(n_second);
    const bool pack = (bf + bs + 7) / 8 < (bf + 7) / 8 + (bs + 7) / 8;
    const unsigned pgrid = grid_for(cap, 256, 16384);
    if (pack) {
        hipLaunchKernelGGL(k_pack_pairs_dev, dim3(pgrid), dim3(256), 0, s, pairs, n_dev, cap, bs, 0,
                           (const uint32_t *)nullptr);
        MJ_LAUNCH_CHECK();
    }
    auto ones = [](int b) { return b >= 64 ? ~0ull : ((1ull << b) - 1); };
    uint64_t *sorted = pairs;  // where the sorted keys end up (no copy back)
    radix_sort(pairs, nullptr, cap, pack ? ones(bf + bs) : (ones(bf) << 32) | ones(bs), ws, s, n_dev,
               nullptr, nullptr, &sorted);
    uint8_t *f = ws.get_n<uint8_t>(cap);
    hipLaunchKernelGGL(k_unique_flags_dev, dim3(pgrid), dim3(256), 0, s, sorted, cap, n_dev, f);
    MJ_LAUNCH_CHECK();
    int64_t *idx = ws.get_n<int64_t>(cap + 1);
    const uint32_t *u = compact_flags_async(f, cap, idx, ws, s);
    uint64_t *res = ws.get_n<uint64_t>(cap + 1);
    gather_u64(sorted, idx, res, cap, s, u);
    if (pack) {
        hipLaunchKernelGGL(k_pack_pairs_dev, dim3(pgrid), dim3(256), 0, s, res, n_dev, cap, bs, 1, u);
        MJ_LAUNCH_CHECK();
    }
    *result = res;
    return u;
}

// ---------------------------------------------------------------- search probe
// For each query record, the equal-key range of the sorted index records.
__global__ void k_probe_ranges(const uint64_t *qkey, int64_t RQ, const uint64_t *ikey, int64_t RI,
                               int64_t *lo_out, uint64_t *cnt) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < RQ; i += stride) {
        uint64_t k = qkey[i];
        int64_t lo = 0, hi = RI;  // first index with ikey >= k
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if (ikey[mid] < k) lo = mid + 1; else hi = mid;
        }
        int64_t e = lo, hi2 = RI;  // first index with ikey > k
        while (e < hi2) {
            int64_t mid = (e + hi2) >> 1;
            if (ikey[mid] <= k) e = mid + 1; else hi2 = mid;
        }
        lo_out[i] = lo;
        cnt[i] = (uint64_t)(e - lo);
    }
}

__global__ __launch_bounds__(EMIT_BLOCK) void k_probe_emit(const uint64_t *__restrict__ qval,
                                                    const int64_t *__restrict__ lo_arr,
                                                    const uint64_t *__restrict__ ts, int64_t RQ,
                                                    uint64_t P, const uint64_t *__restrict__ ival,
                                                    const int32_t *__restrict__ qlen,
                                                    const int32_t *__restrict__ qk,
                                                    const int32_t *__restrict__ ilen,
                                                    uint64_t *out, int64_t cap,
                                                    unsigned long long *counter) {
    __shared__ EmitStage st;
    if (threadIdx.x == 0) st.n = 0;
    __syncthreads();
    const uint64_t nthreads = (uint64_t)gridDim.x * EMIT_BLOCK;
    for (uint64_t t0 = ((uint64_t)blockIdx.x * EMIT_BLOCK + threadIdx.x) * EMIT_CHUNK; ;
         t0 += nthreads * EMIT_CHUNK) {
        if (t0 - (uint64_t)threadIdx.x * EMIT_CHUNK >= P) break;
        bool active = t0 < P;
        int64_t r = 0;
        uint64_t j = 0;
        if (active) {
            int64_t lo = 0, hi = RQ;  // largest r with ts[r] <= t0
            while (hi - lo > 1) {
                int64_t mid = (lo + hi) >> 1;
                if (ts[mid] <= t0) lo = mid; else hi = mid;
            }
            r = lo;
            j = t0 - ts[r];
        }
        for (int c = 0; c < EMIT_CHUNK; c++) {
            uint64_t t = t0 + c;
            bool live = active && t < P;
            bool pass = false;
            uint64_t pairkey = 0;
            if (live) {
                // skip query records with empty ranges
                while (j >= ts[r + 1] - ts[r]) {
                    j = 0;
                    r++;
                }
                uint64_t qv = qval[r];
                uint64_t iv = ival[lo_arr[r] + (int64_t)j];
                int32_t qi = (int32_t)(qv >> 32), si = (int32_t)(iv >> 32);
                pass = pass_filter(qlen[qi], (int64_t)(uint32_t)qv, ilen[si], (int64_t)(uint32_t)iv,
                                   qk[qi]);
                pairkey = ((uint64_t)(uint32_t)qi << 32) | (uint64_t)(uint32_t)si;
                j++;
            }
            stage(pass, pairkey, st);
        }
        flush(st, counter, out, cap);
    }
}

int64_t probe_candidates(const uint64_t *qkey, const uint64_t *qval, int64_t RQ,
                         const uint64_t *ikey, const uint64_t *ival, int64_t RI,
                         const DevStrings &qd, const DevStrings &id, uint64_t *out, int64_t cap,
                         uint64_t *tests_out, Workspace &ws, hipStream_t s, uint64_t *host_scratch) {
    *tests_out = 0;
    if (RQ == 0 || RI == 0) return 0;
    int64_t *lo = ws.get_n<int64_t>(RQ + 1);
    uint64_t *cnt = ws.get_n<uint64_t>(RQ + 1);
    uint64_t *ts = ws.get_n<uint64_t>(RQ + 1);
    hipLaunchKernelGGL(k_probe_ranges, dim3(grid_for(RQ, 256, 16384)), dim3(256), 0, s, qkey, RQ,
                       ikey, RI, lo, cnt);
    MJ_LAUNCH_CHECK();
    exclusive_scan_u64(cnt, ts, RQ, ws, s);
    uint64_t P = read_back<uint64_t>(ts + RQ, s, host_scratch);
    *tests_out = P;
    if (P == 0) return 0;
    if (cap < 0) return -(int64_t)P;
    unsigned long long *counter = (unsigned long long *)ws.get_n<uint64_t>(2);
    fill_u64((uint64_t *)counter, 0, 1, s);
    uint64_t threads = (P + EMIT_CHUNK - 1) / EMIT_CHUNK;
    unsigned grid = (unsigned)std::min<uint64_t>((threads + EMIT_BLOCK - 1) / EMIT_BLOCK, 1u << 16);
    hipLaunchKernelGGL(k_probe_emit, dim3(grid), dim3(EMIT_BLOCK), 0, s, qval, lo, ts, RQ, P, ival,
                       qd.len, qd.kk, id.len, out, cap, counter);
    MJ_LAUNCH_CHECK();
    uint64_t c = read_back<uint64_t>((const uint64_t *)counter, s, host_scratch);
    if ((int64_t)c > cap) throw Error(MJ_ECAPACITY, "candidate buffer overflow");
    return (int64_t)c;
}

}  // namespace mj
