// Device primitives: workspace, fills, exclusive scans, stream compaction and an LSD radix
// sort of (key, value) records.  All loops are bounds-checked; grids come from host-known
// sizes.
#include <string.h>

#include <algorithm>
#include <mutex>

#include "mj_common.h"

namespace mj {

// ---------------------------------------------------------------- workspace / alloc
thread_local mj_allocator t_dev_alloc{};

void *dev_alloc(size_t bytes, const mj_allocator &a) {
    void *p = nullptr;
    if (bytes == 0) bytes = 16;
    if (a.alloc) {
        p = a.alloc(bytes, a.user);
        if (!p) throw Error(MJ_ENOMEM, "the caller's allocator refused " + std::to_string(bytes) + " bytes");
        return p;
    }
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        throw Error(MJ_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    return p;
}

void dev_free(void *p, const mj_allocator &a) {
    if (!p) return;
    if (a.alloc) a.free(p, a.user);
    else (void)hipFree(p);
}

void *dev_alloc(size_t bytes) { return dev_alloc(bytes, t_dev_alloc); }
void dev_free(void *p) { dev_free(p, t_dev_alloc); }

// One pool per device, made on first use and kept for the life of the process.
static hipMemPool_t result_pool(int dev) {
    static std::mutex mu;
    static std::vector<hipMemPool_t> pools;
    std::lock_guard<std::mutex> lock(mu);
    if ((int)pools.size() <= dev) pools.resize(dev + 1, nullptr);
    if (!pools[dev]) {
        hipMemPoolProps props{};
        props.allocType = hipMemAllocationTypePinned;
        props.handleTypes = hipMemHandleTypeNone;
        props.location.type = hipMemLocationTypeDevice;
        props.location.id = dev;
        hipMemPool_t p = nullptr;
        if (hipMemPoolCreate(&p, &props) != hipSuccess) {
            (void)hipGetLastError();
            throw Error(MJ_EDEVICE, "result memory pool creation failed");
        }
        uint64_t keep = RESULT_POOL_KEEP;
        (void)hipMemPoolSetAttribute(p, hipMemPoolAttrReleaseThreshold, &keep);
        pools[dev] = p;
    }
    return pools[dev];
}

void *result_alloc(size_t bytes, const mj_allocator &a, hipStream_t s) {
    if (a.alloc) return dev_alloc(bytes, a);
    if (bytes == 0) bytes = 16;
    int dev = 0;
    MJ_HIP(hipGetDevice(&dev));
    void *p = nullptr;
    if (hipMallocFromPoolAsync(&p, bytes, result_pool(dev), s) != hipSuccess) {
        (void)hipGetLastError();
        throw Error(MJ_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    return p;
}

void result_free(void *p, const mj_allocator &a, hipStream_t s) {
    if (!p) return;
    if (a.alloc) a.free(p, a.user);
    else (void)hipFreeAsync(p, s);
}

Workspace::~Workspace() {
    for (auto &b : blocks_) dev_free(b.p, alloc);
    if (scan.state && !arena()) dev_free(scan.state, alloc);
}

void Workspace::bind_arena(void *base, size_t bytes) {
    arena_base_ = static_cast<uint8_t *>(base);
    arena_bytes_ = bytes;
    arena_used_ = ARENA_SCAN_BYTES;
    // the ticket on a line of its own after the tile words (as in scan_u32_single_pass)
    scan.state = reinterpret_cast<uint64_t *>(arena_base_);
    scan.ticket = reinterpret_cast<unsigned long long *>(scan.state + ARENA_SCAN_BYTES / 8 - 32);
    scan.base = 0;
    scan.epoch = 0;
}

void *Workspace::get(size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    if (arena()) {
        if (bytes > arena_bytes_ - arena_used_)
            throw Error(MJ_ECAPACITY, "the call needs more than the " +
                                          std::to_string(arena_bytes_ >> 20) +
                                          " MiB of fixed scratch memory");
        void *p = arena_base_ + arena_used_;
        arena_used_ += bytes;
        return p;
    }
    Block *best = nullptr;
    for (auto &b : blocks_)
        if (!b.used && b.n >= bytes && (!best || b.n < best->n)) best = &b;
    if (best && best->n <= 4 * bytes + (1 << 20)) {
        best->used = true;
        best->held = holding_;
        return best->p;
    }
    void *p = nullptr;
    try {
        p = dev_alloc(bytes, alloc);
    } catch (const Error &) {
        // free idle blocks and retry once (the stream work of earlier calls is complete:
        // every entry point synchronises before it returns)
        for (auto it = blocks_.begin(); it != blocks_.end();) {
            if (!it->used) { dev_free(it->p, alloc); held_ -= it->n; it = blocks_.erase(it); }
            else ++it;
        }
        p = dev_alloc(bytes, alloc);
    }
    blocks_.push_back({p, bytes, true, holding_});
    held_ += bytes;
    return p;
}

void Workspace::release_all() {
    size_t used = 0;
    for (auto &b : blocks_) {
        if (b.used) used += b.n;
        if (!b.held) b.used = false;
    }
    last_used_ = arena() ? arena_used_ : used;
    if (arena()) arena_used_ = ARENA_SCAN_BYTES;
}

void Workspace::drop_holds() {
    for (auto &b : blocks_)
        if (b.held) {
            b.held = false;
            b.used = false;
        }
}


// ---------------------------------------------------------------- kernel timers
void KTimer::create() {
    for (auto &e : ev) MJ_HIP(hipEventCreate(&e));
}

void KTimer::destroy() {
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
}

int KTimer::begin(int slot, hipStream_t s) {
    if (used + 2 > POOL) return -1;
    int h = used;
    used += 2;
    slot_of[h / 2] = slot;
    MJ_HIP(hipEventRecord(ev[h], s));
    return h;
}

void KTimer::end(int h, hipStream_t s, int launches) {
    if (h < 0) return;
    count_of[h / 2] = launches;
    MJ_HIP(hipEventRecord(ev[h + 1], s));
}

void KTimer::collect(float *ms, int32_t *launches) {
    for (int i = 0; i < SLOTS; i++) {
        ms[i] = 0.f;
        launches[i] = 0;
    }
    for (int h = 0; h + 1 < used; h += 2) {
        float t = 0.f;
        MJ_HIP(hipEventElapsedTime(&t, ev[h], ev[h + 1]));
        ms[slot_of[h / 2]] += t;
        launches[slot_of[h / 2]] += count_of[h / 2];
    }
}

// ---------------------------------------------------------------- fills
template <class T>
__global__ void k_fill(T *p, T v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

static unsigned grid_for(int64_t n, int block, unsigned cap = 65535u) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    return (unsigned)std::min<int64_t>(g, cap);
}

void fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill<uint32_t>, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, p, v, n);
    MJ_LAUNCH_CHECK();
}

void fill_u64(uint64_t *p, uint64_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill<uint64_t>, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, p, v, n);
    MJ_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- scan
constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

template <class T>
__device__ __forceinline__ T shfl_up_t(T v, int d) {
    if constexpr (sizeof(T) == 8) {
        uint32_t lo = (uint32_t)v, hi = (uint32_t)((uint64_t)v >> 32);
        lo = __shfl_up(lo, d, 64);
        hi = __shfl_up(hi, d, 64);
        return (T)(((uint64_t)hi << 32) | lo);
    } else {
        return (T)__shfl_up((uint32_t)v, d, 64);
    }
}

// Exclusive scan of one value per thread across the block; returns the prefix and
// writes the block total to *total (all threads).
template <class T>
__device__ T block_exclusive_scan(T v, T *smem /* >= 4 entries */, T *total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    T inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        T o = shfl_up_t(inc, d);
        if (lane >= d) inc += o;
    }
    if (lane == 63) smem[wid] = inc;
    __syncthreads();
    T wpre = 0, tot = 0;
    const int nw = blockDim.x >> 6;
    for (int w = 0; w < nw; w++) {
        T x = smem[w];
        if (w < wid) wpre += x;
        tot += x;
    }
    __syncthreads();
    *total = tot;
    return wpre + inc - v;
}

// ndev (optional): the element count is min(n, *ndev), a device value; tiles past it
// contribute 0 and write nothing.
template <class In, class T>
__global__ void k_scan_reduce(const In *in, int64_t n, T *partial, const uint32_t *ndev) {
    __shared__ T smem[8];
    if (ndev) n = min<int64_t>(n, *ndev);
    if ((int64_t)blockIdx.x * SCAN_TILE >= n) {  // block-uniform
        if (threadIdx.x == 0) partial[blockIdx.x] = 0;
        return;
    }
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    T s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; k++)
        if (base + k < n) s += (T)in[base + k];
    T tot;
    (void)block_exclusive_scan<T>(s, smem, &tot);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// ndev as for k_scan_reduce; total_out (optional) receives the grand total as well.
template <class In, class T>
__global__ void k_scan_apply(const In *in, int64_t n, const T *partial_scan, T *out,
                             const uint32_t *ndev, T *total_out) {
    __shared__ T smem[8];
    if (ndev) n = min<int64_t>(n, *ndev);
    if ((int64_t)blockIdx.x * SCAN_TILE >= n) {  // block-uniform
        if (n == 0 && blockIdx.x == 0 && threadIdx.x == 0) {
            out[0] = 0;
            if (total_out) *total_out = 0;
        }
        return;
    }
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    T v[SCAN_ITEMS];
    T s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; k++) {
        v[k] = (base + k < n) ? (T)in[base + k] : (T)0;
        s += v[k];
    }
    T tot;
    T pre = block_exclusive_scan<T>(s, smem, &tot);
    T off = partial_scan ? partial_scan[blockIdx.x] : (T)0;
    T run = off + pre;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; k++) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
    // the block holding element n-1 writes the grand total at out[n]
    int64_t last = n - 1;
    if (last >= base && last < base + SCAN_ITEMS) {
        out[n] = run;
        if (total_out) *total_out = run;
    }
}

// Single-pass scan of 32-bit sums (decoupled look-back).  A workgroup takes the next tile
// from a ticket counter, so every tile below its own belongs to a workgroup that has
// already started.  It publishes its tile's sum as soon as it has it (status 1), then its
// first wave looks back over the preceding tiles 64 at a time, adding their published
// sums until it meets a tile that has published its inclusive prefix (status 2), and
// publishes its own inclusive prefix.  It only ever waits for sums that running
// workgroups publish before they wait themselves, so the launch cannot deadlock.  A state
// word is epoch << 34 | status << 32 | value, written and read whole with device-scope
// atomics; words of other calls (other epochs) read as not yet published.
// Device-scope atomics are slow enough here that the look-back chain of a long scan costs
// more than the two extra launches of the reduce-then-scan path, which long scans keep:
// measured, 1,800 tiles ran slower this way and 115 tiles faster.
constexpr int64_t SCAN_LOOKBACK_MAX_TILES = 256;
constexpr int64_t SCAN_MAX_TILES = SCAN_LOOKBACK_MAX_TILES;

__device__ __forceinline__ uint64_t scan_state_load(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void scan_state_store(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <class In>
__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_lookback(const In *in, int64_t n, uint32_t *out,
                                                              uint64_t *state,
                                                              unsigned long long *ticket,
                                                              uint64_t tbase, uint32_t epoch) {
    __shared__ uint32_t smem[8];
    __shared__ uint32_t tile_s, excl_s;
    if (threadIdx.x == 0) tile_s = (uint32_t)(atomicAdd(ticket, 1ull) - tbase);
    __syncthreads();
    const int64_t tile = tile_s;
    const int64_t base = tile * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    uint32_t v[SCAN_ITEMS];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; k++) {
        v[k] = (base + k < n) ? (uint32_t)in[base + k] : 0u;
        sum += v[k];
    }
    uint32_t tot;
    const uint32_t pre = block_exclusive_scan<uint32_t>(sum, smem, &tot);
    const uint64_t tag = (uint64_t)epoch << 34;
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        uint32_t excl = 0;
        if (tile == 0) {
            if (lane == 0) scan_state_store(state, tag | (2ull << 32) | tot);
        } else {
            if (lane == 0) scan_state_store(state + tile, tag | (1ull << 32) | tot);
            for (int64_t j = tile - 1;; j -= 64) {
                const int64_t idx = j - lane;  // lane 0 is the nearest tile
                uint64_t w = 0;
                int st = 2;  // before tile 0: an inclusive prefix of 0
                int fi;
                for (;;) {
                    if (idx >= 0) {
                        w = scan_state_load(state + idx);
                        st = (uint32_t)(w >> 34) == epoch ? (int)((w >> 32) & 3u) : 0;
                    }
                    const uint64_t incl = __ballot(st == 2), wait = __ballot(st == 0);
                    fi = incl ? __ffsll((unsigned long long)incl) - 1 : 63;
                    if ((wait & (~0ull >> (63 - fi))) == 0) break;  // lanes 0..fi published
                }
                uint32_t part = lane <= fi ? (uint32_t)w : 0u;
                for (int d = 32; d >= 1; d >>= 1) part += (uint32_t)__shfl_xor((int)part, d, 64);
                excl += part;
                if (__ballot(st == 2) & (~0ull >> (63 - fi)) & (1ull << fi)) break;
            }
            if (lane == 0) scan_state_store(state + tile, tag | (2ull << 32) | (uint32_t)(excl + tot));
        }
        if (lane == 0) excl_s = excl;
    }
    __syncthreads();
    uint32_t run = excl_s + pre;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; k++) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
    if (n - 1 >= base && n - 1 < base + SCAN_ITEMS) out[n] = run;
}

template <class In, class T>
static void scan_impl(const In *in, T *out, int64_t n, Workspace &ws, hipStream_t s,
                      const uint32_t *ndev = nullptr, T *total_out = nullptr);

template <class In>
static void scan_u32_single_pass(const In *in, uint32_t *out, int64_t n, int64_t nb, Workspace &ws,
                                 hipStream_t s) {
    if (nb > SCAN_MAX_TILES) throw Error(MJ_ECAPACITY, "scan too large");
    auto &sc = ws.scan;
    static_assert((SCAN_MAX_TILES + 64) * 8 <= Workspace::ARENA_SCAN_BYTES, "arena scan state");
    if (!sc.state) {
        // the ticket on a line of its own after the tile words; all zero (epoch 0 unused)
        sc.state = (uint64_t *)dev_alloc((size_t)(SCAN_MAX_TILES + 64) * 8, ws.alloc);
        sc.ticket = (unsigned long long *)(sc.state + SCAN_MAX_TILES + 32);
        fill_u64(sc.state, 0, SCAN_MAX_TILES + 64, s);
        sc.base = 0;
        sc.epoch = 0;
    }
    if (++sc.epoch >= (1u << 30)) {
        fill_u64(sc.state, 0, SCAN_MAX_TILES, s);
        sc.epoch = 1;
    }
    hipLaunchKernelGGL(k_scan_lookback<In>, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, in, n, out,
                       sc.state, sc.ticket, sc.base, sc.epoch);
    MJ_LAUNCH_CHECK();
    sc.base += (uint64_t)nb;
}

template <class In, class T>
static void scan_impl(const In *in, T *out, int64_t n, Workspace &ws, hipStream_t s,
                      const uint32_t *ndev, T *total_out) {
    if (n <= 0) {
        hipLaunchKernelGGL(k_fill<T>, dim3(1), dim3(64), 0, s, out, (T)0, (int64_t)1);
        MJ_LAUNCH_CHECK();
        return;
    }
    int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb == 1) {
        hipLaunchKernelGGL((k_scan_apply<In, T>), dim3(1), dim3(SCAN_BLOCK), 0, s, in, n,
                           (const T *)nullptr, out, ndev, total_out);
        MJ_LAUNCH_CHECK();
        return;
    }
    if (nb > 2147483647LL) throw Error(MJ_ECAPACITY, "scan too large");
    if constexpr (sizeof(T) == 4) {
        if (nb <= SCAN_LOOKBACK_MAX_TILES && !ndev && !total_out && !ws.no_lookback) {
            scan_u32_single_pass<In>(in, out, n, nb, ws, s);
            return;
        }
    }
    T *partial = ws.get_n<T>(nb + 1);
    T *pscan = ws.get_n<T>(nb + 1);
    hipLaunchKernelGGL((k_scan_reduce<In, T>), dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, in, n,
                       partial, ndev);
    MJ_LAUNCH_CHECK();
    scan_impl<T, T>(partial, pscan, nb, ws, s);
    hipLaunchKernelGGL((k_scan_apply<In, T>), dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, in, n,
                       (const T *)pscan, out, ndev, total_out);
    MJ_LAUNCH_CHECK();
}

void exclusive_scan_u32(const uint32_t *in, uint32_t *out, int64_t n, Workspace &ws, hipStream_t s) {
    scan_impl<uint32_t, uint32_t>(in, out, n, ws, s);
}
void exclusive_scan_u64(const uint64_t *in, uint64_t *out, int64_t n, Workspace &ws, hipStream_t s) {
    scan_impl<uint64_t, uint64_t>(in, out, n, ws, s);
}
void exclusive_scan_u64_dev(const uint64_t *in, uint64_t *out, int64_t n, const uint32_t *count,
                            uint64_t *total_out, Workspace &ws, hipStream_t s) {
    scan_impl<uint64_t, uint64_t>(in, out, std::max<int64_t>(n, 1), ws, s, count, total_out);
}

// ---------------------------------------------------------------- compaction
// Indices of the nonzero flags, in order, in three launches and two passes over the
// flags: per-tile counts, a scan of the tile counts, and a compaction in which each tile
// ranks its flags with one block-wide prefix (no per-element prefix array).
constexpr int CT_ITEMS = 16;                      // flags per thread (one 16-byte load)
constexpr int CT_TILE = SCAN_BLOCK * CT_ITEMS;    // 4,096 flags per tile

// the CT_ITEMS flags of this thread as bits (bit k: element base + k is flagged)
__device__ __forceinline__ uint32_t flag_bits(const uint8_t *flags, int64_t n, int64_t base) {
    uint32_t m = 0;
    if (base + CT_ITEMS <= n && ((uintptr_t)(flags + base) & 15) == 0) {
        const uint4 v = *reinterpret_cast<const uint4 *>(flags + base);
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < CT_ITEMS; k++) m |= ((w[k >> 2] >> (8 * (k & 3))) & 0xFFu) ? 1u << k : 0u;
    } else {
        for (int k = 0; k < CT_ITEMS; k++)
            if (base + k < n && flags[base + k]) m |= 1u << k;
    }
    return m;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_flag_counts(const uint8_t *flags, int64_t n,
                                                            uint32_t *tile_count) {
    __shared__ uint32_t smem[8];
    const int64_t base = (int64_t)blockIdx.x * CT_TILE + (int64_t)threadIdx.x * CT_ITEMS;
    uint32_t tot;
    (void)block_exclusive_scan<uint32_t>((uint32_t)__popc(flag_bits(flags, n, base)), smem, &tot);
    if (threadIdx.x == 0) tile_count[blockIdx.x] = tot;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_compact_tiles(const uint8_t *flags, int64_t n,
                                                              const uint32_t *tile_pre,
                                                              int64_t *idx) {
    __shared__ uint32_t smem[8];
    const int64_t base = (int64_t)blockIdx.x * CT_TILE + (int64_t)threadIdx.x * CT_ITEMS;
    uint32_t m = flag_bits(flags, n, base);
    uint32_t tot;
    uint32_t r = tile_pre[blockIdx.x] + block_exclusive_scan<uint32_t>((uint32_t)__popc(m), smem, &tot);
    while (m) {
        idx[r++] = base + __ffs(m) - 1;
        m &= m - 1;
    }
}

const uint32_t *compact_flags_async(const uint8_t *flags, int64_t n, int64_t *idx_out,
                                    Workspace &ws, hipStream_t s) {
    // 32-bit ranks: the count of kept elements must stay below 2^32
    if (n > 0xFFFFFFF0LL) throw Error(MJ_ECAPACITY, "compaction of more than 2^32 elements");
    const int64_t nb = std::max<int64_t>((n + CT_TILE - 1) / CT_TILE, 1);
    uint32_t *cnt = ws.get_n<uint32_t>(nb + 1);
    uint32_t *pre = ws.get_n<uint32_t>(nb + 1);
    hipLaunchKernelGGL(k_flag_counts, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, flags, n, cnt);
    MJ_LAUNCH_CHECK();
    scan_impl<uint32_t, uint32_t>(cnt, pre, nb, ws, s);
    hipLaunchKernelGGL(k_compact_tiles, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, flags, n, pre,
                       idx_out);
    MJ_LAUNCH_CHECK();
    return pre + nb;
}

int64_t compact_flags(const uint8_t *flags, int64_t n, int64_t *idx_out, Workspace &ws,
                      hipStream_t s, uint64_t *host_scratch) {
    if (n <= 0) return 0;
    return (int64_t)read_back<uint32_t>(compact_flags_async(flags, n, idx_out, ws, s), s,
                                        host_scratch);
}

__global__ void k_gather_u64(const uint64_t *src, const int64_t *idx, uint64_t *dst, int64_t n,
                             const uint32_t *n_dev) {
    if (n_dev) n = min(n, (int64_t)*n_dev);
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) dst[i] = src[idx[i]];
}

void gather_u64(const uint64_t *src, const int64_t *idx, uint64_t *dst, int64_t n, hipStream_t s,
                const uint32_t *n_dev) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_gather_u64, dim3(grid_for(n, 256, 16384)), dim3(256), 0, s, src, idx, dst, n,
                       n_dev);
    MJ_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- radix sort
// Least-significant-digit radix sort on 8-bit digits, stable, keys with an optional
// 64-bit payload.  One pass: per-tile digit counts (k_rs_tile_counts), an exclusive
// scan over (digit, tile), and a scatter (k_rs_scatter) in which every element's rank
// among equal digits of its tile comes from LDS counters.  Inside a wave, the lanes that
// share a digit find each other with one ballot per digit bit, so each group updates
// its counter once (no serialisation on frequent digits).  Digit positions at which all
// keys are known to be zero (the caller's bit mask) are skipped.
constexpr int RS_THREADS = 256;
constexpr int RS_WAVES = RS_THREADS / 64;
constexpr int RS_ITEMS = 16;                      // chunks of 64 per wave
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;    // 4096 elements per tile
constexpr int RS_WAVE_SPAN = 64 * RS_ITEMS;       // a wave owns 1024 consecutive elements

// Lanes of this wave (among `valid`) whose 8-bit digit equals this lane's.
__device__ __forceinline__ uint64_t digit_peers(uint32_t d, uint64_t valid) {
    uint64_t peers = valid;
#pragma unroll
    for (int b = 0; b < 8; b++) {
        const bool bit = (d >> b) & 1u;
        const uint64_t m = __ballot(bit);
        peers &= bit ? m : ~m;
    }
    return peers;
}

// The tile a workgroup takes.  Workgroups are dispatched round-robin over the 8 XCDs, each
// with its own L2; giving XCD x the contiguous tiles [start(x), start(x) + count(x)) keeps
// the digit-major counts and offsets of neighbouring tiles (one cache line holds 32) and
// the seams between their output runs within one L2.  A bijection of [0, ntiles).
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t ntiles) {
    const int64_t per = ntiles >> 3, rem = ntiles & 7, x = b & 7;
    return x * per + min(x, rem) + (b >> 3);
}

// The tile of workgroup b when only the first nt_act of ntiles tiles hold elements (a
// count known on the device): those are spread over the XCDs as above, and workgroups
// b >= nt_act take the empty tiles b (whose counts are zero).
__device__ __forceinline__ int64_t xcd_tile_act(int64_t b, int64_t n) {
    const int64_t nt_act = (n + RS_TILE - 1) / RS_TILE;
    return b < nt_act ? xcd_tile(b, nt_act) : b;
}

__device__ __forceinline__ uint64_t lanes_below() {
    const int lane = threadIdx.x & 63;
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Digit counts of one tile, written digit-major: cnt[d * ntiles + tile].
// n_dev (nullable): the element count on the device (n is then the capacity the tiles
// cover; tiles past the count write zero counts).
__global__ __launch_bounds__(RS_THREADS) void k_rs_tile_counts(const uint64_t *__restrict__ key,
                                                               int64_t n, int shift, int64_t ntiles,
                                                               uint32_t *__restrict__ cnt,
                                                               const int64_t *__restrict__ n_dev) {
    if (n_dev) n = min(n, *n_dev);
    const int64_t tile = xcd_tile_act(blockIdx.x, n);
    if (tile * RS_TILE >= n) {  // an empty tile: zero counts (the whole workgroup)
        cnt[(int64_t)threadIdx.x * ntiles + tile] = 0;
        return;
    }
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t base = tile * RS_TILE + (int64_t)wave * RS_WAVE_SPAN;
    const uint64_t below = lanes_below();
    for (int c = 0; c < RS_ITEMS; c++) {
        const int64_t i = base + (int64_t)c * 64 + lane;
        const bool ok = i < n;
        const uint32_t d = ok ? (uint32_t)(key[i] >> shift) & 255u : 0u;
        const uint64_t peers = digit_peers(d, __ballot(ok));
        if (ok && (peers & below) == 0) atomicAdd(&h[d], (uint32_t)__popcll(peers));
    }
    __syncthreads();
    cnt[(int64_t)threadIdx.x * ntiles + tile] = h[threadIdx.x];
}

// Exclusive scan of one value per thread over a 256-thread block (v of thread t ->
// sum of v over threads < t); `tmp` holds RS_WAVES words.
__device__ __forceinline__ uint32_t block_exclusive_scan_256(uint32_t v, uint32_t *tmp) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) tmp[wave] = x;
    __syncthreads();
    uint32_t before = 0;
    for (int w = 0; w < wave; w++) before += tmp[w];
    return before + x - v;
}

// Scatter of one tile: ranks among equal digits (wave peer groups and per-wave LDS
// counters), the tile staged in LDS in digit order, then written out so that
// consecutive lanes write consecutive addresses of a digit's run.  Keys and payloads
// take turns in one LDS buffer (38 KB per workgroup instead of 70 KB), and the payloads
// are loaded only once the keys are ranked, which keeps the kernel within 128 registers:
// four workgroups fit a CU where two did.  BUILD (keys only): each input key k at index i
// is written as (top half of k) << 32 | i, the narrow element of the member filter.
template <bool HASV, bool BUILD = false>
__global__ __launch_bounds__(RS_THREADS) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_rs_scatter(
    const uint64_t *__restrict__ kin, const uint64_t *__restrict__ vin, uint64_t *__restrict__ kout,
    uint64_t *__restrict__ vout, int64_t n, int shift, int64_t ntiles,
    const uint32_t *__restrict__ off, const int64_t *__restrict__ n_dev) {
    if (n_dev) n = min(n, *n_dev);
    if ((int64_t)blockIdx.x * RS_TILE >= n) return;  // an empty tile (whole workgroup)
    __shared__ uint32_t wc[RS_WAVES][256];  // per-wave digit counts, then per-wave offsets
    __shared__ uint32_t gbase[256];         // global position minus tile-local position
    __shared__ uint32_t tmp[RS_WAVES];
    __shared__ uint64_t sk[RS_TILE];  // the tile's keys in digit order, then its payloads
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int w = 0; w < RS_WAVES; w++) wc[w][threadIdx.x] = 0;
    __syncthreads();
    const int64_t tile = xcd_tile_act(blockIdx.x, n);
    const int64_t tile0 = tile * RS_TILE;
    const int64_t base = tile0 + (int64_t)wave * RS_WAVE_SPAN;
    const uint64_t below = lanes_below();
    uint64_t k[RS_ITEMS];
    uint64_t v[HASV ? RS_ITEMS : 1];
    uint32_t dr[RS_ITEMS];  // digit << 16 | rank inside the wave's span
#pragma unroll
    for (int c = 0; c < RS_ITEMS; c++) {
        const int64_t i = base + (int64_t)c * 64 + lane;
        const bool ok = i < n;
        k[c] = ok ? kin[i] : 0;
        if (BUILD) k[c] = (k[c] & 0xFFFFFFFF00000000ull) | (uint64_t)(uint32_t)i;
        const uint32_t d = (uint32_t)(k[c] >> shift) & 255u;
        const uint64_t peers = digit_peers(d, __ballot(ok));
        const uint32_t before = wc[wave][d];
        __builtin_amdgcn_wave_barrier();
        if (ok && (peers & below) == 0) wc[wave][d] = before + (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
        dr[c] = (d << 16) | (before + (uint32_t)__popcll(peers & below));
    }
    __syncthreads();
    {
        const int d = threadIdx.x;  // one digit per thread
        uint32_t cw[RS_WAVES], tot = 0;
        for (int w = 0; w < RS_WAVES; w++) {
            cw[w] = wc[w][d];
            tot += cw[w];
        }
        const uint32_t tb = block_exclusive_scan_256(tot, tmp);  // tile-local start of digit d
        gbase[d] = off[(int64_t)d * ntiles + tile] - tb;  // modulo 2^32
        uint32_t acc = tb;
        for (int w = 0; w < RS_WAVES; w++) {
            wc[w][d] = acc;
            acc += cw[w];
        }
    }
    __syncthreads();
    uint32_t li_of[RS_ITEMS];
#pragma unroll
    for (int c = 0; c < RS_ITEMS; c++) {
        const int64_t i = base + (int64_t)c * 64 + lane;
        li_of[c] = wc[wave][dr[c] >> 16] + (dr[c] & 0xFFFFu);
        if (i < n) sk[li_of[c]] = k[c];
    }
    if (HASV) {  // payload loads in flight while the keys are written
#pragma unroll
        for (int c = 0; c < RS_ITEMS; c++) {
            const int64_t i = base + (int64_t)c * 64 + lane;
            v[HASV ? c : 0] = i < n ? vin[i] : 0;
        }
    }
    __syncthreads();
    const int cnt = (int)min<int64_t>(RS_TILE, n - tile0);
    uint32_t pos[RS_ITEMS];
#pragma unroll
    for (int j = 0; j < RS_ITEMS; j++) {
        const int li = threadIdx.x + j * RS_THREADS;
        if (li < cnt) {
            const uint64_t key = sk[li];
            pos[j] = gbase[(uint32_t)(key >> shift) & 255u] + (uint32_t)li;
            kout[pos[j]] = key;
        }
    }
    if (!HASV) return;
    __syncthreads();  // every key read from the buffer before payloads overwrite it
#pragma unroll
    for (int c = 0; c < RS_ITEMS; c++) {
        const int64_t i = base + (int64_t)c * 64 + lane;
        if (i < n) sk[li_of[c]] = v[HASV ? c : 0];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < RS_ITEMS; j++) {
        const int li = threadIdx.x + j * RS_THREADS;
        if (li < cnt) vout[pos[j]] = sk[li];
    }
}

void radix_sort(uint64_t *key, uint64_t *val, int64_t n, uint64_t key_mask, Workspace &ws,
                hipStream_t s, const int64_t *n_dev, uint64_t *k2, uint64_t *v2,
                uint64_t **sorted_keys) {
    if (sorted_keys) {
        if (val) throw Error(MJ_EINVAL, "radix_sort: sorted_keys is for keys only");
        *sorted_keys = key;
    }
    if (n <= 1) return;
    if (n > 0xFFFFFFF0LL) throw Error(MJ_ECAPACITY, "sort of more than 2^32 elements");
    int passes[8], np = 0;
    for (int p = 0; p < 8; p++)
        if ((key_mask >> (8 * p)) & 0xFFu) passes[np++] = p;
    if (np == 0) return;
    const int64_t ntiles = (n + RS_TILE - 1) / RS_TILE;
    if (ntiles > 0x7FFFFFFFLL || 256 * ntiles > 0xFFFFFFF0LL)
        throw Error(MJ_ECAPACITY, "radix_sort: too many tiles");
    uint32_t *cnt = ws.get_n<uint32_t>(256 * ntiles + 1);
    uint32_t *off = ws.get_n<uint32_t>(256 * ntiles + 1);
    if (!k2) k2 = ws.get_n<uint64_t>(n);
    if (val && !v2) v2 = ws.get_n<uint64_t>(n);
    uint64_t *ka = key, *va = val, *kb = k2, *vb = v2;
    for (int t = 0; t < np; t++) {
        const int shift = 8 * passes[t];
        hipLaunchKernelGGL(k_rs_tile_counts, dim3((unsigned)ntiles), dim3(RS_THREADS), 0, s, ka, n,
                           shift, ntiles, cnt, n_dev);
        MJ_LAUNCH_CHECK();
        exclusive_scan_u32(cnt, off, 256 * ntiles, ws, s);
        if (val)
            hipLaunchKernelGGL(k_rs_scatter<true>, dim3((unsigned)ntiles), dim3(RS_THREADS), 0, s,
                               ka, va, kb, vb, n, shift, ntiles, off, n_dev);
        else
            hipLaunchKernelGGL(k_rs_scatter<false>, dim3((unsigned)ntiles), dim3(RS_THREADS), 0, s,
                               ka, nullptr, kb, nullptr, n, shift, ntiles, off, n_dev);
        MJ_LAUNCH_CHECK();
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (ka != key) {
        if (sorted_keys) {
            *sorted_keys = ka;
            return;
        }
        MJ_HIP(hipMemcpyAsync(key, ka, (size_t)n * 8, hipMemcpyDeviceToDevice, s));
        if (val) MJ_HIP(hipMemcpyAsync(val, va, (size_t)n * 8, hipMemcpyDeviceToDevice, s));
    }
}

// ---------------------------------------------------------------- record sort
// Records sorted by full 64-bit key with four radix passes: a stable sort by the top 32
// bits, then a repair of the runs of equal top halves that hold more than one key.  Such
// runs are rare (about n^2 / 2^33 pairs of keys share a top half).  k_run_bits marks, one
// bit per record, where a run starts and where the key changes inside a run; k_mixed_runs
// (read-only) lets the first change of each run record the run's bounds, found by
// scanning those bitmaps 64 records per step; k_sort_runs_short and k_sort_runs_long
// then order each listed run by the full key (insertion sort, a thread per short run and
// a wave per long one: a run that holds a frequent key has few inversions).  The run list
// is split into RUN_SEGS segments, segment j taking the runs whose first change lies in
// its share of bitmap words, each with a counter on a line of its own (device-scope
// atomics on one address serialise: 64 segments left the repair at 0.9 ms on 78 M text
// records, 1,024 took 0.4 ms off the sort).  Two runs are disjoint and hold two records
// each around their first change, so W words of 64 positions hold at most 32 W + 1 first
// changes: a segment can never overflow.
constexpr int RUN_SEGS = 1024;
constexpr int RUN_CSTRIDE = 64;  // uint64 words between two segment counters
__global__ void k_run_bits(const uint64_t *__restrict__ key, int64_t n, uint64_t *__restrict__ rsb,
                           uint64_t *__restrict__ brb, const int64_t *__restrict__ n_dev) {
    if (n_dev) n = min(n, *n_dev);
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;  // a multiple of 64
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i - lane < n; i += stride) {
        const bool ok = i < n;
        const uint64_t b = ok ? key[i] : 0, a = (ok && i > 0) ? key[i - 1] : 0;
        const bool same_top = i > 0 && (a >> 32) == (b >> 32);
        const uint64_t ms = __ballot(ok && !same_top);
        const uint64_t mb = __ballot(ok && same_top && a != b);
        if (lane == 0) {
            rsb[i >> 6] = ms;
            brb[i >> 6] = mb;
        }
    }
}

__global__ void k_mixed_runs(const uint64_t *__restrict__ rsb, const uint64_t *__restrict__ brb,
                             int64_t n, int64_t seg_words, int64_t *runs, int64_t seg_cap,
                             unsigned long long *count, const int64_t *__restrict__ n_dev) {
    if (n_dev) n = min(n, *n_dev);
    const int64_t nw = (n + 63) >> 6;
    for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < nw;
         w += (int64_t)gridDim.x * blockDim.x) {
        uint64_t bits = brb[w];
        const int64_t seg = w / seg_words;
        while (bits) {
            const int b = __ffsll((unsigned long long)bits) - 1;
            bits &= bits - 1;
            const int64_t i = 64 * w + b;  // key[i-1] != key[i], same top half
            // run start: the last run-start bit at or before i-1 (position 0 always is one)
            int64_t pw = (i - 1) >> 6;
            uint64_t m = rsb[pw] & (~0ull >> (63 - ((i - 1) & 63)));
            while (m == 0) m = rsb[--pw];
            const int64_t rs = 64 * pw + 63 - __clzll((long long)m);
            // the run's first change owns it: no change bit in (rs, i)
            bool first = true;
            if (i - 1 > rs) {
                int64_t qw = (i - 1) >> 6;
                uint64_t mq = brb[qw] & (~0ull >> (63 - ((i - 1) & 63)));
                for (;;) {
                    const int64_t lo = 64 * qw;
                    if (rs + 1 > lo) mq &= ~0ull << (rs + 1 - lo);
                    if (mq) {
                        first = false;
                        break;
                    }
                    if (lo <= rs + 1) break;
                    mq = brb[--qw];
                }
            }
            if (!first) continue;
            // run end: the next run-start bit after i, else n
            int64_t ew = (i + 1) >> 6, re = n;
            if (i + 1 < n) {
                uint64_t me = rsb[ew] & (~0ull << ((i + 1) & 63));
                while (me == 0 && ++ew < nw) me = rsb[ew];
                if (me) re = min(n, 64 * ew + (__ffsll((unsigned long long)me) - 1));
            }
            const unsigned long long slot = atomicAdd(count + seg * RUN_CSTRIDE, 1ull);
            if ((int64_t)slot < seg_cap) {
                int64_t *r = runs + 2 * (seg * seg_cap + (int64_t)slot);
                r[0] = rs;
                r[1] = re;
            }
        }
    }
}

constexpr int64_t RUN_SHORT = 64;

// grid.y = segment; one thread per run of at most RUN_SHORT records
__global__ void k_sort_runs_short(uint64_t *__restrict__ key, uint64_t *__restrict__ val,
                            const int64_t *__restrict__ runs, int64_t seg_cap,
                            const unsigned long long *count) {
    const int64_t seg = blockIdx.y;
    const int64_t nr = min((int64_t)count[seg * RUN_CSTRIDE], seg_cap);
    const int64_t *sr = runs + 2 * seg * seg_cap;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nr;
         r += (int64_t)gridDim.x * blockDim.x) {
        const int64_t rs = sr[2 * r], re = sr[2 * r + 1];
        if (re - rs > RUN_SHORT) continue;  // k_sort_runs_long's
        // Mixed runs are mostly one frequent key and a rare colliding one, so nearly every
        // record is already in place.  The largest key of the sorted prefix stays in a
        // register and keys are loaded RS_FIX at a time (all in flight together): an
        // insertion at position j writes only positions <= j, so the keys loaded beyond j
        // are still current.
        constexpr int RS_FIX = 16;
        uint64_t top = key[rs];
        for (int64_t j0 = rs + 1; j0 < re; j0 += RS_FIX) {
            const int cnt = (int)min<int64_t>(RS_FIX, re - j0);
            uint64_t kc[RS_FIX];
#pragma unroll
            for (int c = 0; c < RS_FIX; c++) kc[c] = c < cnt ? key[j0 + c] : 0;
#pragma unroll
            for (int c = 0; c < RS_FIX; c++) {
                if (c >= cnt) break;
                const uint64_t k = kc[c];
                if (k >= top) {  // in place (equal keys keep their order)
                    top = k;
                    continue;
                }
                int64_t p = j0 + c;
                const uint64_t v = val[p];
                while (p > rs && key[p - 1] > k) {
                    key[p] = key[p - 1];
                    val[p] = val[p - 1];
                    p--;
                }
                key[p] = k;
                val[p] = v;
            }
        }
    }
}

// grid.y = segment; one wave per run of more than RUN_SHORT records.  The records of a
// run share the key's top half, and a mixed run is mostly one frequent key and a few
// colliding ones, met in any order: the wave sorts it by counting.  Pass 1 lists the
// run's distinct keys (at most RUN_KEYS) in LDS and counts each; their order gives each
// key's first position; pass 2 writes every record to its position in the scratch arrays
// (ranks among equal keys of 64 records from ballots, so equal keys keep their order);
// pass 3 copies the run back.  A run with more distinct keys is insertion-sorted instead
// (k_insert_run).
constexpr int RUN_KEYS = 64;

__device__ void k_insert_run(uint64_t *__restrict__ key, uint64_t *__restrict__ val, int64_t rs,
                             int64_t re, int lane) {
    // Keys below the largest key before them (a max-scan over the lanes, seeded with the
    // sorted prefix's largest key) are inserted into the sorted prefix: a binary search for
    // the place, then the wave moves the keys between the place and the old position up
    // by one, 64 at a time from the top (a chunk's loads complete before its stores, and
    // each chunk writes only above the next chunk's range).  An insertion writes only
    // positions <= its old one, so the keys held for later lanes stay current.
    uint64_t top = key[rs];
    for (int64_t j0 = rs + 1; j0 < re; j0 += 64) {
        const bool ok = j0 + lane < re;
        const uint64_t k = ok ? key[j0 + lane] : 0;
        uint64_t incl = k;  // largest key of lanes <= this one
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint64_t o = shfl_up_t(incl, d);
            if (lane >= d) incl = o > incl ? o : incl;
        }
        uint64_t before = shfl_up_t(incl, 1);
        if (lane == 0) before = 0;
        if (top > before) before = top;
        uint64_t bad = __ballot(ok && k < before);
        const uint64_t cmax = (uint64_t)__shfl((long long)incl, 63, 64);
        while (bad) {
            const int b = __ffsll((unsigned long long)bad) - 1;
            bad &= bad - 1;
            const int64_t jb = j0 + b;
            const uint64_t kb = (uint64_t)__shfl((long long)k, b, 64);
            const uint64_t vb = val[jb];
            int64_t a = rs, z = jb;  // the place: the first key of the prefix above kb
            while (a < z) {
                const int64_t mid = (a + z) >> 1;
                if (key[mid] <= kb) a = mid + 1;
                else z = mid;
            }
            for (int64_t hi = jb; hi > a; hi -= 64) {
                const int64_t lo = max(a, hi - 64), i = lo + lane;
                uint64_t kk = 0, vv = 0;
                if (i < hi) {
                    kk = key[i];
                    vv = val[i];
                }
                if (i < hi) {
                    key[i + 1] = kk;
                    val[i + 1] = vv;
                }
            }
            if (lane == 0) {
                key[a] = kb;
                val[a] = vb;
            }
            __threadfence_block();  // the moves complete before the next search
        }
        if (cmax > top) top = cmax;
    }
}

__global__ __launch_bounds__(256) void k_sort_runs_long(uint64_t *__restrict__ key,
                                                        uint64_t *__restrict__ val,
                                                        uint64_t *__restrict__ tk,
                                                        uint64_t *__restrict__ tv,
                                                        const int64_t *__restrict__ runs,
                                                        int64_t seg_cap,
                                                        const unsigned long long *count) {
    __shared__ uint64_t tkey[4][RUN_KEYS];
    __shared__ uint32_t tcnt[4][RUN_KEYS];
    const int64_t seg = blockIdx.y;
    const int64_t nr = min((int64_t)count[seg * RUN_CSTRIDE], seg_cap);
    const int64_t *sr = runs + 2 * seg * seg_cap;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint64_t below = lanes_below();
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    // the wave reads 64 runs' bounds at a time and takes the long ones among them
    for (int64_t r0 = (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * 64; r0 < nr;
         r0 += nwaves * 64) {
        const int64_t rl = r0 + lane;
        const int64_t rs_l = rl < nr ? sr[2 * rl] : 0, re_l = rl < nr ? sr[2 * rl + 1] : 0;
        for (uint64_t longs = __ballot(re_l - rs_l > RUN_SHORT); longs; longs &= longs - 1) {
            const int src = __ffsll((unsigned long long)longs) - 1;
            const int64_t rs = __shfl((long long)rs_l, src, 64), re = __shfl((long long)re_l, src, 64);
            // the index of key k in the table of nd distinct keys, or -1
            auto find = [&](uint64_t k, int nd) {
                int idx = -1;
                for (int t = 0; t < nd; t++)
                    if (tkey[wv][t] == k) idx = t;
                return idx;
            };
            tcnt[wv][lane] = 0;
            __builtin_amdgcn_wave_barrier();
            int nd = 0;  // pass 1: the distinct keys and their counts
            bool over = false;
            for (int64_t s0 = rs; s0 < re && !over; s0 += 64) {
                const bool ok = s0 + lane < re;
                const uint64_t k = ok ? key[s0 + lane] : 0;
                int idx = ok ? find(k, nd) : 0;
                for (uint64_t un = __ballot(idx < 0); un; un = __ballot(idx < 0)) {
                    if (nd == RUN_KEYS) {
                        over = true;
                        break;
                    }
                    const uint64_t nk = (uint64_t)__shfl((long long)k, __ffsll((unsigned long long)un) - 1, 64);
                    if (lane == 0) tkey[wv][nd] = nk;
                    __builtin_amdgcn_wave_barrier();
                    if (idx < 0 && k == nk) idx = nd;
                    nd++;
                }
                if (over) break;
                const uint64_t peers = digit_peers((uint32_t)idx, __ballot(ok));
                if (ok && (peers & below) == 0) tcnt[wv][idx] += (uint32_t)__popcll(peers);
                __builtin_amdgcn_wave_barrier();
            }
            if (over) {
                k_insert_run(key, val, rs, re, lane);
                continue;
            }
            // each key's first position: the counts of the smaller keys
            const uint64_t mk = lane < nd ? tkey[wv][lane] : ~0ull;
            const uint32_t mc = lane < nd ? tcnt[wv][lane] : 0u;
            uint32_t first = 0;
            for (int t = 0; t < nd; t++) {
                const uint64_t ok2 = (uint64_t)__shfl((long long)mk, t, 64);
                const uint32_t c = (uint32_t)__shfl((int)mc, t, 64);
                if (ok2 < mk) first += c;
            }
            __builtin_amdgcn_wave_barrier();
            if (lane < nd) tcnt[wv][lane] = first;
            __builtin_amdgcn_wave_barrier();
            for (int64_t s0 = rs; s0 < re; s0 += 64) {  // pass 2: records to their places
                const bool ok = s0 + lane < re;
                const uint64_t k = ok ? key[s0 + lane] : 0, v = ok ? val[s0 + lane] : 0;
                const int idx = ok ? find(k, nd) : 0;
                const uint64_t peers = digit_peers((uint32_t)idx, __ballot(ok));
                const uint32_t base = tcnt[wv][idx];
                __builtin_amdgcn_wave_barrier();
                if (ok) {
                    const int64_t pos = rs + base + (uint32_t)__popcll(peers & below);
                    tk[pos] = k;
                    tv[pos] = v;
                }
                if (ok && (peers & below) == 0) tcnt[wv][idx] = base + (uint32_t)__popcll(peers);
                __builtin_amdgcn_wave_barrier();
            }
            __threadfence_block();  // the scratch writes complete before other lanes read them
            for (int64_t j = rs + lane; j < re; j += 64) {  // pass 3: back
                key[j] = tk[j];
                val[j] = tv[j];
            }
            __threadfence_block();
        }
    }
}

void sort_records(uint64_t *key, uint64_t *val, int64_t n, Workspace &ws, hipStream_t s,
                  uint64_t *host_scratch, const int64_t *n_dev) {
    if (n <= 1) return;
    // the radix sort's second buffers, then the long-run repair's
    uint64_t *k2 = ws.get_n<uint64_t>(n), *v2 = ws.get_n<uint64_t>(n);
    radix_sort(key, val, n, 0xFFFFFFFF00000000ull, ws, s, n_dev, k2, v2);
    const int64_t nw = (n + 63) / 64;
    const int64_t seg_words = (nw + RUN_SEGS - 1) / RUN_SEGS;
    const int64_t seg_cap = 32 * seg_words + 1;  // first changes a segment can hold
    int64_t *runs = ws.get_n<int64_t>(2 * RUN_SEGS * seg_cap);
    uint64_t *rsb = ws.get_n<uint64_t>(nw + 1);
    uint64_t *brb = ws.get_n<uint64_t>(nw + 1);
    unsigned long long *count = (unsigned long long *)ws.get_n<uint64_t>(RUN_SEGS * RUN_CSTRIDE);
    fill_u64((uint64_t *)count, 0, RUN_SEGS * RUN_CSTRIDE, s);
    hipLaunchKernelGGL(k_run_bits, dim3(grid_for(n, 256, 16384)), dim3(256), 0, s, key, n, rsb, brb,
                       n_dev);
    MJ_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_mixed_runs, dim3(grid_for(nw, 256, 16384)), dim3(256), 0, s, rsb, brb, n,
                       seg_words, runs, seg_cap, count, n_dev);
    MJ_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sort_runs_short, dim3(4, RUN_SEGS), dim3(256), 0, s, key, val, runs, seg_cap,
                       count);
    MJ_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sort_runs_long, dim3(1, RUN_SEGS), dim3(256), 0, s, key, val, k2, v2, runs,
                       seg_cap, count);
    MJ_LAUNCH_CHECK();
    (void)host_scratch;
}

// ---------------------------------------------------------------- group members
// Only records whose key occurs at least twice can form a group (Alg. 3 pairs records of
// equal key); on the large workloads they are 5-25% of all records.  The filter keeps a
// superset of them -- every record whose key's top half occurs twice -- without sorting the
// full records:
//  1. two radix passes over narrow elements (top half of the key << 32 | record index,
//     built by the first pass from the keys) order them by the key's top 16 bits, which
//     puts each "bucket" of equal top 16 bits in one contiguous range;
//  2. k_mb_bounds finds each bucket's range (a binary search per bucket), and k_mb_flags
//     gives each bucket one workgroup with two LDS bitmaps over the next 16 bits (seen /
//     seen again), flagging the records whose key's top half was seen again in a byte
//     array indexed by record (a bucket of more than `big` elements, default 2^16, is kept
//     whole, which only costs time);
//  3. the flagged records are compacted in record order and gathered: ascending reads of
//     the key and payload arrays (gathering them in bucket order read lines at random,
//     fetching 20 times the bytes kept).
// The kept records then go through the full record sort; any superset of the group
// members gives the same groups.
constexpr int MB_BUCKETS = 1 << 16;

__device__ __forceinline__ uint32_t mb_top16(uint64_t x) { return (uint32_t)(x >> 48); }

// bs[b] = the first index whose top 16 bits are >= b (b = 0..2^16; bs[2^16] = n): one
// binary search per thread over the sorted elements.  Every record flag (up to the
// capacity) is cleared on the way.
__global__ void k_mb_bounds(const uint64_t *__restrict__ w, int64_t cap, const int64_t *n_dev,
                            uint32_t *__restrict__ bs, uint8_t *__restrict__ flags) {
    const int64_t n = n_dev ? min(cap, *n_dev) : cap;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g <= MB_BUCKETS) {
        int64_t a = 0, z = n;
        while (a < z) {
            const int64_t mid = (a + z) >> 1;
            if (mb_top16(w[mid]) < (uint32_t)g) a = mid + 1;
            else z = mid;
        }
        bs[g] = (uint32_t)a;
    }
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = g; i < cap; i += stride) flags[i] = 0;
}

// One workgroup per bucket [bs[b], bs[b+1]): LDS bitmaps over bits 32..47 (seen / seen
// again); an element is kept when its bits were seen again, i.e. when its key's top half
// occurs twice, by setting its record's flag (flags are indexed by record: the element's
// low half).  A bucket of more than `big` elements is kept whole.
__global__ __launch_bounds__(256) void k_mb_flags(const uint64_t *__restrict__ w,
                                                  const uint32_t *__restrict__ bs, uint32_t big,
                                                  uint8_t *__restrict__ flags) {
    const uint32_t lo = bs[blockIdx.x], hi = bs[blockIdx.x + 1];
    if (hi - lo > big) {
        for (uint32_t i = lo + threadIdx.x; i < hi; i += 256) flags[(uint32_t)w[i]] = 1;
        return;
    }
    if (hi <= lo + 1) return;  // empty, or one element: not kept
    __shared__ uint32_t seen[2048], again[2048];
    for (int j = threadIdx.x; j < 2048; j += 256) {
        seen[j] = 0;
        again[j] = 0;
    }
    // a bucket of up to MB_KEEP * 256 elements is read once, its elements kept in registers
    // between the two sweeps (loads issued before the bitmaps are cleared)
    constexpr int MB_KEEP = 8;
    const bool keep = hi - lo <= MB_KEEP * 256;
    uint64_t x[MB_KEEP];
    if (keep) {
#pragma unroll
        for (int u = 0; u < MB_KEEP; u++) {
            const uint32_t i = lo + threadIdx.x + 256 * u;
            x[u] = i < hi ? w[i] : 0;
        }
    }
    __syncthreads();
    auto see = [&](uint64_t e) {
        const uint32_t sub = (uint32_t)(e >> 32) & 0xFFFFu, bit = 1u << (sub & 31);
        if (atomicOr(&seen[sub >> 5], bit) & bit) atomicOr(&again[sub >> 5], bit);
    };
    auto mark = [&](uint64_t e) {
        const uint32_t sub = (uint32_t)(e >> 32) & 0xFFFFu;
        if ((again[sub >> 5] >> (sub & 31)) & 1u) flags[(uint32_t)e] = 1;
    };
    if (keep) {
#pragma unroll
        for (int u = 0; u < MB_KEEP; u++)
            if (lo + threadIdx.x + 256 * u < hi) see(x[u]);
        __syncthreads();
#pragma unroll
        for (int u = 0; u < MB_KEEP; u++)
            if (lo + threadIdx.x + 256 * u < hi) mark(x[u]);
    } else {
        for (uint32_t i = lo + threadIdx.x; i < hi; i += 256) see(w[i]);
        __syncthreads();
        for (uint32_t i = lo + threadIdx.x; i < hi; i += 256) mark(w[i]);
    }
}

// mkey[j], mval[j] = the record of the j-th kept record (j < min(count, mcap)), idx
// holding kept record indices in ascending order; m_dev gets the count (which may exceed
// mcap: the caller checks).  Four records per thread, their loads issued together.
constexpr int MB_GATHER = 4;
__global__ void k_mb_gather(const int64_t *__restrict__ idx, const uint32_t *__restrict__ count,
                            const uint64_t *__restrict__ key, const uint64_t *__restrict__ val,
                            uint64_t *__restrict__ mkey, uint64_t *__restrict__ mval, int64_t mcap,
                            int64_t *m_dev) {
    const int64_t m = min((int64_t)*count, mcap);
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g == 0) *m_dev = (int64_t)*count;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j0 = g; j0 < m; j0 += stride * MB_GATHER) {
        int64_t r[MB_GATHER];
#pragma unroll
        for (int u = 0; u < MB_GATHER; u++) {
            const int64_t j = j0 + u * stride;
            r[u] = j < m ? idx[j] : 0;
        }
        uint64_t k[MB_GATHER], v[MB_GATHER];
#pragma unroll
        for (int u = 0; u < MB_GATHER; u++) {
            k[u] = key[r[u]];
            v[u] = val[r[u]];
        }
#pragma unroll
        for (int u = 0; u < MB_GATHER; u++) {
            const int64_t j = j0 + u * stride;
            if (j < m) {
                mkey[j] = k[u];
                mval[j] = v[u];
            }
        }
    }
}

static void mb_radix_pass(const uint64_t *kin, uint64_t *kout, int64_t n, int shift, bool build,
                          Workspace &ws, hipStream_t s, const int64_t *n_dev) {
    const int64_t ntiles = (n + RS_TILE - 1) / RS_TILE;
    uint32_t *cnt = ws.get_n<uint32_t>(256 * ntiles + 1);
    uint32_t *off = ws.get_n<uint32_t>(256 * ntiles + 1);
    hipLaunchKernelGGL(k_rs_tile_counts, dim3((unsigned)ntiles), dim3(RS_THREADS), 0, s, kin, n,
                       shift, ntiles, cnt, n_dev);
    MJ_LAUNCH_CHECK();
    exclusive_scan_u32(cnt, off, 256 * ntiles, ws, s);
    if (build)
        hipLaunchKernelGGL((k_rs_scatter<false, true>), dim3((unsigned)ntiles), dim3(RS_THREADS), 0,
                           s, kin, nullptr, kout, nullptr, n, shift, ntiles, off, n_dev);
    else
        hipLaunchKernelGGL((k_rs_scatter<false, false>), dim3((unsigned)ntiles), dim3(RS_THREADS), 0,
                           s, kin, nullptr, kout, nullptr, n, shift, ntiles, off, n_dev);
    MJ_LAUNCH_CHECK();
}

void group_members(const uint64_t *key, const uint64_t *val, int64_t n, const int64_t *n_dev,
                   uint64_t *mkey, uint64_t *mval, int64_t mcap, int64_t *m_dev, uint32_t big,
                   Workspace &ws, hipStream_t s) {
    if (big < 1) throw Error(MJ_EINVAL, "member filter bucket limit must be >= 1");
    if (n > 0xFFFFFFF0LL) throw Error(MJ_ECAPACITY, "member filter of more than 2^32 records");
    if (n <= 0) {
        fill_u64(reinterpret_cast<uint64_t *>(m_dev), 0, 1, s);
        return;
    }
    const int64_t ntiles = (n + RS_TILE - 1) / RS_TILE;
    if (ntiles > 0x7FFFFFFFLL || 256 * ntiles > 0xFFFFFFF0LL)
        throw Error(MJ_ECAPACITY, "member filter: too many tiles");
    uint64_t *w1 = ws.get_n<uint64_t>(n + 1);
    uint64_t *w2 = ws.get_n<uint64_t>(n + 1);
    mb_radix_pass(key, w1, n, 48, true, ws, s, n_dev);
    mb_radix_pass(w1, w2, n, 56, false, ws, s, n_dev);
    uint8_t *flags = ws.get_n<uint8_t>(n + 16);
    uint32_t *bs = ws.get_n<uint32_t>(MB_BUCKETS + 1);
    hipLaunchKernelGGL(k_mb_bounds, dim3(grid_for(std::max<int64_t>(n, MB_BUCKETS + 1), 256, 16384)),
                       dim3(256), 0, s, w2, n, n_dev, bs, flags);
    MJ_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_mb_flags, dim3(MB_BUCKETS), dim3(256), 0, s, w2, bs, big, flags);
    MJ_LAUNCH_CHECK();
    int64_t *idx = ws.get_n<int64_t>(n + 1);
    const uint32_t *count = compact_flags_async(flags, n, idx, ws, s);
    hipLaunchKernelGGL(k_mb_gather, dim3(grid_for((std::min(n, mcap) + MB_GATHER - 1) / MB_GATHER, 256, 16384)),
                       dim3(256), 0, s, idx, count, key, val, mkey, mval, mcap, m_dev);
    MJ_LAUNCH_CHECK();
}

}  // namespace mj
