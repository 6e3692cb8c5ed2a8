// Device primitives: fills, exclusive scans, stream compaction and a bucketed
// (key, value) sort.  All loops are bounds-checked; grids come from host-known sizes.
#include <string.h>

#include <algorithm>

#include "mj_common.h"

namespace mj {

// ---------------------------------------------------------------- workspace / alloc
Workspace::~Workspace() {
    for (auto &b : blocks_) (void)hipFree(b.p);
}

void *Workspace::get(size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    Block *best = nullptr;
    for (auto &b : blocks_)
        if (!b.used && b.n >= bytes && (!best || b.n < best->n)) best = &b;
    if (best && best->n <= 4 * bytes + (1 << 20)) {
        best->used = true;
        return best->p;
    }
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        // free idle blocks and retry once
        for (auto it = blocks_.begin(); it != blocks_.end();) {
            if (!it->used) { (void)hipFree(it->p); held_ -= it->n; it = blocks_.erase(it); }
            else ++it;
        }
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            throw Error(MJ_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
        }
    }
    blocks_.push_back({p, bytes, true});
    held_ += bytes;
    return p;
}

void Workspace::release_all() {
    for (auto &b : blocks_) b.used = false;
}

void *dev_alloc(size_t bytes) {
    void *p = nullptr;
    if (bytes == 0) bytes = 16;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        throw Error(MJ_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    return p;
}

void dev_free(void *p) {
    if (p) (void)hipFree(p);
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

void KTimer::end(int h, hipStream_t s) {
    if (h >= 0) MJ_HIP(hipEventRecord(ev[h + 1], s));
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
        launches[slot_of[h / 2]] += 1;
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

template <class In, class T>
__global__ void k_scan_reduce(const In *in, int64_t n, T *partial) {
    __shared__ T smem[8];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    T s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; k++)
        if (base + k < n) s += (T)in[base + k];
    T tot;
    (void)block_exclusive_scan<T>(s, smem, &tot);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

template <class In, class T>
__global__ void k_scan_apply(const In *in, int64_t n, const T *partial_scan, T *out) {
    __shared__ T smem[8];
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
    if (last >= base && last < base + SCAN_ITEMS) out[n] = run;
}

template <class In, class T>
static void scan_impl(const In *in, T *out, int64_t n, Workspace &ws, hipStream_t s) {
    if (n <= 0) {
        hipLaunchKernelGGL(k_fill<T>, dim3(1), dim3(64), 0, s, out, (T)0, (int64_t)1);
        MJ_LAUNCH_CHECK();
        return;
    }
    int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb == 1) {
        hipLaunchKernelGGL((k_scan_apply<In, T>), dim3(1), dim3(SCAN_BLOCK), 0, s, in, n,
                           (const T *)nullptr, out);
        MJ_LAUNCH_CHECK();
        return;
    }
    if (nb > 2147483647LL) throw Error(MJ_ECAPACITY, "scan too large");
    T *partial = ws.get_n<T>(nb + 1);
    T *pscan = ws.get_n<T>(nb + 1);
    hipLaunchKernelGGL((k_scan_reduce<In, T>), dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, in, n,
                       partial);
    MJ_LAUNCH_CHECK();
    scan_impl<T, T>(partial, pscan, nb, ws, s);
    hipLaunchKernelGGL((k_scan_apply<In, T>), dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, in, n,
                       (const T *)pscan, out);
    MJ_LAUNCH_CHECK();
}

void exclusive_scan_u32(const uint32_t *in, uint32_t *out, int64_t n, Workspace &ws, hipStream_t s) {
    scan_impl<uint32_t, uint32_t>(in, out, n, ws, s);
}
void exclusive_scan_u64(const uint64_t *in, uint64_t *out, int64_t n, Workspace &ws, hipStream_t s) {
    scan_impl<uint64_t, uint64_t>(in, out, n, ws, s);
}

// ---------------------------------------------------------------- compaction
__global__ void k_compact_scatter(const uint8_t *flags, const uint32_t *pre, int64_t n,
                                  int64_t *idx) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride)
        if (flags[i]) idx[pre[i]] = i;
}

int64_t compact_flags(const uint8_t *flags, int64_t n, int64_t *idx_out, Workspace &ws,
                      hipStream_t s, uint64_t *host_scratch) {
    if (n <= 0) return 0;
    // 32-bit ranks: the count of kept elements must stay below 2^32
    if (n > 0xFFFFFFF0LL) throw Error(MJ_ECAPACITY, "compaction of more than 2^32 elements");
    uint32_t *pre = ws.get_n<uint32_t>(n + 1);
    scan_impl<uint8_t, uint32_t>(flags, pre, n, ws, s);
    hipLaunchKernelGGL(k_compact_scatter, dim3(grid_for(n, 256, 16384)), dim3(256), 0, s, flags,
                       pre, n, idx_out);
    MJ_LAUNCH_CHECK();
    return (int64_t)read_back<uint32_t>(pre + n, s, host_scratch);
}

__global__ void k_gather_u64(const uint64_t *src, const int64_t *idx, uint64_t *dst, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) dst[i] = src[idx[i]];
}

void gather_u64(const uint64_t *src, const int64_t *idx, uint64_t *dst, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_gather_u64, dim3(grid_for(n, 256, 16384)), dim3(256), 0, s, src, idx, dst, n);
    MJ_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- bucketed sort
// Pass 1 histograms buckets (key >> shift), pass 2 scatters into bucket ranges of a
// temporary array, pass 3 sorts each bucket in LDS (or, for buckets above LDS capacity,
// in global memory by one workgroup) and writes it back in place.  The result is
// ordered by (key, val) and does not depend on the scatter order.
constexpr int LOCAL_MAX = 2048;

template <bool HASV>
__global__ void k_bucket_hist(const uint64_t *key, int64_t n, int shift, uint32_t *cnt) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) atomicAdd(&cnt[key[i] >> shift], 1u);
}

template <bool HASV>
__global__ void k_bucket_scatter(const uint64_t *key, const uint64_t *val, int64_t n, int shift,
                                 const uint32_t *boff, uint32_t *fill, uint64_t *k2, uint64_t *v2) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) {
        uint64_t k = key[i];
        uint64_t b = k >> shift;
        uint32_t p = boff[b] + atomicAdd(&fill[b], 1u);
        k2[p] = k;
        if (HASV) v2[p] = val[i];
    }
}

__device__ __forceinline__ bool greater_kv(uint64_t ka, uint64_t va, uint64_t kb, uint64_t vb) {
    return ka > kb || (ka == kb && va > vb);
}

template <bool HASV>
__global__ __launch_bounds__(256) void k_bucket_local_sort(const uint32_t *boff, int64_t nb,
                                                           const uint64_t *k2, const uint64_t *v2,
                                                           uint64_t *key, uint64_t *val,
                                                           uint32_t *big, uint32_t *nbig) {
    __shared__ uint64_t sk[LOCAL_MAX];
    __shared__ uint64_t sv[HASV ? LOCAL_MAX : 1];
    for (int64_t b = blockIdx.x; b < nb; b += gridDim.x) {
        uint32_t start = boff[b], end = boff[b + 1];
        uint32_t sz = end - start;
        if (sz == 0) continue;
        if (sz > (uint32_t)LOCAL_MAX) {
            if (threadIdx.x == 0) {
                uint32_t slot = atomicAdd(nbig, 1u);
                big[slot] = (uint32_t)b;
            }
            continue;
        }
        for (uint32_t i = threadIdx.x; i < sz; i += blockDim.x) {
            sk[i] = k2[start + i];
            if (HASV) sv[i] = v2[start + i];
        }
        __syncthreads();
        uint32_t p2 = 1;
        while (p2 < sz) p2 <<= 1;
        for (uint32_t k = 2; k <= p2; k <<= 1) {
            // mirror step, then half-cleaners; the smaller element always goes low
            for (uint32_t i = threadIdx.x; i < p2 / 2; i += blockDim.x) {
                uint32_t half = k >> 1;
                uint32_t lo = (i / half) * k + (i % half);
                uint32_t hi = lo ^ (k - 1);
                if (hi < sz) {
                    uint64_t a = sk[lo], c = sk[hi];
                    uint64_t av = HASV ? sv[lo] : 0, cv = HASV ? sv[hi] : 0;
                    if (greater_kv(a, av, c, cv)) {
                        sk[lo] = c; sk[hi] = a;
                        if (HASV) { sv[lo] = cv; sv[hi] = av; }
                    }
                }
            }
            __syncthreads();
            for (uint32_t j = k >> 2; j >= 1; j >>= 1) {
                for (uint32_t i = threadIdx.x; i < p2 / 2; i += blockDim.x) {
                    uint32_t lo = (i / j) * (2 * j) + (i % j);
                    uint32_t hi = lo + j;
                    if (hi < sz) {
                        uint64_t a = sk[lo], c = sk[hi];
                        uint64_t av = HASV ? sv[lo] : 0, cv = HASV ? sv[hi] : 0;
                        if (greater_kv(a, av, c, cv)) {
                            sk[lo] = c; sk[hi] = a;
                            if (HASV) { sv[lo] = cv; sv[hi] = av; }
                        }
                    }
                }
                __syncthreads();
            }
        }
        for (uint32_t i = threadIdx.x; i < sz; i += blockDim.x) {
            key[start + i] = sk[i];
            if (HASV) val[start + i] = sv[i];
        }
        __syncthreads();
    }
}

// Buckets larger than LDS: the same network in global memory, one workgroup each.
template <bool HASV>
__global__ __launch_bounds__(1024) void k_bucket_big_sort(const uint32_t *boff, const uint32_t *big,
                                                          const uint32_t *nbig, uint64_t *k2,
                                                          uint64_t *v2, uint64_t *key,
                                                          uint64_t *val) {
    uint32_t count = *nbig;
    for (uint32_t t = blockIdx.x; t < count; t += gridDim.x) {
        uint32_t b = big[t];
        uint32_t start = boff[b], sz = boff[b + 1] - start;
        uint64_t *sk = k2 + start;
        uint64_t *sv = HASV ? v2 + start : nullptr;
        uint32_t p2 = 1;
        while (p2 < sz) p2 <<= 1;
        for (uint32_t k = 2; k <= p2; k <<= 1) {
            for (uint32_t i = threadIdx.x; i < p2 / 2; i += blockDim.x) {
                uint32_t half = k >> 1;
                uint32_t lo = (i / half) * k + (i % half);
                uint32_t hi = lo ^ (k - 1);
                if (hi < sz) {
                    uint64_t a = sk[lo], c = sk[hi];
                    uint64_t av = HASV ? sv[lo] : 0, cv = HASV ? sv[hi] : 0;
                    if (greater_kv(a, av, c, cv)) {
                        sk[lo] = c; sk[hi] = a;
                        if (HASV) { sv[lo] = cv; sv[hi] = av; }
                    }
                }
            }
            __syncthreads();
            for (uint32_t j = k >> 2; j >= 1; j >>= 1) {
                for (uint32_t i = threadIdx.x; i < p2 / 2; i += blockDim.x) {
                    uint32_t lo = (i / j) * (2 * j) + (i % j);
                    uint32_t hi = lo + j;
                    if (hi < sz) {
                        uint64_t a = sk[lo], c = sk[hi];
                        uint64_t av = HASV ? sv[lo] : 0, cv = HASV ? sv[hi] : 0;
                        if (greater_kv(a, av, c, cv)) {
                            sk[lo] = c; sk[hi] = a;
                            if (HASV) { sv[lo] = cv; sv[hi] = av; }
                        }
                    }
                }
                __syncthreads();
            }
        }
        for (uint32_t i = threadIdx.x; i < sz; i += blockDim.x) {
            key[start + i] = sk[i];
            if (HASV) val[start + i] = sv[i];
        }
        __syncthreads();
    }
}

template <bool HASV>
static void sort_impl(uint64_t *key, uint64_t *val, int64_t n, int shift, int bucket_bits,
                      Workspace &ws, hipStream_t s) {
    if (n <= 1) return;
    if (n > 0xFFFFFFF0LL) throw Error(MJ_ECAPACITY, "sort of more than 2^32 elements");
    int64_t nb = 1LL << bucket_bits;
    uint32_t *cnt = ws.get_n<uint32_t>(nb + 1);
    uint32_t *boff = ws.get_n<uint32_t>(nb + 1);
    uint32_t *fillc = ws.get_n<uint32_t>(nb + 1);
    uint32_t *big = ws.get_n<uint32_t>(nb + 1);
    uint32_t *nbig = ws.get_n<uint32_t>(4);
    uint64_t *k2 = ws.get_n<uint64_t>(n);
    uint64_t *v2 = HASV ? ws.get_n<uint64_t>(n) : nullptr;
    fill_u32(cnt, 0, nb, s);
    fill_u32(fillc, 0, nb, s);
    fill_u32(nbig, 0, 1, s);
    unsigned g = grid_for(n, 256, 16384);
    hipLaunchKernelGGL(k_bucket_hist<HASV>, dim3(g), dim3(256), 0, s, key, n, shift, cnt);
    MJ_LAUNCH_CHECK();
    exclusive_scan_u32(cnt, boff, nb, ws, s);
    hipLaunchKernelGGL(k_bucket_scatter<HASV>, dim3(g), dim3(256), 0, s, key, val, n, shift, boff,
                       fillc, k2, v2);
    MJ_LAUNCH_CHECK();
    unsigned gl = (unsigned)std::min<int64_t>(nb, 1 << 16);
    hipLaunchKernelGGL(k_bucket_local_sort<HASV>, dim3(gl), dim3(256), 0, s, boff, nb, k2, v2, key,
                       val, big, nbig);
    MJ_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_bucket_big_sort<HASV>, dim3(64), dim3(1024), 0, s, boff, big, nbig, k2, v2,
                       key, val);
    MJ_LAUNCH_CHECK();
}

void sort_pairs(uint64_t *key, uint64_t *val, int64_t n, int shift, int bucket_bits,
                Workspace &ws, hipStream_t s) {
    if (bucket_bits < 1 || bucket_bits > 24 || shift < 0 || shift > 63)
        throw Error(MJ_EINVAL, "sort_pairs: bad bucket configuration");
    if (val)
        sort_impl<true>(key, val, n, shift, bucket_bits, ws, s);
    else
        sort_impl<false>(key, nullptr, n, shift, bucket_bits, ws, s);
}

}  // namespace mj
