// Partition stage: per-string parameters, bit-plane packing, anchors (Find-Anchor,
// Alg. 2) and partition records (Partition-String, Alg. 1, with the bucket key f of
// Alg. 3).
#include <string.h>

#include <algorithm>
#include <type_traits>
#include <vector>

#include "mj_common.h"

namespace mj {

static unsigned grid_for(int64_t n, int block, unsigned cap = 65535u) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    return (unsigned)std::min<int64_t>(g, cap);
}

// Largest s in [0, n) with off[s] <= g; for 0 <= g < off[n] that string is non-empty
// and contains position g.
__device__ __forceinline__ int32_t owner_of(const int64_t *off, int32_t n, int64_t g) {
    int32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        int32_t mid = (lo + hi) >> 1;
        if (off[mid] <= g) lo = mid; else hi = mid;
    }
    return lo;
}

// ---------------------------------------------------------------- per-string setup
// m_i, K_i, and r_i = max(1, floor((m - q + 1 - T) / (2T + 2))) with T from the rule of
// Remark 1 (Alg. 2 defines r).  The halo needed by the anchor kernel is the largest r
// of a string that has interior positions.
constexpr int32_t WIDE_R = 1920, WIDE_SENTINEL = 0x3FFFFFFF;
// Radii above WIDE_R take the wide path (a tile region holds at most 1,920 positions of
// halo on each side): such a string's radius in rr is WIDE_SENTINEL, which gives it no
// interior position in the tile kernel, and it is listed in wide_ids with its radius.
__global__ void k_prepare(const int64_t *off, int32_t n, int q, int64_t kuni, const int32_t *kps,
                          int t_div, int t_fixed, int32_t *len, int32_t *kk, int32_t *rr,
                          uint32_t *halo, uint32_t *err, unsigned long long *rec_bound,
                          uint32_t *kmax, int32_t *wide_ids, int32_t *wide_r, uint32_t *wide_count,
                          unsigned long long *wide_pos) {
    uint32_t hr = 0;  // the strings' contribution to the halo
    // and to the bound on the partitions of one repetition: interior anchors are strict
    // minima of radius r, so two of them are more than r apart, and a string of npos q-gram
    // starts has at most npos / (r + 1) + 2 partitions (one for m < q, none for m = 0)
    unsigned long long bnd = 0;
    uint32_t km = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        int64_t m = off[i + 1] - off[i];
        int64_t K = kuni >= 0 ? kuni : (int64_t)kps[i];
        if (m < 0 || m > 0x7FFFFFFFLL) atomicOr(err, 1u);
        if (K < 0) atomicOr(err, 2u);
        if (K > 0x3FFFFFFFLL) K = 0x3FFFFFFFLL;
        int64_t T = t_fixed > 0 ? (int64_t)t_fixed : (K + t_div - 1) / t_div;
        if (T < 1) T = 1;
        int64_t num = m - q + 1 - T;
        int64_t r = num <= 0 ? 1 : num / (2 * T + 2);
        if (r < 1) r = 1;
        int64_t npos = m - q + 1;
        bool wide = false;
        if (npos - 1 - r >= r) {  // the string has interior positions
            if (r > WIDE_R) {
                wide = true;
                const uint32_t w = atomicAdd(wide_count, 1u);
                wide_ids[w] = (int32_t)i;
                wide_r[w] = (int32_t)r;
                atomicAdd(wide_pos, (unsigned long long)npos);
            } else {
                hr = max(hr, (uint32_t)r);
            }
        }
        len[i] = (int32_t)m;
        kk[i] = (int32_t)(K < 0 ? 0 : K);
        rr[i] = wide ? WIDE_SENTINEL : (int32_t)std::min<int64_t>(r, 0x7FFFFFFFLL);
        if (m > 0) bnd += npos <= 0 ? 1ull : (unsigned long long)(npos / (r + 1) + 2);
        km = max(km, (uint32_t)(K < 0 ? 0 : K));
    }
    // one atomic per workgroup: device-scope atomics on one address serialise (a wave each
    // took 0.17 ms for 300,000 strings)
    for (int d = 32; d >= 1; d >>= 1) {
        hr = max(hr, (uint32_t)__shfl_xor((int)hr, d, 64));
        km = max(km, (uint32_t)__shfl_xor((int)km, d, 64));
        const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)bnd, d, 64);
        const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(bnd >> 32), d, 64);
        bnd += ((unsigned long long)hi << 32) | lo;
    }
    __shared__ uint32_t s_hr[4], s_km[4];
    __shared__ unsigned long long s_bnd[4];
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_hr[wv] = hr;
        s_km[wv] = km;
        s_bnd[wv] = bnd;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); w++) {
            hr = max(hr, s_hr[w]);
            km = max(km, s_km[w]);
            bnd += s_bnd[w];
        }
        if (hr) atomicMax(halo, hr);
        if (km) atomicMax(kmax, km);
        if (bnd) atomicAdd(rec_bound, bnd);
    }
}

void prepare_launch(DevStrings &d, const PartitionParams &p, Workspace &ws, hipStream_t s,
                    uint64_t *host_dst) {
    int32_t n = d.n;
    d.len = ws.get_n<int32_t>(n + 1);
    d.kk = ws.get_n<int32_t>(n + 1);
    d.rr = ws.get_n<int32_t>(n + 1);
    d.wide_ids = ws.get_n<int32_t>(n + 1);
    d.wide_r = ws.get_n<int32_t>(n + 1);
    // [0] halo, [1] error bits, [2..3] partition bound (u64), [4] largest K, [5] wide
    // strings, [6..7] their q-gram starts (u64)
    uint32_t *flags = ws.get_n<uint32_t>(8);
    fill_u32(flags, 0, 8, s);
    if (n > 0) {
        const unsigned grid = (unsigned)std::min<int64_t>(((int64_t)n + 255) / 256, 128);
        hipLaunchKernelGGL(k_prepare, dim3(grid), dim3(256), 0, s, d.offsets, n, p.q, p.k,
                           p.k_per_string, p.t_div, p.t_fixed, d.len, d.kk, d.rr, flags,
                           flags + 1, reinterpret_cast<unsigned long long *>(flags + 2), flags + 4,
                           d.wide_ids, d.wide_r, flags + 5,
                           reinterpret_cast<unsigned long long *>(flags + 6));
        MJ_LAUNCH_CHECK();
    }
    MJ_HIP(hipMemcpyAsync(host_dst, flags, 32, hipMemcpyDeviceToHost, s));
    if (d.total < 0)  // offsets[n] read back with the flags
        MJ_HIP(hipMemcpyAsync(host_dst + 4, d.offsets + n, 8, hipMemcpyDeviceToHost, s));
}

int32_t prepare_finish(DevStrings &d, const uint64_t *host_src, SetupInfo *info) {
    uint32_t hv[8];
    memcpy(hv, host_src, 32);
    if (d.total < 0) {
        d.total = (int64_t)host_src[4];
        check_total(d);
    }
    d.wide_count = (int32_t)hv[5];
    d.wide_pos = (int64_t)(((uint64_t)hv[7] << 32) | hv[6]);
    if (hv[1] & 1u) throw Error(MJ_EINVAL, "offsets must be non-decreasing with lengths < 2^31");
    if (hv[1] & 2u) throw Error(MJ_EINVAL, "K must be >= 0");
    if (info) {
        info->halo = (int32_t)hv[0];
        info->rec_bound = (int64_t)(((uint64_t)hv[3] << 32) | hv[2]);
        info->kmax = (int32_t)hv[4];
    }
    return (int32_t)hv[0];
}

int32_t prepare_strings(DevStrings &d, const PartitionParams &p, Workspace &ws, hipStream_t s,
                        uint64_t *host_scratch, SetupInfo *info) {
    prepare_launch(d, p, ws, s, host_scratch);
    MJ_HIP(hipStreamSynchronize(s));
    return prepare_finish(d, host_scratch, info);
}

// ---------------------------------------------------------------- bit planes
// planes[w * NP + p] bit t = bit p of the symbol at global position 32w + t (0 past the
// end): the NP planes interleaved word by word, so that a verifier lane reading the planes
// of 32 symbols touches one cache line, not NP.
// With 16-byte aligned symbols a thread reads its 32 symbols as two 16-byte loads and
// transposes each group of 8 as an 8x8 bit matrix (three delta swaps: Hacker's Delight,
// sec. 7-3), after which byte p of the result holds plane p's bits of those 8 symbols.
__device__ __forceinline__ uint64_t transpose8x8(uint64_t x) {
    uint64_t t = (x ^ (x >> 7)) & 0x00AA00AA00AA00AAull;
    x ^= t ^ (t << 7);
    t = (x ^ (x >> 14)) & 0x0000CCCC0000CCCCull;
    x ^= t ^ (t << 14);
    t = (x ^ (x >> 28)) & 0x00000000F0F0F0F0ull;
    x ^= t ^ (t << 28);
    return x;
}

// byte p of each of y[0..3], in that order, as one word (v_perm: bytes 0-3 of the second
// operand, 4-7 of the first; selector 0x0C gives a zero byte)
template <int P>
__device__ __forceinline__ uint32_t gather_byte(const uint64_t y[4]) {
    constexpr int b = P & 3;
    const uint32_t w0 = (uint32_t)(y[0] >> (P < 4 ? 0 : 32)), w1 = (uint32_t)(y[1] >> (P < 4 ? 0 : 32));
    const uint32_t w2 = (uint32_t)(y[2] >> (P < 4 ? 0 : 32)), w3 = (uint32_t)(y[3] >> (P < 4 ? 0 : 32));
    constexpr uint32_t sel = (uint32_t)b | ((uint32_t)(b + 4) << 8) | (0x0Cu << 16) | (0x0Cu << 24);
    const uint32_t lo = __builtin_amdgcn_perm(w1, w0, sel);
    const uint32_t hi = __builtin_amdgcn_perm(w3, w2, sel);
    return lo | (hi << 16);
}

// nonzero when some byte of x is >= sigma
__device__ __forceinline__ uint32_t any_byte_ge(uint32_t x, uint32_t sigma) {
    return (uint32_t)((x & 0xFFu) >= sigma) | (uint32_t)(((x >> 8) & 0xFFu) >= sigma) |
           (uint32_t)(((x >> 16) & 0xFFu) >= sigma) | (uint32_t)((x >> 24) >= sigma);
}

// Also checks every symbol against the alphabet: *err |= 1 when a code is >= sigma (the
// entry points fail with MJ_EINVAL at their next read-back).
template <int NP>
__global__ void k_pack_planes(const uint8_t *chars, int64_t total, uint32_t *planes,
                              int64_t plane_words, int aligned, uint32_t sigma, uint32_t *err) {
    int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    uint32_t over = 0;
    for (; w < plane_words; w += stride) {
        uint32_t acc[NP];
        int64_t base = w * 32;
        if (aligned && base + 32 <= total) {
            const uint4 *v = reinterpret_cast<const uint4 *>(chars + base);
            const uint4 a = v[0], b = v[1];
            over |= any_byte_ge(a.x, sigma) | any_byte_ge(a.y, sigma) | any_byte_ge(a.z, sigma) |
                    any_byte_ge(a.w, sigma) | any_byte_ge(b.x, sigma) | any_byte_ge(b.y, sigma) |
                    any_byte_ge(b.z, sigma) | any_byte_ge(b.w, sigma);
            uint64_t y[4];
            y[0] = transpose8x8(((uint64_t)a.y << 32) | a.x);
            y[1] = transpose8x8(((uint64_t)a.w << 32) | a.z);
            y[2] = transpose8x8(((uint64_t)b.y << 32) | b.x);
            y[3] = transpose8x8(((uint64_t)b.w << 32) | b.z);
            acc[0] = gather_byte<0>(y);
            acc[1] = gather_byte<1>(y);
            if constexpr (NP > 2) {
                acc[2] = gather_byte<2>(y);
                acc[3] = gather_byte<3>(y);
            }
            if constexpr (NP > 4) {
                acc[4] = gather_byte<4>(y);
                acc[5] = gather_byte<5>(y);
            }
            if constexpr (NP > 6) {
                acc[6] = gather_byte<6>(y);
                acc[7] = gather_byte<7>(y);
            }
        } else {
#pragma unroll
            for (int p = 0; p < NP; p++) acc[p] = 0;
            for (int t = 0; t < 32; t++) {
                int64_t g = base + t;
                uint32_t c = g < total ? chars[g] : 0u;
                over |= (uint32_t)(c >= sigma);
#pragma unroll
                for (int p = 0; p < NP; p++) acc[p] |= ((c >> p) & 1u) << t;
            }
        }
#pragma unroll
        for (int p = 0; p < NP; p++) planes[w * NP + p] = acc[p];
    }
    if (over) atomicOr(err, 1u);
}

// Planes of 2-bit packed symbols (four per byte, the first in the low bits): the 32
// symbols of plane word w are the 64 bits of packed words 2w and 2w + 1, plane 0 their
// even bits and plane 1 their odd bits, gathered by halving shift-and-mask steps.  Bits
// past the last symbol are cleared; with sigma < 4 a code >= sigma sets *err.
__device__ __forceinline__ uint32_t even_bits64(uint64_t x) {
    x &= 0x5555555555555555ull;
    x = (x | (x >> 1)) & 0x3333333333333333ull;
    x = (x | (x >> 2)) & 0x0F0F0F0F0F0F0F0Full;
    x = (x | (x >> 4)) & 0x00FF00FF00FF00FFull;
    x = (x | (x >> 8)) & 0x0000FFFF0000FFFFull;
    return (uint32_t)(x | (x >> 16));
}

__global__ void k_pack_planes_2bit(const uint32_t *packed, int64_t total, uint32_t *planes,
                                   int64_t plane_words, uint32_t sigma, uint32_t *err) {
    int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t nin = (total + 15) / 16;  // packed words the caller holds
    uint32_t over = 0;
    for (; w < plane_words; w += stride) {
        const uint32_t lo = 2 * w < nin ? packed[2 * w] : 0u;
        const uint32_t hi = 2 * w + 1 < nin ? packed[2 * w + 1] : 0u;
        const uint64_t x = ((uint64_t)hi << 32) | lo;
        uint32_t p0 = even_bits64(x), p1 = even_bits64(x >> 1);
        const int64_t valid = total - 32 * w;  // symbols of this word inside the input
        if (valid < 32) {
            const uint32_t keep = valid <= 0 ? 0u : (1u << valid) - 1u;
            p0 &= keep;
            p1 &= keep;
        }
        if (sigma == 3) over |= p0 & p1;  // code 3
        if (sigma == 2) over |= p1;       // codes 2 and 3
        planes[2 * w] = p0;
        planes[2 * w + 1] = p1;
    }
    if (over) atomicOr(err, 1u);
}

void pack_planes(DevStrings &d, int np, Workspace &ws, hipStream_t s, uint32_t *dest) {
    d.plane_words = plane_words_for(d.total);
    d.planes = dest ? dest : ws.get_n<uint32_t>((size_t)np * d.plane_words);
    uint32_t *err = ws.get_n<uint32_t>(2);
    fill_u32(err, 0, 1, s);
    d.symbol_err = err;
    int aligned = ((uintptr_t)d.chars & 15) == 0 ? 1 : 0;
    const uint32_t sg = (uint32_t)d.sigma;
    const dim3 grid(grid_for(d.plane_words, 256, 16384));
    if (d.packing == MJ_PACK_2BIT) {
        if (np != 2) throw Error(MJ_EINVAL, "2-bit packing has two planes");
        hipLaunchKernelGGL(k_pack_planes_2bit, grid, dim3(256), 0, s,
                           reinterpret_cast<const uint32_t *>(d.chars), d.total, d.planes,
                           d.plane_words, sg, err);
        MJ_LAUNCH_CHECK();
        return;
    }
    switch (np) {
        case 2: hipLaunchKernelGGL(k_pack_planes<2>, grid, dim3(256), 0, s, d.chars, d.total, d.planes, d.plane_words, aligned, sg, err); break;
        case 4: hipLaunchKernelGGL(k_pack_planes<4>, grid, dim3(256), 0, s, d.chars, d.total, d.planes, d.plane_words, aligned, sg, err); break;
        case 6: hipLaunchKernelGGL(k_pack_planes<6>, grid, dim3(256), 0, s, d.chars, d.total, d.planes, d.plane_words, aligned, sg, err); break;
        case 8: hipLaunchKernelGGL(k_pack_planes<8>, grid, dim3(256), 0, s, d.chars, d.total, d.planes, d.plane_words, aligned, sg, err); break;
        default: throw Error(MJ_EINVAL, "plane count must be 2, 4, 6 or 8");
    }
    MJ_LAUNCH_CHECK();
}

void check_symbols(const DevStrings &d, hipStream_t s, uint64_t *host_scratch) {
    if (!d.symbol_err) return;
    if (read_back<uint32_t>(d.symbol_err, s, host_scratch))
        throw Error(MJ_EINVAL, "a symbol code is not below sigma");
}

// ---------------------------------------------------------------- anchors
// One workgroup handles a tile of TP positions of the concatenated strings within a
// region of REGION positions: H before the tile (H >= every radius used) and the rest,
// at least H, after it.  Each thread hashes the q-grams of RUN consecutive positions of
// the region into LDS; string boundaries come from an LDS copy of the offsets of the
// strings the region overlaps.  A position p is an anchor when h[p] is strictly smaller
// than every other value in [p-r, p+r] (the window test below).  Anchors and string
// starts are flagged in LDS and written as one bit per position.
constexpr int AT_THREADS = 256;

// Order-preserving ranks of the q-gram hash for small code spaces (q*b <= 12 bits):
// rank(G) = number of codes whose hash is strictly smaller than Pi(G).  Pi(a) < Pi(b)
// exactly when rank(a) < rank(b), and equal hashes get equal ranks, so every strict
// window-minimum test gives the same answer on ranks as on the 64-bit hashes.
constexpr int RANK_MAX_BITS = 12;
// One wave per code (four per block): the block hashes every code into LDS, each lane
// counts the smaller hashes among every 64th code, and the wave adds the counts.
__global__ __launch_bounds__(256) void k_rank_table(int ncodes, uint64_t salt,
                                                    const uint64_t *__restrict__ table,
                                                    uint16_t *__restrict__ rank) {
    __shared__ uint64_t v[1 << RANK_MAX_BITS];
    for (int c = threadIdx.x; c < ncodes; c += blockDim.x)
        v[c] = table ? table[c] : mix64((uint64_t)c ^ salt);
    __syncthreads();
    const int c = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (c >= ncodes) return;  // wave-uniform
    const uint64_t x = v[c];
    int below = 0;
    for (int j = lane; j < ncodes; j += 64) below += v[j] < x ? 1 : 0;
    for (int d = 32; d >= 1; d >>= 1) below += __shfl_xor(below, d, 64);
    if (lane == 0) rank[c] = (uint16_t)below;
}

// Per-tile descriptor: the strings overlapping the tile's region (first id, count), and
// for up to TD_STR of them their offsets and radii, so that the anchor kernel reads all
// it needs about string boundaries in one coalesced load.  One thread per tile: the
// binary searches' latency overlaps across tiles.  rmin: the smallest radius of an
// interior position of the tile (0x7FFFFFFF: none), known when ns >= 0.
constexpr int TD_STR = 8;
struct TileDesc {
    int32_t s0, ns;             // ns = -1: more than TD_STR strings (search per position)
    int64_t off[TD_STR + 1];
    int32_t r[TD_STR];
    int32_t rmin;
    int32_t pad[3];             // 128 bytes
};
static_assert(sizeof(TileDesc) == 128, "tile descriptor size");

__global__ void k_tile_desc(const int64_t *__restrict__ off, const int32_t *__restrict__ rr,
                            int32_t n, int64_t total, int64_t ntiles, int TP, int H, int NR,
                            int q, TileDesc *__restrict__ td) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles) return;
    int64_t base = t * TP - H;
    int64_t g0 = base < 0 ? 0 : base;
    int64_t g1 = min(base + NR, total) - 1;
    int32_t s0 = g0 < total ? owner_of(off, n, g0) : n;
    int32_t s1 = g1 >= g0 ? owner_of(off, n, g1) : s0;
    TileDesc d;
    d.s0 = s0;
    d.ns = (s1 - s0 + 1 <= TD_STR) ? (s1 - s0 + 1) : -1;
    for (int k = 0; k <= TD_STR; k++) d.off[k] = (d.ns >= 0 && k <= d.ns) ? off[s0 + k] : 0;
    for (int k = 0; k < TD_STR; k++) d.r[k] = (d.ns >= 0 && k < d.ns) ? rr[s0 + k] : 0;
    // interior positions of a string: i in [r, npos - r) with npos = m - q + 1 full
    // q-grams (none on the wide path); those in the tile's own positions set rmin
    const int64_t c0 = t * TP, c1 = min(c0 + TP, total);
    int32_t rmin = 0x7FFFFFFF;
    for (int k = 0; d.ns >= 0 && k < d.ns; k++) {
        const int32_t r = d.r[k];
        if (r >= WIDE_SENTINEL) continue;
        const int64_t npos = d.off[k + 1] - d.off[k] - q + 1;
        if (max(d.off[k] + r, c0) < min(d.off[k] + npos - r, c1)) rmin = min(rmin, r);
    }
    d.rmin = rmin;
    for (int k = 0; k < 3; k++) d.pad[k] = 0;
    td[t] = d;
}

// Pi of a q-gram code: the injected table's entry (TABLE), else SplitMix64 of code ^ salt.
template <bool TABLE>
__device__ __forceinline__ uint64_t pi_of(uint64_t G, uint64_t salt, const uint64_t *table) {
    if constexpr (TABLE) return table[G];
    else return mix64(G ^ salt);
}

// V = uint64_t: the hash itself (Pi, or the injected table when TABLE); V = uint32_t: its
// rank from the repetition's rank table (code spaces of at most RANK_MAX_BITS bits), staged
// in LDS.  TABLE is a template parameter so that the hashing loop has no branch per position.
// One launch covers every repetition rho < reps: the region's symbols, its string bounds and
// (on the fast paths) the q-gram codes are staged once, then hashed with each repetition's
// salt mix64(seed + rho + GAMMA) (rank table rho at rank + rho * rstride); repetition rho's
// flags go to bitmap + rho * bm_stride and its tile counts to tile_count + rho * tc_stride.
template <int REGION, typename V, bool TABLE>
__global__ __launch_bounds__(AT_THREADS)
// as many resident waves as the LDS allows (7 workgroups per CU for the smaller region):
// the register budget that leaves
__attribute__((amdgpu_waves_per_eu(REGION == 2048 ? 7 : 3))) void k_anchor_tiles(
    const uint8_t *__restrict__ chars, const int64_t *__restrict__ off, int32_t n, int64_t total,
    int q, int bits, uint64_t seed, int reps, const uint64_t *__restrict__ table,
    const uint16_t *__restrict__ rank, int rstride, const int32_t *__restrict__ rr, int TP, int H,
    const TileDesc *__restrict__ tdesc, int aligned4, int packed, uint64_t *__restrict__ bitmap,
    int64_t bm_stride, uint32_t *__restrict__ tile_count, int64_t tc_stride) {
    constexpr bool RANKED = sizeof(V) == 4;
    // LDS slots hold keys: ranks as 16 bits (ranks < 2^12; the sentinel 0xFFFF is above
    // them all), hashes by their top 32 bits (sentinel 0xFFFFFFFF).  Compact slots leave
    // room for more resident workgroups.  Ranks order positions exactly; top halves only
    // decide where they differ: where the key of a candidate equals a competitor's, the
    // full hashes, recomputed from the staged symbols, decide (exact64 below).
    using S = typename std::conditional<RANKED, uint16_t, uint32_t>::type;
    using KT = uint32_t;  // keys in registers
    using Code = typename std::conditional<RANKED, uint32_t, uint64_t>::type;
    // keys, then the suffix (bufA) and prefix (bufB) minima within window-test blocks
    __shared__ __align__(16) S bufA[REGION];
    __shared__ __align__(16) S bufB[REGION];
    // per region slot, written by threads on the general path only: the radius if the
    // position is interior, else 0 (threads on the fast paths keep theirs in registers)
    __shared__ __align__(16) uint16_t pinfo[REGION];
    // symbols, one byte each, word-aligned with the input: NR + q - 1 bytes from offset
    // sh (< 4; < 16 for 2-bit packed input, where q <= 32), read as whole words (and up to
    // 16 bytes past the last q-gram by the hashing loop)
    constexpr int CH_WORDS = (REGION + 64 + 8) / 4 + 4;
    constexpr int CW = (CH_WORDS + AT_THREADS - 1) / AT_THREADS;  // words per thread
    constexpr int CWP = (CH_WORDS / 4 + 1 + AT_THREADS - 1) / AT_THREADS;  // packed words
    __shared__ __align__(16) uint32_t ch32[CH_WORDS];
    uint8_t *const ch = reinterpret_cast<uint8_t *>(ch32);
    // anchor and string-start flags of the tile positions, one bit each
    __shared__ uint32_t aflag[REGION / 32];
    __shared__ TileDesc td;
    // rank table: 2^(q b) entries in dynamic shared memory (sized at launch; none for
    // hashes), so that small code spaces leave room for more resident workgroups
    extern __shared__ __align__(16) uint16_t rank_s[];
    __shared__ int32_t rmin_s;
    const int NR = REGION;
    const int tid = threadIdx.x;
    const int64_t tile_start = (int64_t)blockIdx.x * TP;
    const int64_t base = tile_start - H;
    // Every global load of the set-up is issued before the first of them is used, so a
    // workgroup waits for one memory round trip rather than one per copy loop trip.
    uint32_t tdw = 0;
    if (tid < 32) tdw = reinterpret_cast<const uint32_t *>(tdesc + blockIdx.x)[tid];
    // rank tables: 16-byte copies (each starts on a 16-byte boundary of a workspace block
    // with 16 bytes of slack past its end)
    constexpr int RK = RANKED ? ((1 << RANK_MAX_BITS) / 8 + AT_THREADS - 1) / AT_THREADS : 1;
    uint4 rk[RK];
    const int nr8 = RANKED ? ((1 << (q * bits)) + 7) / 8 : 0;
    auto load_rank = [&](int rho) {
        if constexpr (RANKED) {
            const uint4 *src = reinterpret_cast<const uint4 *>(rank + (int64_t)rho * rstride);
#pragma unroll
            for (int i = 0; i < RK; i++) {
                const int c = tid + AT_THREADS * i;
                rk[i] = c < nr8 ? src[c] : make_uint4(0, 0, 0, 0);
            }
        }
    };
    auto store_rank = [&]() {
        if constexpr (RANKED) {
#pragma unroll
            for (int i = 0; i < RK; i++)
                if (tid + AT_THREADS * i < nr8) reinterpret_cast<uint4 *>(rank_s)[tid + AT_THREADS * i] = rk[i];
        }
    };
    load_rank(0);
    // symbols of the region: byte sh + idx of ch holds global position base + idx, with
    // ch starting at a 4-byte boundary of the input (16 symbols: a 32-bit word of 2-bit
    // packed input) so whole words are copied
    const int sh = (int)(base & (packed ? 15 : 3));
    const int64_t chbase = base - sh;
    const int nwords = (NR + q + sh + 3) / 4;  // <= CH_WORDS (q <= 64; q <= 32 packed)
    uint32_t cw[CW];
    if (packed) {
        // 2-bit input: a thread loads whole packed words (16 symbols) and spreads them to
        // bytes when it stores them (0 outside the input)
        const int64_t pw0 = chbase >> 4, nin = (total + 15) >> 4;
        const int npw = (nwords + 3) / 4;
        const uint32_t *src = reinterpret_cast<const uint32_t *>(chars);
#pragma unroll
        for (int i = 0; i < CWP; i++) {
            const int k = tid + AT_THREADS * i;
            cw[i] = (k < npw && pw0 + k >= 0 && pw0 + k < nin) ? src[pw0 + k] : 0u;
        }
    } else if (aligned4 && chbase >= 0 && chbase + 4 * (int64_t)nwords <= total) {
        const uint32_t *src = reinterpret_cast<const uint32_t *>(chars) + (chbase >> 2);
#pragma unroll
        for (int i = 0; i < CW; i++) {
            const int k = tid + AT_THREADS * i;
            cw[i] = k < nwords ? src[k] : 0u;
        }
    } else {  // the first and last tiles, or unaligned symbols: byte by byte, 0 outside
#pragma unroll
        for (int i = 0; i < CW; i++) {
            const int64_t gp = chbase + 4 * (int64_t)(tid + AT_THREADS * i);
            uint32_t w = 0;
            if (tid + AT_THREADS * i < nwords)
                for (int b = 0; b < 4; b++)
                    if (gp + b >= 0 && gp + b < total) w |= (uint32_t)chars[gp + b] << (8 * b);
            cw[i] = w;
        }
    }
    if (tid == 0) rmin_s = 0x7FFFFFFF;
    for (int w = tid; w < REGION / 32; w += AT_THREADS) aflag[w] = 0;
    if (tid < 32) reinterpret_cast<uint32_t *>(&td)[tid] = tdw;
    if (packed) {
#pragma unroll
        for (int i = 0; i < CWP; i++) {
            const int k = tid + AT_THREADS * i;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                if (4 * k + j < nwords) {
                    // four 2-bit symbols (first in the low bits) to four bytes
                    uint32_t x = (cw[i] >> (8 * j)) & 0xFFu;
                    x = (x | (x << 12)) & 0x000F000Fu;
                    x = (x | (x << 6)) & 0x03030303u;
                    ch32[4 * k + j] = x;
                }
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < CW; i++)
            if (tid + AT_THREADS * i < nwords) ch32[tid + AT_THREADS * i] = cw[i];
    }
    store_rank();
    __syncthreads();
    const int32_t ns = td.ns;
    // string starts inside the tile are flagged like anchors (a few per tile)
    auto flag_start = [&](int idx) {
        if (idx >= H && idx < H + TP) atomicOr(&aflag[(idx - H) >> 5], 1u << ((idx - H) & 31));
    };
    const uint64_t gmask = (q * bits >= 64) ? ~0ull : ((1ull << (q * bits)) - 1);
    constexpr int RUN = REGION / AT_THREADS;
    static_assert(RUN == 8 || RUN == 16, "positions per thread");
    // Each thread takes RUN consecutive region positions.  On the fast paths it keeps, for
    // every repetition: the q-gram codes (Gs), which positions are interior tile positions
    // (bit j of imask for position idx0 + j), their radius (rA for j < jbv, else rB) and
    // the string starts among them (fs0, fs1; -1: none).  The general path (slowp) does all
    // of it per repetition, with the radii in pinfo.
    Code Gs[RUN];
    uint32_t imask = 0;
    int32_t rA = 0, rB = 0;
    int jbv = RUN, fs0 = -1, fs1 = -1;
    bool slowp = false;
    // bits lo .. hi - 1 of a run mask
    auto span = [](int lo, int hi) -> uint32_t {
        lo = max(lo, 0);
        hi = min(hi, RUN);
        return lo < hi ? (0xFFFFFFFFu >> (32 - hi)) & ~((1u << lo) - 1u) : 0u;
    };
    const int idx0 = tid * RUN;
    const int64_t g0 = base + idx0;
    int t = 0;
    int64_t sb0 = 0, se0 = -1;
    if (ns >= 0) {
        for (int k = 1; k < ns; k++) t += (td.off[k] <= g0) ? 1 : 0;
        sb0 = td.off[t];
        se0 = td.off[t + 1];
    }
    {
        // fast paths: the RUN positions lie in string t (fast1: all of them start full
        // q-grams), or in strings t and t + 1 (fast2: positions from jb on belong to t + 1,
        // and some q-grams may run past their string's end)
        const bool in_t = ns >= 0 && q <= 9 && g0 >= sb0 && idx0 + RUN <= NR;
        const bool fast1 = in_t && g0 + RUN + q - 1 <= se0;
        const int64_t se1 = (in_t && t + 1 < ns) ? td.off[t + 2] : se0;
        const bool fast2 = in_t && !fast1 && (se0 >= g0 + RUN || (t + 1 < ns && g0 + RUN <= se1));
        auto codes = [&](auto two) {
            constexpr bool TWO = decltype(two)::value;
            // bytes idx0 .. idx0 + RUN + 7 of the region (the first q-gram and the rest),
            // and the RUN - 1 symbols entering the window, idx0 + q .. idx0 + q + RUN - 2
            constexpr int NA = RUN / 4 + 3;
            uint32_t A[NA], N[RUN / 4];
            {
                const int o = idx0 + sh;
                uint32_t W[NA + 1];
#pragma unroll
                for (int i = 0; i <= NA; i++) W[i] = ch32[(o >> 2) + i];
#pragma unroll
                for (int i = 0; i < NA; i++)
                    A[i] = __builtin_amdgcn_alignbit(W[i + 1], W[i], 8 * (o & 3));
                const int o2 = o + q;
                uint32_t W2[RUN / 4 + 1];
#pragma unroll
                for (int i = 0; i <= RUN / 4; i++) W2[i] = ch32[(o2 >> 2) + i];
#pragma unroll
                for (int i = 0; i < RUN / 4; i++)
                    N[i] = __builtin_amdgcn_alignbit(W2[i + 1], W2[i], 8 * (o2 & 3));
            }
            const Code cmask = (Code)gmask;
            // the first code from its q symbols, q a compile-time constant per case
            Code G = 0;
            auto first = [&](auto qc) {
                constexpr int Q = decltype(qc)::value;
#pragma unroll
                for (int k = 0; k < Q; k++) G = (G << bits) | ((A[k >> 2] >> (8 * (k & 3))) & 0xFFu);
            };
            switch (q) {
                case 1: first(std::integral_constant<int, 1>{}); break;
                case 2: first(std::integral_constant<int, 2>{}); break;
                case 3: first(std::integral_constant<int, 3>{}); break;
                case 4: first(std::integral_constant<int, 4>{}); break;
                case 5: first(std::integral_constant<int, 5>{}); break;
                case 6: first(std::integral_constant<int, 6>{}); break;
                case 7: first(std::integral_constant<int, 7>{}); break;
                case 8: first(std::integral_constant<int, 8>{}); break;
                default: first(std::integral_constant<int, 9>{}); break;  // q <= 9 here
            }
            G &= cmask;  // the code indexes the rank table: never past its 2^(q b) entries
#pragma unroll
            for (int j = 0; j < RUN; j++) {
                Gs[j] = G;
                if (j + 1 < RUN) G = ((G << bits) | ((N[j >> 2] >> (8 * (j & 3))) & 0xFFu)) & cmask;
            }
            // positions inside a string fit in 32 bits (m < 2^31)
            const int32_t i0 = (int32_t)(g0 - sb0);
            const int32_t npos = (int32_t)(se0 - sb0) - q + 1;
            const int32_t r = td.r[t];
            // string t + 1 (fast2): its first run index jb, positions, radius
            const int jb = TWO ? (int)min<int64_t>(se0 - g0, RUN) : RUN;
            const int32_t npos1 = TWO ? (int32_t)(se1 - se0) - q + 1 : 0;
            const int32_t r1 = (TWO && t + 1 < ns) ? td.r[t + 1] : r;
            // Every position's hash is kept, also where its q-gram runs past its string's
            // end: a window-test block holding such a position holds no interior position
            // (an interior position's block lies in its window, inside its string's full
            // q-grams), so its value decides nothing.
            // Interior positions i in [r, npos - r) of string t (i = i0 + j, j < jb) and of
            // string t + 1 (i = j - jb), none on the wide path; tile positions only.
            uint32_t im = r >= WIDE_SENTINEL ? 0u : span(r - i0, min(npos - r - i0, jb));
            if (i0 == 0) fs0 = idx0;
            if constexpr (TWO) {
                if (jb < RUN) {
                    if (r1 < WIDE_SENTINEL) im |= span(jb + r1, jb + npos1 - r1);
                    fs1 = idx0 + jb;
                }
            }
            imask = im & span(H - idx0, H + TP - idx0);
            rA = r;
            rB = r1;
            jbv = jb;
        };
        // one body per wave: where a lane needs fast2, every fast lane of the wave takes it
        // (it covers the fast1 case), so the wave does not run both
        const bool wave_two = __any(fast2);
        if (fast1 && !wave_two) codes(std::false_type{});
        else if (fast1 || fast2) codes(std::true_type{});
        else slowp = true;
    }
    int lrmin = 0x7FFFFFFF;
    for (int rho = 0; rho < reps; rho++) {
        const uint64_t salt = mix64(seed + (uint64_t)rho + GAMMA);
        if (rho > 0) {
            load_rank(rho);
            __syncthreads();  // the previous repetition is done with the flags, keys and table
            for (int w = tid; w < REGION / 32; w += AT_THREADS) aflag[w] = 0;
            store_rank();
            __syncthreads();
        }
        // hashes of the thread's RUN positions into LDS
        if (!slowp) {
            uint32_t hw[RUN * sizeof(S) / 4];
#pragma unroll
            for (int j = 0; j < RUN; j++) {
                if constexpr (RANKED) {
                    const uint32_t h = rank_s[Gs[j]];
                    if (j & 1) hw[j >> 1] |= h << 16;
                    else hw[j >> 1] = h;
                } else {
                    hw[j] = (uint32_t)(pi_of<TABLE>((uint64_t)Gs[j], salt, table) >> 32);
                }
            }
            uint4 *dst = reinterpret_cast<uint4 *>(bufA + idx0);
#pragma unroll
            for (int i = 0; i < (int)(RUN * sizeof(S) / 16); i++)
                dst[i] = make_uint4(hw[4 * i], hw[4 * i + 1], hw[4 * i + 2], hw[4 * i + 3]);
            if (fs0 >= 0) flag_start(fs0);
            if (fs1 >= 0) flag_start(fs1);
        } else {
            int ts = t;
            uint64_t G = 0;
            int64_t have_end = -1;  // G is valid for the previous position in the same string
#pragma unroll 1
            for (int j = 0; j < RUN; j++) {  // rolled: few threads take this path
                const int idx = idx0 + j;
                if (idx >= NR) {  // region padding: a sentinel that is never a strict minimum
                    bufA[idx] = (S)~0ull;
                    pinfo[idx] = 0;
                    continue;
                }
                const int64_t g = base + idx;
                V h = (V)~0ull;
                uint16_t info = 0;
                int32_t r = 0;
                int64_t sbeg = 0, send = 0;
                bool valid = g >= 0 && g < total;
                if (ns >= 0) {
                    while (ts + 1 < ns && td.off[ts + 1] <= g) ts++;
                    sbeg = td.off[ts];
                    send = td.off[ts + 1];
                    r = td.r[ts];
                } else if (valid) {
                    int32_t sidx = owner_of(off, n, g);
                    sbeg = off[sidx];
                    send = off[sidx + 1];
                    r = rr[sidx];
                }
                if (valid) {
                    const int64_t i = g - sbeg;
                    const int64_t npos = (send - sbeg) - q + 1;
                    if (i < npos) {
                        if (have_end == send && i > 0 && j > 0) {
                            G = ((G << bits) | ch[sh + idx + q - 1]) & gmask;
                        } else {
                            G = 0;
                            for (int k = 0; k < q; k++) G = (G << bits) | ch[sh + idx + k];
                            G &= gmask;
                        }
                        have_end = send;
                        if constexpr (RANKED) h = rank_s[G];
                        else h = pi_of<TABLE>(G, salt, table);
                    } else {
                        have_end = -1;
                    }
                    const bool interior = r < WIDE_SENTINEL && (i >= r) && (i <= npos - 1 - r);
                    info = (uint16_t)(interior ? r : 0);
                    if (i == 0) flag_start(idx);
                    if (interior && idx >= H && idx < H + TP) {
                        lrmin = min(lrmin, r);
                        imask |= 1u << j;
                    }
                } else {
                    have_end = -1;
                }
                if constexpr (RANKED) bufA[idx] = (S)h;
                else bufA[idx] = (S)((uint64_t)h >> 32);
                pinfo[idx] = info;
            }
        }
        if (rho == 0) {
            // the smallest interior radius (the same in every repetition): the tile
            // descriptor's, else (more strings than it holds: every thread on the general
            // path) reduced over the block, one LDS atomic per wave, as the lanes' atomics
            // on one address would serialise
            if (ns < 0) {
                for (int d = 32; d >= 1; d >>= 1) lrmin = min(lrmin, __shfl_xor(lrmin, d, 64));
                if ((tid & 63) == 0 && lrmin < 0x7FFFFFFF) atomicMin(&rmin_s, lrmin);
            } else if (tid == 0) {
                rmin_s = td.rmin;
            }
        }
        __syncthreads();
        // the full hash of region slot idx: the tie-break of equal top halves (only blocks
        // and windows of interior positions, where every slot starts a full q-gram, use it)
        auto exact64 = [&](int idx) -> uint64_t {
            uint64_t G = 0;
            for (int k = 0; k < q; k++) G = (G << bits) | ch[sh + idx + k];
            G &= gmask;
            return pi_of<TABLE>(G, salt, table);
        };
        (void)exact64;
        // ---- window test.  Blocks of B = 2^k positions with B - 1 <= every interior radius
        // of the tile and B <= RUN (so a block is a part of one thread's run): a block lies
        // inside the window of each of its positions, so an anchor is the unique minimum of
        // its block.  Each thread finds the unique minima of its blocks and stores the
        // prefix minima (bufB) and suffix minima (bufA) within blocks; each such candidate
        // is then checked against the rest of its window: whole blocks through their minima
        // (the prefix minimum at the block's end), the two partial blocks through one suffix
        // and one prefix minimum.
        if (rmin_s != 0x7FFFFFFF) {  // some tile position is interior
            const int Bv = min(RUN, 1 << (31 - __clz(rmin_s + 1)));
            // the block size as a compile-time constant, so that the block-boundary selects
            // of the prefix and suffix minima and the block loops fold away
            auto window = [&](auto bconst) {
                constexpr int B = decltype(bconst)::value;
                constexpr int bm = B - 1;
                KT v[RUN];
                {
                    uint4 raw[RUN * sizeof(S) / 16];
#pragma unroll
                    for (int i = 0; i < (int)(RUN * sizeof(S) / 16); i++) raw[i] = reinterpret_cast<const uint4 *>(bufA + idx0)[i];
                    const uint32_t *w = reinterpret_cast<const uint32_t *>(raw);
#pragma unroll
                    for (int j = 0; j < RUN; j++) {
                        if constexpr (RANKED) v[j] = (w[j >> 1] >> (16 * (j & 1))) & 0xFFFFu;
                        else v[j] = w[j];
                    }
                }
                KT pre[RUN], suf[RUN];
#pragma unroll
                for (int j = 0; j < RUN; j++) pre[j] = (j & bm) == 0 ? v[j] : min(pre[j > 0 ? j - 1 : 0], v[j]);
#pragma unroll
                for (int j = RUN - 1; j >= 0; j--)
                    suf[j] = ((j + 1) & bm) == 0 ? v[j] : min(suf[j + 1 < RUN ? j + 1 : j], v[j]);
                // bit j: v[j] is strictly below every other key of its block, that is the
                // only key of the block equal to the block's minimum (its last prefix minimum)
                uint32_t cand = 0;
#pragma unroll
                for (int b0 = 0; b0 < RUN; b0 += B) {
                    uint32_t eq = 0;
#pragma unroll
                    for (int j = b0; j < b0 + B; j++) eq |= v[j] == pre[b0 + bm] ? 1u << j : 0u;
                    if (__popc(eq) == 1) {
                        cand |= eq;
                    } else if constexpr (!RANKED) {
                        // several positions hold the minimum top half: their unique minimum,
                        // if any, by their full hashes (equal ranks are equal hashes: none)
                        uint64_t e = ~0ull;
                        int je = -1;
                        bool dup = false;
                        for (; eq; eq &= eq - 1) {
                            const int j = __ffs(eq) - 1;
                            const uint64_t x = exact64(idx0 + j);
                            if (x < e) {
                                e = x;
                                je = j;
                                dup = false;
                            } else if (x == e) {
                                dup = true;
                            }
                        }
                        if (!dup && e != ~0ull) cand |= 1u << je;
                    }
                }
                cand &= imask;  // interior tile positions only
                {
                    uint32_t pw[RUN * sizeof(S) / 4], sw[RUN * sizeof(S) / 4];
#pragma unroll
                    for (int j = 0; j < RUN; j++) {
                        if constexpr (RANKED) {
                            if (j & 1) {
                                pw[j >> 1] |= (uint32_t)pre[j] << 16;
                                sw[j >> 1] |= (uint32_t)suf[j] << 16;
                            } else {
                                pw[j >> 1] = (uint32_t)pre[j];
                                sw[j >> 1] = (uint32_t)suf[j];
                            }
                        } else {
                            pw[j] = pre[j];
                            sw[j] = suf[j];
                        }
                    }
#pragma unroll
                    for (int i = 0; i < (int)(RUN * sizeof(S) / 16); i++) {
                        reinterpret_cast<uint4 *>(bufB + idx0)[i] = make_uint4(pw[4 * i], pw[4 * i + 1], pw[4 * i + 2], pw[4 * i + 3]);
                        reinterpret_cast<uint4 *>(bufA + idx0)[i] = make_uint4(sw[4 * i], sw[4 * i + 1], sw[4 * i + 2], sw[4 * i + 3]);
                    }
                }
                __syncthreads();
                constexpr int lb2 = B >= 16 ? 4 : B >= 8 ? 3 : B >= 4 ? 2 : B >= 2 ? 1 : 0;  // log2 B
                for (; cand; cand &= cand - 1) {
                    const int j = __ffs(cand) - 1;
                    const int p = idx0 + j;
                    const int r = slowp ? (int)pinfo[p] : (j < jbv ? rA : rB);
                    if (r == 0) continue;  // radii are at least 1: kept as a guard
                    const KT hv = bufA[p];  // its key: the suffix minimum from a block's minimum
                    const int bk = p >> lb2;
                    // strictly below every other key of the window: an anchor; above one:
                    // not; equal to one (ranks: equal hashes, not strict): hashes decide by
                    // full value
                    bool below = false, tie = false;
                    auto see = [&](KT x) {
                        below |= x < hv;
                        tie |= x == hv;
                    };
                    const int L = p - r, lb = L >> lb2;
                    if (lb < bk) {
                        see(bufA[L]);
                        for (int b2 = lb + 1; !below && b2 < bk; b2++) see(bufB[(b2 << lb2) + bm]);
                    }
                    const int R = p + r, rb = R >> lb2;
                    if (!below && rb > bk) {
                        for (int b2 = bk + 1; !below && b2 < rb; b2++) see(bufB[(b2 << lb2) + bm]);
                        if (!below) see(bufB[R]);
                    }
                    bool ok = !below && !tie;
                    if constexpr (!RANKED) {
                        if (!below && tie) {
                            const uint64_t ep = exact64(p);
                            ok = true;
                            for (int dd = 1; ok && dd <= r; dd++) ok = exact64(p - dd) > ep && exact64(p + dd) > ep;
                        }
                    }
                    if (ok) atomicOr(&aflag[(p - H) >> 5], 1u << ((p - H) & 31));
                }
                __syncthreads();
            };
            switch (Bv) {
                case 1: window(std::integral_constant<int, 1>{}); break;
                case 2: window(std::integral_constant<int, 2>{}); break;
                case 4: window(std::integral_constant<int, 4>{}); break;
                case 8: window(std::integral_constant<int, 8>{}); break;
                default: window(std::integral_constant<int, RUN>{}); break;  // 16 (RUN == 16)
            }
        }
        // one bit per position: string start or anchor (TP is a multiple of 64)
        const int rem = (int)min<int64_t>(total - tile_start, (int64_t)TP);  // tile positions in the input
        // TP / 64 < 64 words: the first wave writes them all and adds up their bits
        if (tid < 64) {
            uint32_t mine = 0;
            if (64 * tid < rem) {
                uint64_t v = (uint64_t)aflag[2 * tid] | ((uint64_t)aflag[2 * tid + 1] << 32);
                if (rem - 64 * tid < 64) v &= (1ull << (rem - 64 * tid)) - 1ull;
                bitmap[(int64_t)rho * bm_stride + (tile_start >> 6) + tid] = v;
                mine = (uint32_t)__popcll(v);
            }
            for (int d = 32; d >= 1; d >>= 1) mine += (uint32_t)__shfl_xor((int)mine, d, 64);
            if (tid == 0) tile_count[(int64_t)rho * tc_stride + blockIdx.x] = mine;
        }
    }
}

// ---------------------------------------------------------------- wide radii
// Strings whose radius exceeds what a tile region's halo holds.  Their hashes go to global
// memory; so do prefix and suffix minima within blocks of r positions.  Each side of an
// interior position's window, [p - r, p - 1] and [p + 1, p + r], is r positions long, so it
// meets at most two blocks and its minimum is one block suffix minimum and one block prefix
// minimum.  Anchors are ORed into the tile kernel's bitmap and counted into its tile counts
// (the tile kernel sets no bit of these strings but their starts, which are not interior).
__device__ __forceinline__ uint32_t symbol_at(const uint8_t *chars, int packed, int64_t g) {
    return packed ? (uint32_t)(chars[g >> 2] >> (2 * (g & 3))) & 3u : (uint32_t)chars[g];
}

__global__ void k_wide_npos(const int64_t *__restrict__ off, const int32_t *__restrict__ ids,
                            int32_t nw, int q, uint64_t *__restrict__ npos) {
    const int32_t w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w < nw) npos[w] = (uint64_t)(off[ids[w] + 1] - off[ids[w]] - q + 1);
}

__global__ void k_wide_hashes(const uint8_t *__restrict__ chars, int packed,
                              const int64_t *__restrict__ off, const int32_t *__restrict__ ids,
                              int32_t nw, const uint64_t *__restrict__ hoff, int q, int bits,
                              uint64_t salt, const uint64_t *__restrict__ table,
                              uint64_t *__restrict__ h) {
    const uint64_t gmask = (q * bits >= 64) ? ~0ull : ((1ull << (q * bits)) - 1);
    for (int32_t w = blockIdx.x; w < nw; w += gridDim.x) {
        const int64_t s0 = off[ids[w]];
        const int64_t npos = (int64_t)(hoff[w + 1] - hoff[w]);
        uint64_t *hw = h + hoff[w];
        for (int64_t p = threadIdx.x; p < npos; p += blockDim.x) {
            uint64_t G = 0;
            for (int k = 0; k < q; k++) G = (G << bits) | symbol_at(chars, packed, s0 + p + k);
            G &= gmask;
            hw[p] = table ? table[G] : mix64(G ^ salt);
        }
    }
}

__global__ void k_wide_blockmin(const int32_t *__restrict__ wr, int32_t nw,
                                const uint64_t *__restrict__ hoff, const uint64_t *__restrict__ h,
                                uint64_t *__restrict__ P, uint64_t *__restrict__ S) {
    for (int32_t w = blockIdx.x; w < nw; w += gridDim.x) {
        const int64_t o = (int64_t)hoff[w], npos = (int64_t)(hoff[w + 1] - hoff[w]), r = wr[w];
        const int64_t nb = (npos + r - 1) / r;
        for (int64_t b = threadIdx.x; b < nb; b += blockDim.x) {
            const int64_t lo = o + b * r, hi = o + min(npos, (b + 1) * r);
            uint64_t m = ~0ull;
            for (int64_t p = lo; p < hi; p++) {
                m = min(m, h[p]);
                P[p] = m;
            }
            m = ~0ull;
            for (int64_t p = hi - 1; p >= lo; p--) {
                m = min(m, h[p]);
                S[p] = m;
            }
        }
    }
}

__global__ void k_wide_anchors(const int64_t *__restrict__ off, const int32_t *__restrict__ ids,
                               const int32_t *__restrict__ wr, int32_t nw,
                               const uint64_t *__restrict__ hoff, const uint64_t *__restrict__ h,
                               const uint64_t *__restrict__ P, const uint64_t *__restrict__ S,
                               int TP, unsigned long long *bitmap, uint32_t *tcount) {
    for (int32_t w = blockIdx.x; w < nw; w += gridDim.x) {
        const int64_t s0 = off[ids[w]], o = (int64_t)hoff[w];
        const int64_t npos = (int64_t)(hoff[w + 1] - hoff[w]), r = wr[w];
        for (int64_t p = r + threadIdx.x; p <= npos - 1 - r; p += blockDim.x) {
            const uint64_t x = h[o + p];
            const uint64_t left = min(S[o + p - r], P[o + p - 1]);
            const uint64_t right = min(S[o + p + 1], P[o + p + r]);
            if (x < left && x < right) {
                const int64_t g = s0 + p;
                atomicOr(bitmap + (g >> 6), 1ull << (g & 63));
                atomicAdd(tcount + g / TP, 1u);
            }
        }
    }
}

// Buffers of the wide path: each wide string's first slot (hoff, nw + 1 entries), and the
// hashes and block minima of all their q-gram starts.
struct WideBufs {
    uint64_t *hoff = nullptr, *h = nullptr, *P = nullptr, *S = nullptr;
};

static WideBufs wide_setup(const DevStrings &d, int q, Workspace &ws, hipStream_t s) {
    WideBufs wb;
    if (d.wide_count <= 0) return wb;
    const int32_t nw = d.wide_count;
    uint64_t *np = ws.get_n<uint64_t>((size_t)nw + 1);
    wb.hoff = ws.get_n<uint64_t>((size_t)nw + 1);
    hipLaunchKernelGGL(k_wide_npos, dim3((nw + 255) / 256), dim3(256), 0, s, d.offsets, d.wide_ids,
                       nw, q, np);
    MJ_LAUNCH_CHECK();
    exclusive_scan_u64(np, wb.hoff, nw, ws, s);
    wb.h = ws.get_n<uint64_t>((size_t)d.wide_pos + 1);
    wb.P = ws.get_n<uint64_t>((size_t)d.wide_pos + 1);
    wb.S = ws.get_n<uint64_t>((size_t)d.wide_pos + 1);
    return wb;
}

static void wide_anchors(const DevStrings &d, const WideBufs &wb, const PartitionParams &p,
                         uint64_t salt, int TP, uint64_t *bitmap, uint32_t *tcount, hipStream_t s) {
    if (d.wide_count <= 0) return;
    const int32_t nw = d.wide_count;
    const dim3 grid((unsigned)std::min<int32_t>(nw, 65535));
    const int packed = d.packing == MJ_PACK_2BIT ? 1 : 0;
    hipLaunchKernelGGL(k_wide_hashes, grid, dim3(256), 0, s, d.chars, packed, d.offsets,
                       d.wide_ids, nw, wb.hoff, p.q, d.bits, salt, p.pi_table, wb.h);
    MJ_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_wide_blockmin, grid, dim3(256), 0, s, d.wide_r, nw, wb.hoff, wb.h, wb.P,
                       wb.S);
    MJ_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_wide_anchors, grid, dim3(256), 0, s, d.offsets, d.wide_ids, d.wide_r, nw,
                       wb.hoff, wb.h, wb.P, wb.S, TP,
                       reinterpret_cast<unsigned long long *>(bitmap), tcount);
    MJ_LAUNCH_CHECK();
}

// Positions of the flagged bits, in order: one wave per anchor tile (its TP / 64 <= 64
// bitmap words), the tile's first rank from the scan of the tiles' counts, each word's
// from a prefix over the wave.  apos[R] = total closes the last partition.
__global__ __launch_bounds__(64) void k_anchor_scatter(const uint64_t *__restrict__ bm, int64_t nw,
                                                       int words_per_tile,
                                                       const uint32_t *__restrict__ tile_pre,
                                                       int64_t ntiles, int64_t *__restrict__ apos,
                                                       int64_t total) {
    const int lane = threadIdx.x;
    const int64_t t = blockIdx.x;
    const int64_t w = t * words_per_tile + lane;
    uint64_t bits = (lane < words_per_tile && w < nw) ? bm[w] : 0ull;
    const uint32_t c = (uint32_t)__popcll(bits);
    uint32_t incl = c;
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)incl, d, 64);
        if (lane >= d) incl += y;
    }
    uint32_t rank = tile_pre[t] + incl - c;
    while (bits) {
        const int b = __ffsll((unsigned long long)bits) - 1;
        apos[rank++] = w * 64 + b;
        bits &= bits - 1;
    }
    if (t == ntiles - 1 && lane == 63) apos[tile_pre[ntiles]] = total;
}

// ---------------------------------------------------------------- partition records
// Partition records between consecutive flagged positions: key f = M(Phi xor S) with
// Phi the Karp-Rabin polynomial of the content over GF(2^61-1), length folded in as the
// leading coefficient, Phi = L B^L + sum_{g0 <= i < g1} (x_i + 1) B^(g1-1-i) for the
// partition [g0, g1) of length L (Horner's rule started from L); payload (string id << 32 |
// start position).  The owning string comes from the descriptor of the tile holding the
// partition's first position; symbol codes are taken modulo 2^b.
__device__ __forceinline__ uint64_t horner_step(uint64_t h, uint64_t B, uint32_t c) {
    h = mulmod61(h, B) + (uint64_t)c + 1;
    return h >= P61 ? h - P61 : h;
}

// s < 2^64 reduced to [0, 2^61 + 8): 2^61 = 1 modulo 2^61 - 1
__device__ __forceinline__ uint64_t fold61(uint64_t s) { return (s & P61) + (s >> 61); }

// Chunk tables.  Eight power tables P[j 2^b + c] = (c + 1) B^j, j < 8 (8 * 2^b entries):
// a chunk's value is the sum of one entry of each, and P[j 2^b] = B^j.  pt == 0 (b <= 2)
// puts before them T[x] = sum_k (x_k + 1) B^(3-k) for every packed chunk x of 4 symbols
// and the same values times B^4 (2 * 2^(4b) entries).
// lsb != 0 (2-bit packed input): a chunk x holds its first symbol in the low bits, so a
// packed byte is its own table index.
__global__ void k_phi_table(int nc, int bits, uint64_t B, int pt, int lsb, uint64_t *__restrict__ T) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nc) return;
    uint64_t h = 0;
    const int pbase = pt ? 0 : 2 << (4 * bits);  // first power-table entry
    if (idx >= pbase) {
        const int e = idx - pbase;
        h = (uint64_t)(e & ((1 << bits) - 1)) + 1;
        for (int j = 0; j < (e >> bits); j++) h = mulmod61(h, B);
    } else {
        const int x = idx & ((1 << (4 * bits)) - 1);
        for (int k = 0; k < 4; k++)
            h = horner_step(h, B, (uint32_t)(x >> (bits * (lsb ? k : 3 - k))) & ((1u << bits) - 1u));
        if (idx >> (4 * bits))
            for (int k = 0; k < 4; k++) h = mulmod61(h, B);
    }
    T[idx] = h;
}

constexpr int REC_THREADS = 256;
constexpr int REC_STAGE_WORDS = 6144;  // 24 KB: the symbols of a block's records

// Horner's rule over partitions, one thread each, 8 symbols per step: Phi <- Phi B^8 +
// sum_k (x_k + 1) B^(7-k), the sum read from tables in LDS, a shorter tail 4 symbols and
// then 1 symbol at a time (modular arithmetic is exact: the same Phi as one symbol per
// step).  Symbols come four at a time from aligned 32-bit words.  Two uses:
//  - every partition of one repetition, between consecutive positions of apos (R of them,
//    or *Rdev on the device; records from *base_dev when given), a block taking 256
//    consecutive records per sweep.  STAGED (long partitions): their symbols form one
//    contiguous range, which the block first copies to LDS with coalesced word loads (a
//    lane reading its own partition directly touches a line per lane and load); a range
//    longer than the stage is read from global memory instead.  Short partitions are read
//    directly: the copy and its barriers would cost more.
//  - CROSS: the partitions that run past the tile of their first position, from the slots
//    k_records_tiles fills (per repetition and tile: first position, record index; -1:
//    none; ntiles slots per repetition): the partition ends at the next flagged position
//    of the repetition's bitmap, or at the input's end.
// PACKED: 2-bit input (four symbols per byte, the first in the low bits); a packed byte is
// a 4-symbol chunk and, with the chunk tables built in that order, its own table index.
template <bool STAGED, bool PACKED, bool CROSS = false>
__global__ __launch_bounds__(REC_THREADS) void k_records(
    const int64_t *__restrict__ apos, int64_t R, int64_t ntiles, const uint64_t *__restrict__ bitmap,
    int64_t bm_stride, const int64_t *__restrict__ off, int32_t n,
    const uint8_t *__restrict__ chars, int64_t total, int aligned4,
    const TileDesc *__restrict__ td, int TP, uint64_t B, uint64_t salt_f,
    const uint64_t *__restrict__ table, int pt, int bits, uint64_t B4, uint64_t B8, uint64_t *key,
    uint64_t *val, uint32_t *len, const uint32_t *__restrict__ Rdev,
    const int64_t *__restrict__ base_dev) {
    extern __shared__ uint64_t Ts[];
    __shared__ uint32_t stage[STAGED ? REC_STAGE_WORDS : 1];
    // sizes known on the device only: this repetition's record count and where its records
    // go (R is then the bound the grid was sized by)
    if (Rdev) R = min<int64_t>(R, (int64_t)*Rdev);
    if (base_dev) {
        const int64_t b = *base_dev;
        key += b;
        val += b;
        if (len) len += b;
    }
    const int nsym = 1 << bits;
    const int n4 = 1 << (4 * bits);  // pt == 0: chunks of 4 symbols
    const int pbase = pt ? 0 : 2 * n4;  // the power tables
    const int nc = pbase + 8 * nsym;
    for (int t = threadIdx.x; t < nc; t += blockDim.x) Ts[t] = table[t];
    const uint32_t m = (1u << bits) - 1u;
    // a chunk word holds 4 symbols, SU bits apart (bytes; 2-bit fields when packed)
    constexpr int SU = PACKED ? 2 : 8;
    // the table index of a chunk word (pt == 0)
    auto cidx = [&](uint32_t v) -> uint32_t {
        if constexpr (PACKED) return v & 0xFFu;
        return ((v & m) << (3 * bits)) | (((v >> 8) & m) << (2 * bits)) | (((v >> 16) & m) << bits) |
               ((v >> 24) & m);
    };
    // sum over the 4 symbols x_k of v of (x_k + 1) B^(j0 + 3 - k) (pt == 1): four terms
    auto pw4 = [&](uint32_t v, int j0) -> uint64_t {
        return Ts[(j0 + 3) * nsym + (v & m)] + Ts[(j0 + 2) * nsym + ((v >> SU) & m)] +
               Ts[(j0 + 1) * nsym + ((v >> (2 * SU)) & m)] + Ts[j0 * nsym + ((v >> (3 * SU)) & m)];
    };
    // h B^k + sum over the k < 4 symbols x_i in slots 0 .. k-1 of v of (x_i + 1) B^(k-1-i)
    auto partial = [&](uint64_t h, uint32_t v, int k) -> uint64_t {
        uint64_t sum = mulmod61(h, Ts[pbase + k * nsym]);  // P[k 2^b] = B^k
        for (int i = 0; i < k; i++) sum += Ts[pbase + (k - 1 - i) * nsym + ((v >> (SU * i)) & m)];
        const uint64_t x = fold61(sum);
        return x >= P61 ? x - P61 : x;
    };
    // Horner's rule over [g, g1) from symbols sym(i) and chunk words word(i) (i a multiple
    // of 4), a chunk being readable when it ends at or before wend.  Every table entry and
    // h are below p = 2^61 - 1, so a sum of at most five of them stays below 2^64 and one
    // fold brings it below 2^61 + 5 < 2p.  The symbols before the first chunk boundary
    // and after the last whole chunk go in one step each.
    auto hash = [&](uint64_t h, int64_t g, int64_t g1, int64_t wend, auto sym, auto word) -> uint64_t {
        if (PACKED || aligned4) {
            if ((g & 3) && g < g1 && (g | 3) < wend) {
                const int k = (int)min<int64_t>(4 - (g & 3), g1 - g);
                h = partial(h, word(g & ~(int64_t)3) >> (SU * (g & 3)), k);
                g += k;
            }
            for (; g < g1 && (g & 3); g++) h = horner_step(h, B, sym(g) & m);
            for (; g + 8 <= g1; g += 8) {  // h B^8 + (x0..x3) B^4 + (x4..x7)
                const uint32_t v0 = word(g), v1 = word(g + 4);
                uint64_t x;
                if (!pt) {
                    x = fold61(mulmod61(h, B8) + Ts[n4 + cidx(v0)] + Ts[cidx(v1)]);
                } else {
                    x = fold61(mulmod61(h, B8) + pw4(v0, 4));
                    x = fold61(x + pw4(v1, 0));
                }
                h = x >= P61 ? x - P61 : x;
            }
            if (g + 4 <= g1) {
                const uint32_t v = word(g);
                const uint64_t x = fold61(mulmod61(h, B4) + (pt ? pw4(v, 0) : Ts[cidx(v)]));
                h = x >= P61 ? x - P61 : x;
                g += 4;
            }
            if (g < g1 && g + 4 <= wend) {
                h = partial(h, word(g), (int)(g1 - g));
                g = g1;
            }
        }
        for (; g < g1; g++) h = horner_step(h, B, sym(g) & m);
        return h;
    };
    const uint32_t *w = reinterpret_cast<const uint32_t *>(chars);
    // global accessors: a symbol, and the chunk word at a multiple of 4
    auto gsym = [&](int64_t g) -> uint32_t {
        if constexpr (PACKED) return (uint32_t)(chars[g >> 2] >> (2 * (g & 3))) & 3u;
        return chars[g];
    };
    auto gword = [&](int64_t g) -> uint32_t {
        if constexpr (PACKED) return chars[g >> 2];
        return w[g >> 2];
    };
    // packed input: the whole words (16 symbols) the caller holds; unpacked: whole symbols
    const int64_t gend = PACKED ? ((total + 15) & ~(int64_t)15) : total;
    // the string of the partition starting at g0 and its first position
    auto owner = [&](int64_t g0, int32_t &sidx, int64_t &sbeg) {
        const TileDesc &d = td[g0 / TP];
        if (d.ns >= 0) {
            int t = 0;
            for (int j = 1; j < d.ns; j++) t += (d.off[j] <= g0) ? 1 : 0;
            sidx = d.s0 + t;
            sbeg = d.off[t];
        } else {
            sidx = owner_of(off, n, g0);
            sbeg = off[sidx];
        }
    };
    if constexpr (CROSS) {
        static_assert(!STAGED, "partitions that run past their tile are read directly");
        __syncthreads();  // the table is in place
        const int64_t nw = (total + 63) / 64;
        for (int64_t c = (int64_t)blockIdx.x * REC_THREADS + threadIdx.x; c < R;
             c += (int64_t)gridDim.x * REC_THREADS) {
            const int64_t g0 = apos[2 * c], k = apos[2 * c + 1], rho = c / ntiles;
            if (g0 < 0) continue;  // a tile without flags
            // the next flagged position after g0 (past its tile), else the end of the input
            const uint64_t *bm = bitmap + rho * bm_stride;
            int64_t wd = g0 >> 6, g1 = total;
            uint64_t bw = (g0 & 63) == 63 ? 0ull : bm[wd] & (~0ull << ((g0 & 63) + 1));
            while (true) {
                if (bw) {
                    g1 = 64 * wd + __ffsll((unsigned long long)bw) - 1;
                    break;
                }
                if (++wd >= nw) break;
                bw = bm[wd];
            }
            int32_t sidx;
            int64_t sbeg;
            owner(g0, sidx, sbeg);
            const int64_t L = g1 - g0;
            const uint64_t h = hash((uint64_t)L, g0, g1, gend, gsym, gword);  // L < 2^31 < p
            key[k] = mix64(h ^ salt_f);
            val[k] = ((uint64_t)(uint32_t)sidx << 32) | (uint64_t)(uint32_t)(g0 - sbeg);
            if (len) len[k] = (uint32_t)L;
        }
        return;
    }
    if constexpr (!STAGED) {
        __syncthreads();  // the table is in place
        for (int64_t k = (int64_t)blockIdx.x * REC_THREADS + threadIdx.x; k < R;
             k += (int64_t)gridDim.x * REC_THREADS) {
            const int64_t g0 = apos[k], g1 = apos[k + 1];
            int32_t sidx;
            int64_t sbeg;
            owner(g0, sidx, sbeg);
            const int64_t L = g1 - g0;
            const uint64_t h = hash((uint64_t)L, g0, g1, gend, gsym, gword);  // L < 2^31 < p
            key[k] = mix64(h ^ salt_f);
            val[k] = ((uint64_t)(uint32_t)sidx << 32) | (uint64_t)(uint32_t)(g0 - sbeg);
            if (len) len[k] = (uint32_t)L;
        }
        return;
    }
    // symbols per staged word, and the alignment of the staged range
    constexpr int SPW = PACKED ? 16 : 4;
    for (int64_t kb = (int64_t)blockIdx.x * REC_THREADS; kb < R;
         kb += (int64_t)gridDim.x * REC_THREADS) {
        const int64_t kend = min<int64_t>(kb + REC_THREADS, R);
        const int64_t sb = apos[kb] & ~(int64_t)(SPW - 1);  // word-aligned start of the range
        const int64_t nwords = (apos[kend] - sb + SPW - 1) / SPW;
        const bool staged = (PACKED || aligned4) && nwords <= REC_STAGE_WORDS;
        __syncthreads();  // the table is in place; the previous sweep is done with the stage
        if (staged) {
            for (int64_t i = threadIdx.x; i < nwords; i += REC_THREADS) {
                const int64_t gp = sb + SPW * i;
                uint32_t v;
                if (gp + SPW <= gend) {
                    v = w[gp / SPW];
                } else {
                    v = 0;
                    if constexpr (!PACKED)
                        for (int bb = 0; bb < 4; bb++)
                            if (gp + bb < total) v |= (uint32_t)chars[gp + bb] << (8 * bb);
                }
                stage[i] = v;
            }
        }
        __syncthreads();
        const int64_t k = kb + threadIdx.x;
        if (k >= kend) continue;
        const int64_t g0 = apos[k], g1 = apos[k + 1];
        int32_t sidx;
        int64_t sbeg;
        owner(g0, sidx, sbeg);
        const int64_t L = g1 - g0;
        uint64_t h = (uint64_t)L;  // L < 2^31 < p: already reduced
        if (staged) {
            const uint8_t *sbytes = reinterpret_cast<const uint8_t *>(stage);
            auto ssym = [&](int64_t g) -> uint32_t {
                if constexpr (PACKED) return (uint32_t)(sbytes[(g - sb) >> 2] >> (2 * (g & 3))) & 3u;
                return sbytes[g - sb];
            };
            auto sword = [&](int64_t g) -> uint32_t {
                if constexpr (PACKED) return sbytes[(g - sb) >> 2];
                return stage[(g - sb) >> 2];
            };
            h = hash(h, g0, g1, sb + SPW * nwords, ssym, sword);
        } else {
            h = hash(h, g0, g1, gend, gsym, gword);
        }
        key[k] = mix64(h ^ salt_f);
        val[k] = ((uint64_t)(uint32_t)sidx << 32) | (uint64_t)(uint32_t)(g0 - sbeg);
        if (len) len[k] = (uint32_t)L;
    }
}

// Field helpers for values below p = 2^61 - 1.
__device__ __forceinline__ uint64_t addmod61(uint64_t a, uint64_t b) {
    const uint64_t x = a + b;
    return x >= P61 ? x - P61 : x;
}
__device__ __forceinline__ uint64_t submod61(uint64_t a, uint64_t b) {
    return a >= b ? a - b : a + P61 - b;
}
// Inclusive scans over a wave of 64 lanes by DPP moves: row shifts by 1, 2, 4 and 8
// within rows of 16 lanes, then the row totals broadcast (lane 15 into rows 1 and 3, lane
// 31 into rows 2 and 3).  A lane whose source is outside its row, or a row outside the
// move's row mask, receives 0, the identity of the scans' operations.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp0(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xF, true);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ uint64_t dpp0_64(uint64_t v) {
    return ((uint64_t)dpp0<CTRL, ROWS>((uint32_t)(v >> 32)) << 32) | dpp0<CTRL, ROWS>((uint32_t)v);
}
__device__ __forceinline__ uint32_t wave_scan_add(uint32_t x) {
    x += dpp0<0x111, 0xF>(x);
    x += dpp0<0x112, 0xF>(x);
    x += dpp0<0x114, 0xF>(x);
    x += dpp0<0x118, 0xF>(x);
    x += dpp0<0x142, 0xA>(x);
    x += dpp0<0x143, 0xC>(x);
    return x;
}
__device__ __forceinline__ uint64_t wave_scan_addmod61(uint64_t x) {
    x = addmod61(x, dpp0_64<0x111, 0xF>(x));
    x = addmod61(x, dpp0_64<0x112, 0xF>(x));
    x = addmod61(x, dpp0_64<0x114, 0xF>(x));
    x = addmod61(x, dpp0_64<0x118, 0xF>(x));
    x = addmod61(x, dpp0_64<0x142, 0xA>(x));
    x = addmod61(x, dpp0_64<0x143, 0xC>(x));
    return x;
}

// pq[d] = B^d and pq[n + 1 + d] = B^-d (binv = B^-1 modulo p), d <= n: square and multiply.
__global__ void k_pow_tables(uint64_t B, uint64_t binv, int n, uint64_t *__restrict__ pq) {
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d > n) return;
    uint64_t pw = 1, qw = 1, b = B, bi = binv;
    for (int e = d; e; e >>= 1) {
        if (e & 1) {
            pw = mulmod61(pw, b);
            qw = mulmod61(qw, bi);
        }
        b = mulmod61(b, b);
        bi = mulmod61(bi, bi);
    }
    pq[d] = pw;
    pq[n + 1 + d] = qw;
}

// Partition records of every repetition from one pass over the anchor tiles (TP positions
// each, TP < REGION).  Over a tile, with tile-relative positions, the field prefix sums
// U[j] = sum_{i < j} (x_i + 1) B^-i are computed once and serve every repetition: a
// partition [a, b) inside the tile has sum_{a <= i < b} (x_i + 1) B^(b-1-i) =
// B^(b-1) (U[b] - U[a]), so Phi = L B^L + B^(b-1) (U[b] - U[a]) with L = b - a, the same
// field element as Horner's rule gives.  Then each wave takes whole repetitions (wave w:
// repetitions w, w + 4, ...): lane l holds the tile's flag word l, the lanes' count
// prefixes rank the flags, which the lanes list in order in the wave's LDS list, and lane
// i makes the record of flags i and i + 1, at the repetition's base (rbase, on the device)
// plus the tile's count prefix (pre) plus i.  The partition of the tile's last flag runs
// past the tile: it goes to the tile's slot of the list for k_records_cross (first
// position, record index; -1: the tile has no flag).  Blocks stay resident and take tiles
// in turn, loading the next tile's symbols, descriptor, flags (of the wave's first two
// repetitions) and record bases while they work on this one.  A thread always takes the
// same tile positions, so it keeps their powers B^-j in registers; B^d (d <= REGION) is
// copied to LDS once per block.  U is stored with one unused slot after every 8 (index
// j + j / 8), so that the lanes' runs of 8 consecutive positions meet different LDS banks.
constexpr int RT_THREADS = 256;
constexpr int RT_WAVES = RT_THREADS / 64;

// a c modulo p for a < p and c < 2^32 (2^64 = 8 modulo p)
__device__ __forceinline__ uint64_t mulsmall61(uint64_t a, uint32_t c) {
    const uint64_t lo = a * (uint64_t)c, hi = __umul64hi(a, (uint64_t)c);
    const uint64_t r = (lo & P61) + (lo >> 61) + (hi << 3);
    return r >= P61 ? r - P61 : r;
}

// LDS writes of a wave's lanes visible to the wave's other lanes
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int REGION, bool PACKED>
__global__ __launch_bounds__(RT_THREADS)
__attribute__((amdgpu_waves_per_eu(REGION == 2048 ? 4 : 2))) void k_records_tiles(
    const uint8_t *__restrict__ chars, int64_t total, int aligned4, const int64_t *__restrict__ off,
    int32_t n, const TileDesc *__restrict__ tdesc, int64_t ntiles, int TP, int bits,
    const uint64_t *__restrict__ bitmap, int64_t bm_stride, const uint32_t *__restrict__ pre,
    int64_t pre_stride, const int64_t *__restrict__ rbase, int reps,
    const uint64_t *__restrict__ pq, uint64_t salt_f, uint64_t *__restrict__ key,
    uint64_t *__restrict__ val, uint32_t *__restrict__ len, int64_t *__restrict__ cross) {
    constexpr int RUN = REGION / RT_THREADS;  // positions per thread: 8 or 16
    static_assert(RUN == 8 || RUN == 16, "positions per thread");
    static_assert(REGION / 64 <= 64, "a tile's flag words fit a wave");
    constexpr int PADN = REGION + 1 + REGION / 8 + 1;  // padded slots of U
    __shared__ uint64_t U[PADN];
    __shared__ uint16_t flist[RT_WAVES][REGION];  // each wave's list of flagged positions
    __shared__ int64_t r0s[64];                    // the tile's record bases, repetitions < 64
    __shared__ uint64_t wtot[RT_WAVES];
    __shared__ TileDesc td;
    auto pad = [](int j) { return j + (j >> 3); };
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t *__restrict__ Pt = pq;  // B^d: a small table, read through the caches
    const uint32_t m = (1u << bits) - 1u;
    const int nwt = TP / 64;  // TP is a multiple of 64
    const int64_t nw = (total + 63) / 64;
    const int j0 = tid * RUN;  // the thread's first tile position
    uint64_t q[RUN];           // B^-(j0 + k)
#pragma unroll
    for (int k = 0; k < RUN; k++) q[k] = pq[REGION + 1 + j0 + k];
    // loads of one tile: the thread's symbols (0 outside the input), the descriptor's words
    // (threads < 32), the record base of repetition `tid` (threads < 64), and flag word
    // `lane` of the region (the tile's words, then the halo's) of repetitions `wave` and
    // `wave + RT_WAVES`
    uint32_t x[RUN], tdw = 0;
    int64_t r0l = 0;
    uint64_t bw0 = 0, bw1 = 0;
    auto load = [&](int64_t tile) {
        const int64_t g = tile * TP + j0;
        if constexpr (PACKED) {
            // 16 symbols per 32-bit word, the first in the low bits; g is a multiple of 8
            // and the caller holds whole words
            const uint32_t *wp = reinterpret_cast<const uint32_t *>(chars);
            const uint32_t wv = (g >> 4) < ((total + 15) >> 4) ? wp[g >> 4] : 0u;
            const int sh = (int)(g & 15) * 2;
#pragma unroll
            for (int k = 0; k < RUN; k++) x[k] = (wv >> (sh + 2 * k)) & 3u;
        } else if (aligned4 && g + RUN <= total) {
            const uint32_t *wp = reinterpret_cast<const uint32_t *>(chars + g);
#pragma unroll
            for (int i = 0; i < RUN / 4; i++) {
                const uint32_t wv = wp[i];
#pragma unroll
                for (int k = 0; k < 4; k++) x[4 * i + k] = (wv >> (8 * k)) & 0xFFu;
            }
        } else {
#pragma unroll
            for (int k = 0; k < RUN; k++) x[k] = g + k < total ? (uint32_t)chars[g + k] : 0u;
        }
        if (tid < 32) tdw = reinterpret_cast<const uint32_t *>(tdesc + tile)[tid];
        if (tid < 64) r0l = tid < reps ? rbase[tid] + (int64_t)pre[tid * pre_stride + tile] : 0;
        const int64_t w = tile * TP / 64 + lane;
        const bool ok = lane < REGION / 64 && w < nw;
        bw0 = (wave < reps && ok) ? bitmap[wave * bm_stride + w] : 0ull;
        bw1 = (wave + RT_WAVES < reps && ok) ? bitmap[(wave + RT_WAVES) * bm_stride + w] : 0ull;
    };
    if ((int64_t)blockIdx.x < ntiles) load(blockIdx.x);
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t ts = tile * TP;
        __syncthreads();  // the previous tile is done with U, td and the bases
        if (tid < 32) reinterpret_cast<uint32_t *>(&td)[tid] = tdw;
        if (tid < 64) r0s[tid] = r0l;
        const uint64_t bc0 = bw0, bc1 = bw1;
        // U: inclusive sums over the thread's positions, then over the wave, then the block;
        // over the whole region, the halo past the tile included (the partition that runs
        // past the tile usually ends there)
        uint64_t v[RUN];
        uint64_t acc = 0;
#pragma unroll
        for (int k = 0; k < RUN; k++) {
            const uint64_t u = mulsmall61(q[k], (x[k] & m) + 1u);
            acc = addmod61(acc, u);
            v[k] = acc;
        }
        // every register of this tile's loads is consumed: the next tile's are issued now
        // and stay in flight while this one is worked on
        if (tile + gridDim.x < ntiles) load(tile + gridDim.x);
        const uint64_t incl = wave_scan_addmod61(acc);
        if (lane == 63) wtot[wave] = incl;
        __syncthreads();
        uint64_t before = submod61(incl, acc);
        for (int w = 0; w < wave; w++) before = addmod61(before, wtot[w]);
        if (tid == 0) U[pad(0)] = 0;
#pragma unroll
        for (int k = 0; k < RUN; k++) U[pad(j0 + k + 1)] = addmod61(before, v[k]);
        __syncthreads();  // U, td and the bases in place
        uint16_t *fl = flist[wave];
        for (int rho = wave, round = 0; rho < reps; rho += RT_WAVES, round++) {
            // lane l: flag word l of the region; the tile's words (lanes < nwt), their count
            // prefix and the tile's flag count
            const int64_t w = ts / 64 + lane;
            const uint64_t rw = round == 0 ? bc0
                              : round == 1 ? bc1
                                           : ((lane < REGION / 64 && w < nw) ? bitmap[rho * bm_stride + w] : 0ull);
            const uint64_t b = lane < nwt ? rw : 0ull;
            const int64_t r0 = rho < 64 ? r0s[rho] : rbase[rho] + (int64_t)pre[rho * pre_stride + tile];
            const uint32_t c = (uint32_t)__popcll(b);
            const uint32_t ic = wave_scan_add(c);
            const int nf = __builtin_amdgcn_readlane((int)ic, 63);
            // The last flag's partition runs past the tile.  When the next flag lies in the
            // region's halo (flag words nwt .. REGION / 64 - 1, the symbols' U in LDS) it is
            // appended to the list, which makes that partition the list's last one; else the
            // tile's slot lists it (-1: done, or no flag) for the per-partition kernel.
            const uint64_t nz = __ballot(b != 0);
            const uint64_t hnz = __ballot(lane >= nwt && rw != 0);
            int64_t *slot = cross + 2 * ((int64_t)rho * ntiles + tile);
            int nl = nf;  // entries of the list
            if (nz == 0 || hnz) {
                if (lane == 0) slot[0] = -1;
                if (nz != 0) {
                    const int hl = __ffsll((unsigned long long)hnz) - 1;
                    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)rw, hl);
                    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(rw >> 32), hl);
                    const uint64_t hbw = ((uint64_t)hi << 32) | lo;
                    if (lane == 0) fl[nf] = (uint16_t)(64 * hl + __ffsll((unsigned long long)hbw) - 1);
                    nl = nf + 1;
                }
            } else if (lane == 63 - __clzll((long long)nz)) {
                slot[0] = ts + 64 * lane + 63 - __clzll((long long)b);
                slot[1] = r0 + ic - 1;  // the tile's flags before it: all but itself
            }
            // the flags in order
            {
                int rk = (int)(ic - c);
                for (uint64_t f = b; f; f &= f - 1) fl[rk++] = (uint16_t)(64 * lane + __ffsll((unsigned long long)f) - 1);
            }
            wave_sync();
            for (int i = lane; i + 1 < nl; i += 64) {
                const int a = fl[i], bb = fl[i + 1], L = bb - a;
                const uint64_t phi = addmod61(mulsmall61(Pt[L], (uint32_t)L),
                                              mulmod61(Pt[bb - 1], submod61(U[pad(bb)], U[pad(a)])));
                const int64_t g0 = ts + a;
                int32_t sidx;
                int64_t sbeg;
                if (td.ns >= 0) {
                    int t = 0;
                    for (int j = 1; j < td.ns; j++) t += (td.off[j] <= g0) ? 1 : 0;
                    sidx = td.s0 + t;
                    sbeg = td.off[t];
                } else {
                    sidx = owner_of(off, n, g0);
                    sbeg = off[sidx];
                }
                const int64_t rec = r0 + i;
                key[rec] = mix64(phi ^ salt_f);
                val[rec] = ((uint64_t)(uint32_t)sidx << 32) | (uint64_t)(uint32_t)(g0 - sbeg);
                if (len) len[rec] = (uint32_t)L;
            }
            wave_sync();  // the list is read before the wave's next repetition replaces it
        }
    }
}

void RecBuf::reserve(int64_t need, hipStream_t s) {
    if (need <= cap) return;
    int64_t nc = std::max<int64_t>(need, cap + cap / 2);
    auto get = [&](size_t bytes) -> void * { return ws ? ws->get(bytes) : dev_alloc(bytes, alloc); };
    uint64_t *k2 = (uint64_t *)get((size_t)nc * 8);
    uint64_t *v2 = (uint64_t *)get((size_t)nc * 8);
    uint32_t *l2 = with_len ? (uint32_t *)get((size_t)nc * 4) : nullptr;
    if (count > 0) {
        MJ_HIP(hipMemcpyAsync(k2, key, (size_t)count * 8, hipMemcpyDeviceToDevice, s));
        MJ_HIP(hipMemcpyAsync(v2, val, (size_t)count * 8, hipMemcpyDeviceToDevice, s));
        if (with_len) MJ_HIP(hipMemcpyAsync(l2, len, (size_t)count * 4, hipMemcpyDeviceToDevice, s));
        MJ_HIP(hipStreamSynchronize(s));
    }
    if (!ws) {
        dev_free(key, alloc); dev_free(val, alloc); dev_free(len, alloc);
    }
    key = k2; val = v2; len = l2; cap = nc;
}

void RecBuf::release() {
    if (!ws) {
        dev_free(key, alloc); dev_free(val, alloc); dev_free(len, alloc);
    }
    key = val = nullptr; len = nullptr; cap = count = 0;
}

// Anchors and string starts of every repetition: their bitmaps (nw + 1 words each) and
// per-tile counts (ntiles + 1 each) in one workspace block apiece, filled by one launch of
// the tile kernel over all repetitions, then by the wide-radius kernels per repetition.
static void anchor_launch(const DevStrings &d, const PartitionParams &p, int reps, int TP, int H,
                          int region, int64_t ntiles, const TileDesc *ts, Workspace &ws,
                          hipStream_t s, std::vector<uint64_t *> &bitmap,
                          std::vector<uint32_t *> &tcount) {
    const int64_t nw = (d.total + 63) / 64;
    const int code_bits = p.q * d.bits;
    const int aligned4 = ((uintptr_t)d.chars & 3) == 0 ? 1 : 0;
    const int packed = d.packing == MJ_PACK_2BIT ? 1 : 0;
    uint64_t *bm_all = ws.get_n<uint64_t>((size_t)reps * (nw + 1));
    uint32_t *tc_all = ws.get_n<uint32_t>((size_t)reps * (ntiles + 1));
    for (int rho = 0; rho < reps; rho++) {
        bitmap[rho] = bm_all + (int64_t)rho * (nw + 1);
        tcount[rho] = tc_all + (int64_t)rho * (ntiles + 1);
    }
    // rank tables one after another, each on a 16-byte boundary (with 16 bytes of slack)
    const int rstride = code_bits <= RANK_MAX_BITS ? ((1 << code_bits) + 7) & ~7 : 0;
    uint16_t *rank = rstride ? ws.get_n<uint16_t>((size_t)reps * rstride + 8) : nullptr;
    if (rank) {
        const int nc = 1 << code_bits;
        for (int rho = 0; rho < reps; rho++) {
            const uint64_t salt = mix64(p.seed + (uint64_t)rho + GAMMA);
            hipLaunchKernelGGL(k_rank_table, dim3((nc + 3) / 4), dim3(256), 0, s, nc, salt,
                               p.pi_table, rank + (int64_t)rho * rstride);
            MJ_LAUNCH_CHECK();
        }
    }
    const size_t rank_lds = rank ? ((size_t)2 << code_bits) + 16 : 0;
#define MJ_ANCHORS(R, V, T)                                                                     \
    hipLaunchKernelGGL((k_anchor_tiles<R, V, T>), dim3((unsigned)ntiles), dim3(AT_THREADS), rank_lds, s, \
                       d.chars, d.offsets, d.n, d.total, p.q, d.bits, p.seed, reps, p.pi_table, \
                       rank, rstride, d.rr, TP, H, ts, aligned4, packed, bm_all, nw + 1, tc_all, \
                       ntiles + 1)
    if (rank) {
        if (region == 2048) MJ_ANCHORS(2048, uint32_t, false); else MJ_ANCHORS(4096, uint32_t, false);
    } else if (p.pi_table) {
        if (region == 2048) MJ_ANCHORS(2048, uint64_t, true); else MJ_ANCHORS(4096, uint64_t, true);
    } else {
        if (region == 2048) MJ_ANCHORS(2048, uint64_t, false); else MJ_ANCHORS(4096, uint64_t, false);
    }
#undef MJ_ANCHORS
    MJ_LAUNCH_CHECK();
    const WideBufs wb = wide_setup(d, p.q, ws, s);
    for (int rho = 0; rho < reps; rho++)
        wide_anchors(d, wb, p, mix64(p.seed + (uint64_t)rho + GAMMA), TP, bitmap[rho], tcount[rho], s);
}

// Record bases of the repetitions and the record total, from the repetitions' scanned
// anchor-tile counts (pre_all holds reps arrays of ntiles + 1 words, the last one each
// repetition's count).
__global__ void k_rep_bases(const uint32_t *pre_all, int reps, int64_t ntiles, int64_t *base,
                            int64_t *total) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    int64_t acc = 0;
    for (int r = 0; r < reps; r++) {
        base[r] = acc;
        acc += pre_all[(int64_t)r * (ntiles + 1) + ntiles];
    }
    *total = acc;
}

// Persistent grid of a kernel: the workgroups that fit the device at once.
template <class K>
static unsigned resident_grid(K kern, int threads) {
    int dev = 0, cus = 0, per = 0;
    MJ_HIP(hipGetDevice(&dev));
    MJ_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    MJ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, threads, 0));
    return (unsigned)std::max(1, cus * std::max(1, per));
}

// Records of every repetition.  bm_all / pre_all hold the repetitions' anchor bitmaps and
// tile count prefixes one after another (strides nw + 1 and ntiles + 1); rbase their first
// record indices (device).  Several repetitions: the tile kernel, which takes the symbols
// once for all of them, then the partitions that run past their tile.  One repetition:
// the flagged positions in order, then Horner's rule per partition (8 symbols per step from
// chunk tables: cheaper per symbol than the tile kernel's prefix sums when nothing is
// shared); rcap bounds its partitions and stage says whether to stage their symbols.
static void records_launch(const DevStrings &d, const PartitionParams &p, int reps, int TP,
                           int region, int64_t ntiles, const TileDesc *ts, const uint64_t *bm_all,
                           const uint32_t *pre_all, const int64_t *rbase, int64_t rcap, bool stage,
                           uint64_t *key, uint64_t *val, uint32_t *len, Workspace &ws,
                           hipStream_t s) {
    const int64_t nw = (d.total + 63) / 64;
    const int aligned4 = ((uintptr_t)d.chars & 3) == 0 ? 1 : 0;
    const int packed = d.packing == MJ_PACK_2BIT ? 1 : 0;
    const uint64_t B = 2 + mix64(p.seed ^ GAMMA_B) % (P61 - 3);
    const uint64_t salt_f = mix64(p.seed + GAMMA);
    auto mulp = [](uint64_t a, uint64_t b) { return (uint64_t)(((unsigned __int128)a * b) % P61); };
    // Horner steps of 8 symbols (see k_phi_table): power tables, and for b <= 2 tables of
    // all 4-symbol chunks before them (at most 2,048 entries)
    // (2-bit packed input with b = 1 has chunks of 2-bit fields, not 4-bit codes: the
    // power tables serve it)
    const int pt = (d.bits > 2 || (packed && d.bits != 2)) ? 1 : 0;
    uint64_t B4 = 1;
    for (int i = 0; i < 4; i++) B4 = mulp(B4, B);
    const uint64_t B8 = mulp(B4, B4);
    const int nc = (pt ? 0 : 2 << (4 * d.bits)) + (8 << d.bits);
    uint64_t *phi_table = ws.get_n<uint64_t>(nc);
    hipLaunchKernelGGL(k_phi_table, dim3((nc + 255) / 256), dim3(256), 0, s, nc, d.bits, B, pt,
                       packed, phi_table);
    MJ_LAUNCH_CHECK();
    if (reps == 1) {
        int64_t *apos = ws.get_n<int64_t>(rcap + 1);
        hipLaunchKernelGGL(k_anchor_scatter, dim3((unsigned)ntiles), dim3(64), 0, s, bm_all, nw,
                           TP / 64, pre_all, ntiles, apos, d.total);
        MJ_LAUNCH_CHECK();
        auto kern = packed ? (stage ? k_records<true, true> : k_records<false, true>)
                           : (stage ? k_records<true, false> : k_records<false, false>);
        hipLaunchKernelGGL(kern, dim3(grid_for(rcap, REC_THREADS, 65535)), dim3(REC_THREADS),
                           (size_t)nc * 8, s, apos, rcap, (int64_t)0, (const uint64_t *)nullptr,
                           (int64_t)0, d.offsets, d.n, d.chars, d.total, aligned4, ts, TP, B, salt_f,
                           phi_table, pt, d.bits, B4, B8, key, val, len, pre_all + ntiles, rbase);
        MJ_LAUNCH_CHECK();
        return;
    }
    uint64_t binv = 1;  // B^(p - 2) = B^-1 (p prime)
    for (uint64_t e = P61 - 2, bb = B; e; e >>= 1, bb = mulp(bb, bb))
        if (e & 1) binv = mulp(binv, bb);
    uint64_t *pq = ws.get_n<uint64_t>(2 * ((size_t)region + 1));
    hipLaunchKernelGGL(k_pow_tables, dim3((region + 256) / 256), dim3(256), 0, s, B, binv, region, pq);
    MJ_LAUNCH_CHECK();
    const int64_t cap = (int64_t)reps * ntiles;  // one partition per tile and repetition, at most
    int64_t *cross = ws.get_n<int64_t>(2 * (size_t)cap + 2);
#define MJ_RT(R, PK)                                                                              \
    do {                                                                                          \
        static const unsigned grid_ = resident_grid(k_records_tiles<R, PK>, RT_THREADS);          \
        hipLaunchKernelGGL((k_records_tiles<R, PK>), dim3((unsigned)std::min<int64_t>(ntiles, grid_)), \
                           dim3(RT_THREADS), 0, s, d.chars, d.total, aligned4, d.offsets, d.n, ts, \
                           ntiles, TP, d.bits, bm_all, nw + 1, pre_all, ntiles + 1, rbase, reps, pq, \
                           salt_f, key, val, len, cross);                                         \
    } while (0)
    if (region == 2048) {
        if (packed) MJ_RT(2048, true); else MJ_RT(2048, false);
    } else {
        if (packed) MJ_RT(4096, true); else MJ_RT(4096, false);
    }
#undef MJ_RT
    MJ_LAUNCH_CHECK();
    auto kern = packed ? k_records<false, true, true> : k_records<false, false, true>;
    hipLaunchKernelGGL(kern, dim3(grid_for(cap, REC_THREADS, 65535)), dim3(REC_THREADS),
                       (size_t)nc * 8, s, cross, cap, ntiles, bm_all, nw + 1, d.offsets, d.n,
                       d.chars, d.total, aligned4, ts, TP, B, salt_f, phi_table, pt, d.bits, B4,
                       B8, key, val, len, (const uint32_t *)nullptr, (const int64_t *)nullptr);
    MJ_LAUNCH_CHECK();
}

int64_t partition_records(const DevStrings &d, const PartitionParams &p, int32_t halo, RecBuf &out,
                          Workspace &ws, hipStream_t s, uint64_t *host_scratch, KTimer *kt) {
    if (d.total == 0) return 0;
    const int reps = std::max(1, p.reps);
    int H = std::max<int32_t>(halo, 1);  // radii above WIDE_R take the wide path
    // the smaller region (more workgroups per CU) when the halo leaves room for 1024+ positions
    const int region = (2048 - 2 * H >= 1024) ? 2048 : 4096;
    int TP = ((region - 2 * H) / 64) * 64;  // whole bitmap words per tile
    int64_t ntiles = (d.total + TP - 1) / TP;
    if (ntiles > 0x7FFFFFFFLL) throw Error(MJ_ECAPACITY, "too many tiles");
    // flagged positions are string starts plus strict minima of radius >= 1 (at most every
    // other position); their ranks are 32-bit
    if ((int64_t)d.n + d.total / 2 + 2 > 0xFFFFFFF0LL)
        throw Error(MJ_ECAPACITY, "more than 2^32 partitions per repetition");
    if ((size_t)reps * 4 + 4 > HOST_SCRATCH_BYTES / 2) throw Error(MJ_EINVAL, "too many repetitions");

    // phase 1: anchors of every repetition (Pi seeded with seed + rho), their counts
    int th = kt ? kt->begin(KTimer::ANCHORS, s) : -1;
    TileDesc *ts = ws.get_n<TileDesc>(ntiles + 1);
    hipLaunchKernelGGL(k_tile_desc, dim3((unsigned)((ntiles + 255) / 256)), dim3(256), 0, s,
                       d.offsets, d.rr, d.n, d.total, ntiles, TP, H, region, p.q, ts);
    MJ_LAUNCH_CHECK();
    std::vector<uint64_t *> bitmap(reps);
    std::vector<uint32_t *> tcount(reps);  // per tile: flagged positions
    anchor_launch(d, p, reps, TP, H, region, ntiles, ts, ws, s, bitmap, tcount);
    if (kt) kt->end(th, s, 1);
    // their scans, one after another (ntiles + 1 words each, the last the repetition's count)
    uint32_t *pre_all = ws.get_n<uint32_t>((size_t)reps * (ntiles + 1));
    for (int rho = 0; rho < reps; rho++) {
        uint32_t *pre = pre_all + (int64_t)rho * (ntiles + 1);
        exclusive_scan_u32(tcount[rho], pre, ntiles, ws, s);
        MJ_HIP(hipMemcpyAsync((uint8_t *)host_scratch + 4 * rho, pre + ntiles, 4,
                              hipMemcpyDeviceToHost, s));
    }
    // the symbol check of the plane packing comes back with the counts
    uint32_t *sym_err_h = (uint32_t *)host_scratch + reps;
    *sym_err_h = 0;
    if (d.symbol_err)
        MJ_HIP(hipMemcpyAsync(sym_err_h, d.symbol_err, 4, hipMemcpyDeviceToHost, s));
    MJ_HIP(hipStreamSynchronize(s));
    if (*sym_err_h) throw Error(MJ_EINVAL, "a symbol code is not below sigma");
    std::vector<int64_t> R(reps);
    int64_t total = 0;
    for (int rho = 0; rho < reps; rho++) {
        uint32_t v;
        memcpy(&v, (const uint8_t *)host_scratch + 4 * rho, 4);
        R[rho] = v;
        total += v;
    }

    // phase 2: one reservation, then the records of every repetition
    const int64_t base0 = out.count;
    out.reserve(base0 + total + 1, s);
    int64_t *base_dev = ws.get_n<int64_t>(reps + 2);
    hipLaunchKernelGGL(k_rep_bases, dim3(1), dim3(64), 0, s, pre_all, reps, ntiles, base_dev,
                       base_dev + reps + 1);
    MJ_LAUNCH_CHECK();
    if (total > 0) {
        int tr = kt ? kt->begin(KTimer::RECORDS, s) : -1;
        // stage the symbols when partitions average 24 symbols or more
        records_launch(d, p, reps, TP, region, ntiles, ts, bitmap[0], pre_all, base_dev, total,
                       d.total >= 24 * total, out.key + base0, out.val + base0,
                       out.with_len ? out.len + base0 : nullptr, ws, s);
        if (kt) kt->end(tr, s, 1);
    }
    out.count = base0 + total;
    return total;
}

int64_t partition_records_streamed(const DevStrings &d, const PartitionParams &p, const SetupInfo &si,
                                   uint64_t *key, uint64_t *val, int64_t *R_dev, Workspace &ws,
                                   hipStream_t s, KTimer *kt) {
    const int reps = std::max(1, p.reps);
    const int64_t bound = si.rec_bound;  // partitions of one repetition, at most
    if (d.total == 0 || bound == 0) {
        fill_u64(reinterpret_cast<uint64_t *>(R_dev), 0, 1, s);
        return 0;
    }
    int H = std::max<int32_t>(si.halo, 1);  // radii above WIDE_R take the wide path
    const int region = (2048 - 2 * H >= 1024) ? 2048 : 4096;
    int TP = ((region - 2 * H) / 64) * 64;
    int64_t ntiles = (d.total + TP - 1) / TP;
    if (ntiles > 0x7FFFFFFFLL) throw Error(MJ_ECAPACITY, "too many tiles");
    if ((int64_t)d.n + d.total / 2 + 2 > 0xFFFFFFF0LL)
        throw Error(MJ_ECAPACITY, "more than 2^32 partitions per repetition");

    int th = kt ? kt->begin(KTimer::ANCHORS, s) : -1;
    TileDesc *ts = ws.get_n<TileDesc>(ntiles + 1);
    hipLaunchKernelGGL(k_tile_desc, dim3((unsigned)((ntiles + 255) / 256)), dim3(256), 0, s,
                       d.offsets, d.rr, d.n, d.total, ntiles, TP, H, region, p.q, ts);
    MJ_LAUNCH_CHECK();
    std::vector<uint64_t *> bitmap(reps);
    std::vector<uint32_t *> tcount(reps);
    uint32_t *pre_all = ws.get_n<uint32_t>((size_t)reps * (ntiles + 1));
    anchor_launch(d, p, reps, TP, H, region, ntiles, ts, ws, s, bitmap, tcount);
    if (kt) kt->end(th, s, 1);
    for (int rho = 0; rho < reps; rho++)
        exclusive_scan_u32(tcount[rho], pre_all + (int64_t)rho * (ntiles + 1), ntiles, ws, s);
    int64_t *base_dev = ws.get_n<int64_t>(reps + 1);
    hipLaunchKernelGGL(k_rep_bases, dim3(1), dim3(64), 0, s, pre_all, reps, ntiles, base_dev, R_dev);
    MJ_LAUNCH_CHECK();

    int tr = kt ? kt->begin(KTimer::RECORDS, s) : -1;
    // partitions average about half the bound's length (the bound counts anchors r + 1
    // apart, Lemma 1 expects them 2r + 1 apart): stage the symbols when that is 24 or more
    records_launch(d, p, reps, TP, region, ntiles, ts, bitmap[0], pre_all, base_dev, bound,
                   d.total >= 12 * bound, key, val, nullptr, ws, s);
    if (kt) kt->end(tr, s, 1);
    return bound * reps;
}

}  // namespace mj
