// Verification (Alg. 3; Sec. 3): decide ED(x, y) <= K for every candidate pair.
//
// Bit-parallel path (one pair per lane).  The longer string is the pattern (rows, length
// m), the shorter the text (columns, length n), d = m - n <= K.  A path of cost <= K that
// visits diagonal k = i - j makes at least |k| + |d - k| edits, so it stays within the
// K + 1 diagonals lo = ceil((d-K)/2) <= k <= hi = floor((d+K)/2) (Ukkonen's band, tightened
// by the length difference).  Column j keeps the vertical deltas of a window of 32-bit
// words of rows (word w holds rows 32w+1 .. 32w+32).  Columns come in blocks: a first
// block of phi = ((-lo-1) mod 32) + 1 columns, then blocks of 32; the window moves down one
// word between blocks, and phi puts the band's top row lo + (first column of the block)
// on a word boundary at every move.  The window then covers rows j+lo .. j+hi of every
// column j with 1 + ceil((hi-lo)/32) <= ceil(K/32) + 1 words.  Each column applies Myers' bit-vector
// recurrence for global edit distance (hin = +1 at the top) to the whole window as one
// multi-word integer.  Rows above the window are treated as one more than their left
// neighbour, a word entering at the bottom as one more than the row above it, and rows
// above the first pattern row as never-matching rows: every such value is at least the
// true distance, and every cell on an optimal path of cost <= K lies inside the window,
// so the computed value at (m, n) is <= K exactly when ED <= K.  The same holds for the
// early exit: when every window value exceeds K the pair is rejected.
//
// Pattern and text symbols come from bit planes (plane p holds bit p of each symbol),
// so the match mask of 32 pattern rows against one text symbol is the AND over planes
// of XNOR(plane word, text bit), one v_bitop3 per plane.
//
// Wide path (K above the register-resident window): one wavefront per pair computes the
// banded dynamic program row by row, saturated at K+1; the left-to-right dependency of
// a row is resolved with a wavefront prefix-min scan.
#include <string.h>

#include <algorithm>

#include "mj_common.h"
#include "verify_common.h"

namespace mj {

static unsigned grid_for(int64_t n, int block, unsigned cap = 65535u) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    return (unsigned)std::min<int64_t>(g, cap);
}

int verify_planes(int bits) {
    if (bits <= 2) return 2;
    if (bits <= 4) return 4;
    if (bits <= 6) return 6;
    return 8;
}

// ceil(K/32) handled by the bit-parallel kernels (K <= 416); a window of c + 1 words
constexpr int BP_MAX_C = 13;

template <int NW, int NP>
__global__ __launch_bounds__(256) void k_verify_bp(const uint64_t *__restrict__ pairs,
                                                   const int64_t *__restrict__ sel, int64_t n,
                                                   VSet A, VSet B, int kmode,
                                                   uint8_t *__restrict__ flags,
                                                   unsigned long long *cells) {
    int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t my_cells = 0;
    if (it < n) {
        int64_t pi = sel ? sel[it] : it;
        uint64_t pr = pairs[pi];
        int32_t ia = (int32_t)(pr >> 32), ib = (int32_t)(uint32_t)pr;
        int32_t ma = A.len[ia], mb = B.len[ib];
        int32_t K = kmode == 0 ? max(A.kk[ia], B.kk[ib]) : A.kk[ia];
        // pattern X (rows) = longer string, text Y (columns) = shorter
        bool a_is_x = ma >= mb;
        const uint32_t *PX = a_is_x ? A.planes : B.planes;
        const uint32_t *PY = a_is_x ? B.planes : A.planes;
        int64_t offx = a_is_x ? A.off[ia] : B.off[ib];
        int64_t offy = a_is_x ? B.off[ib] : A.off[ia];
        int32_t mp = a_is_x ? ma : mb, nt = a_is_x ? mb : ma;
        uint8_t result;
        const int dlen = mp - nt;
        const int blo = -((K - dlen) >> 1), bhi = (K + dlen) >> 1;  // band diagonals
        const int phi = ((-blo - 1) & 31) + 1;                      // columns of the first block
        const int w0 = ((phi + blo) >> 5) - 1;                      // window word of that block
        if (mp - nt > K) {
            result = 0;
        } else if (nt == 0) {
            result = mp <= K;
        } else if (1 + ((bhi - blo + 31) >> 5) > NW) {
            result = 2;  // not handled by this instance (host bins pairs so this never happens)
        } else {
            uint32_t Pv[NW], Mv[NW], V[NW];
            uint32_t PL[NP][NW];
            int wlo = w0;
#pragma unroll
            for (int s = 0; s < NW; s++) {
                int w = wlo + s;
                bool real = w >= 0;
                Pv[s] = real ? ~0u : 0u;
                Mv[s] = real ? 0u : ~0u;
                V[s] = real ? ~0u : 0u;
#pragma unroll
                for (int p = 0; p < NP; p++)
                    PL[p][s] = real ? load_word<NP>(PX + p, offx + 32 * (int64_t)w) : 0u;
            }
            int S = abs(32 * w0 + 32);  // column 0: row i holds |i| (rows <= 0 are made up)
            bool rejected = false;
            int jb = 0;
            for (int cols = min(phi, nt); jb < nt; jb += cols, cols = min(32, nt - jb)) {
                if (jb > 0) {
                    // early exit: a lower bound of every window value, word by word
                    int Sw = S, lb = S - __popc(Pv[0]);
#pragma unroll
                    for (int s = 1; s < NW; s++) {
                        Sw += __popc(Pv[s]) - __popc(Mv[s]);
                        lb = min(lb, Sw - __popc(Pv[s]));
                    }
                    if (lb > K) {
                        rejected = true;
                        break;
                    }
                    // move the window down one word; the reference row moves to the bottom
                    // of word 1 (for a one-word window, the new word's made-up +1 rows)
                    if constexpr (NW >= 2)
                        S += __popc(Pv[1]) - __popc(Mv[1]);
                    else
                        S += 32;
#pragma unroll
                    for (int s = 0; s + 1 < NW; s++) {
                        Pv[s] = Pv[s + 1];
                        Mv[s] = Mv[s + 1];
                        V[s] = V[s + 1];
#pragma unroll
                        for (int p = 0; p < NP; p++) PL[p][s] = PL[p][s + 1];
                    }
                    wlo++;
                    int w = wlo + NW - 1;
                    Pv[NW - 1] = ~0u;
                    Mv[NW - 1] = 0u;
                    V[NW - 1] = ~0u;
#pragma unroll
                    for (int p = 0; p < NP; p++)
                        PL[p][NW - 1] = load_word<NP>(PX + p, offx + 32 * (int64_t)w);
                }
                uint32_t TY[NP];
#pragma unroll
                for (int p = 0; p < NP; p++) TY[p] = load_word<NP>(PY + p, offy + jb);
                for (int t = 0; t < cols; t++) {
                    uint32_t tb[NP];  // the text symbol's plane bits, each broadcast to a word
#pragma unroll
                    for (int p = 0; p < NP; p++)
                        tb[p] = (uint32_t)__builtin_amdgcn_sbfe((int)TY[p], (unsigned)t, 1u);
                    uint32_t carry = 0, phc = 1, mhc = 0;
                    int dS = 0;
#pragma unroll
                    for (int s = 0; s < NW; s++) {
                        uint32_t eq = V[s];
#pragma unroll
                        for (int p = 0; p < NP; p++) eq = and_xnor(eq, PL[p][s], tb[p]);
                        uint32_t pv = Pv[s], mv = Mv[s];
                        uint32_t xv = eq | mv;
                        uint32_t co;
                        const uint32_t sum = __builtin_addc(eq & pv, pv, carry, &co);
                        carry = co;
                        uint32_t xh = (sum ^ pv) | eq;
                        uint32_t ph = mv | ~(xh | pv);
                        uint32_t mh = pv & xh;
                        if (s == 0) dS = (int)(ph >> 31) - (int)(mh >> 31);
                        uint32_t phs = (ph << 1) | phc;
                        phc = ph >> 31;
                        uint32_t mhs = (mh << 1) | mhc;
                        mhc = mh >> 31;
                        Pv[s] = mhs | ~(xv | phs);
                        Mv[s] = phs & xv;
                    }
                    S += dS;
                }
            }
            my_cells = (uint64_t)min(jb, nt) * (uint64_t)(bhi - blo + 1);
            if (rejected) {
                result = 0;
            } else {
                // value at row mp, relative to the reference row 32*wlo + 32
                int rel = mp - (32 * wlo + 32);
                int val = S;
                if (rel >= 0) {
#pragma unroll
                    for (int s = 1; s < NW; s++) {
                        int cnt = min(32, max(0, 32 + rel - 32 * s));
                        uint32_t mk = cnt >= 32 ? ~0u : ((1u << cnt) - 1u);
                        val += __popc(Pv[s] & mk) - __popc(Mv[s] & mk);
                    }
                } else {
                    uint32_t mk = ~0u << (32 + rel);
                    val -= __popc(Pv[0] & mk) - __popc(Mv[0] & mk);
                }
                result = val <= K;
            }
        }
        flags[pi] = result;
    }
    // wave-reduced cell counter
    for (int d = 32; d >= 1; d >>= 1) {
        uint32_t lo = (uint32_t)my_cells, hi = (uint32_t)(my_cells >> 32);
        lo = __shfl_down(lo, d, 64);
        hi = __shfl_down(hi, d, 64);
        my_cells += ((uint64_t)hi << 32) | lo;
    }
    if ((threadIdx.x & 63) == 0 && my_cells) atomicAdd(cells, (unsigned long long)my_cells);
}

// ---------------------------------------------------------------- wide path
constexpr int DP_MAX_NT = 64;  // cells per lane: band up to 64 * 64 = 4096 (K <= 2047)

// The symbol at global position g, gathered from its bit in each of the np interleaved
// planes (the only copy of the strings the library is sure to hold: the input may be
// 2-bit packed, and an index keeps no symbols).
__device__ __forceinline__ int plane_symbol(const uint32_t *__restrict__ planes, int np, int64_t g) {
    const uint32_t *w = planes + (g >> 5) * np;
    const int b = (int)(g & 31);
    int c = 0;
    for (int p = 0; p < np; p++) c |= (int)((w[p] >> b) & 1u) << p;
    return c;
}

__global__ __launch_bounds__(64) void k_verify_dp(const uint64_t *__restrict__ pairs,
                                                  const int64_t *__restrict__ sel, int64_t n,
                                                  VSet A, VSet B, int kmode, int np,
                                                  uint8_t *__restrict__ flags,
                                                  unsigned long long *cells) {
    const int lane = threadIdx.x;
    for (int64_t it = blockIdx.x; it < n; it += gridDim.x) {
        int64_t pi = sel ? sel[it] : it;
        uint64_t pr = pairs[pi];
        int32_t ia = (int32_t)(pr >> 32), ib = (int32_t)(uint32_t)pr;
        int32_t ma = A.len[ia], mb = B.len[ib];
        int32_t K = kmode == 0 ? max(A.kk[ia], B.kk[ib]) : A.kk[ia];
        // rows over the shorter string x, columns over the longer y
        bool a_short = ma <= mb;
        const uint32_t *XP = a_short ? A.planes : B.planes, *YP = a_short ? B.planes : A.planes;
        const int64_t xo = a_short ? A.off[ia] : B.off[ib], yo = a_short ? B.off[ib] : A.off[ia];
        int32_t mx = a_short ? ma : mb, ny = a_short ? mb : ma;
        uint8_t result = 0;
        const int W = 2 * K + 1;
        const int NT = (W + 63) / 64;
        const int CAP = K + 1;
        uint64_t rows_done = 0;
        if (ny - mx > K) {
            result = 0;
        } else if (NT > DP_MAX_NT) {
            result = 2;
        } else {
            int prev[DP_MAX_NT], cur[DP_MAX_NT];
            for (int t = 0; t < DP_MAX_NT; t++) {
                int d = lane * NT + t;
                int j = d - K;
                prev[t] = (t < NT && d < W && j >= 0 && j <= ny) ? min(j, CAP) : CAP;
            }
            bool ok = true;
            for (int i = 1; i <= mx && ok; i++) {
                int xc = plane_symbol(XP, np, xo + i - 1);
                int up_next = __shfl_down(prev[0], 1, 64);  // first cell of the next lane
                if (lane == 63) up_next = CAP;
                int run = 0x3FFFFFFF;  // lane-local prefix min of U[d] - d
                int pm[DP_MAX_NT];
                for (int t = 0; t < NT; t++) {
                    int d = lane * NT + t;
                    int j = i - K + d;
                    int U;
                    if (d >= W || j < 0 || j > ny) {
                        U = 0x3FFFFFFF;
                    } else if (j == 0) {
                        U = i;
                    } else {
                        int up = (t + 1 < NT) ? prev[t + 1] : up_next;
                        if (d + 1 >= W) up = CAP;
                        int diag = prev[t] + (xc != plane_symbol(YP, np, yo + j - 1) ? 1 : 0);
                        U = min(up + 1, diag);
                    }
                    run = min(run, U - d);
                    pm[t] = run;
                }
                // exclusive prefix min of lane totals
                int ex = run;
                for (int dd = 1; dd < 64; dd <<= 1) {
                    int o = __shfl_up(ex, dd, 64);
                    if (lane >= dd) ex = min(ex, o);
                }
                int excl = __shfl_up(ex, 1, 64);
                if (lane == 0) excl = 0x3FFFFFFF;
                int rmin = CAP;
                for (int t = 0; t < NT; t++) {
                    int d = lane * NT + t;
                    int j = i - K + d;
                    int v = min(pm[t], excl);
                    v = (v >= 0x3FFFFFFF - 4 * W) ? CAP : v + d;
                    v = min(v, CAP);
                    if (d >= W || j < 0 || j > ny) v = CAP;
                    cur[t] = v;
                    rmin = min(rmin, v);
                }
                for (int dd = 32; dd >= 1; dd >>= 1) rmin = min(rmin, __shfl_xor(rmin, dd, 64));
                for (int t = 0; t < NT; t++) prev[t] = cur[t];
                rows_done++;
                if (rmin > K) ok = false;
            }
            if (ok) {
                int dfin = ny - mx + K;
                int owner = dfin / NT, tt = dfin % NT;
                int v = CAP;
                for (int t = 0; t < NT; t++)
                    if (t == tt) v = prev[t];
                v = __shfl(v, owner, 64);
                result = v <= K;
            }
        }
        if (lane == 0) {
            flags[pi] = result;
            // algorithmic work: the K + 1 diagonals a path of cost <= K can visit
            const int dd = ny - mx;
            const uint64_t band = (uint64_t)(((K + dd) >> 1) + ((K - dd) >> 1) + 1);
            atomicAdd(cells, (unsigned long long)(rows_done * band));
        }
    }
}

// ---------------------------------------------------------------- dispatch
// bin of a pair: c = ceil(K/32) for c <= BP_MAX_C (bit-parallel), else the wide path
// Pairs naming a string id outside the collections go to the last bin, which is never
// launched; the host reports them as invalid arguments.  Counts are gathered per block in
// LDS, then added to the global counters once per block.
__global__ void k_bin_pairs(const uint64_t *pairs, int64_t n, VSet A, VSet B, int kmode,
                            uint8_t *bin, uint32_t *counts) {
    constexpr int NBIN = BP_MAX_C + 3;
    __shared__ uint32_t local[NBIN];
    if (threadIdx.x < NBIN) local[threadIdx.x] = 0;
    __syncthreads();
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) {
        uint64_t pr = pairs[i];
        uint32_t ua = (uint32_t)(pr >> 32), ub = (uint32_t)pr;
        int b;
        if (ua >= (uint32_t)A.n || ub >= (uint32_t)B.n) {
            b = BP_MAX_C + 2;
        } else {
            int32_t K = kmode == 0 ? max(A.kk[ua], B.kk[ub]) : A.kk[ua];
            int c = (K + 31) >> 5;
            b = c <= BP_MAX_C ? c : BP_MAX_C + 1;
        }
        bin[i] = (uint8_t)b;
        atomicAdd(&local[b], 1u);
    }
    __syncthreads();
    if (threadIdx.x < NBIN && local[threadIdx.x]) atomicAdd(&counts[threadIdx.x], local[threadIdx.x]);
}

// Scatter pair indices into bin order.  Few bins, so most lanes of a wave share one:
// lanes with equal bins find each other with one ballot per bin bit, each wave counts its
// bins in LDS, and a block reserves its range of each bin with one global atomic.
constexpr int BS_ITEMS = 16;
constexpr int BS_BINS = 16;  // >= BP_MAX_C + 3, a power of two
static_assert(BP_MAX_C + 3 <= BS_BINS, "bin count");

__device__ __forceinline__ uint64_t bin_peers(uint32_t b, uint64_t valid) {
    uint64_t peers = valid;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const bool bit = (b >> k) & 1u;
        const uint64_t m = __ballot(bit);
        peers &= bit ? m : ~m;
    }
    return peers;
}

__global__ __launch_bounds__(256) void k_bin_scatter(const uint8_t *bin, int64_t n,
                                                     const uint32_t *boff, uint32_t *fill,
                                                     int64_t *sel) {
    __shared__ uint32_t wcnt[4][BS_BINS];
    __shared__ uint32_t wbase[4][BS_BINS];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane < BS_BINS) wcnt[wave][lane] = 0;
    __builtin_amdgcn_wave_barrier();
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const int64_t base = (int64_t)blockIdx.x * 256 * BS_ITEMS + (int64_t)wave * 64 * BS_ITEMS;
    uint32_t br[BS_ITEMS];  // bin << 16 | rank inside the wave's span
#pragma unroll
    for (int c = 0; c < BS_ITEMS; c++) {
        const int64_t i = base + (int64_t)c * 64 + lane;
        const bool ok = i < n;
        const uint32_t b = ok ? (uint32_t)bin[i] & (BS_BINS - 1) : 0u;
        const uint64_t peers = bin_peers(b, __ballot(ok));
        const uint32_t before = wcnt[wave][b];
        __builtin_amdgcn_wave_barrier();
        if (ok && (peers & below) == 0) wcnt[wave][b] = before + (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
        br[c] = (b << 16) | (before + (uint32_t)__popcll(peers & below));
    }
    __syncthreads();
    if (threadIdx.x < BS_BINS) {
        const int b = threadIdx.x;
        uint32_t total = 0;
        for (int w = 0; w < 4; w++) total += wcnt[w][b];
        uint32_t acc = total ? boff[b] + atomicAdd(&fill[b], total) : 0u;
        for (int w = 0; w < 4; w++) {
            wbase[w][b] = acc;
            acc += wcnt[w][b];
        }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < BS_ITEMS; c++) {
        const int64_t i = base + (int64_t)c * 64 + lane;
        if (i < n) sel[wbase[wave][br[c] >> 16] + (br[c] & 0xFFFFu)] = i;
    }
}

using BpKernel = void (*)(const uint64_t *, const int64_t *, int64_t, VSet, VSet, int, uint8_t *,
                          unsigned long long *);

template <int NP>
static BpKernel bp_kernel_for(int c) {
    switch (c) {
        case 0: return k_verify_bp<1, NP>;
        case 1: return k_verify_bp<2, NP>;
        case 2: return k_verify_bp<3, NP>;
        case 3: return k_verify_bp<4, NP>;
        case 4: return k_verify_bp<5, NP>;
        case 5: return k_verify_bp<6, NP>;
        case 6: return k_verify_bp<7, NP>;
        case 7: return k_verify_bp<8, NP>;
        case 8: return k_verify_bp<9, NP>;
        case 9: return k_verify_bp<10, NP>;
        case 10: return k_verify_bp<11, NP>;
        case 11: return k_verify_bp<12, NP>;
        case 12: return k_verify_bp<13, NP>;
        default: return k_verify_bp<14, NP>;
    }
}

static BpKernel bp_kernel(int c, int np) {
    switch (np) {
        case 2: return bp_kernel_for<2>(c);
        case 4: return bp_kernel_for<4>(c);
        case 6: return bp_kernel_for<6>(c);
        default: return bp_kernel_for<8>(c);
    }
}


int64_t verify_pairs(const uint64_t *pairs, int64_t n, const DevStrings &A, const DevStrings &B,
                     int kmode, uint8_t *flags, Workspace &ws, hipStream_t s,
                     uint64_t *host_scratch, KTimer *kt, int64_t uniform_k) {
    if (n <= 0) return 0;
    if (A.planes == nullptr || B.planes == nullptr) throw Error(MJ_EINVAL, "strings not packed");
    int np = verify_planes(std::max(A.bits, B.bits));
    VSet va = vset(A), vb = vset(B);
    unsigned long long *cells = (unsigned long long *)ws.get_n<uint64_t>(2);
    fill_u64((uint64_t *)cells, 0, 1, s);
    if (uniform_k >= 0) {
        // every pair has the same threshold and valid ids: one launch, no binning
        int c = (int)((uniform_k + 31) >> 5);
        int th = kt ? kt->begin(KTimer::VERIFY, s) : -1;
        if (c <= BP_MAX_C) {
            hipLaunchKernelGGL(bp_kernel(c, np), dim3(grid_for(n, 256, 0x7FFFFFFF)), dim3(256), 0, s,
                               pairs, (const int64_t *)nullptr, n, va, vb, kmode, flags, cells);
        } else {
            hipLaunchKernelGGL(k_verify_dp, dim3(grid_for(n, 1, 1u << 20)), dim3(64), 0, s, pairs,
                               (const int64_t *)nullptr, n, va, vb, kmode, np, flags, cells);
        }
        MJ_LAUNCH_CHECK();
        if (kt) kt->end(th, s);
        return (int64_t)read_back<uint64_t>((const uint64_t *)cells, s, host_scratch);
    }
    const int NB = BP_MAX_C + 3;  // bit-parallel bins 0..8, wide path, invalid ids
    uint8_t *bin = ws.get_n<uint8_t>(n);
    uint32_t *counts = ws.get_n<uint32_t>(NB + 1);
    uint32_t *boff = ws.get_n<uint32_t>(NB + 1);
    uint32_t *fillc = ws.get_n<uint32_t>(NB + 1);
    int64_t *sel = ws.get_n<int64_t>(n);
    fill_u32(counts, 0, NB, s);
    fill_u32(fillc, 0, NB, s);
    hipLaunchKernelGGL(k_bin_pairs, dim3(grid_for(n, 256, 16384)), dim3(256), 0, s, pairs, n, va, vb,
                       kmode, bin, counts);
    MJ_LAUNCH_CHECK();
    exclusive_scan_u32(counts, boff, NB, ws, s);
    MJ_HIP(hipMemcpyAsync(host_scratch, boff, sizeof(uint32_t) * (NB + 1), hipMemcpyDeviceToHost, s));
    MJ_HIP(hipStreamSynchronize(s));
    uint32_t hoff[NB + 1];
    memcpy(hoff, host_scratch, sizeof(hoff));
    if (hoff[NB] != hoff[NB - 1]) throw Error(MJ_EINVAL, "pair names a string id out of range");
    const int64_t sblocks = (n + 256 * BS_ITEMS - 1) / (256 * BS_ITEMS);
    if (sblocks > 0x7FFFFFFFLL) throw Error(MJ_ECAPACITY, "too many pairs for one verification");
    hipLaunchKernelGGL(k_bin_scatter, dim3((unsigned)sblocks), dim3(256), 0, s, bin, n, boff, fillc,
                       sel);
    MJ_LAUNCH_CHECK();
    for (int b = 0; b < NB - 1; b++) {
        int64_t cnt = (int64_t)hoff[b + 1] - hoff[b];
        if (cnt <= 0) continue;
        const int64_t *bsel = sel + hoff[b];
        int th = kt ? kt->begin(KTimer::VERIFY, s) : -1;
        if (b <= BP_MAX_C) {
            BpKernel kfn = bp_kernel(b, np);
            hipLaunchKernelGGL(kfn, dim3(grid_for(cnt, 256, 0x7FFFFFFF)), dim3(256), 0, s, pairs, bsel,
                               cnt, va, vb, kmode, flags, cells);
        } else {
            hipLaunchKernelGGL(k_verify_dp, dim3(grid_for(cnt, 1, 1u << 20)), dim3(64), 0, s, pairs,
                               bsel, cnt, va, vb, kmode, np, flags, cells);
        }
        MJ_LAUNCH_CHECK();
        if (kt) kt->end(th, s);
    }
    return (int64_t)read_back<uint64_t>((const uint64_t *)cells, s, host_scratch);
}

}  // namespace mj
