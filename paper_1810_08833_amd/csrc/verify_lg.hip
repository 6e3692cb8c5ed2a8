// Batched verification (Alg. 3; Sec. 3): one persistent launch for all candidates.
//
// A pair is owned by a lane group of G lanes; the band window (the K + 1 diagonals a path
// of cost <= K can visit, as in the per-lane kernel) of NW = NWL * G words is split into
// G contiguous chunks, one per lane.  Per column each lane runs Myers'
// bit-vector recurrence on its chunk; the two cross-lane dependencies of a column are
// resolved inside the group: the carry of the multi-word addition with a carry-lookahead
// scan over the lanes (each lane adds with carry-in 0, reports carry-out and whether its
// chunk would propagate a carry, then adds its resolved carry-in), and the bits shifted
// from one chunk into the next.  The window, its column blocks (a first block of phi
// columns, then 32) and its one-word moves between blocks are those of the per-lane
// kernel, so the decision ED <= K is the same.
//
// Groups take pairs from a queue in order of decreasing length (longest first) and,
// whenever their pair ends (accepted, rejected early, or out of columns), refill at the
// next 32-column block boundary, so lanes do not idle behind longer pairs of their wave.
// The queue is split into QUEUES interleaved sub-queues, sub-queue j holding the pairs of
// rank j, j + QUEUES, j + 2 QUEUES, ... in that order, each with a counter on a line of
// its own: device-scope atomics on one address serialise across the chip, so a single
// counter bumped at every refill would pace the whole launch.  A wave starts on the
// sub-queue its number selects and moves to the next one when it finds its own dry.
// The number of lanes per pair G is chosen per (band words, alphabet planes) by timing
// the candidate configurations once per context.
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

// Moves inside a lane group.  Groups of G <= 16 lanes are aligned inside DPP rows of 16
// lanes, so a row shift by d brings lane g the value of lane g - d of its own group for
// every g >= d (the others read 0 and are not used); these run on the VALU, not LDS.
template <int D>
__device__ __forceinline__ uint32_t row_shr(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x110 + D, 0xF, 0xF, true);
}
__device__ __forceinline__ uint32_t row_shl1(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x101, 0xF, 0xF, true);
}
template <int G, int D>
__device__ __forceinline__ uint32_t gshfl_up_c(uint32_t v) {
    if constexpr (G == 1) return v;
    else return row_shr<D>(v);
}
template <int G>
__device__ __forceinline__ uint32_t gshfl_up(uint32_t v, int d) {
    return G > 1 ? (uint32_t)__shfl_up((int)v, d, G) : v;
}
template <int G>
__device__ __forceinline__ uint32_t gshfl_down1(uint32_t v) {
    if constexpr (G == 1) return v;
    else return row_shl1(v);
}
template <int G>
__device__ __forceinline__ int gshfl_xor(int v, int d) {
    return G > 1 ? __shfl_xor(v, d, G) : v;
}

constexpr int QUEUES = 32;
constexpr int QSTRIDE = 64;  // uint64 words between two sub-queue counters (512 bytes)

// The pairs order[0 .. n) with lane groups of G lanes and NWL window words per lane, taken
// from the sub-queues whose counters `next` holds; returns when every sub-queue is dry.
template <int NWL, int G, int NP>
__device__ __forceinline__ void persist_body(const uint64_t *__restrict__ pairs,
                                             const int64_t *__restrict__ order, int64_t n, VSet A,
                                             VSet B, int kmode, uint8_t *__restrict__ flags,
                                             unsigned long long *cells, unsigned long long *next) {
    constexpr int NW = NWL * G;
    const int lane = threadIdx.x & 63;
    const int g = lane & (G - 1);
    const int leader_lane = lane - g;
    bool active = false, exhausted = false;
    // wave-uniform: current sub-queue and how many sub-queues were found dry
    int qj = (int)((blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) % QUEUES);
    int qdry = 0;
    int64_t pi = 0;
    int32_t K = 0, mp = 0, nt = 0, wlo = 0, jb = 0, S = 0, band = 0, phi = 32;
    int64_t offx = 0, offy = 0;
    const uint32_t *PX = nullptr, *PY = nullptr;
    uint32_t Pv[NWL], Mv[NWL], V[NWL], PL[NP][NWL];
    // software pipeline: text words of the current and the next block, and the plane words
    // of the window's next bottom word, loaded one block ahead of their use
    uint32_t TYc[NP], TYn[NP], PLn[NP];
    uint64_t my_cells = 0;
#pragma unroll
    for (int s = 0; s < NWL; s++) {
        Pv[s] = Mv[s] = V[s] = 0;
#pragma unroll
        for (int p = 0; p < NP; p++) PL[p][s] = 0;
    }
    for (;;) {
        // ---- refill: each group without a pair takes the next one
        const bool need = !active && !exhausted;
        const uint64_t req = __ballot(need && g == 0);
        long long got = -1;
        if (req) {
            const int first = __ffsll((unsigned long long)req) - 1;
            const long long qn = n > qj ? (n - qj + QUEUES - 1) / QUEUES : 0;  // sub-queue size
            const long long want = __popcll(req);
            unsigned long long base = 0;
            if (lane == first) base = atomicAdd(next + qj * QSTRIDE, (unsigned long long)want);
            const long long b0 = (long long)__shfl(base, first, 64);
            const long long k = b0 + __popcll(req & ((1ull << lane) - 1));
            if (need && g == 0 && k < qn) got = k * QUEUES + qj;
            if (b0 + want > qn) {  // this sub-queue is dry from now on
                qj = qj + 1 == QUEUES ? 0 : qj + 1;
                if (++qdry == QUEUES) exhausted = true;  // every sub-queue is dry
            }
        }
        got = __shfl(got, leader_lane, 64);
        if (need) {
            if (got < 0 || got >= n) {
                // no pair this time: retried on the next sub-queue unless all are dry
            } else {
                pi = order ? order[got] : got;
                uint64_t pr = pairs[pi];
                int32_t ia = (int32_t)(pr >> 32), ib = (int32_t)(uint32_t)pr;
                int32_t ma = A.len[ia], mb = B.len[ib];
                K = kmode == 0 ? max(A.kk[ia], B.kk[ib]) : A.kk[ia];
                bool a_is_x = ma >= mb;
                PX = a_is_x ? A.planes : B.planes;
                PY = a_is_x ? B.planes : A.planes;
                offx = a_is_x ? A.off[ia] : B.off[ib];
                offy = a_is_x ? B.off[ib] : A.off[ia];
                mp = a_is_x ? ma : mb;
                nt = a_is_x ? mb : ma;
                const int dlen = mp - nt;
                const int blo = -((K - dlen) >> 1), bhi = (K + dlen) >> 1;  // band diagonals
                phi = ((-blo - 1) & 31) + 1;                                // first block's columns
                const int w0 = ((phi + blo) >> 5) - 1;                      // its window word
                uint8_t result = 0;
                bool trivial = true;
                if (mp - nt > K) {
                    result = 0;
                } else if (nt == 0) {
                    result = mp <= K;
                } else if (1 + ((bhi - blo + 31) >> 5) > NW) {
                    result = 2;
                } else {
                    trivial = false;
                }
                if (trivial) {
                    if (g == 0) flags[pi] = result;
                    // a window too small for the band: the call fails (never a silent flag)
                    if (g == 0 && result == 2) atomicOr(cells + 1, 1ull);
                } else {
                    active = true;
                    wlo = w0;
                    jb = 0;
                    S = abs(32 * w0 + 32);  // column 0: row i holds |i| (rows <= 0 made up)
                    band = bhi - blo + 1;
#pragma unroll
                    for (int s = 0; s < NWL; s++) {
                        int w = wlo + g * NWL + s;
                        bool real = w >= 0;
                        Pv[s] = real ? ~0u : 0u;
                        Mv[s] = real ? 0u : ~0u;
                        V[s] = real ? ~0u : 0u;
#pragma unroll
                        for (int p = 0; p < NP; p++)
                            PL[p][s] = real ? load_word<NP>(PX + p, offx + 32 * (int64_t)w) : 0u;
                    }
#pragma unroll
                    for (int p = 0; p < NP; p++) {
                        TYc[p] = load_word<NP>(PY + p, offy);
                        TYn[p] = load_word<NP>(PY + p, offy + phi);
                        // bottom word after the first move: word w0 + NW (read by the last lane)
                        PLn[p] = g == G - 1 ? load_word<NP>(PX + p, offx + 32 * (int64_t)(w0 + NW)) : 0u;
                    }
                }
            }
        }
        if (__all(!active && exhausted)) break;
        if (!active) continue;

        // ---- one block of up to 32 columns
        uint32_t TY[NP];
#pragma unroll
        for (int p = 0; p < NP; p++) TY[p] = TYc[p];
        const int cols = min(jb == 0 ? phi : 32, nt - jb);
        for (int t = 0; t < cols; t++) {
            uint32_t tb[NP];  // the text symbol's plane bits, each broadcast to a word
#pragma unroll
            for (int p = 0; p < NP; p++) tb[p] = (uint32_t)__builtin_amdgcn_sbfe((int)TY[p], (unsigned)t, 1u);
            uint32_t eqv[NWL], sm[NWL];
            uint32_t carry = 0, all1 = ~0u;
#pragma unroll
            for (int s = 0; s < NWL; s++) {
                uint32_t eq = V[s];
#pragma unroll
                for (int p = 0; p < NP; p++) eq = and_xnor(eq, PL[p][s], tb[p]);
                eqv[s] = eq;
                uint32_t co;
                sm[s] = __builtin_addc(eq & Pv[s], Pv[s], carry, &co);  // carry chain in a lane mask
                carry = co;
                all1 &= sm[s];
            }
            if constexpr (G > 1) {
                // carry-lookahead over the group: (carry-out, propagate) combined low to high
                uint32_t cc = carry, pp = (all1 == ~0u) ? 1u : 0u;
                if constexpr (G >= 2) {
                    uint32_t clo = gshfl_up_c<G, 1>(cc), plo = gshfl_up_c<G, 1>(pp);
                    if (g >= 1) { cc = cc | (pp & clo); pp = pp & plo; }
                }
                if constexpr (G >= 4) {
                    uint32_t clo = gshfl_up_c<G, 2>(cc), plo = gshfl_up_c<G, 2>(pp);
                    if (g >= 2) { cc = cc | (pp & clo); pp = pp & plo; }
                }
                if constexpr (G >= 8) {
                    uint32_t clo = gshfl_up_c<G, 4>(cc), plo = gshfl_up_c<G, 4>(pp);
                    if (g >= 4) { cc = cc | (pp & clo); pp = pp & plo; }
                }
                uint32_t cin = gshfl_up_c<G, 1>(cc);
                if (g == 0) cin = 0;
#pragma unroll
                for (int s = 0; s < NWL; s++) {
                    uint32_t co;
                    sm[s] = __builtin_addc(sm[s], 0u, cin, &co);
                    cin = co;
                }
            }
            uint32_t ph[NWL], mh[NWL];
#pragma unroll
            for (int s = 0; s < NWL; s++) {
                uint32_t xh = (sm[s] ^ Pv[s]) | eqv[s];
                ph[s] = Mv[s] | ~(xh | Pv[s]);
                mh[s] = Pv[s] & xh;
            }
            uint32_t phc = 1, mhc = 0;
            if constexpr (G > 1) {
                uint32_t tb = (ph[NWL - 1] >> 31) | ((mh[NWL - 1] >> 31) << 1);
                uint32_t tin = gshfl_up_c<G, 1>(tb);
                if (g != 0) {
                    phc = tin & 1u;
                    mhc = tin >> 1;
                }
            }
            S += (int)(ph[0] >> 31) - (int)(mh[0] >> 31);  // meaningful in the group's lane 0
#pragma unroll
            for (int s = 0; s < NWL; s++) {
                uint32_t xv = eqv[s] | Mv[s];
                uint32_t phs = (ph[s] << 1) | phc;
                phc = ph[s] >> 31;
                uint32_t mhs = (mh[s] << 1) | mhc;
                mhc = mh[s] >> 31;
                Pv[s] = mhs | ~(xv | phs);
                Mv[s] = phs & xv;
            }
        }
        jb += cols;
        if (g == 0) my_cells += (uint64_t)cols * (uint64_t)band;
        const int S0 = __shfl(S, leader_lane, 64);
        int dl[NWL];
        int E = 0;
#pragma unroll
        for (int s = 0; s < NWL; s++) {
            dl[s] = __popc(Pv[s]) - __popc(Mv[s]);
            if (!(g == 0 && s == 0)) E += dl[s];
        }
        if (jb >= nt) {
            // value at row mp, relative to the reference row 32*wlo + 32 (bottom of slot 0)
            int rel = mp - (32 * wlo + 32);
            int part = 0;
            if (rel >= 0) {
#pragma unroll
                for (int s = 0; s < NWL; s++) {
                    int gs = g * NWL + s;
                    if (gs >= 1) {
                        int cnt = min(32, max(0, 32 + rel - 32 * gs));
                        uint32_t mk = cnt >= 32 ? ~0u : ((1u << cnt) - 1u);
                        part += __popc(Pv[s] & mk) - __popc(Mv[s] & mk);
                    }
                }
            } else if (g == 0) {
                uint32_t mk = ~0u << (32 + rel);
                part = -(__popc(Pv[0] & mk) - __popc(Mv[0] & mk));
            }
#pragma unroll
            for (int d = 1; d < G; d <<= 1) part += gshfl_xor<G>(part, d);
            if (g == 0) flags[pi] = (S0 + part) <= K;
            active = false;
            continue;
        }
        // early exit: a lower bound of every window value (word by word, over the group)
        int incl = E;
#pragma unroll
        for (int d = 1; d < G; d <<= 1) {
            int v = (int)gshfl_up<G>((uint32_t)incl, d);
            if (g >= d) incl += v;
        }
        int Sw = S0 + (incl - E);
        int lb = 0x3FFFFFFF;
#pragma unroll
        for (int s = 0; s < NWL; s++) {
            if (!(g == 0 && s == 0)) Sw += dl[s];
            lb = min(lb, Sw - __popc(Pv[s]));
        }
#pragma unroll
        for (int d = 1; d < G; d <<= 1) lb = min(lb, gshfl_xor<G>(lb, d));
        if (lb > K) {
            if (g == 0) flags[pi] = 0;
            active = false;
            continue;
        }
        // move the window down one word: global slot s takes slot s + 1
        int d1;
        if constexpr (NW == 1)
            d1 = 32;
        else if constexpr (NWL >= 2)
            d1 = dl[1];
        else
            d1 = (int)gshfl_down1<G>((uint32_t)dl[0]);
        S += d1;
        uint32_t inP = gshfl_down1<G>(Pv[0]), inM = gshfl_down1<G>(Mv[0]);
        uint32_t inV = gshfl_down1<G>(V[0]);
        uint32_t inL[NP];
#pragma unroll
        for (int p = 0; p < NP; p++) inL[p] = gshfl_down1<G>(PL[p][0]);
#pragma unroll
        for (int s = 0; s + 1 < NWL; s++) {
            Pv[s] = Pv[s + 1];
            Mv[s] = Mv[s + 1];
            V[s] = V[s + 1];
#pragma unroll
            for (int p = 0; p < NP; p++) PL[p][s] = PL[p][s + 1];
        }
        wlo++;
        // next block's text words (prefetched) and the prefetch of the block after it; the
        // bottom word after the following move (word wlo + NW).  Reads past a string's end
        // stay within the padding of the plane arrays.
#pragma unroll
        for (int p = 0; p < NP; p++) {
            TYc[p] = TYn[p];
            TYn[p] = load_word<NP>(PY + p, offy + jb + 32);
        }
        if (g == G - 1) {
            Pv[NWL - 1] = ~0u;
            Mv[NWL - 1] = 0u;
            V[NWL - 1] = ~0u;
#pragma unroll
            for (int p = 0; p < NP; p++) {
                PL[p][NWL - 1] = PLn[p];
                PLn[p] = load_word<NP>(PX + p, offx + 32 * (int64_t)(wlo + NW));
            }
        } else {
            Pv[NWL - 1] = inP;
            Mv[NWL - 1] = inM;
            V[NWL - 1] = inV;
#pragma unroll
            for (int p = 0; p < NP; p++) PL[p][NWL - 1] = inL[p];
        }
    }
    for (int d = 32; d >= 1; d >>= 1) {
        uint32_t lo = (uint32_t)my_cells, hi = (uint32_t)(my_cells >> 32);
        lo = __shfl_down(lo, d, 64);
        hi = __shfl_down(hi, d, 64);
        my_cells += ((uint64_t)hi << 32) | lo;
    }
    if (lane == 0 && my_cells) atomicAdd(cells, (unsigned long long)my_cells);
}

template <int NWL, int G, int NP>
__global__ __launch_bounds__(256) void k_verify_persist(const uint64_t *__restrict__ pairs,
                                                        const int64_t *__restrict__ order,
                                                        int64_t n, VSet A, VSet B, int kmode,
                                                        uint8_t *__restrict__ flags,
                                                        unsigned long long *cells,
                                                        unsigned long long *next,
                                                        const uint32_t *__restrict__ ndev) {
    if (ndev) n = min(n, (int64_t)*ndev);  // the pair count on the device (n: its capacity)
    persist_body<NWL, G, NP>(pairs, order, n, A, B, kmode, flags, cells, next);
}

// ---------------------------------------------------------------- split by columns
// Lanes 2k and 2k + 1 share a pair.  Lane 2k runs the one-lane recurrence over the first
// mid = nt / 2 text columns; lane 2k + 1 runs it over the reversed pattern and the
// reversed remaining text (its cell (i', j') is the forward cell (mp - i', nt - j')).  The
// reversed problem has the same length difference and hence the same band diagonals, so
// each half is the one-lane loop with direction-dependent loads.  Splitting the text at
// column mid (Hirschberg's middle-column decomposition),
//   ED(X, Y) = min over rows i of D(X[0, i), Y[0, mid)) + D(X[i, mp), Y[mid, nt)),
// and an alignment of cost <= K crosses column mid inside the band, where both halves hold
// exact values whenever they are <= K: the decision ED <= K is that of the one-lane kernel.
// A pair's latency halves; texts shorter than 64 columns stay with the first lane alone.
template <int NP>
__device__ __forceinline__ uint32_t load_dir(const uint32_t *plane, int64_t bitpos, bool rev) {
    // forward: symbols bitpos .. bitpos + 31 at bits 0 .. 31; reversed: bit t holds symbol
    // bitpos + 31 - t.  Positions before the start of the planes read as 0.
    uint32_t w;
    if (bitpos >= 0) w = load_word<NP>(plane, bitpos);
    else if (bitpos > -32) w = load_word<NP>(plane, 0) << (uint32_t)(-bitpos);
    else w = 0u;
    return rev ? __builtin_bitreverse32(w) : w;
}

// 32 bits of a padded window (A[0] = 0, A[1 .. NW] = the words, A[NW + 1] = 0) starting
// at bit e of the unpadded words, -32 < e < 32 NW
template <int NW>
__device__ __forceinline__ uint32_t window_bits(const uint32_t (*A)[128], int slot, int e) {
    const int f = e + 32;
    return __builtin_amdgcn_alignbit(A[(f >> 5) + 1][slot], A[f >> 5][slot], (uint32_t)(f & 31));
}

template <int NW, int NP>
__global__ __launch_bounds__(256) void k_verify_bidir(const uint64_t *__restrict__ pairs,
                                                      const int64_t *__restrict__ order,
                                                      int64_t n, VSet A, VSet B, int kmode,
                                                      uint8_t *__restrict__ flags,
                                                      unsigned long long *cells,
                                                      unsigned long long *next,
                                                      const uint32_t *__restrict__ ndev) {
    if (ndev) n = min(n, (int64_t)*ndev);  // the pair count on the device (n: its capacity)
    // meeting of the two halves: the forward and backward windows of each pair's first lane
    __shared__ uint32_t meet[4][NW + 2][128];
    const int lane = threadIdx.x & 63;
    const bool bwd = (lane & 1) != 0;
    const int leader_lane = lane & ~1;
    const int slot = threadIdx.x >> 1;
    bool active = false, exhausted = false, done = false, rej = false, solo = false;
    int lbv = 0;  // lower bound of this half's window values at its current column
    uint8_t solo_res = 0;
    int qj = (int)((blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) % QUEUES);
    int qdry = 0;
    int64_t pi = 0;
    int32_t K = 0, mp = 0, nt = 0, ncols = 0, mid = 0, wlo = 0, jb = 0, S = 0, band = 0;
    int32_t phi = 32, blo = 0, bhi = 0;
    int64_t offx = 0, offy = 0;
    const uint32_t *PX = nullptr, *PY = nullptr;
    uint32_t Pv[NW], Mv[NW], V[NW], PL[NP][NW];
    uint32_t TYc[NP], TYn[NP], PLn[NP];
    uint64_t my_cells = 0;
#pragma unroll
    for (int s = 0; s < NW; s++) {
        Pv[s] = Mv[s] = V[s] = 0;
#pragma unroll
        for (int p = 0; p < NP; p++) PL[p][s] = 0;
    }
    // the half's pattern word w and text word at column j (reversed for the second lane)
    auto xword = [&](int p, int w) -> uint32_t {
        const int64_t pos = bwd ? offx + mp - 32 - 32 * (int64_t)w : offx + 32 * (int64_t)w;
        return load_dir<NP>(PX + p, pos, bwd);
    };
    auto yword = [&](int p, int j) -> uint32_t {
        const int64_t pos = bwd ? offy + nt - 32 - (int64_t)j : offy + (int64_t)j;
        return load_dir<NP>(PY + p, pos, bwd);
    };
    auto swap1 = [](uint32_t v) -> uint32_t {  // the partner lane's value (quad_perm 1,0,3,2)
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);
    };
    for (;;) {
        // ---- resolution of pairs whose halves are both finished, or rejected.  An alignment
        // within the band pays at least the forward bound before the forward lane's column
        // and the backward bound after the backward lane's (disjoint parts of it), so the
        // sum of the two bounds above K rejects the pair as early as one lane would.
        const int plb = (int)swap1((uint32_t)lbv);
        if (active && lbv + plb > K) rej = true;
        const bool pdone = swap1(done ? 1u : 0u) != 0u, prej = swap1(rej ? 1u : 0u) != 0u;
        const bool res_rej = active && (rej || prej);
        const bool res_meet = active && !res_rej && done && pdone && !solo;
        if (__any(res_meet)) {
            uint32_t oP[NW], oM[NW];
#pragma unroll
            for (int s = 0; s < NW; s++) {
                oP[s] = swap1(Pv[s]);
                oM[s] = swap1(Mv[s]);
            }
            const int oS = (int)swap1((uint32_t)S), oW = (int)swap1((uint32_t)wlo);
            if (res_meet && !bwd) {
#pragma unroll
                for (int s = 0; s < NW; s++) {
                    meet[0][s + 1][slot] = Pv[s];
                    meet[1][s + 1][slot] = Mv[s];
                    meet[2][s + 1][slot] = oP[s];
                    meet[3][s + 1][slot] = oM[s];
                }
#pragma unroll
                for (int a = 0; a < 4; a++) {
                    meet[a][0][slot] = 0u;
                    meet[a][NW + 1][slot] = 0u;
                }
                // band rows at column mid, inside the pattern
                const int ilo = max(0, mid + blo), ihi = min(mp, mid + bhi);
                // value of a window at row i from its reference row 32 w + 32 (value Sr)
                auto value_at = [&](int a, int w, int Sr, int i) -> int {
                    const int rel = i - (32 * w + 32);
                    int v = Sr;
                    if (rel >= 0) {
                        for (int e = 32; e < 32 + rel; e += 32) {  // rows 32w + 33 .. i
                            const int cnt = min(32, 32 + rel - e);
                            const uint32_t mk = cnt >= 32 ? ~0u : ((1u << cnt) - 1u);
                            v += __popc(window_bits<NW>(meet[a], slot, e) & mk) -
                                 __popc(window_bits<NW>(meet[a + 1], slot, e) & mk);
                        }
                    } else {  // rows i + 1 .. 32w + 32, all in slot 0
                        const uint32_t mk = ~0u << (32 + rel);
                        v -= __popc(window_bits<NW>(meet[a], slot, 0) & mk) -
                             __popc(window_bits<NW>(meet[a + 1], slot, 0) & mk);
                    }
                    return v;
                };
                int Df = value_at(0, wlo, S, ilo);
                int Db = value_at(2, oW, oS, mp - ilo);
                int best = Df + Db;
                // walk down the band: row i -> i + 1 adds the forward delta of row i + 1
                // (bit i - 32 wlo) and removes the backward delta of row mp - i (bit
                // mp - i - 1 - 32 oW)
                for (int i0 = ilo; i0 < ihi && best > K; i0 += 32) {
                    const int ef = i0 - 32 * wlo;
                    const int eb = mp - i0 - 1 - 32 * oW;  // bit of step 0; later steps go down
                    const uint32_t fP = window_bits<NW>(meet[0], slot, ef);
                    const uint32_t fM = window_bits<NW>(meet[1], slot, ef);
                    const uint32_t bP = __builtin_bitreverse32(window_bits<NW>(meet[2], slot, eb - 31));
                    const uint32_t bM = __builtin_bitreverse32(window_bits<NW>(meet[3], slot, eb - 31));
                    const int steps = min(32, ihi - i0);
                    for (int t = 0; t < steps; t++) {
                        Df += (int)((fP >> t) & 1u) - (int)((fM >> t) & 1u);
                        Db -= (int)((bP >> t) & 1u) - (int)((bM >> t) & 1u);
                        best = min(best, Df + Db);
                    }
                }
                flags[pi] = best <= K ? 1 : 0;
            }
        }
        if (res_rej && !bwd) flags[pi] = 0;
        if (active && !res_rej && done && pdone && solo && !bwd) flags[pi] = solo_res;
        if (res_rej || (active && done && pdone)) {
            active = false;
            done = rej = false;
        }

        // ---- refill: each lane pair without a pair takes the next one
        const bool need = !active && !exhausted;
        const uint64_t req = __ballot(need && !bwd);
        long long got = -1;
        if (req) {
            const int first = __ffsll((unsigned long long)req) - 1;
            const long long qn = n > qj ? (n - qj + QUEUES - 1) / QUEUES : 0;
            const long long want = __popcll(req);
            unsigned long long base = 0;
            if (lane == first) base = atomicAdd(next + qj * QSTRIDE, (unsigned long long)want);
            const long long b0 = (long long)__shfl(base, first, 64);
            const long long k = b0 + __popcll(req & ((1ull << lane) - 1));
            if (need && !bwd && k < qn) got = k * QUEUES + qj;
            if (b0 + want > qn) {
                qj = qj + 1 == QUEUES ? 0 : qj + 1;
                if (++qdry == QUEUES) exhausted = true;
            }
        }
        got = __shfl(got, leader_lane, 64);
        if (need && got >= 0 && got < n) {
            pi = order ? order[got] : got;
            const uint64_t pr = pairs[pi];
            const int32_t ia = (int32_t)(pr >> 32), ib = (int32_t)(uint32_t)pr;
            const int32_t ma = A.len[ia], mb = B.len[ib];
            K = kmode == 0 ? max(A.kk[ia], B.kk[ib]) : A.kk[ia];
            const bool a_is_x = ma >= mb;
            PX = a_is_x ? A.planes : B.planes;
            PY = a_is_x ? B.planes : A.planes;
            offx = a_is_x ? A.off[ia] : B.off[ib];
            offy = a_is_x ? B.off[ib] : A.off[ia];
            mp = a_is_x ? ma : mb;
            nt = a_is_x ? mb : ma;
            const int dlen = mp - nt;
            blo = -((K - dlen) >> 1);
            bhi = (K + dlen) >> 1;
            phi = ((-blo - 1) & 31) + 1;
            const int w0 = ((phi + blo) >> 5) - 1;
            uint8_t result = 0;
            bool trivial = true;
            if (mp - nt > K) {
                result = 0;
            } else if (nt == 0) {
                result = mp <= K;
            } else if (1 + ((bhi - blo + 31) >> 5) > NW) {
                result = 2;
            } else {
                trivial = false;
            }
            if (trivial) {
                if (!bwd) flags[pi] = result;
                if (!bwd && result == 2) atomicOr(cells + 1, 1ull);
            } else {
                active = true;
                solo = nt < 64;
                mid = solo ? nt : nt >> 1;
                ncols = bwd ? nt - mid : mid;
                done = ncols == 0;
                rej = false;
                lbv = 0;
                wlo = w0;
                jb = 0;
                S = abs(32 * w0 + 32);
                band = bhi - blo + 1;
#pragma unroll
                for (int s = 0; s < NW; s++) {
                    const int w = wlo + s;
                    const bool real = w >= 0;
                    Pv[s] = real ? ~0u : 0u;
                    Mv[s] = real ? 0u : ~0u;
                    V[s] = real ? ~0u : 0u;
#pragma unroll
                    for (int p = 0; p < NP; p++) PL[p][s] = real ? xword(p, w) : 0u;
                }
#pragma unroll
                for (int p = 0; p < NP; p++) {
                    TYc[p] = yword(p, 0);
                    TYn[p] = yword(p, phi);
                    PLn[p] = xword(p, w0 + NW);
                }
            }
        }
        if (__all(!active && exhausted)) break;
        if (!active || done || rej) continue;

        // ---- one block of up to 32 columns of this lane's half
        uint32_t TY[NP];
#pragma unroll
        for (int p = 0; p < NP; p++) TY[p] = TYc[p];
        const int cols = min(jb == 0 ? phi : 32, ncols - jb);
        for (int t = 0; t < cols; t++) {
            uint32_t tb[NP];
#pragma unroll
            for (int p = 0; p < NP; p++) tb[p] = (uint32_t)__builtin_amdgcn_sbfe((int)TY[p], (unsigned)t, 1u);
            uint32_t eqv[NW], sm[NW];
            uint32_t carry = 0;
#pragma unroll
            for (int s = 0; s < NW; s++) {
                uint32_t eq = V[s];
#pragma unroll
                for (int p = 0; p < NP; p++) eq = and_xnor(eq, PL[p][s], tb[p]);
                eqv[s] = eq;
                uint32_t co;
                sm[s] = __builtin_addc(eq & Pv[s], Pv[s], carry, &co);
                carry = co;
            }
            uint32_t ph[NW], mh[NW];
#pragma unroll
            for (int s = 0; s < NW; s++) {
                const uint32_t xh = (sm[s] ^ Pv[s]) | eqv[s];
                ph[s] = Mv[s] | ~(xh | Pv[s]);
                mh[s] = Pv[s] & xh;
            }
            S += (int)(ph[0] >> 31) - (int)(mh[0] >> 31);
            uint32_t phc = 1, mhc = 0;
#pragma unroll
            for (int s = 0; s < NW; s++) {
                const uint32_t xv = eqv[s] | Mv[s];
                const uint32_t phs = (ph[s] << 1) | phc;
                phc = ph[s] >> 31;
                const uint32_t mhs = (mh[s] << 1) | mhc;
                mhc = mh[s] >> 31;
                Pv[s] = mhs | ~(xv | phs);
                Mv[s] = phs & xv;
            }
        }
        jb += cols;
        my_cells += (uint64_t)cols * (uint64_t)band;
        int dl[NW];
#pragma unroll
        for (int s = 0; s < NW; s++) dl[s] = __popc(Pv[s]) - __popc(Mv[s]);
        // a lower bound of every window value
        {
            int Sw = S, lb = 0x3FFFFFFF;
#pragma unroll
            for (int s = 0; s < NW; s++) {
                if (s > 0) Sw += dl[s];
                lb = min(lb, Sw - __popc(Pv[s]));
            }
            lbv = lb;
        }
        if (jb >= ncols) {
            if (solo) {
                // the whole text: the value at row mp decides, as in the one-lane kernel
                const int rel = mp - (32 * wlo + 32);
                int part = 0;
                if (rel >= 0) {
#pragma unroll
                    for (int s = 1; s < NW; s++) {
                        const int cnt = min(32, max(0, 32 + rel - 32 * s));
                        const uint32_t mk = cnt >= 32 ? ~0u : ((1u << cnt) - 1u);
                        part += __popc(Pv[s] & mk) - __popc(Mv[s] & mk);
                    }
                } else {
                    const uint32_t mk = ~0u << (32 + rel);
                    part = -(__popc(Pv[0] & mk) - __popc(Mv[0] & mk));
                }
                solo_res = (S + part) <= K ? 1 : 0;
            }
            done = true;
            continue;
        }
        if (lbv > K) {
            rej = true;
            continue;
        }
        // move the window down one word
        if constexpr (NW == 1) S += 32;
        else S += dl[1];
#pragma unroll
        for (int s = 0; s + 1 < NW; s++) {
            Pv[s] = Pv[s + 1];
            Mv[s] = Mv[s + 1];
            V[s] = V[s + 1];
#pragma unroll
            for (int p = 0; p < NP; p++) PL[p][s] = PL[p][s + 1];
        }
        wlo++;
#pragma unroll
        for (int p = 0; p < NP; p++) {
            TYc[p] = TYn[p];
            TYn[p] = yword(p, jb + 32);
        }
        Pv[NW - 1] = ~0u;
        Mv[NW - 1] = 0u;
        V[NW - 1] = ~0u;
#pragma unroll
        for (int p = 0; p < NP; p++) {
            PL[p][NW - 1] = PLn[p];
            PLn[p] = xword(p, wlo + NW);
        }
    }
    for (int d = 32; d >= 1; d >>= 1) {
        uint32_t lo = (uint32_t)my_cells, hi = (uint32_t)(my_cells >> 32);
        lo = __shfl_down(lo, d, 64);
        hi = __shfl_down(hi, d, 64);
        my_cells += ((uint64_t)hi << 32) | lo;
    }
    if (lane == 0 && my_cells) atomicAdd(cells, (unsigned long long)my_cells);
}

// ---------------------------------------------------------------- configurations
using PersistKernel = void (*)(const uint64_t *, const int64_t *, int64_t, VSet, VSet, int,
                               uint8_t *, unsigned long long *, unsigned long long *,
                               const uint32_t *);
using PersistClassKernel = void (*)(const uint64_t *, const int64_t *, const uint32_t *, VSet, VSet,
                                    int, uint8_t *, unsigned long long *, unsigned long long *);
constexpr int VCLS_NW_MAX = 32;  // the widest band class's window words

constexpr int NWL_CHOICES[] = {1, 2, 3, 4, 5, 6, 7, 8, 9, 11};
// g == BIDIR: two lanes per pair, split by columns (each lane holds the whole window);
// g == CLASSES: lanes per pair and window chosen per pair by its band class
constexpr int BIDIR = VERIFY_BIDIR;
constexpr int CLASSES = VERIFY_CLASSES;
constexpr int G_CHOICES[] = {1, 2, BIDIR, 4, 8, CLASSES};

template <int NWL, int G>
static PersistKernel by_np(int np) {
    switch (np) {
        case 2: return k_verify_persist<NWL, G, 2>;
        case 4: return k_verify_persist<NWL, G, 4>;
        case 6: return k_verify_persist<NWL, G, 6>;
        default: return k_verify_persist<NWL, G, 8>;
    }
}

template <int G>
static PersistKernel by_nwl(int nwl, int np) {
    switch (nwl) {
        case 1: return by_np<1, G>(np);
        case 2: return by_np<2, G>(np);
        case 3: return by_np<3, G>(np);
        case 4: return by_np<4, G>(np);
        case 5: return by_np<5, G>(np);
        case 6: return by_np<6, G>(np);
        case 7: return by_np<7, G>(np);
        case 8: return by_np<8, G>(np);
        case 9: return by_np<9, G>(np);
        default: return by_np<11, G>(np);
    }
}

template <int NW>
static PersistKernel bidir_by_np(int np) {
    switch (np) {
        case 2: return k_verify_bidir<NW, 2>;
        case 4: return k_verify_bidir<NW, 4>;
        case 6: return k_verify_bidir<NW, 6>;
        default: return k_verify_bidir<NW, 8>;
    }
}

static PersistKernel bidir_kernel(int nwl, int np) {
    switch (nwl) {
        case 1: return bidir_by_np<1>(np);
        case 2: return bidir_by_np<2>(np);
        case 3: return bidir_by_np<3>(np);
        case 4: return bidir_by_np<4>(np);
        case 5: return bidir_by_np<5>(np);
        case 6: return bidir_by_np<6>(np);
        case 7: return bidir_by_np<7>(np);
        case 8: return bidir_by_np<8>(np);
        case 9: return bidir_by_np<9>(np);
        default: return bidir_by_np<11>(np);
    }
}

static PersistKernel persist_kernel(int nwl, int g, int np) {
    switch (g) {
        case 1: return by_nwl<1>(nwl, np);
        case 2: return by_nwl<2>(nwl, np);
        case BIDIR: return bidir_kernel(nwl, np);
        case 4: return by_nwl<4>(nwl, np);
        case 8: return by_nwl<8>(nwl, np);
        default: throw Error(MJ_EINVAL, "lanes per pair must be 1, 2, 4, 8 or the column split");
    }
}

// smallest supported NWL with NWL * G >= nw (the whole window per lane for BIDIR), or 0;
// for CLASSES 4 (the widest class's words per lane) when the widest class holds nw words
static int nwl_for(int nw, int g) {
    if (g == CLASSES) return nw <= VCLS_NW_MAX ? 4 : 0;
    const int lanes = g == BIDIR ? 1 : g;
    for (int v : NWL_CHOICES)
        if (v * lanes >= nw) return v;
    return 0;
}

// The window needs ceil(K/32) + 1 words (at most 11 * 8); K <= 2047 keeps c <= 64.
int persist_max_c() { return 64; }

// The configuration of calls too small to time: the most lanes per pair that still gives
// each lane more than one word (one lane when the band fits one word).
int verify_small_call_lanes(int cmax) {
    const int nw = cmax + 1;
    int best = 0;
    for (int g : G_CHOICES)
        if (g != BIDIR && g != CLASSES && nwl_for(nw, g) != 0 && (g == 1 || nwl_for(nw, g / 2) > 1))
            best = g;
    return best;
}

// Calls with fewer pairs use a fixed configuration instead of timing the choices.
constexpr int64_t TUNE_MIN_PAIRS = 4096;

// ---------------------------------------------------------------- longest-first order
constexpr int LPT_BINS = 4096;

__global__ void k_pair_cmax(const uint64_t *pairs, int64_t n, VSet A, VSet B, int kmode,
                            uint32_t *cmax, uint32_t *bad) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    uint32_t m = 0;
    for (; i < n; i += stride) {
        uint64_t pr = pairs[i];
        uint32_t ua = (uint32_t)(pr >> 32), ub = (uint32_t)pr;
        if (ua >= (uint32_t)A.n || ub >= (uint32_t)B.n) {
            atomicOr(bad, 1u);
            continue;
        }
        int32_t K = kmode == 0 ? max(A.kk[ua], B.kk[ub]) : A.kk[ua];
        m = max(m, (uint32_t)((K + 31) >> 5));
    }
    for (int d = 32; d >= 1; d >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, d, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(cmax, m);
}

// Band classes: windows of 2, 4, 8, 16 and 32 words (2 words on one lane, 4 on one, then
// 4 words per lane on 2, 4 and 8 lanes).  A pair's class is the smallest whose window
// holds its band, ceil(K/32) + 1 words.  (Eight classes, adding 3-word lanes for windows
// of 3, 6 and 12 words, made the launch slower: 1.54 against 1.44 ms on protein.)
constexpr int VCLS = 5;
constexpr int VCLS_NW[VCLS] = {2, 4, 8, 16, 32};
constexpr int VCLS_BINS = 512;  // length bins per class
static_assert(VCLS * VCLS_BINS <= LPT_BINS, "class bins");
static_assert(VCLS_NW[VCLS - 1] == VCLS_NW_MAX, "widest class");

__device__ __forceinline__ int pair_class(int32_t K) {
    const int nw = ((K + 31) >> 5) + 1;
    int c = 0;
    while (c + 1 < VCLS && VCLS_NW[c] < nw) c++;
    return c;
}

// The bin of a pair: longest first, or (classes) widest class first, then longest first.
__device__ __forceinline__ int lpt_bin(const uint64_t pr, const VSet &A, const VSet &B, int kmode,
                                       int classes) {
    const uint32_t ia = (uint32_t)(pr >> 32), ib = (uint32_t)pr;
    int32_t nt = min(A.len[ia], B.len[ib]);
    if (!classes) return LPT_BINS - 1 - min(nt >> 4, LPT_BINS - 1);
    const int32_t K = kmode == 0 ? max(A.kk[ia], B.kk[ib]) : A.kk[ia];
    return (VCLS - 1 - pair_class(K)) * VCLS_BINS + VCLS_BINS - 1 - min(nt >> 4, VCLS_BINS - 1);
}

__global__ void k_lpt_hist(const uint64_t *pairs, int64_t n, VSet A, VSet B, int kmode,
                           int classes, uint32_t *cnt, const uint32_t *ndev) {
    if (ndev) n = min(n, (int64_t)*ndev);
    __shared__ uint32_t h[LPT_BINS];
    for (int t = threadIdx.x; t < LPT_BINS; t += blockDim.x) h[t] = 0;
    __syncthreads();
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) atomicAdd(&h[lpt_bin(pairs[i], A, B, kmode, classes)], 1u);
    __syncthreads();
    for (int t = threadIdx.x; t < LPT_BINS; t += blockDim.x)
        if (h[t]) atomicAdd(&cnt[t], h[t]);
}

// Scatter into bin order.  Ranks inside a block come from LDS counters; each block then
// reserves its range of every bin it touches with one global atomic (lengths cluster in
// a few bins, so per-pair global atomics would serialise on them).
constexpr int LPT_ITEMS = 16;
__global__ __launch_bounds__(256) void k_lpt_scatter(const uint64_t *pairs, int64_t n, VSet A,
                                                     VSet B, int kmode, int classes,
                                                     const uint32_t *off, uint32_t *fill,
                                                     int64_t *order, const uint32_t *ndev) {
    if (ndev) n = min(n, (int64_t)*ndev);
    __shared__ uint32_t cnt[LPT_BINS];
    __shared__ uint32_t base[LPT_BINS];
    for (int t = threadIdx.x; t < LPT_BINS; t += blockDim.x) cnt[t] = 0;
    __syncthreads();
    const int64_t first = (int64_t)blockIdx.x * blockDim.x * LPT_ITEMS;
    int bin[LPT_ITEMS];
    uint32_t rank[LPT_ITEMS];
#pragma unroll
    for (int k = 0; k < LPT_ITEMS; k++) {
        const int64_t i = first + (int64_t)k * blockDim.x + threadIdx.x;
        bin[k] = 0;
        rank[k] = 0;
        if (i < n) {
            bin[k] = lpt_bin(pairs[i], A, B, kmode, classes);
            rank[k] = atomicAdd(&cnt[bin[k]], 1u);
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < LPT_BINS; t += blockDim.x)
        if (cnt[t]) base[t] = off[t] + atomicAdd(&fill[t], cnt[t]);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < LPT_ITEMS; k++) {
        const int64_t i = first + (int64_t)k * blockDim.x + threadIdx.x;
        if (i < n) order[base[bin[k]] + rank[k]] = i;
    }
}

// One persistent launch over band classes: a wave takes the pairs of the widest class
// first (with that class's lanes per pair and window) and moves to the next narrower class
// when the current one is dry, so each pair's window fits its own band instead of the
// widest band of the call.  The order holds the classes from the widest down, each
// longest first; off[] (the bin offsets of that order) gives each class's range.
template <int NP>
__global__ __launch_bounds__(256) void k_verify_classes(const uint64_t *__restrict__ pairs,
                                                        const int64_t *__restrict__ order,
                                                        const uint32_t *__restrict__ off, VSet A,
                                                        VSet B, int kmode,
                                                        uint8_t *__restrict__ flags,
                                                        unsigned long long *cells,
                                                        unsigned long long *next) {
    for (int c = VCLS - 1; c >= 0; c--) {
        const int b0 = (VCLS - 1 - c) * VCLS_BINS;
        const int64_t base = off[b0], cnt = (int64_t)off[b0 + VCLS_BINS] - base;
        if (cnt <= 0) continue;
        unsigned long long *nx = next + (int64_t)c * QUEUES * QSTRIDE;
        const int64_t *oc = order + base;
        switch (c) {
            case 0: persist_body<2, 1, NP>(pairs, oc, cnt, A, B, kmode, flags, cells, nx); break;
            case 1: persist_body<4, 1, NP>(pairs, oc, cnt, A, B, kmode, flags, cells, nx); break;
            case 2: persist_body<4, 2, NP>(pairs, oc, cnt, A, B, kmode, flags, cells, nx); break;
            case 3: persist_body<4, 4, NP>(pairs, oc, cnt, A, B, kmode, flags, cells, nx); break;
            default: persist_body<4, 8, NP>(pairs, oc, cnt, A, B, kmode, flags, cells, nx); break;
        }
    }
}

// ---------------------------------------------------------------- dispatch
// The pairs in bin order (longest first; class-major when classes) and the bins' offsets
// off[0 .. LPT_BINS]; cnt and fill (LPT_BINS + 4 words each) must be zero.
static void build_order(const uint64_t *pairs, int64_t n, const VSet &va, const VSet &vb,
                        int kmode, int classes, uint32_t *cnt, uint32_t *fill, uint32_t *off,
                        int64_t *order, Workspace &ws, hipStream_t s, const uint32_t *ndev) {
    hipLaunchKernelGGL(k_lpt_hist, dim3(grid_for(n, 256, 1024)), dim3(256), 0, s, pairs, n, va, vb,
                       kmode, classes, cnt, ndev);
    MJ_LAUNCH_CHECK();
    exclusive_scan_u32(cnt, off, LPT_BINS, ws, s);
    const int64_t sblocks = (n + 256 * LPT_ITEMS - 1) / (256 * LPT_ITEMS);
    if (sblocks > 0x7FFFFFFFLL) throw Error(MJ_ECAPACITY, "too many pairs for one verification");
    hipLaunchKernelGGL(k_lpt_scatter, dim3((unsigned)sblocks), dim3(256), 0, s, pairs, n, va, vb,
                       kmode, classes, off, fill, order, ndev);
    MJ_LAUNCH_CHECK();
}

static PersistClassKernel classes_kernel(int np) {
    switch (np) {
        case 2: return k_verify_classes<2>;
        case 4: return k_verify_classes<4>;
        case 6: return k_verify_classes<6>;
        default: return k_verify_classes<8>;
    }
}

// order / off: the longest-first order and its bin offsets (class-major for CLASSES)
static void launch_persist(int nwl, int g, int np, int max_blocks, const uint64_t *pairs,
                           const int64_t *order, int64_t n, const VSet &va, const VSet &vb,
                           int kmode, uint8_t *flags, unsigned long long *cells,
                           unsigned long long *next, hipStream_t s, bool next_zero = false,
                           const uint32_t *ndev = nullptr, const uint32_t *off = nullptr) {
    if (!next_zero) fill_u64((uint64_t *)next, 0, (int64_t)VCLS * QUEUES * QSTRIDE, s);
    // at most max_blocks resident workgroups, and no more than the pairs need
    int64_t groups_per_block = 256 / (g == BIDIR ? 2 : g == CLASSES ? 1 : g);
    int64_t blocks = (n + groups_per_block - 1) / groups_per_block;
    blocks = std::min<int64_t>(blocks, max_blocks);
    if (g == CLASSES) {
        hipLaunchKernelGGL(classes_kernel(np), dim3((unsigned)std::max<int64_t>(blocks, 1)),
                           dim3(256), 0, s, pairs, order, off, va, vb, kmode, flags, cells, next);
        MJ_LAUNCH_CHECK();
        return;
    }
    hipLaunchKernelGGL(persist_kernel(nwl, g, np), dim3((unsigned)std::max<int64_t>(blocks, 1)),
                       dim3(256), 0, s, pairs, order, n, va, vb, kmode, flags, cells, next, ndev);
    MJ_LAUNCH_CHECK();
}

int64_t verify_pairs_batched(const uint64_t *pairs, int64_t n, const DevStrings &A,
                             const DevStrings &B, int kmode, uint8_t *flags, Workspace &ws,
                             hipStream_t s, uint64_t *host_scratch, KTimer *kt,
                             VerifyTuning *tune, int64_t uniform_k, uint64_t *cells_defer,
                             int force_lanes) {
    if (n <= 0) return 0;
    if (A.planes == nullptr || B.planes == nullptr) throw Error(MJ_EINVAL, "strings not packed");
    const int np = verify_planes(std::max(A.bits, B.bits));
    VSet va = vset(A), vb = vset(B);
    // one block cleared by one launch: the sub-queue counters (one set per band class), the
    // band-cell counter, the K pass's two words and two pairs of length-bin counter arrays
    // (longest-first and class-major orders)
    constexpr int64_t ZNEXT = 2 * VCLS * QUEUES * QSTRIDE, ZCNT = LPT_BINS + 4;
    uint32_t *zb = ws.get_n<uint32_t>(ZNEXT + 4 + 4 + 4 * ZCNT);
    unsigned long long *next = (unsigned long long *)zb;
    unsigned long long *cells = (unsigned long long *)(zb + ZNEXT);
    uint32_t *cm = zb + ZNEXT + 4;
    // longest pairs first
    uint32_t *cnt = zb + ZNEXT + 8;
    uint32_t *fillc = cnt + ZCNT;
    fill_u32(zb, 0, ZNEXT + 8 + 4 * ZCNT, s);
    bool next_zero = true;
    uint32_t *off = ws.get_n<uint32_t>(LPT_BINS + 1);
    int64_t *order = ws.get_n<int64_t>(n);
    // the class-major order, built when the band classes are timed or chosen
    uint32_t *off_c = nullptr;
    int64_t *order_c = nullptr;
    auto class_order = [&]() {
        if (order_c) return;
        off_c = ws.get_n<uint32_t>(LPT_BINS + 1);
        order_c = ws.get_n<int64_t>(n);
        build_order(pairs, n, va, vb, kmode, 1, fillc + ZCNT, fillc + 2 * ZCNT, off_c, order_c, ws,
                    s, nullptr);
    };
    int cmax;
    if (uniform_k >= 0) {
        // every pair's K is known (and its ids valid): no pass over the pairs
        cmax = (int)((std::min<int64_t>(uniform_k, 0x3FFFFFFF) + 31) >> 5);
    } else {
        hipLaunchKernelGGL(k_pair_cmax, dim3(grid_for(n, 256, 2048)), dim3(256), 0, s, pairs, n, va,
                           vb, kmode, cm, cm + 1);
        MJ_LAUNCH_CHECK();
        MJ_HIP(hipMemcpyAsync(host_scratch, cm, 8, hipMemcpyDeviceToHost, s));
        MJ_HIP(hipStreamSynchronize(s));
        uint32_t hv[2];
        memcpy(hv, host_scratch, 8);
        if (hv[1]) throw Error(MJ_EINVAL, "pair names a string id out of range");
        cmax = (int)hv[0];
    }
    if (cmax > persist_max_c())
        throw Error(MJ_ECAPACITY, "threshold K above the batched verifier's band limit (K <= 2047)");
    const int nw = cmax + 1;
    // band classes pay off only where the pairs' K differ
    const bool classes_ok = uniform_k < 0 && nwl_for(nw, CLASSES) != 0;
    const int npi = np / 2 - 1;
    const int ci = std::min(cmax, 63);
    int best_g = tune ? tune->best_g[ci][npi] : 0;
    int best_blocks = tune ? tune->best_blocks[ci][npi] : 0;
    if (force_lanes != 0) {
        best_g = force_lanes == -2 ? BIDIR : force_lanes == -3 ? CLASSES : force_lanes;
        best_blocks = 512;
        if (nwl_for(nw, best_g) == 0)
            throw Error(MJ_ECAPACITY, "verify_lanes: the lanes of a pair cannot hold this band");
    }
    if (best_g == CLASSES) class_order();
    else build_order(pairs, n, va, vb, kmode, 0, cnt, fillc, off, order, ws, s, nullptr);
    if (best_g == 0 && (n < TUNE_MIN_PAIRS || !tune)) {
        // a small call leaves most of the chip idle: the most lanes per pair (shortest
        // path per pair); timing the choices would cost more than the work.  Without a
        // tuning table (latency-first callers) the same fixed choice.
        best_g = verify_small_call_lanes(cmax);
        best_blocks = 512;
    }
    if (best_g == 0) {
        // time each (lanes per pair, resident workgroups) once on this call's pairs and
        // keep the fastest.  Back-to-back timing favours more resident workgroups than a
        // launch inside the pipeline does (the column split ran 1.30 ms at 768 and 1.32 ms
        // at 512 here, but 1.59 and 1.35 ms in the join), so each step up the list of
        // workgroup counts must be 3% faster to be taken.
        hipEvent_t e0, e1;
        MJ_HIP(hipEventCreate(&e0));
        MJ_HIP(hipEventCreate(&e1));
        float best = 1e30f;
        best_g = 0;
        for (int g : G_CHOICES) {
            int nwl = nwl_for(nw, g);
            if (nwl == 0 || (g == CLASSES && !classes_ok)) continue;
            if (g == CLASSES) class_order();
            int step = 0;
            for (int mb : {256, 512, 768, 1024, 2048}) {
                const float penalty = 1.0f + 0.03f * (float)step++;
                float ms = 1e30f;
                for (int rep = 0; rep < 2; rep++) {  // best of two: timing noise
                    MJ_HIP(hipEventRecord(e0, s));
                    launch_persist(nwl, g, np, mb, pairs, g == CLASSES ? order_c : order, n, va, vb,
                                   kmode, flags, cells, next, s, next_zero, nullptr,
                                   g == CLASSES ? off_c : off);
                    next_zero = false;
                    MJ_HIP(hipEventRecord(e1, s));
                    MJ_HIP(hipEventSynchronize(e1));
                    float t = 0.f;
                    MJ_HIP(hipEventElapsedTime(&t, e0, e1));
                    ms = std::min(ms, t);
                }
                if (ms * penalty < best) {
                    best = ms * penalty;
                    best_g = g;
                    best_blocks = mb;
                }
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (tune) {
            tune->best_g[ci][npi] = best_g;
            tune->best_blocks[ci][npi] = best_blocks;
        }
        fill_u64((uint64_t *)cells, 0, 1, s);
    }
    int th = kt ? kt->begin(KTimer::VERIFY, s) : -1;
    if (best_g == CLASSES) class_order();
    launch_persist(nwl_for(nw, best_g), best_g, np, best_blocks, pairs,
                   best_g == CLASSES ? order_c : order, n, va, vb, kmode, flags, cells, next, s,
                   next_zero, nullptr, best_g == CLASSES ? off_c : off);
    if (kt) kt->end(th, s);
    if (tune) {
        tune->last_g = best_g;
        tune->last_nwl = nwl_for(nw, best_g);
        tune->last_blocks = best_blocks;
    }
    if (cells_defer) {
        // the caller reads both words after its next synchronisation of the stream:
        // the band-cell count and the undersized-window error word
        MJ_HIP(hipMemcpyAsync(cells_defer, cells, 16, hipMemcpyDeviceToHost, s));
        return 0;
    }
    MJ_HIP(hipMemcpyAsync(host_scratch, cells, 16, hipMemcpyDeviceToHost, s));
    MJ_HIP(hipStreamSynchronize(s));
    uint64_t hv[2];
    memcpy(hv, host_scratch, 16);
    if (hv[1]) throw Error(MJ_ECAPACITY, "a pair's band exceeds the verifier window");
    return (int64_t)hv[0];
}

// The batched verification with the pair count on the device (*n_dev <= cap): pairs
// longest first, then the persistent launch in the configuration the context timed for this
// band size (the caller makes sure one is known: `cmax` words of band from the largest K),
// no host read.  flags[n .. cap) are written 0; the band-cell count and the window error
// word go to cells_out[0..1] (device).
void verify_pairs_batched_streamed(const uint64_t *pairs, int64_t cap, const uint32_t *n_dev,
                                   const DevStrings &A, const DevStrings &B, int kmode, int cmax,
                                   uint8_t *flags, Workspace &ws, hipStream_t s, KTimer *kt,
                                   const VerifyTuning &tune, int force_lanes,
                                   unsigned long long **cells_out) {
    const int np = verify_planes(std::max(A.bits, B.bits));
    VSet va = vset(A), vb = vset(B);
    cap = std::max<int64_t>(cap, 1);
    constexpr int64_t ZNEXT = 2 * VCLS * QUEUES * QSTRIDE, ZCNT = LPT_BINS + 4;
    uint32_t *zb = ws.get_n<uint32_t>(ZNEXT + 4 + 4 + 2 * ZCNT);
    unsigned long long *next = (unsigned long long *)zb;
    unsigned long long *cells = (unsigned long long *)(zb + ZNEXT);
    uint32_t *cnt = zb + ZNEXT + 8;
    uint32_t *fillc = cnt + ZCNT;
    fill_u32(zb, 0, ZNEXT + 8 + 2 * ZCNT, s);
    *cells_out = cells;
    fill_u32(reinterpret_cast<uint32_t *>(flags), 0, (cap + 3) / 4, s);
    uint32_t *off = ws.get_n<uint32_t>(LPT_BINS + 1);
    int64_t *order = ws.get_n<int64_t>(cap);
    if (cmax > persist_max_c())
        throw Error(MJ_ECAPACITY, "threshold K above the batched verifier's band limit (K <= 2047)");
    const int nw = cmax + 1;
    const int npi = np / 2 - 1;
    const int ci = std::min(cmax, 63);
    int g = tune.best_g[ci][npi], blocks = tune.best_blocks[ci][npi];
    if (force_lanes != 0) {
        g = force_lanes == -2 ? BIDIR : force_lanes == -3 ? CLASSES : force_lanes;
        blocks = 512;
    }
    if (g == 0 || nwl_for(nw, g) == 0)
        throw Error(MJ_EINVAL, "no verifier configuration for this band size");
    build_order(pairs, cap, va, vb, kmode, g == CLASSES ? 1 : 0, cnt, fillc, off, order, ws, s, n_dev);
    int th = kt ? kt->begin(KTimer::VERIFY, s) : -1;
    launch_persist(nwl_for(nw, g), g, np, blocks, pairs, order, cap, va, vb, kmode, flags, cells, next,
                   s, true, n_dev, off);
    if (kt) kt->end(th, s);
}

}  // namespace mj
