// Shared pieces of the verification kernels.
#pragma once

#include "mj_common.h"

namespace mj {

// The verifiers read strings through their bit planes only (never the input symbols).
struct VSet {
    int32_t n;
    const int64_t *off;
    const int32_t *len;
    const int32_t *kk;
    const uint32_t *planes;
};

// The NP bit planes are interleaved: word w of plane p is planes[w * NP + p], so the planes
// of 32 consecutive symbols share a cache line.  `plane` points at plane p's first word
// (planes + p); returns 32 symbols' bits starting at global bit position bitpos (>= 0).
template <int NP>
__device__ __forceinline__ uint32_t load_word(const uint32_t *plane, int64_t bitpos) {
    int64_t w = bitpos >> 5;
    uint32_t sh = (uint32_t)(bitpos & 31);
    uint32_t lo = plane[w * NP], hi = plane[(w + 1) * NP];
    return __builtin_amdgcn_alignbit(hi, lo, sh);
}

// a & ~(b ^ c): the bits of a where b and c agree, in one v_bitop3 (truth table indexed
// by a << 2 | b << 1 | c: set at 100b and 111b).  With b a plane word of the pattern and c
// a text symbol's plane bit broadcast to all 32 lanes of the word, it narrows a match mask
// to the rows whose plane bit equals the text's.
__device__ __forceinline__ uint32_t and_xnor(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x90);
}

inline VSet vset(const DevStrings &d) {
    return VSet{d.n, d.offsets, d.len, d.kk, d.planes};
}

}  // namespace mj
