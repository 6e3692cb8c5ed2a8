// Shared pieces of the verification kernels.
#pragma once

#include "mj_common.h"

namespace mj {

struct VSet {
    int32_t n;
    const uint8_t *chars;
    const int64_t *off;
    const int32_t *len;
    const int32_t *kk;
    const uint32_t *planes;
    int64_t pw;
};

__device__ __forceinline__ uint32_t load_word(const uint32_t *plane, int64_t bitpos) {
    // 32 symbols' bits starting at global bit position bitpos (>= 0)
    int64_t w = bitpos >> 5;
    uint32_t sh = (uint32_t)(bitpos & 31);
    uint32_t lo = plane[w], hi = plane[w + 1];
    return __builtin_amdgcn_alignbit(hi, lo, sh);
}

inline VSet vset(const DevStrings &d) {
    return VSet{d.n, d.chars, d.offsets, d.len, d.kk, d.planes, d.plane_words};
}

}  // namespace mj
