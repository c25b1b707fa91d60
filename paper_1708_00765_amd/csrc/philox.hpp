// Counter-based random numbers for the CLS kernels.
//
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
// as 1, 2, 3", SC'11): a 4x32-bit counter is pushed through ten rounds of the
// Philox S-box; each round multiplies words 0 and 2 by the two round constants
// (high halves are mixed into the other words together with the key, low
// halves carried over) and the 2x32-bit key advances by the two Weyl
// increments between rounds.
//
// Stream layout: event step j of history h of a problem with seed s uses the
// block at counter (j, lane, lo32(h), hi32(h)) under key (lo32(s), hi32(s));
// lane is 0 except for the extra source block of the 3D interior source. A
// block yields five 23-bit integers k -- the top 23 bits of the four words, and
// the low 9, 9 and 5 bits of words 0, 1 and 2 -- mapped to U = (k + 1/2) 2^-23,
// a value in (0, 1) that is exact in both FP32 and FP64, so both precisions
// see identical uniforms.
//
// Each k is returned as the bit pattern of the float 1 + k 2^-23 (exponent
// field 127 above the 23 bits, one v_alignbit per word); U is that float minus
// 1 - 2^-24, a subtraction that is exact because U = (2k + 1) 2^-24 needs at
// most 24 significant bits.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cls {

struct Block5 {
    uint32_t k[5];
};

__device__ __forceinline__ Block5 philox_u23(uint32_t step, uint32_t lane, uint64_t h,
                                             uint32_t key_lo, uint32_t key_hi)
{
    uint32_t a = step, b = lane, c = (uint32_t)h, d = (uint32_t)(h >> 32);
    uint32_t k0 = key_lo, k1 = key_hi;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t pa = (uint64_t)a * 0xD2511F53u;   // one v_mad_u64_u32 each
        const uint64_t pc = (uint64_t)c * 0xCD9E8D57u;
        // three-input XOR in one gfx950 bitop3 (truth table 0x96)
        const uint32_t na = __builtin_amdgcn_bitop3_b32((uint32_t)(pc >> 32), b, k0, 0x96);
        const uint32_t nc = __builtin_amdgcn_bitop3_b32((uint32_t)(pa >> 32), d, k1, 0x96);
        b = (uint32_t)pc;
        d = (uint32_t)pa;
        a = na;
        c = nc;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    Block5 o;
    // (0x7F : w) >> 9 = 0x3F800000 | (w >> 9)
    o.k[0] = __builtin_amdgcn_alignbit(0x7Fu, a, 9u);
    o.k[1] = __builtin_amdgcn_alignbit(0x7Fu, b, 9u);
    o.k[2] = __builtin_amdgcn_alignbit(0x7Fu, c, 9u);
    o.k[3] = __builtin_amdgcn_alignbit(0x7Fu, d, 9u);
    o.k[4] = 0x3F800000u | ((a & 0x1FFu) << 14) | ((b & 0x1FFu) << 5) | (c & 0x1Fu);
    return o;
}

// U = (k + 1/2) 2^-23 from the bit pattern w of 1 + k 2^-23 (exact, see above).
template <typename R>
__device__ __forceinline__ R unit(uint32_t w)
{
    if constexpr (sizeof(R) == 4) {
        return __uint_as_float(w) - (1.0f - 0x1p-24f);
    } else {
        return (double)__uint_as_float(w) - (1.0 - 0x1p-24);
    }
}

}  // namespace cls
