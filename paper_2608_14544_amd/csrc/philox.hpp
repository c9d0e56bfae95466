// Philox4x32-10 counter-based generator for gfx950 (Salmon, Moraes, Dror,
// Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11): ten rounds
// of the 4x32 S-box with multipliers 0xD2511F53 / 0xCD9E8D57 and Weyl key
// increments 0x9E3779B9 / 0xBB67AE85.  The key is the 64-bit seed, which
// is wave-uniform, so the key schedule runs on the scalar unit; each
// 32x32->64 product is one v_mad_u64_u32, and each three-way exclusive or
// one v_bitop3_b32 (truth table 0x96, a ^ b ^ c), which the compiler does
// not form from two exclusive ors by itself.
#pragma once

#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>

#include <cstdint>
#endif

namespace qcl {

struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox10(U4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c.z;
        U4 n;
        n.x = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c.y, k0, 0x96);
        n.y = (uint32_t)p1;
        n.z = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c.w, k1, 0x96);
        n.w = (uint32_t)p0;
        c = n;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// (2 floor(x / 2^9) + 1) / 2^24: a uniform in (0,1) that is exact in both
// binary32 and binary64, so both precisions see the same threshold value.
// The top 23 bits of x become the mantissa of 1 + floor(x / 2^9) 2^-23 (one
// funnel shift of the exponent bits 0x7F and x by 9, v_alignbit_b32);
// subtracting 1 - 2^-24 leaves (2 floor(x / 2^9) + 1) 2^-24, which has at
// most 24 significant bits, so the subtraction is exact.
__device__ __forceinline__ float u24f(uint32_t x)
{
    return __uint_as_float(__builtin_amdgcn_alignbit(0x7Fu, x, 9u)) - 0x1.fffffep-1f;
}
__device__ __forceinline__ double u24d(uint32_t x)
{
    return (double)u24f(x);  // exact: the value has 24 significant bits
}

// 52-bit uniform in (0,1): k = hi * 2^20 + floor(lo / 2^12), (2k + 1) / 2^53.
__device__ __forceinline__ double u52(uint32_t hi, uint32_t lo)
{
    const uint64_t k = ((uint64_t)hi << 20) | (uint64_t)(lo >> 12);
    return (double)(2u * k + 1u) * 0x1p-53;
}

__device__ __forceinline__ uint32_t pick_word(const U4 &v, uint32_t i)
{
    // branch-free select of word i (0..3)
    uint32_t lo = (i & 1u) ? v.y : v.x;
    uint32_t hi = (i & 1u) ? v.w : v.z;
    return (i & 2u) ? hi : lo;
}

}  // namespace qcl
