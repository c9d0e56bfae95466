// Fixed-order reduction of per-walker values into one tile partial.
//
// A workgroup of kBlock walkers (4 wavefronts) sums V = 32 doubles per
// walker.  Inside a wavefront a reduce-scatter butterfly pairs lanes l and
// l^32, then l^16, l^8, l^4, l^2, l^1; at each stage a lane keeps half of
// the values it still carries, summed with its partner's copy, so after the
// last stage every lane holds the wavefront total of one value.  Data moves
// with gfx950's register-only crossbar instructions: v_permlane32_swap and
// v_permlane16_swap for the two widest stages (one swap per dword replaces a
// shuffle-and-select), DPP row/quad permutations for the narrow ones.  No
// LDS traffic is needed inside the wavefront.
//
// Which value ends in which lane is a fixed function of the lane index; it
// is obtained by running the same data movement on the value indices
// (scatter_slots), so the code does not depend on which half of a register
// pair a swap instruction moves.  Across the 4 wavefronts the sums continue
// in LDS as (w0 + w1) + (w2 + w3).  Every sum is therefore a fixed binary
// tree over the walker index: bitwise repeatable and independent of how the
// steps are split over launches.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qcl {

namespace rdetail {

__device__ __forceinline__ uint32_t lo32(double x) { return (uint32_t)__double_as_longlong(x); }
__device__ __forceinline__ uint32_t hi32(double x) { return (uint32_t)((uint64_t)__double_as_longlong(x) >> 32); }
__device__ __forceinline__ double mkd(uint32_t lo, uint32_t hi)
{
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// v_permlane32_swap / v_permlane16_swap on a pair of doubles
__device__ __forceinline__ void swap32(double &a, double &b)
{
    auto l = __builtin_amdgcn_permlane32_swap(lo32(a), lo32(b), false, false);
    auto h = __builtin_amdgcn_permlane32_swap(hi32(a), hi32(b), false, false);
    a = mkd(l[0], h[0]);
    b = mkd(l[1], h[1]);
}
__device__ __forceinline__ void swap16(double &a, double &b)
{
    auto l = __builtin_amdgcn_permlane16_swap(lo32(a), lo32(b), false, false);
    auto h = __builtin_amdgcn_permlane16_swap(hi32(a), hi32(b), false, false);
    a = mkd(l[0], h[0]);
    b = mkd(l[1], h[1]);
}
__device__ __forceinline__ void swap32i(int &a, int &b)
{
    auto r = __builtin_amdgcn_permlane32_swap((uint32_t)a, (uint32_t)b, false, false);
    a = (int)r[0];
    b = (int)r[1];
}
__device__ __forceinline__ void swap16i(int &a, int &b)
{
    auto r = __builtin_amdgcn_permlane16_swap((uint32_t)a, (uint32_t)b, false, false);
    a = (int)r[0];
    b = (int)r[1];
}

// value of lane l ^ D for D in {8, 4, 2, 1} (DPP; every lane reads a lane
// of its own row of 16)
template <int D>
__device__ __forceinline__ uint32_t xlane32(uint32_t x)
{
    if constexpr (D == 8) {
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x128, 0xF, 0xF, false);  // row_ror:8
    } else if constexpr (D == 4) {
        // row_half_mirror (l -> l ^ 7 within 8) then quad mirror (l -> l ^ 3)
        const int m = __builtin_amdgcn_update_dpp(0, (int)x, 0x141, 0xF, 0xF, false);
        return (uint32_t)__builtin_amdgcn_update_dpp(0, m, 0x1B, 0xF, 0xF, false);  // quad_perm [3,2,1,0]
    } else if constexpr (D == 2) {
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
    } else {
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
    }
}
template <int D>
__device__ __forceinline__ double xlane(double x)
{
    return mkd(xlane32<D>(lo32(x)), xlane32<D>(hi32(x)));
}

// one narrow stage: lanes with bit D clear keep the lower half
template <int D, int H>
__device__ __forceinline__ void narrow_stage(double *v, bool upper)
{
#pragma unroll
    for (int i = 0; i < H; ++i) {
        const double lo = v[i] + xlane<D>(v[i]);
        const double hi = v[i + H] + xlane<D>(v[i + H]);
        v[i] = upper ? hi : lo;
    }
}

}  // namespace rdetail

// Value index each lane holds after wave_reduce32 (same movement on ints).
__device__ __forceinline__ int scatter_slot32(int lane)
{
    using namespace rdetail;
    int id[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        int a = i, b = i + 16;
        swap32i(a, b);
        id[i] = a;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        int a = id[i], b = id[i + 8];
        swap16i(a, b);
        id[i] = a;
    }
    id[0] = (lane & 8) ? id[4] : id[0];
    id[1] = (lane & 8) ? id[5] : id[1];
    id[2] = (lane & 8) ? id[6] : id[2];
    id[3] = (lane & 8) ? id[7] : id[3];
    id[0] = (lane & 4) ? id[2] : id[0];
    id[1] = (lane & 4) ? id[3] : id[1];
    id[0] = (lane & 2) ? id[1] : id[0];
    return id[0];
}

// Reduce-scatter of 32 doubles over the 64 lanes; lane l ends with the
// wavefront total of value scatter_slot32(l) in v[0] (lanes l and l^1 hold
// the same value).
__device__ __forceinline__ void wave_reduce32(double (&v)[32], int lane)
{
    using namespace rdetail;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        double a = v[i], b = v[i + 16];
        swap32(a, b);
        v[i] = a + b;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        double a = v[i], b = v[i + 8];
        swap16(a, b);
        v[i] = a + b;
    }
    narrow_stage<8, 4>(v, (lane & 8) != 0);
    narrow_stage<4, 2>(v, (lane & 4) != 0);
    narrow_stage<2, 1>(v, (lane & 2) != 0);
    v[0] = v[0] + xlane<1>(v[0]);
}

// Sums v over the workgroup and writes the first n_valid of the 32 totals
// to dst (threads 0..n_valid-1).  lds holds 4*32 doubles;
// slot = scatter_slot32(lane).  All threads call it.
__device__ __forceinline__ void block_reduce_store32(double (&v)[32], int slot, double *__restrict__ dst,
                                                     double *lds, int n_valid = 32)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    wave_reduce32(v, lane);
    if ((lane & 1) == 0)
        lds[wave * 32 + slot] = v[0];
    __syncthreads();
    if (threadIdx.x < n_valid) {
        const int t = threadIdx.x;
        dst[t] = (lds[t] + lds[32 + t]) + (lds[64 + t] + lds[96 + t]);
    }
    __syncthreads();
}

// Value index each lane holds after wave_reduce16.
__device__ __forceinline__ int scatter_slot16(int lane)
{
    using namespace rdetail;
    int id[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        int a = i, b = i + 8;
        swap32i(a, b);
        id[i] = a;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        int a = id[i], b = id[i + 4];
        swap16i(a, b);
        id[i] = a;
    }
    id[0] = (lane & 8) ? id[2] : id[0];
    id[1] = (lane & 8) ? id[3] : id[1];
    id[0] = (lane & 4) ? id[1] : id[0];
    return id[0];
}

// Reduce-scatter of 16 doubles over the 64 lanes (the same stages as
// wave_reduce32 with half the values live): lane l ends with the wavefront
// total of value scatter_slot16(l) in v[0] (lanes l, l^1, l^2, l^3 agree).
__device__ __forceinline__ void wave_reduce16(double (&v)[16], int lane)
{
    using namespace rdetail;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        double a = v[i], b = v[i + 8];
        swap32(a, b);
        v[i] = a + b;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        double a = v[i], b = v[i + 4];
        swap16(a, b);
        v[i] = a + b;
    }
    narrow_stage<8, 2>(v, (lane & 8) != 0);
    narrow_stage<4, 1>(v, (lane & 4) != 0);
    v[0] = v[0] + xlane<2>(v[0]);
    v[0] = v[0] + xlane<1>(v[0]);
}

// block_reduce_store32 for 16 values; lds holds 4*16 doubles,
// slot = scatter_slot16(lane).
__device__ __forceinline__ void block_reduce_store16(double (&v)[16], int slot, double *__restrict__ dst,
                                                     double *lds, int n_valid = 16)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    wave_reduce16(v, lane);
    if ((lane & 3) == 0)
        lds[wave * 16 + slot] = v[0];
    __syncthreads();
    if (threadIdx.x < n_valid) {
        const int t = threadIdx.x;
        dst[t] = (lds[t] + lds[16 + t]) + (lds[32 + t] + lds[48 + t]);
    }
    __syncthreads();
}

}  // namespace qcl
