// Fixed-order reduction of per-walker bin values into one tile partial.
//
// A workgroup of kBlock walkers (4 wavefronts of 64) sums V doubles per
// walker.  The values go through LDS, 8 at a time (one "pass"): every lane
// writes its 8 values as one row of its wavefront's staging area (64 rows,
// padded to 9 doubles so that the rows fall on distinct banks), then lane l
// reads column (l & 7) of the 8 consecutive rows 8 (l >> 3) .. 8 (l >> 3) + 7
// and adds them as a pairwise tree.  The 8 partial sums of a column sit in
// lanes l, l ^ 8, l ^ 16, ..., l ^ 56 and are combined by three butterfly
// stages: a DPP row rotation (l ^ 8), v_permlane16_swap (l ^ 16) and
// v_permlane32_swap (l ^ 32) (see BinReducer::flush).  Each wavefront
// total is therefore a perfect binary tree over its 64 walkers in index
// order; across the 4 wavefronts the totals are added as (w0 + w1) + (w2 + w3)
// from a small LDS area, and the tiles are combined by the same tree in the
// final reduction: the whole sum is a perfect pairwise tree over the global
// walker index, bitwise independent of launch shape, batching and slicing.
//
// Compared with reducing in registers, the transposition moves the data
// through the LDS pipe and leaves about 12 additions and 4 crossbar moves per
// pass on the vector ALU; values that are zero in most lanes (the adiabatic
// slots a walker is not in) are written as zeros and overwritten by the one
// lane-dependent slot under an exec mask, with no per-value select.
//
// The count of walkers excluded from a bin (non-finite weight or phase) is
// gathered with a wavefront ballot and stored after the bin's values.
#pragma once

#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>

#include <cstdint>
#endif

namespace qcl {

constexpr int kPassValues = 8;    // values per LDS pass
constexpr int kStageStride = 9;   // doubles per staging row (8 values + 1 pad)
constexpr int kFlushValues = 32;  // values per cross-wavefront flush (4 passes)

struct BinLds {
    double stage[4][64 * kStageStride];  // one staging area per wavefront
    double wsum[2][4][kFlushValues];     // wavefront totals, double-buffered by flush
    uint32_t excluded[2][4];
};

namespace rdetail {

__device__ __forceinline__ uint32_t lo32(double x) { return (uint32_t)__double_as_longlong(x); }
__device__ __forceinline__ uint32_t hi32(double x) { return (uint32_t)((uint64_t)__double_as_longlong(x) >> 32); }
__device__ __forceinline__ double mkd(uint32_t lo, uint32_t hi)
{
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// x + x(lane ^ 8): row rotation by 8 inside each row of 16 lanes (every
// lane's source is valid, so no old value is needed)
__device__ __forceinline__ double add_xor8(double x)
{
    const uint32_t l = (uint32_t)__builtin_amdgcn_mov_dpp((int)lo32(x), 0x128, 0xF, 0xF, true);
    const uint32_t h = (uint32_t)__builtin_amdgcn_mov_dpp((int)hi32(x), 0x128, 0xF, 0xF, true);
    return x + mkd(l, h);
}

// v_permlane16_swap of a with b swaps the odd rows of a with the even rows
// of b, leaving (a0, b0, a2, b2) and (a1, b1, a3, b3): their sum holds
// a(row 2r) + a(row 2r+1) in rows 0 and 2 and the same of b in rows 1 and 3
__device__ __forceinline__ double add_swap16(double a, double b)
{
    const auto l = __builtin_amdgcn_permlane16_swap(lo32(a), lo32(b), false, false);
    const auto h = __builtin_amdgcn_permlane16_swap(hi32(a), hi32(b), false, false);
    return mkd(l[0], h[0]) + mkd(l[1], h[1]);
}

// v_permlane32_swap of a with b swaps the upper half of a with the lower
// half of b, leaving (a0, a1, b0, b1) and (a2, a3, b2, b3) in rows
__device__ __forceinline__ double add_swap32(double a, double b)
{
    const auto l = __builtin_amdgcn_permlane32_swap(lo32(a), lo32(b), false, false);
    const auto h = __builtin_amdgcn_permlane32_swap(hi32(a), hi32(b), false, false);
    return mkd(l[0], h[0]) + mkd(l[1], h[1]);
}

// x(lane) + x(lane ^ 16): v_permlane16_swap of x with itself leaves rows
// (r0, r0, r2, r2) in the first result and (r1, r1, r3, r3) in the second,
// so every lane adds the even row's value to the odd row's, in that order
__device__ __forceinline__ double add_xor16(double x)
{
    const auto l = __builtin_amdgcn_permlane16_swap(lo32(x), lo32(x), false, false);
    const auto h = __builtin_amdgcn_permlane16_swap(hi32(x), hi32(x), false, false);
    return mkd(l[0], h[0]) + mkd(l[1], h[1]);
}

// x(lane) + x(lane ^ 32), the same with the two halves of the wavefront
__device__ __forceinline__ double add_xor32(double x)
{
    const auto l = __builtin_amdgcn_permlane32_swap(lo32(x), lo32(x), false, false);
    const auto h = __builtin_amdgcn_permlane32_swap(hi32(x), hi32(x), false, false);
    return mkd(l[0], h[0]) + mkd(l[1], h[1]);
}

}  // namespace rdetail

// Reduction state of one bin (or one block of up to kFlushValues values of
// a bin) in one workgroup; every thread of the workgroup makes the same
// calls.  Usage per pass: put() the 8 values (or zero_row() and a masked
// put()), then pass(); after at most 4 passes flush().
//
// pass() leaves in every lane the sum of its column over its 8 rows.  The
// flush combines the (up to) 4 passes across lanes as one reduce-scatter:
// a DPP rotation adds the row halves (l ^ 8) of each pass, v_permlane16_swap
// of passes 0 with 1 and 2 with 3 adds l ^ 16 while sending the two passes
// to alternate rows, and v_permlane32_swap of the two results adds l ^ 32,
// after which row r (lanes 16 r .. 16 r + 15) holds the wavefront totals of
// pass r.  The additions are the same perfect tree over the 64 lanes as a
// butterfly on each pass separately, in fewer crossbar moves.
struct BinReducer {
    BinLds &L;
    int &parity;  // the workgroup's flush counter (kept by the caller across bins)
    int lane, wave;
    double *row;
    int npass = 0;
    double acc[4];

    __device__ __forceinline__ BinReducer(BinLds &lds, int &flush_parity)
        : L(lds), parity(flush_parity), lane(threadIdx.x & 63), wave(threadIdx.x >> 6)
    {
        row = &L.stage[wave][lane * kStageStride];
    }

    __device__ __forceinline__ void zero_row()
    {
#pragma unroll
        for (int j = 0; j < kPassValues; ++j)
            row[j] = 0.0;
    }

    __device__ __forceinline__ void put(int col, double x) { row[col] = x; }

    // column (lane & 7) of the staged rows 8 (lane >> 3) .. 8 (lane >> 3) + 7
    __device__ __forceinline__ void pass()
    {
        __builtin_amdgcn_wave_barrier();
        const double *c = &L.stage[wave][(lane >> 3) * 8 * kStageStride + (lane & 7)];
        const double s01 = c[0 * kStageStride] + c[1 * kStageStride];
        const double s23 = c[2 * kStageStride] + c[3 * kStageStride];
        const double s45 = c[4 * kStageStride] + c[5 * kStageStride];
        const double s67 = c[6 * kStageStride] + c[7 * kStageStride];
        double s = (s01 + s23) + (s45 + s67);
        // one pass at a time: the empty asm makes the sum exist here, so the
        // compiler cannot sink the additions to the flush and hold all four
        // passes' reads in registers (which would cost the kernel occupancy)
        asm volatile("" : "+v"(s));
        acc[npass] = s;
        ++npass;
    }

    // Walkers excluded from this bin (counted per wavefront).
    __device__ __forceinline__ void count_excluded(bool excluded)
    {
        const unsigned long long m = __ballot(excluded);
        if (lane == 0)
            L.excluded[parity & 1][wave] = (uint32_t)__popcll(m);
    }

    // Adds the wavefront totals of the values staged since the last flush
    // over the 4 wavefronts and writes the first n of them to dst (threads
    // 0..n-1); thread 32 writes the excluded count to *count_dst when it is
    // given.  The wavefront totals are double-buffered by the flush counter,
    // so one barrier per flush suffices: a buffer is written again only
    // after the next flush's barrier, which every reader of this flush has
    // passed.
    __device__ __forceinline__ void flush(double *__restrict__ dst, int n, double *__restrict__ count_dst)
    {
        using namespace rdetail;
        const int k = parity & 1;
#pragma unroll
        for (int p = 0; p < 4; ++p)
            acc[p] = p < npass ? add_xor8(acc[p]) : 0.0;
        const double t = add_swap32(add_swap16(acc[0], acc[1]), add_swap16(acc[2], acc[3]));
        if ((lane & 8) == 0)  // row r, lanes 16 r .. 16 r + 7: pass r, value lane & 7
            L.wsum[k][wave][(lane >> 4) * kPassValues + (lane & 7)] = t;
        __syncthreads();
        const int i = threadIdx.x;
        if (i < n)
            dst[i] = (L.wsum[k][0][i] + L.wsum[k][1][i]) + (L.wsum[k][2][i] + L.wsum[k][3][i]);
        if (count_dst && i == kFlushValues)
            *count_dst = (double)((L.excluded[k][0] + L.excluded[k][1]) + (L.excluded[k][2] + L.excluded[k][3]));
        npass = 0;
        parity ^= 1;
    }
};


// The same reduction with each pass combined across lanes on its own (the
// butterfly x + x(l ^ 8), + x(l ^ 16), + x(l ^ 32) on every lane) and its 8
// wavefront totals written to LDS at once: the same additions in the same
// tree as BinReducer, so the sums are bitwise equal, at more crossbar moves
// per pass but with no pass sums held in registers until the flush.  The
// general kernels, whose step code already holds many registers, use this
// form.
struct BinReducerPerPass {
    BinLds &L;
    int &parity;  // the workgroup's flush counter (kept by the caller across bins)
    int lane, wave;
    double *row;
    int npass = 0;

    __device__ __forceinline__ BinReducerPerPass(BinLds &lds, int &flush_parity)
        : L(lds), parity(flush_parity), lane(threadIdx.x & 63), wave(threadIdx.x >> 6)
    {
        row = &L.stage[wave][lane * kStageStride];
    }

    __device__ __forceinline__ void zero_row()
    {
#pragma unroll
        for (int j = 0; j < kPassValues; ++j)
            row[j] = 0.0;
    }

    __device__ __forceinline__ void put(int col, double x) { row[col] = x; }

    // the wavefront totals of the 8 staged values, into the LDS totals
    __device__ __forceinline__ void pass()
    {
        using namespace rdetail;
        __builtin_amdgcn_wave_barrier();
        const double *c = &L.stage[wave][(lane >> 3) * 8 * kStageStride + (lane & 7)];
        const double s01 = c[0 * kStageStride] + c[1 * kStageStride];
        const double s23 = c[2 * kStageStride] + c[3 * kStageStride];
        const double s45 = c[4 * kStageStride] + c[5 * kStageStride];
        const double s67 = c[6 * kStageStride] + c[7 * kStageStride];
        double s = (s01 + s23) + (s45 + s67);
        s = add_xor8(s);
        s = add_xor16(s);
        s = add_xor32(s);
        if (lane < kPassValues)
            L.wsum[parity & 1][wave][npass * kPassValues + lane] = s;
        __builtin_amdgcn_wave_barrier();
        ++npass;
    }

    __device__ __forceinline__ void count_excluded(bool excluded)
    {
        const unsigned long long m = __ballot(excluded);
        if (lane == 0)
            L.excluded[parity & 1][wave] = (uint32_t)__popcll(m);
    }

    // as BinReducer::flush
    __device__ __forceinline__ void flush(double *__restrict__ dst, int n, double *__restrict__ count_dst)
    {
        __syncthreads();
        const int i = threadIdx.x;
        const int k = parity & 1;
        if (i < n)
            dst[i] = (L.wsum[k][0][i] + L.wsum[k][1][i]) + (L.wsum[k][2][i] + L.wsum[k][3][i]);
        if (count_dst && i == kFlushValues)
            *count_dst = (double)((L.excluded[k][0] + L.excluded[k][1]) + (L.excluded[k][2] + L.excluded[k][3]));
        npass = 0;
        parity ^= 1;
    }
};

}  // namespace qcl
