// Fixed-order reduction of per-walker values into one tile partial.
//
// A workgroup of kBlock walkers (4 wavefronts) sums V values per walker.
// Inside a wavefront the sums follow the pairwise tree over lanes
// ((0+1)+(2+3))+...: a reduce-scatter butterfly in which, at the stage
// with lane distance d, each lane keeps half of its remaining values,
// summed with the partner lane's copy.  Every value therefore meets the
// same pairs as in the plain pairwise tree, while each stage halves the
// number of values a lane carries.  Across the 4 wavefronts the tree continues
// in LDS as (w0 + w1) + (w2 + w3).  Together with the pairwise tree over
// tiles this makes every sum a perfect binary tree over the walker index,
// independent of launch geometry.
#pragma once

#include <hip/hip_runtime.h>

namespace qcl {

// After the call, lane l holds (for V <= 64) the wavefront total of value
// index bitrev_log2V(l mod V) in v[0]; for V > 64 it holds V/64 values,
// v[i] being value index  sum_k bit_k(l) * (V >> (k+1)) + i.
template <int V>
__device__ __forceinline__ void wave_reduce_scatter(double (&v)[V], int lane)
{
    static_assert((V & (V - 1)) == 0 && V >= 2, "power of two");
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        const int off = 1 << s;
        const int half = V >> (s + 1);
        if (half >= 1) {
            const bool upper = (lane & off) != 0;
#pragma unroll
            for (int i = 0; i < half; ++i) {
                // both halves cross the lane pair; each lane keeps the sum of
                // the half it owns (selecting sums, not array elements, keeps
                // the array in registers)
                const double lo = v[i] + __shfl_xor(v[i], off, 64);
                const double hi = v[i + half] + __shfl_xor(v[i + half], off, 64);
                v[i] = upper ? hi : lo;
            }
        } else {
            v[0] = v[0] + __shfl_xor(v[0], off, 64);
        }
    }
}

template <int V>
__device__ __forceinline__ int scatter_index(int lane, int i)
{
    int idx = i;
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        const int half = V >> (s + 1);
        if (half >= 1 && (lane & (1 << s)))
            idx += half;
    }
    return idx;
}

// Sums v over the workgroup and writes the V totals to dst (by threads
// 0..V-1).  lds must hold 4*V doubles.  All threads must call it.
template <int V>
__device__ __forceinline__ void block_reduce_store(double (&v)[V], double *__restrict__ dst, double *lds)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    wave_reduce_scatter<V>(v, lane);
    constexpr int per_lane = V > 64 ? V / 64 : 1;
    const bool owner = V >= 64 || lane < V;
    if (owner) {
#pragma unroll
        for (int i = 0; i < per_lane; ++i)
            lds[wave * V + scatter_index<V>(lane, i)] = v[i];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < V; t += blockDim.x)
        dst[t] = (lds[t] + lds[V + t]) + (lds[2 * V + t] + lds[3 * V + t]);
    __syncthreads();
}

}  // namespace qcl
