// Fixed-budget systematic resampling of a walker ensemble for gfx950.
//
// Between propagation calls the T walkers of an ensemble are replaced by T
// copies drawn in proportion to |w| (the paper's CPU code spawned walkers
// instead and let their number grow, Sec. II.B).  Every decision is taken in
// exact integer arithmetic, so the result does not depend on the order in
// which the device adds things up:
//   k_i = ceil(|w_i| / w_max * 2^32)   (0 for zero or non-finite walkers)
//   P_i = k_0 + ... + k_{i-1},  K = P_T
//   output j copies the walker i with P_i <= X_j < P_{i+1},
//   X_j = floor((j 2^32 + U) K / (T 2^32)),  U one 32-bit Philox word,
// and carries the weight w_i K / (T k_i), so each walker's expected total
// weight is unchanged (its mean copy count over the 2^32 offsets is within
// 2^-32 of T k_i / K).
//
// Passes (all bound by HBM bandwidth):
//   1. exact maximum of |w|: per-tile maxima, then one atomic maximum per
//      group of 256 tiles (non-negative doubles order like their bit
//      patterns);
//   2. per 1024-walker tile (four consecutive walkers a lane), the sum of
//      k_i;
//   3. exclusive scan of the tile sums per group of 256 tiles, with the
//      group totals;
//   4. one workgroup: exclusive scan of the group totals, K after the last;
//   5. per walker, P_i from the two scans and an in-tile scan;
//   6. one lane per 256-output workgroup of pass 7: the source of the
//      workgroup's first output, by binary search over P;
//   7. per workgroup: its slice of P (outputs visit sources in order, so
//      every output lies between its own first source and the next
//      workgroup's) staged in LDS, then per output a search in that slice
//      and the copy of the source's state.
// k_i is never stored: passes 5 and 7 recompute it from w_i with the same
// expression, which gives the same integer.  X_j is formed in 64-bit pieces
// (K = cT + d, jd = eT + f, Uc = g 2^32 + h):
//   X_j = jc + e + g + floor((f 2^32 + hT + Ud) / (T 2^32)),
// where the last term is 0, 1 or 2 and each partial sum fits 64 bits
// (T < 2^31, c <= 2^32).
#include <cstdint>

#include "philox.hpp"
#include "qcl_internal.hpp"

namespace qcl {
namespace {

constexpr double kTwo32 = 4294967296.0;
constexpr int kItems = 4;                // consecutive walkers per lane in passes 1, 2 and 5
constexpr int kQTile = kBlock * kItems;  // walkers per quantisation tile

int64_t n_qtiles(int64_t n) { return (n + kQTile - 1) / kQTile; }
int64_t n_groups_of(int64_t tiles) { return (tiles + kBlock - 1) / kBlock; }

__device__ __forceinline__ bool live_weight(double w, double phase) { return isfinite(w) && isfinite(phase) && w != 0.0; }

__device__ __forceinline__ uint64_t quantized(double w, double phase, double wmax)
{
    return (wmax > 0.0 && live_weight(w, phase)) ? (uint64_t)ceil(fabs(w) / wmax * kTwo32) : 0;
}

// sum of one value per thread over the workgroup (kBlock threads)
__device__ __forceinline__ uint64_t block_sum_u64(uint64_t v, uint64_t *lds)
{
    lds[threadIdx.x] = v;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off)
            lds[threadIdx.x] += lds[threadIdx.x + off];
        __syncthreads();
    }
    const uint64_t s = lds[0];
    __syncthreads();
    return s;
}

// exclusive prefix sum of one value per thread over the workgroup; *total
// receives the workgroup's sum
__device__ __forceinline__ uint64_t block_exclusive_u64(uint64_t v, uint64_t *lds, uint64_t *total)
{
    lds[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
        const uint64_t add = (int)threadIdx.x >= off ? lds[threadIdx.x - off] : 0;
        __syncthreads();
        lds[threadIdx.x] += add;
        __syncthreads();
    }
    const uint64_t inclusive = lds[threadIdx.x];
    *total = lds[kBlock - 1];
    __syncthreads();
    return inclusive - v;
}

// largest of one value per thread over the workgroup
__device__ __forceinline__ uint64_t block_max_u64(uint64_t v, uint64_t *lds)
{
    lds[threadIdx.x] = v;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off)
            lds[threadIdx.x] = lds[threadIdx.x] > lds[threadIdx.x + off] ? lds[threadIdx.x] : lds[threadIdx.x + off];
        __syncthreads();
    }
    const uint64_t r = lds[0];
    __syncthreads();
    return r;
}

// per quantisation tile, the bit pattern of the largest |w| of a live walker
// (0 if none)
__global__ __launch_bounds__(kBlock) void rs_tile_max_kernel(const double *__restrict__ w,
                                                             const double *__restrict__ phase, int64_t n,
                                                             uint64_t *__restrict__ tile_max)
{
    __shared__ uint64_t lds[kBlock];
    const int64_t base = (int64_t)blockIdx.x * kQTile + (int64_t)threadIdx.x * kItems;
    double x[kItems], f[kItems];
#pragma unroll
    for (int u = 0; u < kItems; ++u) {  // clamped indices: every load issues at once
        const int64_t i = base + u < n ? base + u : n - 1;
        x[u] = w[i];
        f[u] = phase[i];
    }
    uint64_t bits = 0;
#pragma unroll
    for (int u = 0; u < kItems; ++u) {
        const uint64_t b = base + u < n && live_weight(x[u], f[u]) ? (uint64_t)__double_as_longlong(fabs(x[u])) : 0;
        bits = b > bits ? b : bits;
    }
    const uint64_t mx = block_max_u64(bits, lds);
    if (threadIdx.x == 0)
        tile_max[blockIdx.x] = mx;
}

// per group of kBlock tiles, one atomic maximum into *wmax_bits
__global__ __launch_bounds__(kBlock) void rs_max_groups_kernel(const uint64_t *__restrict__ tile_max, int64_t n_tiles,
                                                               unsigned long long *wmax_bits)
{
    __shared__ uint64_t lds[kBlock];
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const uint64_t mx = block_max_u64(t < n_tiles ? tile_max[t] : 0, lds);
    if (threadIdx.x == 0 && mx != 0)
        atomicMax(wmax_bits, (unsigned long long)mx);
}

// quantised weights of a lane's kItems consecutive walkers (0 past the end)
__device__ __forceinline__ void lane_weights(const double *__restrict__ w, const double *__restrict__ phase, int64_t n,
                                             int64_t base, double wmax, uint64_t (&k)[kItems])
{
    double x[kItems], f[kItems];
#pragma unroll
    for (int u = 0; u < kItems; ++u) {
        const int64_t i = base + u < n ? base + u : n - 1;
        x[u] = w[i];
        f[u] = phase[i];
    }
#pragma unroll
    for (int u = 0; u < kItems; ++u)
        k[u] = base + u < n ? quantized(x[u], f[u], wmax) : 0;
}

__global__ __launch_bounds__(kBlock) void rs_tile_sum_kernel(const double *__restrict__ w,
                                                             const double *__restrict__ phase, int64_t n,
                                                             const unsigned long long *wmax_bits,
                                                             uint64_t *__restrict__ tile_sums)
{
    __shared__ uint64_t lds[kBlock];
    const int64_t base = (int64_t)blockIdx.x * kQTile + (int64_t)threadIdx.x * kItems;
    uint64_t k[kItems];
    lane_weights(w, phase, n, base, __longlong_as_double((long long)*wmax_bits), k);
    uint64_t local = 0;
#pragma unroll
    for (int u = 0; u < kItems; ++u)
        local += k[u];
    const uint64_t s = block_sum_u64(local, lds);
    if (threadIdx.x == 0)
        tile_sums[blockIdx.x] = s;
}

// exclusive scan of each group of kBlock tile sums in place; group totals
// to supers[group]
__global__ __launch_bounds__(kBlock) void rs_scan_groups_kernel(uint64_t *__restrict__ tile_sums, int64_t n_tiles,
                                                                uint64_t *__restrict__ supers)
{
    __shared__ uint64_t lds[kBlock];
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const uint64_t v = t < n_tiles ? tile_sums[t] : 0;
    uint64_t total;
    const uint64_t ex = block_exclusive_u64(v, lds, &total);
    if (t < n_tiles)
        tile_sums[t] = ex;
    if (threadIdx.x == 0)
        supers[blockIdx.x] = total;
}

// one workgroup: exclusive scan of the group totals in place, K at [n_groups]
__global__ __launch_bounds__(kBlock) void rs_scan_top_kernel(uint64_t *supers, int64_t n_groups)
{
    __shared__ uint64_t lds[kBlock];
    uint64_t carry = 0;
    for (int64_t base = 0; base < n_groups; base += kBlock) {
        const int64_t g = base + threadIdx.x;
        const uint64_t v = g < n_groups ? supers[g] : 0;
        uint64_t total;
        const uint64_t ex = block_exclusive_u64(v, lds, &total);
        if (g < n_groups)
            supers[g] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0)
        supers[n_groups] = carry;
}

__global__ __launch_bounds__(kBlock) void rs_prefix_kernel(const double *__restrict__ w, const double *__restrict__ phase,
                                                           int64_t n, const unsigned long long *wmax_bits,
                                                           const uint64_t *__restrict__ tile_sums,
                                                           const uint64_t *__restrict__ supers, int64_t n_groups,
                                                           uint64_t *__restrict__ P)
{
    __shared__ uint64_t lds[kBlock];
    const int64_t base = (int64_t)blockIdx.x * kQTile + (int64_t)threadIdx.x * kItems;
    uint64_t k[kItems];
    lane_weights(w, phase, n, base, __longlong_as_double((long long)*wmax_bits), k);
    uint64_t local = 0;
#pragma unroll
    for (int u = 0; u < kItems; ++u)
        local += k[u];
    uint64_t total;
    uint64_t run = supers[blockIdx.x / kBlock] + tile_sums[blockIdx.x] + block_exclusive_u64(local, lds, &total);
#pragma unroll
    for (int u = 0; u < kItems; ++u) {
        if (base + u < n)
            P[base + u] = run;
        run += k[u];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0)
        P[n] = supers[n_groups];
}

// the per-call constants of the comb: K = c T + d, U c = g 2^32 + h
struct Comb {
    uint64_t c, d, g, h;
    uint32_t U;
};

__device__ __forceinline__ Comb make_comb(uint64_t K, int64_t n, uint32_t U)
{
    const uint64_t c = K / (uint64_t)n;
    const uint64_t Uc = (uint64_t)U * c;
    return Comb{c, K - c * (uint64_t)n, Uc >> 32, Uc & 0xFFFFFFFFull, U};
}

// X_j = floor((j 2^32 + U) K / (T 2^32)), exactly, in 64-bit arithmetic
__device__ __forceinline__ uint64_t comb_point(int64_t j, const Comb &C, int64_t n)
{
    const uint64_t T = (uint64_t)n, TT = T << 32;
    const uint64_t jd = (uint64_t)j * C.d;  // < 2^62
    const uint64_t e = jd / T, f = jd - e * T;
    uint64_t r = (f << 32) + C.h * T;      // < 2 T 2^32
    uint64_t q = 0;
    if (r >= TT) {
        r -= TT;
        q = 1;
    }
    r += (uint64_t)C.U * C.d;               // < 2 T 2^32
    q += r >= TT ? 1 : 0;
    return (uint64_t)j * C.c + e + C.g + q;
}

// the i in [lo, hi) with P[i] <= X < P[i + 1], given P[lo] <= X < P[hi]
template <typename PT>
__device__ __forceinline__ int64_t search(PT P, uint64_t X, int64_t lo, int64_t hi)
{
    while (hi - lo > 1) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if (P[mid] <= X)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// start[b] = source of output b * kBlock for b < n_wg, start[n_wg] = n - 1;
// comb constants to comb[0..4]
__global__ __launch_bounds__(kBlock) void rs_bounds_kernel(const uint64_t *__restrict__ P, int64_t n, int64_t n_wg,
                                                           uint32_t key0, uint32_t key1, uint64_t offset,
                                                           uint64_t step, uint64_t *__restrict__ comb,
                                                           int64_t *__restrict__ start)
{
    const int64_t b = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const uint64_t K = P[n];
    if (K == 0 || b > n_wg)
        return;
    const uint32_t U =
        philox10(U4{(uint32_t)offset, (uint32_t)(offset >> 32), (uint32_t)step, 3u}, key0, key1).x;
    const Comb C = make_comb(K, n, U);
    if (b == 0) {
        comb[0] = C.c;
        comb[1] = C.d;
        comb[2] = C.g;
        comb[3] = C.h;
        comb[4] = C.U;
    }
    start[b] = b < n_wg ? search(P, comb_point(b * kBlock, C, n), 0, n) : n - 1;
}

constexpr int kStage = 1024;  // largest slice of P a workgroup stages in LDS
constexpr int kXcds = 8;      // workgroups are dealt to the XCDs round-robin

// Output tile of a gather workgroup: each XCD (own L2) takes one contiguous
// run of tiles, so the cache lines shared by neighbouring tiles' source
// slices are fetched into one L2 only.  A bijection of [0, n_wg).
__device__ __forceinline__ int64_t xcd_tile(int64_t bid, int64_t n_wg)
{
    const int64_t xcd = bid % kXcds, local = bid / kXcds;
    const int64_t base = n_wg / kXcds, extra = n_wg % kXcds;
    return xcd < extra ? xcd * (base + 1) + local : extra * (base + 1) + (xcd - extra) * base + local;
}

template <typename R>
__global__ __launch_bounds__(kBlock) void rs_gather_kernel(EnsDev<R> S, EnsDev<R> D, int32_t m, int32_t nn,
                                                           const uint64_t *__restrict__ P,
                                                           const uint64_t *__restrict__ comb,
                                                           const int64_t *__restrict__ start,
                                                           const unsigned long long *wmax_bits)
{
    __shared__ uint64_t slice[kStage + 1];
    const int64_t n = S.n_traj;
    const int64_t wg = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t j = wg * kBlock + threadIdx.x;
    const uint64_t K = P[n];
    int64_t i = j;  // K == 0: no walker with a nonzero finite weight, copy unchanged
    double scale = 1.0;
    if (K != 0) {
        // every output of this workgroup has P[lo] <= X_j < P[hi]
        const int64_t lo = start[wg], hi = start[wg + 1] + 1;
        const bool staged = hi - lo <= kStage;  // uniform over the workgroup
        if (staged) {
            for (int64_t t = threadIdx.x; t <= hi - lo; t += kBlock)
                slice[t] = P[lo + t];
            __syncthreads();
        }
        if (j < n) {
            const Comb C{comb[0], comb[1], comb[2], comb[3], (uint32_t)comb[4]};
            const uint64_t X = comb_point(j, C, n);
            i = staged ? lo + search((const uint64_t *)slice, X, 0, hi - lo) : search(P, X, lo, hi);
            const double wmax = __longlong_as_double((long long)*wmax_bits);
            const uint64_t ki = (uint64_t)ceil(fabs(S.w[i]) / wmax * kTwo32);
            scale = (double)K / ((double)n * (double)ki);
        }
    }
    if (j >= n)
        return;
    for (int r = 0; r < m; ++r) {
        D.q[r * D.ld + j] = S.q[r * S.ld + i];
        D.p[r * D.ld + j] = S.p[r * S.ld + i];
    }
    for (int r = 0; r < nn; ++r)
        D.u[r * D.ld + j] = S.u[r * S.ld + i];
    D.w[j] = K == 0 ? S.w[i] : S.w[i] * scale;
    D.phase[j] = S.phase[i];
    D.a[j] = S.a[i];
    D.b[j] = S.b[i];
    if (S.flags && D.flags)
        D.flags[j] = S.flags[i];
}

template <typename R>
EnsDev<R> ens_dev_rs(const qcl_ensemble &e)
{
    return EnsDev<R>{(R *)e.q, (R *)e.p, (R *)e.u, e.w, e.phase, e.a, e.b, e.flags, e.ld, e.n_traj, e.traj_offset};
}

}  // namespace

ResampleLayout resample_layout(int64_t n_traj)
{
    auto up = [](size_t x) { return (x + 255) / 256 * 256; };
    ResampleLayout L{};
    const size_t T = (size_t)n_traj, qt = (size_t)n_qtiles(n_traj), groups = (size_t)n_groups_of(n_qtiles(n_traj));
    L.wmax = 0;
    L.P = 256;
    L.tiles = L.P + up(8 * (T + 1));
    L.supers = L.tiles + up(8 * qt);
    L.comb = L.supers + up(8 * (groups + 1));
    L.start = L.comb + 256;
    L.bytes = L.start + up(8 * ((size_t)n_tiles(n_traj) + 1));
    return L;
}

hipError_t launch_resample(const qcl_model_s &m, const qcl_ensemble &S, const qcl_ensemble &D, uint64_t seed,
                           void *workspace, hipStream_t s)
{
    const int64_t n = S.n_traj;
    if (n == 0)
        return hipSuccess;
    const int64_t qt = n_qtiles(n), groups = n_groups_of(qt), tiles = n_tiles(n);
    const ResampleLayout L = resample_layout(n);
    char *ws = (char *)workspace;
    auto *wmax = (unsigned long long *)(ws + L.wmax);
    auto *P = (uint64_t *)(ws + L.P);
    auto *tsum = (uint64_t *)(ws + L.tiles);
    auto *sup = (uint64_t *)(ws + L.supers);
    auto *comb = (uint64_t *)(ws + L.comb);
    auto *start = (int64_t *)(ws + L.start);
    hipError_t e = zero_words((uint64_t *)wmax, 1, s);
    if (e != hipSuccess)
        return e;
    const dim3 qgrid((unsigned)qt), grid((unsigned)tiles), block(kBlock);
    const auto *cwmax = (const unsigned long long *)wmax;
    // the tile maxima live in the tile-sum array until the tile sums replace them
    hipLaunchKernelGGL(rs_tile_max_kernel, qgrid, block, 0, s, S.w, S.phase, n, tsum);
    hipLaunchKernelGGL(rs_max_groups_kernel, dim3((unsigned)groups), block, 0, s, (const uint64_t *)tsum, qt, wmax);
    hipLaunchKernelGGL(rs_tile_sum_kernel, qgrid, block, 0, s, S.w, S.phase, n, cwmax, tsum);
    hipLaunchKernelGGL(rs_scan_groups_kernel, dim3((unsigned)groups), block, 0, s, tsum, qt, sup);
    hipLaunchKernelGGL(rs_scan_top_kernel, dim3(1), block, 0, s, sup, groups);
    hipLaunchKernelGGL(rs_prefix_kernel, qgrid, block, 0, s, S.w, S.phase, n, cwmax, (const uint64_t *)tsum,
                       (const uint64_t *)sup, groups, P);
    // one lane per gather workgroup plus the closing entry
    hipLaunchKernelGGL(rs_bounds_kernel, dim3((unsigned)n_tiles(tiles + 1)), block, 0, s, (const uint64_t *)P, n,
                       tiles, (uint32_t)seed, (uint32_t)(seed >> 32), (uint64_t)S.traj_offset, (uint64_t)S.step, comb,
                       start);
    if (S.prec == QCL_FP64)
        hipLaunchKernelGGL(rs_gather_kernel<double>, grid, block, 0, s, ens_dev_rs<double>(S), ens_dev_rs<double>(D),
                           m.m, m.n * m.n, (const uint64_t *)P, (const uint64_t *)comb, (const int64_t *)start,
                           cwmax);
    else
        hipLaunchKernelGGL(rs_gather_kernel<float>, grid, block, 0, s, ens_dev_rs<float>(S), ens_dev_rs<float>(D),
                           m.m, m.n * m.n, (const uint64_t *)P, (const uint64_t *)comb, (const int64_t *)start,
                           cwmax);
    return hipGetLastError();
}

}  // namespace qcl
