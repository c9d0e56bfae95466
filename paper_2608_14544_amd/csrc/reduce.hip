// Ensemble averages from tile partials (Sec. II.B: fixed summation order).
//
// The partials hold, per tile of QCL_TILE walkers, the sums of every bin
// value and the number of walkers excluded from each bin.  They are
// combined by a perfect pairwise tree over the tile index (zero-padded):
// each pass adds groups of 8 consecutive rows as
// ((x0+x1)+(x2+x3))+((x4+x5)+(x6+x7)), i.e. three levels of the binary tree,
// until one row remains.  The final kernel turns the sums into means and
// standard errors.  The work is HBM-bound and tiny next to propagation.
#include <algorithm>
#include <cstring>

#include "qcl_internal.hpp"

namespace qcl {
namespace {

__global__ __launch_bounds__(256) void pairwise8_kernel(const double *__restrict__ in, int64_t rows_in, int64_t cols,
                                                        double *__restrict__ out)
{
    const int64_t rows_out = (rows_in + 7) / 8;
    const int64_t n = rows_out * cols;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = idx / cols, c = idx - r * cols;
        double x[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int64_t rr = 8 * r + k;
            x[k] = rr < rows_in ? in[rr * cols + c] : 0.0;
        }
        out[idx] = ((x[0] + x[1]) + (x[2] + x[3])) + ((x[4] + x[5]) + (x[6] + x[7]));
    }
}

// sums: per bin 2 N^2 groups (Re, Im, Re^2, Im^2) followed by the excluded
// count -> out [n_out][2][N][N] (mean Re, mean Im, SE Re, SE Im) and, when
// excluded is given, the counts [n_out]
__global__ __launch_bounds__(256) void finalize_kernel(const double *__restrict__ sums, int32_t n_out,
                                                       int32_t groups_per_bin, double T, double *__restrict__ out,
                                                       int64_t *__restrict__ excluded)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n_groups = (int64_t)n_out * groups_per_bin;
    const int64_t row = 4LL * groups_per_bin + 1;  // doubles per bin
    if (g < n_groups) {
        const int64_t o = g / groups_per_bin, k = g - o * groups_per_bin;
        const double *s = sums + o * row + 4 * k;
        const double s0 = s[0], s1 = s[1], s2 = s[2], s3 = s[3];
        const double vr = (s2 - s0 * s0 / T) / (T * (T - 1.0));
        const double vi = (s3 - s1 * s1 / T) / (T * (T - 1.0));
        out[4 * g + 0] = s0 / T;
        out[4 * g + 1] = s1 / T;
        out[4 * g + 2] = (T > 1.0 && vr > 0.0) ? sqrt(vr) : 0.0;
        out[4 * g + 3] = (T > 1.0 && vi > 0.0) ? sqrt(vi) : 0.0;
    }
    if (excluded && g < n_out)
        excluded[g] = (int64_t)sums[g * row + row - 1];
}

// Host words travel inside the kernel arguments (captured at launch), so the
// copy is asynchronous with no host buffer to keep alive, and graph-safe.
constexpr int kUploadWords = 480;
struct WordChunk {
    uint64_t w[kUploadWords];
    int32_t n;
};

__global__ __launch_bounds__(256) void upload_kernel(WordChunk c, uint64_t *__restrict__ dst)
{
    for (int i = threadIdx.x; i < c.n; i += blockDim.x)
        dst[i] = c.w[i];
}

__global__ __launch_bounds__(256) void zero_kernel(uint64_t *__restrict__ dst, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = 0;
}

}  // namespace

hipError_t upload_words(const uint64_t *words, size_t n_words, uint64_t *dst, hipStream_t s)
{
    for (size_t off = 0; off < n_words; off += kUploadWords) {
        WordChunk c;
        c.n = (int32_t)std::min<size_t>(kUploadWords, n_words - off);
        std::memcpy(c.w, words + off, sizeof(uint64_t) * c.n);
        hipLaunchKernelGGL(upload_kernel, dim3(1), dim3(256), 0, s, c, dst + off);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

hipError_t zero_words(uint64_t *dst, size_t n_words, hipStream_t s)
{
    if (n_words == 0)
        return hipSuccess;
    const int64_t blocks = std::min<int64_t>(((int64_t)n_words + 255) / 256, 1024);
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s, dst, (int64_t)n_words);
    return hipGetLastError();
}

hipError_t launch_reduce(int n_states, double *partials, int64_t n_traj, int32_t n_out, double *out,
                         int64_t *excluded, hipStream_t s)
{
    const int64_t tiles = n_tiles(n_traj);
    const int64_t cols = (int64_t)n_out * tile_values(n_states);
    double *scratch_a = partials + tiles * cols;
    double *scratch_b = scratch_a + ((tiles + 7) / 8) * cols;
    const double *src = partials;
    int64_t rows = tiles;
    bool to_a = true;
    while (rows > 1) {
        double *dst = to_a ? scratch_a : scratch_b;
        const int64_t rows_out = (rows + 7) / 8;
        const int64_t work = rows_out * cols;
        const int64_t blocks = std::min<int64_t>((work + 255) / 256, 8192);
        hipLaunchKernelGGL(pairwise8_kernel, dim3((unsigned)blocks), dim3(256), 0, s, src, rows, cols, dst);
        hipError_t err = hipGetLastError();
        if (err != hipSuccess)
            return err;
        src = dst;
        rows = rows_out;
        to_a = !to_a;
    }
    const int32_t gpb = 2 * n_states * n_states;
    const int64_t threads = std::max<int64_t>((int64_t)n_out * gpb, n_out);
    hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, src, n_out, gpb,
                       (double)n_traj, out, excluded);
    return hipGetLastError();
}

}  // namespace qcl
