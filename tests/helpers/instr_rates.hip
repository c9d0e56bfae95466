// Issue cost of single gfx950 vector instructions, measured with
// independent chains: every lane runs CH chains of ITERS dependent copies of
// one operation, 8 workgroups of 256 lanes per compute unit (8 waves per
// SIMD), timed with HIP events (best of three launches).  Printed: SIMD
// cycles per wave64 operation at 2.4 GHz, where an operation is the short
// sequence named (the chain needs a second instruction for some kinds).
//
//     hipcc --offload-arch=gfx950 -O3 -Xclang -target-feature -Xclang -packed-fp32-ops \
//         tests/helpers/instr_rates.hip -o /tmp/instr_rates && /tmp/instr_rates
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

namespace {

constexpr int CH = 8;
constexpr int ITERS = 4096;
constexpr int kOps = 14;

template <int OP>
__global__ __launch_bounds__(256) void chains(uint32_t *out, uint32_t seed, uint32_t m0)
{
    uint32_t x[CH], y[CH];
    float f[CH], g[CH], h[CH];
    double d[CH], e[CH];
    const uint32_t t = blockIdx.x * 256 + threadIdx.x;
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        x[c] = t * 2654435761u + c * 977u + seed;
        y[c] = x[c] * 747796405u;
        f[c] = (float)(x[c] & 1023) * 1e-3f;
        g[c] = 0.999f - (float)(y[c] & 15) * 1e-6f;
        h[c] = (float)(y[c] & 255) * 1e-6f;
        d[c] = f[c];
        e[c] = g[c];
    }
    for (int it = 0; it < ITERS; ++it) {
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            if constexpr (OP == 0) f[c] = f[c] + g[c];                                          // v_add_f32
            if constexpr (OP == 1) f[c] = f[c] * g[c];                                          // v_mul_f32
            if constexpr (OP == 2) f[c] = __builtin_fmaf(f[c], 0.999f, 1e-3f);                  // v_fmamk_f32
            if constexpr (OP == 3) f[c] = __builtin_fmaf(f[c], g[c], h[c]);                     // v_fma_f32
            if constexpr (OP == 4) d[c] = d[c] + e[c];                                          // v_add_f64
            if constexpr (OP == 5) d[c] = d[c] * e[c];                                          // v_mul_f64
            if constexpr (OP == 6) d[c] = __builtin_fma(d[c], e[c], d[c]);                      // v_fma_f64
            if constexpr (OP == 7) f[c] = __builtin_amdgcn_rsqf(f[c] + 1.0f);                   // add + v_rsq_f32
            if constexpr (OP == 8) x[c] = (x[c] ^ m0) + 0x9e3779b9u;                            // xor + add
            if constexpr (OP == 9) x[c] = __builtin_amdgcn_bitop3_b32(x[c], y[c], m0, 0x96) + 1u;  // bitop3 + add
            if constexpr (OP == 10) {                                                           // v_mad_u64_u32 + xor
                const uint64_t p = (uint64_t)x[c] * m0;
                x[c] = (uint32_t)(p >> 32) ^ (uint32_t)p;
            }
            if constexpr (OP == 11) x[c] = __umulhi(x[c], m0) + x[c];                           // v_mul_hi_u32 + add
            if constexpr (OP == 12) x[c] = x[c] * m0 + 1u;                                      // v_mul_lo_u32 + add
            if constexpr (OP == 13) f[c] = (f[c] < g[c]) ? h[c] + f[c] : g[c] * f[c];           // cmp, cndmask, 2 f32
        }
    }
    uint32_t acc = 0;
#pragma unroll
    for (int c = 0; c < CH; ++c)
        acc ^= x[c] ^ __float_as_uint(f[c]) ^ (uint32_t)__double_as_longlong(d[c]);
    out[t] = acc;
}

template <int... I>
struct Table {
    static constexpr void (*k[sizeof...(I)])(uint32_t *, uint32_t, uint32_t) = {chains<I>...};
};

}  // namespace

int main()
{
    const int wg = 256 * 8;  // 8 workgroups per compute unit on 256 CUs
    const int n = wg * 256;  // one output word per lane: every write in bounds
    uint32_t *out = nullptr;
    if (hipMalloc(&out, n * sizeof(uint32_t)) != hipSuccess) {
        printf("hipMalloc failed\n");
        return 1;
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        printf("hipEventCreate failed\n");
        return 1;
    }
    const char *names[kOps] = {"v_add_f32", "v_mul_f32", "v_fmamk_f32 (one literal)", "v_fma_f32 (three registers)",
                               "v_add_f64", "v_mul_f64", "v_fma_f64", "v_add_f32 + v_rsq_f32", "v_xor + v_add_u32",
                               "v_bitop3_b32 + v_add_u32", "v_mad_u64_u32 + v_xor", "v_mul_hi_u32 + v_add_u32",
                               "v_mul_lo_u32 + v_add_u32", "v_cmp + v_cndmask + 2 f32"};
    using T = Table<0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13>;
    printf("%-30s %10s %22s\n", "operation", "best ms", "SIMD cycles per wave-op");
    for (int op = 0; op < kOps; ++op) {
        float best = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
            hipEventRecord(e0, 0);
            hipLaunchKernelGGL(T::k[op], dim3(wg), dim3(256), 0, 0, out, 12345u + rep, 0xD2511F53u);
            hipEventRecord(e1, 0);
            if (hipEventSynchronize(e1) != hipSuccess) {
                printf("launch failed\n");
                return 1;
            }
            float ms = 0.0f;
            hipEventElapsedTime(&ms, e0, e1);
            best = ms < best ? ms : best;
        }
        const double wave_ops_per_simd = (double)n / 64 * ITERS * CH / 1024;
        printf("%-30s %10.3f %22.2f\n", names[op], best, best * 1e-3 * 2.4e9 / wave_ops_per_simd);
        fflush(stdout);
    }
    hipFree(out);
    return hipGetLastError() == hipSuccess ? 0 : 1;
}
