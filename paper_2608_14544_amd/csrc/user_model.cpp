// Models with a supplied potential: the caller's device source is compiled
// with the library's N-state kernels (user_kernels.hpp) by hipRTC when the
// model is built, for gfx950, and the code object is loaded on the current
// device.  The program is
//
//   constants (QCL_TILE, flag bits, QCL_N, QCL_M, qcl_param[], 1/m_j)
//   the caller's source (qcl_potential, qcl_force, qcl_coupling)
//   #include "user_kernels.hpp"   (from the headers built into the library)
//   two extern "C" kernels: qcl_user_sample_kernel, qcl_user_propagate_kernel
//
// Parameters and masses enter as hexadecimal floating literals, exact.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <algorithm>
#include <cinttypes>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "qcl_internal.hpp"

namespace qcl {
namespace rtc {
// the device headers the run-time program includes (generated at build time)
extern const int n_headers;
extern const char *const header_names[];
extern const char *const header_texts[];
}  // namespace rtc

namespace {

constexpr const char *kSampleName = "qcl_user_sample_kernel";
constexpr const char *kPropagateName = "qcl_user_propagate_kernel";
constexpr const char *kBatchName = "qcl_user_batch_kernel";
constexpr const char *kSample32Name = "qcl_user_sample32_kernel";
constexpr const char *kPropagate32Name = "qcl_user_propagate32_kernel";
constexpr const char *kBatch32Name = "qcl_user_batch32_kernel";

// the same rotation threshold as the built-in binary64 kernels
constexpr double kRotEps64 = 64.0 * 1.1102230246251565e-16;

std::string hex_literal(double x)
{
    char buf[64];
    std::snprintf(buf, sizeof(buf), "%a", x);
    return buf;
}

std::string program_text(const qcl_model_s &m, const char *source, const double *params, int n_params)
{
    std::string s;
    char buf[160];
    auto line = [&](const char *fmt, auto... v) {
        std::snprintf(buf, sizeof(buf), fmt, v...);
        s += buf;
        s += '\n';
    };
    line("#define QCL_TILE %d", QCL_TILE);
    line("#define QCL_MAX_MODES %d", QCL_MAX_MODES);
    line("#define QCL_FLAG_NONFINITE %uu", QCL_FLAG_NONFINITE);
    line("#define QCL_FLAG_DEGENERATE %uu", QCL_FLAG_DEGENERATE);
    line("#define QCL_FLAG_RESOLVED64 %uu", QCL_FLAG_RESOLVED64);
    line("#define QCL_FLAG_FALLBACK %uu", QCL_FLAG_FALLBACK);
    line("#define QCL_TRANS_LINEAR %d", (int)QCL_TRANS_LINEAR);
    line("#define QCL_INIT_ADIABATIC %d", (int)QCL_INIT_ADIABATIC);
    line("#define QCL_N %d", m.n);
    line("#define QCL_M %d", m.m);
    line("#define QCL_N_PARAMS %d", n_params);
    s += "#include <cstdint>\n";
    s += "__device__ constexpr double qcl_param[";
    s += std::to_string(n_params > 0 ? n_params : 1);
    s += "] = {";
    for (int i = 0; i < n_params; ++i)
        s += (i ? ", " : "") + hex_literal(params[i]);
    if (n_params == 0)
        s += "0.0";
    s += "};\n#line 1 \"source\"\n";
    s += source;
    s += "\n#line 1 \"qcl_user_program\"\n#include \"user_kernels.hpp\"\n";
    s += "__device__ constexpr double qcl_inv_mass[QCL_M] = {";
    for (int j = 0; j < m.m; ++j)
        s += (j ? ", " : "") + hex_literal(1.0 / m.mass[j]);
    s += "};\n";
    // the three kernels per precision; the binary32 ones exist when the
    // source provides binary32 functions and says so (QCL_SOURCE_FP32)
    auto kernels = [&](const char *suffix, const char *R) {
        char b[2048];
        std::snprintf(
            b, sizeof(b),
            "extern \"C\" __global__ __launch_bounds__(QCL_TILE) void qcl_user_sample%s_kernel(\n"
            "    qcl::SampleArgs S, qcl::UserArgs A, qcl::EnsDev<%s> E, double *partials, int32_t n_out)\n"
            "{\n"
            "    __shared__ qcl::BinLds lds;\n"
            "    qcl::user_sample<QCL_N, QCL_M, %s>(S, A, E, partials, n_out, lds);\n"
            "}\n"
            "extern \"C\" __global__ __launch_bounds__(QCL_TILE) void qcl_user_propagate%s_kernel(\n"
            "    qcl::UserArgs A, qcl::PropArgs P, qcl::EnsDev<%s> E, double *partials)\n"
            "{\n"
            "    __shared__ qcl::BinLds lds;\n"
            "    qcl::user_propagate<QCL_N, QCL_M, %s>(A, P, E, qcl_inv_mass, partials, lds);\n"
            "}\n"
            "extern \"C\" __global__ __launch_bounds__(QCL_TILE) void qcl_user_batch%s_kernel(\n"
            "    const qcl::UserBatchItem<%s> *items, int32_t n_items, int64_t total_tiles,\n"
            "    unsigned long long *counter)\n"
            "{\n"
            "    __shared__ qcl::BinLds lds;\n"
            "    __shared__ long long item_sh;\n"
            "    qcl::user_batch<QCL_N, QCL_M, %s>(items, n_items, total_tiles, counter, qcl_inv_mass, lds,\n"
            "                                     item_sh);\n"
            "}\n",
            suffix, R, R, suffix, R, R, suffix, R, R);
        s += b;
    };
    kernels("", "double");
    s += "#ifdef QCL_SOURCE_FP32\n";
    kernels("32", "float");
    s += "#endif\n";
    return s;
}

// Jacobi thresholds as in the built-in kernels; the binary32 re-solve
// threshold is 1e-4 of the harmonic reference's largest quantum hbar w
UserArgs user_args(const qcl_model_s &m, double dt, bool fp32)
{
    double scale = 0.0;
    for (int j = 0; j < m.m; ++j)
        scale = std::max(scale, m.hbar * m.omega[j]);
    return UserArgs{dt, 0.5 * dt, dt / m.hbar, fp32 ? 64.0 * 5.9604644775390625e-08 : kRotEps64, 1e-4 * scale};
}

template <typename R>
EnsDev<R> ens_user(const qcl_ensemble &e)
{
    return EnsDev<R>{(R *)e.q, (R *)e.p, (R *)e.u, e.w, e.phase, e.a, e.b, e.flags, e.ld, e.n_traj, e.traj_offset};
}


}  // namespace

qcl_status user_compile(qcl_model_s &m, const char *source, const double *params, int n_params)
{
    const std::string text = program_text(m, source, params, n_params);
    hiprtcProgram prog = nullptr;
    hiprtcResult r = hiprtcCreateProgram(&prog, text.c_str(), "qcl_user_program.hip", rtc::n_headers,
                                         rtc::header_texts, rtc::header_names);
    if (r != HIPRTC_SUCCESS)
        return set_error(QCL_ERR_DEVICE, "hiprtcCreateProgram: %s", hiprtcGetErrorString(r));
    // No contraction of separate multiplies and adds: the supplied functions
    // are inlined at the start of a call and inside the step loop, and both
    // copies must round alike for a run split over calls to reproduce the
    // uninterrupted one bit for bit (fma() in the source still fuses).
    const char *opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off", "-Xclang",
                          "-target-feature", "-Xclang", "-packed-fp32-ops"};
    r = hiprtcCompileProgram(prog, (int)(sizeof(opts) / sizeof(opts[0])), opts);
    if (r != HIPRTC_SUCCESS) {
        size_t n = 0;
        std::string log;
        if (hiprtcGetProgramLogSize(prog, &n) == HIPRTC_SUCCESS && n > 1) {
            log.resize(n);
            (void)hiprtcGetProgramLog(prog, &log[0]);
        }
        (void)hiprtcDestroyProgram(&prog);
        // the first lines of the log name the failing line of the source
        if (log.size() > 400)
            log.resize(400);
        return set_error(QCL_ERR_INVALID_ARG, "the potential source does not compile: %s", log.c_str());
    }
    size_t code_size = 0;
    r = hiprtcGetCodeSize(prog, &code_size);
    if (r == HIPRTC_SUCCESS) {
        m.user_code.resize(code_size);
        r = hiprtcGetCode(prog, m.user_code.data());
    }
    (void)hiprtcDestroyProgram(&prog);
    if (r != HIPRTC_SUCCESS)
        return set_error(QCL_ERR_DEVICE, "hiprtcGetCode: %s", hiprtcGetErrorString(r));
    return QCL_OK;
}

qcl_status user_load(qcl_model_s &m)
{
    hipModule_t mod = nullptr;
    hipError_t e = hipModuleLoadData(&mod, m.user_code.data());
    if (e != hipSuccess)
        return set_error(QCL_ERR_DEVICE, "hipModuleLoadData: %s", hipGetErrorString(e));
    hipFunction_t fs = nullptr, fp = nullptr, fb = nullptr;
    e = hipModuleGetFunction(&fs, mod, kSampleName);
    if (e == hipSuccess)
        e = hipModuleGetFunction(&fp, mod, kPropagateName);
    if (e == hipSuccess)
        e = hipModuleGetFunction(&fb, mod, kBatchName);
    if (e != hipSuccess) {
        (void)hipModuleUnload(mod);
        return set_error(QCL_ERR_DEVICE, "hipModuleGetFunction: %s", hipGetErrorString(e));
    }
    m.user_module = mod;
    m.user_sample = (void *)fs;
    m.user_propagate = (void *)fp;
    m.user_batch = (void *)fb;
    // binary32 kernels: present only when the source provides them
    hipFunction_t fs32 = nullptr, fp32 = nullptr, fb32 = nullptr;
    if (hipModuleGetFunction(&fs32, mod, kSample32Name) == hipSuccess &&
        hipModuleGetFunction(&fp32, mod, kPropagate32Name) == hipSuccess &&
        hipModuleGetFunction(&fb32, mod, kBatch32Name) == hipSuccess) {
        m.user_sample32 = (void *)fs32;
        m.user_propagate32 = (void *)fp32;
        m.user_batch32 = (void *)fb32;
    }
    (void)hipGetLastError();  // a kernel the source did not ask for is no error
    return QCL_OK;
}

void user_release(qcl_model_s &m)
{
    if (m.user_module)
        (void)hipModuleUnload((hipModule_t)m.user_module);
    m.user_module = m.user_sample = m.user_propagate = m.user_batch = nullptr;
    m.user_sample32 = m.user_propagate32 = m.user_batch32 = nullptr;
}

hipError_t launch_user_sample(const qcl_model_s &m, const SampleArgs &sa_in, const qcl_ensemble &ens,
                              double *partials, int32_t n_out, hipStream_t s)
{
    SampleArgs sa = sa_in;
    sa.m = m.m;
    UserArgs A = user_args(m, 1.0, false);  // sampling is binary64 in both precisions
    const unsigned grid = (unsigned)n_tiles(ens.n_traj);
    if (ens.prec == QCL_FP32_ACC64) {
        EnsDev<float> E = ens_user<float>(ens);
        void *args[] = {&sa, &A, &E, &partials, &n_out};
        return hipModuleLaunchKernel((hipFunction_t)m.user_sample32, grid, 1, 1, kBlock, 1, 1, 0, s, args, nullptr);
    }
    EnsDev<double> E = ens_user<double>(ens);
    void *args[] = {&sa, &A, &E, &partials, &n_out};
    return hipModuleLaunchKernel((hipFunction_t)m.user_sample, grid, 1, 1, kBlock, 1, 1, 0, s, args, nullptr);
}

hipError_t launch_user_propagate(const qcl_model_s &m, const qcl_ensemble &ens, const qcl_prop_desc &pd,
                                 double *partials, hipStream_t s)
{
    const bool fp32 = ens.prec == QCL_FP32_ACC64;
    UserArgs A = user_args(m, pd.dt, fp32);
    PropArgs P{ens.step, pd.n_steps, pd.cadence, pd.n_out, pd.scheme, (uint32_t)pd.seed, (uint32_t)(pd.seed >> 32),
               m.m};
    const unsigned grid = (unsigned)n_tiles(ens.n_traj);
    if (fp32) {
        EnsDev<float> E = ens_user<float>(ens);
        void *args[] = {&A, &P, &E, &partials};
        return hipModuleLaunchKernel((hipFunction_t)m.user_propagate32, grid, 1, 1, kBlock, 1, 1, 0, s, args,
                                     nullptr);
    }
    EnsDev<double> E = ens_user<double>(ens);
    void *args[] = {&A, &P, &E, &partials};
    return hipModuleLaunchKernel((hipFunction_t)m.user_propagate, grid, 1, 1, kBlock, 1, 1, 0, s, args, nullptr);
}

template <typename R>
void write_user_item(const qcl_model_s &m, const qcl_ensemble &ens, const qcl_prop_desc &pd, double *partials,
                     int64_t tile_begin, void *out)
{
    UserBatchItem<R> it{};
    it.A = user_args(m, pd.dt, sizeof(R) == 4);
    it.P = PropArgs{ens.step, pd.n_steps, pd.cadence, pd.n_out, pd.scheme, (uint32_t)pd.seed,
                    (uint32_t)(pd.seed >> 32), m.m};
    it.E = ens_user<R>(ens);
    it.partials = partials;
    it.tile_begin = tile_begin;
    std::memcpy(out, &it, sizeof(it));
}

size_t batch_item_user(const qcl_model_s &m, const qcl_ensemble &ens, const qcl_prop_desc &pd, double *partials,
                       int64_t tile_begin, void *out)
{
    if (out) {
        if (ens.prec == QCL_FP32_ACC64)
            write_user_item<float>(m, ens, pd, partials, tile_begin, out);
        else
            write_user_item<double>(m, ens, pd, partials, tile_begin, out);
    }
    return sizeof(UserBatchItem<double>);
}

hipError_t launch_user_batch(const qcl_model_s &m, int prec, int wpc, const void *items, int32_t n_items,
                             int64_t total_tiles, unsigned long long *counter, hipStream_t s)
{
    const hipFunction_t fn = (hipFunction_t)(prec == QCL_FP32_ACC64 ? m.user_batch32 : m.user_batch);
    int cus = 0, per_cu = 0, dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBlock, 0);
    const int64_t grid = persistent_grid(total_tiles, cus, per_cu, wpc);
    const void *it = items;
    void *args[] = {&it, &n_items, &total_tiles, &counter};
    return hipModuleLaunchKernel(fn, (unsigned)grid, 1, 1, kBlock, 1, 1, 0, s, args, nullptr);
}

}  // namespace qcl
