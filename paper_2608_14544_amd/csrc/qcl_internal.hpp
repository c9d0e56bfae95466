// Internal declarations shared by the host API and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <type_traits>
#include <vector>

#include "qcl.h"
#include "qcl_device.hpp"

namespace qcl {


// Two-state model in the form the analytic kernels use: with
// V(q) = Vbar(q) I + [[dl, cc], [cc, -dl]],
//   dl(q) = dlt0 + sum_j dlt_j q_j,  cc(q) = c0 + sum_j cpl_j q_j,
// the adiabatic energies are Vbar -+ r, r = sqrt(dl^2 + cc^2), and
// dE_{0,1}/dq_j = kbar_j -+ (dl dlt_j + cc cpl_j)/r.  Constants that only
// ever appear multiplied by a step length are stored pre-multiplied.
template <int M, typename R>
struct N2Const {
    R dlt[M];   // (K_00 - K_11)/2
    R cpl[M];   // K_01
    R vdl[M];   // dt/m_j (K_00 - K_11)/2: p_j vdl_j sums to dt dl_v
    R vcp[M];   // dt/m_j K_01
    R hk[M];    // (dt/2) m_j w_j^2
    R hb[M];    // (dt/2) (K_00 + K_11)/2
    R dtm[M];   // dt/m_j
    R dlt0;     // (V0_00 - V0_11)/2
    R c0;       // V0_01
    R hdt;      // dt/2
    R hdt2;     // dt/4 (the kick factor (a + b - 1) (dt/2)/r is (sa + sb) (dt/4)/r with sa = 2a - 1)
    R gap_half; // binary32 path: points with r below this (a gap 2r below 1e-4 of the
                // model's energy scale) are re-solved in binary64
    double dt_hbar;
    double dt_hbar2;  // dt/(2 hbar), the phase factor for sa - sb = 2 (a - b)
    // binary64 copies [dlt0, c0, dlt_0..M-1, cpl_0..M-1] in device memory,
    // read only by the binary32 path's near-degenerate re-solve
    const double *c64;
};

// General-N model constants in device memory (both precisions).  The
// mode couplings are factored as K_j = sum_r C_jr B_r over an orthonormal
// basis {B_r} of the span of the K_j (rank R <= T = N(N+1)/2 upper-triangle
// slots), padded with zero rows to a rank bucket RB in {1, N, T}:
//   v0    [T]                        upper triangle of V0 (row-major)
//   basis [RB][T]                    B_r
//   modes [kMaxModesPad][2 + 2 RB]   m w^2, 1/m, C_j0..C_j(RB-1), C_jr/m_j
// zero-padded past the model's modes so that padded modes stay at rest.
// When every direction is kept (RB = T) the basis is the slot basis (B_r
// the unit matrix of slot r) and C_jr the slot values of K_j; the kernels
// then skip the contractions with it.
// A model with higher powers (V(q) = V0 + sum_j sum_{k=1..4} q_j^k A_jk,
// A_j1 = K_j) factors all its A_jk over one basis, A_jk = sum_r C_jkr B_r,
// with RB = T, and its mode rows hold per direction r the coefficients of
// phi_jr(x) = sum_k C_jkr x^k and of its derivative:
//   modes [kMaxModesPad][2 + 8 RB]   m w^2, 1/m, then per r:
//                                    C_j1r..C_j4r, 1 C_j1r, 2 C_j2r, 3 C_j3r, 4 C_j4r
constexpr int kMaxModesPad = 128;

template <typename R>
struct GenConst {
    const R *v0;
    const R *basis;
    const R *modes;
    const R *sq;  // bilinear models: [kSq][RB] slot weights of the squared mode combinations
    R dt, hdt;
    double dt_hbar;
    R gap_thr;  // binary32 path: gaps below this are re-solved in binary64
    R rot_eps;  // Jacobi: rotate while |a_pq| > rot_eps * ||A||_F
    int32_t basis_diag;  // rank one: the one coupling direction is diagonal
};

// squared mode combinations of a bilinear model: the kernels are built for
// 4, 8 and kSq of them (kSq: at most 16 modes)
constexpr int kSq = 16;
inline int sq_pad(int n_sq) { return n_sq <= 4 ? 4 : n_sq <= 8 ? 8 : kSq; }

inline int64_t n_tiles(int64_t n_traj) { return (n_traj + kBlock - 1) / kBlock; }

// Workgroups of a persistent batched launch: every compute unit gets the
// workgroups that fit (per_cu), or at most wpc of them when wpc > 0; never
// more than there are tiles.
inline int64_t persistent_grid(int64_t total_tiles, int cus, int per_cu, int wpc)
{
    const int per = wpc > 0 ? std::min(wpc, std::max(1, per_cu)) : std::max(1, per_cu);
    return std::min<int64_t>(total_tiles, (int64_t)std::max(1, cus) * per);
}

inline int padded_modes(int m)
{
    return m <= 4 ? 4 : m <= 8 ? 8 : m <= 16 ? 16 : m <= 32 ? 32 : m <= 64 ? 64 : 128;
}

// rank bucket: 1, N or T = N(N+1)/2 (for more than 4 states only 1 or T)
inline int rank_bucket(int rank, int n)
{
    return rank <= 1 ? 1 : (rank <= n && n <= 4) ? n : n * (n + 1) / 2;
}


// Two-state model with higher powers of each mode: per mode j the
// polynomials (no constant term) of dl, of cc and of Vbar, each in four
// coefficients c_1..c_4 (value) and 1c_1..4c_4 (slope); the linear part K_j
// is c_1.  dl = dlt0 + sum_j phi^d_j(q_j), cc = c0 + sum_j phi^c_j(q_j), and
// the mean force needs only the slope of phi^b_j.
template <int M, typename R>
struct N2Poly {
    R dv[M][4], ds[M][4];  // dl: value and slope coefficients
    R cv[M][4], cs[M][4];  // cc
    R bs[M][4];            // Vbar: slope coefficients
    // binary64 copies [dlt0, c0, dv[M][4], cv[M][4]] in device memory, read
    // only by the binary32 path's near-degenerate re-solve
    const double *c64;
};
struct N2Linear {};  // no extra constants for a linear model

template <int M, typename R, bool POLY>
using N2Extra = std::conditional_t<POLY, N2Poly<M, R>, N2Linear>;

// Batched work: one descriptor per instance, tile_begin = prefix sum of the
// tiles of the preceding descriptors of the same kernel class.
template <int M, typename R, bool POLY = false>
struct BatchItemN2 {
    N2Const<M, R> C;
    N2Extra<M, R, POLY> Q;
    PropArgs P;
    EnsDev<R> E;
    double *partials;
    int64_t tile_begin;
};

template <typename R>
struct BatchItemGen {
    GenConst<R> C;
    GenConst<double> C64;
    PropArgs P;
    EnsDev<R> E;
    double *partials;
    int64_t tile_begin;
};

}  // namespace qcl

struct qcl_model_s {
    int32_t n;
    int32_t m;
    double hbar;
    std::vector<double> mass, omega, v0, k;
    // two-state derived constants (binary64)
    std::vector<double> kq, minv, kbar, dlt, cpl;  // m w^2, 1/m, (K00+K11)/2, (K00-K11)/2, K01
    double dlt0 = 0.0, c0 = 0.0;
    double energy_scale = 1.0;
    int device = 0;
    // built from device source (qcl_create_model_source): the code object
    // compiled for it and its two kernels (hipModule_t, hipFunction_t)
    bool source = false;
    std::vector<char> user_code;
    void *user_module = nullptr;
    void *user_sample = nullptr;
    void *user_propagate = nullptr;
    void *user_batch = nullptr;
    void *user_sample32 = nullptr;  // binary32 kernels, when the source provides binary32 functions
    void *user_propagate32 = nullptr;
    void *user_batch32 = nullptr;
    double *d_model = nullptr;  // device: V0 [N*N], K [M*N*N], then two-state binary64
                                // constants [dlt0, c0, dlt[M], cpl[M]]
    size_t c64_offset = 0;      // element offset of the two-state constants
    size_t n2poly64_offset = 0; // element offset of the two-state polynomial constants (binary64)
    std::vector<double> n2poly; // [M][5][4]: dv, ds, cv, cs, bs per mode (two states, higher powers)
    size_t gen64_offset = 0;    // element offset of the general-N binary64 constants
    size_t gen32_byte_offset = 0;  // byte offset of the general-N binary32 constants
    int32_t rank = 0;           // rank of the mode couplings (general-N factorisation)
    int32_t rank_pad = 1;       // rank bucket RB the general kernels are specialised on
    int32_t basis_diag = 0;     // rank one: the coupling direction has no off-diagonal slots
    int32_t degree = 1;         // highest power of q_j in V(q) (> 1: kernels_poly{N}.hip)
    std::vector<double> poly;   // [M][degree-1][N][N] higher-power matrices A_jk (k >= 2)
    int32_t n_pairs = 0;        // bilinear terms (> 0: kernels_bil{,h,w}{N}.hip)
    std::vector<int32_t> pairs; // [n_pairs][2] modes of each term
    std::vector<double> bpair;  // [n_pairs][N][N] B_p
    int32_t n_sq = 0;           // squared mode combinations representing them
    std::vector<double> sq_c;   // [n_sq][M] mode coefficients of each combination
    std::vector<double> sq_lam; // [n_sq][T] slot weights (X_r += lam_sr y_s^2 / 2)
    bool fast2 = false;         // two-state closed-form kernels apply (N = 2, M <= 8)
};

namespace qcl {

hipError_t launch_sample_n2(const qcl_model_s &m, const SampleArgs &sa, const qcl_ensemble &ens,
                            double *partials, int32_t n_out, hipStream_t stream);
hipError_t launch_propagate_n2(const qcl_model_s &m, const qcl_ensemble &ens, const qcl_prop_desc &pd,
                               double *partials, hipStream_t stream);
template <int K>
struct int_ {};  // general kernels of K states, linear couplings (kernels_gen{K}.hip)
template <int K>
struct poly_ {};  // general kernels of K states, higher powers (kernels_poly{K}.hip)
template <int K>
struct bil_ {};   // general kernels of K states, higher powers and bilinear terms as 8 squares (kernels_bil{K}.hip)
template <int K>
struct bilh_ {};  // the same with 4 squares (kernels_bilh{K}.hip)
template <int K>
struct bilw_ {};  // the same with 16 squares, at most 16 modes (kernels_bilw{K}.hip)

#define QCL_DECLARE_GENERAL(TAG)                                                                              \
    hipError_t launch_sample_general_n(const qcl_model_s &m, const SampleArgs &sa, const qcl_ensemble &ens,   \
                                       double *partials, int32_t n_out, hipStream_t s, TAG);                 \
    hipError_t launch_propagate_general_n(const qcl_model_s &m, const qcl_ensemble &ens,                     \
                                          const qcl_prop_desc &pd, double *partials, hipStream_t s, TAG);    \
    size_t batch_item_general_n(const qcl_model_s &m, const qcl_ensemble &ens, const qcl_prop_desc &pd,      \
                                double *partials, int64_t tile_begin, void *out, TAG);                       \
    hipError_t launch_batch_general_n(int mp, int rb, int prec, int occ, int wpc, const void *items,           \
                                      int32_t n_items,                                                     \
                                      int64_t total_tiles, unsigned long long *counter, hipStream_t s, TAG);
QCL_DECLARE_GENERAL(int_<2>)
QCL_DECLARE_GENERAL(int_<3>)
QCL_DECLARE_GENERAL(int_<4>)
QCL_DECLARE_GENERAL(int_<5>)
QCL_DECLARE_GENERAL(int_<6>)
QCL_DECLARE_GENERAL(int_<7>)
QCL_DECLARE_GENERAL(int_<8>)
QCL_DECLARE_GENERAL(poly_<2>)
QCL_DECLARE_GENERAL(poly_<3>)
QCL_DECLARE_GENERAL(poly_<4>)
QCL_DECLARE_GENERAL(bil_<2>)
QCL_DECLARE_GENERAL(bil_<3>)
QCL_DECLARE_GENERAL(bil_<4>)
QCL_DECLARE_GENERAL(bilh_<2>)
QCL_DECLARE_GENERAL(bilh_<3>)
QCL_DECLARE_GENERAL(bilh_<4>)
QCL_DECLARE_GENERAL(bilw_<2>)
QCL_DECLARE_GENERAL(bilw_<3>)
QCL_DECLARE_GENERAL(bilw_<4>)
#undef QCL_DECLARE_GENERAL

// Calls fn with the tag of the general kernels a model runs on; `none` when
// the state count has none (never, for a validated model).
template <typename Ret, typename F>
inline Ret with_general(const qcl_model_s &m, Ret none, F &&fn)
{
    if (m.n_pairs > 0 && sq_pad(m.n_sq) == 4) {
        switch (m.n) {
        case 2: return fn(bilh_<2>{});
        case 3: return fn(bilh_<3>{});
        case 4: return fn(bilh_<4>{});
        default: return none;
        }
    }
    if (m.n_pairs > 0 && sq_pad(m.n_sq) == kSq) {
        switch (m.n) {
        case 2: return fn(bilw_<2>{});
        case 3: return fn(bilw_<3>{});
        case 4: return fn(bilw_<4>{});
        default: return none;
        }
    }
    if (m.n_pairs > 0) {
        switch (m.n) {
        case 2: return fn(bil_<2>{});
        case 3: return fn(bil_<3>{});
        case 4: return fn(bil_<4>{});
        default: return none;
        }
    }
    if (m.degree > 1) {
        switch (m.n) {
        case 2: return fn(poly_<2>{});
        case 3: return fn(poly_<3>{});
        case 4: return fn(poly_<4>{});
        default: return none;
        }
    }
    switch (m.n) {
    case 2: return fn(int_<2>{});
    case 3: return fn(int_<3>{});
    case 4: return fn(int_<4>{});
    case 5: return fn(int_<5>{});
    case 6: return fn(int_<6>{});
    case 7: return fn(int_<7>{});
    case 8: return fn(int_<8>{});
    default: return none;
    }
}

size_t batch_item_n2(const qcl_model_s &m, const qcl_ensemble &ens, const qcl_prop_desc &pd, double *partials,
                     int64_t tile_begin, void *out);
hipError_t launch_batch_n2(int modes, bool poly, int prec, int scheme, int wpc, const void *items, int32_t n_items,
                           int64_t total_tiles, unsigned long long *counter, hipStream_t s);
// device-side copy of host words carried in kernel arguments; zeroing of counters
hipError_t upload_words(const uint64_t *words, size_t n_words, uint64_t *dst, hipStream_t s);
hipError_t zero_words(uint64_t *dst, size_t n_words, hipStream_t s);

size_t batch_item_user(const qcl_model_s &m, const qcl_ensemble &ens, const qcl_prop_desc &pd, double *partials,
                       int64_t tile_begin, void *out);

inline size_t batch_item(const qcl_model_s &m, const qcl_ensemble &ens, const qcl_prop_desc &pd, double *partials,
                         int64_t tile_begin, void *out)
{
    if (m.source)
        return batch_item_user(m, ens, pd, partials, tile_begin, out);
    if (m.fast2)
        return batch_item_n2(m, ens, pd, partials, tile_begin, out);
    return with_general(m, size_t(0),
                        [&](auto tag) { return batch_item_general_n(m, ens, pd, partials, tile_begin, out, tag); });
}

// The register-budget variant a call runs: the one asked for where such
// kernels exist (binary32, general kernels of a linear model; 3 with at most
// 32 padded modes (16 for four states), 2 with 64), else 0.
inline int occupancy_variant(const qcl_model_s &m, int prec, int requested)
{
    if (m.source || m.fast2 || m.degree != 1 || m.n > 4 || prec != QCL_FP32_ACC64)
        return 0;
    const int mp = padded_modes(m.m);
    if (requested == 3 && mp <= (m.n >= 4 ? 16 : 32))
        return 3;
    if (requested == 2 && mp == 64)
        return 2;
    return 0;
}

// Models with a supplied potential (user_model.cpp): compilation of the
// caller's source with the library's kernels, loading on the current
// device, launches and release.
qcl_status user_compile(qcl_model_s &m, const char *source, const double *params, int n_params);
qcl_status user_load(qcl_model_s &m);
void user_release(qcl_model_s &m);
hipError_t launch_user_sample(const qcl_model_s &m, const SampleArgs &sa, const qcl_ensemble &ens, double *partials,
                              int32_t n_out, hipStream_t s);
hipError_t launch_user_propagate(const qcl_model_s &m, const qcl_ensemble &ens, const qcl_prop_desc &pd,
                                 double *partials, hipStream_t s);
hipError_t launch_user_batch(const qcl_model_s &m, int prec, int wpc, const void *items, int32_t n_items,
                             int64_t total_tiles, unsigned long long *counter, hipStream_t s);

// wpc: workgroups per compute unit of the persistent launch (0: as many as
// fit, else at most that many)
inline hipError_t launch_batch(const qcl_model_s &m, int prec, int scheme, int occ, int wpc, const void *items,
                               int32_t n_items, int64_t total_tiles, unsigned long long *counter, hipStream_t s)
{
    if (m.source)  // each supplied potential is its own compiled program
        return launch_user_batch(m, prec, wpc, items, n_items, total_tiles, counter, s);
    if (m.fast2)  // the transition rule is a template parameter of the two-state kernels
        return launch_batch_n2(m.m, m.degree > 1, prec, scheme, wpc, items, n_items, total_tiles, counter, s);
    const int mp = padded_modes(m.m), rb = m.rank_pad;
    return with_general(m, hipErrorNotSupported, [&](auto tag) {
        return launch_batch_general_n(mp, rb, prec, occ, wpc, items, n_items, total_tiles, counter, s, tag);
    });
}

inline hipError_t launch_sample_general(const qcl_model_s &m, const SampleArgs &sa, const qcl_ensemble &ens,
                                        double *partials, int32_t n_out, hipStream_t s)
{
    return with_general(m, hipErrorNotSupported,
                        [&](auto tag) { return launch_sample_general_n(m, sa, ens, partials, n_out, s, tag); });
}

inline hipError_t launch_propagate_general(const qcl_model_s &m, const qcl_ensemble &ens, const qcl_prop_desc &pd,
                                           double *partials, hipStream_t s)
{
    return with_general(m, hipErrorNotSupported,
                        [&](auto tag) { return launch_propagate_general_n(m, ens, pd, partials, s, tag); });
}
// Records the thread's last error (qcl_last_error) and returns st.
qcl_status set_error(qcl_status st, const char *fmt, ...);

// qcl_propagate_batch with a given workspace; fixed_workspace marks the
// library's static per-device array (limit reported as such, no side streams).
qcl_status propagate_batch_in(const qcl_batch_item *items, int32_t n_items, void *workspace, size_t workspace_bytes,
                              void *stream, bool fixed_workspace);

// Reduces the tile partials to out [n_out][2][N][N][4]; when excluded is
// not NULL, also writes there the number of walkers excluded from each bin
// (int64 [n_out]).
hipError_t launch_reduce(int n_states, double *partials, int64_t n_traj, int32_t n_out, double *out,
                         int64_t *excluded, hipStream_t stream);

// workspace of qcl_resample: byte offsets of its parts and the total
struct ResampleLayout {
    size_t wmax, P, tiles, supers, comb, start, bytes;  // byte offsets into the workspace, total size
};
ResampleLayout resample_layout(int64_t n_traj);
hipError_t launch_resample(const qcl_model_s &m, const qcl_ensemble &src, const qcl_ensemble &dst, uint64_t seed,
                           void *workspace, hipStream_t stream);


}  // namespace qcl
