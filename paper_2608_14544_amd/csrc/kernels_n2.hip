// Two-state kernels for gfx950: initial sampling and multi-step propagation
// of the QCL walker ensemble (Eq. 1), one walker per lane, whole state in
// registers for the entire step loop.
//
// For N = 2 the adiabatic problem is solved in closed form (no iteration):
// with V(q) = Vbar I + [[dl, cc], [cc, -dl]] the energies are Vbar -+ r,
// r = sqrt(dl^2 + cc^2) (computed without cancellation, also near a
// conical intersection).  The upper eigenvector is parallel to
//     x = (r + dl, cc) for dl >= 0,   x = (cc, r - dl) otherwise,
// (both forms are the same direction up to sign; each is free of
// cancellation on its side), and the lower one to (-x1, x0).  The tracked
// frame is U = [s0 (-x1, x0), s1 (x0, x1)] / |x| with column signs s0, s1.
//
// The step needs no eigenvector:
//   * the mean force of element (a,b) is a gradient of Vbar -+ r,
//       (F_a + F_b)_j / 2 = -m w^2 q_j - kbar_j - (a+b-1)(dl dlt_j + cc cpl_j)/r;
//   * the velocity-projected coupling is
//       v.d_01 = s0 s1 (dl c_v - cc dl_v) / (2 r^2),
//     dl_v = sum_j v_j dlt_j, c_v = sum_j v_j cpl_j;
//   * keeping each column continuous (flip when its overlap with the
//     previous column is negative) flips s0 and s1 together, exactly when
//     x_old . x_new < 0, so s0 s1 is constant along a walker.
// Normalised eigenvectors are formed only for output bins and for the
// frame stored at the end of a call.
//
// Models with higher powers of each mode (POLY) keep the closed form: dl,
// cc and Vbar become sums of per-mode polynomials, evaluated by Horner's
// rule, and the constants dlt_j, cpl_j, kbar_j above become the slopes of
// those polynomials at q_j, computed once per point and kept in registers
// for the coupling and the two kicks that use them.
#include <algorithm>
#include <cstring>

#include "block_reduce.hpp"
#include "phase_math.hpp"
#include "philox.hpp"
#include "qcl_internal.hpp"

// Floating-point contraction is off in this file: every fused multiply-add
// is written out (fma2), so each copy of the step body in the unrolled loop
// below computes exactly the same operations, and a walker's result does
// not depend on which copy ran a given step (calls split anywhere give the
// same bits).
#pragma clang fp contract(off)

namespace qcl {
namespace {

__device__ __forceinline__ float fma2(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma2(double a, double b, double c) { return __builtin_fma(a, b, c); }

// 1/sqrt.  binary32: the hardware v_rsq_f32 (about 1 ulp); arguments are
// squared gaps that are either well above the binary32 denormal range or
// re-solved in binary64.  binary64: the library rsqrt.
__device__ __forceinline__ double rsq(double x) { return rsqrt(x); }
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }

// Geometry of the 2x2 problem at one point: dl, cc, r = sqrt(dl^2+cc^2),
// 1/r and the unnormalised canonical upper eigenvector x.
template <typename R>
struct Geo2 {
    R dl, cc, r, rinv, x0, x1;
};

template <typename R>
__device__ __forceinline__ void geo2(R dl, R cc, Geo2<R> &g)
{
    const R r2 = fma2(dl, dl, cc * cc);
    const R rinv = rsq(r2);
    const R r = r2 * rinv;
    const bool pos = dl >= R(0);
    g.dl = dl;
    g.cc = cc;
    g.r = r;
    g.rinv = rinv;
    g.x0 = pos ? fma2(r2, rinv, dl) : cc;   // r + dl
    g.x1 = pos ? cc : fma2(r2, rinv, -dl);  // r - dl
}

// normalised canonical upper eigenvector (c0, c1); the lower one is (-c1, c0)
template <typename R>
__device__ __forceinline__ void canon2(const Geo2<R> &g, R &c0, R &c1)
{
    const R n = rsq(fma2(g.x0, g.x0, g.x1 * g.x1));
    c0 = g.x0 * n;
    c1 = g.x1 * n;
}

// Mode classes of a linear model, fixed per kernel build.  With MT >= 0 the
// first MT modes only tune the gap (K_01 = 0) and the others only couple the
// two states (K_00 = K_11 = 0, so no bath force either); MT < 0 treats every
// mode as both.  Linear-vibronic models are commonly of this form (tuning
// modes of the totally symmetric irrep, coupling modes of the irrep of the
// coupling).  The terms a build leaves out are products with exact zeros,
// so it computes the same values as the general build (up to the sign of an
// exact zero).
template <int MT>
__device__ constexpr bool tunes(int j) { return MT < 0 || j < MT; }
template <int MT>
__device__ constexpr bool couples(int j) { return MT < 0 || j >= MT; }

template <int M, typename R, int MT>
__device__ __forceinline__ void coupling_coords(const N2Const<M, R> &C, const R (&q)[M], R &dl, R &cc)
{
    dl = C.dlt0;
    cc = C.c0;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        if (tunes<MT>(j))
            dl = fma2(C.dlt[j], q[j], dl);
        if (couples<MT>(j))
            cc = fma2(C.cpl[j], q[j], cc);
    }
}

// dt (dl_v, c_v) = (sum_j p_j vdl_j, sum_j p_j vcp_j) over the modes of each class
template <int M, typename R, int MT>
__device__ __forceinline__ void velocity_coords(const N2Const<M, R> &C, const R (&p)[M], R &dlv, R &cv)
{
    constexpr int jc = MT < 0 ? 0 : MT;  // first coupling mode
    dlv = R(0);
    cv = R(0);
    if constexpr (MT != 0) {
        dlv = p[0] * C.vdl[0];
#pragma unroll
        for (int j = 1; j < M; ++j)
            if (tunes<MT>(j))
                dlv = fma2(p[j], C.vdl[j], dlv);
    }
    if constexpr (jc < M) {
        cv = p[jc] * C.vcp[jc];
#pragma unroll
        for (int j = jc + 1; j < M; ++j)
            cv = fma2(p[j], C.vcp[j], cv);
    }
}

// c1 + x (c2 + x (c3 + x c4)): phi(x) = x times this for value coefficients,
// phi'(x) itself for slope coefficients
template <typename R>
__device__ __forceinline__ R horner4(const R *c, R x)
{
    return fma2(x, fma2(x, fma2(x, c[3], c[2]), c[1]), c[0]);
}

template <int M, typename R>
__device__ __forceinline__ void poly_coords(const N2Const<M, R> &C, const N2Poly<M, R> &Q, const R (&q)[M], R &dl,
                                            R &cc)
{
    dl = C.dlt0;
    cc = C.c0;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        dl = fma2(q[j], horner4<R>(Q.dv[j], q[j]), dl);
        cc = fma2(q[j], horner4<R>(Q.cv[j], q[j]), cc);
    }
}

// slopes of the dl, cc and Vbar polynomials of every mode at q
template <int M, typename R>
__device__ __forceinline__ void poly_slopes(const N2Poly<M, R> &Q, const R (&q)[M], R (&SD)[M], R (&SC)[M],
                                            R (&SB)[M])
{
#pragma unroll
    for (int j = 0; j < M; ++j) {
        SD[j] = horner4<R>(Q.ds[j], q[j]);
        SC[j] = horner4<R>(Q.cs[j], q[j]);
        SB[j] = horner4<R>(Q.bs[j], q[j]);
    }
}

// binary64 re-solve of a near-degenerate point for the binary32 path; the
// binary64 constants are read from device memory only when needed
template <int M>
__device__ __forceinline__ Geo2<float> resolve64(const double *__restrict__ c64, const float (&q)[M])
{
    double dl = c64[0], cc = c64[1];
#pragma unroll
    for (int j = 0; j < M; ++j) {
        dl = fma2(c64[2 + j], (double)q[j], dl);
        cc = fma2(c64[2 + M + j], (double)q[j], cc);
    }
    Geo2<double> d;
    geo2<double>(dl, cc, d);
    return Geo2<float>{(float)d.dl, (float)d.cc, (float)d.r, (float)d.rinv, (float)d.x0, (float)d.x1};
}

// the same for a model with higher powers: [dlt0, c0, dv[M][4], cv[M][4]]
template <int M>
__device__ __forceinline__ Geo2<float> resolve64_poly(const double *__restrict__ c64, const float (&q)[M])
{
    double dl = c64[0], cc = c64[1];
#pragma unroll
    for (int j = 0; j < M; ++j) {
        const double x = (double)q[j];
        dl = fma2(x, horner4<double>(c64 + 2 + 4 * j, x), dl);
        cc = fma2(x, horner4<double>(c64 + 2 + 4 * M + 4 * j, x), cc);
    }
    Geo2<double> d;
    geo2<double>(dl, cc, d);
    return Geo2<float>{(float)d.dl, (float)d.cc, (float)d.r, (float)d.rinv, (float)d.x0, (float)d.x1};
}

// Geometry at q.  binary32: a gap 2r below the model threshold is re-solved
// in binary64 (a rare, divergent branch); an exact degeneracy can only
// occur there, so it is checked there.  binary64: checked at every point.
// (r is compared with half the threshold: doubling is exact, so the
// decision is the one on 2r.)
template <int M, typename R, bool POLY, int MT = -1>
__device__ __forceinline__ void geo_at(const N2Const<M, R> &C, const N2Extra<M, R, POLY> &Q, const R (&q)[M],
                                       Geo2<R> &g, uint32_t &flag)
{
    R dl, cc;
    if constexpr (POLY)
        poly_coords<M, R>(C, Q, q, dl, cc);
    else
        coupling_coords<M, R, MT>(C, q, dl, cc);
    geo2<R>(dl, cc, g);
    if constexpr (sizeof(R) == 4) {
        if (!(g.r >= C.gap_half)) {
            if constexpr (POLY)
                g = resolve64_poly<M>(Q.c64, q);
            else
                g = resolve64<M>(C.c64, q);
            flag |= kFlagResolved;
            if (!(R(2) * g.r > R(0)))
                flag |= kFlagDegenerate;
        }
    } else {
        if (!(g.r > R(0x1p-1023)))  // 2r below the smallest normal double
            flag |= kFlagDegenerate;
    }
}

// One output bin of the workgroup's tile, reduced into dst (tile_values(2)
// doubles: [slot][stat] with slots 0..3 adiabatic (a*2+b) and 4..7 diabatic
// (i*2+j), stats Re, Im, Re^2, Im^2, then the excluded count).  The
// adiabatic terms sit in the walker's own slot only: the staging rows are
// cleared and that slot written under an exec mask.  Diabatic terms use
// U_ia U_jb = (a == b ? 1 : s0 s1) C_ia C_jb with the canonical frame C.
// Every thread of the workgroup calls it.
template <typename R>
__device__ __forceinline__ void bin_n2(BinLds &L, int &parity, bool live, int a, int b, double w, double phase,
                                       R c0, R c1, R sig, double *__restrict__ dst)
{
    double sn, cs;
    if constexpr (sizeof(R) == 4) {
        float s32, c32;
        sincos_phase32(phase, s32, c32);
        sn = (double)s32;
        cs = (double)c32;
    } else {
        sincos_phase(phase, sn, cs);
    }
    const bool ok = live && isfinite(w) && isfinite(phase);
    const double re = ok ? w * cs : 0.0;
    const double im = ok ? -w * sn : 0.0;
    const double re2 = re * re, im2 = im * im;
    BinReducer B(L, parity);
    const int s = a * 2 + b;
#pragma unroll
    for (int p = 0; p < 2; ++p) {  // adiabatic slots 2p and 2p + 1
        B.zero_row();
        if ((s >> 1) == p) {
            const int c = 4 * (s & 1);
            B.put(c + 0, re);
            B.put(c + 1, im);
            B.put(c + 2, re2);
            B.put(c + 3, im2);
        }
        B.pass();
    }
    // an excluded walker contributes exact zeros (its frame may be NaN)
    const double d0 = ok ? (double)c0 : 0.0, d1 = ok ? (double)c1 : 0.0;
    const double ua0 = a ? d0 : -d1;  // C_0a
    const double ua1 = a ? d1 : d0;   // C_1a
    const double ub0 = b ? d0 : -d1;  // C_0b
    const double ub1 = b ? d1 : d0;   // C_1b
    // the sign s0 s1 (off-diagonal elements) scales the weight: an exact
    // sign change, the same bits as scaling each product
    const bool flip = (a != b) && sig < R(0);
    const double res = flip ? -re : re, ims = flip ? -im : im;
    const double cf[4] = {ua0 * ub0, ua0 * ub1, ua1 * ub0, ua1 * ub1};
#pragma unroll
    for (int p = 0; p < 2; ++p) {  // diabatic cells 2p and 2p + 1
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const double r = res * cf[2 * p + h], m = ims * cf[2 * p + h];
            B.put(4 * h + 0, r);
            B.put(4 * h + 1, m);
            B.put(4 * h + 2, r * r);
            B.put(4 * h + 3, m * m);
        }
        B.pass();
    }
    B.count_excluded(live && !ok);
    B.flush(dst, 32, dst + 32);
}

// ---------------------------------------------------------------- sampling

template <int M, typename R, bool POLY>
__global__ __launch_bounds__(kBlock) void sample_n2_kernel(N2Const<M, double> C, N2Extra<M, double, POLY> Q,
                                                           SampleArgs S, EnsDev<R> E, double *__restrict__ partials,
                                                           int32_t n_out)
{
    __shared__ BinLds lds;
    int parity = 0;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool live = i < E.n_traj;
    const uint64_t gid = (uint64_t)(E.traj_offset + (live ? i : 0));
    const double two_pi = 6.283185307179586476925286766559;

    double q[M], p[M];
#pragma unroll
    for (int j = 0; j < M; ++j) {
        const U4 x = philox10(U4{(uint32_t)gid, (uint32_t)(gid >> 32), (uint32_t)j, 1u}, S.key0, S.key1);
        const double u1 = u52(x.x, x.y);
        const double u2 = u52(x.z, x.w);
        const double rr = sqrt(-2.0 * log(u1));
        double sn, cs;
        sincos_phase(two_pi * u2, sn, cs);
        q[j] = S.q0[j] + S.sq[j] * (rr * cs);
        p[j] = S.sp[j] * (rr * sn);
    }
    Geo2<double> g;
    uint32_t flag = 0;
    geo_at<M, double, POLY>(C, Q, q, g, flag);
    double c0, c1;
    canon2<double>(g, c0, c1);
    if (!(g.r > 0.0)) {  // exact degeneracy: any basis diagonalises V; take the identity
        c0 = 0.0;
        c1 = 1.0;
    }
    // column signs without a previous frame: U_kk > 0, else the first
    // nonzero entry of the column positive.  Column 0 = s0 (-c1, c0),
    // column 1 = s1 (c0, c1).
    const double l0 = (-c1 != 0.0) ? -c1 : c0;
    const double l1 = (c1 != 0.0) ? c1 : c0;
    const double s0 = l0 < 0.0 ? -1.0 : 1.0;
    const double s1 = l1 < 0.0 ? -1.0 : 1.0;
    const double u00 = -s0 * c1, u10 = s0 * c0, u01 = s1 * c0, u11 = s1 * c1;

    int a, b;
    double w;
    if (S.basis == QCL_INIT_ADIABATIC) {
        a = b = S.state;
        w = 1.0;
    } else {
        // diabatic |k><k| in the adiabatic basis: rho_ab = U_ka U_kb
        const int k = S.state;
        const double uk0 = k ? u10 : u00;  // U_k0
        const double uk1 = k ? u11 : u01;  // U_k1
        const double rs = fabs(uk0) + fabs(uk1);
        const double Z = rs * rs;
        const U4 x = philox10(U4{(uint32_t)gid, (uint32_t)(gid >> 32), 0u, 2u}, S.key0, S.key1);
        const double t = u52(x.x, x.y) * Z;
        const double w00 = fabs(uk0 * uk0), w01 = fabs(uk0 * uk1), w11 = fabs(uk1 * uk1);
        double Cm = w00;
        int pa = -1, pb = -1;
        if (t < Cm) { pa = 0; pb = 0; }
        Cm += w01;
        if (pa < 0 && t < Cm) { pa = 0; pb = 1; }
        Cm += w01;
        if (pa < 0 && t < Cm) { pa = 1; pb = 0; }
        Cm += w11;
        if (pa < 0 && t < Cm) { pa = 1; pb = 1; }
        if (pa < 0) {  // rounding: last element with nonzero weight
            if (w11 > 0.0) { pa = 1; pb = 1; }
            else if (w01 > 0.0) { pa = 1; pb = 0; }
            else { pa = 0; pb = 0; }
        }
        a = pa;
        b = pb;
        const double prod = (pa ? uk1 : uk0) * (pb ? uk1 : uk0);
        w = (prod > 0.0 ? 1.0 : -1.0) * Z;
    }

    bin_n2<double>(lds, parity, live, a, b, w, 0.0, c0, c1, s0 * s1,
                   partials + ((int64_t)blockIdx.x * n_out + 0) * tile_values(2));

    if (live) {
        const int64_t ld = E.ld;
#pragma unroll
        for (int j = 0; j < M; ++j) {
            E.q[j * ld + i] = (R)q[j];
            E.p[j * ld + i] = (R)p[j];
        }
        E.u[0 * ld + i] = (R)u00;
        E.u[1 * ld + i] = (R)u01;
        E.u[2 * ld + i] = (R)u10;
        E.u[3 * ld + i] = (R)u11;
        E.w[i] = w;
        E.phase[i] = 0.0;
        E.a[i] = (uint8_t)a;
        E.b[i] = (uint8_t)b;
        if (E.flags)
            E.flags[i] = flag;
    }
}

// ---------------------------------------------------------------- propagation

// One walker between steps, in registers.  G_j = dl dlt_j + cc cpl_j (or,
// with higher powers, dl phi^d'_j + cc phi^c'_j) is the element-independent
// part of the Hellmann-Feynman force at the current point, so that
// dE_{0,1}/dq_j = kbar_j -+ G_j/r; hr = (dt/4)/r and kx = s0 s1/(2 r^2) are
// kept with it for the two kicks and the next coupling.  The element (a, b)
// is held as the signs sa = 2a - 1, sb = 2b - 1 (a move negates one, and
// a + b - 1 and a - b are (sa + sb)/2 and (sa - sb)/2, the halves folded
// into hr and the phase factor exactly).
template <int M, typename R, bool POLY>
struct WalkerN2 {
    static constexpr int MP = POLY ? M : 1;
    R q[M], p[M];
    Geo2<R> g;
    R G[M];
    R SD[MP], SC[MP], SB[MP];  // polynomial slopes at the current point (POLY)
    R hr, kx, hsig, s1;
    double w, phase, r_old;
    float sa, sb;
    uint32_t flag;
};

// geometry, force terms and the per-point factors at the walker's q
template <int M, typename R, bool POLY, int MT>
__device__ __forceinline__ void point_n2(const N2Const<M, R> &C, const N2Extra<M, R, POLY> &Q, WalkerN2<M, R, POLY> &k)
{
    geo_at<M, R, POLY, MT>(C, Q, k.q, k.g, k.flag);
    if constexpr (POLY) {
        poly_slopes<M, R>(Q, k.q, k.SD, k.SC, k.SB);
#pragma unroll
        for (int j = 0; j < M; ++j)
            k.G[j] = fma2(k.g.dl, k.SD[j], k.g.cc * k.SC[j]);
    } else {
#pragma unroll
        for (int j = 0; j < M; ++j) {
            if constexpr (MT < 0)
                k.G[j] = fma2(k.g.dl, C.dlt[j], k.g.cc * C.cpl[j]);
            else if (tunes<MT>(j))
                k.G[j] = k.g.dl * C.dlt[j];
            else
                k.G[j] = k.g.cc * C.cpl[j];
        }
    }
    k.hr = C.hdt2 * k.g.rinv;
    k.kx = k.hsig * (k.g.rinv * k.g.rinv);
}

// p += (dt/2) * mean force of element (a,b), h = (a + b - 1) (dt/2)/r:
// (dt/2)(F_a + F_b)/2 = -hk q - hb - h G  (hb_j = (dt/2) phi^b'_j with
// higher powers; hb_j = 0 for coupling modes)
template <int M, typename R, bool POLY, int MT>
__device__ __forceinline__ void kick_n2(const N2Const<M, R> &C, WalkerN2<M, R, POLY> &k, R h)
{
#pragma unroll
    for (int j = 0; j < M; ++j) {
        R t;
        if constexpr (POLY)
            t = fma2(-C.hdt, k.SB[j], k.p[j]);
        else
            t = tunes<MT>(j) ? k.p[j] - C.hb[j] : k.p[j];
        k.p[j] = fma2(-h, k.G[j], fma2(-C.hk[j], k.q[j], t));
    }
}

// One step n -> n+1 of one walker; word is its Philox output for step n.
template <int M, typename R, int SCHEME, bool POLY, int MT>
__device__ __forceinline__ void step_n2(const N2Const<M, R> &C, const N2Extra<M, R, POLY> &Q, WalkerN2<M, R, POLY> &k,
                                        uint32_t word)
{
    R u;
    if constexpr (sizeof(R) == 4) u = u24f(word); else u = u24d(word);

    // 1. Monte Carlo move between elements at (q_n, p_n).
    // dt v.d_01 = s0 s1 (dl c_v - cc dl_v) / (2 r^2); the two candidates
    // (1-a, b) and (a, 1-b) carry f0 = +-x, f1 = +-x.
    R dlv, cv;
    if constexpr (POLY) {
        const R v0 = k.p[0] * C.dtm[0];
        dlv = v0 * k.SD[0];
        cv = v0 * k.SC[0];
#pragma unroll
        for (int j = 1; j < M; ++j) {
            const R vj = k.p[j] * C.dtm[j];
            dlv = fma2(vj, k.SD[j], dlv);
            cv = fma2(vj, k.SC[j], cv);
        }
    } else {
        velocity_coords<M, R, MT>(C, k.p, dlv, cv);
    }
    R xs;  // dl c_v - cc dl_v
    if constexpr (!POLY && MT == 0)
        xs = k.g.dl * cv;  // no tuning mode: dl_v = 0
    else if constexpr (!POLY && MT == M)
        xs = -(k.g.cc * dlv);  // no coupling mode: c_v = 0
    else
        xs = fma2(k.g.dl, cv, -(k.g.cc * dlv));
    const R x = xs * k.kx;
    const R ax = __builtin_fabs(x);
    const R S = ax + ax;
    int pick;  // -1 stay, 0 -> (1-a, b), 1 -> (a, 1-b)
    R mul;     // weight factor (normalized rule) or divisor (linear rule, staying)
    if (SCHEME == QCL_TRANS_LINEAR && S < R(1)) {
        pick = (u < ax) ? 0 : ((u < S) ? 1 : -1);
        mul = R(1) - S;
    } else {
        if (SCHEME == QCL_TRANS_LINEAR)
            k.flag |= kFlagFallback;
        const R one_s = R(1) + S;
        const R t = u * one_s;
        const bool stay = t < R(1), first = t < R(1) + ax;
        pick = stay ? -1 : (first ? 0 : 1);
        mul = one_s;
    }
    // sign of the chosen candidate's factor: f0 = (a ? -x : x), f1 = (b ? -x : x)
    const float sc = (pick == 0) ? k.sa : k.sb;
    const bool fpos = (x > R(0)) != (sc > 0.0f);
    if (SCHEME == QCL_TRANS_LINEAR && S < R(1)) {
        if (pick < 0) k.w = k.w / (double)mul;
        else k.w = fpos ? k.w : -k.w;
    } else {
        // the factor's sign goes into the multiplier: w (-m) = -(w m) exactly
        k.w = k.w * (double)((pick < 0 || fpos) ? mul : -mul);
    }
    k.sa = (pick == 0) ? -k.sa : k.sa;
    k.sb = (pick == 1) ? -k.sb : k.sb;

    // 2. velocity Verlet on the mean force of the current element:
    // (a + b - 1) (dt/2)/r = (sa + sb) hr
    const R lam2 = R(k.sa + k.sb);
    const R xo0 = k.g.x0, xo1 = k.g.x1;
    kick_n2<M, R, POLY, MT>(C, k, lam2 * k.hr);
#pragma unroll
    for (int j = 0; j < M; ++j)
        k.q[j] = fma2(C.dtm[j], k.p[j], k.q[j]);
    point_n2<M, R, POLY, MT>(C, Q, k);
    k.s1 = (fma2(xo0, k.g.x0, xo1 * k.g.x1) < R(0)) ? -k.s1 : k.s1;  // frame continuity
    kick_n2<M, R, POLY, MT>(C, k, lam2 * k.hr);

    // 3. phase: trapezoid of w_ab = (E_a - E_b)/hbar = 2 (a - b) r / hbar,
    // (a - b) dt/hbar = (sa - sb) dt/(2 hbar)
    const double r_new = (double)k.g.r;
    k.phase = fma2((double)(k.sa - k.sb), C.dt_hbar2 * (k.r_old + r_new), k.phase);
    k.r_old = r_new;
}

// All steps of one tile of kBlock walkers (the whole workgroup calls it).
// The steps run four at a time, aligned to the Philox blocks (one block of
// four words per four steps), so that each copy of the step reads its word
// directly; steps before the first aligned step and after the last whole
// block run one at a time with the word selected at run time.  Every copy
// performs the same operations (no contraction), so the bits do not depend
// on the copy.  Bins fall between stretches.
template <int M, typename R, int SCHEME, bool POLY, int MT>
__device__ __forceinline__ void propagate_n2_tile(const N2Const<M, R> &C_in, const N2Extra<M, R, POLY> &Q,
                                                  const PropArgs &P, const EnsDev<R> &E,
                                                  double *__restrict__ partials, int64_t tile, BinLds &lds,
                                                  int &parity)
{
    // dlt0 and c0 start the two coupling coordinates at every point; held in
    // vector registers (the empty asm pins them there), the first fused
    // multiply-add of each needs no copy of a second scalar operand
    N2Const<M, R> C = C_in;
    asm volatile("" : "+v"(C.dlt0), "+v"(C.c0));
    const int64_t i = tile * kBlock + threadIdx.x;
    const bool live = i < E.n_traj;
    const int64_t li = live ? i : E.n_traj - 1;  // idle lanes shadow a valid walker
    const int64_t ld = E.ld;
    const uint64_t gid = (uint64_t)(E.traj_offset + li);
    const uint32_t g_lo = (uint32_t)gid, g_hi = (uint32_t)(gid >> 32);

    WalkerN2<M, R, POLY> k;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        k.q[j] = E.q[j * ld + li];
        k.p[j] = E.p[j * ld + li];
    }
    const R p00 = E.u[0 * ld + li], p01 = E.u[1 * ld + li], p10 = E.u[2 * ld + li], p11 = E.u[3 * ld + li];
    k.w = E.w[li];
    k.phase = E.phase[li];
    k.sa = E.a[li] ? 1.0f : -1.0f;
    k.sb = E.b[li] ? 1.0f : -1.0f;
    k.flag = 0;
    k.hsig = R(0.5);
    point_n2<M, R, POLY, MT>(C, Q, k);
    // column signs of the stored frame relative to the canonical one; the
    // product s0 s1 is invariant along the walker, s1 is tracked
    const R s0_in = fma2(p00, -k.g.x1, p10 * k.g.x0) < R(0) ? R(-1) : R(1);
    k.s1 = fma2(p01, k.g.x0, p11 * k.g.x1) < R(0) ? R(-1) : R(1);
    const R sig = s0_in * k.s1;
    k.hsig = R(0.5) * sig;
    k.kx = k.hsig * (k.g.rinv * k.g.rinv);
    k.r_old = (double)k.g.r;

    int64_t step = P.step0;
    const int64_t end = P.step0 + P.n_steps;
    int64_t obin = step / P.cadence + 1;  // next bin and its global step
    int64_t next_bin = obin * P.cadence;
    U4 rnd{0, 0, 0, 0};
    if (step & 3)
        rnd = philox10(U4{g_lo, g_hi, (uint32_t)(step >> 2), 0u}, P.key0, P.key1);
    while (step < end) {
        const int64_t stop = next_bin < end ? next_bin : end;
        int n = (int)(stop - step);
        for (; n > 0 && (step & 3); --n, ++step)
            step_n2<M, R, SCHEME, POLY, MT>(C, Q, k, pick_word(rnd, (uint32_t)(step & 3)));
        for (; n >= 4; n -= 4, step += 4) {
            rnd = philox10(U4{g_lo, g_hi, (uint32_t)(step >> 2), 0u}, P.key0, P.key1);
            step_n2<M, R, SCHEME, POLY, MT>(C, Q, k, rnd.x);
            step_n2<M, R, SCHEME, POLY, MT>(C, Q, k, rnd.y);
            step_n2<M, R, SCHEME, POLY, MT>(C, Q, k, rnd.z);
            step_n2<M, R, SCHEME, POLY, MT>(C, Q, k, rnd.w);
        }
        for (; n > 0; --n, ++step) {
            if ((step & 3) == 0)
                rnd = philox10(U4{g_lo, g_hi, (uint32_t)(step >> 2), 0u}, P.key0, P.key1);
            step_n2<M, R, SCHEME, POLY, MT>(C, Q, k, pick_word(rnd, (uint32_t)(step & 3)));
        }
        // 4. output bin at global step next_bin
        if (step == next_bin) {
            if (obin < P.n_out) {
                R c0, c1;
                canon2<R>(k.g, c0, c1);
                bin_n2<R>(lds, parity, live, k.sa > 0.0f, k.sb > 0.0f, k.w, k.phase, c0, c1, sig,
                          partials + (tile * P.n_out + obin) * tile_values(2));
            }
            ++obin;
            next_bin += P.cadence;
        }
    }
    if (!(isfinite(k.w) && isfinite(k.phase)))
        k.flag |= kFlagNonfinite;

    if (live) {
        R c0, c1;
        canon2<R>(k.g, c0, c1);
        const R s0 = sig * k.s1;
#pragma unroll
        for (int j = 0; j < M; ++j) {
            E.q[j * ld + i] = k.q[j];
            E.p[j * ld + i] = k.p[j];
        }
        E.u[0 * ld + i] = -s0 * c1;
        E.u[1 * ld + i] = k.s1 * c0;
        E.u[2 * ld + i] = s0 * c0;
        E.u[3 * ld + i] = k.s1 * c1;
        E.w[i] = k.w;
        E.phase[i] = k.phase;
        E.a[i] = k.sa > 0.0f ? 1 : 0;
        E.b[i] = k.sb > 0.0f ? 1 : 0;
        if (E.flags)
            E.flags[i] |= k.flag;
    }
}

// Resident workgroups per CU the propagation kernels are built for: five
// for the binary32 linear models up to 4 modes (the step loop and the bins
// fit 96 registers, five waves per SIMD), four for the models with higher
// powers up to 3 modes and, in binary32, 4 modes (128 registers), no
// constraint otherwise.
template <int M, typename R, bool POLY>
constexpr int kN2Occupancy = (sizeof(R) == 4 && !POLY && M <= 4)            ? 5
                             : (POLY && (M <= 3 || (sizeof(R) == 4 && M <= 4))) ? 4
                                                                                 : 1;

template <int M, typename R, int SCHEME, bool POLY, int MT = -1>
__global__ __launch_bounds__(kBlock, (kN2Occupancy<M, R, POLY>)) void propagate_n2_kernel(N2Const<M, R> C, N2Extra<M, R, POLY> Q, PropArgs P,
                                                              EnsDev<R> E, double *__restrict__ partials)
{
    __shared__ BinLds lds;
    int parity = 0;
    propagate_n2_tile<M, R, SCHEME, POLY, MT>(C, Q, P, E, partials, (int64_t)blockIdx.x, lds, parity);
}

// Persistent launch over (instance, tile) work items of many two-state
// instances of one kernel class; items are taken from an atomic counter
// (descriptors are sorted by decreasing work per tile).
template <int M, typename R, int SCHEME, bool POLY>
__global__ __launch_bounds__(kBlock, (kN2Occupancy<M, R, POLY>)) void batch_n2_kernel(const BatchItemN2<M, R, POLY> *__restrict__ items,
                                                          int32_t n_items, int64_t total_tiles,
                                                          unsigned long long *counter)
{
    __shared__ BinLds lds;
    __shared__ long long item_sh;
    int parity = 0;
    for (;;) {
        if (threadIdx.x == 0)
            item_sh = (long long)atomicAdd(counter, 1ull);
        __syncthreads();
        // wave-uniform by construction; readfirstlane lets the descriptor
        // loads below go through the scalar unit
        const long long raw = item_sh;
        const long long item = (long long)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(raw >> 32)) << 32) |
                                           (uint32_t)__builtin_amdgcn_readfirstlane((int)raw));
        __syncthreads();
        if (item >= total_tiles)
            break;
        int lo = 0, hi = n_items - 1;  // last descriptor with tile_begin <= item
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (items[mid].tile_begin <= item) lo = mid; else hi = mid - 1;
        }
        const BatchItemN2<M, R, POLY> &it = items[lo];
        propagate_n2_tile<M, R, SCHEME, POLY, -1>(it.C, it.Q, it.P, it.E, it.partials, item - it.tile_begin, lds,
                                                  parity);
        __syncthreads();
    }
}

template <int M, typename R>
N2Const<M, R> make_const(const qcl_model_s &m, double dt)
{
    N2Const<M, R> C{};
    const double hdt = 0.5 * dt;
    for (int j = 0; j < M; ++j) {
        const bool real = j < m.m;  // padded modes are inert
        C.dlt[j] = (R)(real ? m.dlt[j] : 0.0);
        C.cpl[j] = (R)(real ? m.cpl[j] : 0.0);
        C.vdl[j] = (R)(real ? dt * m.minv[j] * m.dlt[j] : 0.0);
        C.vcp[j] = (R)(real ? dt * m.minv[j] * m.cpl[j] : 0.0);
        C.hk[j] = (R)(real ? hdt * m.kq[j] : 0.0);
        C.hb[j] = (R)(real ? hdt * m.kbar[j] : 0.0);
        C.dtm[j] = (R)(real ? dt * m.minv[j] : 0.0);
    }
    C.dlt0 = (R)m.dlt0;
    C.c0 = (R)m.c0;
    C.hdt = (R)hdt;
    C.hdt2 = (R)(0.5 * hdt);
    C.gap_half = (R)(0.5 * (1e-4 * m.energy_scale));
    C.dt_hbar = dt / m.hbar;
    C.dt_hbar2 = 0.5 * C.dt_hbar;
    C.c64 = m.d_model + m.c64_offset;
    return C;
}

template <int M, typename R>
N2Poly<M, R> make_poly(const qcl_model_s &m)
{
    N2Poly<M, R> Q{};
    for (int j = 0; j < M && j < m.m; ++j)  // padded modes: zero coefficients
        for (int k = 0; k < 4; ++k) {
            const double *row = &m.n2poly[(size_t)j * 20];
            Q.dv[j][k] = (R)row[0 + k];
            Q.ds[j][k] = (R)row[4 + k];
            Q.cv[j][k] = (R)row[8 + k];
            Q.cs[j][k] = (R)row[12 + k];
            Q.bs[j][k] = (R)row[16 + k];
        }
    Q.c64 = m.d_model + m.n2poly64_offset;
    return Q;
}

template <typename R>
EnsDev<R> ens_dev(const qcl_ensemble &e)
{
    return EnsDev<R>{(R *)e.q, (R *)e.p, (R *)e.u, e.w, e.phase, e.a, e.b, e.flags, e.ld, e.n_traj, e.traj_offset};
}

template <int M>
hipError_t sample_m(const qcl_model_s &m, const SampleArgs &sa, const qcl_ensemble &ens, double *partials,
                    int32_t n_out, hipStream_t s)
{
    const dim3 grid((unsigned)n_tiles(ens.n_traj)), block(kBlock);
    const N2Const<M, double> C = make_const<M, double>(m, 1.0);
    if (m.degree > 1) {
        const N2Poly<M, double> Q = make_poly<M, double>(m);
        if (ens.prec == QCL_FP64)
            hipLaunchKernelGGL((sample_n2_kernel<M, double, true>), grid, block, 0, s, C, Q, sa, ens_dev<double>(ens),
                               partials, n_out);
        else
            hipLaunchKernelGGL((sample_n2_kernel<M, float, true>), grid, block, 0, s, C, Q, sa, ens_dev<float>(ens),
                               partials, n_out);
    } else {
        if (ens.prec == QCL_FP64)
            hipLaunchKernelGGL((sample_n2_kernel<M, double, false>), grid, block, 0, s, C, N2Linear{}, sa,
                               ens_dev<double>(ens), partials, n_out);
        else
            hipLaunchKernelGGL((sample_n2_kernel<M, float, false>), grid, block, 0, s, C, N2Linear{}, sa,
                               ens_dev<float>(ens), partials, n_out);
    }
    return hipGetLastError();
}

// Mode-class builds exist for linear models with up to this many modes and
// the normalized transition rule; other models take the general build.
constexpr int kSplitMaxModes = 4;

// The mode classes of a linear two-state model: the smallest MT such that
// the modes before it have K_01 = 0 and the others K_00 = K_11 = 0, or -1
// when the modes are not ordered that way.
int mode_split(const qcl_model_s &m)
{
    for (int mt = 0; mt <= m.m; ++mt) {
        bool ok = true;
        for (int j = 0; j < m.m && ok; ++j)
            ok = j < mt ? m.cpl[j] == 0.0 : (m.dlt[j] == 0.0 && m.kbar[j] == 0.0);
        if (ok)
            return mt;
    }
    return -1;
}

template <int M, typename R, int MT>
void launch_split(int mt, dim3 grid, const N2Const<M, R> &C, const PropArgs &P, const EnsDev<R> &E, double *partials,
                  hipStream_t s)
{
    if constexpr (MT <= M) {
        if (mt == MT) {
            hipLaunchKernelGGL((propagate_n2_kernel<M, R, QCL_TRANS_NORMALIZED, false, MT>), grid, dim3(kBlock), 0, s,
                               C, N2Linear{}, P, E, partials);
            return;
        }
        launch_split<M, R, MT + 1>(mt, grid, C, P, E, partials, s);
    }
}

template <int M, typename R>
void propagate_mr(const qcl_model_s &m, const qcl_ensemble &ens, const qcl_prop_desc &pd, double *partials,
                  hipStream_t s)
{
    const dim3 grid((unsigned)n_tiles(ens.n_traj)), block(kBlock);
    const PropArgs P{ens.step, pd.n_steps, pd.cadence, pd.n_out, pd.scheme, (uint32_t)pd.seed,
                     (uint32_t)(pd.seed >> 32)};
    const N2Const<M, R> C = make_const<M, R>(m, pd.dt);
    if constexpr (M <= kSplitMaxModes) {
        const int mt = m.degree > 1 || pd.scheme == QCL_TRANS_LINEAR ? -1 : mode_split(m);
        if (mt >= 0) {
            launch_split<M, R, 0>(mt, grid, C, P, ens_dev<R>(ens), partials, s);
            return;
        }
    }
    if (m.degree > 1) {
        const N2Poly<M, R> Q = make_poly<M, R>(m);
        if (pd.scheme == QCL_TRANS_LINEAR)
            hipLaunchKernelGGL((propagate_n2_kernel<M, R, QCL_TRANS_LINEAR, true>), grid, block, 0, s, C, Q, P,
                               ens_dev<R>(ens), partials);
        else
            hipLaunchKernelGGL((propagate_n2_kernel<M, R, QCL_TRANS_NORMALIZED, true>), grid, block, 0, s, C, Q, P,
                               ens_dev<R>(ens), partials);
        return;
    }
    if (pd.scheme == QCL_TRANS_LINEAR)
        hipLaunchKernelGGL((propagate_n2_kernel<M, R, QCL_TRANS_LINEAR, false>), grid, block, 0, s, C, N2Linear{}, P,
                           ens_dev<R>(ens), partials);
    else
        hipLaunchKernelGGL((propagate_n2_kernel<M, R, QCL_TRANS_NORMALIZED, false>), grid, block, 0, s, C,
                           N2Linear{}, P, ens_dev<R>(ens), partials);
}

template <int M>
hipError_t propagate_m(const qcl_model_s &m, const qcl_ensemble &ens, const qcl_prop_desc &pd, double *partials,
                       hipStream_t s)
{
    if (ens.prec == QCL_FP64)
        propagate_mr<M, double>(m, ens, pd, partials, s);
    else
        propagate_mr<M, float>(m, ens, pd, partials, s);
    return hipGetLastError();
}

template <int M, typename R, bool POLY>
size_t item_n2(const qcl_model_s &m, const qcl_ensemble &ens, const qcl_prop_desc &pd, double *partials,
               int64_t tile_begin, void *out)
{
    if (out) {
        BatchItemN2<M, R, POLY> it{};
        it.C = make_const<M, R>(m, pd.dt);
        if constexpr (POLY)
            it.Q = make_poly<M, R>(m);
        it.P = PropArgs{ens.step, pd.n_steps, pd.cadence, pd.n_out, pd.scheme, (uint32_t)pd.seed,
                        (uint32_t)(pd.seed >> 32), m.m};
        it.E = ens_dev<R>(ens);
        it.partials = partials;
        it.tile_begin = tile_begin;
        std::memcpy(out, &it, sizeof(it));
    }
    return sizeof(BatchItemN2<M, R, POLY>);
}

template <int M, typename R, bool POLY>
hipError_t batch_m_r(int scheme, int wpc, const void *items, int32_t n_items, int64_t total_tiles,
                     unsigned long long *counter, hipStream_t s)
{
    int cus = 0, per_cu = 0, dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const void *fn = scheme == QCL_TRANS_LINEAR ? (const void *)batch_n2_kernel<M, R, QCL_TRANS_LINEAR, POLY>
                                                : (const void *)batch_n2_kernel<M, R, QCL_TRANS_NORMALIZED, POLY>;
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBlock, 0);
    const int64_t grid = persistent_grid(total_tiles, cus, per_cu, wpc);
    const BatchItemN2<M, R, POLY> *it = (const BatchItemN2<M, R, POLY> *)items;
    if (scheme == QCL_TRANS_LINEAR)
        hipLaunchKernelGGL((batch_n2_kernel<M, R, QCL_TRANS_LINEAR, POLY>), dim3((unsigned)grid), dim3(kBlock), 0, s,
                           it, n_items, total_tiles, counter);
    else
        hipLaunchKernelGGL((batch_n2_kernel<M, R, QCL_TRANS_NORMALIZED, POLY>), dim3((unsigned)grid), dim3(kBlock), 0,
                           s, it, n_items, total_tiles, counter);
    return hipGetLastError();
}

template <int M>
size_t item_m(const qcl_model_s &m, const qcl_ensemble &ens, const qcl_prop_desc &pd, double *partials,
              int64_t tile_begin, void *out)
{
    if (m.degree > 1)
        return ens.prec == QCL_FP64 ? item_n2<M, double, true>(m, ens, pd, partials, tile_begin, out)
                                    : item_n2<M, float, true>(m, ens, pd, partials, tile_begin, out);
    return ens.prec == QCL_FP64 ? item_n2<M, double, false>(m, ens, pd, partials, tile_begin, out)
                                : item_n2<M, float, false>(m, ens, pd, partials, tile_begin, out);
}

template <int M>
hipError_t batch_m(bool poly, int prec, int scheme, int wpc, const void *items, int32_t n_items, int64_t total_tiles,
                   unsigned long long *counter, hipStream_t s)
{
    if (poly)
        return prec == QCL_FP64 ? batch_m_r<M, double, true>(scheme, wpc, items, n_items, total_tiles, counter, s)
                                : batch_m_r<M, float, true>(scheme, wpc, items, n_items, total_tiles, counter, s);
    return prec == QCL_FP64 ? batch_m_r<M, double, false>(scheme, wpc, items, n_items, total_tiles, counter, s)
                            : batch_m_r<M, float, false>(scheme, wpc, items, n_items, total_tiles, counter, s);
}

}  // namespace

size_t batch_item_n2(const qcl_model_s &m, const qcl_ensemble &ens, const qcl_prop_desc &pd, double *partials,
                     int64_t tile_begin, void *out)
{
    switch (m.m) {
    case 1: return item_m<1>(m, ens, pd, partials, tile_begin, out);
    case 2: return item_m<2>(m, ens, pd, partials, tile_begin, out);
    case 3: return item_m<3>(m, ens, pd, partials, tile_begin, out);
    case 4: return item_m<4>(m, ens, pd, partials, tile_begin, out);
    case 5: return item_m<5>(m, ens, pd, partials, tile_begin, out);
    case 6: return item_m<6>(m, ens, pd, partials, tile_begin, out);
    case 7: return item_m<7>(m, ens, pd, partials, tile_begin, out);
    case 8: return item_m<8>(m, ens, pd, partials, tile_begin, out);
    default: return 0;
    }
}

hipError_t launch_batch_n2(int modes, bool poly, int prec, int scheme, int wpc, const void *items, int32_t n_items,
                           int64_t total_tiles, unsigned long long *counter, hipStream_t s)
{
    switch (modes) {
    case 1: return batch_m<1>(poly, prec, scheme, wpc, items, n_items, total_tiles, counter, s);
    case 2: return batch_m<2>(poly, prec, scheme, wpc, items, n_items, total_tiles, counter, s);
    case 3: return batch_m<3>(poly, prec, scheme, wpc, items, n_items, total_tiles, counter, s);
    case 4: return batch_m<4>(poly, prec, scheme, wpc, items, n_items, total_tiles, counter, s);
    case 5: return batch_m<5>(poly, prec, scheme, wpc, items, n_items, total_tiles, counter, s);
    case 6: return batch_m<6>(poly, prec, scheme, wpc, items, n_items, total_tiles, counter, s);
    case 7: return batch_m<7>(poly, prec, scheme, wpc, items, n_items, total_tiles, counter, s);
    case 8: return batch_m<8>(poly, prec, scheme, wpc, items, n_items, total_tiles, counter, s);
    default: return hipErrorNotSupported;
    }
}

hipError_t launch_sample_n2(const qcl_model_s &m, const SampleArgs &sa, const qcl_ensemble &ens, double *partials,
                            int32_t n_out, hipStream_t s)
{
    switch (m.m) {
    case 1: return sample_m<1>(m, sa, ens, partials, n_out, s);
    case 2: return sample_m<2>(m, sa, ens, partials, n_out, s);
    case 3: return sample_m<3>(m, sa, ens, partials, n_out, s);
    case 4: return sample_m<4>(m, sa, ens, partials, n_out, s);
    case 5: return sample_m<5>(m, sa, ens, partials, n_out, s);
    case 6: return sample_m<6>(m, sa, ens, partials, n_out, s);
    case 7: return sample_m<7>(m, sa, ens, partials, n_out, s);
    case 8: return sample_m<8>(m, sa, ens, partials, n_out, s);
    default: return hipErrorNotSupported;
    }
}

hipError_t launch_propagate_n2(const qcl_model_s &m, const qcl_ensemble &ens, const qcl_prop_desc &pd,
                               double *partials, hipStream_t s)
{
    switch (m.m) {
    case 1: return propagate_m<1>(m, ens, pd, partials, s);
    case 2: return propagate_m<2>(m, ens, pd, partials, s);
    case 3: return propagate_m<3>(m, ens, pd, partials, s);
    case 4: return propagate_m<4>(m, ens, pd, partials, s);
    case 5: return propagate_m<5>(m, ens, pd, partials, s);
    case 6: return propagate_m<6>(m, ens, pd, partials, s);
    case 7: return propagate_m<7>(m, ens, pd, partials, s);
    case 8: return propagate_m<8>(m, ens, pd, partials, s);
    default: return hipErrorNotSupported;
    }
}

}  // namespace qcl
