// Per-walker N-state frame arithmetic on gfx950, shared by the general
// kernels (N = 2..8, model tables in device memory) and by the kernels
// compiled at run time for models with a supplied potential: the symmetric
// eigen-solve of the diabatic matrix by cyclic Jacobi rotations warm-started
// from the previous frame (Golub & Van Loan, Sec. 8.5), ordering and sign
// continuity of the eigenvectors, Rayleigh energies, register-resident
// selection by a runtime index, and one output bin of a walker tile.
#pragma once

#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>

#include <cstdint>
#endif

#include "block_reduce.hpp"
#include "phase_math.hpp"
#include "philox.hpp"
#include "qcl_device.hpp"

namespace qcl {

template <int N>
constexpr int kTri = N * (N + 1) / 2;

template <int N>
__host__ __device__ constexpr int tri_index(int k, int l)
{
    return k * N - k * (k - 1) / 2 + (l - k);  // k <= l, row-major upper triangle
}

template <int N>
__host__ __device__ constexpr int sym_index(int k, int l)
{
    return k <= l ? tri_index<N>(k, l) : tri_index<N>(l, k);
}

// a table of model constants seen through the constant address space
template <typename R>
using ctab_t = const __attribute__((address_space(4))) R *;

// The table at p (a wave-uniform address) as an opaque scalar value:
// loads through the result are scalar loads that the compiler can neither
// hoist above this point nor merge with loads through another call's
// result.  The address is moved to scalar registers first, since a value
// that is uniform but was loaded by the vector unit (a batch descriptor
// field) may sit in vector registers.
template <typename R>
__device__ __forceinline__ ctab_t<R> ctab(const R *p)
{
    const uint64_t v = (uint64_t)p;
    uint64_t u = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32)) << 32) |
                 (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    asm volatile("" : "+s"(u));
    return (ctab_t<R>)u;
}

__device__ __forceinline__ float fma_g(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_g(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float abs_g(float x) { return __builtin_fabsf(x); }
__device__ __forceinline__ double abs_g(double x) { return __builtin_fabs(x); }
__device__ __forceinline__ float sqrt_g(float x) { return __builtin_sqrtf(x); }
__device__ __forceinline__ double sqrt_g(double x) { return __builtin_sqrt(x); }
// reciprocal: hardware estimate, refined twice by Newton steps in binary64
__device__ __forceinline__ float rcp_g(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_g(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma_g(r, fma_g(-x, r, 1.0), r);
    return fma_g(r, fma_g(-x, r, 1.0), r);
}
// 1/sqrt: hardware estimate; in binary64 refined by two Newton steps
// r <- r (3/2 - x r^2 / 2)
__device__ __forceinline__ float rsq_g(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsq_g(double x)
{
    double r = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    r = r * fma_g(-h * r, r, 1.5);
    return r * fma_g(-h * r, r, 1.5);
}
// sqrt of an argument >= 1 (no denormal or zero cases): x / sqrt(x), a
// couple of instructions instead of the correctly rounded expansion
template <typename R>
__device__ __forceinline__ R sqrt_ge1(R x) { return x * rsq_g(x); }
__device__ __forceinline__ float div_g(float a, float b) { return a * rcp_g(b); }
__device__ __forceinline__ double div_g(double a, double b) { return a * rcp_g(b); }

template <int N, typename R>
struct Frame {
    R U[N][N];  // U[i][k]: component i of eigenvector k
    R E[N];     // ascending energies
};

// E_k = u_k^T V u_k
template <int N, typename R>
__device__ __forceinline__ void rayleigh(const R (&V)[kTri<N>], const R (&U)[N][N], R (&E)[N])
{
#pragma unroll
    for (int k = 0; k < N; ++k) {
        R d = R(0), o = R(0);
#pragma unroll
        for (int i = 0; i < N; ++i) {
            d = fma_g(V[tri_index<N>(i, i)], U[i][k] * U[i][k], d);
#pragma unroll
            for (int l = i + 1; l < N; ++l)
                o = fma_g(V[tri_index<N>(i, l)], U[i][k] * U[l][k], o);
        }
        E[k] = fma_g(R(2), o, d);
    }
}

// A = U^T V U (upper triangle), one column of V U at a time
template <int N, typename R>
__device__ __forceinline__ void congruence(const R (&V)[kTri<N>], const R (&U)[N][N], R (&A)[kTri<N>])
{
#pragma unroll
    for (int l = 0; l < N; ++l) {
        R w[N];  // column l of V U
#pragma unroll
        for (int i = 0; i < N; ++i) {
            R s = R(0);
#pragma unroll
            for (int r = 0; r < N; ++r)
                s = fma_g(V[sym_index<N>(i, r)], U[r][l], s);
            w[i] = s;
        }
#pragma unroll
        for (int k = 0; k <= l; ++k) {
            R s = R(0);
#pragma unroll
            for (int i = 0; i < N; ++i)
                s = fma_g(U[i][k], w[i], s);
            A[tri_index<N>(k, l)] = s;
        }
    }
}

// cyclic Jacobi on the symmetric triangle A, rotations accumulated into U
// (A <- J^T A J, U <- U J with J_pp = J_qq = c, J_pq = s = -J_qp).  A pair
// is rotated while |A_pq| exceeds thr; otherwise its rotation is the
// identity (t = 0, c = 1, s = 0 leave every finite entry's value unchanged),
// so the sweeps run without per-pair branches and stop when no pair of any
// lane of the wavefront exceeds thr.  A lane's result depends on its own
// matrix only: further sweeps on a converged lane are identities.
// Returns the sum of |t| = |tan(angle)| over the lane's rotations.
template <int N, typename R>
__device__ __forceinline__ R jacobi(R (&A)[kTri<N>], R (&U)[N][N], R eps, int max_sweeps)
{
    R f2 = R(0);
#pragma unroll
    for (int k = 0; k < N; ++k)
#pragma unroll
        for (int l = k; l < N; ++l)
            f2 = fma_g((k == l ? R(1) : R(2)) * A[tri_index<N>(k, l)], A[tri_index<N>(k, l)], f2);
    const R thr = eps * sqrt_g(f2);
    R turned = R(0);
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        bool need = false;
#pragma unroll
        for (int p = 0; p < N - 1; ++p)
#pragma unroll
            for (int q = p + 1; q < N; ++q)
                need |= abs_g(A[tri_index<N>(p, q)]) > thr;
        if (!__any(need))
            break;
#pragma unroll
        for (int p = 0; p < N - 1; ++p) {
#pragma unroll
            for (int q = p + 1; q < N; ++q) {
                const R apq = A[tri_index<N>(p, q)];
                const bool rot = abs_g(apq) > thr;
                const R app = A[tri_index<N>(p, p)], aqq = A[tri_index<N>(q, q)];
                const R theta = (aqq - app) * rcp_g(R(2) * (rot ? apq : R(1)));
                R t = rcp_g(abs_g(theta) + sqrt_ge1<R>(fma_g(theta, theta, R(1))));
                t = theta < R(0) ? -t : t;
                t = rot ? t : R(0);
                turned += abs_g(t);
                const R c = rsq_g(fma_g(t, t, R(1)));
                const R s = t * c;
                const R h = t * apq;
                A[tri_index<N>(p, p)] = app - h;
                A[tri_index<N>(q, q)] = aqq + h;
                A[tri_index<N>(p, q)] = rot ? R(0) : apq;
#pragma unroll
                for (int r = 0; r < N; ++r) {
                    if (r == p || r == q)
                        continue;
                    const R arp = A[sym_index<N>(r, p)], arq = A[sym_index<N>(r, q)];
                    A[sym_index<N>(r, p)] = fma_g(c, arp, -s * arq);
                    A[sym_index<N>(r, q)] = fma_g(s, arp, c * arq);
                }
#pragma unroll
                for (int r = 0; r < N; ++r) {
                    const R urp = U[r][p], urq = U[r][q];
                    U[r][p] = fma_g(c, urp, -s * urq);
                    U[r][q] = fma_g(s, urp, c * urq);
                }
            }
        }
    }
    return turned;
}

template <int N, typename R>
__device__ __forceinline__ void cswap(Frame<N, R> &f, int i, int j)
{
    const bool sw = f.E[j] < f.E[i];
    const R ei = f.E[i], ej = f.E[j];
    f.E[i] = sw ? ej : ei;
    f.E[j] = sw ? ei : ej;
#pragma unroll
    for (int r = 0; r < N; ++r) {
        const R ui = f.U[r][i], uj = f.U[r][j];
        f.U[r][i] = sw ? uj : ui;
        f.U[r][j] = sw ? ui : uj;
    }
}

// ascending order (sorting networks for N <= 4; odd-even transposition,
// N rounds of compare-exchanges of neighbours, above)
template <int N, typename R>
__device__ __forceinline__ void sort_frame(Frame<N, R> &f)
{
    if constexpr (N == 2) {
        cswap<N, R>(f, 0, 1);
    } else if constexpr (N == 3) {
        cswap<N, R>(f, 0, 1);
        cswap<N, R>(f, 1, 2);
        cswap<N, R>(f, 0, 1);
    } else if constexpr (N == 4) {
        cswap<N, R>(f, 0, 1);
        cswap<N, R>(f, 2, 3);
        cswap<N, R>(f, 0, 2);
        cswap<N, R>(f, 1, 3);
        cswap<N, R>(f, 1, 2);
    } else {
#pragma unroll
        for (int round = 0; round < N; ++round)
#pragma unroll
            for (int i = round & 1; i + 1 < N; i += 2)
                cswap<N, R>(f, i, i + 1);
    }
}

// eigen-solve of V from the previous frame U0: rotate, Jacobi, sort,
// sign-align with U0, Rayleigh energies
template <int N, typename R>
__device__ __forceinline__ void solve_warm(const R (&V)[kTri<N>], const R (&U0)[N][N], R eps, Frame<N, R> &f)
{
    R A[kTri<N>];
    congruence<N, R>(V, U0, A);
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int k = 0; k < N; ++k)
            f.U[i][k] = U0[i][k];
    const R turned = jacobi<N, R>(A, f.U, eps, sizeof(R) == 8 ? 10 : 8);
#pragma unroll
    for (int k = 0; k < N; ++k)
        f.E[k] = A[tri_index<N>(k, k)];
    // The sorting network leaves sorted energies as they are, so it runs
    // only when some lane of the wavefront has them out of order.
    bool unsorted = false;
#pragma unroll
    for (int k = 0; k + 1 < N; ++k)
        unsorted |= f.E[k + 1] < f.E[k];
    const bool resorted = __any(unsorted);
    if (resorted)
        sort_frame<N, R>(f);
    // Sign alignment.  Without a reordering, U = U0 J with J the product of
    // the lane's rotations, and ||J - I||_2 <= sum ||R_i - I||_2 =
    // sum 2 |sin(angle_i / 2)| <= sum |t_i|; so when that sum is below 1/2,
    // every u0_k . u_k = J_kk > 1/2 and no column changes sign: the check
    // runs only when some lane turned further or was reordered.
    if (resorted || __any(turned >= R(0.5))) {
#pragma unroll
        for (int k = 0; k < N; ++k) {
            R d = R(0);
#pragma unroll
            for (int r = 0; r < N; ++r)
                d = fma_g(U0[r][k], f.U[r][k], d);
            if (d < R(0)) {
#pragma unroll
                for (int r = 0; r < N; ++r)
                    f.U[r][k] = -f.U[r][k];
            }
        }
    }
    rayleigh<N, R>(V, f.U, f.E);
}

// eigen-solve from the identity; each column's first nonzero entry on the
// diagonal or below made positive (U_kk > 0 when U_kk != 0)
template <int N>
__device__ __forceinline__ void solve_cold(const double (&V)[kTri<N>], double eps, Frame<N, double> &f)
{
    double A[kTri<N>];
#pragma unroll
    for (int k = 0; k < kTri<N>; ++k)
        A[k] = V[k];
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int k = 0; k < N; ++k)
            f.U[i][k] = (i == k) ? 1.0 : 0.0;
    jacobi<N, double>(A, f.U, eps, 40);
#pragma unroll
    for (int k = 0; k < N; ++k)
        f.E[k] = A[tri_index<N>(k, k)];
    sort_frame<N, double>(f);
#pragma unroll
    for (int k = 0; k < N; ++k) {
        double lead = f.U[k][k];
#pragma unroll
        for (int r = 0; r < N; ++r)
            lead = (lead == 0.0) ? f.U[r][k] : lead;
        if (lead < 0.0) {
#pragma unroll
            for (int r = 0; r < N; ++r)
                f.U[r][k] = -f.U[r][k];
        }
    }
    rayleigh<N, double>(V, f.U, f.E);
}

template <int N, typename R>
__device__ __forceinline__ R min_gap(const Frame<N, R> &f)
{
    R g = f.E[1] - f.E[0];
#pragma unroll
    for (int k = 1; k + 1 < N; ++k)
        g = (f.E[k + 1] - f.E[k]) < g ? (f.E[k + 1] - f.E[k]) : g;
    return g;
}

// x[a] for a runtime index a < N.  A chain of selects over the elements of
// an array is turned by the compiler into an indexed private (scratch) copy
// of the array; the sum of x[k] weighted by 0 or 1 is exact for finite
// entries and keeps everything in registers.
template <int N, typename R>
__device__ __forceinline__ R pick(const R (&x)[N], int a)
{
    R s = R(0);
#pragma unroll
    for (int k = 0; k < N; ++k)
        s = fma_g(x[k], (a == k) ? R(1) : R(0), s);
    return s;
}

template <int N, typename R>
__device__ __forceinline__ void column(const Frame<N, R> &f, int a, R (&u)[N])
{
#pragma unroll
    for (int r = 0; r < N; ++r)
        u[r] = pick<N, R>(f.U[r], a);
}

template <int N, typename R>
__device__ __forceinline__ R energy(const Frame<N, R> &f, int a)
{
    return pick<N, R>(f.E, a);
}

// row a of the symmetric triangle M
template <int N, typename R>
__device__ __forceinline__ void tri_row(const R (&M)[kTri<N>], int a, R (&row)[N])
{
#pragma unroll
    for (int c = 0; c < N; ++c) {
        R x[N];
#pragma unroll
        for (int k = 0; k < N; ++k)
            x[k] = M[sym_index<N>(k, c)];
        row[c] = pick<N, R>(x, a);
    }
}

// One output bin of the workgroup's tile, reduced into dst (tile_values(N)
// doubles): the per-walker values [basis][i][j][stat] (basis 0 adiabatic
// W [a==i][b==j], basis 1 diabatic W U_ia U_jb; stats Re, Im, Re^2, Im^2),
// two cells of 4 stats per LDS pass, then the excluded count.  A walker's
// adiabatic terms sit in its own cell only: the staging row is cleared and
// that cell written under an exec mask.  Every thread of the workgroup
// calls it.
template <int N, typename R>
__device__ __forceinline__ void bin_store(BinLds &L, int &parity, bool live, int a, int b, double w, double phase,
                                          const Frame<N, R> &f, double *__restrict__ dst)
{
    constexpr int NN = N * N;
    constexpr int NV = 8 * NN;
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
    R ua[N], ub[N];
    column<N, R>(f, a, ua);
    column<N, R>(f, b, ub);
    const int cell = a * N + b;  // the walker's adiabatic cell
    BinReducerPerPass B(L, parity);
#pragma unroll
    for (int p = 0; p < NN; ++p) {  // pass p: cells 2p and 2p + 1 of the 2 N^2
        if (2 * p < NN)
            B.zero_row();
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int c = 2 * p + h;
            if (c >= NN) {  // diabatic cell (i, j)
                const int ii = (c - NN) / N, jj = (c - NN) % N;
                // an excluded walker contributes exact zeros (its frame may be NaN)
                const double cij = ok ? (double)ua[ii] * (double)ub[jj] : 0.0;
                const double r = re * cij, m = im * cij;
                B.put(4 * h + 0, r);
                B.put(4 * h + 1, m);
                B.put(4 * h + 2, r * r);
                B.put(4 * h + 3, m * m);
            }
        }
        if (2 * p < NN && (cell >> 1) == p) {
            const int col = 4 * (cell & 1);
            B.put(col + 0, re);
            B.put(col + 1, im);
            B.put(col + 2, re * re);
            B.put(col + 3, im * im);
        }
        B.pass();
        const bool last = p == NN - 1;
        if ((p & 3) == 3 || last) {
            const int c0 = (p & ~3) * kPassValues;
            if (last)
                B.count_excluded(live && !ok);
            B.flush(dst + c0, (NV - c0) < kFlushValues ? (NV - c0) : kFlushValues, last ? dst + NV : nullptr);
        }
    }
}

// Weights of the slots of a symmetric matrix A in the mean of element
// (a, b): sum_{k<=l} A_kl P_kl = [(U^T A U)_aa + (U^T A U)_bb] / 2, with
// P_kk = (U_ka^2 + U_kb^2) / 2 and P_kl = U_ka U_la + U_kb U_lb (k < l).
// The binary32 solve leaves each eigenvector accurate to O(eps32 ||V||/gap)
// per gap; only the mixing inside the closest pair (k, k+1) degrades as
// their gap closes.  That pair's 2x2 block of V is rebuilt in binary64 in
// the binary32 columns (vslot(s) gives slot s of V in binary64), diagonalised
// by one binary64 Jacobi rotation, and the two columns are rotated, ordered
// by their binary64 energies and sign-aligned with the previous frame U0.
template <int N, typename VSlot>
__device__ __forceinline__ void refine_pair64_with(VSlot vslot, const float (&U0)[N][N], Frame<N, float> &f)
{
    // the pair with the smallest gap
    int k = 0;
    float g = f.E[1] - f.E[0];
#pragma unroll
    for (int c = 1; c + 1 < N; ++c) {
        const float gc = f.E[c + 1] - f.E[c];
        k = gc < g ? c : k;
        g = gc < g ? gc : g;
    }
    // the 2x2 block of V in the pair's binary32 columns u, v (their entries
    // are exact in binary64), slot by slot
    float u[N], v[N];
#pragma unroll
    for (int r = 0; r < N; ++r) {
        u[r] = pick<N, float>(f.U[r], k);
        v[r] = pick<N, float>(f.U[r], k + 1);
    }
    double a = 0.0, b = 0.0, c = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int l = i; l < N; ++l) {
            const double vs = vslot(tri_index<N>(i, l));
            const double ui = u[i], ul = u[l], vi = v[i], vl = v[l];
            if (i == l) {
                a = fma_g(vs, ui * ui, a);
                b = fma_g(vs, vi * vi, b);
                c = fma_g(vs, ui * vi, c);
            } else {
                a = fma_g(vs, 2.0 * (ui * ul), a);
                b = fma_g(vs, 2.0 * (vi * vl), b);
                c = fma_g(vs, fma_g(ui, vl, ul * vi), c);
            }
        }
    double cs = 1.0, sn = 0.0;
    if (c != 0.0) {
        const double theta = (b - a) * rcp_g(2.0 * c);
        double t = rcp_g(abs_g(theta) + sqrt_ge1<double>(fma_g(theta, theta, 1.0)));
        t = theta < 0.0 ? -t : t;
        cs = rsq_g(fma_g(t, t, 1.0));
        sn = t * cs;
        a -= t * c;
        b += t * c;
    }
    // rotated columns, lower energy first, signs continuous with U0
    const bool swap = b < a;
    float nu[N], nv[N];
#pragma unroll
    for (int r = 0; r < N; ++r) {
        const double x = fma_g(cs, (double)u[r], -sn * (double)v[r]);
        const double y = fma_g(sn, (double)u[r], cs * (double)v[r]);
        nu[r] = (float)(swap ? y : x);
        nv[r] = (float)(swap ? x : y);
    }
    // sign alignment against the previous frame's columns k, k+1
    double d0 = 0.0, d1 = 0.0;
#pragma unroll
    for (int r = 0; r < N; ++r) {
        d0 = fma_g((double)pick<N, float>(U0[r], k), (double)nu[r], d0);
        d1 = fma_g((double)pick<N, float>(U0[r], k + 1), (double)nv[r], d1);
    }
#pragma unroll
    for (int r = 0; r < N; ++r) {
        nu[r] = d0 < 0.0 ? -nu[r] : nu[r];
        nv[r] = d1 < 0.0 ? -nv[r] : nv[r];
    }
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
        for (int col = 0; col < N; ++col) {
            const float x = f.U[r][col];
            f.U[r][col] = (col == k) ? nu[r] : (col == k + 1) ? nv[r] : x;
        }
}

template <int N, typename R>
__device__ __forceinline__ void pair_weights(const Frame<N, R> &f, int a, int b, R (&P)[kTri<N>])
{
    R ua[N], ub[N];
    column<N, R>(f, a, ua);
    column<N, R>(f, b, ub);
#pragma unroll
    for (int k = 0; k < N; ++k)
#pragma unroll
        for (int l = k; l < N; ++l)
            P[tri_index<N>(k, l)] = (k == l) ? R(0.5) * fma_g(ua[k], ua[k], ub[k] * ub[k])
                                             : fma_g(ua[k], ua[l], ub[k] * ub[l]);
}

// The Monte Carlo move of one step at the walker's current point (Eq. 1's
// coupling term): from rows a and b of D = U^T (sum_j v_j dV/dq_j) U, the
// candidate factors f = dt D_ac / (E_c - E_a) towards (c, b) and
// dt D_bc / (E_c - E_b) towards (a, c), in that fixed order, with
// S = sum |f|.  Normalized rule: stay with probability 1/(1+S), else take
// the first candidate whose cumulative |f| passes t - 1, t = u (1 + S);
// w <- w (1 + S) sgn(f).  Linear rule (while S < 1, else the normalized one
// with kFlagFallback): candidate k with probability |f_k|, w <- w sgn(f_k),
// or stay with w <- w / (1 - S).  A pick that rounding leaves empty takes
// the last candidate with f != 0.
template <int N, typename R>
__device__ __forceinline__ void transition(const Frame<N, R> &f, const R (&Da)[N], const R (&Db)[N], R u, R dt,
                                           bool linear_rule, int &a, int &b, double &w, uint32_t &flag)
{
    constexpr int NC = 2 * N;  // candidate slots (two are always empty)
    const R Ea = energy<N, R>(f, a), Eb = energy<N, R>(f, b);
    R fc[NC], af[NC];
    R S = R(0);
#pragma unroll
    for (int c = 0; c < N; ++c) {
        fc[c] = (c != a) ? dt * div_g(Da[c], f.E[c] - Ea) : R(0);      // -> (c, b)
        fc[N + c] = (c != b) ? dt * div_g(Db[c], f.E[c] - Eb) : R(0);  // -> (a, c)
    }
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        af[k] = abs_g(fc[k]);
        S += af[k];
    }
    int choice = -1;
    const bool linear = linear_rule && S < R(1);
    if (linear_rule && !linear)
        flag |= kFlagFallback;
    const R t = linear ? u : u * (R(1) + S);
    const R base = linear ? R(0) : R(1);
    const bool stay = !linear && (t < R(1));
    R Cm = R(0);
    int last = -1;
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        Cm += af[k];
        const bool valid = (k < N) ? (k != a) : (k - N != b);
        if (!stay && choice < 0 && valid && t < base + Cm)
            choice = k;
        last = (valid && af[k] > R(0)) ? k : last;
    }
    if (!linear && !stay && choice < 0)
        choice = last;
    bool positive = true;  // sign of the chosen factor (true when staying)
#pragma unroll
    for (int k = 0; k < NC; ++k)
        positive = (choice == k) ? (fc[k] > R(0)) : positive;
    const double sg = positive ? 1.0 : -1.0;
    // The rule is a kernel argument, uniform over the wave: a scalar
    // branch on it, and per-lane selects inside.  A divergent
    // if/else here let the compiler place the copy of w that lives
    // across the join before the exec mask was restored, so lanes
    // of the other side kept no copy of their weight.
    if (linear_rule) {
        const double w_lin = (choice < 0) ? w / (double)(R(1) - S) : w * sg;
        const double w_norm = w * (double)(R(1) + S) * sg;
        w = linear ? w_lin : w_norm;
    } else {
        w = w * (double)(R(1) + S) * sg;
    }
    if (choice >= 0) {
        if (choice < N) a = choice;
        else b = choice - N;
    }
}

// The initial density-matrix element (a, b) and weight w of a walker from
// its frame f at the sampled q: adiabatic state k gives (k, k) and w = 1; a
// diabatic state k gives rho_ab = U_ka U_kb, drawn with probability
// |U_ka U_kb| / Z, Z = (sum_c |U_kc|)^2, and w = sgn(U_ka U_kb) Z (an
// unbiased estimator of rho).  The uniform comes from the walker's Philox
// block (gid, 0, 0, 2).
template <int N>
__device__ __forceinline__ void initial_element(const Frame<N, double> &f, const SampleArgs &S, uint64_t gid, int &a,
                                                int &b, double &w)
{
    if (S.basis == QCL_INIT_ADIABATIC) {
        a = b = S.state;
        w = 1.0;
    } else {
        // diabatic |k><k| in the adiabatic basis: rho_ab = U_ka U_kb
        double uk[N];
#pragma unroll
        for (int c = 0; c < N; ++c) {
            double col[N];
#pragma unroll
            for (int r = 0; r < N; ++r)
                col[r] = f.U[r][c];
            uk[c] = pick<N, double>(col, S.state);
        }
        double rs = 0.0;
#pragma unroll
        for (int c = 0; c < N; ++c)
            rs += __builtin_fabs(uk[c]);
        const double Z = rs * rs;
        const U4 x = philox10(U4{(uint32_t)gid, (uint32_t)(gid >> 32), 0u, 2u}, S.key0, S.key1);
        const double t = u52(x.x, x.y) * Z;
        int pa = -1, pb = -1, la = 0, lb = 0;
        double Cm = 0.0;
#pragma unroll
        for (int ia = 0; ia < N; ++ia)
#pragma unroll
            for (int ib = 0; ib < N; ++ib) {
                const double wgt = __builtin_fabs(uk[ia] * uk[ib]);
                if (wgt > 0.0) { la = ia; lb = ib; }
                Cm += wgt;
                if (pa < 0 && t < Cm) { pa = ia; pb = ib; }
            }
        if (pa < 0) { pa = la; pb = lb; }
        a = pa;
        b = pb;
        const double ua = pick<N, double>(uk, pa), ubv = pick<N, double>(uk, pb);
        w = (ua * ubv > 0.0 ? 1.0 : -1.0) * Z;
    }
}

}  // namespace qcl
