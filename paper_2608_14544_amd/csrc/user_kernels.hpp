// Kernels for a model with a supplied potential (the general form of Eq. 1:
// any real symmetric N x N diabatic matrix V(q) of the classical modes,
// H = sum_j p_j^2 / (2 m_j) + V(q)), compiled at run time with the caller's
// device source in front.  That source defines
//
//   __device__ void qcl_potential(const double *q, double *V);
//       V(q): the N(N+1)/2 upper-triangle entries V_kl (k <= l), row by row
//   __device__ void qcl_force(const double *q, const double *w, double *f);
//       f_j = -sum_s w_s dV_s/dq_j for the M modes (w: one weight per slot)
//   __device__ void qcl_coupling(const double *q, const double *v, double *K);
//       K_s = sum_j v_j dV_s/dq_j (v: one value per mode)
//
// and may read QCL_N, QCL_M and the caller's parameters qcl_param[], which
// the compilation defines before it.  The functions are binary64; a source
// that also defines them for float arguments (overloads or templates) and
// defines QCL_SOURCE_FP32 gets the binary32 kernels too (binary32 state and
// step, binary64 weight, phase and sums, and a binary64 re-solve of the
// closest pair of states, from the binary64 potential, where the smallest
// gap falls below the model's threshold).  The step is
// the one of the built-in models (Monte Carlo move from rows a and b of
// D = U^T K(v) U at (q_n, p_n), velocity Verlet on the mean force of the
// new element, eigen-solve at q_{n+1} warm-started from the previous
// frame, trapezoid phase, bins every cadence steps), with the force and the
// velocity coupling taken from the caller's functions: the mean force is
// qcl_force with the slot weights of element (a, b), so that it equals
// -[(U^T dV/dq_j U)_aa + (U^T dV/dq_j U)_bb] / 2.
#pragma once

#include "nstate_frame.hpp"

namespace qcl {

// p_j += dt/2 f_j with the mean force of element (a, b) in frame f at q
template <int N, int M, typename R>
__device__ __forceinline__ void user_kick(const R (&q)[M], const Frame<N, R> &f, int a, int b, R hdt, R (&p)[M])
{
    R P[kTri<N>], F[M];
    pair_weights<N, R>(f, a, b, P);
    qcl_force(q, P, F);
#pragma unroll
    for (int j = 0; j < M; ++j)
        p[j] = fma_g(hdt, F[j], p[j]);
}

// K(v) = sum_j v_j dV/dq_j at q, v = p/m
template <int N, int M, typename R>
__device__ __forceinline__ void user_velocity_coupling(const R (&q)[M], const R (&p)[M], const double (&inv_mass)[M],
                                                       R (&K)[kTri<N>])
{
    R v[M];
#pragma unroll
    for (int j = 0; j < M; ++j)
        v[j] = p[j] * (R)inv_mass[j];
    qcl_coupling(q, v, K);
}

// rows a and b of D = U^T K U
template <int N, typename R>
__device__ __forceinline__ void coupling_rows(const R (&K)[kTri<N>], const Frame<N, R> &f, int a, int b, R (&Da)[N],
                                              R (&Db)[N])
{
    R ua[N], ub[N], wa[N], wb[N];
    column<N, R>(f, a, ua);
    column<N, R>(f, b, ub);
#pragma unroll
    for (int k = 0; k < N; ++k) {
        R sa = R(0), sb = R(0);
#pragma unroll
        for (int l = 0; l < N; ++l) {
            const R kv = K[sym_index<N>(k, l)];
            sa = fma_g(kv, ua[l], sa);
            sb = fma_g(kv, ub[l], sb);
        }
        wa[k] = sa;
        wb[k] = sb;
    }
#pragma unroll
    for (int c = 0; c < N; ++c) {
        R da = R(0), db = R(0);
#pragma unroll
        for (int k = 0; k < N; ++k) {
            da = fma_g(f.U[k][c], wa[k], da);
            db = fma_g(f.U[k][c], wb[k], db);
        }
        Da[c] = da;
        Db[c] = db;
    }
}

// Wigner sampling of the harmonic reference (the same draws as the built-in
// models: Philox block (gid, j, 1) per mode, Box-Muller), frame from the
// identity, initial element, bin 0; all in binary64, stored in the
// ensemble's precision R.
template <int N, int M, typename R>
__device__ __forceinline__ void user_sample(const SampleArgs &S, const UserArgs &A, const EnsDev<R> &E,
                                            double *__restrict__ partials, int32_t n_out, BinLds &lds)
{
    int parity = 0;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool live = i < E.n_traj;
    const uint64_t gid = (uint64_t)(E.traj_offset + (live ? i : 0));
    const double two_pi = 6.283185307179586476925286766559;
    const int64_t ld = E.ld;
    double q[M];
#pragma unroll
    for (int j = 0; j < M; ++j) {
        const U4 x = philox10(U4{(uint32_t)gid, (uint32_t)(gid >> 32), (uint32_t)j, 1u}, S.key0, S.key1);
        const double u1 = u52(x.x, x.y);
        const double u2 = u52(x.z, x.w);
        const double rr = sqrt(-2.0 * log(u1));
        double sn, cs;
        sincos_phase(two_pi * u2, sn, cs);
        q[j] = S.q0[j] + S.sq[j] * (rr * cs);
        const double pj = S.sp[j] * (rr * sn);
        if (live) {
            E.q[j * ld + i] = (R)q[j];
            E.p[j * ld + i] = (R)pj;
        }
    }
    double V[kTri<N>];
    qcl_potential(q, V);
    Frame<N, double> f;
    solve_cold<N>(V, A.rot_eps, f);
    uint32_t flag = 0;
    if (!(min_gap<N, double>(f) > 2.2250738585072014e-308))
        flag |= kFlagDegenerate;
    int a, b;
    double w;
    initial_element<N>(f, S, gid, a, b, w);
    bin_store<N, double>(lds, parity, live, a, b, w, 0.0, f,
                         partials + ((int64_t)blockIdx.x * n_out + 0) * tile_values(N));
    if (live) {
#pragma unroll
        for (int r = 0; r < N; ++r)
#pragma unroll
            for (int k = 0; k < N; ++k)
                E.u[(r * N + k) * ld + i] = (R)f.U[r][k];
        E.w[i] = w;
        E.phase[i] = 0.0;
        E.a[i] = (uint8_t)a;
        E.b[i] = (uint8_t)b;
        if (E.flags)
            E.flags[i] = flag;
    }
}

// All steps of one tile of kBlock walkers (the whole workgroup calls it).
template <int N, int M, typename R>
__device__ __forceinline__ void user_propagate_tile(const UserArgs &A, const PropArgs &P, const EnsDev<R> &E,
                                                    const double (&inv_mass)[M], double *__restrict__ partials,
                                                    int64_t tile, BinLds &lds, int &parity)
{
    constexpr int T = kTri<N>;
    const int64_t i = tile * kBlock + threadIdx.x;
    const bool live = i < E.n_traj;
    const int64_t li = live ? i : E.n_traj - 1;
    const int64_t ld = E.ld;
    const uint64_t gid = (uint64_t)(E.traj_offset + li);
    const uint32_t g_lo = (uint32_t)gid, g_hi = (uint32_t)(gid >> 32);
    const bool linear_rule = P.scheme == QCL_TRANS_LINEAR;
    const R dt = (R)A.dt, hdt = (R)A.hdt, eps = (R)A.rot_eps;

    R q[M], p[M];
#pragma unroll
    for (int j = 0; j < M; ++j) {
        q[j] = E.q[j * ld + li];
        p[j] = E.p[j * ld + li];
    }
    double w = E.w[li];
    double phase = E.phase[li];
    int a = E.a[li];
    int b = E.b[li];
    uint32_t flag = 0;
    Frame<N, R> f;
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
        for (int k = 0; k < N; ++k)
            f.U[r][k] = E.u[(r * N + k) * ld + li];
    R K[T];
    {
        R V[T];
        qcl_potential(q, V);
        rayleigh<N, R>(V, f.U, f.E);
        user_velocity_coupling<N, M, R>(q, p, inv_mass, K);
    }

    int64_t step = P.step0;
    const int64_t end = P.step0 + P.n_steps;
    U4 rnd{0, 0, 0, 0};
    if (step & 3)
        rnd = philox10(U4{g_lo, g_hi, (uint32_t)(step >> 2), 0u}, P.key0, P.key1);
    while (step < end) {
        const int64_t next_bin = (step / P.cadence + 1) * P.cadence;
        const int64_t stop = next_bin < end ? next_bin : end;
        for (; step < stop; ++step) {
            if ((step & 3) == 0)
                rnd = philox10(U4{g_lo, g_hi, (uint32_t)(step >> 2), 0u}, P.key0, P.key1);
            const uint32_t word = pick_word(rnd, (uint32_t)(step & 3));
            R u;
            if constexpr (sizeof(R) == 4) u = u24f(word); else u = u24d(word);

            // 1. Monte Carlo move at (q_n, p_n)
            R Da[N], Db[N];
            coupling_rows<N, R>(K, f, a, b, Da, Db);
            transition<N, R>(f, Da, Db, u, dt, linear_rule, a, b, w, flag);

            // 2. velocity Verlet on the mean force of the current element
            const R dE0 = energy<N, R>(f, a) - energy<N, R>(f, b);
            user_kick<N, M, R>(q, f, a, b, hdt, p);
#pragma unroll
            for (int j = 0; j < M; ++j)
                q[j] = fma_g(dt, p[j] * (R)inv_mass[j], q[j]);
            {
                R V[T], U0[N][N];
                qcl_potential(q, V);
#pragma unroll
                for (int r = 0; r < N; ++r)
#pragma unroll
                    for (int k = 0; k < N; ++k)
                        U0[r][k] = f.U[r][k];
                solve_warm<N, R>(V, U0, eps, f);
                if constexpr (sizeof(R) == 4) {
                    if (!(min_gap<N, R>(f) >= (R)A.gap_thr)) {  // near-degenerate: binary64
                        double q64[M], V64[T];
#pragma unroll
                        for (int j = 0; j < M; ++j)
                            q64[j] = (double)q[j];
                        qcl_potential(q64, V64);
                        refine_pair64_with<N>([&](int sl) { return V64[sl]; }, U0, f);
                        rayleigh<N, R>(V, f.U, f.E);
                        flag |= kFlagResolved;
                    }
                }
            }
            if (!(min_gap<N, R>(f) > R(2.2250738585072014e-308)))
                flag |= kFlagDegenerate;
            user_kick<N, M, R>(q, f, a, b, hdt, p);
            user_velocity_coupling<N, M, R>(q, p, inv_mass, K);

            // 3. phase: trapezoid of w_ab = (E_a - E_b)/hbar
            const R dE1 = energy<N, R>(f, a) - energy<N, R>(f, b);
            phase += A.dt_hbar * 0.5 * ((double)dE0 + (double)dE1);
        }
        // 4. output bin at global step next_bin
        if (step == next_bin && next_bin / P.cadence < P.n_out) {
            bin_store<N, R>(lds, parity, live, a, b, w, phase, f,
                            partials + (tile * P.n_out + next_bin / P.cadence) * tile_values(N));
        }
    }
    if (!(__builtin_isfinite(w) && __builtin_isfinite(phase)))
        flag |= kFlagNonfinite;

    if (live) {
#pragma unroll
        for (int j = 0; j < M; ++j) {
            E.q[j * ld + i] = q[j];
            E.p[j * ld + i] = p[j];
        }
#pragma unroll
        for (int r = 0; r < N; ++r)
#pragma unroll
            for (int k = 0; k < N; ++k)
                E.u[(r * N + k) * ld + i] = f.U[r][k];
        E.w[i] = w;
        E.phase[i] = phase;
        E.a[i] = (uint8_t)a;
        E.b[i] = (uint8_t)b;
        if (E.flags)
            E.flags[i] |= flag;
    }
}

template <int N, int M, typename R>
__device__ __forceinline__ void user_propagate(const UserArgs &A, const PropArgs &P, const EnsDev<R> &E,
                                               const double (&inv_mass)[M], double *__restrict__ partials,
                                               BinLds &lds)
{
    int parity = 0;
    user_propagate_tile<N, M, R>(A, P, E, inv_mass, partials, (int64_t)blockIdx.x, lds, parity);
}

// Persistent launch over the (instance, tile) items of many ensembles of
// this model: items are taken from a device counter (descriptors sorted by
// decreasing work per tile), as in the built-in batched kernels.
template <int N, int M, typename R>
__device__ __forceinline__ void user_batch(const UserBatchItem<R> *__restrict__ items, int32_t n_items,
                                           int64_t total_tiles, unsigned long long *counter,
                                           const double (&inv_mass)[M], BinLds &lds, long long &item_sh)
{
    int parity = 0;
    for (;;) {
        if (threadIdx.x == 0)
            item_sh = (long long)atomicAdd(counter, 1ull);
        __syncthreads();
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
        const UserBatchItem<R> &it = items[lo];
        user_propagate_tile<N, M, R>(it.A, it.P, it.E, inv_mass, it.partials, item - it.tile_begin, lds, parity);
        __syncthreads();
    }
}

}  // namespace qcl
