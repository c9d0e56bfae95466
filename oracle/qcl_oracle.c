/*
 * qcl_oracle.c -- plain FP64 CPU oracle of the momentum-jump-free
 * quantum-classical Liouville (QCL) trajectory ensemble.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code,
 * header, table or constant with the HIP path: it has its own Philox, its
 * own Jacobi eigensolver and its own reduction.
 *
 * What is computed (paper Sec. II.A, Eq. 1): each walker carries one
 * density-matrix element (a,b) of the adiabatic basis, classical (q,p), a
 * real weight w and a phase Phi, so that its contribution to rho_ab is
 * W = w exp(-i Phi).  The four terms of Eq. 1 are realised as
 *   -i w_ab rho            -> Phi += int w_ab dt      (trapezoid)
 *   -(P/M) sum_g (d rho - rho d)
 *                          -> Monte Carlo move to (c,b) or (a,c) with a
 *                             weight update; P is not changed (Sec. II.A:
 *                             no off-diagonal Hellmann-Feynman force)
 *   -(P/M) d/dR rho - (F_a+F_b)/2 d/dP rho
 *                          -> velocity Verlet on the mean force (F_a+F_b)/2
 * with a fixed number of walkers and no spawning (Sec. II.B).
 *
 * Conventions where the paper is silent (each one a stated reading):
 *   - step order: transition at (q_n, p_n), then Verlet, then phase;
 *   - transition rule: stay with probability 1/(1+S), move to candidate k
 *     with probability |f_k|/(1+S), w *= (1+S) sgn(f_k) ("normalized"),
 *     or the "linear" rule when S < 1;
 *   - RNG: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) keyed by the
 *     64-bit seed, counters built from (trajectory id, step);
 *   - eigenvalues ascending; eigenvector signs: U_kk > 0 at t = 0, then
 *     each column kept continuous by overlap with the previous step;
 *   - observables normalised by the number of walkers.
 *
 * Beyond the linear-vibronic form V(q) = V0 + sum_j q_j K_j, a model may
 * carry higher separable powers sum_{k=2..4} q_j^k A_jk (state-dependent
 * frequencies and anharmonicity); forces and couplings then use
 * dV/dq_j = K_j + sum_k k q_j^(k-1) A_jk, evaluated directly.
 *
 * Floating point: IEEE binary64, compiled without fast-math and without
 * FMA contraction.
 */
#include <math.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdlib.h>
#include <string.h>

#define OR_MAXN 8
#define OR_MAXM 128
#define OR_CHUNK 1024

typedef struct {
    int32_t n_states;
    int32_t n_modes;
    const double *mass;   /* [M] */
    const double *omega;  /* [M] */
    const double *v0;     /* [N][N] */
    const double *k;      /* [M][N][N] */
    double hbar;
    int32_t degree;       /* highest power of q_j in V(q): 1 (linear) .. 4 */
    const double *a;      /* [M][degree-1][N][N]: A_jk for k = 2..degree, or NULL */
    int32_t n_pairs;      /* bilinear terms q_i q_j B_p, i != j (0: none) */
    const int32_t *pairs; /* [n_pairs][2]: the modes (i, j) of each term */
    const double *bpair;  /* [n_pairs][N][N]: B_p */
    /* A supplied potential (the general form of Eq. 1): when user_v is set,
     * V(q) and dV/dq_j come from these functions of (q, user_prm) and are
     * the whole q-dependent Hamiltonian -- v0, k, the higher powers, the
     * bilinear terms and the harmonic bath term m w^2 q^2 / 2 are not used
     * (mass and omega still give the kinetic term and the Wigner widths). */
    void (*user_v)(const double *q, const double *prm, double *V);           /* V [N][N] */
    void (*user_dv)(int j, const double *q, const double *prm, double *Gj);  /* dV/dq_j [N][N] */
    const double *user_prm;
} or_model;

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11): 10 rounds of the 4x32 S-box   */
/* with multipliers 0xD2511F53, 0xCD9E8D57 and Weyl key increments     */
/* 0x9E3779B9, 0xBB67AE85.                                             */
/* ------------------------------------------------------------------ */
void or_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void philox_block(uint64_t seed, uint64_t traj, uint32_t c2, uint32_t c3, uint32_t out[4])
{
    uint32_t ctr[4] = {(uint32_t)traj, (uint32_t)(traj >> 32), c2, c3};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    or_philox4x32_10(ctr, key, out);
}

/* 24-bit uniform in (0,1): (2 floor(x/2^9) + 1) / 2^24, exact in binary32. */
double or_uniform24(uint32_t x)
{
    return (double)(2u * (x >> 9) + 1u) / 16777216.0;
}

/* 52-bit uniform in (0,1) from two words: k = hi*2^20 + floor(lo/2^12). */
double or_uniform52(uint32_t hi, uint32_t lo)
{
    uint64_t k = ((uint64_t)hi << 20) | (uint64_t)(lo >> 12);
    return (double)(2u * k + 1u) / 9007199254740992.0;
}

/* ------------------------------------------------------------------ */
/* Symmetric eigenproblem by cyclic Jacobi rotations (Golub & Van Loan, */
/* Matrix Computations, Sec. 8.5).  A is n x n row-major and symmetric; */
/* on return E holds the eigenvalues ascending and the columns of U the */
/* eigenvectors (A = U diag(E) U^T).                                   */
/* ------------------------------------------------------------------ */
void or_jacobi_eigh(int n, const double *a_in, double *E, double *U)
{
    double A[OR_MAXN * OR_MAXN];
    memcpy(A, a_in, sizeof(double) * n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            U[i * n + j] = (i == j) ? 1.0 : 0.0;

    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int p = 0; p < n; ++p) {
            diag += A[p * n + p] * A[p * n + p];
            for (int q = p + 1; q < n; ++q)
                off += A[p * n + q] * A[p * n + q];
        }
        if (off == 0.0 || off <= 1e-40 * diag)
            break;
        for (int p = 0; p < n - 1; ++p) {
            for (int q = p + 1; q < n; ++q) {
                double apq = A[p * n + q];
                if (apq == 0.0)
                    continue;
                /* rotation [[c, s], [-s, c]] in the (p,q) plane zeroing A_pq */
                double tau = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
                double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                double c = 1.0 / sqrt(1.0 + t * t);
                double s = t * c;
                for (int r = 0; r < n; ++r) { /* A <- A J */
                    double arp = A[r * n + p], arq = A[r * n + q];
                    A[r * n + p] = c * arp - s * arq;
                    A[r * n + q] = s * arp + c * arq;
                }
                for (int r = 0; r < n; ++r) { /* A <- J^T A */
                    double apr = A[p * n + r], aqr = A[q * n + r];
                    A[p * n + r] = c * apr - s * aqr;
                    A[q * n + r] = s * apr + c * aqr;
                }
                A[p * n + q] = 0.0;
                A[q * n + p] = 0.0;
                for (int r = 0; r < n; ++r) { /* U <- U J */
                    double urp = U[r * n + p], urq = U[r * n + q];
                    U[r * n + p] = c * urp - s * urq;
                    U[r * n + q] = s * urp + c * urq;
                }
            }
        }
    }
    for (int i = 0; i < n; ++i)
        E[i] = A[i * n + i];
    /* ascending order (selection sort, columns follow) */
    for (int i = 0; i < n - 1; ++i) {
        int m = i;
        for (int j = i + 1; j < n; ++j)
            if (E[j] < E[m])
                m = j;
        if (m != i) {
            double te = E[i]; E[i] = E[m]; E[m] = te;
            for (int r = 0; r < n; ++r) {
                double tu = U[r * n + i]; U[r * n + i] = U[r * n + m]; U[r * n + m] = tu;
            }
        }
    }
}

static void flip_column(int n, double *U, int k)
{
    for (int r = 0; r < n; ++r)
        U[r * n + k] = -U[r * n + k];
}

/* Eigenvector sign convention.  Without a previous frame: U_kk > 0 (if
 * U_kk == 0, the first nonzero entry of the column is made positive).
 * With a previous frame: column k is flipped when its overlap with the
 * previous column k is negative (an overlap of exactly zero keeps it). */
void or_gauge(int n, const double *Uprev, double *U)
{
    for (int k = 0; k < n; ++k) {
        if (Uprev) {
            double dot = 0.0;
            for (int r = 0; r < n; ++r)
                dot += Uprev[r * n + k] * U[r * n + k];
            if (dot < 0.0)
                flip_column(n, U, k);
        } else {
            double lead = U[k * n + k];
            if (lead == 0.0)
                for (int r = 0; r < n && lead == 0.0; ++r)
                    lead = U[r * n + k];
            if (lead < 0.0)
                flip_column(n, U, k);
        }
    }
}

/* Entry i of A_jk (k >= 2) of a model with higher powers. */
static double poly_entry(const or_model *m, int j, int k, int i)
{
    int n = m->n_states;
    return m->a[((size_t)j * (m->degree - 1) + (k - 2)) * n * n + i];
}

/* Electronic Hamiltonian V(q) = V0 + sum_j [q_j K_j + sum_{k=2..D} q_j^k A_jk]
 * + sum_p q_{i_p} q_{j_p} B_p (cross-mode bilinear terms). */
void or_potential(const or_model *m, const double *q, double *V)
{
    int n = m->n_states, M = m->n_modes;
    if (m->user_v) {
        m->user_v(q, m->user_prm, V);
        return;
    }
    for (int i = 0; i < n * n; ++i) {
        double v = m->v0[i];
        for (int j = 0; j < M; ++j) {
            v += q[j] * m->k[j * n * n + i];
            double qk = q[j];
            for (int k = 2; k <= m->degree; ++k) {
                qk *= q[j];
                v += qk * poly_entry(m, j, k, i);
            }
        }
        for (int pr = 0; pr < m->n_pairs; ++pr)
            v += q[m->pairs[2 * pr]] * q[m->pairs[2 * pr + 1]] * m->bpair[(size_t)pr * n * n + i];
        V[i] = v;
    }
}

/* dV/dq_j = K_j + sum_{k=2..D} k q_j^(k-1) A_jk + sum over the bilinear
 * terms that hold mode j of (the other mode's q) B_p, an N x N matrix.
 * q may be NULL for a linear model. */
static void mode_gradient(const or_model *m, int j, const double *q, double *Gj)
{
    int n = m->n_states;
    if (m->user_dv) {
        m->user_dv(j, q, m->user_prm, Gj);
        return;
    }
    const double qj = q ? q[j] : 0.0;
    for (int i = 0; i < n * n; ++i) {
        double g = m->k[(size_t)j * n * n + i];
        double qk = 1.0;
        for (int k = 2; k <= m->degree; ++k) {
            qk *= qj;
            g += k * qk * poly_entry(m, j, k, i);
        }
        for (int pr = 0; q && pr < m->n_pairs; ++pr) {
            const int pi = m->pairs[2 * pr], pj = m->pairs[2 * pr + 1];
            if (pi == j)
                g += q[pj] * m->bpair[(size_t)pr * n * n + i];
            if (pj == j)
                g += q[pi] * m->bpair[(size_t)pr * n * n + i];
        }
        Gj[i] = g;
    }
}

/* Adiabatic data at q: energies E (ascending) and gauge-fixed U. */
void or_adiabatic(const or_model *m, const double *q, const double *Uprev, double *E, double *U)
{
    double V[OR_MAXN * OR_MAXN];
    or_potential(m, q, V);
    or_jacobi_eigh(m->n_states, V, E, U);
    or_gauge(m->n_states, Uprev, U);
}

/* X = U^T A U for symmetric A (n x n). */
static void rotate_to_adiabatic(int n, const double *U, const double *Amat, double *X)
{
    double T[OR_MAXN * OR_MAXN];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int r = 0; r < n; ++r)
                s += Amat[i * n + r] * U[r * n + j];
            T[i * n + j] = s;
        }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int r = 0; r < n; ++r)
                s += U[r * n + i] * T[r * n + j];
            X[i * n + j] = s;
        }
}

/* Mean classical force on element (a,b):
 * F_j = -m_j w_j^2 q_j - [ (U^T dV/dq_j U)_aa + (U^T dV/dq_j U)_bb ] / 2
 * (without the first term for a supplied potential, whose V holds it),
 * i.e. (F_a + F_b)/2 with Hellmann-Feynman F_alpha (Eq. 1, last term). */
void or_mean_force(const or_model *m, const double *q, const double *U, int a, int b, double *F)
{
    int n = m->n_states;
    double G[OR_MAXN * OR_MAXN], Gj[OR_MAXN * OR_MAXN];
    for (int j = 0; j < m->n_modes; ++j) {
        mode_gradient(m, j, q, Gj);
        rotate_to_adiabatic(n, U, Gj, G);
        const double bath = m->user_v ? 0.0 : m->mass[j] * m->omega[j] * m->omega[j] * q[j];
        F[j] = -bath - 0.5 * (G[a * n + a] + G[b * n + b]);
    }
}

/* (P/M).d_ab for all pairs: D = U^T (sum_j v_j dV/dq_j) U, v.d_ab =
 * D_ab/(E_b - E_a) for a != b and 0 on the diagonal.  Output vd [N][N].
 * q may be NULL for a linear model (dV/dq_j = K_j does not depend on it). */
void or_velocity_nac(const or_model *m, const double *q, const double *p, const double *E, const double *U,
                     double *vd)
{
    int n = m->n_states;
    double Kv[OR_MAXN * OR_MAXN], D[OR_MAXN * OR_MAXN], Gj[OR_MAXN * OR_MAXN];
    for (int i = 0; i < n * n; ++i)
        Kv[i] = 0.0;
    for (int j = 0; j < m->n_modes; ++j) {
        mode_gradient(m, j, q, Gj);
        for (int i = 0; i < n * n; ++i)
            Kv[i] += (p[j] / m->mass[j]) * Gj[i];
    }
    rotate_to_adiabatic(n, U, Kv, D);
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b)
            vd[a * n + b] = (a == b) ? 0.0 : D[a * n + b] / (E[b] - E[a]);
}

/* Candidate moves out of element (a,b) in their fixed order: first (c,b)
 * for c != a with factor f = dt v.d_ac, then (a,c) for c != b with factor
 * f = dt v.d_bc.  These are the coefficients with which rho_ab feeds the
 * other elements through the coupling term of Eq. 1 over one step. */
int or_candidates(int n, const double *vd, double dt, int a, int b,
                  double *f, int32_t *ta, int32_t *tb)
{
    int nc = 0;
    for (int c = 0; c < n; ++c) {
        if (c == a) continue;
        f[nc] = dt * vd[a * n + c];
        ta[nc] = c; tb[nc] = b; ++nc;
    }
    for (int c = 0; c < n; ++c) {
        if (c == b) continue;
        f[nc] = dt * vd[b * n + c];
        ta[nc] = a; tb[nc] = c; ++nc;
    }
    return nc;
}

enum { OR_NORMALIZED = 0, OR_LINEAR = 1 };

/* One Monte Carlo transition.  Returns the chosen candidate (-1 = stay)
 * and updates (a, b, w).  *fallback is set when the linear rule cannot be
 * used (S >= 1) and the normalized rule was applied instead. */
int or_transition(int n, const double *vd, double dt, double u, int scheme,
                  int32_t *a, int32_t *b, double *w, int *fallback)
{
    double f[2 * OR_MAXN];
    int32_t ta[2 * OR_MAXN], tb[2 * OR_MAXN];
    int nc = or_candidates(n, vd, dt, *a, *b, f, ta, tb);
    double S = 0.0;
    for (int k = 0; k < nc; ++k)
        S += fabs(f[k]);
    int pick = -1;
    *fallback = 0;
    if (scheme == OR_LINEAR && S < 1.0) {
        double C = 0.0;
        for (int k = 0; k < nc; ++k) {
            C += fabs(f[k]);
            if (u < C) { pick = k; break; }
        }
        if (pick < 0) {
            *w = *w / (1.0 - S);
        } else {
            *w = *w * (f[pick] > 0.0 ? 1.0 : -1.0);
        }
    } else {
        if (scheme == OR_LINEAR)
            *fallback = 1;
        double t = u * (1.0 + S);
        if (!(t < 1.0)) {
            double C = 0.0;
            for (int k = 0; k < nc; ++k) {
                C += fabs(f[k]);
                if (t < 1.0 + C) { pick = k; break; }
            }
            if (pick < 0) /* rounding: take the last candidate with |f| > 0 */
                for (int k = nc - 1; k >= 0 && pick < 0; --k)
                    if (fabs(f[k]) > 0.0) pick = k;
        }
        *w = *w * (1.0 + S) * (pick < 0 ? 1.0 : (f[pick] > 0.0 ? 1.0 : -1.0));
    }
    if (pick >= 0) {
        *a = ta[pick];
        *b = tb[pick];
    }
    return pick;
}

/* ------------------------------------------------------------------ */
/* Observables (per walker).  slot layout [2][N][N][4]:                */
/*   basis 0: adiabatic rho_ab  <- W if (a,b) matches, else 0          */
/*   basis 1: diabatic  rho_ij  <- W U_ia U_jb                         */
/*   stat: Re, Im, Re^2, Im^2 with W = w (cos Phi - i sin Phi).        */
/* Non-finite walkers contribute nothing (they are counted instead).   */
/* ------------------------------------------------------------------ */
static void add_walker(int n, const double *U, int a, int b, double w, double phase, double *sums)
{
    if (!isfinite(w) || !isfinite(phase))
        return;
    double re = w * cos(phase), im = -w * sin(phase);
    double *ad = sums, *dia = sums + 4 * n * n;
    int s = a * n + b;
    ad[4 * s + 0] += re;
    ad[4 * s + 1] += im;
    ad[4 * s + 2] += re * re;
    ad[4 * s + 3] += im * im;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double cij = U[i * n + a] * U[j * n + b];
            double r = re * cij, m = im * cij;
            int t = i * n + j;
            dia[4 * t + 0] += r;
            dia[4 * t + 1] += m;
            dia[4 * t + 2] += r * r;
            dia[4 * t + 3] += m * m;
        }
}

/* ------------------------------------------------------------------ */
/* Initial sampling (Sec. II.A: partial Wigner transform; Wigner (q,p)). */
/* ------------------------------------------------------------------ */
enum { OR_INIT_DIABATIC = 0, OR_INIT_ADIABATIC = 1 };

/* Thermal Wigner widths of one harmonic mode:
 * var_q = hbar / (2 m w tanh(hbar w / 2kT)), var_p = hbar m w / (2 tanh(.)),
 * tanh -> 1 at kT = 0 (ground state). */
static void wigner_widths(double hbar, double mass, double omega, double kT, double *sq, double *sp)
{
    double th = (kT > 0.0) ? tanh(hbar * omega / (2.0 * kT)) : 1.0;
    *sq = sqrt(hbar / (2.0 * mass * omega * th));
    *sp = sqrt(hbar * mass * omega / (2.0 * th));
}

static void sample_one(const or_model *m, double kT, const double *q0, int init_state, int basis,
                       uint64_t seed, uint64_t gid,
                       double *q, double *p, double *w, double *phase, int32_t *a, int32_t *b, double *U)
{
    const double two_pi = 6.283185307179586476925286766559;
    int n = m->n_states;
    for (int j = 0; j < m->n_modes; ++j) {
        uint32_t x[4];
        philox_block(seed, gid, (uint32_t)j, 1u, x);
        double u1 = or_uniform52(x[0], x[1]);
        double u2 = or_uniform52(x[2], x[3]);
        double r = sqrt(-2.0 * log(u1));
        double zq = r * cos(two_pi * u2), zp = r * sin(two_pi * u2);
        double sq, sp;
        wigner_widths(m->hbar, m->mass[j], m->omega[j], kT, &sq, &sp);
        q[j] = q0[j] + sq * zq;
        p[j] = sp * zp;
    }
    double E[OR_MAXN];
    or_adiabatic(m, q, NULL, E, U);
    if (basis == OR_INIT_ADIABATIC) {
        *a = init_state; *b = init_state; *w = 1.0;
    } else {
        /* diabatic |k><k| seen in the adiabatic basis: rho_ab = U_ka U_kb.
         * Draw (a,b) with probability |U_ka U_kb| / Z, Z = (sum_a |U_ka|)^2,
         * and carry w = sgn(U_ka U_kb) Z (unbiased). */
        int k = init_state;
        double rowsum = 0.0;
        for (int c = 0; c < n; ++c)
            rowsum += fabs(U[k * n + c]);
        double Z = rowsum * rowsum;
        uint32_t x[4];
        philox_block(seed, gid, 0u, 2u, x);
        double t = or_uniform52(x[0], x[1]) * Z;
        int pa = -1, pb = -1, la = -1, lb = -1;
        double C = 0.0;
        for (int ia = 0; ia < n && pa < 0; ++ia)
            for (int ib = 0; ib < n; ++ib) {
                double wgt = fabs(U[k * n + ia] * U[k * n + ib]);
                if (wgt > 0.0) { la = ia; lb = ib; }
                C += wgt;
                if (t < C) { pa = ia; pb = ib; break; }
            }
        if (pa < 0) { pa = la; pb = lb; }
        double prod = U[k * n + pa] * U[k * n + pb];
        *a = pa; *b = pb;
        *w = (prod > 0.0 ? 1.0 : -1.0) * Z;
    }
    *phase = 0.0;
}

/* Sample n_traj walkers with global ids traj_offset .. traj_offset+n_traj-1.
 * State arrays are per walker (AoS): q,p [T][M], U [T][N][N].  sums0
 * ([2][N][N][4], accumulated, may be NULL) receives the t = 0 bin. */
void or_sample(const or_model *m, double kT, const double *q0, int init_state, int basis,
               uint64_t seed, int64_t traj_offset, int64_t n_traj,
               double *q, double *p, double *w, double *phase, int32_t *a, int32_t *b, double *U,
               double *sums0)
{
    int n = m->n_states, M = m->n_modes, nslot = 8 * n * n;
    int64_t n_chunks = (n_traj + OR_CHUNK - 1) / OR_CHUNK;
    double *part = sums0 ? (double *)calloc((size_t)(n_chunks > 0 ? n_chunks : 1) * nslot, sizeof(double)) : NULL;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < n_chunks; ++c) {
        int64_t lo = c * OR_CHUNK, hi = lo + OR_CHUNK < n_traj ? lo + OR_CHUNK : n_traj;
        for (int64_t t = lo; t < hi; ++t) {
            sample_one(m, kT, q0, init_state, basis, seed, (uint64_t)(traj_offset + t),
                       q + t * M, p + t * M, w + t, phase + t, a + t, b + t, U + t * n * n);
            if (part)
                add_walker(n, U + t * n * n, a[t], b[t], w[t], phase[t], part + c * nslot);
        }
    }
    if (part) {
        for (int64_t c = 0; c < n_chunks; ++c)
            for (int s = 0; s < nslot; ++s)
                sums0[s] += part[c * nslot + s];
        free(part);
    }
}

/* ------------------------------------------------------------------ */
/* Propagation: n_steps steps from global step step0.                  */
/* ------------------------------------------------------------------ */
enum { OR_FLAG_NONFINITE = 1u, OR_FLAG_DEGENERATE = 2u, OR_FLAG_FALLBACK = 8u };

static void propagate_one(const or_model *m, uint64_t gid, int64_t step0, int n_steps, double dt,
                          int cadence, uint64_t seed, int scheme,
                          double *q, double *p, double *w, double *phase, int32_t *a, int32_t *b,
                          double *U, int32_t n_out, double *sums, uint32_t *flag, int64_t *n_fb)
{
    int n = m->n_states, M = m->n_modes;
    double E[OR_MAXN], Un[OR_MAXN * OR_MAXN], vd[OR_MAXN * OR_MAXN];
    double F[OR_MAXM], qn[OR_MAXM];
    /* eigen-data at the current q, aligned to the stored frame */
    double Ucur[OR_MAXN * OR_MAXN];
    or_adiabatic(m, q, U, E, Ucur);
    memcpy(U, Ucur, sizeof(double) * n * n);

    for (int it = 0; it < n_steps; ++it) {
        int64_t step = step0 + it;
        /* 1. Monte Carlo transition at (q_n, p_n) */
        for (int i = 0; i + 1 < n; ++i)
            if (!(E[i + 1] - E[i] > 2.2250738585072014e-308))
                *flag |= OR_FLAG_DEGENERATE;
        or_velocity_nac(m, q, p, E, U, vd);
        uint32_t x[4];
        philox_block(seed, gid, (uint32_t)(step >> 2), 0u, x);
        double u = or_uniform24(x[step & 3]);
        int fb = 0;
        or_transition(n, vd, dt, u, scheme, a, b, w, &fb);
        if (fb) { *flag |= OR_FLAG_FALLBACK; ++*n_fb; }

        /* 2. velocity Verlet on the mean force of the (new) element */
        double dE0 = E[*a] - E[*b];
        or_mean_force(m, q, U, *a, *b, F);
        for (int j = 0; j < M; ++j)
            p[j] += 0.5 * dt * F[j];
        for (int j = 0; j < M; ++j)
            qn[j] = q[j] + dt * p[j] / m->mass[j];
        memcpy(q, qn, sizeof(double) * M);
        or_adiabatic(m, q, U, E, Un);
        memcpy(U, Un, sizeof(double) * n * n);
        or_mean_force(m, q, U, *a, *b, F);
        for (int j = 0; j < M; ++j)
            p[j] += 0.5 * dt * F[j];

        /* 3. phase: trapezoid of w_ab = (E_a - E_b)/hbar over the step */
        double dE1 = E[*a] - E[*b];
        *phase += 0.5 * dt * (dE0 + dE1) / m->hbar;

        if (!isfinite(*w) || !isfinite(*phase))
            *flag |= OR_FLAG_NONFINITE;

        /* 4. output bin */
        int64_t s1 = step + 1;
        if (s1 % cadence == 0) {
            int64_t o = s1 / cadence;
            if (o < n_out)
                add_walker(n, U, *a, *b, *w, *phase, sums + o * 8 * n * n);
        }
    }
}

int or_propagate(const or_model *m, int64_t n_traj, int64_t traj_offset, int64_t step0,
                 int n_steps, double dt, int cadence, uint64_t seed, int scheme,
                 double *q, double *p, double *w, double *phase, int32_t *a, int32_t *b, double *U,
                 int32_t n_out, double *sums, uint32_t *flags, int64_t *n_fallback)
{
    int n = m->n_states, M = m->n_modes, nslot = 8 * n * n;
    if (n < 2 || n > OR_MAXN || M < 1 || M > OR_MAXM || cadence < 1 || n_steps < 0 || m->n_pairs < 0)
        return 1;
    for (int pr = 0; pr < m->n_pairs; ++pr) {
        const int pi = m->pairs[2 * pr], pj = m->pairs[2 * pr + 1];
        if (pi < 0 || pj < 0 || pi >= M || pj >= M || pi == pj)
            return 1;
    }
    int64_t n_chunks = (n_traj + OR_CHUNK - 1) / OR_CHUNK;
    size_t per = (size_t)n_out * nslot;
    double *part = (double *)calloc((size_t)(n_chunks > 0 ? n_chunks : 1) * per, sizeof(double));
    int64_t *fb = (int64_t *)calloc((size_t)(n_chunks > 0 ? n_chunks : 1), sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < n_chunks; ++c) {
        int64_t lo = c * OR_CHUNK, hi = lo + OR_CHUNK < n_traj ? lo + OR_CHUNK : n_traj;
        for (int64_t t = lo; t < hi; ++t) {
            uint32_t fl = 0;
            propagate_one(m, (uint64_t)(traj_offset + t), step0, n_steps, dt, cadence, seed, scheme,
                          q + t * M, p + t * M, w + t, phase + t, a + t, b + t, U + t * n * n,
                          n_out, part + c * per, &fl, fb + c);
            if (flags)
                flags[t] |= fl;
        }
    }
    for (int64_t c = 0; c < n_chunks; ++c) {
        for (size_t s = 0; s < per; ++s)
            sums[s] += part[c * per + s];
        if (n_fallback)
            *n_fallback += fb[c];
    }
    free(part);
    free(fb);
    return 0;
}

/* Threads the OpenMP loops over walkers use. */
int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Ensemble averages from bin sums: out [n_out][2][N][N][4] =
 * (mean Re, mean Im, standard error Re, standard error Im), means over
 * n_traj walkers, SE = sqrt((S2 - S1^2/T) / (T (T-1))). */
void or_finalize(int n, int64_t n_traj, int32_t n_out, const double *sums, double *out)
{
    double T = (double)n_traj;
    for (int64_t i = 0; i < (int64_t)n_out * 2 * n * n; ++i) {
        const double *s = sums + 4 * i;
        double *o = out + 4 * i;
        o[0] = s[0] / T;
        o[1] = s[1] / T;
        double vr = (s[2] - s[0] * s[0] / T) / (T * (T - 1.0));
        double vi = (s[3] - s[1] * s[1] / T) / (T * (T - 1.0));
        o[2] = n_traj > 1 && vr > 0.0 ? sqrt(vr) : 0.0;
        o[3] = n_traj > 1 && vi > 0.0 ? sqrt(vi) : 0.0;
    }
}
