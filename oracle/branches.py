"""Exact expectation of the Monte Carlo estimator by enumerating branches.

Test infrastructure (independent of ``qcl_oracle.c``: numpy eigensolver,
finite-difference couplings and forces, coupling term written as the
matrix commutator of Eq. 1).

Over one step of length dt the coupling term of Eq. 1 maps a walker that
carries W on element (a,b) to W (1 + dt L) E_ab with

    L E_ab = -(v.d E_ab - E_ab v.d),   E_ab = unit matrix at (a,b),

so the exact expectation over all Monte Carlo choices, for fixed initial
(q, p), is the sum over every path of elements of the product of the
matrix entries of (1 + dt L) along the path, each path carrying its own
classical trajectory (velocity Verlet on the mean force of its current
element) and phase (trapezoid of w_ab).  The Monte Carlo transition rule
samples exactly this sum, so its mean over many random streams must agree
with the enumeration within the statistical error.

The step order (coupling at (q_n, p_n), then Verlet, then phase) is the
same reading the propagator uses.
"""
from __future__ import annotations

import numpy as np


class Enumerator:
    def __init__(self, model, fd_h: float = 1e-5):
        self.m = model
        self.n = model.n_states
        self.M = model.n_modes
        self.h = fd_h

    # -- electronic structure (numpy eigh + sign conventions) -------------
    def V(self, q):
        """V0 + sum_j q_j K_j (+ sum_j sum_k q_j^k A_jk for models with higher
        powers, + sum_p q_i q_j B_p for cross-mode bilinear terms)."""
        v = self.m.v0 + np.tensordot(q, self.m.k, axes=(0, 0))
        poly = getattr(self.m, "poly", None)
        if poly is not None:
            for k in range(2, poly.shape[1] + 2):
                v = v + np.tensordot(np.asarray(q) ** k, poly[:, k - 2], axes=(0, 0))
        for i, j, B in getattr(self.m, "bilinear", None) or []:
            v = v + q[i] * q[j] * np.asarray(B)
        return v

    def eig(self, q, Uprev=None):
        E, U = np.linalg.eigh(self.V(q))
        U = U.copy()
        for k in range(self.n):
            if Uprev is not None:
                if float(Uprev[:, k] @ U[:, k]) < 0.0:
                    U[:, k] = -U[:, k]
            else:
                lead = U[k, k] if U[k, k] != 0.0 else U[np.nonzero(U[:, k])[0][0], k]
                if lead < 0.0:
                    U[:, k] = -U[:, k]
        return E, U

    def vd(self, q, p, U):
        """v.d_ab = sum_j (p_j/m_j) <u_a | d u_b / d q_j> by central differences."""
        out = np.zeros((self.n, self.n))
        for j in range(self.M):
            e = np.zeros(self.M)
            e[j] = self.h
            _, Up = self.eig(q + e, U)
            _, Um = self.eig(q - e, U)
            out += (p[j] / self.m.mass[j]) * (U.T @ (Up - Um)) / (2 * self.h)
        np.fill_diagonal(out, 0.0)
        return out

    def force(self, q, a, b):
        """-(m w^2 q) - (dE_a/dq + dE_b/dq)/2 by central differences."""
        g = np.zeros(self.M)
        for j in range(self.M):
            e = np.zeros(self.M)
            e[j] = self.h
            Ep = np.linalg.eigvalsh(self.V(q + e))
            Em = np.linalg.eigvalsh(self.V(q - e))
            g[j] = 0.5 * ((Ep[a] - Em[a]) + (Ep[b] - Em[b])) / (2 * self.h)
        return -self.m.mass * self.m.omega ** 2 * q - g

    # -- enumeration -------------------------------------------------------
    def expectation(self, q0, p0, a0, b0, U0, dt, n_steps, w0=1.0):
        """Exact expectation of the per-step observables [n_steps, 2, N, N]
        (complex; basis 0 adiabatic, 1 diabatic) after steps 1..n_steps."""
        n = self.n
        out = np.zeros((n_steps, 2, n, n), complex)

        def rec(step, q, p, a, b, W, U):
            if step == n_steps:
                return
            vd = self.vd(q, p, U)
            Eab = np.zeros((n, n))
            Eab[a, b] = 1.0
            T = Eab - dt * (vd @ Eab - Eab @ vd)
            E0, _ = self.eig(q, U)
            for (i, j) in zip(*np.nonzero(T)):
                fac = T[i, j]
                pn = p + 0.5 * dt * self.force(q, i, j)
                qn = q + dt * pn / self.m.mass
                E1, Un = self.eig(qn, U)
                pn = pn + 0.5 * dt * self.force(qn, i, j)
                dphi = 0.5 * dt * ((E0[i] - E0[j]) + (E1[i] - E1[j])) / self.m.hbar
                Wn = W * fac * np.exp(-1j * dphi)
                out[step, 0, i, j] += Wn
                out[step, 1] += Wn * np.outer(Un[:, i], Un[:, j])
                rec(step + 1, qn, pn, i, j, Wn, Un)

        rec(0, np.asarray(q0, float), np.asarray(p0, float), int(a0), int(b0), complex(w0),
            np.asarray(U0, float))
        return out
