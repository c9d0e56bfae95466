"""Phase-space grid solution of Eq. 1 for one mode and two states.

Test infrastructure, independent of the trajectory oracle: it solves the
partial differential equation of Eq. 1 on a (q, p) grid instead of sampling
it, so it pins the whole estimator (sampling, transitions, classical flow,
phase and averaging) rather than one implementation of it.

Splitting (Strang): per step h

    A(h/2)  advection of each element rho_ab along the mean-force flow
            dq/dt = p/m, dp/dt = (F_a + F_b)/2 with the phase factor
            exp(-i int w_ab dt) along the characteristic (semi-Lagrangian,
            bicubic Lagrange interpolation at the foot points);
    B(h)    coupling term d rho/dt = -[v.d, rho] at every grid point, solved
            exactly: for two states v.d = x [[0,1],[-1,0]] and
            rho <- R rho R^T with R = exp(-h v.d), a plane rotation;
    A(h/2).

Adiabatic basis: numpy eigenvectors with U_kk > 0, which is smooth in q
for models whose off-diagonal coupling never vanishes (the one-mode
spin-boson model).  Couplings d_01 come from central differences of these
eigenvectors.  Initial condition: thermal Wigner Gaussian times the
diabatic projector |k><k| seen in the adiabatic basis, rho_ab = U_ka U_kb.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp


def _eig_grid(model, q):
    Vg = model.v0[None, :, :] + q[:, None, None] * model.k[0][None, :, :]
    E, U = np.linalg.eigh(Vg)
    for kk in range(2):
        s = np.where(U[:, kk, kk] < 0.0, -1.0, 1.0)
        U[:, :, kk] *= s[:, None]
    return E, U


def _cubic_weights(t):
    """Lagrange cubic weights on nodes -1, 0, 1, 2 for offset t in [0, 1)."""
    return np.stack([
        -t * (t - 1) * (t - 2) / 6.0,
        (t + 1) * (t - 1) * (t - 2) / 2.0,
        -(t + 1) * t * (t - 2) / 2.0,
        (t + 1) * t * (t - 1) / 6.0,
    ], axis=-1)


def _interp_matrix(qf, pf, qg, pg):
    """Sparse matrix evaluating a grid function at foot points (qf, pf)
    (bicubic Lagrange, zero outside the grid)."""
    nq, npp = len(qg), len(pg)
    dq, dp = qg[1] - qg[0], pg[1] - pg[0]
    xq = (qf - qg[0]) / dq
    xp = (pf - pg[0]) / dp
    iq = np.floor(xq).astype(np.int64)
    ip = np.floor(xp).astype(np.int64)
    wq = _cubic_weights(xq - iq)
    wp = _cubic_weights(xp - ip)
    rows, cols, vals = [], [], []
    r = np.arange(qf.size)
    for a in range(4):
        for b in range(4):
            jq = iq - 1 + a
            jp = ip - 1 + b
            ok = (jq >= 0) & (jq < nq) & (jp >= 0) & (jp < npp)
            rows.append(r[ok])
            cols.append(jq[ok] * npp + jp[ok])
            vals.append(wq[ok, a] * wp[ok, b])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(qf.size, nq * npp))


class GridSolver:
    def __init__(self, model, init, q_range=(-6.0, 5.0), p_range=(-5.5, 5.5),
                 nq=221, npp=221, h=0.01, fd=1e-5, substeps=4):
        assert model.n_states == 2 and model.n_modes == 1
        self.m = model
        self.qg = np.linspace(q_range[0], q_range[1], nq)
        self.pg = np.linspace(p_range[0], p_range[1], npp)
        self.dA = (self.qg[1] - self.qg[0]) * (self.pg[1] - self.pg[0])
        Q, P = np.meshgrid(self.qg, self.pg, indexing="ij")
        self.Q, self.P = Q.ravel(), P.ravel()
        self.h = h
        mass, om, hb = model.mass[0], model.omega[0], model.hbar
        self.mass = mass

        def surfaces(q):
            E, _ = _eig_grid(model, np.atleast_1d(q))
            return E

        def dEdq(q):
            return (surfaces(q + fd) - surfaces(q - fd)) / (2 * fd)

        # foot points and phase factors for a full step h (the half steps at
        # the two ends are handled separately)
        def flow(a, b, tau):
            q, p = self.Q.copy(), self.P.copy()
            hs = -tau / substeps  # integrate backwards in time

            def rhs(q, p):
                g = dEdq(q)
                F = -mass * om * om * q - 0.5 * (g[:, a] + g[:, b])
                return p / mass, F

            def wab(q):
                E = surfaces(q)
                return (E[:, a] - E[:, b]) / hb

            phase = np.zeros_like(q)
            for _ in range(substeps):  # RK4 with Simpson phase
                k1q, k1p = rhs(q, p)
                k2q, k2p = rhs(q + 0.5 * hs * k1q, p + 0.5 * hs * k1p)
                k3q, k3p = rhs(q + 0.5 * hs * k2q, p + 0.5 * hs * k2p)
                k4q, k4p = rhs(q + hs * k3q, p + hs * k3p)
                qn = q + hs / 6 * (k1q + 2 * k2q + 2 * k3q + k4q)
                pn = p + hs / 6 * (k1p + 2 * k2p + 2 * k3p + k4p)
                phase += (abs(hs) / 6.0) * (wab(q) + 4 * wab(0.5 * (q + qn)) + wab(qn))
                q, p = qn, pn
            return _interp_matrix(q, p, self.qg, self.pg), np.exp(-1j * phase)

        self.elements = [(0, 0), (0, 1), (1, 0), (1, 1)]
        self.full = {}
        self.half = {}
        for (a, b) in self.elements:
            self.full[(a, b)] = flow(a, b, h)
            self.half[(a, b)] = flow(a, b, 0.5 * h)

        # coupling rotation per grid point: x = v.d_01
        _, U = _eig_grid(model, self.Q)
        _, Up = _eig_grid(model, self.Q + fd)
        _, Um = _eig_grid(model, self.Q - fd)
        d01 = np.einsum("ni,ni->n", U[:, :, 0], (Up[:, :, 1] - Um[:, :, 1]) / (2 * fd))
        x = (self.P / mass) * d01
        self.c, self.s = np.cos(h * x), np.sin(h * x)
        self.U = U

        # initial condition
        kT, q0, k = init.kT, float(init.q0[0]), init.state
        th = math.tanh(hb * om / (2 * kT)) if kT > 0 else 1.0
        vq = hb / (2 * mass * om * th)
        vp = hb * mass * om / (2 * th)
        wig = np.exp(-(self.Q - q0) ** 2 / (2 * vq) - self.P ** 2 / (2 * vp)) / (2 * math.pi * math.sqrt(vq * vp))
        self.rho = {(a, b): (wig * U[:, k, a] * U[:, k, b]).astype(complex) for (a, b) in self.elements}
        self.t = 0.0

    def _advect(self, table):
        for e in self.elements:
            Mx, ph = table[e]
            self.rho[e] = (Mx @ self.rho[e]) * ph

    def _couple(self):
        # rho <- R rho R^T with R = exp(-h x J), J = [[0,1],[-1,0]]:
        # R = [[c, -s], [s, c]]
        c, s = self.c, self.s
        r00, r01, r10, r11 = (self.rho[e] for e in self.elements)
        # T = R rho
        t00 = c * r00 - s * r10
        t01 = c * r01 - s * r11
        t10 = s * r00 + c * r10
        t11 = s * r01 + c * r11
        # rho' = T R^T, R^T = [[c, s], [-s, c]]
        self.rho[(0, 0)] = t00 * c - t01 * s
        self.rho[(0, 1)] = t00 * s + t01 * c
        self.rho[(1, 0)] = t10 * c - t11 * s
        self.rho[(1, 1)] = t10 * s + t11 * c

    def run(self, t_out):
        """Observables at the (increasing) times t_out: array [len, 2, 2, 2]
        complex, basis 0 adiabatic, 1 diabatic."""
        res = []
        n_total = int(round(max(t_out) / self.h))
        marks = {int(round(t / self.h)): i for i, t in enumerate(t_out)}
        out = [None] * len(t_out)
        if 0 in marks:
            out[marks[0]] = self.observables()
        self._advect(self.half)
        for n in range(1, n_total + 1):
            self._couple()
            if n in marks:
                saved = dict(self.rho)
                self._advect(self.half)
                out[marks[n]] = self.observables()
                self.rho = saved
            if n < n_total:
                self._advect(self.full)
        return np.array(out)

    def observables(self):
        ad = np.zeros((2, 2), complex)
        dia = np.zeros((2, 2), complex)
        U = self.U
        for (a, b) in self.elements:
            r = self.rho[(a, b)]
            ad[a, b] = r.sum() * self.dA
            for i in range(2):
                for j in range(2):
                    dia[i, j] += (r * U[:, i, a] * U[:, j, b]).sum() * self.dA
        return np.stack([ad, dia])
