"""Pins of the oracle's adiabatic quantities (Sec. II.A: w_ab, d_ab, F_a).

* eigenvalues/eigenvectors vs LAPACK (scipy.linalg.eigh);
* Hellmann-Feynman mean force vs central differences of the surfaces;
* P/M . d_ab vs central differences of the gauge-fixed eigenvectors;
* two-state closed forms: E = Vbar +- r, r^2 = delta^2 + c^2, and for the
  spin-boson coupling v.d_01 = -+ v g Delta / (2 r^2);
* sign convention: U_kk > 0 without a previous frame, continuity with one.
"""
import numpy as np
import pytest
import scipy.linalg as sl

import workloads as W


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 7, 8])
def test_jacobi_vs_lapack(oracle_lib, n):
    oc = oracle_lib
    rng = np.random.default_rng(n)
    for t in range(300):
        A = rng.normal(size=(n, n))
        A = A + A.T
        if t % 10 == 0:  # near-degenerate spectra
            Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
            ev = np.sort(rng.normal(size=n))
            ev[1] = ev[0] + 1e-9
            A = Q @ np.diag(ev) @ Q.T
            A = 0.5 * (A + A.T)
        E, U = oc.jacobi_eigh(A)
        E2 = sl.eigh(A, eigvals_only=True)
        assert np.all(np.diff(E) >= 0)
        np.testing.assert_allclose(E, E2, rtol=0, atol=1e-13 * max(1.0, np.abs(E2).max()))
        np.testing.assert_allclose(U @ np.diag(E) @ U.T, A, atol=2e-13 * max(1.0, np.abs(A).max()))
        np.testing.assert_allclose(U.T @ U, np.eye(n), atol=1e-13)


def test_jacobi_diagonal_and_permuted(oracle_lib):
    oc = oracle_lib
    E, U = oc.jacobi_eigh(np.diag([3.0, -1.0, 2.0]))
    assert E.tolist() == [-1.0, 2.0, 3.0]
    assert np.array_equal(np.abs(U), np.array([[0, 0, 1], [1, 0, 0], [0, 1, 0]], float))


def test_gauge_conventions(oracle_lib):
    oc = oracle_lib
    m = oc.Model(W.pyrazine_ci().model)
    rng = np.random.default_rng(5)
    for _ in range(100):
        q = rng.normal(size=3)
        E, U = oc.adiabatic(m, q)
        assert np.all(np.diag(U) > 0)
        # a frame with flipped columns is followed by continuity
        Uprev = U * np.array([-1.0, 1.0])
        E2, U2 = oc.adiabatic(m, q + 1e-3, Uprev)
        assert U2[:, 0] @ Uprev[:, 0] > 0 and U2[:, 1] @ Uprev[:, 1] > 0


@pytest.mark.parametrize("wl", [W.pyrazine_ci(), W.spin_boson_ohmic(), W.random_lvc(3, n_states=3, n_modes=4),
                                W.random_lvc(7, n_states=4, n_modes=5), W.random_lvc(8, n_states=6, n_modes=4),
                                W.random_lvc(9, n_states=8, n_modes=3)])
def test_force_and_nac_vs_finite_differences(oracle_lib, wl):
    oc = oracle_lib
    model = wl.model
    m = oc.Model(model)
    n, M = model.n_states, model.n_modes
    rng = np.random.default_rng(11)
    h = 1e-6
    for _ in range(10):
        q = wl.init.q0 + 0.7 * rng.normal(size=M)
        p = rng.normal(size=M)
        E, U = oc.adiabatic(m, q)
        # eigenvalues vs LAPACK on the same V(q)
        V = model.v0 + np.tensordot(q, model.k, axes=(0, 0))
        np.testing.assert_allclose(E, sl.eigh(V, eigvals_only=True), atol=1e-13)
        dE = np.zeros((M, n))
        dU = np.zeros((M, n, n))
        for j in range(M):
            e = np.zeros(M)
            e[j] = h
            Ep, Up = oc.adiabatic(m, q + e, U)
            Em, Um = oc.adiabatic(m, q - e, U)
            dE[j] = (Ep - Em) / (2 * h)
            dU[j] = (Up - Um) / (2 * h)
        for a in range(n):
            for b in range(n):
                F = oc.mean_force(m, q, U, a, b)
                Fr = -model.mass * model.omega ** 2 * q - 0.5 * (dE[:, a] + dE[:, b])
                np.testing.assert_allclose(F, Fr, atol=2e-8)
        vd = oc.velocity_nac(m, p, E, U)
        vd_fd = np.einsum("j,jab->ab", p / model.mass, np.einsum("ia,jib->jab", U, dU))
        np.fill_diagonal(vd_fd, 0.0)
        scale = np.abs(vd).max() + 1e-3
        np.testing.assert_allclose(vd, vd_fd, atol=1e-6 * scale)
        np.testing.assert_allclose(vd, -vd.T, atol=1e-14 * scale)


def test_two_state_closed_forms(oracle_lib):
    oc = oracle_lib
    wl = W.spin_boson_1mode()
    m = oc.Model(wl.model)
    eps, delta, g = 0.5, 0.2, 0.5
    for q in np.linspace(-4, 3, 29):
        E, U = oc.adiabatic(m, [q])
        dl = eps + g * q
        r = np.hypot(dl, delta)
        np.testing.assert_allclose(E, [-r, r], atol=1e-14)
        vd = oc.velocity_nac(m, [1.3], E, U)
        # |v.d_01| = v g Delta / (2 r^2); with U_kk > 0 the sign is +
        np.testing.assert_allclose(vd[0, 1], 1.3 * g * delta / (2 * r * r), rtol=1e-12)
