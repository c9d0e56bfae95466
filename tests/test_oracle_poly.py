"""Pins of the oracle for models with separable higher powers,
V(q) = V0 + sum_j [q_j K_j + sum_{k=2..D} q_j^k A_jk]: LAPACK eigenvalues
of V(q), forces and couplings against finite differences, the exact
discrete velocity-Verlet map of a diagonal model with state-dependent
frequencies (and its phase as the exact trapezoid sum over that orbit),
energy conservation of order dt^2 on a quartic surface, the all-branches
enumeration (independent numpy implementation), and exact reduction to the
linear model when the higher powers vanish."""
import numpy as np
import pytest
import scipy.linalg as sl

import workloads as W
from oracle.branches import Enumerator


def _V(model, q):
    v = model.v0 + np.tensordot(q, model.k, axes=(0, 0))
    for k in range(2, model.degree + 1):
        v = v + np.tensordot(q ** k, model.poly[:, k - 2], axes=(0, 0))
    return v


@pytest.mark.parametrize("wl", [W.pyrazine_qvc(), W.random_poly(0, n_states=2, n_modes=3, degree=2),
                                W.random_poly(1, n_states=3, n_modes=4, degree=3),
                                W.random_poly(2, n_states=4, n_modes=3, degree=4)])
def test_poly_force_and_nac_vs_finite_differences(oracle_lib, wl):
    oc = oracle_lib
    model = wl.model
    m = oc.Model(model)
    n, M = model.n_states, model.n_modes
    rng = np.random.default_rng(5)
    h = 1e-6
    for _ in range(8):
        q = wl.init.q0 + 0.8 * rng.normal(size=M)
        p = rng.normal(size=M)
        E, U = oc.adiabatic(m, q)
        np.testing.assert_allclose(E, sl.eigh(_V(model, q), eigvals_only=True), atol=1e-12)
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
                np.testing.assert_allclose(F, Fr, atol=5e-8 * (1 + np.abs(Fr).max()))
        vd = oc.velocity_nac(m, p, E, U, q=q)
        vd_fd = np.einsum("j,jab->ab", p / model.mass, np.einsum("ia,jib->jab", U, dU))
        np.fill_diagonal(vd_fd, 0.0)
        scale = np.abs(vd).max() + 1e-3
        np.testing.assert_allclose(vd, vd_fd, atol=1e-6 * scale)
    with pytest.raises(ValueError):
        oc.velocity_nac(m, p, E, U)  # q is required


def _diag_qvc():
    """Two states, three modes, everything diagonal: no coupling, each
    element moves on an effective harmonic surface."""
    M = 3
    kap = np.array([[0.3, -0.2], [-0.1, 0.25], [0.05, 0.0]])  # kappa_j per state
    g = np.array([[0.1, -0.15], [0.0, 0.2], [-0.05, 0.05]])   # q^2 coefficient per state
    k = np.stack([np.diag(kap[j]) for j in range(M)])
    poly = np.stack([np.diag(g[j]) for j in range(M)])[:, None]
    model = W.LVCModel(name="diag_qvc", mass=[1.0, 0.6, 2.0], omega=[1.0, 1.4, 0.7], v0=np.diag([-4.0, 4.0]),
                       k=k, poly=poly)
    init = W.InitSpec(kT=0.3, q0=np.zeros(M), state=0)
    return W.Workload(model, init, W.RunSpec(400, 200, 0.04, 10, 21)), kap, g


def _verlet_matrix(m, k_eff, dt):
    # one velocity-Verlet step of x'' = -(k_eff/m) x on (x, p)
    w2 = k_eff / m
    return np.array([[1 - 0.5 * (w2 * dt * dt), dt / m],
                     [-k_eff * dt * (1 - 0.25 * w2 * dt * dt), 1 - 0.5 * w2 * dt * dt]])


def test_diagonal_qvc_exact_verlet_map_and_phase(oracle_lib):
    oc = oracle_lib
    wl, kap, g = _diag_qvc()
    model, r = wl.model, wl.run
    st0, _ = oc.sample(model, wl.init, r.seed, r.n_traj)
    # put half the walkers on the coherence (0, 1) and some on (1, 1)
    st0.a[: r.n_traj // 2] = 0
    st0.b[: r.n_traj // 2] = 1
    st0.a[r.n_traj // 2:] = 1
    st0.b[r.n_traj // 2:] = 1
    st0.w[:] = 1.0
    st0.U[:] = np.eye(2)
    st = st0.copy()
    oc.propagate(model, st, r.dt, r.n_steps, r.cadence, r.seed, r.n_out)
    assert np.array_equal(st.a, st0.a) and np.array_equal(st.b, st0.b) and np.all(st.w == 1.0)
    a, b = st0.a, st0.b
    dV0 = model.v0[a, a] - model.v0[b, b]
    phase = np.zeros(r.n_traj)
    gap = np.zeros(r.n_traj)
    for j in range(model.n_modes):
        m = model.mass[j]
        k_eff = m * model.omega[j] ** 2 + g[j, a] + g[j, b]           # per walker
        qs = -(kap[j, a] + kap[j, b]) / (2 * k_eff)                     # centre of the mean-force well
        qj = np.zeros((r.n_steps + 1, r.n_traj))
        x, pj = st0.q[:, j] - qs, st0.p[:, j].copy()
        qj[0] = st0.q[:, j]
        for i in range(r.n_traj):
            Mv = _verlet_matrix(m, k_eff[i], r.dt)
            y = np.array([x[i], pj[i]])
            for s in range(r.n_steps):
                y = Mv @ y
                qj[s + 1, i] = y[0] + qs[i]
            x[i], pj[i] = y
        np.testing.assert_allclose(st.q[:, j], x + qs, rtol=1e-10, atol=1e-11)
        np.testing.assert_allclose(st.p[:, j], pj, rtol=1e-10, atol=1e-11)
        dE = (kap[j, a] - kap[j, b]) * qj + (g[j, a] - g[j, b]) * qj ** 2
        gap += np.abs(dE).max(axis=0)
        phase += r.dt * (0.5 * dE[0] + dE[1:-1].sum(axis=0) + 0.5 * dE[-1])
    assert np.all(gap < 8.0)  # the diabatic order never changes along the orbits: adiabatic labels hold
    phase += dV0 * r.n_steps * r.dt
    np.testing.assert_allclose(st.phase, phase, rtol=1e-11, atol=1e-11)


def test_quartic_energy_second_order(oracle_lib):
    """A single adiabatic surface with quartic and cubic terms: velocity
    Verlet keeps the energy within O(dt^2)."""
    oc = oracle_lib
    M = 2
    k = np.zeros((M, 2, 2))
    poly = np.zeros((M, 3, 2, 2))
    poly[0, 1] = np.diag([0.05, 0.0])
    poly[0, 2] = np.diag([0.2, 0.2])
    poly[1, 2] = np.diag([0.1, 0.3])
    model = W.LVCModel(name="quartic", mass=[1.0, 2.0], omega=[1.0, 0.5], v0=np.diag([-1.0, 1.0]), k=k, poly=poly)
    init = W.InitSpec(kT=0.5, q0=np.zeros(M), state=0)
    mm = oc.Model(model)
    st0, _ = oc.sample(mm, init, 3, 200)
    assert np.all(st0.a == 0) and np.all(st0.b == 0)

    def energy(st):
        e = 0.5 * st.p ** 2 / model.mass + 0.5 * model.mass * model.omega ** 2 * st.q ** 2
        e = e.sum(axis=1) + model.v0[0, 0]
        for kk in range(2, 5):
            e += (st.q ** kk * poly[:, kk - 2, 0, 0]).sum(axis=1)
        return e

    drift = []
    for dt, n in ((0.05, 400), (0.025, 800)):
        st = st0.copy()
        e0 = energy(st)
        worst = 0.0
        for _ in range(8):
            oc.propagate(mm, st, dt, n // 8, n // 8, 3, 9)
            worst = max(worst, float(np.abs(energy(st) - e0).max()))
        drift.append(worst)
    print("energy drift", drift)
    assert drift[0] < 0.05  # energies are O(1)
    assert 3.0 < drift[0] / drift[1] < 5.0, drift


def test_zero_higher_powers_reduce_to_linear(oracle_lib):
    oc = oracle_lib
    base = W.pyrazine_ci(n_traj=300, n_steps=60, cadence=10)
    lin = base.model
    zero = W.LVCModel(name="zero_poly", mass=lin.mass, omega=lin.omega, v0=lin.v0, k=lin.k, hbar=lin.hbar,
                      poly=np.zeros((3, 3, 2, 2)))
    out_l, st_l, _ = oc.run(base)
    out_z, st_z, _ = oc.run(W.Workload(zero, base.init, base.run))
    assert np.array_equal(out_l, out_z)
    for key in ("q", "p", "w", "phase", "U"):
        assert np.array_equal(getattr(st_l, key), getattr(st_z, key)), key


def test_poly_all_branches_enumeration(oracle_lib):
    oc = oracle_lib
    wl = W.random_poly(3, n_states=3, n_modes=1, degree=4)
    mm = oc.Model(wl.model)
    q0, p0 = np.array([0.4]), np.array([1.4])
    _, U0 = oc.adiabatic(mm, q0)
    k, dt, T = 3, 0.2, 200_000
    ex = Enumerator(wl.model).expectation(q0, p0, 2, 2, U0, dt, k)
    st = oc.State(T, 3, 1)
    st.q[:] = q0
    st.p[:] = p0
    st.a[:] = 2
    st.b[:] = 2
    st.w[:] = 1.0
    st.U[:] = U0
    sums, _ = oc.propagate(mm, st, dt, k, 1, 23, k + 1)
    out = oc.finalize(sums, T)
    mc = out[1:, ..., 0] + 1j * out[1:, ..., 1]
    grain = 10 * np.abs(st.w).max() / T
    assert np.abs(ex[..., 0, :, :]).max() > 0.05  # the coupling moves weight off (2, 2)
    assert np.all(np.abs(mc.real - ex.real) <= 4.5 * out[1:, ..., 2] + grain)
    assert np.all(np.abs(mc.imag - ex.imag) <= 4.5 * out[1:, ..., 3] + grain)
