"""Pins of the oracle's propagation (Eq. 1 realised by walkers).

* zero coupling: no transitions, populations exactly constant, coherence
  phase equal to the closed form of the discrete trapezoid over the exact
  discrete Verlet orbit, O(dt^2) to the continuous integral, and the
  ensemble coherence equal to the Gaussian characteristic function;
* uncoupled harmonic: (q, p) equal the exact discrete velocity-Verlet map
  (2x2 matrix power) and the continuous orbit to O(dt^2);
* per-step weight invariant |w'| = |w| (1 + S) with S from
  finite-difference couplings;
* one-step transition expectation exactly (1 + dt L) on the element;
* all-branches enumeration (deterministic "spawn everything" limit) equals
  the Monte Carlo mean within the statistical error, both transition rules;
* the phase-space grid solution of Eq. 1 (tests/golden) equals the Monte
  Carlo populations and coherences within the statistical error;
* the bias against that grid solution is first order in dt;
* trace and Hermiticity in expectation.
"""
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle.branches import Enumerator

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _grid_fixture():
    with open(os.path.join(GOLDEN, "grid_spin_boson_1mode.json")) as f:
        d = json.load(f)
    return np.array(d["t"]), np.array(d["rho_re"]) + 1j * np.array(d["rho_im"])


# ----------------------------------------------------------------- zero coupling

def _zero_coupling_phase_coefficients(model, t, hbar=1.0):
    """Phi(t) = A + sum_j (B_j q0_j + C_j p0_j) for element (0,1) on a
    diagonal LVC model: continuous harmonic orbit on the mean surface."""
    dv = model.v0[0, 0] - model.v0[1, 1]
    dk = model.k[:, 0, 0] - model.k[:, 1, 1]
    fbar = 0.5 * (model.k[:, 0, 0] + model.k[:, 1, 1])
    m, w = model.mass, model.omega
    qbar = -fbar / (m * w ** 2)
    A = (dv * t + np.sum(dk * qbar * (t - np.sin(w * t) / w))) / hbar
    B = dk * np.sin(w * t) / (w * hbar)
    C = dk * (1 - np.cos(w * t)) / (m * w ** 2 * hbar)
    return A, B, C


def _verlet_matrix(m, w, dt):
    c = 1 - 0.5 * dt * dt * w * w
    return np.array([[c, dt / m], [-m * w * w * dt * (1 - 0.25 * dt * dt * w * w), c]])


def test_zero_coupling_populations_exact(oracle_lib):
    oc = oracle_lib
    wl = W.zero_coupling()
    r = wl.run
    out, st, sums = oc.run(wl)
    st0, _ = oc.sample(wl.model, wl.init, r.seed, r.n_traj)
    assert np.array_equal(st.a, st0.a) and np.array_equal(st.b, st0.b)
    assert np.array_equal(st.w, st0.w)
    for o in range(1, r.n_out):
        assert np.array_equal(sums[o, 0, :, :, 0], sums[0, 0, :, :, 0])
    assert np.all(st.flags == 0)


def test_zero_coupling_phase_discrete_and_continuous(oracle_lib):
    oc = oracle_lib
    wl = W.zero_coupling()
    model = wl.model
    T = 50
    st, _ = oc.sample(model, wl.init, 3, T)
    st.a[:] = 0
    st.b[:] = 1
    st.w[:] = 1.0
    q0, p0 = st.q.copy(), st.p.copy()
    n_steps, dt = 400, 0.025
    oc.propagate(model, st, dt, n_steps, n_steps, 3, 2)
    # exact discrete orbit on the mean force -m w^2 q - fbar
    fbar = 0.5 * (model.k[:, 0, 0] + model.k[:, 1, 1])
    dk = model.k[:, 0, 0] - model.k[:, 1, 1]
    dv = model.v0[0, 0] - model.v0[1, 1]
    for t in range(T):
        phi = 0.0
        qs = []
        for j in range(model.n_modes):
            m, w = model.mass[j], model.omega[j]
            qbar = -fbar[j] / (m * w * w)
            Mx = _verlet_matrix(m, w, dt)
            x = np.array([q0[t, j] - qbar, p0[t, j]])
            traj = [x]
            for _ in range(n_steps):
                traj.append(Mx @ traj[-1])
            traj = np.array(traj)
            qs.append(traj[:, 0] + qbar)
            np.testing.assert_allclose(st.q[t, j], qs[-1][-1], rtol=1e-11, atol=1e-12)
            np.testing.assert_allclose(st.p[t, j], traj[-1, 1], rtol=1e-11, atol=1e-12)
        qs = np.array(qs)  # [M, n+1]
        dE = dv + dk @ qs
        phi_discrete = 0.5 * dt * np.sum(dE[:-1] + dE[1:])
        np.testing.assert_allclose(st.phase[t], phi_discrete, rtol=1e-12, atol=1e-12)
        A, B, C = _zero_coupling_phase_coefficients(model, n_steps * dt)
        phi_cont = A + B @ q0[t] + C @ p0[t]
        assert abs(st.phase[t] - phi_cont) < 0.05 * dt * dt * n_steps * dt + 1e-9
    assert np.all(st.a == 0) and np.all(st.b == 1) and np.all(st.w == 1.0)


def test_zero_coupling_phase_second_order(oracle_lib):
    oc = oracle_lib
    wl = W.zero_coupling()
    model = wl.model
    st0, _ = oc.sample(model, wl.init, 8, 20)
    st0.a[:] = 0
    st0.b[:] = 1
    tf = 6.0
    A, B, C = _zero_coupling_phase_coefficients(model, tf)
    exact = A + st0.q @ B + st0.p @ C
    errs = []
    for dt in (0.1, 0.05, 0.025):
        st = st0.copy()
        n = int(round(tf / dt))
        oc.propagate(model, st, dt, n, n, 8, 2)
        errs.append(np.max(np.abs(st.phase - exact)))
    assert 3.3 < errs[0] / errs[1] < 4.7 and 3.3 < errs[1] / errs[2] < 4.7, errs


def test_zero_coupling_gaussian_characteristic_function(oracle_lib):
    oc = oracle_lib
    wl = W.zero_coupling(n_traj=200_000, n_steps=160, dt=0.025, cadence=40)
    model = wl.model
    st, _ = oc.sample(model, wl.init, wl.run.seed, wl.run.n_traj)
    st.a[:] = 0
    st.b[:] = 1
    st.w[:] = 1.0
    sums, _ = oc.propagate(model, st, wl.run.dt, wl.run.n_steps, wl.run.cadence, wl.run.seed, wl.run.n_out)
    out = oc.finalize(sums, wl.run.n_traj)
    kT = wl.init.kT
    th = np.tanh(model.hbar * model.omega / (2 * kT))
    vq = model.hbar / (2 * model.mass * model.omega * th)
    vp = model.hbar * model.mass * model.omega / (2 * th)
    for o in range(1, wl.run.n_out):
        t = o * wl.run.cadence * wl.run.dt
        A, B, C = _zero_coupling_phase_coefficients(model, t)
        mean = A + B @ wl.init.q0
        var = np.sum(B * B * vq + C * C * vp)
        cf = np.exp(-1j * mean - 0.5 * var)
        mc = out[o, 0, 0, 1, 0] + 1j * out[o, 0, 0, 1, 1]
        se = math.hypot(out[o, 0, 0, 1, 2], out[o, 0, 0, 1, 3])
        assert abs(mc - cf) < 4.5 * se + 2e-3 * t * wl.run.dt, (o, mc, cf, se)


# ------------------------------------------------------------ uncoupled harmonic

def test_uncoupled_harmonic_exact_verlet_map(oracle_lib):
    oc = oracle_lib
    wl = W.uncoupled_harmonic()
    model, r = wl.model, wl.run
    st0, _ = oc.sample(model, wl.init, r.seed, r.n_traj)
    st = st0.copy()
    sums, _ = oc.propagate(model, st, r.dt, r.n_steps, r.cadence, r.seed, r.n_out)
    assert np.array_equal(st.a, st0.a) and np.array_equal(st.b, st0.b) and np.array_equal(st.w, st0.w)
    for j in range(model.n_modes):
        Mn = np.linalg.matrix_power(_verlet_matrix(model.mass[j], model.omega[j], r.dt), r.n_steps)
        x = Mn @ np.stack([st0.q[:, j], st0.p[:, j]])
        np.testing.assert_allclose(st.q[:, j], x[0], rtol=1e-11, atol=1e-12)
        np.testing.assert_allclose(st.p[:, j], x[1], rtol=1e-11, atol=1e-12)
        # continuous orbit to O(dt^2)
        m, w, t = model.mass[j], model.omega[j], r.n_steps * r.dt
        qc = st0.q[:, j] * np.cos(w * t) + st0.p[:, j] / (m * w) * np.sin(w * t)
        assert np.max(np.abs(st.q[:, j] - qc)) < (w * r.dt) ** 2 * w * t * (np.abs(st0.q[:, j]).max() + 5)
    # constant surfaces: phase of (a,b) is (E_a - E_b) t exactly
    E = np.linalg.eigvalsh(model.v0)
    expect = (E[st.a] - E[st.b]) * r.n_steps * r.dt
    np.testing.assert_allclose(st.phase, expect, atol=1e-12)


# ------------------------------------------------------------ weights, transitions

def test_weight_growth_invariant(oracle_lib):
    oc = oracle_lib
    for wl in (W.pyrazine_ci(), W.spin_boson_1mode(), W.random_lvc(5, n_states=3, n_modes=2),
               W.random_lvc(6, n_states=4, n_modes=3)):
        model = wl.model
        en = Enumerator(model)
        st, _ = oc.sample(model, wl.init, 21, 300)
        w0 = st.w.copy()
        S = np.zeros(st.n_traj)
        for t in range(st.n_traj):
            vd = en.vd(st.q[t], st.p[t], st.U[t])
            a, b = st.a[t], st.b[t]
            S[t] = wl.run.dt * (sum(abs(vd[a, c]) for c in range(model.n_states) if c != a)
                                + sum(abs(vd[b, c]) for c in range(model.n_states) if c != b))
        oc.propagate(model, st, wl.run.dt, 1, 1000, 21, 1)
        np.testing.assert_allclose(np.abs(st.w) / np.abs(w0) - 1.0, S, rtol=1e-5, atol=1e-9)


@pytest.mark.parametrize("scheme", [0, 1])
def test_one_step_transition_expectation(oracle_lib, scheme):
    """Integrating the transition over u gives exactly w (1 + dt L) E_ab."""
    oc = oracle_lib
    rng = np.random.default_rng(2)
    n_u = 1 << 15
    us = (np.arange(n_u) + 0.5) / n_u
    for n in (2, 3, 4):
        for _ in range(4):
            x = rng.normal(size=(n, n)) * (0.3 if scheme == 1 else 3.0) / n
            vd = x - x.T
            dt = 0.1
            a, b = rng.integers(0, n, size=2)
            acc = np.zeros((n, n))
            for u in us:
                _, a1, b1, w1, fb = oc.transition(vd, dt, u, scheme, a, b, 1.0)
                acc[a1, b1] += w1
            acc /= n_u
            Eab = np.zeros((n, n))
            Eab[a, b] = 1.0
            expect = Eab - dt * (vd @ Eab - Eab @ vd)
            S = np.abs(expect).sum() - 1.0
            np.testing.assert_allclose(acc, expect, atol=4 * (1 + S) * (2 * n) / n_u)


@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("start", [(0, 0), (0, 1), (1, 1)])
def test_all_branches_enumeration(oracle_lib, scheme, start):
    oc = oracle_lib
    wl = W.spin_boson_1mode()
    mm = oc.Model(wl.model)
    q0, p0 = np.array([-0.9]), np.array([1.2])
    E0, U0 = oc.adiabatic(mm, q0)
    k, dt, T = 5, 0.1, 200_000
    ex = Enumerator(wl.model).expectation(q0, p0, start[0], start[1], U0, dt, k)
    st = oc.State(T, 2, 1)
    st.q[:] = q0
    st.p[:] = p0
    st.a[:] = start[0]
    st.b[:] = start[1]
    st.w[:] = 1.0
    st.U[:] = U0
    sums, _ = oc.propagate(mm, st, dt, k, 1, 7 + scheme, k + 1, scheme=scheme)
    out = oc.finalize(sums, T)
    mc = out[1:, ..., 0] + 1j * out[1:, ..., 1]
    se_r, se_i = out[1:, ..., 2], out[1:, ..., 3]
    grain = 10 * np.abs(st.w).max() / T  # a few walkers' worth: rare branches may go unsampled
    assert np.all(np.abs(mc.real - ex.real) <= 4.5 * se_r + grain)
    assert np.all(np.abs(mc.imag - ex.imag) <= 4.5 * se_i + grain)


@pytest.mark.parametrize("n_states,k", [(3, 3), (5, 2), (8, 2)])
def test_many_state_enumeration(oracle_lib, n_states, k):
    oc = oracle_lib
    wl = W.random_lvc(1, n_states=n_states, n_modes=1)
    mm = oc.Model(wl.model)
    rng = np.random.default_rng(0)
    q0 = wl.init.q0 + 0.3 * rng.normal(size=1)
    p0 = np.array([1.5])
    _, U0 = oc.adiabatic(mm, q0)
    dt, T = 0.2, 200_000
    s0 = n_states // 2
    ex = Enumerator(wl.model).expectation(q0, p0, s0, s0, U0, dt, k)
    st = oc.State(T, n_states, 1)
    st.q[:] = q0
    st.p[:] = p0
    st.a[:] = s0
    st.b[:] = s0
    st.w[:] = 1.0
    st.U[:] = U0
    sums, _ = oc.propagate(mm, st, dt, k, 1, 17, k + 1)
    out = oc.finalize(sums, T)
    mc = out[1:, ..., 0] + 1j * out[1:, ..., 1]
    grain = 10 * np.abs(st.w).max() / T  # a few walkers' worth: rare branches may go unsampled
    assert np.all(np.abs(mc.real - ex.real) <= 4.5 * out[1:, ..., 2] + grain)
    assert np.all(np.abs(mc.imag - ex.imag) <= 4.5 * out[1:, ..., 3] + grain)


# ------------------------------------------------------------ whole estimator

def test_grid_solution_agreement(oracle_lib):
    oc = oracle_lib
    ts, rho = _grid_fixture()
    dt = 0.0125
    wl = W.spin_boson_1mode(n_traj=200_000, n_steps=int(round(3.0 / dt)), dt=dt,
                            cadence=int(round(0.5 / dt)), seed=5)
    out, _, _ = oc.run(wl)
    n = out.shape[0]
    g = rho[:n]
    for basis in (0, 1):
        for i in range(2):
            for j in range(2):
                mre, mim = out[:, basis, i, j, 0], out[:, basis, i, j, 1]
                sre, sim = out[:, basis, i, j, 2], out[:, basis, i, j, 3]
                # statistical error plus a first-order splitting bias allowance
                assert np.all(np.abs(mre - g[:, basis, i, j].real) <= 4.5 * sre + 0.4 * dt), (basis, i, j)
                assert np.all(np.abs(mim - g[:, basis, i, j].imag) <= 4.5 * sim + 0.4 * dt), (basis, i, j)


@pytest.mark.slow
def test_step_size_bias_first_order(oracle_lib):
    oc = oracle_lib
    ts, rho = _grid_fixture()
    biases, ses = [], []
    for dt in (0.1, 0.05, 0.025):
        wl = W.spin_boson_1mode(n_traj=1_000_000, n_steps=int(round(1.5 / dt)), dt=dt,
                                cadence=int(round(0.5 / dt)), seed=6)
        out, _, _ = oc.run(wl)
        biases.append(out[2:4, 1, 0, 0, 0] - rho[2:4, 1, 0, 0].real)  # t = 1.0, 1.5
        ses.append(out[2:4, 1, 0, 0, 2])
    b = np.array(biases)
    se = np.array(ses)
    assert np.all(b[0] > 6 * se[0])  # visible bias at the largest step
    # the bias shrinks between first order (ratio 2) and second order (4) per halving
    ratio = b[0] / b[1]
    assert np.all((ratio > 1.4) & (ratio < 5.5)), ratio
    assert np.all(np.abs(b[2]) < np.abs(b[1]) + 2 * se[2])
    assert np.all(np.abs(b[2]) < 0.5 * b[0] + 3 * se[2])


def test_trace_and_hermiticity_in_expectation(oracle_lib):
    oc = oracle_lib
    for wl in (W.spin_boson_1mode(n_traj=100_000, n_steps=60, dt=0.05, cadence=20, seed=9),
               W.pyrazine_ci(n_traj=100_000, n_steps=30, cadence=10, seed=9),
               W.random_lvc(4, n_states=3, n_modes=4, n_traj=100_000, n_steps=40),
               W.random_lvc(8, n_states=4, n_modes=2, n_traj=100_000, n_steps=40)):
        out, _, _ = oc.run(wl)
        n = wl.model.n_states
        for basis in (0, 1):
            tr = sum(out[:, basis, i, i, 0] for i in range(n))
            se = np.sqrt(sum(out[:, basis, i, i, 2] ** 2 for i in range(n)))
            assert np.all(np.abs(tr - 1.0) <= 5 * se * math.sqrt(n) + 1e-12), (wl.model.name, basis, tr, se)
            for i in range(n):
                for j in range(i + 1, n):
                    re = out[:, basis, i, j, 0] - out[:, basis, j, i, 0]
                    im = out[:, basis, i, j, 1] + out[:, basis, j, i, 1]
                    sr = np.hypot(out[:, basis, i, j, 2], out[:, basis, j, i, 2])
                    si = np.hypot(out[:, basis, i, j, 3], out[:, basis, j, i, 3])
                    assert np.all(np.abs(re) <= 5 * sr + 1e-12), (wl.model.name, basis, i, j)
                    assert np.all(np.abs(im) <= 5 * si + 1e-12), (wl.model.name, basis, i, j)
