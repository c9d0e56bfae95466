"""Pins of the oracle for models with cross-mode bilinear terms,
V(q) = V0 + sum_j [q_j K_j + sum_{k=2..D} q_j^k A_jk] + sum_p q_{i_p} q_{j_p} B_p:
LAPACK eigenvalues of V(q) built here from the model definition, forces and
couplings against finite differences, the exact discrete velocity-Verlet
map of a diagonal model whose bilinear terms couple the modes (a linear
map of (q, p), applied as a matrix power) with its phase as the exact
trapezoid sum over that orbit, the all-branches enumeration of the
independent numpy enumerator, and exact reduction to the model without
them when every B_p vanishes."""
import numpy as np
import pytest
import scipy.linalg as sl

import workloads as W
from oracle.branches import Enumerator


def _V(model, q):
    v = model.v0 + np.tensordot(q, model.k, axes=(0, 0))
    for k in range(2, model.degree + 1):
        v = v + np.tensordot(q ** k, model.poly[:, k - 2], axes=(0, 0))
    for i, j, B in model.bilinear or []:
        v = v + q[i] * q[j] * B
    return v


@pytest.mark.parametrize("wl", [W.pyrazine_bilinear(),
                                W.random_bilinear(0, n_states=2, n_modes=3, n_pairs=2),
                                W.random_bilinear(1, n_states=3, n_modes=5, n_pairs=4, degree=3),
                                W.random_bilinear(2, n_states=4, n_modes=4, n_pairs=3, degree=4),
                                W.random_bilinear(5, n_states=3, n_modes=6, n_pairs=8, degree=2),
                                W.random_bilinear(15, n_states=2, n_modes=5, all_pairs=True, degree=3)])
def test_bilinear_force_and_nac_vs_finite_differences(oracle_lib, wl):
    oc = oracle_lib
    model = wl.model
    m = oc.Model(model)
    n, M = model.n_states, model.n_modes
    rng = np.random.default_rng(9)
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


def _diag_bilinear():
    """Two states, three modes, every matrix diagonal, two bilinear terms:
    no electronic coupling, so each element moves on one quadratic
    surface whose force couples the modes."""
    M = 3
    kap = np.array([[0.3, -0.2], [-0.1, 0.25], [0.05, 0.0]])   # kappa_j per state
    g = np.array([[0.1, -0.15], [0.0, 0.2], [-0.05, 0.05]])    # q_j^2 coefficient per state
    bil = [(0, 1, np.diag([0.12, -0.08])), (1, 2, np.diag([-0.05, 0.1]))]
    k = np.stack([np.diag(kap[j]) for j in range(M)])
    poly = np.stack([np.diag(g[j]) for j in range(M)])[:, None]
    model = W.LVCModel(name="diag_bilinear", mass=[1.0, 0.6, 2.0], omega=[1.0, 1.4, 0.7], v0=np.diag([-4.0, 4.0]),
                       k=k, poly=poly, bilinear=bil)
    init = W.InitSpec(kT=0.3, q0=np.zeros(M), state=0)
    return W.Workload(model, init, W.RunSpec(200, 150, 0.04, 10, 27)), kap, g, bil


def test_diagonal_bilinear_exact_verlet_map_and_phase(oracle_lib):
    oc = oracle_lib
    wl, kap, g, bil = _diag_bilinear()
    model, r = wl.model, wl.run
    M = model.n_modes
    st0, _ = oc.sample(model, wl.init, r.seed, r.n_traj)
    half = r.n_traj // 2
    st0.a[:half], st0.b[:half] = 0, 1   # the coherence (0, 1)
    st0.a[half:], st0.b[half:] = 1, 1   # the population (1, 1)
    st0.w[:] = 1.0
    st0.U[:] = np.eye(2)
    st = st0.copy()
    oc.propagate(model, st, r.dt, r.n_steps, r.cadence, r.seed, r.n_out)
    assert np.array_equal(st.a, st0.a) and np.array_equal(st.b, st0.b) and np.all(st.w == 1.0)
    minv = np.diag(1.0 / model.mass)
    for a, b, sel in ((0, 1, slice(0, half)), (1, 1, slice(half, None))):
        # mean force F = -K q - c of element (a, b): K couples the modes
        K = np.diag(model.mass * model.omega ** 2 + g[:, a] + g[:, b])
        for i, j, B in bil:
            K[i, j] += 0.5 * (B[a, a] + B[b, b])
            K[j, i] += 0.5 * (B[a, a] + B[b, b])
        c = 0.5 * (kap[:, a] + kap[:, b])
        qs = -np.linalg.solve(K, c)
        kick = np.block([[np.eye(M), np.zeros((M, M))], [-0.5 * r.dt * K, np.eye(M)]])
        drift = np.block([[np.eye(M), r.dt * minv], [np.zeros((M, M)), np.eye(M)]])
        A = kick @ drift @ kick
        y = np.concatenate([(st0.q[sel] - qs).T, st0.p[sel].T])   # [2M, walkers]
        # the gap along the orbit, V_aa - V_bb, and its trapezoid sum
        def gap(yq):
            qq = yq[:M] + qs[:, None]
            d = (kap[:, a] - kap[:, b]) @ qq + (g[:, a] - g[:, b]) @ qq ** 2
            for i, j, B in bil:
                d = d + (B[a, a] - B[b, b]) * qq[i] * qq[j]
            return d + (model.v0[a, a] - model.v0[b, b])
        phase = 0.5 * gap(y)
        for s in range(r.n_steps):
            y = A @ y
            phase = phase + (gap(y) if s + 1 < r.n_steps else 0.5 * gap(y))
        np.testing.assert_allclose(st.q[sel], (y[:M] + qs[:, None]).T, rtol=1e-10, atol=1e-11)
        np.testing.assert_allclose(st.p[sel], y[M:].T, rtol=1e-10, atol=1e-11)
        np.testing.assert_allclose(st.phase[sel], r.dt * phase, rtol=1e-11, atol=1e-11)


def test_zero_bilinear_terms_reduce_to_the_model_without_them(oracle_lib):
    oc = oracle_lib
    base = W.pyrazine_qvc(n_traj=300, n_steps=60, cadence=10)
    m0 = base.model
    zero = W.LVCModel(name="zero_bilinear", mass=m0.mass, omega=m0.omega, v0=m0.v0, k=m0.k, hbar=m0.hbar,
                      poly=m0.poly, bilinear=[(0, 2, np.zeros((2, 2))), (1, 2, np.zeros((2, 2)))])
    out_0, st_0, _ = oc.run(base)
    out_z, st_z, _ = oc.run(W.Workload(zero, base.init, base.run))
    assert np.array_equal(out_0, out_z)
    for key in ("q", "p", "w", "phase", "U"):
        assert np.array_equal(getattr(st_0, key), getattr(st_z, key)), key


def test_bilinear_all_branches_enumeration(oracle_lib):
    oc = oracle_lib
    wl = W.random_bilinear(3, n_states=3, n_modes=2, n_pairs=1, degree=2)
    mm = oc.Model(wl.model)
    q0, p0 = np.array([0.4, -0.3]), np.array([1.4, 0.9])
    _, U0 = oc.adiabatic(mm, q0)
    k, dt, T = 3, 0.2, 200_000
    ex = Enumerator(wl.model).expectation(q0, p0, 2, 2, U0, dt, k)
    st = oc.State(T, 3, 2)
    st.q[:] = q0
    st.p[:] = p0
    st.a[:] = 2
    st.b[:] = 2
    st.w[:] = 1.0
    st.U[:] = U0
    sums, _ = oc.propagate(mm, st, dt, k, 1, 29, k + 1)
    out = oc.finalize(sums, T)
    mc = out[1:, ..., 0] + 1j * out[1:, ..., 1]
    grain = 10 * np.abs(st.w).max() / T
    assert np.abs(ex[..., 0, :, :]).max() > 0.05  # the coupling moves weight off (2, 2)
    assert np.all(np.abs(mc.real - ex.real) <= 4.5 * out[1:, ..., 2] + grain)
    assert np.all(np.abs(mc.imag - ex.imag) <= 4.5 * out[1:, ..., 3] + grain)


def test_invalid_pairs_rejected_by_the_oracle(oracle_lib):
    oc = oracle_lib
    wl = W.random_bilinear(4, n_states=2, n_modes=3, n_pairs=1)
    for i, j in ((1, 1), (0, 3), (-1, 2)):
        m = wl.model
        bad = W.LVCModel(name="bad", mass=m.mass, omega=m.omega, v0=m.v0, k=m.k, poly=m.poly,
                         bilinear=[(i, j, np.eye(2))])
        st, _ = oc.sample(bad, wl.init, 1, 4)
        with pytest.raises(ValueError):
            oc.propagate(bad, st, 0.05, 2, 1, 1, 3)
