"""Pins of the oracle's initial sampling (partial Wigner transform, Sec. II.A).

* thermal Wigner moments of every mode in closed form:
  <q> = q0, var q = hbar/(2 m w tanh(hbar w/2kT)), var p = hbar m w/(2 tanh(.)),
  cov(q, p) = 0, and the 1-mode spin-boson value var = 1/(2 tanh 1);
* the diabatic initial projector |k><k| is recovered exactly in
  expectation: the t = 0 diabatic bin equals e_k e_k^T within its SE;
* adiabatic start: (a, b) = (k, k), w = 1 for every walker;
* reproducibility and trajectory-offset slicing.
"""
import math

import numpy as np
import pytest

import workloads as W


@pytest.mark.parametrize("wl", [W.spin_boson_1mode(), W.spin_boson_ohmic(kT=1.0), W.pyrazine_ci()])
def test_wigner_moments(oracle_lib, wl):
    oc = oracle_lib
    T = 200_000
    st, _ = oc.sample(wl.model, wl.init, 99, T)
    m = wl.model
    for j in range(m.n_modes):
        kT = wl.init.kT
        th = math.tanh(m.hbar * m.omega[j] / (2 * kT)) if kT > 0 else 1.0
        vq = m.hbar / (2 * m.mass[j] * m.omega[j] * th)
        vp = m.hbar * m.mass[j] * m.omega[j] / (2 * th)
        q, p = st.q[:, j], st.p[:, j]
        assert abs(q.mean() - wl.init.q0[j]) < 4.5 * math.sqrt(vq / T)
        assert abs(p.mean()) < 4.5 * math.sqrt(vp / T)
        assert abs(q.var() / vq - 1) < 4.5 * math.sqrt(2 / T)
        assert abs(p.var() / vp - 1) < 4.5 * math.sqrt(2 / T)
        assert abs(np.corrcoef(q, p)[0, 1]) < 4.5 / math.sqrt(T)
        # fourth moment of a Gaussian: kurtosis 3
        kq = ((q - q.mean()) ** 4).mean() / q.var() ** 2
        assert abs(kq - 3) < 4.5 * math.sqrt(96 / T)


def test_spin_boson_width_value(oracle_lib):
    oc = oracle_lib
    wl = W.spin_boson_1mode()
    st, _ = oc.sample(wl.model, wl.init, 0, 100_000)
    assert abs(st.q[:, 0].var() - 0.656518) < 0.01
    assert abs(0.5 / math.tanh(1.0) - 0.656518) < 1e-6


@pytest.mark.parametrize("wl", [W.spin_boson_1mode(), W.pyrazine_ci(), W.random_lvc(2, n_states=3, n_modes=3),
                                W.random_lvc(9, n_states=4, n_modes=2)])
def test_initial_projector_unbiased(oracle_lib, wl):
    oc = oracle_lib
    T = 100_000
    st, s0 = oc.sample(wl.model, wl.init, 5, T)
    out = oc.finalize(s0[None], T)[0]
    n = wl.model.n_states
    k = wl.init.state
    target = np.zeros((n, n))
    target[k, k] = 1.0
    mean = out[1, :, :, 0]
    se = out[1, :, :, 2]
    assert np.all(np.abs(mean - target) <= 4.5 * se + 1e-12), (mean, se)
    assert np.all(out[1, :, :, 1] == 0.0)  # no phase at t = 0
    # every walker's |w| is Z = (sum_a |U_ka|)^2
    Z = np.abs(st.U[:, k, :]).sum(axis=1) ** 2
    np.testing.assert_allclose(np.abs(st.w), Z, rtol=1e-15)
    assert np.all(st.U[np.arange(T), st.a, st.a] > 0)


def test_adiabatic_start(oracle_lib):
    oc = oracle_lib
    wl = W.pyrazine_ci()
    wl.init.basis = W.INIT_ADIABATIC
    wl.init.state = 1
    st, s0 = oc.sample(wl.model, wl.init, 1, 1000)
    assert np.all(st.a == 1) and np.all(st.b == 1) and np.all(st.w == 1.0)
    assert s0[0, 1, 1, 0] == 1000.0


def test_sampling_reproducible_and_sliced(oracle_lib):
    oc = oracle_lib
    wl = W.pyrazine_ci()
    st1, _ = oc.sample(wl.model, wl.init, 3, 3000)
    st2, _ = oc.sample(wl.model, wl.init, 3, 1000, traj_offset=2000)
    for f in ("q", "p", "w", "a", "b", "U"):
        assert np.array_equal(getattr(st1, f)[2000:], getattr(st2, f))
    st3, _ = oc.sample(wl.model, wl.init, 4, 3000)
    assert not np.array_equal(st1.q, st3.q)
