"""The oracle's supplied-potential path (the general form of Eq. 1, Sec. IV's
next step): a model whose V(q) and dV/dq come from compiled C callbacks.

Pins, none of which re-types the oracle's own arithmetic:
  * the test models' gradients against central finite differences of their
    potentials (the callbacks agree with themselves);
  * a linear-vibronic model written as a supplied potential reproduces the
    built-in linear-vibronic oracle (itself pinned by the other oracle
    tests) walker by walker to rounding, which ties the callback plumbing --
    mean force without a separate bath term, couplings from the supplied
    gradient -- to the pinned path;
  * an uncoupled Morse oscillator keeps the textbook classical period
    T(E) = 2 pi / (a sqrt(2 (D - E) / m)) within the Verlet error, and the
    harmonic spectator mode its period 2 pi / sqrt(k / m).
"""
import ctypes as C
import math

import numpy as np
import pytest

import oracle.core as oc
import workloads as W

_dp = C.POINTER(C.c_double)


def _ptr(a):
    return a.ctypes.data_as(_dp)


def _potential(m, q):
    V = np.zeros(m.n * m.n)
    m.user.qcl_oracle_potential(_ptr(q), _ptr(m.params), _ptr(V))
    return V.reshape(m.n, m.n)


def _gradient(m, j, q):
    G = np.zeros(m.n * m.n)
    m.user.qcl_oracle_gradient(int(j), _ptr(q), _ptr(m.params), _ptr(G))
    return G.reshape(m.n, m.n)


@pytest.mark.parametrize("make", [lambda: W.morse_coupled().model,
                                  lambda: W.lvc_as_source(W.random_lvc(7, n_modes=4).model)],
                         ids=["morse", "lvc_n3_m4"])
def test_gradient_matches_finite_differences(make):
    m = oc.Model(make())
    rng = np.random.default_rng(1)
    for _ in range(5):
        q = rng.normal(0.0, 0.5, m.M)
        V = _potential(m, q)
        assert np.allclose(V, V.T, rtol=0, atol=0)
        for j in range(m.M):
            h = 1e-5
            qp, qm = q.copy(), q.copy()
            qp[j] += h
            qm[j] -= h
            fd = (_potential(m, qp) - _potential(m, qm)) / (2 * h)
            assert np.allclose(_gradient(m, j, q), fd, rtol=1e-7, atol=1e-9)


def _run(model, wl, T, S, scheme=oc.NORMALIZED):
    r = wl.run
    m = oc.Model(model)
    st, s0 = oc.sample(m, wl.init, r.seed, T)
    n_out = S // r.cadence + 1
    sums = np.zeros((n_out, 2, m.n, m.n, 4))
    sums[0] = s0
    oc.propagate(m, st, r.dt, S, r.cadence, r.seed, n_out, sums, scheme)
    return oc.finalize(sums, T), st


@pytest.mark.parametrize("index,n_modes,scheme", [(7, 4, oc.NORMALIZED), (3, 2, oc.LINEAR)])
def test_lvc_as_source_reproduces_builtin(index, n_modes, scheme):
    wl = W.random_lvc(index, n_modes=n_modes)
    src = W.lvc_as_source(wl.model)
    o1, s1 = _run(wl.model, wl, 600, 120, scheme)
    o2, s2 = _run(src, wl, 600, 120, scheme)
    assert np.array_equal(s1.a, s2.a) and np.array_equal(s1.b, s2.b)
    for key in ("q", "p", "phase"):
        x, y = getattr(s1, key), getattr(s2, key)
        assert np.max(np.abs(x - y)) <= 1e-11 * max(1.0, float(np.abs(x).max())), key
    assert np.max(np.abs(s1.w - s2.w) / np.abs(s1.w)) <= 1e-11
    rms = np.sqrt(o1[..., 2:] ** 2 * 599 + o1[..., :2] ** 2)
    assert np.all(np.abs(o1[..., :2] - o2[..., :2]) <= 1e-11 * np.maximum(1.0, rms))


def _turning_times(ts, p):
    """Times at which p crosses zero from below (linear interpolation)."""
    out = []
    for i in range(1, len(p)):
        if p[i - 1] < 0.0 <= p[i]:
            out.append(ts[i - 1] + (ts[i] - ts[i - 1]) * (-p[i - 1]) / (p[i] - p[i - 1]))
    return np.array(out)


def test_uncoupled_morse_period_closed_form():
    wl = W.morse_coupled()
    model = wl.model
    model.params = model.params.copy()
    model.params[8] = 0.0  # no diabatic coupling: each walker stays on its surface
    D, a, x0, k1 = model.params[0], model.params[2], model.params[3], model.params[6]
    m = oc.Model(model)
    init = W.InitSpec(kT=0.0, q0=[0.0, 0.0], state=0, basis=W.INIT_ADIABATIC)
    st, _ = oc.sample(m, init, 1, 1)
    A = 0.3
    st.q[0] = [x0 - A, 0.2]
    st.p[0] = [0.0, 0.0]
    st.U[0] = np.eye(2)
    E = D * (1.0 - math.exp(a * A)) ** 2  # at the left turning point
    dt, every = 0.005, 8  # momenta recorded every 8 steps (0.04)
    ts, p0, p1 = [0.0], [0.0], [0.0]
    for i in range(500):
        oc.propagate(m, st, dt, every, every, 1, 1)
        ts.append((i + 1) * every * dt)
        p0.append(st.p[0, 0])
        p1.append(st.p[0, 1])
    assert st.a[0] == 0 and st.b[0] == 0 and st.w[0] == 1.0  # never left the lower surface
    # mode 0 starts at rest at its left turning point: p0 first rises from 0
    t0 = _turning_times(np.array(ts), np.array(p0))
    T_morse = 2.0 * math.pi / (a * math.sqrt(2.0 * (D - E) / model.mass[0]))
    periods = np.diff(np.concatenate([[0.0], t0]))
    assert len(periods) >= 2
    assert np.all(np.abs(periods / T_morse - 1.0) < 2e-4), (periods, T_morse)
    # mode 1 starts at its right turning point; successive minima of p1 one period apart
    t1 = _turning_times(np.array(ts), np.array(p1))
    T_h = 2.0 * math.pi / math.sqrt(k1 / model.mass[1])
    assert np.all(np.abs(np.diff(t1) / T_h - 1.0) < 2e-4), (np.diff(t1), T_h)
