"""Pins of the oracle's ensemble averages (``or_finalize``) and of its bin
sums, independent of the formula the oracle uses: each walker of a small
ensemble is run on its own (its random streams are keyed by its global
id, so it is the same walker), its own bin terms are read from its
one-walker sums, and numpy's mean and sample standard deviation of those
terms give the expected means and standard errors."""
import numpy as np
import pytest

import oracle.core as oc
import workloads as W


def _per_walker_terms(wl, T, S):
    """[T, n_out, 2, N, N, 2] per-walker (Re, Im) terms and their squares."""
    r = wl.run
    n_out = S // r.cadence + 1
    m = oc.Model(wl.model)
    terms = []
    for i in range(T):
        st, s0 = oc.sample(m, wl.init, r.seed, 1, traj_offset=i)
        sums = np.zeros((n_out, 2, m.n, m.n, 4))
        sums[0] = s0
        oc.propagate(m, st, r.dt, S, r.cadence, r.seed, n_out, sums)
        terms.append(sums)
    return np.array(terms)


@pytest.mark.parametrize("name", ["pyrazine", "n3"])
def test_finalize_mean_and_standard_error(oracle_lib, name):
    T, S = 97, 40
    wl = {"pyrazine": W.pyrazine_ci(n_traj=T, n_steps=S, cadence=5),
          "n3": W.random_lvc(3, n_states=3, n_modes=4, n_traj=T, n_steps=S, cadence=5)}[name]
    out, _, sums = oc.run(wl)
    terms = _per_walker_terms(wl, T, S)
    # a one-walker sum holds the term itself and its exact square
    np.testing.assert_array_equal(terms[..., 2], terms[..., 0] ** 2)
    np.testing.assert_array_equal(terms[..., 3], terms[..., 1] ** 2)
    # the ensemble's sums are the sums of its walkers' terms (to rounding)
    scale = np.abs(terms).sum(axis=0)
    assert np.all(np.abs(sums - terms.sum(axis=0)) <= 1e-13 * np.maximum(scale, 1e-300))
    x = terms[..., :2]
    mean = x.mean(axis=0)
    se = x.std(axis=0, ddof=1) / np.sqrt(T)
    np.testing.assert_allclose(out[..., :2], mean, rtol=1e-12, atol=1e-15)
    # the oracle's one-pass formula against numpy's two-pass deviation:
    # relative agreement to ~1e-9 where the spread is not lost to cancellation
    big = se > 1e-6 * np.maximum(np.abs(mean), 1e-300)
    assert big.sum() > 50
    np.testing.assert_allclose(out[..., 2:][big], se[big], rtol=1e-9)
    assert np.all(np.abs(out[..., 2:] - se) <= 1e-7 * np.maximum(np.abs(mean), se) + 1e-15)


def test_finalize_single_walker_and_constant_terms(oracle_lib):
    """T = 1 has no standard error; a bin whose terms are all equal has SE 0."""
    s = np.zeros((1, 2, 2, 2, 4))
    s[0, 0, 0, 0] = [0.7, -0.2, 0.49, 0.04]
    o = oc.finalize(s, 1)
    np.testing.assert_array_equal(o[0, 0, 0, 0], [0.7, -0.2, 0.0, 0.0])
    s = np.zeros((1, 2, 2, 2, 4))
    s[0, 1, 1, 0] = [3 * 0.5, 3 * -0.25, 3 * 0.25, 3 * 0.0625]
    o = oc.finalize(s, 3)
    np.testing.assert_allclose(o[0, 1, 1, 0], [0.5, -0.25, 0.0, 0.0], atol=1e-12)
