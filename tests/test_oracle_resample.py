"""Pins of the oracle's fixed-budget systematic resampling."""
import math

import numpy as np
import pytest

import oracle.core as oc
import oracle.resample as R


def _state(w, n_states=2, n_modes=2, seed=0):
    rng = np.random.default_rng(seed)
    T = len(w)
    st = oc.State(T, n_states, n_modes)
    st.q[:] = rng.normal(size=(T, n_modes))
    st.p[:] = rng.normal(size=(T, n_modes))
    st.w[:] = w
    st.phase[:] = rng.uniform(0, 6, size=T)
    st.a[:] = rng.integers(0, n_states, size=T)
    st.b[:] = rng.integers(0, n_states, size=T)
    st.U[:] = np.eye(n_states)
    return st


def test_copy_counts_are_floor_or_ceil_and_order_kept():
    rng = np.random.default_rng(1)
    w = rng.lognormal(0, 1.5, size=500) * rng.choice([-1, 1], size=500)
    k, _ = R.quantized(w.tolist(), [0.0] * 500)
    for U in (0, 1, 123456789, (1 << 32) - 1):
        src, K = R.indices(k, U)
        assert len(src) == 500 and all(a <= b for a, b in zip(src, src[1:]))
        counts = np.bincount(src, minlength=500)
        expect = [500 * x / K for x in k]
        assert all(math.floor(e) <= c <= math.ceil(e) for c, e in zip(counts, expect))


def test_equal_weights_give_the_identity():
    st = _state([-2.5] * 37)
    out = R.resample(st, seed=9)
    assert np.array_equal(out.q, st.q) and np.array_equal(out.w, st.w) and np.array_equal(out.a, st.a)


def test_unbiased_over_offsets():
    rng = np.random.default_rng(2)
    T = 40
    w = rng.lognormal(0, 1.0, size=T) * rng.choice([-1, 1], size=T)
    k, _ = R.quantized(w.tolist(), [0.0] * T)
    acc = np.zeros(T)
    n = 20000
    for U in rng.integers(0, 1 << 32, size=n):
        src, K = R.indices(k, int(U))
        for i in src:
            acc[i] += w[i] * (float(K) / (float(T) * float(k[i])))
    est = acc / n
    # each walker's expected total weight after resampling is its own weight;
    # its copy count is floor(e) or ceil(e), e = T k/K, so one draw's
    # contribution has standard deviation at most |w|/(2e)
    e = T * np.array(k, dtype=float) / sum(k)
    sd = np.abs(w) / (2 * e)
    assert np.all(np.abs(est - w) <= 5 * sd / math.sqrt(n) + 1e-12 * np.abs(w))


def test_zero_and_nonfinite_weights_are_dropped():
    w = [1.0, 0.0, float("nan"), 3.0, float("inf"), 2.0]
    st = _state(w)
    out = R.resample(st, seed=4)
    src_w = set(out.w.tolist())
    assert all(np.isfinite(out.w)) and 0.0 not in src_w
    k, wmax = R.quantized(w, [0.0] * 6)
    assert wmax == 3.0 and k[1] == k[2] == k[4] == 0 and k[3] == 1 << 32
    # walkers keep their weight sign and magnitudes become K/(T k_i) |w_i|
    K = sum(k)
    for x in out.w:
        assert any(math.isclose(abs(x), abs(v) * K / (6 * kk), rel_tol=1e-15) for v, kk in zip(w, k) if kk)


def test_all_zero_weights_copy_unchanged():
    st = _state([0.0] * 8)
    out = R.resample(st, seed=1)
    assert np.array_equal(out.q, st.q) and np.array_equal(out.w, st.w)


def test_quantization_and_offset_definitions():
    k, wmax = R.quantized([0.5, -1.0, 1e-30], [0.0, 0.0, 0.0])
    assert wmax == 1.0 and k == [1 << 31, 1 << 32, 1]   # ceil keeps tiny weights alive
    # the offset is word 0 of the Philox block at counter (offset, step, 3)
    x = oc.philox([7, 0, 11, 3], [5, 0])
    assert R.offset_word(5, 7, 11) == int(x[0])


def test_per_output_source_matches_the_sequential_walk():
    # zero weights in the middle and at both ends give empty intervals that
    # the search must step over
    rng = np.random.default_rng(4)
    w = rng.lognormal(0, 2.0, size=300)
    w[[0, 5, 6, 7, 150, 299]] = 0.0
    k, _ = R.quantized(w.tolist(), [0.0] * 300)
    P = R.prefix(k)
    assert P[-1] == sum(k) and len(P) == 301
    for U in (0, 77, (1 << 32) - 1):
        src, _ = R.indices(k, U)
        assert [R.source(P, U, j) for j in range(300)] == src
