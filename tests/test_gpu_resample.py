"""Parity of fixed-budget systematic resampling (HIP, through the C ABI)
with the oracle.

Every decision (the quantised weights, their prefix sums, the comb points
and the search) is integer arithmetic and every copy weight is the same
binary64 expression on both sides, so the bar is bit-exact: each output
walker's source, weight and copied state.  The source walker is read back
through the flags word, which the resampling copies verbatim: the tests
set it to the walker index beforehand.
"""
import numpy as np
import pytest

import oracle.core as oc
import oracle.resample as R
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2608_14544_amd as pkg
    pkg.load_library()
    return pkg


def _random_state(T, N, M, seed, prec, w=None, phase=None):
    """Seeded walker state; real arrays rounded to binary32 on the host for
    a binary32 ensemble, flags = walker index (to read sources back)."""
    rng = np.random.default_rng(seed)
    if w is None:
        w = rng.lognormal(0.0, 2.0, size=T) * rng.choice([-1.0, 1.0], size=T)
    rnd = (lambda x: x.astype(np.float32).astype(np.float64)) if prec == "fp32" else (lambda x: x)
    return {"q": rnd(rng.normal(size=(T, M))), "p": rnd(rng.normal(size=(T, M))),
            "U": rnd(rng.normal(size=(T, N, N))), "w": np.asarray(w, np.float64),
            "phase": rng.uniform(-20, 20, T) if phase is None else np.asarray(phase, np.float64),
            "a": rng.integers(0, N, T).astype(np.int32), "b": rng.integers(0, N, T).astype(np.int32),
            "flags": np.arange(T, dtype=np.uint32)}


def _device_pair(P, model, T, prec, traj_offset, step, state):
    import torch
    src = P.Ensemble(model, T, prec, traj_offset=traj_offset)
    dst = P.Ensemble(model, T, prec, traj_offset=traj_offset)
    if T:
        src.load_numpy(dict(state, step=step))
        src.tensors()["flags"][:T] = torch.as_tensor(state["flags"].view(np.int32), device=src.buffer.device)
    src.c.step = step
    return src, dst


def _oracle_state(g, N, M, traj_offset, step):
    T = len(g["w"])
    st = oc.State(T, N, M)
    for k in ("q", "p", "U", "w", "phase", "a", "b", "flags"):
        setattr(st, k, g[k].copy())
    st.traj_offset, st.step = traj_offset, step
    return st


def _same(x, y):
    if np.issubdtype(np.asarray(x).dtype, np.floating):
        return np.array_equal(x, y, equal_nan=True)
    return np.array_equal(x, y)


def _resample_both(P, model, N, M, T, prec, seed, traj_offset=0, step=0, state=None):
    import torch
    state = _random_state(T, N, M, seed, prec) if state is None else state
    src, dst = _device_pair(P, model, T, prec, traj_offset, step, state)
    assert _all_same(src.to_numpy(), state)
    P.qcl_resample(model, src, dst, seed)
    torch.cuda.synchronize()
    g = dst.to_numpy()
    assert dst.step == step and _all_same(src.to_numpy(), state)   # src is not changed
    o = R.resample(_oracle_state(state, N, M, traj_offset, step), seed)
    return g, o, state


def _all_same(a, b):
    return all(_same(a[k], b[k]) for k in b)


def _check(g, o, label):
    for k in ("q", "p", "U", "w", "phase", "a", "b", "flags"):
        assert _same(g[k], getattr(o, k)), (label, k)
    print(f"[{label}] bit-exact, {len(np.unique(g['flags']))} distinct sources of {len(g['w'])}", flush=True)


def _model(P, N, M, index=1):
    return P.Model(W.random_lvc(index, n_states=N, n_modes=M).model)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("N,M,T", [(2, 3, 1), (2, 3, 255), (3, 5, 257), (4, 7, 3000), (6, 4, 1000)])
def test_bit_exact(P, prec, N, M, T):
    model = _model(P, N, M)
    # a trajectory offset above 2^32 exercises both counter words
    g, o, _ = _resample_both(P, model, N, M, T, prec, seed=0x1234_5678_9ABC, traj_offset=(5 << 32) + 17, step=123)
    _check(g, o, f"{prec} N={N} M={M} T={T}")


def test_dropped_and_nonfinite_walkers(P):
    N, M, T = 2, 3, 777
    model = _model(P, N, M)
    rng = np.random.default_rng(3)
    w = rng.lognormal(0, 1.0, T) * rng.choice([-1.0, 1.0], T)
    w[[0, 1, 100, 776]] = 0.0
    w[[5, 300]] = np.nan
    w[[6, 301]] = np.inf
    w[7] = -np.inf
    w[8] = 1e-300           # survives quantisation with k = 1
    phase = rng.uniform(-3, 3, T)
    phase[[9, 500]] = np.nan
    phase[10] = np.inf
    st = _random_state(T, N, M, 4, "fp64", w=w, phase=phase)
    g, o, before = _resample_both(P, model, N, M, T, "fp64", seed=77, step=9, state=st)
    _check(g, o, "dropped")
    dead = {0, 1, 100, 776, 5, 300, 6, 301, 7, 9, 500, 10}
    assert not dead & set(g["flags"].tolist())
    assert np.all(np.isfinite(g["w"]))


@pytest.mark.parametrize("stride", [3000, 7])
def test_sparse_weights(P, stride):
    """Live walkers only every ``stride`` walkers: with stride 3000 a
    workgroup's outputs span more sources than it stages in LDS (the
    direct search over P), with stride 7 the slices are wide but staged."""
    N, M, T = 2, 3, 200_000
    model = _model(P, N, M)
    rng = np.random.default_rng(stride)
    w = np.zeros(T)
    live = np.arange(5, T, stride)
    w[live] = rng.lognormal(0, 1.5, live.size) * rng.choice([-1.0, 1.0], live.size)
    st = _random_state(T, N, M, 8, "fp64", w=w)
    g, o, _ = _resample_both(P, model, N, M, T, "fp64", seed=stride, step=2, state=st)
    _check(g, o, f"sparse/{stride}")
    assert set(g["flags"].tolist()) <= set(live.tolist())


def test_all_weights_zero_copies_unchanged(P):
    N, M, T = 3, 2, 300
    model = _model(P, N, M)
    st = _random_state(T, N, M, 5, "fp64", w=np.zeros(T))
    g, o, before = _resample_both(P, model, N, M, T, "fp64", seed=1, step=4, state=st)
    _check(g, o, "K=0")
    assert _all_same(g, before)


def test_equal_weights_give_the_identity(P):
    N, M, T = 2, 4, 4099
    model = _model(P, N, M)
    st = _random_state(T, N, M, 6, "fp32", w=np.full(T, -0.75))
    g, o, before = _resample_both(P, model, N, M, T, "fp32", seed=2, step=1, state=st)
    _check(g, o, "equal")
    assert _all_same(g, before)


def test_empty_ensemble(P):
    model = _model(P, 2, 3)
    src = P.Ensemble(model, 0, "fp64")
    dst = P.Ensemble(model, 0, "fp64")
    src.c.step = 5
    P.qcl_resample(model, src, dst, 3)
    assert dst.step == 5


def test_invalid_pairs_rejected(P):
    model = _model(P, 2, 3)
    a = P.Ensemble(model, 100, "fp64")
    with pytest.raises(P.QCLError):
        P.qcl_resample(model, a, P.Ensemble(model, 101, "fp64"), 1)
    with pytest.raises(P.QCLError):
        P.qcl_resample(model, a, P.Ensemble(model, 100, "fp32"), 1)
    with pytest.raises(P.QCLError):
        P.qcl_resample(model, a, P.Ensemble(model, 100, "fp64", traj_offset=1), 1)
    with pytest.raises(P.QCLError):
        P.qcl_resample(model, a, a, 1)


def test_million_walkers_bit_exact(P):
    N, M, T = 2, 3, 1_000_000
    model = _model(P, N, M)
    g, o, _ = _resample_both(P, model, N, M, T, "fp32", seed=11, traj_offset=3, step=200)
    _check(g, o, "1e6")


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_full_size_sampled(P, prec):
    """Ten million walkers of the pyrazine-like model (the ensemble of the
    throughput runs, both precisions of the resampling leg) with
    heavy-tailed signed weights, 0.5% of them zero: every output's source is
    checked for order and liveness, and 4096 sampled outputs against the
    oracle's per-output definition (source, weight and state bit-exact)."""
    import torch
    wl = W.pyrazine_ci()
    T, seed, step = 10_000_000, 21, 200
    model = P.Model(wl.model)
    N, M = model.n_states, model.n_modes
    rng = np.random.default_rng(seed)
    w = rng.lognormal(0.0, 2.5, T) * rng.choice([-1.0, 1.0], T)
    w[rng.integers(0, T, T // 200)] = 0.0
    s = _random_state(T, N, M, seed, prec, w=w)
    src, dst = _device_pair(P, model, T, prec, 0, step, s)
    P.qcl_resample(model, src, dst, seed)
    torch.cuda.synchronize()
    g = dst.to_numpy()
    k, _ = R.quantized(s["w"].tolist(), s["phase"].tolist())
    Pk = R.prefix(k)
    K = Pk[-1]
    U = R.offset_word(seed, 0, step)
    idx = g["flags"].astype(np.int64)
    assert np.all(np.diff(idx) >= 0)
    assert np.all(np.asarray(k, dtype=np.uint64)[idx] > 0)
    sample = np.unique(np.concatenate([[0, 1, T - 2, T - 1], rng.integers(0, T, 4092)]))
    for j in sample.tolist():
        i = R.source(Pk, U, j)
        assert idx[j] == i, j
        assert g["w"][j] == s["w"][i] * (float(K) / (float(T) * float(k[i]))), j
        for key in ("q", "p", "U", "phase", "a", "b"):
            assert _same(g[key][j], s[key][i]), (j, key)
    print(f"[1e7 {prec}] K={K} U={U} distinct sources={len(np.unique(idx))}", flush=True)


def test_propagate_resample_propagate_matches_oracle(P):
    """The composed path, binary64: sample, 20 steps, resample, 20 steps, on
    the device (run_resampled) and on the oracle.  The propagation agrees
    to rounding, so a walker's quantised weight k_i = ceil(|w_i|/w_max 2^32)
    can differ by one between the two; its copies' weights then differ by
    1/k_i relative, which the weight tolerance allows.  Everything else is
    held to the binary64 propagation tolerance, walkers whose transition
    decisions differ excluded (at most 0.2%)."""
    from paper_2608_14544_amd import branching
    from parity import check_ensemble64
    wl = W.pyrazine_ci(n_traj=0, n_steps=40, cadence=4)
    r, T, half = wl.run, 3000, 20
    out_g, ens, _ = branching.run_resampled(wl, T, 0, half, "fp64")
    g = ens.to_numpy()
    m = oc.Model(wl.model)
    st, s0 = oc.sample(m, wl.init, r.seed, T)
    n_out = r.n_steps // r.cadence + 1
    sums = np.zeros((n_out, 2, m.n, m.n, 4))
    sums[0] = s0
    oc.propagate(m, st, r.dt, half, r.cadence, r.seed, n_out, sums)
    k, _ = R.quantized(st.w.tolist(), st.phase.tolist())
    src, _ = R.indices(k, R.offset_word(r.seed, 0, half))
    st = R.resample(st, r.seed)
    oc.propagate(m, st, r.dt, half, r.cadence, r.seed, n_out, sums)
    out_o = oc.finalize(sums, T)
    flip = (g["a"] != st.a) | (g["b"] != st.b)
    flip |= ~(np.abs(np.abs(g["w"]) - np.abs(st.w)) <= 1e-6 * np.abs(st.w))
    ok = ~flip
    worst = {}
    for key in ("q", "p", "U", "phase"):
        o = getattr(st, key)
        scale = max(float(np.sqrt(np.mean(o ** 2))), 1e-300)
        worst[key] = float((np.abs(g[key] - o) / np.maximum(np.abs(o), scale))[ok].max())
    tol_w = 1e-9 + 2.0 / np.array([k[i] for i in src], dtype=np.float64)
    werr = np.abs(g["w"] - st.w) / np.abs(st.w)
    print(f"[composed] flips={int(flip.sum())} worst={worst} w-err/tol={float((werr / tol_w)[ok].max())} "
          f"sources={len(set(src))}", flush=True)
    assert flip.sum() <= 0.002 * T
    assert all(v <= 1e-9 for v in worst.values()), worst
    assert np.all(werr[ok] <= tol_w[ok])
    # every bin: a copy's relative weight difference is set at the resampling
    # and kept by the common factors (1 + S) afterwards, so the final
    # |w_gpu - w_oracle| of the agreeing walkers bounds their terms' difference
    # in every later bin; flipped walkers are bounded by their |w|
    quant = float(np.abs(g["w"][ok] - st.w[ok]).sum() / T)
    check_ensemble64(out_g, out_o, T, flip, g, {"w": st.w}, tol=1e-8, label="composed", extra_allow=quant)


def test_branching_without_resampling_is_the_plain_run(P):
    from paper_2608_14544_amd import branching
    wl = W.pyrazine_ci(n_traj=0, n_steps=60, cadence=2)
    plain, _, _ = branching.run_resampled(wl, 5000, 777, None, "fp32")
    ref, _ = P.run(wl, "fp32", n_traj=5000, traj_offset=777)
    assert np.array_equal(plain, ref)
    a, _, _ = branching.run_resampled(wl, 5000, 777, 4, "fp32")
    b, _, _ = branching.run_resampled(wl, 5000, 777, 4, "fp32")
    assert np.array_equal(a, b)
    # bins up to the first resampling are the plain run's, later ones differ
    assert np.array_equal(a[:3], plain[:3]) and not np.array_equal(a, plain)


def test_replica_study_structure(P):
    """The replica study on a small case: every interval reports its
    times, means and spreads, the runs without resampling match the plain
    runs' populations, and the same call twice gives the same numbers."""
    from paper_2608_14544_amd import branching, study
    wl = W.pyrazine_ci(n_traj=0, n_steps=20, cadence=2)
    res = branching.replica_spread(wl, 2000, 3, [None, 4], [5.0, 10.0], "fp32")
    assert set(res) == {"none", "every_4_steps"}
    for v in res.values():
        assert len(v["times"]) == len(v["mean"]) == len(v["replica_sd"]) == 2
        assert all(np.isfinite(v["mean"])) and all(x >= 0 for x in v["replica_sd"])
    ref = [study.population(P.run(wl, "fp32", n_traj=2000, traj_offset=k * 2000)[0])[0] for k in range(3)]
    t = np.arange(ref[0].size) * wl.run.cadence * wl.run.dt * wl.model.time_unit_fs
    i = int(np.argmin(np.abs(t - 10.0)))
    assert res["none"]["mean"][1] == pytest.approx(float(np.mean([r[i] for r in ref])), rel=1e-12)
    again = branching.replica_spread(wl, 2000, 3, [None, 4], [5.0, 10.0], "fp32")
    for k in res:
        assert res[k]["mean"] == again[k]["mean"] and res[k]["replica_sd"] == again[k]["replica_sd"]
