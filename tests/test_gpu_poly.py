"""Models with separable higher powers of each mode (V(q) = V0 + sum_j sum_k
q_j^k A_jk, k <= 4) on the general kernels: binary64 walkers against the
oracle, binary32 ensembles, bitwise slicing and batching, the largest mode
buckets."""
import numpy as np
import pytest

import workloads as W
from test_gpu_batch import _assert_same, _batched, _solo
from parity import (check_ensemble32, check_ensemble64, compare_walkers, gpu_run, oracle_run, oracle_walkers,
                    sample_ids, sampled_state)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2608_14544_amd as pkg
    pkg.load_library()
    return pkg


CASES = {
    "qvc_pyrazine": lambda: W.pyrazine_qvc(n_traj=2000, n_steps=60, cadence=6),
    "n2_m3_d2": lambda: W.random_poly(0, n_states=2, n_modes=3, degree=2),
    "n3_m4_d3": lambda: W.random_poly(1, n_states=3, n_modes=4, degree=3),
    "n4_m3_d4": lambda: W.random_poly(2, n_states=4, n_modes=3, degree=4),
    "n3_m12_d4": lambda: W.random_poly(4, n_states=3, n_modes=12, degree=4, rank_full=False, n_traj=1000),
}


def test_model_degree_and_rank(P):
    m = P.Model(W.random_poly(2, n_states=4, n_modes=3, degree=4).model)
    assert m.degree == 4 and m.rank == 10
    m2 = P.Model(W.pyrazine_qvc().model)
    assert m2.degree == 4 and 1 <= m2.rank <= 3
    assert P.Model(W.pyrazine_ci().model).degree == 1


@pytest.mark.parametrize("name", list(CASES))
def test_poly_fp64_parity(P, name):
    wl = CASES[name]()
    out_g, st_g, s0_g, _ = gpu_run(P, wl)
    out_o, st_o, s0_o, _ = oracle_run(wl)
    compare_walkers(s0_g, s0_o, rtol=1e-11, label=name + " sample")
    flip = compare_walkers(st_g, st_o, rtol=1e-10, max_flip_frac=0.005, label=name)
    check_ensemble64(out_g, out_o, wl.run.n_traj, flip, st_g, st_o, label=name)


@pytest.mark.parametrize("name", ["qvc_pyrazine", "n4_m3_d4"])
def test_poly_fp32_ensemble(P, name):
    wl = CASES[name]()
    wl.run.n_traj = 40_000
    out_g, st_g, _, _ = gpu_run(P, wl, prec="fp32")
    out_o, st_o, _, _ = oracle_run(wl)
    check_ensemble32(out_g, out_o, wl.run.n_traj, label=name, g=st_g, o=st_o)


def test_poly_linear_rule(P):
    wl = CASES["n3_m4_d3"]()
    out_g, st_g, _, _ = gpu_run(P, wl, scheme=1)
    out_o, st_o, _, fl_o = oracle_run(wl, scheme=1)
    assert np.array_equal(st_g["flags"] & 8, np.asarray(fl_o) & 8)
    flip = compare_walkers(st_g, st_o, rtol=1e-10, max_flip_frac=0.005, label="poly linear")
    check_ensemble64(out_g, out_o, wl.run.n_traj, flip, st_g, st_o, label="poly linear")


def test_poly_slicing_bitwise(P):
    wl = W.random_poly(5, n_states=4, n_modes=6, degree=4, n_traj=3000, n_steps=90, cadence=10)
    for prec in ("fp64", "fp32"):
        out1, st1, _, _ = gpu_run(P, wl, prec=prec)
        out2, st2, _, _ = gpu_run(P, wl, prec=prec, split=[13, 27, 50])
        for k in st1:
            assert np.array_equal(st1[k], st2[k]), (prec, k)
        assert np.array_equal(out1, out2), prec


def test_poly_in_mixed_batch_bitwise(P):
    mix = [
        (W.pyrazine_qvc(n_traj=700, n_steps=60, cadence=6), "fp32", 0, 700),
        (W.pyrazine_ci(n_traj=500, n_steps=60, cadence=6), "fp32", 0, 500),
        (W.random_poly(6, n_states=3, n_modes=5, degree=3, n_traj=300, n_steps=40, cadence=10), "fp64", 1, 300),
        (W.random_poly(7, n_states=4, n_modes=20, degree=4, n_traj=257, n_steps=30, cadence=10), "fp32", 0, 257),
        (W.random_lvc(8, n_states=3, n_modes=4, n_traj=400, n_steps=40, cadence=10), "fp32", 0, 400),
    ]
    solo = [_solo(P, wl, prec, scheme, T) for wl, prec, scheme, T in mix]
    for slices in ((None,), (0.5, None)):
        got = _batched(P, mix, slices)
        for i, (a, b) in enumerate(zip(solo, got)):
            _assert_same(a, b, f"poly batch item {i} slices {slices}")


@pytest.mark.parametrize("n_states,n_modes", [(2, 40), (3, 100)])
def test_poly_large_mode_buckets(P, n_states, n_modes):
    """64 and 128 padded modes: binary64 against the oracle."""
    wl = W.random_poly(9 + n_states, n_states=n_states, n_modes=n_modes, degree=4, n_traj=300, n_steps=30,
                       cadence=10, rank_full=False)
    out_g, st_g, _, _ = gpu_run(P, wl)
    out_o, st_o, _, _ = oracle_run(wl)
    flip = compare_walkers(st_g, st_o, rtol=1e-10, max_flip_frac=0.01, label=f"poly N{n_states} M{n_modes}")
    check_ensemble64(out_g, out_o, wl.run.n_traj, flip, st_g, st_o, label=f"poly N{n_states} M{n_modes}")


def test_poly_bench_configuration_full_size(P):
    """The bench's polynomial workload at full size (pyrazine_qvc, 1e7
    walkers, 200 steps, one launch): binary64 walkers sampled across the
    ensemble recomputed one by one by the oracle, and the binary32 run's
    populations within 2e-3 of the binary64 run's while resolved."""
    import torch
    wl = W.pyrazine_qvc(n_traj=10_000_000, n_steps=200, cadence=10)
    r = wl.run
    model = P.Model(wl.model)
    outs = {}
    for prec in ("fp64", "fp32"):
        ens = P.Ensemble(model, r.n_traj, prec, zero=False)
        part = P.Partials(model, r.n_traj, r.n_out)
        P.qcl_sample_initial(model, wl.init, r.seed, ens, part)
        P.qcl_propagate(model, ens, r.dt, r.n_steps, r.cadence, r.seed, part)
        outs[prec] = P.qcl_reduce_observables(model, part, r.n_traj).cpu().numpy()
        if prec == "fp64":
            ids = sample_ids(r.n_traj, 120, seed=3, extra=[1 << 20, 5_555_555])
            g = sampled_state(ens, ids)
        del ens, part
        torch.cuda.empty_cache()
    o = oracle_walkers(wl, ids)
    compare_walkers(g, o, rtol=1e-10, max_flip_frac=0.01, label="pyrazine_qvc 1e7 sampled")
    # binary32 against binary64 on every bin
    check_ensemble32(outs["fp32"], outs["fp64"], r.n_traj, label="pyrazine_qvc fp32 vs fp64")


@pytest.mark.parametrize("T", [0, 1, 255, 257])
def test_poly_empty_and_ragged(P, T):
    wl = W.random_poly(30, n_states=3, n_modes=5, degree=4, n_traj=T, n_steps=40, cadence=7)
    out_g, st_g, _, _ = gpu_run(P, wl)
    if T == 0:
        assert out_g is None and st_g["w"].size == 0
        return
    out_o, st_o, _, _ = oracle_run(wl)
    flip = compare_walkers(st_g, st_o, rtol=1e-10, label=f"poly T={T}")
    check_ensemble64(out_g, out_o, T, flip, st_g, st_o, label=f"poly T={T}")


def test_poly_largest_bucket_n4_m128(P):
    """Four states, 128 modes, quartic: the largest polynomial class (its
    binary64 build spills to scratch), against the oracle, both precisions."""
    wl = W.random_poly(31, n_states=4, n_modes=128, degree=4, n_traj=256, n_steps=20, cadence=10,
                       rank_full=False)
    out_g, st_g, _, _ = gpu_run(P, wl)
    out_o, st_o, _, _ = oracle_run(wl)
    flip = compare_walkers(st_g, st_o, rtol=1e-10, max_flip_frac=0.02, label="poly N4 M128")
    check_ensemble64(out_g, out_o, wl.run.n_traj, flip, st_g, st_o, label="poly N4 M128")
    out32, st32, _, _ = gpu_run(P, wl, prec="fp32")
    assert np.all(np.isfinite(st32["w"])) and np.all(np.isfinite(out32))


def test_poly_two_state_closed_form_slicing_and_linear_rule(P):
    """Two states, at most 8 modes: the closed-form kernels with polynomial
    dl, cc and Vbar; bitwise slicing in both precisions and the linear
    rule against the oracle."""
    wl = W.pyrazine_qvc(n_traj=3000, n_steps=90, cadence=10)
    for prec in ("fp64", "fp32"):
        out1, st1, _, _ = gpu_run(P, wl, prec=prec)
        out2, st2, _, _ = gpu_run(P, wl, prec=prec, split=[13, 27, 50])
        for k in st1:
            assert np.array_equal(st1[k], st2[k]), (prec, k)
        assert np.array_equal(out1, out2), prec
    wl = W.random_poly(8, n_states=2, n_modes=8, degree=4, n_traj=1500, n_steps=60, cadence=10)
    out_g, st_g, _, _ = gpu_run(P, wl, scheme=1)
    out_o, st_o, _, fl_o = oracle_run(wl, scheme=1)
    assert np.array_equal(st_g["flags"] & 8, np.asarray(fl_o) & 8)
    flip = compare_walkers(st_g, st_o, rtol=1e-10, max_flip_frac=0.005, label="poly n2 m8 linear")
    check_ensemble64(out_g, out_o, wl.run.n_traj, flip, st_g, st_o, label="poly n2 m8 linear")
