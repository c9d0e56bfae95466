"""Models with cross-mode bilinear terms (V(q) += sum_p q_i q_j B_p, with or
without higher powers of each mode) on the general kernels: binary64
walkers against the oracle, binary32 ensembles, the linear rule, bitwise
slicing and batching, ragged sizes and the full-size workload of the bench.

The device splits each term as ((q_i + q_j)^2 - (q_i - q_j)^2) / 4, the
oracle evaluates q_i q_j B_p directly: the two agree to rounding, so the
binary64 tolerances are those of the other general-kernel models.  Models
needing up to 4, 8 or 16 squared combinations run the builds for 4, 8 or
16; the cases cover all three, and both ways of forming the combinations
(per term, and per slot from the eigendecomposition of the slot's mode-mode
matrix, for models where every pair of modes is coupled)."""
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
    "pyrazine_bilinear": lambda: W.pyrazine_bilinear(n_traj=2000, n_steps=60, cadence=6),
    "n2_m3_p2": lambda: W.random_bilinear(0, n_states=2, n_modes=3, n_pairs=2),
    "n3_m5_p4_d3": lambda: W.random_bilinear(1, n_states=3, n_modes=5, n_pairs=4, degree=3),
    "n4_m4_p3_d4": lambda: W.random_bilinear(2, n_states=4, n_modes=4, n_pairs=3, degree=4),
    "n3_m20_p4": lambda: W.random_bilinear(5, n_states=3, n_modes=20, n_pairs=4, n_traj=1000),
    "n3_m6_p1_d3": lambda: W.random_bilinear(11, n_states=3, n_modes=6, n_pairs=1, degree=3),
    "n2_m6_p8_d2": lambda: W.random_bilinear(12, n_states=2, n_modes=6, n_pairs=8),
    "n4_m16_p6_d4": lambda: W.random_bilinear(13, n_states=4, n_modes=16, n_pairs=6, degree=4, n_traj=1000),
    # every pair of modes coupled: the slot eigendecompositions need fewer combinations
    "n2_m5_all_d3": lambda: W.random_bilinear(15, n_states=2, n_modes=5, all_pairs=True, degree=3),
    "n2_m8_all_shared": lambda: W.random_bilinear(16, n_states=2, n_modes=8, all_pairs=True, shared=True),
}


def test_model_pairs_and_degree(P):
    m = P.Model(W.random_bilinear(1, n_states=3, n_modes=5, n_pairs=4, degree=3).model)
    assert m.n_pairs == 4 and m.degree == 3
    lin = W.pyrazine_ci().model
    only = W.LVCModel(name="bil_only", mass=lin.mass, omega=lin.omega, v0=lin.v0, k=lin.k, hbar=lin.hbar,
                      bilinear=[(0, 2, np.diag([0.01, -0.01]))])
    m2 = P.Model(only)
    assert m2.n_pairs == 1 and m2.degree == 2
    assert P.Model(W.pyrazine_qvc().model).n_pairs == 0


@pytest.mark.parametrize("name", list(CASES))
def test_bilinear_fp64_parity(P, name):
    wl = CASES[name]()
    out_g, st_g, s0_g, _ = gpu_run(P, wl)
    out_o, st_o, s0_o, _ = oracle_run(wl)
    compare_walkers(s0_g, s0_o, rtol=1e-11, label=name + " sample")
    flip = compare_walkers(st_g, st_o, rtol=1e-10, max_flip_frac=0.005, label=name)
    check_ensemble64(out_g, out_o, wl.run.n_traj, flip, st_g, st_o, label=name)


def test_bilinear_only_model_fp64_parity(P):
    """Bilinear terms without higher powers (the kernels take A = 0)."""
    base = W.pyrazine_ci(n_traj=1500, n_steps=60, cadence=6)
    lin = base.model
    only = W.LVCModel(name="bil_only", mass=lin.mass, omega=lin.omega, v0=lin.v0, k=lin.k, hbar=lin.hbar,
                      time_unit_fs=lin.time_unit_fs,
                      bilinear=[(0, 1, np.diag([-0.01, 0.012])), (2, 0, np.array([[0.0, 0.015], [0.015, 0.0]]))])
    wl = W.Workload(only, base.init, base.run)
    out_g, st_g, _, _ = gpu_run(P, wl)
    out_o, st_o, _, _ = oracle_run(wl)
    flip = compare_walkers(st_g, st_o, rtol=1e-10, max_flip_frac=0.005, label="bilinear only")
    check_ensemble64(out_g, out_o, wl.run.n_traj, flip, st_g, st_o, label="bilinear only")


@pytest.mark.parametrize("name", ["pyrazine_bilinear", "n4_m4_p3_d4"])
def test_bilinear_fp32_ensemble(P, name):
    wl = CASES[name]()
    wl.run.n_traj = 40_000
    out_g, st_g, _, _ = gpu_run(P, wl, prec="fp32")
    out_o, st_o, _, _ = oracle_run(wl)
    check_ensemble32(out_g, out_o, wl.run.n_traj, label=name, g=st_g, o=st_o)


def test_bilinear_linear_rule(P):
    wl = CASES["n3_m5_p4_d3"]()
    out_g, st_g, _, _ = gpu_run(P, wl, scheme=1)
    out_o, st_o, _, fl_o = oracle_run(wl, scheme=1)
    assert np.array_equal(st_g["flags"] & 8, np.asarray(fl_o) & 8)
    flip = compare_walkers(st_g, st_o, rtol=1e-10, max_flip_frac=0.005, label="bilinear linear")
    check_ensemble64(out_g, out_o, wl.run.n_traj, flip, st_g, st_o, label="bilinear linear")


@pytest.mark.parametrize("T", [0, 1, 255, 257])
def test_bilinear_empty_and_ragged(P, T):
    wl = W.random_bilinear(6, n_states=3, n_modes=4, n_pairs=2, n_traj=T, n_steps=40, cadence=7)
    out_g, st_g, _, _ = gpu_run(P, wl)
    if T == 0:
        assert out_g is None and st_g["w"].size == 0
        return
    out_o, st_o, _, _ = oracle_run(wl)
    flip = compare_walkers(st_g, st_o, rtol=1e-10, label=f"bilinear T={T}")
    check_ensemble64(out_g, out_o, T, flip, st_g, st_o, label=f"bilinear T={T}")


def test_bilinear_slicing_bitwise(P):
    wl = W.random_bilinear(7, n_states=4, n_modes=6, n_pairs=4, degree=4, n_traj=3000, n_steps=90, cadence=10)
    for prec in ("fp64", "fp32"):
        out1, st1, _, _ = gpu_run(P, wl, prec=prec)
        out2, st2, _, _ = gpu_run(P, wl, prec=prec, split=[13, 27, 50])
        for k in st1:
            assert np.array_equal(st1[k], st2[k]), (prec, k)
        assert np.array_equal(out1, out2), prec


def test_bilinear_in_mixed_batch_bitwise(P):
    mix = [
        (W.pyrazine_bilinear(n_traj=700, n_steps=60, cadence=6), "fp32", 0, 700),
        (W.pyrazine_qvc(n_traj=500, n_steps=60, cadence=6), "fp32", 0, 500),
        (W.random_bilinear(8, n_states=3, n_modes=5, n_pairs=3, degree=3, n_traj=300, n_steps=40, cadence=10),
         "fp64", 1, 300),
        (W.random_bilinear(9, n_states=4, n_modes=20, n_pairs=4, n_traj=257, n_steps=30, cadence=10), "fp32", 0, 257),
        (W.random_lvc(8, n_states=3, n_modes=4, n_traj=400, n_steps=40, cadence=10), "fp32", 0, 400),
        (W.random_bilinear(14, n_states=3, n_modes=8, n_pairs=7, degree=3, n_traj=300, n_steps=40, cadence=10),
         "fp32", 0, 300),
    ]
    solo = [_solo(P, wl, prec, scheme, T) for wl, prec, scheme, T in mix]
    for slices in ((None,), (0.5, None)):
        got = _batched(P, mix, slices)
        for i, (a, b) in enumerate(zip(solo, got)):
            _assert_same(a, b, f"bilinear batch item {i} slices {slices}")


def test_bilinear_32_modes(P):
    """The largest mode bucket of bilinear models (32 padded modes)."""
    wl = W.random_bilinear(10, n_states=3, n_modes=30, n_pairs=4, degree=4, n_traj=300, n_steps=30, cadence=10)
    out_g, st_g, _, _ = gpu_run(P, wl)
    out_o, st_o, _, _ = oracle_run(wl)
    flip = compare_walkers(st_g, st_o, rtol=1e-10, max_flip_frac=0.01, label="bilinear M30")
    check_ensemble64(out_g, out_o, wl.run.n_traj, flip, st_g, st_o, label="bilinear M30")


def test_bilinear_bench_configuration_full_size(P):
    """The bench's bilinear workload at full size (pyrazine_bilinear, 1e7
    walkers, 200 steps, one launch): binary64 walkers sampled across the
    ensemble recomputed one by one by the oracle, and the binary32 run's
    populations within 2e-3 of the binary64 run's while resolved."""
    import torch
    wl = W.pyrazine_bilinear(n_traj=10_000_000, n_steps=200, cadence=10)
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
    compare_walkers(g, o, rtol=1e-10, max_flip_frac=0.01, label="pyrazine_bilinear 1e7 sampled")
    # binary32 against binary64 on every bin
    check_ensemble32(outs["fp32"], outs["fp64"], r.n_traj, label="pyrazine_bilinear fp32 vs fp64")
