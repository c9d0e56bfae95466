"""Models with 5 to 8 electronic states on the general kernels (odd-even
transposition sort of the eigenpairs, couplings factored over rank 1 or
all N(N+1)/2 directions, at most 32 modes): binary64 walkers against the
oracle, binary32 ensembles, bitwise slicing and batching."""
import numpy as np
import pytest

import workloads as W
from test_gpu_batch import _assert_same, _batched, _solo
from parity import check_ensemble32, check_ensemble64, compare_walkers, gpu_run, oracle_run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2608_14544_amd as pkg
    pkg.load_library()
    return pkg


def _dense(index, n_states, n_modes, **kw):
    """A model whose couplings span all N(N+1)/2 directions: random_lvc's
    rank-1 couplings plus a dense symmetric part per mode."""
    wl = W.random_lvc(index, n_states=n_states, n_modes=n_modes, **kw)
    rng = np.random.Generator(np.random.Philox(key=[9, index]))
    k = wl.model.k.copy()
    for j in range(n_modes):
        a = rng.uniform(-0.05, 0.05, size=(n_states, n_states))
        k[j] += 0.5 * (a + a.T)
    wl.model = W.LVCModel(name=wl.model.name + "_dense", mass=wl.model.mass, omega=wl.model.omega,
                          v0=wl.model.v0, k=k)
    return wl


CASES = {
    "n5_m3": lambda: W.random_lvc(40, n_states=5, n_modes=3, n_traj=1000, n_steps=60, cadence=20),
    "n6_m8_dense": lambda: _dense(41, 6, 8, n_traj=600, n_steps=40, cadence=20),
    "n7_m12": lambda: W.random_lvc(42, n_states=7, n_modes=12, n_traj=500, n_steps=40, cadence=20),
    "n8_m4_dense": lambda: _dense(43, 8, 4, n_traj=400, n_steps=40, cadence=20),
    "n8_m32": lambda: W.random_lvc(44, n_states=8, n_modes=32, n_traj=300, n_steps=20, cadence=10),
}


def test_model_ranks(P):
    # rank-1 couplings, and dense ones that span as many directions as there
    # are modes (the kernels then keep all N(N+1)/2 directions)
    assert P.Model(CASES["n5_m3"]().model).rank == 1
    assert P.Model(CASES["n8_m4_dense"]().model).rank == 4
    assert P.Model(CASES["n6_m8_dense"]().model).rank == 8


@pytest.mark.parametrize("name", list(CASES))
def test_many_states_fp64_parity(P, name):
    wl = CASES[name]()
    out_g, st_g, s0_g, _ = gpu_run(P, wl)
    out_o, st_o, s0_o, _ = oracle_run(wl)
    compare_walkers(s0_g, s0_o, rtol=1e-10, label=name + " sample")
    flip = compare_walkers(st_g, st_o, rtol=1e-10, max_flip_frac=0.01, label=name)
    check_ensemble64(out_g, out_o, wl.run.n_traj, flip, st_g, st_o, label=name)


@pytest.mark.parametrize("name", ["n6_m8_dense", "n8_m4_dense"])
def test_many_states_fp32_ensemble(P, name):
    wl = CASES[name]()
    wl.run.n_traj = 20_000
    out_g, st_g, _, _ = gpu_run(P, wl, prec="fp32")
    out_o, st_o, _, _ = oracle_run(wl)
    check_ensemble32(out_g, out_o, wl.run.n_traj, label=name, g=st_g, o=st_o)


def test_many_states_linear_rule_and_ragged(P):
    wl = W.random_lvc(45, n_states=6, n_modes=5, n_traj=257, n_steps=30, cadence=7)
    out_g, st_g, _, _ = gpu_run(P, wl, scheme=1)
    out_o, st_o, _, fl_o = oracle_run(wl, scheme=1)
    assert np.array_equal(st_g["flags"] & 8, np.asarray(fl_o) & 8)
    flip = compare_walkers(st_g, st_o, rtol=1e-10, max_flip_frac=0.01, label="n6 linear ragged")
    check_ensemble64(out_g, out_o, wl.run.n_traj, flip, st_g, st_o, label="n6 linear ragged")


def test_many_states_slicing_and_batch_bitwise(P):
    wl = CASES["n8_m4_dense"]()
    for prec in ("fp64", "fp32"):
        out1, st1, _, _ = gpu_run(P, wl, prec=prec)
        out2, st2, _, _ = gpu_run(P, wl, prec=prec, split=[7, 13, 20])
        for k in st1:
            assert np.array_equal(st1[k], st2[k]), (prec, k)
        assert np.array_equal(out1, out2), prec
    mix = [
        (W.random_lvc(46, n_states=6, n_modes=10, n_traj=300, n_steps=30, cadence=10), "fp32", 0, 300),
        (_dense(47, 8, 5, n_traj=257, n_steps=20, cadence=10), "fp64", 1, 257),
        (W.random_lvc(48, n_states=4, n_modes=6, n_traj=500, n_steps=30, cadence=10), "fp32", 0, 500),
        (W.pyrazine_ci(n_traj=400, n_steps=30, cadence=10), "fp32", 0, 400),
    ]
    solo = [_solo(P, w, prec, scheme, T) for w, prec, scheme, T in mix]
    for slices in ((None,), (0.5, None)):
        got = _batched(P, mix, slices)
        for i, (a, b) in enumerate(zip(solo, got)):
            _assert_same(a, b, f"many-state batch item {i} slices {slices}")
