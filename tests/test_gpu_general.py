"""Parity of the general-N HIP kernels (N = 2..4 states, up to 128 modes)
with the FP64 CPU oracle, through the C ABI.

The general kernels finish each eigen-solve with Jacobi rotations started
from the previous frame, whereas the oracle starts every solve from the
identity: both converge to the same eigenpairs, so FP64 walkers agree to
rounding (tolerance as for the two-state path, 1e-10 relative, with a
small allowance for walkers whose transition decisions flip).
"""
import numpy as np
import pytest

import workloads as W
from parity import check_ensemble32, check_ensemble64, compare_walkers, gpu_run, oracle_run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2608_14544_amd as pkg
    pkg.load_library()
    return pkg


CASES = {
    "n3_m3": lambda: W.random_lvc(1, n_states=3, n_modes=3, n_traj=2000, n_steps=200, cadence=20),
    "n4_m5": lambda: W.random_lvc(2, n_states=4, n_modes=5, n_traj=2000, n_steps=200, cadence=20),
    "n2_m12": lambda: W.spin_boson_ohmic(kT=1.0, n_traj=2000, n_steps=200, cadence=20, n_modes=12),
    "n3_m20": lambda: W.random_lvc(5, n_states=3, n_modes=20, n_traj=1000, n_steps=100, cadence=20),
    "n4_m40": lambda: W.random_lvc(6, n_states=4, n_modes=40, n_traj=600, n_steps=60, cadence=20),
}


@pytest.mark.parametrize("name", list(CASES))
def test_general_fp64_parity(P, name):
    wl = CASES[name]()
    out_g, st_g, s0_g, _ = gpu_run(P, wl)
    out_o, st_o, s0_o, _ = oracle_run(wl)
    compare_walkers(s0_g, s0_o, rtol=1e-11, label=name + " sample")
    flip = compare_walkers(st_g, st_o, rtol=1e-10, max_flip_frac=0.005, label=name)
    check_ensemble64(out_g, out_o, wl.run.n_traj, flip, st_g, st_o, label=name)


@pytest.mark.parametrize("name", ["n3_m3", "n4_m5", "n2_m12"])
def test_general_fp32_ensemble(P, name):
    wl = CASES[name]()
    wl.run.n_traj = 40_000
    out_g, st_g, _, _ = gpu_run(P, wl, prec="fp32")
    out_o, st_o, _, _ = oracle_run(wl)
    check_ensemble32(out_g, out_o, wl.run.n_traj, label=name, g=st_g, o=st_o)


@pytest.mark.parametrize("T", [1, 255, 257])
def test_general_ragged(P, T):
    wl = W.random_lvc(3, n_states=3, n_modes=4, n_traj=T, n_steps=40, cadence=7)
    out_g, st_g, _, _ = gpu_run(P, wl)
    out_o, st_o, _, _ = oracle_run(wl)
    flip = compare_walkers(st_g, st_o, rtol=1e-10, label=f"general T={T}")
    check_ensemble64(out_g, out_o, T, flip, st_g, st_o, label=f"general T={T}")


def test_general_determinism_and_slicing(P):
    wl = W.random_lvc(4, n_states=4, n_modes=6, n_traj=3000, n_steps=90, cadence=10)
    for prec in ("fp64", "fp32"):
        out1, st1, _, _ = gpu_run(P, wl, prec=prec)
        out2, st2, _, _ = gpu_run(P, wl, prec=prec, split=[13, 27, 50])
        for k in st1:
            assert np.array_equal(st1[k], st2[k]), (prec, k)
        assert np.array_equal(out1, out2), prec


def _with_spectators(wl, n_extra):
    """The same model with ``n_extra`` uncoupled harmonic modes appended
    (K_j = 0, at rest at the origin on average)."""
    m = wl.model
    N = m.v0.shape[0]
    poly = None if m.poly is None else np.concatenate([m.poly, np.zeros((n_extra,) + m.poly.shape[1:])])
    lvc = W.LVCModel(name=m.name + "_spectators", mass=np.concatenate([m.mass, np.ones(n_extra)]),
                     omega=np.concatenate([m.omega, np.full(n_extra, float(m.omega.min()))]), v0=m.v0,
                     k=np.concatenate([m.k, np.zeros((n_extra, N, N))]), hbar=m.hbar, poly=poly)
    init = W.InitSpec(kT=wl.init.kT, q0=np.concatenate([wl.init.q0, np.zeros(n_extra)]), state=wl.init.state)
    return W.Workload(lvc, init, wl.run)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("kind", ["lvc3", "lvc4", "poly3"])
def test_four_mode_build_equals_eight_mode_build(P, prec, kind):
    """A 3-mode model runs the four-mode build; the same model with two
    uncoupled spectator modes runs the eight-mode build.  The spectators
    add exact zeros to every coupling coordinate and draw their own random
    numbers, so both builds give the same bits for the elements, weights,
    phases, frames and flags, the three coupled modes and every bin."""
    if kind == "poly3":
        wl = W.random_poly(44, n_states=3, n_modes=3, degree=3, n_traj=3000, n_steps=80, cadence=10)
    else:
        n_states = int(kind[-1])
        wl = W.random_lvc(40 + n_states, n_states=n_states, n_modes=3, n_traj=3000, n_steps=80, cadence=10)
    ws = _with_spectators(wl, 2)
    assert P.Model(wl.model).n_modes == 3 and P.Model(ws.model).n_modes == 5
    out_a, st_a, _, _ = gpu_run(P, wl, prec=prec)
    out_b, st_b, _, _ = gpu_run(P, ws, prec=prec)
    for k in ("a", "b", "w", "phase", "U", "flags"):
        assert np.array_equal(st_a[k], st_b[k]), (prec, k)
    assert np.array_equal(st_a["q"], st_b["q"][:, :3]) and np.array_equal(st_a["p"], st_b["p"][:, :3]), prec
    assert np.array_equal(out_a, out_b), prec


def _crossing_model(coupling=5e-5):
    """Three states whose diagonal energies cross as mode 0 moves, with a
    weak coupling between states 0 and 1: the adiabatic gap of that pair
    falls far below the binary32 threshold around the crossing seam."""
    v0 = np.array([[0.05, coupling, 0.0], [coupling, -0.05, 0.02], [0.0, 0.02, 0.4]])
    k = np.zeros((3, 3, 3))
    k[0] = np.diag([-0.3, 0.3, 0.0])
    k[1] = np.diag([0.05, -0.05, 0.1])
    k[2] = [[0.0, 0.0, 0.01], [0.0, 0.0, 0.0], [0.01, 0.0, 0.0]]
    lvc = W.LVCModel(name="crossing3", mass=np.ones(3), omega=np.array([0.2, 0.5, 0.8]), v0=v0, k=k)
    init = W.InitSpec(kT=0.05, q0=np.zeros(3), state=0)
    return W.Workload(lvc, init, W.RunSpec(40_000, 120, 0.05, 20, 17))


def test_general_fp32_near_degenerate(P):
    """The binary32 path refines the closest pair in binary64 below the gap
    threshold; ensemble averages stay within 1e-3 * max(1, rms) of the oracle."""
    wl = _crossing_model()
    out_g, st_g, _, _ = gpu_run(P, wl, prec="fp32")
    out_o, st_o, _, _ = oracle_run(wl)
    refined = (st_g["flags"] & 4) != 0
    print("refined walkers", refined.mean(), flush=True)
    assert refined.mean() > 0.002  # the refinement ran for a few hundred walkers
    check_ensemble32(out_g, out_o, wl.run.n_traj, label="crossing3", g=st_g, o=st_o)


@pytest.mark.parametrize("name", ["n3_m3", "n4_m5"])
def test_general_linear_rule_parity(P, name):
    """The linear transition rule (with its fallback to the normalized one
    when S >= 1) on the general kernels, binary64, per walker."""
    wl = CASES[name]()
    out_g, st_g, _, _ = gpu_run(P, wl, scheme=1)
    out_o, st_o, _, fl_o = oracle_run(wl, scheme=1)
    assert np.array_equal(st_g["flags"] & 8, np.asarray(fl_o) & 8)  # same walkers fell back
    flip = compare_walkers(st_g, st_o, rtol=1e-10, max_flip_frac=0.005, label=name + " linear")
    check_ensemble64(out_g, out_o, wl.run.n_traj, flip, st_g, st_o, label=name + " linear")


@pytest.mark.parametrize("n_states", [2, 3, 4])
def test_adiabatic_initial_state(P, n_states):
    """Start in an adiabatic state (element (k, k), weight 1) on both kernel
    families: samples and propagated walkers against the oracle."""
    if n_states == 2:
        wl = W.pyrazine_ci(n_traj=2000, n_steps=60, cadence=10)
    else:
        wl = W.random_lvc(30 + n_states, n_states=n_states, n_modes=6, n_traj=2000, n_steps=60, cadence=10)
    wl.init.basis = W.INIT_ADIABATIC
    wl.init.state = n_states - 1
    out_g, st_g, s0_g, _ = gpu_run(P, wl)
    out_o, st_o, s0_o, _ = oracle_run(wl)
    assert np.all(s0_g["a"] == n_states - 1) and np.all(s0_g["b"] == n_states - 1) and np.all(s0_g["w"] == 1.0)
    compare_walkers(s0_g, s0_o, rtol=1e-11, label=f"adiabatic N{n_states} sample")
    flip = compare_walkers(st_g, st_o, rtol=1e-10, max_flip_frac=0.005, label=f"adiabatic N{n_states}")
    check_ensemble64(out_g, out_o, wl.run.n_traj, flip, st_g, st_o, label=f"adiabatic N{n_states}")
