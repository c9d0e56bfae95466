"""Edge cases of the GPU path against the oracle: a model that is exactly
degenerate everywhere, the largest mode bucket (up to 128 modes) of the
general kernels, and the headline model at 1e8 walkers (global walker ids
above 2^26)."""
import numpy as np
import pytest

import oracle.core as oc
import workloads as W
from test_gpu_parity import _oracle_state, compare_walkers, ensemble_close, gpu_run, oracle_run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2608_14544_amd as pkg
    pkg.load_library()
    return pkg


@pytest.mark.parametrize("n_states,n_modes", [(2, 1), (3, 2), (4, 12)])
def test_exactly_degenerate_model(P, n_states, n_modes):
    """V = 0 everywhere: every walker meets a zero gap, is flagged degenerate
    and non-finite, and is left out of the sums, as in the oracle."""
    lvc = W.LVCModel(name="flat", mass=np.ones(n_modes), omega=np.ones(n_modes),
                     v0=np.zeros((n_states, n_states)), k=np.zeros((n_modes, n_states, n_states)))
    wl = W.Workload(lvc, W.InitSpec(kT=0.5, q0=np.zeros(n_modes), state=0), W.RunSpec(300, 20, 0.05, 10, 5))
    for prec in ("fp64", "fp32"):
        out_g, st_g, _, _ = gpu_run(P, wl, prec=prec)
        out_o, st_o, _, fl_o = oracle_run(wl)
        assert np.array_equal(st_g["flags"] & 3, np.asarray(fl_o) & 3), prec
        assert np.all(np.isfinite(out_g)), prec
        assert np.array_equal(out_g[1:], out_o[1:]), prec  # all walkers excluded: zeros


@pytest.mark.parametrize("n_states,n_modes", [(3, 100), (4, 128)])
def test_general_largest_mode_bucket(P, n_states, n_modes):
    wl = W.random_lvc(20 + n_states, n_states=n_states, n_modes=n_modes, n_traj=300, n_steps=30, cadence=10)
    out_g, st_g, s0_g, _ = gpu_run(P, wl)
    out_o, st_o, s0_o, _ = oracle_run(wl)
    compare_walkers(s0_g, s0_o, rtol=1e-11, label=f"N{n_states} M{n_modes} sample")
    nflip = compare_walkers(st_g, st_o, rtol=1e-9, max_flip_frac=0.01, label=f"N{n_states} M{n_modes}")
    if nflip == 0:
        assert ensemble_close(out_g, out_o, wl.run.n_traj)
    out32, _, _, _ = gpu_run(P, wl, prec="fp32")
    d = np.abs(out32[..., :2] - out_o[..., :2])
    se = np.maximum(out_o[..., 2:], 1e-300)
    assert np.all((d <= 1e-3) | (d <= 3 * se))


def test_headline_model_at_1e8_walkers(P):
    """The pyrazine-like model at 1e8 walkers (the top of the scaling sweep),
    binary64: sampled walkers, among them ids above 2^26 and the last one,
    recomputed one by one by the oracle."""
    import torch
    wl = W.pyrazine_ci(n_traj=100_000_000, n_steps=200)
    r = wl.run
    model = P.Model(wl.model)
    ens = P.Ensemble(model, r.n_traj, "fp64", zero=False)
    part = P.Partials(model, r.n_traj, r.n_out)
    P.qcl_sample_initial(model, wl.init, r.seed, ens, part)
    P.qcl_propagate(model, ens, r.dt, r.n_steps, r.cadence, r.seed, part)
    torch.cuda.synchronize()
    t = ens.tensors()
    ids = np.array([0, 1 << 24, (1 << 26) + 3, 77_777_777, r.n_traj - 257, r.n_traj - 1])
    g = {"q": t["q"][:, ids].cpu().numpy().T, "p": t["p"][:, ids].cpu().numpy().T,
         "U": t["u"][:, ids].cpu().numpy().T.reshape(-1, 2, 2), "w": t["w"][ids].cpu().numpy(),
         "phase": t["phase"][ids].cpu().numpy(), "a": t["a"][ids].cpu().numpy().astype(np.int32),
         "b": t["b"][ids].cpu().numpy().astype(np.int32)}
    del ens, part
    torch.cuda.empty_cache()
    m = oc.Model(wl.model)
    o = {k: [] for k in g}
    for i in ids:
        st, _ = oc.sample(m, wl.init, r.seed, 1, traj_offset=int(i))
        oc.propagate(m, st, r.dt, r.n_steps, r.cadence, r.seed, r.n_out)
        for k, v in _oracle_state(st).items():
            o[k].append(v[0])
    o = {k: np.array(v) for k, v in o.items()}
    compare_walkers(g, o, rtol=1e-8, max_flip_frac=0.2, label="pyrazine 1e8 sampled")
