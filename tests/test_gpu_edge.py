"""Edge cases of the GPU path against the oracle: a model that is exactly
degenerate everywhere, the largest mode bucket (up to 128 modes) of the
general kernels, and the headline model at 1e8 walkers (global walker ids
above 2^26)."""
import numpy as np
import pytest

import workloads as W
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


@pytest.mark.parametrize("n_states,n_modes", [(2, 1), (3, 2), (4, 12)])
def test_exactly_degenerate_model(P, n_states, n_modes):
    """V = 0 everywhere: every walker meets a zero gap, is flagged degenerate
    and non-finite, and is left out of the sums, as in the oracle; the
    reduction reports them (QCL_ERR_NONFINITE, with the count per bin from
    the asynchronous call)."""
    import torch
    lvc = W.LVCModel(name="flat", mass=np.ones(n_modes), omega=np.ones(n_modes),
                     v0=np.zeros((n_states, n_states)), k=np.zeros((n_modes, n_states, n_states)))
    wl = W.Workload(lvc, W.InitSpec(kT=0.5, q0=np.zeros(n_modes), state=0), W.RunSpec(300, 20, 0.05, 10, 5))
    for prec in ("fp64", "fp32"):
        out_g, st_g, _, ens = gpu_run(P, wl, prec=prec, expect_excluded=True)
        out_o, st_o, _, fl_o = oracle_run(wl)
        assert np.array_equal(st_g["flags"] & 3, np.asarray(fl_o) & 3), prec
        assert np.all(np.isfinite(out_g)), prec
        assert np.array_equal(out_g[1:], out_o[1:]), prec  # all walkers excluded: zeros
        # the per-bin counts: bin 0 (sampled state, finite) none, every later bin all 300
        r = wl.run
        model = P.Model(wl.model)
        e2 = P.Ensemble(model, r.n_traj, prec)
        part = P.Partials(model, r.n_traj, r.n_out)
        P.qcl_sample_initial(model, wl.init, r.seed, e2, part)
        P.qcl_propagate(model, e2, r.dt, r.n_steps, r.cadence, r.seed, part)
        _, excl = P.qcl_reduce_observables_async(model, part, r.n_traj)
        torch.cuda.synchronize()
        assert excl.cpu().tolist() == [0] + [r.n_traj] * (r.n_out - 1), (prec, excl.cpu().tolist())


@pytest.mark.parametrize("n_states,n_modes", [(3, 100), (4, 128)])
def test_general_largest_mode_bucket(P, n_states, n_modes):
    wl = W.random_lvc(20 + n_states, n_states=n_states, n_modes=n_modes, n_traj=300, n_steps=30, cadence=10)
    out_g, st_g, s0_g, _ = gpu_run(P, wl)
    out_o, st_o, s0_o, _ = oracle_run(wl)
    compare_walkers(s0_g, s0_o, rtol=1e-11, label=f"N{n_states} M{n_modes} sample")
    flip = compare_walkers(st_g, st_o, rtol=1e-10, max_flip_frac=0.01, label=f"N{n_states} M{n_modes}")
    check_ensemble64(out_g, out_o, wl.run.n_traj, flip, st_g, st_o, label=f"N{n_states} M{n_modes}")
    out32, st32, _, _ = gpu_run(P, wl, prec="fp32")
    check_ensemble32(out32, out_o, wl.run.n_traj, label=f"N{n_states} M{n_modes} fp32", g=st32, o=st_o)


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
    ids = sample_ids(r.n_traj, 120, seed=8, extra=[1 << 24, (1 << 26) + 3, 77_777_777])
    g = sampled_state(ens, ids)
    del ens, part
    torch.cuda.empty_cache()
    o = oracle_walkers(wl, ids)
    compare_walkers(g, o, rtol=1e-10, max_flip_frac=0.01, label="pyrazine 1e8 sampled")
