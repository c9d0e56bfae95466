"""Batched propagation (one persistent launch per kernel class over
(instance, tile) work items): every instance's walkers and observables
must be bitwise those of its solo qcl_propagate run, whatever else shares
the launch, and a batch must agree with the FP64 oracle like a solo run."""
import numpy as np
import pytest

import workloads as W
from parity import (check_ensemble32, check_ensemble64, compare_walkers, oracle_run, oracle_walkers, sample_ids,
                    sampled_state)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2608_14544_amd as pkg
    pkg.load_library()
    return pkg


def _mix():
    """Uneven instances covering every kernel family: two-state closed form
    (1, 3 and 8 modes), general N = 2 (12 modes), 3 and 4 states, both
    precisions and both transition rules, ragged walker counts."""
    return [
        (W.spin_boson_1mode(), "fp64", 0, 700),
        (W.pyrazine_ci(n_traj=1000, n_steps=120, cadence=10), "fp32", 0, 1000),
        (W.pyrazine_ci(n_traj=257, n_steps=77, cadence=7, seed=11), "fp32", 0, 257),
        (W.random_lvc(7, n_states=2, n_modes=8, n_traj=513, n_steps=90, cadence=9), "fp64", 1, 513),
        (W.spin_boson_ohmic(kT=1.0, n_traj=300, n_steps=60, cadence=20, n_modes=12), "fp64", 0, 300),
        (W.random_lvc(8, n_states=3, n_modes=4, n_traj=900, n_steps=100, cadence=10), "fp32", 0, 900),
        (W.random_lvc(9, n_states=3, n_modes=4, n_traj=64, n_steps=30, cadence=10), "fp32", 0, 64),
        (W.random_lvc(10, n_states=4, n_modes=6, n_traj=1, n_steps=50, cadence=25), "fp64", 0, 1),
        (W.random_lvc(11, n_states=4, n_modes=20, n_traj=400, n_steps=40, cadence=20), "fp64", 1, 400),
    ]


def _setup(P, wl, prec, T):
    r = wl.run
    model = P.Model(wl.model)
    ens = P.Ensemble(model, T, prec)
    part = P.Partials(model, T, r.n_steps // r.cadence + 1)
    P.qcl_sample_initial(model, wl.init, r.seed, ens, part)
    return model, ens, part


def _solo(P, wl, prec, scheme, T):
    model, ens, part = _setup(P, wl, prec, T)
    r = wl.run
    P.qcl_propagate(model, ens, r.dt, r.n_steps, r.cadence, r.seed, part, scheme)
    out = P.qcl_reduce_observables(model, part, T)
    return out.cpu().numpy(), ens.to_numpy()


def _batched(P, mix, slices=(None,)):
    import torch
    runs = [(_setup(P, wl, prec, T), wl, scheme, T) for wl, prec, scheme, T in mix]
    ws = P.Workspace()
    done = [0] * len(runs)
    for frac in slices:
        jobs = []
        for i, ((model, ens, part), wl, scheme, T) in enumerate(runs):
            r = wl.run
            n = r.n_steps - done[i] if frac is None else min(r.n_steps - done[i], int(r.n_steps * frac))
            done[i] += n
            jobs.append(P.BatchJob(model, ens, part, r.dt, n, r.cadence, r.seed, scheme))
        P.qcl_propagate_batch(jobs, ws)
    outs = []
    for i, ((model, ens, part), wl, scheme, T) in enumerate(runs):
        assert done[i] == wl.run.n_steps and ens.step == wl.run.n_steps
        outs.append((P.qcl_reduce_observables(model, part, T).cpu().numpy(), ens.to_numpy()))
    torch.cuda.synchronize()
    return outs


def _assert_same(a, b, label):
    out_a, st_a = a
    out_b, st_b = b
    for k in st_a:
        assert np.array_equal(st_a[k], st_b[k]), (label, k)
    assert np.array_equal(out_a, out_b), label


def test_batch_bitwise_equals_solo(P):
    mix = _mix()
    solo = [_solo(P, wl, prec, scheme, T) for wl, prec, scheme, T in mix]
    batch = _batched(P, mix)
    for i, (s, b) in enumerate(zip(solo, batch)):
        _assert_same(s, b, f"item {i}")


def _classed_model(n_modes, mt, seed):
    """A two-state linear model whose first ``mt`` modes only tune the gap
    (K_01 = 0) and whose other modes only couple the states
    (K_00 = K_11 = 0), with a constant coupling in V0."""
    rng = np.random.default_rng(seed)
    k = np.zeros((n_modes, 2, 2))
    for j in range(n_modes):
        if j < mt:
            k[j] = np.diag(rng.uniform(-0.6, 0.6, 2))
        else:
            c = rng.uniform(-0.4, 0.4)
            k[j] = [[0.0, c], [c, 0.0]]
    model = W.LVCModel(name=f"classes_{mt}_of_{n_modes}", mass=rng.uniform(0.5, 2.0, n_modes),
                       omega=rng.uniform(0.5, 1.5, n_modes), v0=[[-0.3, 0.05], [0.05, 0.3]], k=k)
    init = W.InitSpec(kT=0.3, q0=np.zeros(n_modes), state=1)
    return W.Workload(model, init, W.RunSpec(700, 90, 0.05, 9, seed))


@pytest.mark.parametrize("n_modes,mt", [(1, 0), (1, 1), (3, 0), (3, 1), (3, 2), (3, 3), (4, 2), (4, 4)])
def test_mode_class_builds_equal_general(P, n_modes, mt):
    """Solo calls of these models (normalized rule, up to four modes) run the
    two-state build specialised to the mode classes, batched calls the
    general build: walkers and bins agree bit for bit in both precisions
    (the class build only leaves out products with exact zeros), and the
    binary64 run agrees with the oracle."""
    wl = _classed_model(n_modes, mt, 100 + 10 * n_modes + mt)
    for prec in ("fp32", "fp64"):
        s = _solo(P, wl, prec, 0, 700)
        b = _batched(P, [(wl, prec, 0, 700)])[0]
        _assert_same(s, b, f"{wl.model.name} {prec}")
    out_o, st_o, _, _ = oracle_run(wl)
    out_g, st_g = s
    flip = compare_walkers(st_g, st_o, rtol=1e-10, label=wl.model.name)
    check_ensemble64(out_g, out_o, 700, flip, st_g, st_o, label=wl.model.name)


def test_batch_sliced_equals_solo(P):
    """K-step slices of a batch (continuous-batching quanta) change nothing."""
    mix = _mix()[:6]
    solo = [_solo(P, wl, prec, scheme, T) for wl, prec, scheme, T in mix]
    batch = _batched(P, mix, slices=(0.3, 0.3, None))
    for i, (s, b) in enumerate(zip(solo, batch)):
        _assert_same(s, b, f"item {i}")


def test_batch_matches_oracle(P):
    mix = [m for m in _mix() if m[1] == "fp64" and m[2] == 0]
    batch = _batched(P, mix)
    for (wl, prec, scheme, T), (out_g, st_g) in zip(mix, batch):
        out_o, st_o, _, _ = oracle_run(wl, n_traj=T)
        flip = compare_walkers(st_g, st_o, rtol=1e-10, max_flip_frac=0.005, label="batch")
        check_ensemble64(out_g, out_o, T, flip, st_g, st_o, label="batch")


def test_batch_rejects_shared_ensemble(P):
    wl = W.pyrazine_ci(n_traj=100, n_steps=20, cadence=10)
    model, ens, part = _setup(P, wl, "fp64", 100)
    r = wl.run
    jobs = [P.BatchJob(model, ens, part, r.dt, 10, r.cadence, r.seed)] * 2
    with pytest.raises(P.QCLError):
        P.qcl_propagate_batch(jobs)
    assert ens.step == 0


@pytest.mark.parametrize("n_states,n_modes,budget", [(3, 20, 3), (4, 50, 2), (2, 40, 2)])
def test_register_budget_variants_bitwise(P, n_states, n_modes, budget):
    """The register-budget build of a general kernel (3 waves per SIMD up to
    32 padded modes, 2 at 64) gives the same bits, alone and batched; the
    tuner picks one of the two builds."""
    import torch
    from paper_2608_14544_amd.tune import TuningTable
    wl = W.random_lvc(12 + n_modes, n_states=n_states, n_modes=n_modes, n_traj=1500, n_steps=60, cadence=20)
    r = wl.run
    outs = []
    for occ in (0, budget):
        model, ens, part = _setup(P, wl, "fp32", r.n_traj)
        P.qcl_propagate(model, ens, r.dt, r.n_steps, r.cadence, r.seed, part, occupancy=occ)
        outs.append((P.qcl_reduce_observables(model, part, r.n_traj).cpu().numpy(), ens.to_numpy()))
    model, ens, part = _setup(P, wl, "fp32", r.n_traj)
    P.qcl_propagate_batch([P.BatchJob(model, ens, part, r.dt, r.n_steps, r.cadence, r.seed, occupancy=budget)])
    outs.append((P.qcl_reduce_observables(model, part, r.n_traj).cpu().numpy(), ens.to_numpy()))
    torch.cuda.synchronize()
    _assert_same(outs[0], outs[1], f"occupancy {budget}")
    _assert_same(outs[0], outs[2], f"batched occupancy {budget}")
    t = TuningTable()
    choice = t.tune(wl, "fp32", n_traj=1 << 16, n_steps=20)
    print("tuned", n_states, n_modes, t.timings, flush=True)
    assert choice in (0, budget) and t.occupancy(P.Model(wl.model), "fp32") == choice


@pytest.mark.parametrize("wpc", [1, 2])
def test_workgroups_per_cu_bitwise(P, wpc):
    """A cap on the workgroups per compute unit of the persistent launch
    changes the launch shape only: every item of a mixed batch (two-state
    closed form, general N, both precisions) is bitwise its uncapped result,
    and items that differ in the cap run in separate launches of the same
    call."""
    import torch
    mix = _mix()
    ref = _batched(P, mix)
    runs, jobs = [], []
    for i, (wl, prec, scheme, T) in enumerate(mix):
        r = wl.run
        model, ens, part = _setup(P, wl, prec, T)
        runs.append((model, ens, part, T))
        jobs.append(P.BatchJob(model, ens, part, r.dt, r.n_steps, r.cadence, r.seed, scheme,
                               workgroups_per_cu=wpc if i % 2 == 0 else 0))
    P.qcl_propagate_batch(jobs)
    torch.cuda.synchronize()
    for i, (model, ens, part, T) in enumerate(runs):
        got = (P.qcl_reduce_observables(model, part, T).cpu().numpy(), ens.to_numpy())
        _assert_same(ref[i], got, f"item {i} wpc {wpc}")


def test_tuner_workgroups_per_cu(P):
    from paper_2608_14544_amd.tune import WPC_CANDIDATES, TuningTable, launch_class
    wl = W.random_lvc(3, n_states=3, n_modes=20, n_traj=2000, n_steps=60, cadence=20)
    t = TuningTable()
    choice = t.tune_workgroups(wl, "fp32", n_traj=1 << 16, n_steps=20)
    k = launch_class(P.Model(wl.model), "fp32")
    print("workgroups per CU", t.wpc_timings, flush=True)
    assert choice in WPC_CANDIDATES and t.wpc[k] == choice and set(t.wpc_timings[k]) == set(WPC_CANDIDATES)


def test_batched_workload_full_size():
    """The 256-instance batched workload at full size in the benchmark's
    launch configuration (binary32, tuned register budgets, one batched
    call): the smallest instances' ensembles against the FP64 oracle run
    in full (1e-3 x max(1, rms) per bin); then a binary64 batch of full-size instances
    covering N = 2, 3, 4 and up to 64 modes, with sampled walkers
    recomputed one by one by the oracle."""
    import torch
    import paper_2608_14544_amd as P
    from paper_2608_14544_amd.tune import autotune
    P.load_library()
    wls = W.batched_instances(256)
    table = autotune(wls, "fp32")
    runs, jobs = [], []
    for wl in wls:
        r = wl.run
        model, ens, part = _setup(P, wl, "fp32", r.n_traj)
        runs.append((model, ens, part))
        jobs.append(P.BatchJob(model, ens, part, r.dt, r.n_steps, r.cadence, r.seed,
                               occupancy=table.occupancy(model, "fp32")))
    P.qcl_propagate_batch(jobs)
    torch.cuda.synchronize()
    order = sorted(range(len(wls)), key=lambda i: wls[i].run.n_traj * wls[i].run.n_steps * wls[i].model.n_states)
    checked = 0
    for i in order:
        wl = wls[i]
        if wl.model.n_states == 4:  # keep the host oracle's share of the test short
            continue
        model, ens, part = runs[i]
        out_g = P.qcl_reduce_observables(model, part, wl.run.n_traj).cpu().numpy()
        out_o, st_o, _, _ = oracle_run(wl)
        check_ensemble32(out_g, out_o, wl.run.n_traj, g=ens.to_numpy(), o=st_o,
                         label=f"instance {i}: N={wl.model.n_states} M={wl.model.n_modes} T={wl.run.n_traj} "
                               f"steps={wl.run.n_steps}")
        checked += 1
        if checked == 4:
            break
    del runs, jobs
    torch.cuda.empty_cache()
    # binary64: full-size instances, per-walker parity on sampled walkers
    picks = [10, 13, 82, 97, 168, 214]
    sub = [wls[i] for i in picks]
    runs, jobs = [], []
    for wl in sub:
        r = wl.run
        model, ens, part = _setup(P, wl, "fp64", r.n_traj)
        runs.append((model, ens, part))
        jobs.append(P.BatchJob(model, ens, part, r.dt, r.n_steps, r.cadence, r.seed))
    P.qcl_propagate_batch(jobs)
    torch.cuda.synchronize()
    for wl, (model, ens, part), idx in zip(sub, runs, picks):
        ids = sample_ids(wl.run.n_traj, 60, seed=idx)
        g = sampled_state(ens, ids)
        o = oracle_walkers(wl, ids)
        compare_walkers(g, o, rtol=1e-10, max_flip_frac=0.01, label=f"batched instance {idx} fp64 sampled")
