"""The job server on the device: jobs that arrive while others run are
admitted by memory footprint and advanced together in batched quanta; each
result must be bitwise the result of the same job run alone."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2608_14544_amd as pkg
    pkg.load_library()
    return pkg


def _alone(P, wl, prec, scheme=0):
    import torch
    r = wl.run
    model = P.Model(wl.model)
    ens = P.Ensemble(model, r.n_traj, prec)
    part = P.Partials(model, r.n_traj, r.n_out)
    P.qcl_sample_initial(model, wl.init, r.seed, ens, part)
    P.qcl_propagate(model, ens, r.dt, r.n_steps, r.cadence, r.seed, part, scheme)
    out = P.qcl_reduce_observables(model, part, r.n_traj).cpu().numpy()
    torch.cuda.synchronize()
    return out


def test_served_results_equal_alone(P):
    from paper_2608_14544_amd.serve import DeviceBackend, JobSpec, Server, latency_stats
    arrivals, wls = W.served_stream(14, rate=200.0, seed=7, traj_scale=2e-3, step_scale=0.1, max_modes=40)
    specs = [JobSpec(wl, prec="fp64" if i % 3 == 0 else "fp32", name=f"job{i}") for i, wl in enumerate(wls)]
    be = DeviceBackend()
    fps = [be.footprint(s) for s in specs]
    # room for a few jobs at a time, so that some wait and are admitted later
    srv = Server(be, memory_budget=max(fps) * 2, max_slots=6, quantum_steps=16)
    results = srv.run(arrivals, specs)
    assert len(results) == len(specs) and not any(r.error for r in results)
    assert srv.rounds > 3 and srv.used == 0
    waited = [r for r in results if r.admitted > r.arrival + 1e-4]
    print("jobs", len(results), "rounds", srv.rounds, "admitted late", len(waited), latency_stats(results),
          flush=True)
    by_name = {r.name: r for r in results}
    for s in specs:
        ref = _alone(P, s.workload, s.prec)
        assert np.array_equal(by_name[s.name].out, ref), s.name


def test_server_rejects_oversized(P):
    from paper_2608_14544_amd.serve import DeviceBackend, JobSpec, Server
    be = DeviceBackend()
    small = JobSpec(W.spin_boson_1mode(n_traj=500, n_steps=20), name="small")
    big = JobSpec(W.pyrazine_ci(n_traj=200000, n_steps=20), name="big")
    srv = Server(be, memory_budget=be.footprint(small) * 3, quantum_steps=8)
    res = {r.name: r for r in srv.run([0.0, 0.0], [big, small])}
    assert res["big"].error and res["big"].out is None
    assert np.array_equal(res["small"].out, _alone(P, small.workload, "fp32"))


def test_served_mixed_model_families_equal_alone(P):
    """Every model family through the server at once: linear, higher powers,
    more than four states and bilinear terms of each combination count
    (4, 8 and 16), in both precisions; each result bitwise the job alone."""
    from paper_2608_14544_amd.serve import DeviceBackend, JobSpec, Server
    wls = [
        W.pyrazine_ci(n_traj=3000, n_steps=60, cadence=6),
        W.pyrazine_qvc(n_traj=2000, n_steps=60, cadence=6),
        W.random_poly(40, n_states=3, n_modes=12, degree=4, n_traj=1500, n_steps=40, cadence=10),
        W.random_lvc(41, n_states=6, n_modes=5, n_traj=1000, n_steps=40, cadence=10),
        W.pyrazine_bilinear(n_traj=2500, n_steps=60, cadence=6),
        W.random_bilinear(42, n_states=3, n_modes=6, n_pairs=4, degree=3, n_traj=1200, n_steps=40, cadence=10),
        W.random_bilinear(43, n_states=2, n_modes=8, all_pairs=True, shared=True, n_traj=1800, n_steps=40,
                          cadence=10),
    ]
    specs = [JobSpec(wl, prec="fp64" if i % 2 else "fp32", name=f"job{i}") for i, wl in enumerate(wls)]
    be = DeviceBackend()
    fps = [be.footprint(s) for s in specs]
    srv = Server(be, memory_budget=max(fps) * 3, max_slots=4, quantum_steps=16)
    results = srv.run([0.002 * i for i in range(len(specs))], specs)
    assert len(results) == len(specs) and not any(r.error for r in results)
    by_name = {r.name: r for r in results}
    for s in specs:
        assert np.array_equal(by_name[s.name].out, _alone(P, s.workload, s.prec)), s.name


def test_served_fp64_jobs_match_oracle(P):
    """Binary64 jobs of every batched model family through the server, admitted
    at different times and advanced in quanta beside each other, against the
    FP64 oracle run of the same job: every mean of every bin within
    1e-9 * max(1, rms of its summed terms).  The served path returns only the
    reduced observables, so no flip allowance is taken: at these sizes a
    binary64 walker whose decision differs from the oracle's is not expected
    (its uniform number would have to fall within ~1e-13 of a threshold)."""
    from paper_2608_14544_amd.serve import DeviceBackend, JobSpec, Server
    from parity import check_ensemble64, oracle_run
    wls = [
        W.spin_boson_1mode(n_traj=700, n_steps=80, cadence=8),
        W.pyrazine_ci(n_traj=1000, n_steps=60, cadence=6),
        W.random_lvc(5, n_states=3, n_modes=6, n_traj=600, n_steps=50, cadence=10),
        W.random_lvc(9, n_states=4, n_modes=10, n_traj=500, n_steps=40, cadence=8),
        W.pyrazine_qvc(n_traj=800, n_steps=40, cadence=8),
        W.random_bilinear(42, n_states=3, n_modes=6, n_pairs=4, degree=3, n_traj=600, n_steps=40, cadence=10),
    ]
    specs = [JobSpec(wl, prec="fp64", name=f"job{i}") for i, wl in enumerate(wls)]
    be = DeviceBackend()
    fps = [be.footprint(s) for s in specs]
    srv = Server(be, memory_budget=max(fps) * 3, max_slots=3, quantum_steps=16)
    results = srv.run([0.003 * i for i in range(len(specs))], specs)
    assert len(results) == len(specs) and not any(r.error for r in results)
    assert srv.rounds > 3
    by_name = {r.name: r for r in results}
    for s in specs:
        out_o = oracle_run(s.workload)[0]
        check_ensemble64(by_name[s.name].out, out_o, s.workload.run.n_traj, label="served " + s.workload.model.name)
