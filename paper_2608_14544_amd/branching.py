"""Fixed-budget branching: propagation with systematic resampling between
calls, and the replica study that measures whether it pays.

The paper's CPU code spawned a walker whenever a transition was taken
(Sec. II.B), so the weight growth prod(1 + S) along a walker became growth
of the walker count; its GPU code keeps the count fixed and lets the weights
grow.  Here the count stays fixed and, every ``every`` time steps, the
ensemble is resampled in proportion to |w| on the device (qcl_resample):
walkers with large weights are split into copies that then branch on their
own random streams, walkers with small weights are dropped, and every
copy's weight keeps the expected contribution unchanged.

A resampled ensemble's copies are correlated, so the per-run standard error
of the reduced observables no longer measures the run's error; the honest
measure is the spread over independent replicas (disjoint walker-id
ranges), which ``replica_spread`` reports beside the plain runs.
"""
from __future__ import annotations

import time
from typing import Dict, Optional, Sequence

import numpy as np

from . import qcl as Q
from . import study


def run_resampled(workload, n_traj: int, traj_offset: int, every: Optional[int], prec: str = "fp32",
                  n_steps: Optional[int] = None, model: Optional[Q.Model] = None,
                  resample_seed: Optional[int] = None):
    """Sample, propagate and reduce one ensemble, resampling it every
    ``every`` steps (never when ``every`` is None or 0).  Returns (reduced
    output [n_out][2][N][N][4] as numpy, final Ensemble, device seconds)."""
    import torch
    r = workload.run
    S = r.n_steps if n_steps is None else int(n_steps)
    n_out = S // r.cadence + 1
    model = model or Q.Model(workload.model)
    seed = r.seed if resample_seed is None else int(resample_seed)
    a = Q.Ensemble(model, n_traj, prec, traj_offset)
    b = Q.Ensemble(model, n_traj, prec, traj_offset) if every else None
    part = Q.Partials(model, n_traj, n_out)
    ws = Q.Workspace()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Q.qcl_sample_initial(model, workload.init, r.seed, a, part)
    done = 0
    chunk = int(every) if every else S
    while done < S:
        c = min(chunk, S - done)
        Q.qcl_propagate(model, a, r.dt, c, r.cadence, r.seed, part)
        done += c
        if every and done < S:
            Q.qcl_resample(model, a, b, seed, ws)
            a, b = b, a
    out = Q.qcl_reduce_observables(model, part, n_traj)
    torch.cuda.synchronize()
    seconds = time.perf_counter() - t0
    return out.cpu().numpy(), a, seconds


def replica_spread(workload, n_traj: int, replicas: int, intervals: Sequence[Optional[int]],
                   times: Sequence[float], prec: str = "fp32", n_steps: Optional[int] = None,
                   state: Optional[int] = None) -> Dict[str, dict]:
    """For each resampling interval (in steps; None = never), ``replicas``
    runs of ``n_traj`` walkers on disjoint id ranges: the replica mean and
    standard deviation of the excited adiabatic population at the bins
    nearest ``times``, with the mean per-run standard error and the device
    time.  Every interval uses the same id ranges, so the runs differ only
    in the resampling."""
    r = workload.run
    model = Q.Model(workload.model)
    dt_unit = r.cadence * r.dt * (workload.model.time_unit_fs or 1.0)
    res = {}
    for every in intervals:
        ps, ses, secs = [], [], 0.0
        for k in range(replicas):
            out, ens, s = run_resampled(workload, n_traj, k * n_traj, every, prec, n_steps, model)
            del ens
            p, se = study.population(out, state)
            ps.append(p)
            ses.append(se)
            secs += s
        ps, ses = np.array(ps), np.array(ses)
        t = np.arange(ps.shape[1]) * dt_unit
        bins = [int(np.argmin(np.abs(t - x))) for x in times]
        key = "none" if not every else f"every_{every}_steps"
        res[key] = {
            "every_steps": every or None,
            "times": [float(t[i]) for i in bins],
            "mean": [float(ps[:, i].mean()) for i in bins],
            "replica_sd": [float(ps[:, i].std(ddof=1)) for i in bins],
            "mean_run_se": [float(ses[:, i].mean()) for i in bins],
            "seconds": secs,
        }
    return res
