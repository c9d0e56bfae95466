"""Autotuner: three launch knobs, each measured where it applies.

1. Register budget of the general kernels (qcl_prop_desc.occupancy).

The general kernels of linear models (N > 2, or N = 2 with M > 8) exist in
binary32 in two builds of the same code: one where the compiler chooses
the register count (often 150-240 registers, two or three waves per SIMD;
at 64 modes all 256 and some accumulation registers, one wave), and one
with a register budget: a third of the register file (three waves per
SIMD) up to 32 padded modes, half of it (two waves) at 64.  Which one is
faster depends on the kernel class -- more resident waves hide the step's
long dependency chains, the cap can force spills -- so it is measured.  The
arithmetic is identical: the choice never changes a result bit.

A class is (N, padded modes MP, coupling-rank bucket RB, precision); the
tuner times one propagate call per build on a synthetic ensemble of the
given workload and records the faster one.

2. Workgroups per compute unit of the persistent batched launch
(qcl_prop_desc.workgroups_per_cu): all that fit (the default), or at most
1 or 2.  Fewer resident workgroups leave room to the other classes of a
batch that run beside it, at the cost of latency hiding; timed per launch
class (the kernel a batch item runs) with one batched call of a synthetic
ensemble.

3. The serving quantum: walker-steps each resident job advances per
scheduling round (serve.Server quantum_work), with a floor in steps
(serve.Server min_steps).  Short rounds answer small jobs sooner, long
rounds spend less on per-round launches and on moving each job's state in
and out of registers (a job of 1e8 walkers at 2e8 walker-steps per round
would advance two steps per round); timed on a prefix of the served
stream, the candidate with the lowest p99 latency kept.

None of the three changes a result bit.  ``TuningTable`` keeps the choices
and their timings and can save and load them as JSON.
"""
from __future__ import annotations

import json
import os
import time
from typing import Dict, Iterable, Optional, Tuple

from . import qcl as Q

Key = Tuple[int, int, int, str]
VARIANTS = (0, 2, 3)
WPC_CANDIDATES = (0, 1, 2)
QUANTUM_CANDIDATES = ((5e7, 1), (2e8, 1), (8e8, 1), (2e8, 16), (8e8, 16))  # (quantum_work, min_steps)


def budget_variant(mp: int, n_states: int = 3) -> int:
    """The register-budget build that exists for ``mp`` padded modes: 3
    (three waves per SIMD) up to 32 modes (16 for four states), 2 (two
    waves) at 64, else 0 (none)."""
    if mp <= (16 if n_states >= 4 else 32):
        return 3
    return 2 if mp == 64 else 0


def padded_modes(m: int) -> int:
    """Mode count the general kernels are specialised on."""
    for mp in (4, 8, 16, 32, 64):
        if m <= mp:
            return mp
    return 128


def rank_bucket(rank: int, n: int) -> int:
    return 1 if rank <= 1 else n if (rank <= n and n <= 4) else n * (n + 1) // 2


def kernel_class(n_states: int, n_modes: int, rank: int, prec: str) -> Optional[Key]:
    """The tunable kernel class of a model, or None when only one build
    exists (two-state closed form, more than 4 states, binary64, more than
    64 padded modes)."""
    if (n_states == 2 and n_modes <= 8) or n_states > 4:
        return None
    mp = padded_modes(n_modes)
    if prec != "fp32" or budget_variant(mp, n_states) == 0:
        return None
    return (n_states, mp, rank_bucket(rank, n_states), prec)


def launch_class(model: "Q.Model", prec: str) -> tuple:
    """The kernel a batch item of ``model`` runs: the closed-form two-state
    kernels per mode count, the general kernels per padded modes and rank
    bucket, each per model form and precision; a model with a supplied
    potential runs the kernel of its own program."""
    if getattr(model, "is_source", False):
        return ("source", int(model.handle.value), prec)
    n, m = int(model.n_states), int(model.n_modes)
    closed = n == 2 and m <= 8 and not getattr(model, "n_pairs", 0)
    modes = m if closed else padded_modes(m)
    return (n, modes, 0 if closed else rank_bucket(int(model.rank), n), int(getattr(model, "degree", 1) > 1),
            int(getattr(model, "n_pairs", 0) > 0), prec)


class TuningTable:
    def __init__(self, path: Optional[str] = None):
        self.choice: Dict[Key, int] = {}
        self.timings: Dict[Key, Dict[int, float]] = {}
        self.wpc: Dict[tuple, int] = {}
        self.wpc_timings: Dict[tuple, Dict[int, float]] = {}
        self.serving: Dict[str, float] = {}
        self.serving_timings: Dict[tuple, dict] = {}
        if path and os.path.exists(path):
            self.load(path)

    def key(self, model: "Q.Model", prec: str) -> Optional[Key]:
        # one build only for models with higher powers and supplied potentials
        if getattr(model, "degree", 1) > 1 or getattr(model, "is_source", False):
            return None
        return kernel_class(model.n_states, model.n_modes, model.rank, prec)

    def occupancy(self, model: "Q.Model", prec: str) -> int:
        k = self.key(model, prec)
        return self.choice.get(k, 0) if k is not None else 0

    def workgroups_per_cu(self, model: "Q.Model", prec: str) -> int:
        return self.wpc.get(launch_class(model, prec), 0)

    def quantum_work(self, default: float = 2e8) -> float:
        return float(self.serving.get("quantum_work", default))

    def min_steps(self, default: int = 1) -> int:
        return int(self.serving.get("min_steps", default))

    def save(self, path: str):
        rows = [{"n": k[0], "mp": k[1], "rb": k[2], "prec": k[3], "occupancy": v,
                 "ms": {str(o): t for o, t in self.timings.get(k, {}).items()}}
                for k, v in sorted(self.choice.items())]
        wrows = [{"class": list(k), "workgroups_per_cu": v,
                  "ms": {str(o): t for o, t in self.wpc_timings.get(k, {}).items()}}
                 for k, v in sorted(self.wpc.items())]
        with open(path, "w") as f:
            json.dump({"occupancy": rows, "workgroups_per_cu": wrows, "serving": self.serving}, f, indent=1)

    def load(self, path: str):
        with open(path) as f:
            doc = json.load(f)
        rows = doc["occupancy"] if isinstance(doc, dict) else doc
        for r in rows:
            k = (int(r["n"]), int(r["mp"]), int(r["rb"]), str(r["prec"]))
            occ = int(r["occupancy"])
            if occ not in VARIANTS:
                raise ValueError(f"unknown occupancy {occ} in {path}")
            self.choice[k] = occ
        if isinstance(doc, dict):
            for r in doc.get("workgroups_per_cu", []):
                k = tuple(r["class"][:5]) + (str(r["class"][5]),)
                if int(r["workgroups_per_cu"]) not in WPC_CANDIDATES:
                    raise ValueError(f"unknown workgroups_per_cu in {path}")
                self.wpc[k] = int(r["workgroups_per_cu"])
            self.serving.update({k: float(v) for k, v in doc.get("serving", {}).items()})

    def tune_workgroups(self, workload, prec: str = "fp32", model: Optional["Q.Model"] = None,
                        n_traj: int = 1 << 18, n_steps: int = 40, min_gain: float = 0.03) -> int:
        """Times one batched call of ``workload``'s model per candidate
        workgroups-per-CU (register budget as tuned) and records the
        fastest; a cap must win by ``min_gain`` over all-that-fit."""
        import torch
        model = model or Q.Model(workload.model)
        k = launch_class(model, prec)
        if k in self.wpc:
            return self.wpc[k]
        r = workload.run
        ens = Q.Ensemble(model, n_traj, prec, zero=False)
        part = Q.Partials(model, n_traj, 2 * (n_steps // r.cadence) + 4)
        Q.qcl_sample_initial(model, workload.init, r.seed, ens, part)
        ws = Q.Workspace()
        occ = self.occupancy(model, prec)
        s = torch.cuda.current_stream()
        times = {}
        for wpc in WPC_CANDIDATES + WPC_CANDIDATES:  # the first round warms each launch up
            job = Q.BatchJob(model, ens, part, r.dt, n_steps // 2, r.cadence, r.seed, occupancy=occ,
                             workgroups_per_cu=wpc)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            Q.qcl_propagate_batch([job], ws, stream=s)
            e1.record(s)
            torch.cuda.synchronize()
            times[wpc] = e0.elapsed_time(e1)
        base = times[0]
        best = min(WPC_CANDIDATES, key=lambda w: times[w])
        best = best if times[best] < (1.0 - min_gain) * base else 0
        self.wpc[k] = best
        self.wpc_timings[k] = times
        del ens, part
        return best

    def tune_quantum(self, run_stream, candidates=QUANTUM_CANDIDATES) -> tuple:
        """``run_stream(quantum_work, min_steps)`` serves a stream and
        returns its latency statistics; keeps the candidate pair with the
        lowest p99."""
        stats = {(float(q), int(m)): run_stream(float(q), int(m)) for q, m in candidates}
        def p99(c):
            v = stats[c].get("p99_s")
            return float("inf") if v is None else v
        best = min(stats, key=p99)
        self.serving["quantum_work"] = best[0]
        self.serving["min_steps"] = float(best[1])
        self.serving_timings = stats
        return best

    def tune(self, workload, prec: str = "fp32", model: Optional["Q.Model"] = None,
             n_traj: int = 1 << 20, n_steps: int = 60, min_gain: float = 0.03) -> int:
        """Times both builds on ``workload``'s model and records the faster
        (the capped build must win by ``min_gain``).  Returns the choice."""
        import torch
        model = model or Q.Model(workload.model)
        k = self.key(model, prec)
        if k is None:
            return 0
        if k in self.choice:
            return self.choice[k]
        r = workload.run
        ens = Q.Ensemble(model, n_traj, prec, zero=False)
        part = Q.Partials(model, n_traj, 2 * (n_steps // r.cadence) + 4)
        Q.qcl_sample_initial(model, workload.init, r.seed, ens, part)
        alt = budget_variant(k[1], k[0])
        times = {}
        for occ in (0, alt):  # warm both builds first
            Q.qcl_propagate(model, ens, r.dt, r.cadence, r.cadence, r.seed, part, occupancy=occ)
        torch.cuda.synchronize()
        for occ in (0, alt):
            t0 = time.perf_counter()
            Q.qcl_propagate(model, ens, r.dt, n_steps // 2, r.cadence, r.seed, part, occupancy=occ)
            torch.cuda.synchronize()
            times[occ] = (time.perf_counter() - t0) * 1e3
        best = alt if times[alt] < (1.0 - min_gain) * times[0] else 0
        self.choice[k] = best
        self.timings[k] = times
        del ens, part
        return best


def autotune(workloads: Iterable, prec: str = "fp32", table: Optional[TuningTable] = None) -> TuningTable:
    """Tunes every distinct kernel class among ``workloads`` once."""
    table = table or TuningTable()
    for wl in workloads:
        m = Q.Model(wl.model)
        if table.key(m, prec) is not None and table.key(m, prec) not in table.choice:
            table.tune(wl, prec, model=m)
    return table
