"""Autotuner for the general kernels' register budget.

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
given workload and records the faster one.  ``TuningTable`` keeps the
choices (and can save and load them as JSON); ``occupancy(model, prec)``
gives the value for ``qcl_prop_desc.occupancy``.
"""
from __future__ import annotations

import json
import os
import time
from typing import Dict, Iterable, Optional, Tuple

from . import qcl as Q

Key = Tuple[int, int, int, str]
VARIANTS = (0, 2, 3)


def budget_variant(mp: int) -> int:
    """The register-budget build that exists for ``mp`` padded modes."""
    return 3 if mp <= 32 else 2


def padded_modes(m: int) -> int:
    """Mode count the general kernels are specialised on."""
    for mp in (8, 16, 32, 64):
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
    if prec != "fp32" or mp > 64:
        return None
    return (n_states, mp, rank_bucket(rank, n_states), prec)


class TuningTable:
    def __init__(self, path: Optional[str] = None):
        self.choice: Dict[Key, int] = {}
        self.timings: Dict[Key, Dict[int, float]] = {}
        if path and os.path.exists(path):
            self.load(path)

    def key(self, model: "Q.Model", prec: str) -> Optional[Key]:
        if getattr(model, "degree", 1) > 1:  # one build only for models with higher powers
            return None
        return kernel_class(model.n_states, model.n_modes, model.rank, prec)

    def occupancy(self, model: "Q.Model", prec: str) -> int:
        k = self.key(model, prec)
        return self.choice.get(k, 0) if k is not None else 0

    def save(self, path: str):
        rows = [{"n": k[0], "mp": k[1], "rb": k[2], "prec": k[3], "occupancy": v,
                 "ms": {str(o): t for o, t in self.timings.get(k, {}).items()}}
                for k, v in sorted(self.choice.items())]
        with open(path, "w") as f:
            json.dump(rows, f, indent=1)

    def load(self, path: str):
        with open(path) as f:
            for r in json.load(f):
                k = (int(r["n"]), int(r["mp"]), int(r["rb"]), str(r["prec"]))
                occ = int(r["occupancy"])
                if occ not in VARIANTS:
                    raise ValueError(f"unknown occupancy {occ} in {path}")
                self.choice[k] = occ

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
        alt = budget_variant(k[1])
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
