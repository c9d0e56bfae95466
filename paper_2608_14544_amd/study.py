"""Walker-count convergence and decay-rate study (the paper's Sec. III.B,
Figs. 3-4): one model run at several walker counts, the excited adiabatic
population P(t) of each run compared with the largest run, and the decay
rate of P(t) fitted on each.

Every run draws its walkers from its own range of global walker ids (the
random streams are keyed by global id), so the runs are independent samples
of one large ensemble: a run of N walkers is not a prefix of the reference
run.  The device does the whole ensemble work (sampling, propagation,
reduction); this module only reads the reduced observables, n_out x 2 x N x N
values per run, and does the analysis on them.

Analysis definitions (the paper judges convergence and the decay by eye; the
numbers below are this module's readings of it):

- population: P(t_k) = Re rho^ad_{N-1,N-1}(t_k) with its standard error, the
  excited adiabatic state of Figs. 1-4;
- resolved horizon: the last bin time before the standard error of P first
  exceeds ``tol``;
- agreement horizon: the last bin time before |P_N - P_ref| first exceeds
  ``tol``;
- decay rate: weighted least squares of ln P(t) = ln A - k t over the bins
  whose times lie in a window [t0, t1], each bin weighted by (P/SE)^2, the
  inverse of the first-order variance of ln P; the window defaults to the
  first times the reference curve falls to ``p_hi`` = 0.8 and to ``p_lo`` =
  0.3, the fast segment of the decay (the pyrazine-like population drops
  from 0.8 to 0.3 within about 5 fs and then flattens near 0.2).  A run
  whose P is not positive somewhere in the window has no log fit; its rate
  is reported as None;
- fit quality: chi^2 per degree of freedom of that fit.  Above 1 the single
  exponential does not describe the window within the bins' errors, and the
  reported rate error ``rate_se`` is the statistical one (``rate_se_stat``)
  times sqrt(chi^2/dof), the Birge ratio.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import qcl as Q


@dataclass
class Curve:
    n_traj: int
    traj_offset: int
    t: np.ndarray  # bin times: fs for models in eV, else the model's reduced unit
    p: np.ndarray
    se: np.ndarray
    seconds: float = 0.0
    flags: Dict[str, int] = field(default_factory=dict)


def population(out: np.ndarray, state: Optional[int] = None) -> Tuple[np.ndarray, np.ndarray]:
    """Mean and standard error of Re rho^ad_ss over bins (default: the top
    adiabatic state) from a reduced output [n_out][2][N][N][4]."""
    n = out.shape[2]
    s = n - 1 if state is None else int(state)
    return out[:, 0, s, s, 0].copy(), out[:, 0, s, s, 2].copy()


def first_exceed(values: np.ndarray, tol: float) -> int:
    """Index of the first entry above ``tol`` (NaN counts as above), or
    len(values) when none is."""
    bad = ~(np.abs(values) <= tol)
    idx = np.flatnonzero(bad)
    return int(idx[0]) if idx.size else len(values)


def horizon(t: np.ndarray, values: np.ndarray, tol: float) -> float:
    """The last time before |values| first exceeds ``tol``; -inf when the
    first bin already does, +inf when none does."""
    k = first_exceed(values, tol)
    if k == len(values):
        return float("inf")
    return float(t[k - 1]) if k > 0 else float("-inf")


def crossing_time(t: np.ndarray, p: np.ndarray, level: float) -> float:
    """The first bin time at which p <= level (inf when it never is)."""
    idx = np.flatnonzero(p <= level)
    return float(t[idx[0]]) if idx.size else float("inf")


@dataclass
class DecayFit:
    rate: float
    rate_se: float        # statistical error of the slope
    amplitude: float
    window: Tuple[float, float]
    n_bins: int
    chi2_per_dof: float

    @property
    def rate_se_scaled(self) -> float:
        """The rate's error scaled by sqrt(chi^2/dof) when that exceeds 1."""
        return self.rate_se * float(np.sqrt(max(1.0, self.chi2_per_dof)))


def decay_fit(t: np.ndarray, p: np.ndarray, se: np.ndarray, window: Tuple[float, float]) -> DecayFit:
    """Weighted least-squares fit of ln p = ln A - k t over the bins with
    window[0] <= t <= window[1]; needs two bins with p > 0 and se > 0."""
    sel = (t >= window[0]) & (t <= window[1])
    if not np.all(p[sel] > 0) or not np.all(se[sel] > 0):
        raise ValueError("decay window holds a bin with P <= 0 or a zero standard error")
    x, y = t[sel], np.log(p[sel])
    sw = p[sel] / se[sel]  # square roots of the weights
    if x.size < 2:
        raise ValueError(f"decay window {window} holds {x.size} bin(s); two are needed")
    a = np.stack([np.ones_like(x), -x], axis=1) * sw[:, None]
    coef, _, _, _ = np.linalg.lstsq(a, y * sw, rcond=None)
    cov = np.linalg.inv(a.T @ a)
    resid = (y - (coef[0] - coef[1] * x)) * sw
    dof = x.size - 2
    chi2 = float(resid @ resid / dof) if dof > 0 else 0.0
    return DecayFit(rate=float(coef[1]), rate_se=float(np.sqrt(cov[1, 1])), amplitude=float(np.exp(coef[0])),
                    window=(float(window[0]), float(window[1])), n_bins=int(x.size), chi2_per_dof=chi2)


def default_window(ref: Curve, p_hi: float = 0.8, p_lo: float = 0.3) -> Tuple[float, float]:
    return crossing_time(ref.t, ref.p, p_hi), crossing_time(ref.t, ref.p, p_lo)


def run_curve(workload, n_traj: int, traj_offset: int, prec: str = "fp32", n_steps: Optional[int] = None,
              model: Optional["Q.Model"] = None, state: Optional[int] = None) -> Curve:
    """Sample, propagate and reduce ``n_traj`` walkers with global ids from
    ``traj_offset`` on the device; returns the population curve and the
    time of the run (sampling, propagation and reduction; the buffers are
    allocated before the clock starts)."""
    import torch
    r = workload.run
    S = r.n_steps if n_steps is None else int(n_steps)
    n_out = S // r.cadence + 1
    model = model or Q.Model(workload.model)
    ens = Q.Ensemble(model, int(n_traj), prec, int(traj_offset))
    part = Q.Partials(model, int(n_traj), n_out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Q.qcl_sample_initial(model, workload.init, r.seed, ens, part)
    Q.qcl_propagate(model, ens, r.dt, S, r.cadence, r.seed, part, Q.QCL_TRANS_NORMALIZED)
    out = Q.qcl_reduce_observables(model, part, int(n_traj))
    torch.cuda.synchronize()
    seconds = time.perf_counter() - t0
    out = out.cpu().numpy()
    del part
    fl = ens.tensors()["flags"][:n_traj]
    flags = {name: int(((fl & bit) != 0).sum().item()) for name, bit in
             (("nonfinite", Q.FLAG_NONFINITE), ("degenerate", Q.FLAG_DEGENERATE), ("resolved64", Q.FLAG_RESOLVED64))}
    del ens
    p, se = population(out, state)
    t = np.arange(out.shape[0]) * (r.cadence * r.dt * (workload.model.time_unit_fs or 1.0))
    return Curve(int(n_traj), int(traj_offset), t, p, se, seconds, flags)


def disjoint_offsets(walker_counts: Sequence[int]) -> List[int]:
    """Global id ranges: the largest run first from id 0, the others after
    it in decreasing size, none overlapping."""
    order = sorted(range(len(walker_counts)), key=lambda i: -int(walker_counts[i]))
    offsets = [0] * len(walker_counts)
    nxt = 0
    for i in order:
        offsets[i] = nxt
        nxt += int(walker_counts[i])
    return offsets


def summarize(curves: Sequence[Curve], tol: float = 0.02, window: Optional[Tuple[float, float]] = None,
              p_hi: float = 0.8, p_lo: float = 0.3, fit: bool = True) -> dict:
    """Horizons of every curve against the largest one and, when ``fit``,
    the decay rate of each over one common window."""
    ref = max(curves, key=lambda c: c.n_traj)
    if fit and window is None:
        window = default_window(ref, p_hi, p_lo)
    rows = []
    for c in curves:
        row = {"n_traj": c.n_traj, "traj_offset": c.traj_offset, "seconds": c.seconds,
               "resolved_until": horizon(c.t, c.se, tol), **c.flags}
        if c is not ref:
            row["agrees_until"] = horizon(c.t, c.p - ref.p, tol)
            row["max_dev_resolved"] = float(np.max(np.abs(c.p - ref.p)[: first_exceed(c.se, tol)], initial=0.0))
        if fit:
            try:
                f = decay_fit(c.t, c.p, c.se, window)
                row.update(rate=f.rate, rate_se=f.rate_se_scaled, rate_se_stat=f.rate_se, amplitude=f.amplitude,
                           fit_bins=f.n_bins, chi2_per_dof=f.chi2_per_dof)
            except ValueError as e:  # a noisy run with P <= 0 inside the window has no log fit
                row.update(rate=None, fit_error=str(e))
        rows.append(row)
    res = {"tol": tol, "reference_n_traj": ref.n_traj, "runs": rows}
    if fit:
        res["window"] = list(window)
    return res


def walker_study(workload, walker_counts: Sequence[int] = (10**6, 10**7, 10**8), prec: str = "fp32",
                 n_steps: Optional[int] = None, tol: float = 0.02, fit: bool = True,
                 window: Optional[Tuple[float, float]] = None) -> Tuple[dict, List[Curve]]:
    """Runs ``workload`` at every walker count on disjoint id ranges and
    summarizes the curves (see the module docstring)."""
    model = Q.Model(workload.model)
    offsets = disjoint_offsets(walker_counts)
    curves = [run_curve(workload, n, off, prec, n_steps, model) for n, off in zip(walker_counts, offsets)]
    return summarize(curves, tol=tol, window=window, fit=fit), curves
