"""Walker-count convergence and decay-rate analysis of reduced observables --
test infrastructure, written independently of the package's study module.

The paper compares runs of 1e6, 1e7 and 1e8 walkers by eye and states where
each one is accurate and that the smallest already fixes the decay rate of
the excited adiabatic population (Sec. III.B, Figs. 3-4).  The quantities
here turn that into numbers, with plain loops and closed-form sums:

- the excited population P(t_k) is Re rho^ad of the top adiabatic state
  (mean and standard error of the estimator);
- a horizon is the last bin time before a sequence first leaves [-tol, tol]
  (a NaN leaves it too);
- the decay rate k of P(t) = A exp(-k t) comes from the weighted
  least-squares line through (t_k, ln P_k) with weights (P_k/SE_k)^2, the
  inverse of the first-order variance of ln P_k; the normal equations are
  solved in closed form, and the rate's standard error is the square root of
  the slope's variance, W / (W Sxx - Sx^2);
- the fit's quality is chi^2 per degree of freedom, the weighted sum of
  squared residuals of ln P over (bins - 2); when it exceeds 1 the single
  exponential does not describe the window within the bins' errors, and the
  rate's error is scaled by sqrt(chi^2/dof) (the Birge ratio), so the quoted
  error covers the scatter the fit leaves.
"""
from __future__ import annotations

import math


def excited_population(out):
    """(mean, SE) lists of Re rho^ad of the top adiabatic state, from an
    observable array [n_out][2][N][N][4] after averaging."""
    n = len(out[0][0])
    mean = [float(out[k][0][n - 1][n - 1][0]) for k in range(len(out))]
    se = [float(out[k][0][n - 1][n - 1][2]) for k in range(len(out))]
    return mean, se


def horizon(t, values, tol):
    last = -math.inf
    for tk, v in zip(t, values):
        if not (abs(v) <= tol):
            return last
        last = float(tk)
    return math.inf


def first_time_at_or_below(t, p, level):
    for tk, pk in zip(t, p):
        if pk <= level:
            return float(tk)
    return math.inf


def decay_rate(t, p, se, t0, t1):
    """(k, SE of k, A, bins used) of the weighted line through ln P over
    t0 <= t <= t1."""
    W = Sx = Sy = Sxx = Sxy = 0.0
    used = 0
    for tk, pk, sk in zip(t, p, se):
        if t0 <= tk <= t1:
            if not (pk > 0.0 and sk > 0.0):
                raise ValueError("bin with P <= 0 or zero standard error inside the window")
            w = (pk / sk) ** 2
            y = math.log(pk)
            W += w
            Sx += w * tk
            Sy += w * y
            Sxx += w * tk * tk
            Sxy += w * tk * y
            used += 1
    if used < 2:
        raise ValueError("fewer than two bins inside the window")
    det = W * Sxx - Sx * Sx
    slope = (W * Sxy - Sx * Sy) / det
    intercept = (Sy - slope * Sx) / W
    return -slope, math.sqrt(W / det), math.exp(intercept), used


def fit_quality(t, p, se, t0, t1, k, amp):
    """chi^2 per degree of freedom of ln P = ln A - k t over t0 <= t <= t1,
    each bin weighted by (P/SE)^2 (0 with fewer than three bins)."""
    chi2 = 0.0
    used = 0
    for tk, pk, sk in zip(t, p, se):
        if t0 <= tk <= t1:
            r = math.log(pk) - (math.log(amp) - k * tk)
            chi2 += (pk / sk) ** 2 * r * r
            used += 1
    return chi2 / (used - 2) if used > 2 else 0.0


def scaled_rate_error(rate_se, chi2_per_dof):
    """The rate's error scaled by the Birge ratio when the fit is poor."""
    return rate_se * math.sqrt(max(1.0, chi2_per_dof))
