"""Pins of the oracle's convergence and decay-rate analysis (Sec. III.B,
Figs. 3-4), and agreement of the package's study module with it on
synthetic curves (host arithmetic only, no device)."""
import math

import numpy as np
import pytest

import oracle.decay as D


def test_exact_exponential_any_weights():
    t = np.linspace(0.0, 30.0, 31)
    A, k = 0.93, 0.173
    p = A * np.exp(-k * t)
    se = np.random.default_rng(1).uniform(1e-3, 5e-2, t.size)
    rate, _, amp, used = D.decay_rate(t, p, se, 5.0, 20.0)
    assert used == 16
    assert abs(rate - k) <= 1e-12 * k and abs(amp - A) <= 1e-12


def test_two_bins_closed_form():
    # two points: the line through them, and first-order error propagation of
    # ln(p1/p2)/(t2-t1) for the rate's standard error
    t, p, se = [2.0, 7.0], [0.6, 0.15], [0.01, 0.02]
    rate, rse, amp, used = D.decay_rate(t, p, se, 0.0, 10.0)
    assert used == 2
    assert math.isclose(rate, math.log(p[0] / p[1]) / 5.0, rel_tol=1e-13)
    assert math.isclose(rse, math.sqrt((se[0] / p[0]) ** 2 + (se[1] / p[1]) ** 2) / 5.0, rel_tol=1e-12)
    assert math.isclose(amp * math.exp(-rate * 2.0), p[0], rel_tol=1e-12)


def test_equal_relative_errors_textbook_slope_error():
    # constant relative error r: ordinary least squares on ln p, slope variance r^2 / sum (t - mean t)^2
    rng = np.random.default_rng(2)
    t = np.arange(10.0)
    p = 0.8 * np.exp(-0.3 * t) * np.exp(rng.normal(0, 0.05, t.size))
    r = 0.05
    rate, rse, _, _ = D.decay_rate(t, p, p * r, -1.0, 100.0)
    slope_ols = np.polyfit(t, np.log(p), 1)[0]
    assert math.isclose(rate, -slope_ols, rel_tol=1e-10)
    assert math.isclose(rse, r / math.sqrt(((t - t.mean()) ** 2).sum()), rel_tol=1e-12)


def test_fit_minimises_weighted_squares():
    rng = np.random.default_rng(3)
    t = np.linspace(1.0, 12.0, 12)
    se = rng.uniform(0.002, 0.02, t.size)
    p = 0.9 * np.exp(-0.25 * t) + rng.normal(0, 1, t.size) * se * 0.3
    rate, _, amp, _ = D.decay_rate(t, p, se, 0.0, 20.0)

    def chi2(k, a):
        return float((((np.log(p) - math.log(a) + k * t) * p / se) ** 2).sum())

    best = chi2(rate, amp)
    for dk in (-1e-4, 1e-4):
        for da in (-1e-4, 0.0, 1e-4):
            assert chi2(rate + dk, amp * (1 + da)) > best
    assert chi2(rate, amp * (1 + 1e-4)) > best and chi2(rate, amp * (1 - 1e-4)) > best


def test_rate_error_covers_scatter():
    # the reported standard error matches the spread of rates fitted on
    # independent noisy copies of one exponential; the log fit's bias is of
    # second order in SE/P (at most 2% here), far inside the bound
    rng = np.random.default_rng(4)
    t = np.linspace(0.0, 10.0, 11)
    p0 = 0.9 * np.exp(-0.2 * t)
    se = 0.002 * np.ones_like(t)
    rates, errs = [], []
    for _ in range(4000):
        p = p0 + rng.normal(0, 1, t.size) * se
        k, s, _, _ = D.decay_rate(t, p, se, 0.0, 10.0)
        rates.append(k)
        errs.append(s)
    rates = np.array(rates)
    assert abs(rates.mean() - 0.2) < 4 * rates.std() / math.sqrt(rates.size) + 2e-5
    assert abs(rates.std() / np.mean(errs) - 1.0) < 0.08


def test_fit_quality():
    """chi^2/dof is 0 on an exact exponential, averages 1 over noisy copies
    whose errors are the stated ones, and grows when one exponential does
    not fit (a plateau); the scaled error then covers the scatter."""
    t = np.linspace(0.0, 10.0, 11)
    p0 = 0.9 * np.exp(-0.2 * t)
    k, ks, a, _ = D.decay_rate(t, p0, 0.01 * p0, 0.0, 10.0)
    assert D.fit_quality(t, p0, 0.01 * p0, 0.0, 10.0, k, a) < 1e-20
    assert D.scaled_rate_error(ks, 0.3) == ks
    rng = np.random.default_rng(11)
    se = 0.002 * np.ones_like(t)
    chis = []
    for _ in range(2000):
        p = p0 + rng.normal(0, 1, t.size) * se
        k, ks, a, _ = D.decay_rate(t, p, se, 0.0, 10.0)
        chis.append(D.fit_quality(t, p, se, 0.0, 10.0, k, a))
    # mean of chi^2/9 is 1 (up to the log's second-order bias), SE 0.47/sqrt(2000)
    assert abs(np.mean(chis) - 1.0) < 0.05
    # a decay onto a plateau fitted by one exponential
    pp = 0.7 * np.exp(-0.5 * t) + 0.2
    rates, errs, scaled = [], [], []
    for _ in range(2000):
        p = pp + rng.normal(0, 1, t.size) * se
        k, ks, a, _ = D.decay_rate(t, p, se, 0.0, 10.0)
        c = D.fit_quality(t, p, se, 0.0, 10.0, k, a)
        assert c > 10.0
        rates.append(k)
        scaled.append(D.scaled_rate_error(ks, c))
        errs.append(ks)
    assert np.mean(scaled) > 3.0 * np.mean(errs)


def test_horizon_and_crossing():
    t = [0.0, 1.0, 2.0, 3.0]
    assert D.horizon(t, [0.01, -0.015, 0.03, 0.0], 0.02) == 1.0
    assert D.horizon(t, [0.05, 0.0, 0.0, 0.0], 0.02) == -math.inf
    assert D.horizon(t, [0.0, 0.02, -0.02, 0.0], 0.02) == math.inf  # the bound is inside
    assert D.horizon(t, [0.0, float("nan"), 0.0, 0.0], 0.02) == 0.0
    assert D.first_time_at_or_below(t, [1.0, 0.5, 0.1, 0.3], 0.1) == 2.0
    assert D.first_time_at_or_below(t, [1.0, 0.5, 0.2, 0.3], 0.1) == math.inf


def test_window_edges_inclusive_and_errors():
    t = [0.0, 1.0, 2.0, 3.0]
    p = [0.9, 0.5, 0.3, 0.1]
    se = [0.01] * 4
    assert D.decay_rate(t, p, se, 1.0, 3.0)[3] == 3
    with pytest.raises(ValueError):
        D.decay_rate(t, p, se, 0.5, 1.5)
    with pytest.raises(ValueError):
        D.decay_rate(t, [0.9, -0.1, 0.3, 0.1], se, 0.0, 3.0)
    with pytest.raises(ValueError):
        D.decay_rate(t, p, [0.01, 0.0, 0.01, 0.01], 0.0, 3.0)


def test_excited_population_indexing():
    out = np.zeros((3, 2, 3, 3, 4))
    out[:, 0, 2, 2, 0] = [0.7, 0.6, 0.5]
    out[:, 0, 2, 2, 2] = [0.01, 0.02, 0.03]
    out[:, 1, 2, 2, 0] = 9.0  # diabatic: not read
    out[:, 0, 1, 1, 0] = 9.0
    m, s = D.excited_population(out)
    assert m == [0.7, 0.6, 0.5] and s == [0.01, 0.02, 0.03]


# ---------------------------------------------- package analysis vs oracle

def _curves(rng, n_bins=40):
    t = np.arange(n_bins) * 0.5
    base = 0.95 * np.exp(-0.2 * np.maximum(t - 3.0, 0.0))
    out = []
    for n in (10**4, 10**5, 10**6):
        se = 4e-4 * np.exp(0.1 * t) * math.sqrt(1e6 / n)
        out.append((n, t, base + rng.normal(0, 1, n_bins) * se, se))
    return out


def test_study_analysis_matches_oracle():
    from paper_2608_14544_amd import study as S
    rng = np.random.default_rng(7)
    raw = _curves(rng)
    curves = [S.Curve(n, 0, t, p, se) for n, t, p, se in raw]
    res = S.summarize(curves, tol=0.02)
    _, t_ref, p_ref, _ = raw[-1]
    t0 = D.first_time_at_or_below(t_ref, p_ref, 0.8)
    t1 = D.first_time_at_or_below(t_ref, p_ref, 0.3)
    assert res["window"] == [t0, t1]
    for row, (n, t, p, se) in zip(res["runs"], raw):
        k, ks, a, used = D.decay_rate(t, p, se, t0, t1)
        chi2 = D.fit_quality(t, p, se, t0, t1, k, a)
        assert math.isclose(row["rate"], k, rel_tol=1e-12) and math.isclose(row["rate_se_stat"], ks, rel_tol=1e-12)
        assert math.isclose(row["chi2_per_dof"], chi2, rel_tol=1e-9, abs_tol=1e-12)
        assert math.isclose(row["rate_se"], D.scaled_rate_error(ks, chi2), rel_tol=1e-9)
        assert math.isclose(row["amplitude"], a, rel_tol=1e-12) and row["fit_bins"] == used
        assert row["resolved_until"] == D.horizon(t, se, 0.02)
        if n != 10**6:
            assert row["agrees_until"] == D.horizon(t, p - p_ref, 0.02)


def test_disjoint_offsets():
    from paper_2608_14544_amd import study as S
    counts = [10**6, 10**8, 10**7]
    assert S.disjoint_offsets(counts) == [10**8 + 10**7, 0, 10**8]
