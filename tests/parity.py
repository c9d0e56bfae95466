"""Parity helpers shared by the GPU tests: the HIP path (through the C ABI)
against the FP64 CPU oracle on the same seeded inputs.

Tolerances
  * FP64 path, per walker: q, p, U, Phi within 1e-10 relative to
    max(|value|, ensemble rms of that quantity); w within 1e-10 relative.
    Walkers whose transition decisions differ ("flips": a different final
    element, or |w| off by more than 1e-6 relative) are counted, printed
    and excluded from the per-walker comparison; the caller caps their
    number.
  * FP64 path, ensemble means: every bin is asserted, flips or not.  The
    bound of bin k is
        1e-9 * max(1, rms_k)  +  sum over flipped walkers of (|w_gpu| + |w_oracle|) / T,
    where rms_k is the root mean square of the per-walker terms of that
    bin (from the oracle's mean and standard error).  The first term is
    1e-9 absolute on unit-scale bins and 1e-9 relative to the summed terms
    where weights have grown past 1 (the weights grow as prod(1 + S) along
    a walker: the sign problem).  The second term bounds what the flipped
    walkers can contribute: under both transition rules |w| never
    decreases along a walker, so a walker's final |w| bounds its term in
    every bin (a diabatic term is |w| |U_ia U_jb| <= |w|).
  * FP32 path (binary32 propagation, binary64 weight, phase and sums):
    ensemble means within 1e-3 * max(1, rms_k) of the oracle on every bin:
    1e-3 absolute on unit-scale bins, 1e-3 relative to the summed terms
    elsewhere.  (The two paths share their random streams, so sampling
    noise is common to both and a standard error is not the yardstick.)
    Where both final states are at hand, walkers whose decisions differ
    from the oracle's are counted and widen the bound by their |w|, as
    above: binary32 rounding changes a decision now and then, and a walker
    that took another branch is another sample of the same estimator.
"""
from __future__ import annotations

import numpy as np

import oracle.core as oc


def oracle_state(st):
    return {"q": st.q, "p": st.p, "U": st.U, "w": st.w, "phase": st.phase, "a": st.a, "b": st.b}


def flip_mask(g, o):
    """Walkers whose transition decisions differ between the two runs."""
    flip = (g["a"] != o["a"]) | (g["b"] != o["b"])
    flip |= ~(np.abs(np.abs(g["w"]) - np.abs(o["w"])) <= 1e-6 * np.abs(o["w"]))
    return flip


def compare_walkers(g, o, rtol=1e-10, max_flip_frac=0.0, label=""):
    """Per-walker FP64 parity; returns the boolean mask of flipped walkers."""
    flip = flip_mask(g, o)
    ok = ~flip
    worst = {}
    for key in ("q", "p", "U", "phase"):
        gv, ov = g[key][ok], o[key][ok]
        scale = max(float(np.sqrt(np.mean(o[key] ** 2))) if o[key].size else 1.0, 1e-300)
        err = np.abs(gv - ov) / np.maximum(np.abs(ov), scale)
        worst[key] = float(err.max()) if err.size else 0.0
    errw = np.abs(g["w"][ok] - o["w"][ok]) / np.abs(o["w"][ok])
    worst["w"] = float(errw.max()) if errw.size else 0.0
    nflip = int(flip.sum())
    print(f"[{label}] walkers={len(ok)} flips={nflip} ({nflip / max(len(ok), 1):.2%}) "
          f"worst-rel={ {k: f'{v:.2e}' for k, v in worst.items()} }", flush=True)
    assert nflip <= max_flip_frac * len(ok), (label, nflip, len(ok))
    for key, v in worst.items():
        assert v <= rtol, (label, key, v)
    return flip


def rms_terms(out_o, n_traj):
    """Root mean square of the per-walker terms behind each mean of an
    [n_out, 2, N, N, 4] result: SE^2 = (S2 - S1^2/T) / (T (T - 1)), so
    S2 / T = SE^2 (T - 1) + mean^2."""
    T = float(n_traj)
    return np.sqrt(out_o[..., 2:] ** 2 * (T - 1.0) + out_o[..., :2] ** 2)


def flip_allowance(flip, g, o, n_traj):
    """Largest change the flipped walkers can make to any mean."""
    if flip is None or not np.any(flip):
        return 0.0
    wg = np.abs(g["w"][flip])
    wo = np.abs(o["w"][flip])
    assert np.all(np.isfinite(wg)) and np.all(np.isfinite(wo)), "a flipped walker is non-finite"
    return float((wg.sum() + wo.sum()) / n_traj)


def check_ensemble64(out_g, out_o, n_traj, flip=None, g=None, o=None, tol=1e-9, label="", extra_allow=0.0):
    """Asserts every bin of an FP64 result against the oracle's;
    ``extra_allow`` is a further absolute allowance the caller derives (and
    states) for a known per-walker difference."""
    rms = rms_terms(out_o, n_traj)
    allow = flip_allowance(flip, g, o, n_traj) + float(extra_allow)
    bound = tol * np.maximum(1.0, rms) + allow
    err = np.abs(out_g[..., :2] - out_o[..., :2])
    unit = rms <= 1.0
    abs_unit = float(err[unit].max()) if unit.any() else 0.0
    rel_big = float((err[~unit] / rms[~unit]).max()) if (~unit).any() else 0.0
    print(f"[{label}] fp64 ensemble: {int(unit.sum())} unit-scale means, max abs err {abs_unit:.3g}; "
          f"{int((~unit).sum())} means with rms > 1 (largest {float(rms.max()):.3g}), max err/rms {rel_big:.3g}; "
          f"flip allowance {allow:.3g}; max err/bound {float((err / bound).max()):.3g}", flush=True)
    assert np.all(err <= bound), (label, float((err / bound).max()))


def flip_mask32(g, o):
    """Walkers of a binary32 run whose transition decisions differ from the
    binary64 oracle's: a different final element, |w| off by more than 1e-3
    relative (the decisions are the same, so |w| = prod(1 + S) agrees to the
    binary32 rounding of the S), or a weight that is finite on one side only."""
    flip = (g["a"] != o["a"]) | (g["b"] != o["b"])
    flip |= ~(np.abs(np.abs(g["w"]) - np.abs(o["w"])) <= 1e-3 * np.abs(o["w"]))
    return flip


def check_ensemble32(out_g, out_o, n_traj, tol=1e-3, label="", g=None, o=None):
    """Asserts every bin of a binary32-propagated result against the FP64
    oracle's: 1e-3 absolute on unit-scale means, 1e-3 relative to the rms
    of the summed terms elsewhere.  With the final states of both runs
    (``g`` binary32, ``o`` oracle), walkers whose decisions differ are
    counted and the bound is widened by their |w| as in the FP64 check: a
    walker that took another branch is another sample, not an error of the
    arithmetic."""
    rms = rms_terms(out_o, n_traj)
    flip = None
    allow = 0.0
    if g is not None:
        flip = flip_mask32(g, o)
        allow = flip_allowance(flip, g, o, n_traj)
    bound = tol * np.maximum(1.0, rms) + allow
    err = np.abs(out_g[..., :2] - out_o[..., :2])
    unit = rms <= 1.0
    abs_unit = float(err[unit].max()) if unit.any() else 0.0
    rel_big = float((err[~unit] / rms[~unit]).max()) if (~unit).any() else 0.0
    fl = "" if flip is None else f"flips {int(flip.sum())}/{flip.size} ({flip.mean():.2%}), allowance {allow:.3g}; "
    print(f"[{label}] fp32 ensemble: {int(unit.sum())} unit-scale means, max abs err {abs_unit:.3g}; "
          f"{int((~unit).sum())} means with rms > 1 (largest {float(rms.max()):.3g}), max err/rms {rel_big:.3g}; "
          f"{fl}max err/bound {float((err / bound).max()):.3g}", flush=True)
    assert np.all(err <= bound), (label, float((err / bound).max()))
    return flip


def gpu_run(P, wl, prec="fp64", n_traj=None, n_steps=None, scheme=0, split=None, expect_excluded=False):
    """Sample, propagate (optionally in several calls) and reduce on the
    device; returns (out, final state, sampled state, ensemble).  With
    ``expect_excluded`` the reduction must report walkers left out of the
    sums (QCL_ERR_NONFINITE); its averages are returned all the same."""
    import torch
    r = wl.run
    T = r.n_traj if n_traj is None else n_traj
    S = r.n_steps if n_steps is None else n_steps
    n_out = S // r.cadence + 1
    model = P.Model(wl.model)
    ens = P.Ensemble(model, T, prec)
    part = P.Partials(model, T, n_out)
    P.qcl_sample_initial(model, wl.init, r.seed, ens, part)
    sample_state = ens.to_numpy()
    chunks = [S] if split is None else split
    assert sum(chunks) == S
    for c in chunks:
        P.qcl_propagate(model, ens, r.dt, c, r.cadence, r.seed, part, scheme)
    out = None
    if T > 0 and expect_excluded:
        try:
            P.qcl_reduce_observables(model, part, T)
        except P.QCLError as e:
            assert e.status == P.QCL_ERR_NONFINITE, e
            print("reduce:", e, flush=True)
            out = e.out
        assert out is not None, "the reduction did not report the excluded walkers"
    elif T > 0:
        out = P.qcl_reduce_observables(model, part, T)
    torch.cuda.synchronize()
    return (out.cpu().numpy() if out is not None else None), ens.to_numpy(), sample_state, ens


def oracle_run(wl, n_traj=None, n_steps=None, scheme=0):
    """The oracle on the same workload; returns (out, final state, sampled
    state, flags)."""
    r = wl.run
    T = r.n_traj if n_traj is None else n_traj
    S = r.n_steps if n_steps is None else n_steps
    n_out = S // r.cadence + 1
    m = oc.Model(wl.model)
    st, s0 = oc.sample(m, wl.init, r.seed, T)
    samp = oracle_state(st.copy())
    sums = np.zeros((n_out, 2, m.n, m.n, 4))
    sums[0] = s0
    oc.propagate(m, st, r.dt, S, r.cadence, r.seed, n_out, sums, scheme)
    return oc.finalize(sums, T), oracle_state(st), samp, st.flags


def sampled_state(ens, ids):
    """Walker-major state of the walkers ``ids`` of a device ensemble."""
    N = ens.model.n_states
    t = ens.tensors()
    import torch
    ix = torch.as_tensor(np.asarray(ids, np.int64), device=t["w"].device)
    return {"q": t["q"][:, ix].cpu().numpy().T.astype(np.float64),
            "p": t["p"][:, ix].cpu().numpy().T.astype(np.float64),
            "U": t["u"][:, ix].cpu().numpy().T.reshape(-1, N, N).astype(np.float64),
            "w": t["w"][ix].cpu().numpy(), "phase": t["phase"][ix].cpu().numpy(),
            "a": t["a"][ix].cpu().numpy().astype(np.int32), "b": t["b"][ix].cpu().numpy().astype(np.int32)}


def oracle_walkers(wl, ids, n_steps=None, scheme=0):
    """The oracle's final state of the walkers with global ids ``ids``, each
    recomputed on its own (its random streams are keyed by its id)."""
    r = wl.run
    S = r.n_steps if n_steps is None else n_steps
    m = oc.Model(wl.model)
    o = {k: [] for k in ("q", "p", "U", "w", "phase", "a", "b")}
    for i in ids:
        st, _ = oc.sample(m, wl.init, r.seed, 1, traj_offset=int(i))
        oc.propagate(m, st, r.dt, S, r.cadence, r.seed, S // r.cadence + 1, scheme=scheme)
        for k, v in oracle_state(st).items():
            o[k].append(v[0])
    return {k: np.array(v) for k, v in o.items()}


def sample_ids(n_traj, n_random, seed=0, extra=()):
    """Walker ids for a sampled check: the first and last walkers, tile
    edges, any ``extra`` ids and ``n_random`` uniform draws."""
    rng = np.random.default_rng(seed)
    edge = [0, 1, 255, 256, 257, n_traj // 2, n_traj - 257, n_traj - 2, n_traj - 1]
    ids = np.concatenate([np.array(edge + list(extra), np.int64), rng.integers(0, n_traj, n_random)])
    ids = ids[(ids >= 0) & (ids < n_traj)]
    return np.unique(ids)
