"""The full-size workloads against the oracle's full runs.

``pyrazine_ci`` (2-state 3-mode conical-intersection model, 1e7 walkers,
1000 steps of 0.5 fs, bins every 10 steps) and the 3-mode Ohmic spin-boson
model at kT 0.2 and 1.0 (1e6 walkers, 2000 steps of 0.02) are run on the
device in both precisions, one launch each as the benchmark does, and
every bin of the reduced result is compared with the oracle's run of the
same walkers (``tests/golden/*_oracle.json``, written by
``tests/golden/make_golden.py`` from the oracle only).

Binary64: every mean within 1e-9 x max(1, rms of its terms), widened by the
|w| of walkers whose decisions differ from the oracle's.  Those walkers are
found from per-group digests of the final state stored with the golden
(sum of |w| and of 2a + b per 4096 consecutive walkers): a group whose
digests differ is recomputed walker by walker by the oracle.

Binary32: every mean within 1e-3 x max(1, rms): 1e-3 absolute while the
terms are of unit scale, 1e-3 relative to them once the weights have
grown.  The binary32 run shares its random streams with the oracle, so the
standard error is not the yardstick.
"""
import json
import os

import numpy as np
import pytest

import oracle.core as oc
import workloads as W
from parity import check_ensemble32, check_ensemble64, flip_mask, oracle_state, rms_terms

pytestmark = pytest.mark.gpu
GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
CASES = {
    "pyrazine_ci": (W.pyrazine_ci, "pyrazine_ci_1e7_oracle.json"),
    "spin_boson_kT0.2": (lambda: W.spin_boson_ohmic(kT=0.2), "spin_boson_ohmic_m3_kT0.2_1e6_oracle.json"),
    "spin_boson_kT1.0": (lambda: W.spin_boson_ohmic(kT=1.0), "spin_boson_ohmic_m3_kT1.0_1e6_oracle.json"),
}


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2608_14544_amd as pkg
    pkg.load_library()
    return pkg


@pytest.fixture(scope="module", params=list(CASES))
def golden(request):
    make, fname = CASES[request.param]
    with open(os.path.join(GOLDEN_DIR, fname)) as f:
        d = json.load(f)
    wl = make()
    d["workload"] = wl
    d["label"] = request.param
    r = wl.run
    assert (d["n_traj"], d["n_steps"], d["cadence"], d["seed"]) == (r.n_traj, r.n_steps, r.cadence, r.seed)
    assert d["dt"] == r.dt
    d["out"] = np.array(d["out"])
    d["group_abs_w"] = np.array(d["group_abs_w"])
    d["group_ab"] = np.array(d["group_ab"], dtype=np.int64)
    return d


def _run(P, prec, wl):
    import torch
    r = wl.run
    model = P.Model(wl.model)
    ens = P.Ensemble(model, r.n_traj, prec, zero=False)
    part = P.Partials(model, r.n_traj, r.n_out)
    P.qcl_sample_initial(model, wl.init, r.seed, ens, part)
    P.qcl_propagate(model, ens, r.dt, r.n_steps, r.cadence, r.seed, part)
    out = P.qcl_reduce_observables(model, part, r.n_traj).cpu().numpy()
    t = ens.tensors()
    T = r.n_traj
    w = t["w"][:T]
    ab = 2 * t["a"][:T].to(torch.int64) + t["b"][:T].to(torch.int64)
    torch.cuda.synchronize()
    return wl, out, w, ab, t


def _group_digests(w, ab, group):
    import torch
    T = w.shape[0]
    n = (T + group - 1) // group
    pad = n * group - T
    aw = torch.nn.functional.pad(w.abs(), (0, pad)).view(n, group)
    abp = torch.nn.functional.pad(ab, (0, pad)).view(n, group)
    # the oracle sums each group's |w| in order with numpy; here the sum only
    # locates groups, so its rounding order does not matter at 1e-9
    return aw.sum(dim=1).cpu().numpy(), abp.sum(dim=1).cpu().numpy()


def test_headline_fp64_every_bin_against_oracle(P, golden):
    wl, out, w, ab, t = _run(P, "fp64", golden["workload"])
    r = wl.run
    G = golden["group"]
    gw, gab = _group_digests(w, ab, G)
    ow, oab = golden["group_abs_w"], golden["group_ab"]
    suspect = np.nonzero((gab != oab) | ~(np.abs(gw - ow) <= 1e-9 * np.abs(ow)))[0]
    print(f"groups whose digests differ: {suspect.size} of {gw.size}", flush=True)
    assert suspect.size <= 20, "too many groups differ from the oracle's"
    # recompute the suspect groups walker by walker
    m = oc.Model(wl.model)
    allow, n_flip = 0.0, 0
    for gi in suspect:
        lo = int(gi) * G
        n = min(G, r.n_traj - lo)
        st, _ = oc.sample(m, wl.init, r.seed, n, traj_offset=lo)
        oc.propagate(m, st, r.dt, r.n_steps, r.cadence, r.seed, r.n_out)
        o = oracle_state(st)
        g = {"w": t["w"][lo:lo + n].cpu().numpy(), "a": t["a"][lo:lo + n].cpu().numpy().astype(np.int32),
             "b": t["b"][lo:lo + n].cpu().numpy().astype(np.int32)}
        flip = flip_mask(g, o)
        n_flip += int(flip.sum())
        allow += float((np.abs(g["w"][flip]).sum() + np.abs(o["w"][flip]).sum()) / r.n_traj)
    print(f"walkers whose decisions differ from the oracle's: {n_flip} of {r.n_traj}", flush=True)
    assert n_flip <= 1e-4 * r.n_traj
    check_ensemble64(out, golden["out"], r.n_traj, tol=1e-9, label=golden["label"] + " fp64", extra_allow=allow)
    # standard errors too, at the same bound relative to the terms' rms
    rms = rms_terms(golden["out"], r.n_traj)
    d_se = np.abs(out[..., 2:] - golden["out"][..., 2:])
    assert np.all(d_se <= 1e-9 * np.maximum(1.0, rms) + allow), float(d_se.max())


def test_headline_fp32_every_bin_against_oracle(P, golden):
    wl, out, w, ab, t = _run(P, "fp32", golden["workload"])
    r = wl.run
    flags = t["flags"][:r.n_traj].cpu().numpy().view(np.uint32)
    print(f"flags: resolved in binary64 {int(np.count_nonzero(flags & 4))}, "
          f"non-finite {int(np.count_nonzero(flags & 1))} (oracle {golden['nonfinite']})", flush=True)
    check_ensemble32(out, golden["out"], r.n_traj, tol=1e-3, label=golden["label"] + " fp32")
    P_up = out[:, 0, 1, 1, 0]
    P_or = golden["out"][:, 0, 1, 1, 0]
    within = np.abs(P_up - P_or) <= 1e-3
    print(f"upper adiabatic population: max |fp32 - oracle| {np.abs(P_up - P_or).max():.3g}, "
          f"{int(within.sum())} of {within.size} bins within 1e-3", flush=True)
