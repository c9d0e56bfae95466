"""Throughput of the QCL walker-ensemble hot path on one MI355X.

One benchmark step = one pass of the whole path over one ensemble:
qcl_sample_initial + qcl_propagate (all time steps) + qcl_reduce_observables
for the two-state three-mode conical-intersection model (pyrazine-like
S2/S1, 1e7 walkers, 1000 steps of 0.5 fs, bins every 10 steps).  Inputs are
synthetic and seeded; the ensemble lives in HBM before timing starts.

value = walkers * time steps / wall time of the step, in trajectory-steps/s,
for the headline precision (binary32 propagation with binary64 phase,
weights and sums).  The plain binary64 path is timed the same way and
reported beside it, with the largest population difference between the
two.  Two further legs are reported in the same line:

  batched  256 seeded N-state (2-4) harmonic instances (1-64 modes, 1e4-1e6
           walkers, 500-4000 steps, binary32) advanced by one
           qcl_propagate_batch call: walker-steps/s of that call;
  served   a Poisson stream of 200 jobs (20 jobs/s) through the
           continuous-batching server: walker-steps/s and p50/p99 latency;
  scaling  the headline model at 1e4..1e8 walkers in both precisions;
  spin_boson  the 3-mode Ohmic spin-boson runs (1e6 walkers, 2000 steps,
           kT 0.2 and 1.0) in both precisions with their population difference;
  convergence  the pyrazine-like and spin-boson (kT 0.2) models at 1e6, 1e7
           and 1e8 walkers: horizons of agreement and the decay rate;
  poly     models with higher powers of each mode (state-dependent
           frequencies, anharmonicity) and with cross-mode bilinear terms;
  many_states  6- and 8-state models on the general kernels.
  resample qcl_resample of the headline ensemble (1e7 walkers) against HBM
           bandwidth, and the replica spread of P(t) with and without
           resampling every 1-10 fs (64 x 1e6 walkers).
  served_full  the served stream with 1e5-1e8 walkers per random job, whose
           offered load exceeds the device.
  general  the general-N kernel classes (4,64), (4,32), (3,64) alone.
  source   models with a supplied potential (coupled Morse states; a
           linear-vibronic model as source and on the built-in kernels).

Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--prec fp32|fp64] [--n-traj T]
                    [--legs headline,batched,served]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3}  # MI355X published dense vector peaks

# HBM bytes of one propagate launch, from the committed rocprofv3 counter
# summary; valid only while the kernel's sources are the ones it measured.
HBM_PROFILE = os.path.join(ROOT, "profiles", "propagate_n2_pyrazine_1e7_hbm_counters.md")
KERNEL_SOURCES = ["kernels_n2.hip", "block_reduce.hpp", "phase_math.hpp", "philox.hpp", "qcl_internal.hpp",
                  "qcl_device.hpp"]


def kernel_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2608_14544_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(n_traj: int, prec: str):
    """Counter-derived bytes per launch if they apply to this build and
    workload, else None."""
    if not os.path.exists(HBM_PROFILE):
        return None
    vals = {}
    for line in open(HBM_PROFILE):
        k, _, v = line.strip().partition(":")
        if k in ("traffic_bytes_per_launch", "n_traj", "precision", "kernel_sources_sha256"):
            vals[k] = v.strip()
    if (vals.get("kernel_sources_sha256") != kernel_sources_sha256() or vals.get("n_traj") != str(n_traj)
            or vals.get("precision") != prec or "traffic_bytes_per_launch" not in vals):
        return None
    return int(vals["traffic_bytes_per_launch"])


def flops_per_traj_step(n_states: int, n_modes: int, slots_per_mode: float, eigen: int = 15) -> float:
    """Algorithmic floating-point work of one walker step (FMA = 2), the
    count the hot-path scope fixes for the linear-vibronic family:
        2 [M (3 s + 4) + E_N + 4 N^2 + 4 (N - 1)]
    with s the mean number of nonzero coupling slots per mode (three
    contractions of V, the forces and the velocity coupling per slot, and
    the kick/drift per mode), E_N the eigen-solve (about 15 for the 2 x 2
    closed form), 4 N^2 for the frame and the phase, 4 (N - 1) for the
    transition.  For the pyrazine-like model (N = 2, M = 3, s = 5/3) it is
    124 flops.  Philox integer work and the bins are not counted."""
    return 2.0 * (n_modes * (3.0 * slots_per_mode + 4.0) + eigen + 4 * n_states * n_states + 4 * (n_states - 1))


def coupling_slots(lvc) -> float:
    """Mean number of nonzero upper-triangle entries of the K_j per mode."""
    import numpy as np
    n = lvc.v0.shape[0]
    iu = np.triu_indices(n)
    return float(np.mean([np.count_nonzero(np.asarray(k)[iu]) for k in lvc.k]))


GOLDEN = os.path.join(ROOT, "tests", "golden", "pyrazine_ci_1e7_oracle.json")


def spin_boson_golden(kT):
    return os.path.join(ROOT, "tests", "golden", f"spin_boson_ohmic_m3_kT{kT}_1e6_oracle.json")


def oracle_accuracy(out, wl, n_traj, prec, golden=GOLDEN):
    """Every bin of a full-size result against the oracle's run of the same
    walkers stored in tests/golden (written from the oracle alone); None
    when the workload differs from the stored one."""
    import numpy as np
    r = wl.run
    if not os.path.exists(golden) or n_traj != r.n_traj:
        return None
    with open(golden) as f:
        g = json.load(f)
    if (g["n_traj"], g["n_steps"], g["cadence"], g["seed"]) != (r.n_traj, r.n_steps, r.cadence, r.seed):
        return None
    ref = np.array(g["out"])
    T = float(n_traj)
    rms = np.sqrt(ref[..., 2:] ** 2 * (T - 1.0) + ref[..., :2] ** 2)
    err = np.abs(out[..., :2] - ref[..., :2])
    tol = 1e-9 if prec == "fp64" else 1e-3
    d_pop = np.abs(out[:, 0, 1, 1, 0] - ref[:, 0, 1, 1, 0])
    fs = wl.model.time_unit_fs
    se = ref[:, 0, 1, 1, 2]
    unresolved = np.nonzero(~(se < 0.01))[0]
    n_res = int(unresolved[0]) if len(unresolved) else len(se)
    until = (n_res - 1) * r.cadence * r.dt * (fs or 1.0) if n_res else None
    return {
        "max_abs_upper_population_diff": float(d_pop.max()),
        "max_abs_upper_population_diff_resolved_bins": float(d_pop[:n_res].max()) if n_res else None,
        "resolved_bins": n_res,
        ("resolved_until_fs" if fs else "resolved_until"): until,
        "bins_within_1e-3": int(np.count_nonzero(d_pop <= 1e-3)),
        "bins": int(d_pop.size),
        "max_err_over_rms_scaled_bound": float((err / (tol * np.maximum(1.0, rms))).max()),
        "bound": f"{tol:g} x max(1, rms of the summed terms), every mean of every bin",
    }


def time_path(P, torch, model, wl, prec, n_traj, steps, warmup):
    r = wl.run
    ens = P.Ensemble(model, n_traj, prec)
    part = P.Partials(model, n_traj, r.n_out)
    n = model.n_states
    out = torch.empty((r.n_out, 2, n, n, 4), dtype=torch.float64, device="cuda")
    excl = torch.empty(r.n_out, dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]

    def one(i=None):
        P.qcl_sample_initial(model, wl.init, r.seed, ens, part, stream)
        if i is not None:
            ev[i][0].record(stream)
        P.qcl_propagate(model, ens, r.dt, r.n_steps, r.cadence, r.seed, part, 0, stream)
        if i is not None:
            ev[i][1].record(stream)
        P.qcl_reduce_observables_async(model, part, n_traj, out, excl, stream)

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        one(i)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / steps
    ms_prop = sum(a.elapsed_time(b) for a, b in ev) / steps
    res = out.cpu().numpy()
    fl = ens.tensors()["flags"][:n_traj]
    time_path.flag_counts = {name: int(((fl & bit) != 0).sum().item())
                             for name, bit in (("nonfinite", 1), ("degenerate", 2), ("resolved64", 4))}
    del ens, part
    return ms_step, ms_prop, res


def _oracle_rate(wl, n):
    """Walker-steps/s of the FP64 oracle on n walkers of ``wl`` (sample +
    propagate + reduce), and the seconds it took."""
    import numpy as np
    import oracle.core as oc
    r = wl.run
    m = oc.Model(wl.model)
    t = time.perf_counter()
    st, s0 = oc.sample(m, wl.init, r.seed, n)
    sums = np.zeros((r.n_out, 2, m.n, m.n, 4))
    sums[0] = s0
    oc.propagate(m, st, r.dt, r.n_steps, r.cadence, r.seed, r.n_out, sums)
    oc.finalize(sums, n)
    dt = time.perf_counter() - t
    return n * r.n_steps / dt, dt


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, target_s: float):
    """The FP64 oracle on the host cores, on a bounded slice of the same
    workload (same model, same 1000 steps, fewer walkers): all threads, and
    one thread in a child process (OMP_NUM_THREADS=1)."""
    import subprocess
    import oracle.core as oc
    cal_n = 16384
    _, dt_cal = _oracle_rate(wl, cal_n)
    n = int(max(cal_n, min(20_000_000, cal_n * target_s / max(dt_cal, 1e-6))))
    n = (n // 1024) * 1024
    rate, dt = _oracle_rate(wl, n)
    # about 5 s on one thread
    n1 = max(1024, (int(5.0 * rate / max(oc.num_threads(), 1) / wl.run.n_steps) // 1024) * 1024)
    code = ("import sys; sys.path.insert(0, %r); import bench, workloads as W; "
            "r, dt = bench._oracle_rate(W.pyrazine_ci(), %d); print(r, dt)" % (ROOT, n1))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    single = None
    try:
        out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=600)
        if out.returncode == 0:
            r1, dt1 = (float(x) for x in out.stdout.split()[-2:])
            single = {"value": r1, "walkers": n1, "seconds": dt1}
    except (subprocess.TimeoutExpired, ValueError):
        single = None
    return {"value": rate, "unit": "trajectory-steps/s", "cores": oc.num_threads(), "kind": "oracle",
            "sample": f"{n} walkers x {wl.run.n_steps} steps of the same model (sample+propagate+reduce), "
                      f"{dt:.1f} s, FP64 C oracle, OpenMP over walkers",
            "cpu_model": _cpu_model(), "single_thread": single, "other_legs": _oracle_other_legs()}


def _oracle_other_legs():
    """The oracle on the other configurations and beside two further legs,
    each bounded to a few seconds: the one-mode spin-boson run at its full
    size (1e4 walkers x 200 steps), the 3-mode Ohmic spin-boson run at kT
    0.2 on 65536 of its 1e6 walkers (all 2000 steps), the bilinear model's
    propagation (65536 walkers x 200 steps) and fixed-budget resampling
    (pure Python, 1e6 walkers with heavy-tailed signed weights)."""
    import numpy as np
    import oracle.core as oc
    import oracle.resample as orr
    import workloads as W
    s1 = W.spin_boson_1mode()
    r1, dt1 = _oracle_rate(s1, s1.run.n_traj)
    so = W.spin_boson_ohmic(kT=0.2)
    ro, dto = _oracle_rate(so, 65536)
    bw = W.pyrazine_bilinear(n_traj=0, n_steps=200, cadence=10)
    rb, dtb = _oracle_rate(bw, 65536)
    T = 1_000_000
    rng = np.random.default_rng(1)
    st = oc.State(T, 2, 3)
    st.q[:] = rng.normal(size=(T, 3))
    st.p[:] = rng.normal(size=(T, 3))
    st.w[:] = rng.lognormal(0.0, 2.5, T) * rng.choice([-1.0, 1.0], T)
    st.phase[:] = rng.uniform(-20, 20, T)
    t0 = time.perf_counter()
    orr.resample(st, 21)
    dtr = time.perf_counter() - t0
    return {"spin_boson_1mode_full": {"value": r1, "unit": "trajectory-steps/s", "cores": oc.num_threads(),
                                      "sample": f"{s1.run.n_traj} walkers x {s1.run.n_steps} steps (the whole "
                                                f"run), {dt1:.3f} s"},
            "spin_boson_ohmic_kT0.2": {"value": ro, "unit": "trajectory-steps/s", "cores": oc.num_threads(),
                                       "sample": f"65536 of {so.run.n_traj} walkers x {so.run.n_steps} steps, "
                                                 f"{dto:.2f} s"},
            "pyrazine_bilinear": {"value": rb, "unit": "trajectory-steps/s", "cores": oc.num_threads(),
                                  "sample": f"65536 walkers x 200 steps, {dtb:.2f} s"},
            "resample": {"value": T / dtr, "unit": "walkers/s", "cores": 1,
                         "sample": f"{T} walkers (2 states, 3 modes), {dtr:.2f} s, Python integers"}}


def spin_boson_leg(P, torch):
    """The 3-mode Ohmic spin-boson runs (1e6 walkers, 2000 steps) at kT 0.2
    and 1.0, FP32_ACC64 beside FP64, with the largest population difference
    between the two over the bins the FP64 run resolves (SE < 0.01), and
    every bin of each against the oracle's run of the same walkers."""
    import numpy as np
    import workloads as W
    out = []
    for kT in (0.2, 1.0):
        wl = W.spin_boson_ohmic(kT=kT)
        r = wl.run
        model = P.Model(wl.model)
        res = {}
        for prec in ("fp32", "fp64"):
            ms_step, ms_prop, o = time_path(P, torch, model, wl, prec, r.n_traj, 3, 1)
            res[prec] = (ms_step, ms_prop, o)
        r64, r32 = res["fp64"][2], res["fp32"][2]
        se = np.max(np.stack([r64[:, 0, i, i, 2] for i in range(2)]), axis=0)
        bad = np.nonzero(~(se < 0.01))[0]
        n_res = int(bad[0]) if len(bad) else len(se)
        dpop = max(float(np.max(np.abs(r32[:n_res, 0, i, i, 0] - r64[:n_res, 0, i, i, 0]))) for i in range(2))
        gold = spin_boson_golden(kT)
        out.append({"kT": kT, "n_traj": r.n_traj, "n_steps": r.n_steps,
                    "fp32": {"value": r.n_traj * r.n_steps / (res["fp32"][0] / 1e3), "ms": res["fp32"][0]},
                    "fp64": {"value": r.n_traj * r.n_steps / (res["fp64"][0] / 1e3), "ms": res["fp64"][0]},
                    "fp32_vs_fp64_max_abs_population_diff": dpop, "resolved_bins": n_res, "bins": len(se),
                    "fp32_vs_oracle": oracle_accuracy(r32, wl, r.n_traj, "fp32", gold),
                    "fp64_vs_oracle": oracle_accuracy(r64, wl, r.n_traj, "fp64", gold),
                    "oracle": f"FP64 CPU oracle run of the same 1e6 walkers ({os.path.relpath(gold, ROOT)})"})
        torch.cuda.empty_cache()
    return out


def poly_leg(P, torch):
    """Models with higher powers of each mode (general kernels, every
    coupling direction kept): the pyrazine-like model with state-dependent
    frequencies and a quartic tuning mode (1e7 walkers, 200 steps of 0.5 fs)
    and a 3-state, 16-mode quartic model (1e6 walkers, 200 steps), then the
    same pyrazine-like model with two cross-mode bilinear terms (1e7
    walkers, 200 steps), a 3-state, 16-mode quartic model with four, and a
    2-state, 8-mode model with every pair of modes coupled by a mixing
    shared by the states (sixteen squared combinations; 1e6 walkers), both
    precisions; walker-steps/s of sample + propagate + reduce and the
    propagate kernel's own time."""
    import workloads as W
    cases = (("pyrazine_qvc", W.pyrazine_qvc(n_traj=10_000_000, n_steps=200, cadence=10)),
             ("poly_n3_m16_d4", W.random_poly(20, n_states=3, n_modes=16, degree=4, n_traj=1_000_000,
                                               n_steps=200, cadence=10, dt=0.02)),
             ("pyrazine_bilinear", W.pyrazine_bilinear(n_traj=10_000_000, n_steps=200, cadence=10)),
             ("bilinear_n3_m16_d4_p4", W.random_bilinear(20, n_states=3, n_modes=16, n_pairs=4, degree=4,
                                                         n_traj=1_000_000, n_steps=200, cadence=10, dt=0.02)),
             ("bilinear_n2_m8_all_shared", W.random_bilinear(21, n_states=2, n_modes=8, all_pairs=True, shared=True,
                                                             n_traj=1_000_000, n_steps=200, cadence=10)))
    return _model_runs(P, torch, cases)


def many_states_leg(P, torch):
    """Models with 6 and 8 electronic states (general kernels, odd-even
    transposition sort): a 6-state, 8-mode model with rank-1 couplings and an
    8-state, 8-mode model whose couplings span 8 directions (all 36 kept),
    1e6 walkers x 200 steps, both precisions."""
    import numpy as np
    import workloads as W
    dense = W.random_lvc(61, n_states=8, n_modes=8, n_traj=1_000_000, n_steps=200, cadence=10)
    rng = np.random.Generator(np.random.Philox(key=[9, 61]))
    k = dense.model.k.copy()
    for j in range(8):
        a = rng.uniform(-0.05, 0.05, size=(8, 8))
        k[j] += 0.5 * (a + a.T)
    dense.model = W.LVCModel(name="random_lvc_n8_dense", mass=dense.model.mass, omega=dense.model.omega,
                             v0=dense.model.v0, k=k)
    cases = (("lvc_n6_m8_rank1", W.random_lvc(60, n_states=6, n_modes=8, n_traj=1_000_000, n_steps=200,
                                              cadence=10)),
             ("lvc_n8_m8_dense", dense))
    return _model_runs(P, torch, cases)


def resample_leg(P, torch, n_traj=10_000_000, reps=20, replicas=64, replica_traj=1_000_000):
    """Fixed-budget resampling (qcl_resample) of the headline ensemble
    (pyrazine-like model, 1e7 walkers, binary32, after 200 steps): device
    time per call from HIP events on the launch stream and the rate against
    HBM, counting the algorithmic bytes (every walker's state read once and
    written once).  Then the replica study: 64 runs of 1e6 walkers on
    disjoint id ranges over 30 fs (1 fs bins), resampled every 1, 2, 5 or
    10 fs or never, with the replica spread of the excited population at
    10, 20 and 30 fs."""
    import workloads as W
    from paper_2608_14544_amd import branching
    wl = W.pyrazine_ci()
    r = wl.run
    prec = "fp32"
    model = P.Model(wl.model)
    src = P.Ensemble(model, n_traj, prec)
    dst = P.Ensemble(model, n_traj, prec)
    part = P.Partials(model, n_traj, 2)
    stream = torch.cuda.current_stream()
    P.qcl_sample_initial(model, wl.init, r.seed, src, part, stream)
    P.qcl_propagate(model, src, r.dt, 200, 200, r.seed, part, 0, stream)
    ws = P.qcl_resample(model, src, dst, r.seed, None, stream)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record(stream)
        P.qcl_resample(model, src, dst, r.seed, ws, stream)
        b.record(stream)
    torch.cuda.synchronize()
    ms = sum(a.elapsed_time(b) for a, b in ev) / reps
    M, N = model.n_modes, model.n_states
    rs = 4 if prec == "fp32" else 8
    state_bytes = (2 * M + N * N) * rs + 8 + 8 + 1 + 1 + 4
    alg = 2 * state_bytes * n_traj
    del src, dst, part, ws
    torch.cuda.empty_cache()
    out = {"n_traj": n_traj, "prec": prec, "ms": ms, "walkers_per_s": n_traj / (ms / 1e3),
           "algorithmic_bytes_per_walker": 2 * state_bytes, "GB_per_s": alg / (ms / 1e3) / 1e9,
           "frac_of_hbm_peak": alg / (ms / 1e3) / 8e12}
    # the same on a binary64 ensemble (sampled; the state arrays double in size)
    src = P.Ensemble(model, n_traj, "fp64")
    dst = P.Ensemble(model, n_traj, "fp64")
    part = P.Partials(model, n_traj, 2)
    P.qcl_sample_initial(model, wl.init, r.seed, src, part, stream)
    P.qcl_propagate(model, src, r.dt, 200, 200, r.seed, part, 0, stream)
    ws = P.qcl_resample(model, src, dst, r.seed, None, stream)
    for a, b in ev:
        a.record(stream)
        P.qcl_resample(model, src, dst, r.seed, ws, stream)
        b.record(stream)
    torch.cuda.synchronize()
    ms64 = sum(a.elapsed_time(b) for a, b in ev) / reps
    sb64 = (2 * M + N * N) * 8 + 22
    out["fp64"] = {"ms": ms64, "algorithmic_bytes_per_walker": 2 * sb64,
                   "GB_per_s": 2 * sb64 * n_traj / (ms64 / 1e3) / 1e9,
                   "frac_of_hbm_peak": 2 * sb64 * n_traj / (ms64 / 1e3) / 8e12}
    del src, dst, part, ws
    torch.cuda.empty_cache()
    sw = W.pyrazine_ci(n_traj=0, n_steps=60, cadence=2)
    if not replicas:
        return out
    out["replicas"] = {"n_traj": replica_traj, "replicas": replicas, "steps": 60,
                       "dt_fs": sw.run.dt * sw.model.time_unit_fs,
                       "by_interval": branching.replica_spread(sw, replica_traj, replicas, [None, 2, 4, 10, 20],
                                                               [10.0, 20.0, 30.0], prec)}
    return out


def _model_runs(P, torch, cases):
    out = []
    for name, wl in cases:
        r = wl.run
        model = P.Model(wl.model)
        row = {"model": name, "n_states": model.n_states, "n_modes": model.n_modes, "degree": model.degree,
               "pairs": model.n_pairs, "rank": model.rank, "n_traj": r.n_traj, "n_steps": r.n_steps}
        for prec in ("fp32", "fp64"):
            ms_step, ms_prop, _ = time_path(P, torch, model, wl, prec, r.n_traj, 3, 1)
            row[prec] = {"value": r.n_traj * r.n_steps / (ms_step / 1e3), "ms": ms_step, "propagate_ms": ms_prop,
                         "flags": dict(time_path.flag_counts)}
            torch.cuda.empty_cache()
        out.append(row)
    return out


def batched_leg(P, torch, n_instances=256):
    """One qcl_propagate_batch call over the seeded heterogeneous instances
    (ensembles sampled beforehand, resident in HBM)."""
    import workloads as W
    from paper_2608_14544_amd.tune import autotune, launch_class
    wls = W.batched_instances(n_instances)
    t0 = time.perf_counter()
    table = autotune(wls, "fp32")  # untimed: one short run per kernel class and build
    seen = {}
    for wl in wls:  # workgroups per CU, per launch class (the instance with the most walkers)
        m = P.Model(wl.model)
        k = launch_class(m, "fp32")
        if k not in seen or wl.run.n_traj > seen[k][0].run.n_traj:
            seen[k] = (wl, m)
    for wl, m in seen.values():
        table.tune_workgroups(wl, "fp32", model=m)
    tune_s = time.perf_counter() - t0
    jobs, tot = [], 0
    stream = torch.cuda.current_stream()
    for wl in wls:
        r = wl.run
        model = P.Model(wl.model)
        ens = P.Ensemble(model, r.n_traj, "fp32", zero=False)
        part = P.Partials(model, r.n_traj, r.n_out)
        P.qcl_sample_initial(model, wl.init, r.seed, ens, part, stream)
        jobs.append(P.BatchJob(model, ens, part, r.dt, r.n_steps, r.cadence, r.seed,
                               occupancy=table.occupancy(model, "fp32"),
                               workgroups_per_cu=table.workgroups_per_cu(model, "fp32")))
        tot += r.n_traj * r.n_steps
    ws = P.Workspace()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    P.qcl_propagate_batch(jobs, ws, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    return {"workload": f"{n_instances} seeded N-state harmonic instances (N 2-4, M 1-64, 1e4-1e6 walkers, "
                        "500-4000 steps), fp32, one qcl_propagate_batch call",
            "value": tot / (ms / 1e3), "unit": "trajectory-steps/s", "walker_steps": tot,
            "ms": ms, "wall_ms": wall * 1e3,
            "autotune": {
                "seconds": tune_s,
                "register_budget": {"classes": len(table.choice), "capped": sum(1 for v in table.choice.values() if v),
                                    "chosen": {"x".join(map(str, k[:3])): v for k, v in table.choice.items()},
                                    "gain": {"x".join(map(str, k[:3])): t[0] / min(t.values())
                                             for k, t in table.timings.items()}},
                "workgroups_per_cu": {"classes": len(table.wpc), "capped": sum(1 for v in table.wpc.values() if v),
                                      "chosen": {"x".join(map(str, k[:5])): v for k, v in table.wpc.items()},
                                      "gain": {"x".join(map(str, k[:5])): t[0] / min(t.values())
                                               for k, t in table.wpc_timings.items()}}}}, table


GENERAL_CLASSES = ((4, 64), (4, 32), (3, 64))


def general_leg(P, torch, n_traj=1 << 20, n_steps=200):
    """The general-N kernel classes that dominate the batched workload, each
    on one of its instances run alone (binary32 at the tuner's register
    budget, and binary64): walker-steps/s of one qcl_propagate call."""
    import workloads as W
    from paper_2608_14544_amd.tune import TuningTable, padded_modes
    wls = W.batched_instances(256)
    table = TuningTable()
    rows = []
    for n, mp in GENERAL_CLASSES:
        cands = [wl for wl in wls if wl.model.n_states == n and padded_modes(wl.model.n_modes) == mp]
        wl = max(cands, key=lambda w: w.model.n_modes)
        r = wl.run
        model = P.Model(wl.model)
        row = {"class": f"N={n} padded modes {mp}", "instance": wl.model.name, "n_modes": wl.model.n_modes,
               "n_traj": n_traj, "n_steps": n_steps}
        for prec in ("fp32", "fp64"):
            occ = table.tune(wl, prec, model=model) if prec == "fp32" else 0
            ens = P.Ensemble(model, n_traj, prec, zero=False)
            part = P.Partials(model, n_traj, n_steps // r.cadence + 1)
            P.qcl_sample_initial(model, wl.init, r.seed, ens, part)
            P.qcl_propagate(model, ens, r.dt, r.cadence, r.cadence, r.seed, part, occupancy=occ)  # warm-up
            torch.cuda.synchronize()
            s = torch.cuda.current_stream()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            P.qcl_propagate(model, ens, r.dt, n_steps - r.cadence, r.cadence, r.seed, part, 0, s, occupancy=occ)
            e1.record(s)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            row[prec] = {"ms": ms, "value": n_traj * (n_steps - r.cadence) / (ms / 1e3), "occupancy": occ}
            del ens, part
            torch.cuda.empty_cache()
        rows.append(row)
    return rows


def source_leg(P, torch, n_traj=1 << 20, n_steps=200):
    """Models with a supplied potential: the coupled Morse model, and a
    3-state 4-mode linear-vibronic model both as a supplied potential and on
    the built-in general kernels (the cost of the generic path); in binary64
    and binary32, walker-steps/s of one qcl_propagate call, and the time to
    build the model (run-time compilation)."""
    import workloads as W
    lvc = W.random_lvc(7, n_states=3, n_modes=4)
    cases = [("morse_coupled", W.morse_coupled()), ("random_lvc_3_4_source", W.Workload(
        W.lvc_as_source(lvc.model), lvc.init, lvc.run)), ("random_lvc_3_4_builtin", lvc)]
    rows = []
    for name, wl in cases:
        r = wl.run
        t0 = time.perf_counter()
        model = P.Model(wl.model)
        build_s = time.perf_counter() - t0
        row = {"model": name, "n_states": wl.model.n_states, "n_modes": wl.model.n_modes, "n_traj": n_traj,
               "n_steps": n_steps - r.cadence, "model_build_s": build_s}
        for prec in ("fp64", "fp32"):
            ens = P.Ensemble(model, n_traj, prec, zero=False)
            part = P.Partials(model, n_traj, n_steps // r.cadence + 1)
            P.qcl_sample_initial(model, wl.init, r.seed, ens, part)
            P.qcl_propagate(model, ens, r.dt, r.cadence, r.cadence, r.seed, part)  # warm-up
            torch.cuda.synchronize()
            s = torch.cuda.current_stream()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            P.qcl_propagate(model, ens, r.dt, n_steps - r.cadence, r.cadence, r.seed, part, 0, s)
            e1.record(s)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            row[prec] = {"ms": ms, "value": n_traj * (n_steps - r.cadence) / (ms / 1e3)}
            del ens, part
            torch.cuda.empty_cache()
        row["value"] = row["fp64"]["value"]  # binary64 rate (earlier lines' key)
        rows.append(row)
        del model
    return rows


def served_leg(P, torch, n_jobs=200, rate=20.0, quantum=2000, full=False, table=None, quantum_work=2e8,
               tune_quantum=True, min_steps=1):
    """The served stream through the continuous-batching server.  Default:
    the sub-saturation variant (walkers log-uniform over 1e5-1e7); ``full``
    uses 1e5-1e8, whose offered load exceeds one device.  The serving
    quantum and its step floor are tuned on the first 30 % of this stream
    (each stream its own) unless ``tune_quantum`` is false, in which case
    every job advances ``quantum_work`` walker-steps and at least
    ``min_steps`` steps per round."""
    import workloads as W
    from paper_2608_14544_amd.serve import DeviceBackend, JobSpec, Server, latency_stats
    traj_range = (1e5, 1e8) if full else (1e5, 1e7)
    arrivals, wls = W.served_stream(n_jobs, rate=rate, traj_range=traj_range)
    specs = [JobSpec(wl, prec="fp32", name=f"{i}:{wl.model.name}") for i, wl in enumerate(wls)]
    from paper_2608_14544_amd.tune import TuningTable, autotune
    table = autotune(wls, "fp32", table if table is not None else TuningTable())  # untimed; kept if tuned
    if tune_quantum:
        k = max(1, n_jobs * 3 // 10)  # the first 30 % of the stream, served once per candidate

        def run_prefix(q, ms):
            s = Server(DeviceBackend(tuning=table), quantum_steps=quantum, quantum_work=q, min_steps=ms)
            return latency_stats(s.run(arrivals[:k], specs[:k]))
        table.tune_quantum(run_prefix)
        print(f"[bench] serving quantum: {table.quantum_work():.0e} walker-steps per job per round, at least "
              f"{table.min_steps()} steps (p99 on the first {k} jobs: " +
              ", ".join(f"{q:.0e}/{ms}: {v['p99_s']:.3f} s" for (q, ms), v in table.serving_timings.items()) + ")",
              file=sys.stderr, flush=True)
        quantum_work = table.quantum_work(quantum_work)
        min_steps = table.min_steps(min_steps)
    backend = DeviceBackend(tuning=table)
    srv = Server(backend, quantum_steps=quantum, quantum_work=quantum_work, min_steps=min_steps)
    done = []

    def progress(r):
        done.append(r)
        if len(done) % 20 == 0 or len(done) == n_jobs:
            print(f"[bench] served ({'full' if full else 'sub-saturation'}): {len(done)}/{n_jobs} jobs done at "
                  f"{r.finished:.1f} s", file=sys.stderr, flush=True)

    res = srv.run(arrivals, specs, on_result=progress)
    st = latency_stats(res)
    if not full:  # the same stream with a fixed 50-step quantum per job, for comparison
        srv2 = Server(DeviceBackend(tuning=table), quantum_steps=50)
        st2 = latency_stats(srv2.run(arrivals, specs))
        st["fixed_50_step_quantum"] = {k: st2[k] for k in ("p50_s", "p99_s", "walker_steps_per_s", "makespan_s")}
    kinds = {}
    for rr in res:
        kind = rr.name.split(":", 1)[1] if ":" in rr.name else "job"
        kind = "random_lvc" if kind.startswith("random_lvc") else kind
        kinds.setdefault(kind, []).append(rr)
    st["by_kind"] = {k: {kk: latency_stats(v)[kk] for kk in ("n_jobs", "p50_s", "p99_s")} for k, v in kinds.items()}
    offered = sum(sp.walker_steps for sp in specs) / max(arrivals[-1], 1e-9)
    st.update({"workload": f"{n_jobs} jobs, Poisson arrivals at {rate} jobs/s, equal odds of: 1-mode spin-boson, "
                           "3-mode spin-boson kT 0.2, the same at kT 1.0, pyrazine-like CI (1e7 walkers), N-state "
                           f"(2-4) harmonic model with M log-U[1,100], walkers log-U[{traj_range[0]:.0e},"
                           f"{traj_range[1]:.0e}], 500-2000 steps; fp32",
               "variant": "full" if full else "sub-saturation",
               "offered_walker_steps_per_s": offered,
               "rounds": srv.rounds, "quantum": f"{quantum_work:.0e} walker-steps per job per round, "
                                                 f"at least {min_steps} and at most {quantum} steps",
               "quantum_tuning": {f"{q:.0e} walker-steps, at least {ms} steps":
                                  {kk: v.get(kk) for kk in ("p50_s", "p99_s", "walker_steps_per_s")}
                                  for (q, ms), v in table.serving_timings.items()} if tune_quantum else None,
               "host_enqueue_s": backend.host_s, "host_enqueue_s_per_round": backend.host_s / max(srv.rounds, 1),
               "host_enqueue_fraction_of_makespan": backend.host_s / st["makespan_s"] if st.get("makespan_s") else None,
               "memory_budget_GB": srv.budget / 1e9})
    return st


def scaling_leg(P, torch, wl, sizes=(10_000, 100_000, 1_000_000, 10_000_000, 100_000_000)):
    """Time of one sample+propagate+reduce pass of the headline model
    against the walker count, both precisions (time should be linear)."""
    out = []
    r = wl.run
    model = P.Model(wl.model)
    for prec in ("fp32", "fp64"):
        for T in sizes:
            ms_step, ms_prop, _ = time_path(P, torch, model, wl, prec, T, 1, 1 if T <= 1_000_000 else 0)
            out.append({"prec": prec, "n_traj": T, "ms": ms_step, "propagate_ms": ms_prop,
                        "walker_steps_per_s": T * r.n_steps / (ms_step / 1e3)})
            torch.cuda.empty_cache()
    return out


def _json_safe(x):
    """inf/NaN -> None (the JSON line stays strict JSON)."""
    if isinstance(x, float):
        return x if math.isfinite(x) else None
    if isinstance(x, dict):
        return {k: _json_safe(v) for k, v in x.items()}
    if isinstance(x, (list, tuple)):
        return [_json_safe(v) for v in x]
    return x


def convergence_leg(P, torch, counts=(10**6, 10**7, 10**8)):
    """Walker-count convergence (the paper's Figs. 3-4): the pyrazine-like
    model over 100 fs in 1 fs bins and the 3-mode spin-boson model (kT 0.2)
    at 1e6, 1e7 and 1e8 walkers on disjoint walker-id ranges, both
    precisions; per run the device time, the resolved and agreement
    horizons (tolerance 0.02 in population) and, for the pyrazine-like
    model, the decay rate of the excited adiabatic population."""
    import workloads as W
    from paper_2608_14544_amd import study
    res = {}
    cases = (("pyrazine_ci", W.pyrazine_ci(n_traj=0, n_steps=200, cadence=2), True),
             ("spin_boson_kT0.2", W.spin_boson_ohmic(kT=0.2, n_traj=0), False))
    for name, wl, fit in cases:
        for prec in ("fp32", "fp64"):
            summary, _ = study.walker_study(wl, counts, prec=prec, tol=0.02, fit=fit)
            summary["time_unit"] = "fs" if wl.model.time_unit_fs else "reduced"
            summary["n_steps"], summary["cadence"] = wl.run.n_steps, wl.run.cadence
            res[f"{name}_{prec}"] = _json_safe(summary)
            torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--prec", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--n-traj", type=int, default=None)
    ap.add_argument("--no-compare", action="store_true", help="skip timing the other precision")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--legs", default="headline,spin_boson,batched,served,served_full,scaling,convergence,poly,"
                    "many_states,resample,general,source",
                    help="comma-separated subset of the default legs")
    ap.add_argument("--resample-replicas", type=int, default=64,
                    help="replicas of the resampling study (0: time the resampling only)")
    ap.add_argument("--served-jobs", type=int, default=200)
    ap.add_argument("--served-quantum-work", type=float, default=2e8,
                    help="walker-steps per resident job per serving round")
    ap.add_argument("--served-min-steps", type=int, default=1,
                    help="with --served-no-tune: steps every resident job advances at least per serving round")
    ap.add_argument("--served-no-tune", action="store_true",
                    help="serve at --served-quantum-work instead of tuning the quantum on a prefix")
    ap.add_argument("--served-full", action="store_true",
                    help="the served leg uses 1e5-1e8 walkers per random job (as the served_full leg does)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the walker ensemble would shard by global walker id, each GPU reducing its own "
              "tiles, with one gather of the per-GPU partial sums at the end)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2608_14544_amd as P
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        n = 1 << 30
        src = torch.ones(n // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "copies": 3}), flush=True)
        return
    wl = W.pyrazine_ci()
    n_traj = args.n_traj or wl.run.n_traj
    r = wl.run
    model = P.Model(wl.model)
    print(f"[bench] {wl.model.name}: {n_traj} walkers x {r.n_steps} steps, prec {args.prec}", file=sys.stderr,
          flush=True)

    ms_step, ms_prop, res = time_path(P, torch, model, wl, args.prec, n_traj, args.steps, args.warmup)
    flags = dict(time_path.flag_counts)
    tsteps = n_traj * r.n_steps
    value = tsteps / (ms_step / 1e3)
    fl = flops_per_traj_step(wl.model.n_states, wl.model.n_modes, coupling_slots(wl.model))
    achieved = fl * tsteps / (ms_prop / 1e3) / 1e12
    peak = PEAK_TFLOPS[args.prec]
    line = {
        "metric": "trajectory-steps/s FP32 vs FP64 (3-mode CI model, 1e7 traj); p50/p99 job latency",
        "value": value,
        "unit": "trajectory-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64acc" if args.prec == "fp32" else "f64",
        "data": "synthetic (seeded Wigner sampling of the model; no dataset)",
        "config": {"workload": "pyrazine_ci: 2-state 3-mode LVC conical intersection, "
                               f"{n_traj} walkers, {r.n_steps} steps of 0.5 fs, bins every {r.cadence} steps",
                   "n_traj": n_traj, "n_steps": r.n_steps, "cadence": r.cadence, "precision": args.prec},
        "propagate_ms": ms_prop,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": measured_traffic(n_traj, args.prec),
                     "traffic_unit": "bytes per launch (HBM, FETCH_SIZE x2 + WRITE_SIZE, copy-calibrated)",
                     "kernel": "propagate_n2_kernel", "flops_per_traj_step": fl},
    }
    print(f"[bench] {args.prec}: {ms_step:.2f} ms/step, propagate {ms_prop:.2f} ms", file=sys.stderr, flush=True)

    if not args.no_compare:
        other = "fp64" if args.prec == "fp32" else "fp32"
        ms2, mp2, res2 = time_path(P, torch, model, wl, other, n_traj, args.steps, args.warmup)
        r64 = res2 if other == "fp64" else res
        r32 = res if other == "fp64" else res2
        # The estimator's variance grows with the walker weights (prod(1+S));
        # compare the two precisions over the bins the ensemble resolves
        # (population standard error below 0.01).
        se_pop = np.max(np.stack([r64[:, 0, i, i, 2] for i in range(2)]), axis=0)
        unresolved = np.nonzero(~(se_pop < 0.01))[0]
        n_res = int(unresolved[0]) if len(unresolved) else len(se_pop)
        window = slice(0, n_res)
        dpop = max(float(np.max(np.abs(r32[window, 0, i, i, 0] - r64[window, 0, i, i, 0]))) for i in range(2)) \
            if n_res else None
        dcoh = float(np.max(np.abs(r32[window, 1, 0, 1, :2] - r64[window, 1, 0, 1, :2]))) if n_res else None
        dt_fs = r.dt * (wl.model.time_unit_fs or 1.0)
        line[other] = {"value": tsteps / (ms2 / 1e3), "ms_per_step": ms2, "propagate_ms": mp2,
                       "roofline_frac": fl * tsteps / (mp2 / 1e3) / 1e12 / PEAK_TFLOPS[other]}
        line["accuracy"] = {
            "fp32_vs_oracle": oracle_accuracy(r32, wl, n_traj, "fp32"),
            "fp64_vs_oracle": oracle_accuracy(r64, wl, n_traj, "fp64"),
            "oracle": "FP64 CPU oracle run of the same 1e7 walkers (tests/golden/pyrazine_ci_1e7_oracle.json)",
            "fp32_vs_fp64_max_abs_population_diff_resolved": dpop,
            "fp32_vs_fp64_max_abs_diabatic_coherence_diff_resolved": dcoh,
            "resolved_bins": n_res,
            "resolved_until_fs": (n_res - 1) * r.cadence * dt_fs if n_res else 0.0,
            "resolved_criterion": "population SE < 0.01 (fp64 run); later bins are dominated by the weight growth "
                                  "prod(1 + S) (sign problem)",
            "population_se_at_last_bin": float(se_pop[-1]),
            f"{args.prec}_walker_flags": flags,
        }
        print(f"[bench] {other}: {ms2:.2f} ms/step, propagate {mp2:.2f} ms; max |dP| {dpop} over {n_res} "
              f"resolved bins", file=sys.stderr, flush=True)

    legs = set(args.legs.split(","))
    if "spin_boson" in legs:
        line["spin_boson"] = spin_boson_leg(P, torch)
        print(f"[bench] spin-boson: " + ", ".join(
            f"kT {x['kT']}: fp32 {x['fp32']['value']:.3e}, fp64 {x['fp64']['value']:.3e}, "
            f"|dP| {x['fp32_vs_fp64_max_abs_population_diff']:.1e} over {x['resolved_bins']}/{x['bins']} bins"
            for x in line["spin_boson"]), file=sys.stderr, flush=True)
    table = None
    if "batched" in legs:
        line["batched"], table = batched_leg(P, torch)
        print(f"[bench] batched: {line['batched']['value']:.3e} trajectory-steps/s "
              f"({line['batched']['ms']:.0f} ms)", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
    if "served" in legs:
        line["served"] = served_leg(P, torch, args.served_jobs, full=args.served_full, table=table,
                                    quantum_work=args.served_quantum_work, tune_quantum=not args.served_no_tune,
                                    min_steps=args.served_min_steps)
        print(f"[bench] served: {line['served']}", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
    if "served_full" in legs and not args.served_full:
        line["served_full"] = served_leg(P, torch, args.served_jobs, full=True, table=table,
                                         quantum_work=args.served_quantum_work,
                                         tune_quantum=not args.served_no_tune, min_steps=args.served_min_steps)
        print(f"[bench] served (1e5-1e8 walkers): {line['served_full']}", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
    if "general" in legs:
        line["general"] = general_leg(P, torch)
        print("[bench] general: " + "; ".join(f"{x['class']} fp32 {x['fp32']['value']:.3e}, fp64 {x['fp64']['value']:.3e}"
                                              for x in line["general"]), file=sys.stderr, flush=True)
    if "source" in legs:
        line["source"] = source_leg(P, torch)
        print("[bench] supplied potentials: " + "; ".join(
            f"{x['model']} fp64 {x['fp64']['value']:.3e} fp32 {x['fp32']['value']:.3e} (build {x['model_build_s']:.2f} s)"
            for x in line["source"]),
            file=sys.stderr, flush=True)
    if "scaling" in legs:
        line["scaling_sweep"] = scaling_leg(P, torch, wl)
        print(f"[bench] scaling sweep: " + ", ".join(f"{x['prec']} {x['n_traj']:.0e}: {x['ms']:.1f} ms"
                                                    for x in line["scaling_sweep"]), file=sys.stderr, flush=True)
    if "poly" in legs:
        line["poly"] = poly_leg(P, torch)
        print("[bench] poly: " + "; ".join(f"{x['model']} fp32 {x['fp32']['value']:.3e}, fp64 {x['fp64']['value']:.3e}"
                                           for x in line["poly"]), file=sys.stderr, flush=True)
    if "many_states" in legs:
        line["many_states"] = many_states_leg(P, torch)
        print("[bench] many states: " + "; ".join(
            f"{x['model']} fp32 {x['fp32']['value']:.3e}, fp64 {x['fp64']['value']:.3e}"
            for x in line["many_states"]), file=sys.stderr, flush=True)
    if "resample" in legs:
        line["resample"] = resample_leg(P, torch, replicas=args.resample_replicas)
        rs = line["resample"]
        print(f"[bench] resample: {rs['ms']:.3f} ms per 1e7 walkers, {rs['GB_per_s']:.0f} GB/s"
              + ("; replica SD " + ", ".join(f"{k} {v['replica_sd']}" for k, v in rs["replicas"]["by_interval"].items())
                 if "replicas" in rs else ""), file=sys.stderr, flush=True)
    if "convergence" in legs:
        line["convergence"] = convergence_leg(P, torch)
        for key, v in line["convergence"].items():
            print(f"[bench] convergence {key}: " + "; ".join(
                f"{r['n_traj']:.0e} {r['seconds']:.2f} s resolved<={r['resolved_until']}"
                + (f" rate {r['rate']:.4f}+-{r['rate_se']:.4f}" if r.get("rate") is not None else "")
                for r in v["runs"]), file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
