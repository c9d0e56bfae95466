"""Writes the stored expected values under tests/golden/.

Calls only the oracle package (the phase-space grid solver of Eq. 1 and the
FP64 oracle propagator); no value here comes from the HIP path.

    python tests/golden/make_golden.py            # every file
    python tests/golden/make_golden.py pyrazine   # one of them (grid, pyrazine, spin_boson)
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle.core as oc  # noqa: E402
import workloads as W  # noqa: E402
from oracle.grid import GridSolver  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def grid_spin_boson_1mode():
    wl = W.spin_boson_1mode()
    params = dict(q_range=(-6.0, 5.0), p_range=(-5.5, 5.5), nq=221, npp=221, h=0.01)
    g = GridSolver(wl.model, wl.init, **params)
    ts = [round(0.5 * i, 6) for i in range(11)]
    res = g.run(ts)
    doc = {
        "what": "Eq. 1 solved on a (q,p) grid for the 1-mode 2-state spin-boson model "
                "(eps=0.5, Delta=0.2, g=0.5, w=m=1, kT=0.5, Wigner start on diabatic state 0 "
                "centred at q0=-0.5): ensemble density matrix vs time, adiabatic (U_kk>0 gauge) "
                "and diabatic bases",
        "source": "oracle/grid.py (Strang splitting, semi-Lagrangian bicubic advection, "
                  "exact two-state coupling rotation)",
        "grid": {k: list(v) if isinstance(v, tuple) else v for k, v in params.items()},
        "t": ts,
        "rho_re": res.real.tolist(),   # [t][basis][i][j]
        "rho_im": res.imag.tolist(),
    }
    with open(os.path.join(HERE, "grid_spin_boson_1mode.json"), "w") as f:
        json.dump(doc, f, indent=1)


GROUP = 4096  # walkers per digest group


def full_run(wl, fname, what):
    """One workload at its full size run by the oracle, in slices of 2^20
    walkers (the sums are additive over walkers): the bin sums, the averaged
    observables, and per group of 4096 consecutive walkers two digests of
    the final state, the sum of |w| and the sum of 2a + b, which let a test
    find the groups holding a walker whose transition decisions differ from
    the oracle's."""
    r = wl.run
    m = oc.Model(wl.model)
    T = r.n_traj
    n = m.n
    sums = np.zeros((r.n_out, 2, n, n, 4))
    abs_w, ab = [], []
    nonfinite = 0
    sl = GROUP * 256
    for lo in range(0, T, sl):
        k = min(sl, T - lo)
        st, s0 = oc.sample(m, wl.init, r.seed, k, traj_offset=lo)
        part = np.zeros_like(sums)
        part[0] = s0
        oc.propagate(m, st, r.dt, r.n_steps, r.cadence, r.seed, r.n_out, part)
        sums += part
        nonfinite += int(np.count_nonzero(st.flags & oc.FLAG_NONFINITE))
        for g0 in range(0, k, GROUP):
            w = st.w[g0:g0 + GROUP]
            abs_w.append(float(np.abs(w).sum()))
            ab.append(int((2 * st.a[g0:g0 + GROUP] + st.b[g0:g0 + GROUP]).sum()))
        print(f"{wl.model.name} oracle: {lo + k}/{T} walkers", flush=True)
    out = oc.finalize(sums, T)
    doc = {
        "what": what + " by the oracle: bin sums [n_out][basis][i][j][Re, Im, Re^2, Im^2], averaged "
                "observables [n_out][basis][i][j][mean Re, mean Im, SE Re, SE Im], and per group of 4096 "
                "consecutive walkers the sum of |w| and of 2a + b of the final state",
        "source": "oracle/qcl_oracle.c through oracle/core.py (sample, propagate, finalize)",
        "n_traj": T, "n_steps": r.n_steps, "dt": r.dt, "cadence": r.cadence, "seed": r.seed,
        "group": GROUP, "nonfinite": nonfinite,
        "sums": sums.tolist(), "out": out.tolist(),
        "group_abs_w": abs_w, "group_ab": ab,
    }
    with open(os.path.join(HERE, fname), "w") as f:
        json.dump(doc, f)


def pyrazine_ci_full():
    full_run(W.pyrazine_ci(), "pyrazine_ci_1e7_oracle.json",
             "pyrazine_ci at full size (2-state 3-mode conical-intersection model, 1e7 walkers, 1000 steps "
             "of 0.5 fs, bins every 10 steps, Philox seed 3, diabatic start on the upper state, FP64)")


def spin_boson_full(kT):
    wl = W.spin_boson_ohmic(kT=kT)
    r = wl.run
    full_run(wl, f"spin_boson_ohmic_m3_kT{kT}_1e6_oracle.json",
             f"3-mode Ohmic spin-boson model at kT {kT} at full size (eps 0, Delta 0.5, Kondo parameter 0.1, "
             f"w_c 1; 1e6 walkers, 2000 steps of 0.02, bins every 10 steps, Philox seed {r.seed}, Wigner start "
             f"on diabatic state 0 centred at its minimum, FP64)")


if __name__ == "__main__":
    which = sys.argv[1:] or ["grid", "pyrazine", "spin_boson"]
    if "grid" in which:
        grid_spin_boson_1mode()
    if "pyrazine" in which:
        pyrazine_ci_full()
    if "spin_boson" in which:
        spin_boson_full(0.2)
        spin_boson_full(1.0)
