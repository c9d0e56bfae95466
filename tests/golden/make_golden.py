"""Writes the stored expected values under tests/golden/.

Calls only the oracle package (the phase-space grid solver of Eq. 1); no
value here comes from the HIP path.

    python tests/golden/make_golden.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

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


if __name__ == "__main__":
    grid_spin_boson_1mode()
