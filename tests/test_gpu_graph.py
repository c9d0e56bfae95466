"""The hot path under HIP graph capture: sample + propagate + reduce of one
ensemble captured once and replayed several times, with eager work and
synchronisations between the replays; every replay must equal the eager
result bit for bit (the calls allocate nothing, never synchronise and put
no memset node in the graph)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def test_captured_step_replays_bitwise():
    import torch
    import paper_2608_14544_amd as P
    P.load_library()
    for prec, wl in (("fp32", W.pyrazine_ci(n_traj=20_000, n_steps=60, cadence=10)),
                     ("fp64", W.random_lvc(13, n_states=3, n_modes=12, n_traj=3000, n_steps=40, cadence=10))):
        r = wl.run
        model = P.Model(wl.model)
        N = model.n_states
        ens = P.Ensemble(model, r.n_traj, prec)
        part = P.Partials(model, r.n_traj, r.n_out)
        out = torch.empty((r.n_out, 2, N, N, 4), dtype=torch.float64, device="cuda")
        excl = torch.empty(r.n_out, dtype=torch.int64, device="cuda")
        side = torch.cuda.Stream()  # default priority

        def step(stream):
            P.qcl_sample_initial(model, wl.init, r.seed, ens, part, stream)
            ens.c.step = 0  # the host-side counter is what the next call reads
            P.qcl_propagate(model, ens, r.dt, r.n_steps, r.cadence, r.seed, part, stream=stream)
            P.qcl_reduce_observables_async(model, part, r.n_traj, out, excl, stream)

        with torch.cuda.stream(side):
            step(side)
        torch.cuda.synchronize()
        eager = out.cpu().numpy().copy()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            step(side)
        for rep in range(3):
            out.zero_()
            junk = torch.randn(1 << 16, device="cuda").sum()  # eager work between replays
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy(), eager), (prec, rep)
            assert int(excl.max()) == 0
            del junk
