"""Models with a supplied potential (qcl_create_model_source): the device
source is compiled with the library's kernels at model creation, and the
binary64 path is compared with the FP64 oracle's callback path
(``c_source``, an independent C transcription of the same formulas).

Cases: two coupled Morse states whose coupling depends on both modes (not
separable, not linear-vibronic), and linear-vibronic models written as
supplied potentials (N = 3 and 4, normalized and linear rules), whose GPU
results must also agree with the built-in kernels' to the same tolerance.
Tolerances as for the built-in binary64 path: 1e-10 relative per walker
with flipped decisions counted, every bin within 1e-9 (rms-scaled where
the weights have grown) plus the flipped walkers' allowance.
"""
import numpy as np
import pytest

import workloads as W
from parity import check_ensemble64, compare_walkers, gpu_run, oracle_run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2608_14544_amd as pkg
    pkg.load_library()
    return pkg


def _lvc_source(index, n_states, n_modes, **kw):
    wl = W.random_lvc(index, n_states=n_states, n_modes=n_modes, **kw)
    return W.Workload(W.lvc_as_source(wl.model), wl.init, wl.run), wl


CASES = {
    "morse": lambda: W.morse_coupled(n_traj=3000, n_steps=160, cadence=10),
    "morse_ragged": lambda: W.morse_coupled(n_traj=777, n_steps=97, cadence=7),
    "lvc_n3_m4": lambda: _lvc_source(7, 3, 4, n_traj=2000, n_steps=150, cadence=15)[0],
    "lvc_n4_m6": lambda: _lvc_source(2, 4, 6, n_traj=1500, n_steps=120, cadence=20)[0],
}


@pytest.mark.parametrize("name", list(CASES))
def test_source_fp64_parity(P, name):
    wl = CASES[name]()
    model = P.Model(wl.model)
    assert model.is_source
    out_g, st_g, s0_g, _ = gpu_run(P, wl)
    out_o, st_o, s0_o, _ = oracle_run(wl)
    compare_walkers(s0_g, s0_o, rtol=1e-11, label=name + " sample")
    flip = compare_walkers(st_g, st_o, rtol=1e-10, max_flip_frac=0.005, label=name)
    check_ensemble64(out_g, out_o, wl.run.n_traj, flip, st_g, st_o, label=name)


def test_source_linear_rule(P):
    wl = CASES["lvc_n3_m4"]()
    out_g, st_g, _, _ = gpu_run(P, wl, scheme=1)
    out_o, st_o, _, _ = oracle_run(wl, scheme=1)
    flip = compare_walkers(st_g, st_o, rtol=1e-10, max_flip_frac=0.005, label="linear")
    check_ensemble64(out_g, out_o, wl.run.n_traj, flip, st_g, st_o, label="linear")


def test_source_matches_builtin_kernels(P):
    """The same linear-vibronic model through the supplied-potential kernels
    and through the built-in general kernels."""
    src, lvc = _lvc_source(2, 4, 6, n_traj=1500, n_steps=120, cadence=20)
    out_s, st_s, _, _ = gpu_run(P, src)
    out_b, st_b, _, _ = gpu_run(P, lvc)
    flip = compare_walkers(st_s, st_b, rtol=1e-10, max_flip_frac=0.005, label="source vs built-in")
    check_ensemble64(out_s, out_b, src.run.n_traj, flip, st_s, st_b, label="source vs built-in")


def test_source_split_run_bitwise(P):
    wl = CASES["morse"]()
    out1, st1, _, _ = gpu_run(P, wl)
    out2, st2, _, _ = gpu_run(P, wl, split=[37, 3, 120])
    for k in st1:
        assert np.array_equal(st1[k], st2[k]), k
    assert np.array_equal(out1, out2)


def test_source_rejects_fp32_and_batches(P):
    import ctypes as C
    wl = CASES["morse"]()
    model = P.Model(wl.model)
    with pytest.raises(P.QCLError) as e:
        ens = P.Ensemble(model, 256, "fp32")
        part = P.Partials(model, 256, 2)
        P.qcl_sample_initial(model, wl.init, 1, ens, part)
    assert e.value.status == P.QCL_ERR_UNSUPPORTED
    ens = P.Ensemble(model, 256, "fp64")
    part = P.Partials(model, 256, 3)
    P.qcl_sample_initial(model, wl.init, 1, ens, part)
    L = P.load_library()
    item = P.qcl.qcl_batch_item(model.handle, C.pointer(ens.c),
                                P.qcl.qcl_prop_desc(0.05, 10, 10, 3, 0, 1, 0, 0), part.ptr)
    items = (P.qcl.qcl_batch_item * 1)(item)
    nbytes = C.c_size_t()
    st = L.qcl_batch_workspace_bytes(items, 1, C.byref(nbytes))
    assert st == P.QCL_ERR_UNSUPPORTED
    assert b"supplied potential" in L.qcl_last_error()


def test_source_compile_error_is_reported(P):
    wl = CASES["morse"]()
    bad = W.SourceModel(name="bad", n_states_=2, mass=[1.0, 1.0], omega=[1.0, 1.0], params=[1.0],
                        hip_source="__device__ void qcl_potential(const double *q, double *V) { V[0] = q[0] +; }",
                        c_source="")
    with pytest.raises(P.QCLError) as e:
        P.Model(bad)
    assert e.value.status == P.QCL_ERR_INVALID_ARG
    assert "does not compile" in str(e.value)
    del wl
