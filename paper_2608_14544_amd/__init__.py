"""MI355X (gfx950) propagator for the momentum-jump-free quantum-classical
Liouville trajectory ensemble: C-ABI library ``libqcl.so`` (include/qcl.h)
with a thin ctypes binding (:mod:`paper_2608_14544_amd.qcl`)."""
from . import qcl  # noqa: F401
from .qcl import (  # noqa: F401
    BatchJob, Ensemble, Model, Partials, QCLError, Workspace, load_library, qcl_batch_workspace_bytes,
    qcl_propagate, qcl_propagate_batch, qcl_propagate_batch_static, qcl_reduce_observables, qcl_reduce_observables_async, qcl_resample,
    qcl_resample_workspace_bytes, qcl_sample_initial, run, QCL_ERR_DEVICE, QCL_ERR_INVALID_ARG, QCL_ERR_NONFINITE,
    QCL_ERR_UNSUPPORTED, QCL_FP64, QCL_FP32_ACC64,
    QCL_TRANS_LINEAR, QCL_TRANS_NORMALIZED,
)
