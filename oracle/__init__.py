"""FP64 CPU oracle of the QCL trajectory ensemble -- test infrastructure.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It never imports the HIP package and shares no code
with it; both sides read model numbers from :mod:`workloads`.

``oracle.core``      ctypes wrapper of ``qcl_oracle.c`` (the propagator).
``oracle.branches``  exact all-branches expectation for tiny cases.
``oracle.grid``      phase-space grid solution of Eq. 1 (one mode, two states).
``oracle.decay``     horizons and decay rate of the excited population.
``oracle.resample``  fixed-budget systematic resampling of an ensemble.
"""
