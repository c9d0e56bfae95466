"""ctypes front end of the plain FP64 C oracle (``qcl_oracle.c``).

Test infrastructure only: see the package docstring.  State arrays here are
per walker (array-of-structures): q, p ``[T, M]``, U ``[T, N, N]``.
Observable arrays follow ``[n_out, 2, N, N, 4]`` with basis 0 = adiabatic,
1 = diabatic and the last axis (Re, Im, Re^2, Im^2) for sums or
(mean Re, mean Im, SE Re, SE Im) after :func:`finalize`.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qcl_oracle.c")
_LIB = os.path.join(_HERE, "_qcl_oracle.so")
_lock = threading.Lock()
_lib = None

NORMALIZED = 0
LINEAR = 1
FLAG_NONFINITE = 1
FLAG_DEGENERATE = 2
FLAG_FALLBACK = 8


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: IEEE binary64, no fast-math, no FMA
    contraction, OpenMP over walkers."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fno-fast-math", "-ffp-contract=off",
               "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Model(C.Structure):
    _fields_ = [("n_states", C.c_int32), ("n_modes", C.c_int32),
                ("mass", C.POINTER(C.c_double)), ("omega", C.POINTER(C.c_double)),
                ("v0", C.POINTER(C.c_double)), ("k", C.POINTER(C.c_double)),
                ("hbar", C.c_double), ("degree", C.c_int32), ("a", C.POINTER(C.c_double)),
                ("n_pairs", C.c_int32), ("pairs", C.POINTER(C.c_int32)), ("bpair", C.POINTER(C.c_double)),
                ("user_v", C.c_void_p), ("user_dv", C.c_void_p), ("user_prm", C.POINTER(C.c_double))]


_USER_DIR = os.path.join(_HERE, "_user")


def user_library(c_source: str) -> C.CDLL:
    """Compiles the C transcription of a supplied potential (functions
    ``qcl_oracle_potential(q, prm, V)``, V the full N x N matrix, and
    ``qcl_oracle_gradient(j, q, prm, G)``, G = dV/dq_j) with the oracle's
    floating-point options, cached by the source's hash."""
    import hashlib
    h = hashlib.sha256(c_source.encode()).hexdigest()[:16]
    os.makedirs(_USER_DIR, exist_ok=True)
    so = os.path.join(_USER_DIR, f"potential_{h}.so")
    if not os.path.exists(so):
        src = os.path.join(_USER_DIR, f"potential_{h}.c")
        with open(src, "w") as f:
            f.write("#include <math.h>\n" + c_source)
        tmp = so + f".{os.getpid()}.tmp"
        subprocess.run(["gcc", "-O2", "-std=c99", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared",
                        src, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, so)
    return C.CDLL(so)


_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_up = C.POINTER(C.c_uint32)


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)  # missing, or older than its source
            L = C.CDLL(_LIB)
            L.or_philox4x32_10.argtypes = [_up, _up, _up]
            L.or_uniform24.argtypes = [C.c_uint32]
            L.or_uniform24.restype = C.c_double
            L.or_uniform52.argtypes = [C.c_uint32, C.c_uint32]
            L.or_uniform52.restype = C.c_double
            L.or_jacobi_eigh.argtypes = [C.c_int, _dp, _dp, _dp]
            L.or_gauge.argtypes = [C.c_int, _dp, _dp]
            L.or_adiabatic.argtypes = [C.POINTER(_Model), _dp, _dp, _dp, _dp]
            L.or_mean_force.argtypes = [C.POINTER(_Model), _dp, _dp, C.c_int, C.c_int, _dp]
            L.or_velocity_nac.argtypes = [C.POINTER(_Model), _dp, _dp, _dp, _dp, _dp]
            L.or_candidates.argtypes = [C.c_int, _dp, C.c_double, C.c_int, C.c_int, _dp, _ip, _ip]
            L.or_candidates.restype = C.c_int
            L.or_transition.argtypes = [C.c_int, _dp, C.c_double, C.c_double, C.c_int,
                                        _ip, _ip, _dp, C.POINTER(C.c_int)]
            L.or_transition.restype = C.c_int
            L.or_sample.argtypes = [C.POINTER(_Model), C.c_double, _dp, C.c_int, C.c_int,
                                    C.c_uint64, C.c_int64, C.c_int64,
                                    _dp, _dp, _dp, _dp, _ip, _ip, _dp, _dp]
            L.or_propagate.argtypes = [C.POINTER(_Model), C.c_int64, C.c_int64, C.c_int64,
                                       C.c_int, C.c_double, C.c_int, C.c_uint64, C.c_int,
                                       _dp, _dp, _dp, _dp, _ip, _ip, _dp,
                                       C.c_int32, _dp, _up, C.POINTER(C.c_int64)]
            L.or_propagate.restype = C.c_int
            L.or_finalize.argtypes = [C.c_int, C.c_int64, C.c_int32, _dp, _dp]
            L.or_num_threads.argtypes = []
            L.or_num_threads.restype = C.c_int
            _lib = L
    return _lib


def _d(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _i(a: np.ndarray):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(_ip)


class Model:
    """Keeps the numpy buffers of a ``workloads.LVCModel`` (or
    ``workloads.SourceModel``) alive for C."""

    def __init__(self, m):
        self.src = m
        self.mass = np.ascontiguousarray(m.mass, np.float64)
        self.omega = np.ascontiguousarray(m.omega, np.float64)
        self.v0 = np.ascontiguousarray(m.v0, np.float64)
        self.k = np.ascontiguousarray(m.k, np.float64)
        self.n = int(self.v0.shape[0])
        self.M = int(self.mass.shape[0])
        poly = getattr(m, "poly", None)
        self.degree = 1 if poly is None else int(poly.shape[1]) + 1
        self.a = None if poly is None else np.ascontiguousarray(poly, np.float64)
        bil = getattr(m, "bilinear", None) or []
        self.n_pairs = len(bil)
        self.pairs = np.ascontiguousarray([[int(i), int(j)] for i, j, _ in bil] or np.zeros((0, 2)), np.int32)
        self.bpair = np.ascontiguousarray([np.asarray(B, np.float64) for _, _, B in bil]
                                          or np.zeros((0, self.n, self.n)), np.float64)
        # a supplied potential: the model's C transcription, compiled here
        c_src = getattr(m, "c_source", None)
        self.user = user_library(c_src) if c_src else None
        self.params = np.ascontiguousarray(np.append(np.asarray(getattr(m, "params", ()), np.float64), 0.0))
        user_v = user_dv = prm = None
        if self.user is not None:
            user_v = C.cast(self.user.qcl_oracle_potential, C.c_void_p)
            user_dv = C.cast(self.user.qcl_oracle_gradient, C.c_void_p)
            prm = _d(self.params)
        self.c = _Model(self.n, self.M, _d(self.mass), _d(self.omega), _d(self.v0), _d(self.k),
                        float(m.hbar), self.degree, _d(self.a) if self.a is not None else None,
                        self.n_pairs, _i(self.pairs) if self.n_pairs else None,
                        _d(self.bpair) if self.n_pairs else None, user_v, user_dv, prm)

    @property
    def ref(self):
        return C.byref(self.c)


def _model(m) -> Model:
    return m if isinstance(m, Model) else Model(m)


# ---------------------------------------------------------------- primitives

def philox(counter, key) -> np.ndarray:
    c = np.ascontiguousarray(counter, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    o = np.zeros(4, np.uint32)
    lib().or_philox4x32_10(c.ctypes.data_as(_up), k.ctypes.data_as(_up), o.ctypes.data_as(_up))
    return o


def uniform24(x: int) -> float:
    return lib().or_uniform24(int(x))


def uniform52(hi: int, lo: int) -> float:
    return lib().or_uniform52(int(hi), int(lo))


def jacobi_eigh(A: np.ndarray):
    A = np.ascontiguousarray(A, np.float64)
    n = A.shape[0]
    E = np.zeros(n)
    U = np.zeros((n, n))
    lib().or_jacobi_eigh(n, _d(A), _d(E), _d(U))
    return E, U


def adiabatic(m, q, Uprev: Optional[np.ndarray] = None):
    mm = _model(m)
    q = np.ascontiguousarray(q, np.float64)
    E = np.zeros(mm.n)
    U = np.zeros((mm.n, mm.n))
    up = _d(np.ascontiguousarray(Uprev, np.float64)) if Uprev is not None else None
    lib().or_adiabatic(mm.ref, _d(q), up, _d(E), _d(U))
    return E, U


def mean_force(m, q, U, a, b):
    mm = _model(m)
    F = np.zeros(mm.M)
    lib().or_mean_force(mm.ref, _d(np.ascontiguousarray(q, np.float64)),
                        _d(np.ascontiguousarray(U, np.float64)), int(a), int(b), _d(F))
    return F


def velocity_nac(m, p, E, U, q=None):
    """v.d for all pairs; q is needed when the model has powers above 1 or
    cross-mode bilinear terms."""
    mm = _model(m)
    vd = np.zeros((mm.n, mm.n))
    if q is None and (mm.degree > 1 or mm.n_pairs):
        raise ValueError("velocity_nac of a model with higher powers or bilinear terms needs q")
    qp = _d(np.ascontiguousarray(q, np.float64)) if q is not None else None
    lib().or_velocity_nac(mm.ref, qp, _d(np.ascontiguousarray(p, np.float64)),
                          _d(np.ascontiguousarray(E, np.float64)),
                          _d(np.ascontiguousarray(U, np.float64)), _d(vd))
    return vd


def candidates(vd, dt, a, b):
    vd = np.ascontiguousarray(vd, np.float64)
    n = vd.shape[0]
    f = np.zeros(2 * n)
    ta = np.zeros(2 * n, np.int32)
    tb = np.zeros(2 * n, np.int32)
    nc = lib().or_candidates(n, _d(vd), float(dt), int(a), int(b), _d(f), _i(ta), _i(tb))
    return f[:nc], ta[:nc], tb[:nc]


def transition(vd, dt, u, scheme, a, b, w):
    vd = np.ascontiguousarray(vd, np.float64)
    aa = C.c_int32(a)
    bb = C.c_int32(b)
    ww = C.c_double(w)
    fb = C.c_int(0)
    k = lib().or_transition(vd.shape[0], _d(vd), float(dt), float(u), int(scheme),
                            C.byref(aa), C.byref(bb), C.byref(ww), C.byref(fb))
    return k, aa.value, bb.value, ww.value, fb.value


# ---------------------------------------------------------------- ensemble

class State:
    """Per-walker oracle state (AoS)."""

    def __init__(self, n_traj: int, n_states: int, n_modes: int):
        T = int(n_traj)
        self.q = np.zeros((T, n_modes))
        self.p = np.zeros((T, n_modes))
        self.w = np.zeros(T)
        self.phase = np.zeros(T)
        self.a = np.zeros(T, np.int32)
        self.b = np.zeros(T, np.int32)
        self.U = np.zeros((T, n_states, n_states))
        self.flags = np.zeros(T, np.uint32)
        self.step = 0
        self.traj_offset = 0

    @property
    def n_traj(self) -> int:
        return int(self.w.shape[0])

    def copy(self) -> "State":
        s = State.__new__(State)
        for k, v in self.__dict__.items():
            setattr(s, k, v.copy() if isinstance(v, np.ndarray) else v)
        return s

    def subset(self, idx) -> "State":
        s = State.__new__(State)
        for k, v in self.__dict__.items():
            setattr(s, k, np.ascontiguousarray(v[idx]) if isinstance(v, np.ndarray) else v)
        return s


def sample(m, init, seed: int, n_traj: int, traj_offset: int = 0):
    """Wigner sampling of (q, p) and of the initial element; returns
    (state, sums0) with sums0 the t = 0 bin [2, N, N, 4]."""
    mm = _model(m)
    st = State(n_traj, mm.n, mm.M)
    st.traj_offset = int(traj_offset)
    sums0 = np.zeros((2, mm.n, mm.n, 4))
    q0 = np.ascontiguousarray(init.q0, np.float64)
    lib().or_sample(mm.ref, float(init.kT), _d(q0), int(init.state), int(init.basis),
                    C.c_uint64(int(seed)), int(traj_offset), int(n_traj),
                    _d(st.q), _d(st.p), _d(st.w), _d(st.phase), _i(st.a), _i(st.b), _d(st.U),
                    _d(sums0))
    return st, sums0


def propagate(m, st: State, dt: float, n_steps: int, cadence: int, seed: int, n_out: int,
              sums: Optional[np.ndarray] = None, scheme: int = NORMALIZED):
    """Advance every walker n_steps steps (in place) from st.step; bin
    contributions at global steps that are multiples of ``cadence`` are
    accumulated into ``sums`` [n_out, 2, N, N, 4].  Returns (sums, n_fallback)."""
    mm = _model(m)
    if sums is None:
        sums = np.zeros((n_out, 2, mm.n, mm.n, 4))
    nfb = C.c_int64(0)
    rc = lib().or_propagate(mm.ref, st.n_traj, st.traj_offset, st.step, int(n_steps), float(dt),
                            int(cadence), C.c_uint64(int(seed)), int(scheme),
                            _d(st.q), _d(st.p), _d(st.w), _d(st.phase), _i(st.a), _i(st.b),
                            _d(st.U), int(n_out), _d(sums),
                            st.flags.ctypes.data_as(_up), C.byref(nfb))
    if rc != 0:
        raise ValueError("oracle propagate: invalid arguments")
    st.step += int(n_steps)
    return sums, int(nfb.value)


def num_threads() -> int:
    return int(lib().or_num_threads())


def finalize(sums: np.ndarray, n_traj: int) -> np.ndarray:
    sums = np.ascontiguousarray(sums, np.float64)
    n = sums.shape[-2]
    n_out = sums.shape[0]
    out = np.zeros_like(sums)
    lib().or_finalize(n, int(n_traj), n_out, _d(sums), _d(out))
    return out


def run(workload, n_traj: Optional[int] = None, n_steps: Optional[int] = None,
        scheme: int = NORMALIZED, traj_offset: int = 0):
    """Sample, propagate and average one workload; returns (out, state, sums)."""
    m, init, r = workload.model, workload.init, workload.run
    T = r.n_traj if n_traj is None else int(n_traj)
    S = r.n_steps if n_steps is None else int(n_steps)
    n_out = S // r.cadence + 1
    mm = Model(m)
    st, s0 = sample(mm, init, r.seed, T, traj_offset)
    sums = np.zeros((n_out, 2, mm.n, mm.n, 4))
    sums[0] = s0
    propagate(mm, st, r.dt, S, r.cadence, r.seed, n_out, sums, scheme)
    return finalize(sums, T), st, sums
