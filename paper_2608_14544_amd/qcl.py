"""Python binding of libqcl (the C ABI in include/qcl.h).

Argument marshalling only: every step of the hot path runs in the HIP
kernels of libqcl.so.  PyTorch provides device memory and streams.  The
library must have been built (``python -m paper_2608_14544_amd.build``);
there is no fallback of any kind.
"""
from __future__ import annotations

import ctypes as C
import os
import threading
from typing import Optional

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libqcl.so")

QCL_OK = 0
QCL_ERR_INVALID_ARG = 1
QCL_ERR_UNSUPPORTED = 2
QCL_ERR_OUT_OF_MEMORY = 3
QCL_ERR_DEVICE = 4
QCL_ERR_NONFINITE = 5

QCL_FP64 = 0
QCL_FP32_ACC64 = 1
QCL_INIT_DIABATIC = 0
QCL_INIT_ADIABATIC = 1
QCL_TRANS_NORMALIZED = 0
QCL_TRANS_LINEAR = 1
QCL_TILE = 256

FLAG_NONFINITE = 1
FLAG_DEGENERATE = 2
FLAG_RESOLVED64 = 4
FLAG_FALLBACK = 8

PRECISIONS = {"fp64": QCL_FP64, "fp32": QCL_FP32_ACC64, "f64": QCL_FP64, "f32": QCL_FP32_ACC64}


class QCLError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"qcl status {status}: {msg}")
        self.status = status
        self.out = None  # QCL_ERR_NONFINITE: the averages, which are written regardless


class qcl_model_desc(C.Structure):
    _fields_ = [("n_states", C.c_int32), ("n_modes", C.c_int32),
                ("mass", C.POINTER(C.c_double)), ("omega", C.POINTER(C.c_double)),
                ("v0", C.POINTER(C.c_double)), ("k", C.POINTER(C.c_double)),
                ("hbar", C.c_double)]


class qcl_poly_desc(C.Structure):
    _fields_ = [("degree", C.c_int32), ("reserved", C.c_int32), ("a", C.POINTER(C.c_double))]


class qcl_bilinear_desc(C.Structure):
    _fields_ = [("n_pairs", C.c_int32), ("reserved", C.c_int32), ("pairs", C.POINTER(C.c_int32)),
                ("b", C.POINTER(C.c_double))]


class qcl_source_desc(C.Structure):
    _fields_ = [("source", C.c_char_p), ("params", C.POINTER(C.c_double)), ("n_params", C.c_int32),
                ("reserved", C.c_int32)]


class qcl_init_desc(C.Structure):
    _fields_ = [("kT", C.c_double), ("q0", C.POINTER(C.c_double)),
                ("state", C.c_int32), ("basis", C.c_int32)]


class qcl_ensemble(C.Structure):
    _fields_ = [("n_traj", C.c_int64), ("ld", C.c_int64), ("traj_offset", C.c_int64),
                ("step", C.c_int64), ("prec", C.c_int32), ("reserved", C.c_int32),
                ("q", C.c_void_p), ("p", C.c_void_p), ("u", C.c_void_p),
                ("w", C.c_void_p), ("phase", C.c_void_p), ("a", C.c_void_p),
                ("b", C.c_void_p), ("flags", C.c_void_p)]


class qcl_prop_desc(C.Structure):
    _fields_ = [("dt", C.c_double), ("n_steps", C.c_int32), ("cadence", C.c_int32),
                ("n_out", C.c_int32), ("scheme", C.c_int32), ("seed", C.c_uint64),
                ("occupancy", C.c_int32), ("workgroups_per_cu", C.c_int32)]


class qcl_batch_item(C.Structure):
    _fields_ = [("model", C.c_void_p), ("ens", C.POINTER(qcl_ensemble)), ("prop", qcl_prop_desc),
                ("partials", C.c_void_p)]


EXPORTS = ("qcl_create_model", "qcl_create_model_poly", "qcl_create_model_bilinear", "qcl_create_model_source",
           "qcl_model_is_source", "qcl_destroy_model",
           "qcl_model_states", "qcl_model_modes", "qcl_model_rank", "qcl_model_degree", "qcl_model_pairs",
           "qcl_ensemble_bytes", "qcl_ensemble_bind", "qcl_partials_bytes",
           "qcl_sample_initial", "qcl_propagate", "qcl_batch_workspace_bytes", "qcl_propagate_batch",
           "qcl_propagate_batch_static",
           "qcl_reduce_observables", "qcl_reduce_observables_async", "qcl_resample_workspace_bytes", "qcl_resample",
           "qcl_last_error")

_lock = threading.Lock()
_lib = None


def load_library(path: str = LIB_PATH):
    """Loads libqcl.so; raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with `python -m paper_2608_14544_amd.build`")
        L = C.CDLL(path)
        vp, i32, i64, u64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_size_t
        L.qcl_create_model.argtypes = [C.POINTER(qcl_model_desc), C.POINTER(vp)]
        L.qcl_create_model_poly.argtypes = [C.POINTER(qcl_model_desc), C.POINTER(qcl_poly_desc), C.POINTER(vp)]
        L.qcl_model_degree.argtypes = [vp]
        L.qcl_model_degree.restype = i32
        L.qcl_create_model_bilinear.argtypes = [C.POINTER(qcl_model_desc), C.POINTER(qcl_poly_desc),
                                                C.POINTER(qcl_bilinear_desc), C.POINTER(vp)]
        L.qcl_create_model_source.argtypes = [C.POINTER(qcl_model_desc), C.POINTER(qcl_source_desc), C.POINTER(vp)]
        L.qcl_model_is_source.argtypes = [vp]
        L.qcl_model_is_source.restype = i32
        L.qcl_model_pairs.argtypes = [vp]
        L.qcl_model_pairs.restype = i32
        L.qcl_destroy_model.argtypes = [vp]
        L.qcl_model_states.argtypes = [vp]
        L.qcl_model_states.restype = i32
        L.qcl_model_modes.argtypes = [vp]
        L.qcl_model_modes.restype = i32
        L.qcl_model_rank.argtypes = [vp]
        L.qcl_model_rank.restype = i32
        L.qcl_ensemble_bytes.argtypes = [vp, i64, i32, C.POINTER(i64), C.POINTER(sz)]
        L.qcl_ensemble_bind.argtypes = [vp, vp, i64, i32, i64, C.POINTER(qcl_ensemble)]
        L.qcl_partials_bytes.argtypes = [vp, i64, i32, C.POINTER(sz)]
        L.qcl_sample_initial.argtypes = [vp, C.POINTER(qcl_init_desc), u64, C.POINTER(qcl_ensemble),
                                         vp, i32, vp]
        L.qcl_propagate.argtypes = [vp, C.POINTER(qcl_ensemble), C.POINTER(qcl_prop_desc), vp, vp]
        L.qcl_batch_workspace_bytes.argtypes = [C.POINTER(qcl_batch_item), i32, C.POINTER(sz)]
        L.qcl_propagate_batch.argtypes = [C.POINTER(qcl_batch_item), i32, vp, sz, vp]
        L.qcl_propagate_batch_static.argtypes = [C.POINTER(qcl_batch_item), i32, vp]
        L.qcl_reduce_observables.argtypes = [vp, vp, i64, i32, vp, vp]
        L.qcl_reduce_observables_async.argtypes = [vp, vp, i64, i32, vp, vp, vp]
        L.qcl_resample_workspace_bytes.argtypes = [i64, C.POINTER(sz)]
        L.qcl_resample.argtypes = [vp, C.POINTER(qcl_ensemble), C.POINTER(qcl_ensemble), u64, vp, sz, vp]
        L.qcl_last_error.argtypes = []
        L.qcl_last_error.restype = C.c_char_p
        for name in EXPORTS[:-1]:
            if getattr(L, name).restype is C.c_int:
                getattr(L, name).restype = C.c_int
        _lib = L
        return _lib


def _check(status: int):
    if status != QCL_OK:
        msg = load_library().qcl_last_error()
        raise QCLError(status, msg.decode() if msg else "")


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _torch():
    import torch
    return torch


def _stream_handle(stream=None) -> Optional[int]:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


# --------------------------------------------------------------------- model

class Model:
    """Library-owned model handle built from a ``workloads.LVCModel``."""

    def __init__(self, lvc):
        L = load_library()
        self.lvc = lvc
        if getattr(lvc, "hip_source", None) is not None:
            self._init_source(L, lvc)
            return
        self._arrays = [np.ascontiguousarray(x, np.float64) for x in (lvc.mass, lvc.omega, lvc.v0, lvc.k)]
        mass, omega, v0, k = self._arrays
        desc = qcl_model_desc(int(v0.shape[0]), int(mass.shape[0]), _dptr(mass), _dptr(omega),
                              _dptr(v0), _dptr(k), float(lvc.hbar))
        h = C.c_void_p()
        poly = getattr(lvc, "poly", None)
        bil = getattr(lvc, "bilinear", None)
        pd = None
        if poly is not None:
            a = np.ascontiguousarray(poly, np.float64)
            self._arrays.append(a)
            pd = qcl_poly_desc(int(a.shape[1]) + 1, 0, _dptr(a))
        if bil:
            pairs = np.ascontiguousarray([[int(i), int(j)] for i, j, _ in bil], np.int32)
            b = np.ascontiguousarray(np.stack([np.asarray(B, np.float64) for _, _, B in bil]), np.float64)
            self._arrays += [pairs, b]
            bd = qcl_bilinear_desc(len(bil), 0, pairs.ctypes.data_as(C.POINTER(C.c_int32)), _dptr(b))
            _check(L.qcl_create_model_bilinear(C.byref(desc), C.byref(pd) if pd is not None else None,
                                               C.byref(bd), C.byref(h)))
        elif pd is not None:
            _check(L.qcl_create_model_poly(C.byref(desc), C.byref(pd), C.byref(h)))
        else:
            _check(L.qcl_create_model(C.byref(desc), C.byref(h)))
        self.handle = h
        self.n_states = int(L.qcl_model_states(h))
        self.n_modes = int(L.qcl_model_modes(h))
        self.rank = int(L.qcl_model_rank(h))
        self.degree = int(L.qcl_model_degree(h))
        self.n_pairs = int(L.qcl_model_pairs(h))

    def _init_source(self, L, sm):
        """A model with a supplied potential (``workloads.SourceModel``):
        its device source is compiled by the library for the current device."""
        mass = np.ascontiguousarray(sm.mass, np.float64)
        omega = np.ascontiguousarray(sm.omega, np.float64)
        prm = np.ascontiguousarray(sm.params, np.float64)
        self._arrays = [mass, omega, prm]
        desc = qcl_model_desc(int(sm.n_states), int(mass.shape[0]), _dptr(mass), _dptr(omega), None, None,
                              float(sm.hbar))
        self._source = sm.hip_source.encode()
        src = qcl_source_desc(self._source, _dptr(prm) if prm.size else None, int(prm.size), 0)
        h = C.c_void_p()
        _check(L.qcl_create_model_source(C.byref(desc), C.byref(src), C.byref(h)))
        self.handle = h
        self.n_states = int(L.qcl_model_states(h))
        self.n_modes = int(L.qcl_model_modes(h))
        self.rank = int(L.qcl_model_rank(h))
        self.degree = 1
        self.n_pairs = 0

    @property
    def is_source(self) -> bool:
        return bool(load_library().qcl_model_is_source(self.handle))

    def close(self):
        if getattr(self, "handle", None):
            load_library().qcl_destroy_model(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def ensemble_bytes(handle, n_traj: int, prec) -> int:
        ld = C.c_int64()
        b = C.c_size_t()
        pr = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
        _check(load_library().qcl_ensemble_bytes(handle, int(n_traj), pr, C.byref(ld), C.byref(b)))
        return int(b.value)

    def partials_bytes(self, n_traj: int, n_out: int) -> int:
        b = C.c_size_t()
        _check(load_library().qcl_partials_bytes(self.handle, int(n_traj), int(n_out), C.byref(b)))
        return int(b.value)


# ------------------------------------------------------------------ ensemble

class Ensemble:
    """Device-resident walker ensemble in one torch allocation."""

    def __init__(self, model: Model, n_traj: int, prec="fp64", traj_offset: int = 0, device="cuda",
                 zero: bool = True):
        torch = _torch()
        L = load_library()
        self.model = model
        self.prec = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
        ld = C.c_int64()
        nbytes = C.c_size_t()
        _check(L.qcl_ensemble_bytes(model.handle, int(n_traj), self.prec, C.byref(ld), C.byref(nbytes)))
        # qcl_sample_initial writes every array entry a kernel reads, so an
        # ensemble that is sampled next need not be cleared
        alloc = torch.zeros if zero else torch.empty
        self.buffer = alloc(int(nbytes.value), dtype=torch.uint8, device=device)
        self.c = qcl_ensemble()
        _check(L.qcl_ensemble_bind(model.handle, C.c_void_p(self.buffer.data_ptr()), int(n_traj), self.prec,
                                   int(traj_offset), C.byref(self.c)))
        self.n_traj = int(n_traj)
        self.ld = int(ld.value)

    @property
    def step(self) -> int:
        return int(self.c.step)

    def _view(self, ptr, dtype, shape):
        torch = _torch()
        base = self.buffer.data_ptr()
        off = int(ptr) - base
        itemsize = torch.tensor([], dtype=dtype).element_size()
        n = int(np.prod(shape))
        return self.buffer[off:off + n * itemsize].view(dtype).view(*shape)

    def tensors(self):
        """Torch views of the arrays: q, p [M, ld], u [N*N, ld], w, phase, a, b, flags [ld]."""
        torch = _torch()
        rt = torch.float64 if self.prec == QCL_FP64 else torch.float32
        M, N, ld = self.model.n_modes, self.model.n_states, self.ld
        c = self.c
        return {
            "q": self._view(c.q, rt, (M, ld)), "p": self._view(c.p, rt, (M, ld)),
            "u": self._view(c.u, rt, (N * N, ld)),
            "w": self._view(c.w, torch.float64, (ld,)), "phase": self._view(c.phase, torch.float64, (ld,)),
            "a": self._view(c.a, torch.uint8, (ld,)), "b": self._view(c.b, torch.uint8, (ld,)),
            "flags": self._view(c.flags, torch.int32, (ld,)),
        }

    def to_numpy(self):
        """Per-walker arrays in walker-major layout: q, p [T, M], U [T, N, N]."""
        T, N = self.n_traj, self.model.n_states
        t = {k: v.cpu().numpy() for k, v in self.tensors().items()}
        return {
            "q": t["q"][:, :T].T.astype(np.float64), "p": t["p"][:, :T].T.astype(np.float64),
            "U": t["u"][:, :T].T.reshape(T, N, N).astype(np.float64),
            "w": t["w"][:T].copy(), "phase": t["phase"][:T].copy(),
            "a": t["a"][:T].astype(np.int32), "b": t["b"][:T].astype(np.int32),
            "flags": t["flags"][:T].view(np.uint32).copy(),
        }

    def load_numpy(self, state):
        """Writes walker-major arrays (oracle layout) into the device ensemble."""
        torch = _torch()
        T, N = self.n_traj, self.model.n_states
        t = self.tensors()
        dev = self.buffer.device
        rt = t["q"].dtype
        t["q"][:, :T] = torch.as_tensor(np.ascontiguousarray(state["q"].T), device=dev).to(rt)
        t["p"][:, :T] = torch.as_tensor(np.ascontiguousarray(state["p"].T), device=dev).to(rt)
        t["u"][:, :T] = torch.as_tensor(np.ascontiguousarray(state["U"].reshape(T, N * N).T), device=dev).to(rt)
        t["w"][:T] = torch.as_tensor(state["w"], device=dev)
        t["phase"][:T] = torch.as_tensor(state["phase"], device=dev)
        t["a"][:T] = torch.as_tensor(state["a"].astype(np.uint8), device=dev)
        t["b"][:T] = torch.as_tensor(state["b"].astype(np.uint8), device=dev)
        t["flags"][:T] = 0
        self.c.step = int(state.get("step", 0))


class Partials:
    """Tile partial sums of one ensemble (qcl_partials_bytes of them)."""

    def __init__(self, model: Model, n_traj: int, n_out: int, device="cuda"):
        torch = _torch()
        nb = model.partials_bytes(n_traj, n_out)
        self.tensor = torch.zeros(max(nb // 8, 1), dtype=torch.float64, device=device)
        self.n_out = int(n_out)
        self.n_traj = int(n_traj)
        self.n_states = int(model.n_states)

    @property
    def ptr(self):
        return C.c_void_p(self.tensor.data_ptr())


# ------------------------------------------------------------- entry points

def _match(model: Model, ens: Optional[Ensemble] = None, partials: Optional[Partials] = None):
    """Raises before any launch when the buffers were not made for this
    model and for each other: the C ABI takes raw pointers, so a
    mismatch would write past the end of a device buffer."""
    if ens is not None:
        if ens.model is not model and ens.model.handle.value != model.handle.value:
            raise ValueError("the ensemble was made for another model")
        if partials is not None and partials.n_traj != ens.n_traj:
            raise ValueError(f"partials hold {partials.n_traj} walkers, the ensemble {ens.n_traj}")
    if partials is not None and partials.n_states != model.n_states:
        raise ValueError(f"partials hold {partials.n_states} states, the model {model.n_states}")


def qcl_sample_initial(model: Model, init, seed: int, ens: Ensemble, partials: Partials, stream=None):
    _match(model, ens, partials)
    q0 = np.ascontiguousarray(init.q0, np.float64)
    d = qcl_init_desc(float(init.kT), _dptr(q0), int(init.state), int(init.basis))
    _check(load_library().qcl_sample_initial(model.handle, C.byref(d), C.c_uint64(int(seed)), C.byref(ens.c),
                                             partials.ptr, partials.n_out, C.c_void_p(_stream_handle(stream))))


def qcl_propagate(model: Model, ens: Ensemble, dt: float, n_steps: int, cadence: int, seed: int,
                  partials: Partials, scheme: int = QCL_TRANS_NORMALIZED, stream=None, occupancy: int = 0):
    _match(model, ens, partials)
    pd = qcl_prop_desc(float(dt), int(n_steps), int(cadence), partials.n_out, int(scheme), int(seed),
                       int(occupancy), 0)
    _check(load_library().qcl_propagate(model.handle, C.byref(ens.c), C.byref(pd), partials.ptr,
                                        C.c_void_p(_stream_handle(stream))))


class BatchJob:
    """Arguments of one qcl_propagate call, as an item of a batch."""

    def __init__(self, model: Model, ens: Ensemble, partials: Partials, dt: float, n_steps: int,
                 cadence: int, seed: int, scheme: int = QCL_TRANS_NORMALIZED, occupancy: int = 0,
                 workgroups_per_cu: int = 0):
        self.model, self.ens, self.partials = model, ens, partials
        self.dt, self.n_steps, self.cadence = float(dt), int(n_steps), int(cadence)
        self.seed, self.scheme, self.occupancy = int(seed), int(scheme), int(occupancy)
        self.workgroups_per_cu = int(workgroups_per_cu)

    def item(self) -> qcl_batch_item:
        _match(self.model, self.ens, self.partials)
        pd = qcl_prop_desc(self.dt, self.n_steps, self.cadence, self.partials.n_out, self.scheme,
                           self.seed, self.occupancy, self.workgroups_per_cu)
        return qcl_batch_item(self.model.handle, C.pointer(self.ens.c), pd, self.partials.ptr)


class Workspace:
    """Device workspace for qcl_propagate_batch, grown on demand."""

    def __init__(self, device="cuda"):
        self.device = device
        self.tensor = None

    def get(self, nbytes: int):
        torch = _torch()
        if nbytes == 0:
            return None, 0
        if self.tensor is None or self.tensor.numel() < nbytes:
            # torch's caching allocator returns 512-byte aligned blocks
            self.tensor = torch.empty(max(nbytes, 1 << 16), dtype=torch.uint8, device=self.device)
        return C.c_void_p(self.tensor.data_ptr()), self.tensor.numel()


def qcl_batch_workspace_bytes(jobs) -> int:
    arr = (qcl_batch_item * len(jobs))(*[j.item() for j in jobs])
    nb = C.c_size_t(0)
    _check(load_library().qcl_batch_workspace_bytes(arr, len(jobs), C.byref(nb)))
    return nb.value


def qcl_propagate_batch(jobs, workspace: Optional[Workspace] = None, stream=None):
    """Advances every job by its n_steps in per-class persistent launches;
    each job's result is bitwise its solo qcl_propagate result."""
    L = load_library()
    arr = (qcl_batch_item * len(jobs))(*[j.item() for j in jobs])
    nb = C.c_size_t(0)
    _check(L.qcl_batch_workspace_bytes(arr, len(jobs), C.byref(nb)))
    ws = workspace or Workspace()
    ptr, have = ws.get(nb.value)
    _check(L.qcl_propagate_batch(arr, len(jobs), ptr, have, C.c_void_p(_stream_handle(stream))))
    return ws


def _reduce_args(model: Model, partials: Partials, n_traj: int, out):
    torch = _torch()
    _match(model, None, partials)
    if int(n_traj) != partials.n_traj:
        # the reduction's scratch rows sit after the tile rows of
        # partials.n_traj walkers; another count would place them over live rows
        raise ValueError(f"n_traj {n_traj} differs from the {partials.n_traj} walkers of the partials")
    N = model.n_states
    shape = (partials.n_out, 2, N, N, 4)
    if out is None:
        out = torch.empty(shape, dtype=torch.float64, device=partials.tensor.device)
    elif tuple(out.shape) != shape or out.dtype != torch.float64 or not out.is_contiguous() \
            or out.device != partials.tensor.device:
        raise ValueError(f"out must be a contiguous float64 tensor of shape {shape} on {partials.tensor.device}")
    return out


def qcl_propagate_batch_static(jobs, stream=None):
    """qcl_propagate_batch with the library's own per-device workspace (no
    device allocation by the library or here)."""
    arr = (qcl_batch_item * len(jobs))(*[j.item() for j in jobs])
    _check(load_library().qcl_propagate_batch_static(arr, len(jobs), C.c_void_p(_stream_handle(stream))))


def qcl_reduce_observables(model: Model, partials: Partials, n_traj: int, out=None, stream=None):
    """Returns a device tensor [n_out, 2, N, N, 4]: mean Re, mean Im, SE Re, SE Im.
    Waits for the reduction; raises QCLError (status QCL_ERR_NONFINITE, the
    result in its ``out``) when walkers with a non-finite weight or phase
    were left out of a bin."""
    out = _reduce_args(model, partials, n_traj, out)
    st = load_library().qcl_reduce_observables(model.handle, partials.ptr, int(n_traj), partials.n_out,
                                               C.c_void_p(out.data_ptr()), C.c_void_p(_stream_handle(stream)))
    if st == QCL_ERR_NONFINITE:
        err = QCLError(st, load_library().qcl_last_error().decode())
        err.out = out
        raise err
    _check(st)
    return out


def qcl_reduce_observables_async(model: Model, partials: Partials, n_traj: int, out=None, excluded=None,
                                 stream=None):
    """Enqueues the reduction without waiting; returns (out, excluded) device
    tensors, excluded [n_out] int64 holding the walkers left out of each bin."""
    torch = _torch()
    out = _reduce_args(model, partials, n_traj, out)
    if excluded is None:
        excluded = torch.empty(partials.n_out, dtype=torch.int64, device=out.device)
    elif tuple(excluded.shape) != (partials.n_out,) or excluded.dtype != torch.int64 or \
            not excluded.is_contiguous() or excluded.device != out.device:
        raise ValueError(f"excluded must be a contiguous int64 tensor of shape ({partials.n_out},) on {out.device}")
    _check(load_library().qcl_reduce_observables_async(model.handle, partials.ptr, int(n_traj), partials.n_out,
                                                       C.c_void_p(out.data_ptr()), C.c_void_p(excluded.data_ptr()),
                                                       C.c_void_p(_stream_handle(stream))))
    return out, excluded


def qcl_resample_workspace_bytes(n_traj: int) -> int:
    nb = C.c_size_t(0)
    _check(load_library().qcl_resample_workspace_bytes(int(n_traj), C.byref(nb)))
    return nb.value


def qcl_resample(model: Model, src: Ensemble, dst: Ensemble, seed: int, workspace: Optional[Workspace] = None,
                 stream=None):
    """Fixed-budget systematic resampling of src into dst (same size, precision
    and traj_offset); dst continues at src's step.  Returns the workspace."""
    L = load_library()
    _match(model, src)
    _match(model, dst)
    nb = C.c_size_t(0)
    _check(L.qcl_resample_workspace_bytes(src.n_traj, C.byref(nb)))
    ws = workspace or Workspace(device=src.buffer.device)
    ptr, have = ws.get(nb.value)
    _check(L.qcl_resample(model.handle, C.byref(src.c), C.byref(dst.c), int(seed) & 0xFFFFFFFFFFFFFFFF, ptr, have,
                          C.c_void_p(_stream_handle(stream))))
    return ws


def run(workload, prec="fp64", n_traj: Optional[int] = None, n_steps: Optional[int] = None,
        scheme: int = QCL_TRANS_NORMALIZED, traj_offset: int = 0, model: Optional[Model] = None):
    """Sample, propagate and reduce one workload; returns (out numpy, Ensemble)."""
    torch = _torch()
    r = workload.run
    T = r.n_traj if n_traj is None else int(n_traj)
    S = r.n_steps if n_steps is None else int(n_steps)
    n_out = S // r.cadence + 1
    model = model or Model(workload.model)
    ens = Ensemble(model, T, prec, traj_offset)
    part = Partials(model, T, n_out)
    qcl_sample_initial(model, workload.init, r.seed, ens, part)
    qcl_propagate(model, ens, r.dt, S, r.cadence, r.seed, part, scheme)
    out = qcl_reduce_observables(model, part, T)
    torch.cuda.synchronize()
    return out.cpu().numpy(), ens
