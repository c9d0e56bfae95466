"""Continuous-batching job server for QCL ensembles on one GPU.

Jobs (a model, an initial state, a walker count, a step count, a
precision) arrive over time.  The server keeps every admitted ensemble
resident in device memory and advances all of them together in quanta,
one ``qcl_propagate_batch`` call per quantum (Sec. II.B: walkers are independent, so ensembles of different
models and sizes can share a launch).  Between quanta it

  * admits queued jobs while their device footprint (walker arrays,
    partial sums, result buffer) fits the memory budget and a slot is free
    (first come first served; a job that does not fit lets smaller ones
    behind it start, until it has waited ``max_backfill_wait`` seconds);
  * retires jobs whose last step has been enqueued: their observables are
    reduced on the device and copied to host memory asynchronously; their
    device buffers, and their share of the memory budget, are given back
    once that copy has completed.

A quantum is either a fixed step count per job (``quantum_steps``) or a
fixed amount of work per job (``quantum_work`` walker-steps, i.e.
quantum_work / n_traj steps, at least ``min_steps`` and at most
``quantum_steps``): the second shares the device roughly equally between
resident jobs, so a small job is not held back by rounds sized for large
ones.  The floor is there because every round loads and stores each
resident walker's whole state once (the kernels keep it in registers for
the length of a call): that round trip costs as much as a few to about 17
steps of the step arithmetic (per mode, 16 bytes in and out at HBM speed
against about 10 instructions per step; the electronic part adds more
arithmetic than state for N > 2), so a job of many walkers advanced one
or two steps per round would spend most of its device time moving its
state.

Because a batched launch and any split of the steps into calls leave each
ensemble's arithmetic unchanged, a job's result is bitwise the one it gets
when run alone.

The device work sits behind a small backend interface so that the
scheduling logic can be exercised without a GPU (see ``SimBackend``).
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Deque, Dict, List, Optional

import numpy as np


@dataclasses.dataclass
class JobSpec:
    """One simulation request: ``workload`` is a ``workloads.Workload``."""
    workload: object
    prec: str = "fp32"
    scheme: int = 0
    name: str = ""

    @property
    def n_traj(self) -> int:
        return int(self.workload.run.n_traj)

    @property
    def n_steps(self) -> int:
        return int(self.workload.run.n_steps)

    @property
    def walker_steps(self) -> int:
        return self.n_traj * self.n_steps


@dataclasses.dataclass
class JobResult:
    job_id: int
    name: str
    out: Optional[np.ndarray]     # [n_out, 2, N, N, 4] (mean Re, mean Im, SE Re, SE Im)
    arrival: float                # seconds on the server clock
    admitted: float
    finished: float
    walker_steps: int
    error: str = ""
    excluded: int = 0             # walkers left out of a bin (non-finite weight or phase), largest over bins

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclasses.dataclass
class _Job:
    job_id: int
    spec: JobSpec
    arrival: float
    footprint: int
    admitted: float = -1.0
    done_steps: int = 0
    handle: object = None
    pending: object = None        # backend result future once retired


class DeviceBackend:
    """Device work through the C ABI (one stream, default priority)."""

    def __init__(self, stream=None, tuning=None):
        import torch
        from . import qcl as Q
        self.Q = Q
        self.torch = torch
        self.tuning = tuning  # tune.TuningTable: register budget and workgroups per CU per class
        Q.load_library()
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        # descriptors are uploaded by a kernel on the same stream, so one
        # workspace serves every round
        self.ws = Q.Workspace()
        self._models: Dict[tuple, object] = {}
        self.host_s = 0.0  # host time spent enqueueing rounds

    @staticmethod
    def _model_key(lvc):
        """Everything that defines a model's device tables (or, for a
        supplied potential, its compiled program)."""
        key = [lvc.name, lvc.hbar, np.asarray(lvc.mass).tobytes(), np.asarray(lvc.omega).tobytes(),
               np.asarray(lvc.v0).tobytes(), np.asarray(lvc.k).tobytes()]
        poly = getattr(lvc, "poly", None)
        key.append(None if poly is None else np.asarray(poly).tobytes())
        bil = getattr(lvc, "bilinear", None)
        key.append(None if bil is None else tuple((i, j, np.asarray(B).tobytes()) for i, j, B in bil))
        src = getattr(lvc, "hip_source", None)
        key.append(src)
        params = getattr(lvc, "params", None)
        key.append(None if params is None else np.asarray(params, dtype=np.float64).tobytes())
        return tuple(key)

    def _model(self, lvc):
        key = self._model_key(lvc)
        m = self._models.get(key)
        if m is None:
            m = self.Q.Model(lvc)
            self._models[key] = m
        return m

    def footprint(self, spec: JobSpec) -> int:
        m = self._model(spec.workload.model)
        r = spec.workload.run
        n_out = r.n_steps // r.cadence + 1
        N = m.n_states
        return (self.Q.Model.ensemble_bytes(m.handle, r.n_traj, spec.prec)
                + m.partials_bytes(r.n_traj, n_out) + n_out * 2 * N * N * 4 * 8)

    def start(self, spec: JobSpec):
        Q = self.Q
        wl = spec.workload
        r = wl.run
        m = self._model(wl.model)
        with self.torch.cuda.stream(self.stream):
            ens = Q.Ensemble(m, r.n_traj, spec.prec, zero=False)
            part = Q.Partials(m, r.n_traj, r.n_steps // r.cadence + 1)
            Q.qcl_sample_initial(m, wl.init, r.seed, ens, part, stream=self.stream)
        return (m, ens, part)

    def advance(self, work):
        """work: list of (handle, spec, n_steps); one batched launch.  The
        host time spent enqueueing it is added to ``host_s``."""
        Q = self.Q
        t0 = time.perf_counter()
        tn = self.tuning
        jobs = [Q.BatchJob(h[0], h[1], h[2], s.workload.run.dt, n, s.workload.run.cadence,
                           s.workload.run.seed, s.scheme,
                           occupancy=tn.occupancy(h[0], s.prec) if tn is not None else 0,
                           workgroups_per_cu=tn.workgroups_per_cu(h[0], s.prec) if tn is not None else 0)
                for h, s, n in work]
        with self.torch.cuda.stream(self.stream):
            Q.qcl_propagate_batch(jobs, self.ws, stream=self.stream)
        self.host_s += time.perf_counter() - t0

    def finish(self, handle, spec: JobSpec):
        """Enqueues the reduction and the copy to host; returns a future."""
        torch = self.torch
        m, ens, part = handle
        with torch.cuda.stream(self.stream):
            out, excl = self.Q.qcl_reduce_observables_async(m, part, spec.n_traj, stream=self.stream)
            host = torch.empty(out.shape, dtype=out.dtype, pin_memory=True)
            host.copy_(out, non_blocking=True)
            host_excl = torch.empty(excl.shape, dtype=excl.dtype, pin_memory=True)
            host_excl.copy_(excl, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self.stream)
        return _DeviceFuture(ev, host, (out, excl, part, ens), host_excl)

    def release(self, handle):
        pass  # tensors go back to the stream-ordered caching allocator with the handle

    def barrier(self):
        ev = self.torch.cuda.Event()
        ev.record(self.stream)
        return ev

    def wait(self, token):
        token.synchronize()


class _DeviceFuture:
    def __init__(self, ev, host, keep, host_excluded=None):
        self.ev, self.host, self.keep, self.host_excluded = ev, host, keep, host_excluded

    def ready(self) -> bool:
        if self.ev.query():
            self.keep = None
            return True
        return False

    def result(self) -> np.ndarray:
        self.ev.synchronize()
        self.keep = None
        return self.host.numpy().copy()

    def excluded(self) -> int:
        """Largest number of walkers a bin left out (non-finite weight or phase)."""
        self.ev.synchronize()
        return int(self.host_excluded.max()) if self.host_excluded is not None else 0


class Server:
    def __init__(self, backend=None, memory_budget: Optional[int] = None, max_slots: int = 64,
                 quantum_steps: int = 50, max_backfill_wait: float = 2.0,
                 clock: Callable[[], float] = time.perf_counter, max_in_flight: int = 2,
                 quantum_work: Optional[float] = None, min_steps: int = 1):
        self.backend = backend if backend is not None else DeviceBackend()
        if memory_budget is None:
            import torch
            free, _ = torch.cuda.mem_get_info()
            memory_budget = int(0.85 * free)
        self.budget = int(memory_budget)
        self.max_slots = int(max_slots)
        self.quantum = int(quantum_steps)
        self.quantum_work = None if quantum_work is None else float(quantum_work)
        self.min_steps = max(1, int(min_steps))
        self.max_backfill_wait = float(max_backfill_wait)
        self.clock = clock
        self.t0 = clock()
        self.max_in_flight = max(1, int(max_in_flight))
        self.queue: Deque[_Job] = collections.deque()
        self.active: List[_Job] = []
        self.draining: List[_Job] = []
        self.results: List[JobResult] = []
        self.used = 0
        self.next_id = 0
        self.tokens: Deque[object] = collections.deque()
        self.rounds = 0

    def now(self) -> float:
        return self.clock() - self.t0

    # ---------------------------------------------------------------- API
    def submit(self, spec: JobSpec, arrival: Optional[float] = None) -> int:
        jid = self.next_id
        self.next_id += 1
        t = self.now() if arrival is None else float(arrival)
        try:
            fp = int(self.backend.footprint(spec))
        except Exception as exc:  # an invalid job is answered, not fatal to the server
            self.results.append(JobResult(jid, spec.name, None, t, t, t, 0, error=f"rejected: {exc}"))
            return jid
        job = _Job(jid, spec, t, fp)
        if fp > self.budget:
            self.results.append(JobResult(jid, spec.name, None, t, t, t, 0,
                                          error=f"footprint {fp} B exceeds the memory budget {self.budget} B"))
        else:
            self.queue.append(job)
        return jid

    def idle(self) -> bool:
        return not (self.queue or self.active or self.draining)

    def step(self) -> List[JobResult]:
        """One scheduling round: retire, admit, launch one quantum."""
        done = self._collect()
        self._admit()
        if self.active:
            while len(self.tokens) >= self.max_in_flight:
                self.backend.wait(self.tokens.popleft())
            work = []
            for j in self.active:
                n = min(self._steps_per_round(j.spec), j.spec.n_steps - j.done_steps)
                work.append((j.handle, j.spec, n))
                j.done_steps += n
            self.backend.advance([w for w in work if w[2] > 0])
            self.tokens.append(self.backend.barrier())
            self.rounds += 1
            still = []
            for j in self.active:
                if j.done_steps >= j.spec.n_steps:
                    j.pending = self.backend.finish(j.handle, j.spec)
                    self.backend.release(j.handle)
                    j.handle = None
                    # the job's buffers stay alive until its reduction and
                    # copy have completed: its footprint is given back in
                    # _collect, once the result is ready
                    self.draining.append(j)
                else:
                    still.append(j)
            self.active = still
        return done

    def run(self, arrivals: Optional[List[float]] = None, specs: Optional[List[JobSpec]] = None,
            idle_sleep: float = 2e-4, on_result: Optional[Callable[[JobResult], None]] = None) -> List[JobResult]:
        """Serves ``specs`` arriving at ``arrivals`` (seconds from now) and
        returns every result in completion order; ``on_result`` is called
        with each result as it is retired."""
        specs = specs or []
        arrivals = list(arrivals or [0.0] * len(specs))
        assert len(arrivals) == len(specs) and arrivals == sorted(arrivals)
        self.t0 = self.clock()
        k = 0
        while k < len(specs) or not self.idle():
            t = self.now()
            while k < len(specs) and arrivals[k] <= t:
                self.submit(specs[k], arrival=arrivals[k])
                k += 1
            for r in self.step():
                if on_result is not None:
                    on_result(r)
            if not self.active and not self.draining and not self.queue and k < len(specs):
                time.sleep(max(0.0, min(idle_sleep * 50, arrivals[k] - self.now())))
            elif not self.active and self.draining:
                time.sleep(idle_sleep)
        return self.results

    # ------------------------------------------------------------ internals
    def _steps_per_round(self, spec: JobSpec) -> int:
        if self.quantum_work is None:
            return self.quantum
        return max(1, min(self.quantum, max(self.min_steps, int(self.quantum_work // max(spec.n_traj, 1)))))

    def _collect(self) -> List[JobResult]:
        done, keep = [], []
        for j in self.draining:
            if j.pending.ready():
                self.used -= j.footprint
                r = JobResult(j.job_id, j.spec.name, j.pending.result(), j.arrival, j.admitted, self.now(),
                              j.spec.walker_steps, excluded=j.pending.excluded())
                self.results.append(r)
                done.append(r)
            else:
                keep.append(j)
        self.draining = keep
        return done

    def _admit(self):
        now = self.now()
        blocked_head = None
        for j in list(self.queue):
            if len(self.active) >= self.max_slots:
                break
            fits = self.used + j.footprint <= self.budget
            if blocked_head is not None and now - blocked_head.arrival > self.max_backfill_wait:
                break  # stop backfilling so memory drains for the head
            if not fits:
                if blocked_head is None:
                    blocked_head = j
                continue
            self.queue.remove(j)
            try:
                j.handle = self.backend.start(j.spec)
            except Exception as exc:  # e.g. the device ran out of memory: answer the job, keep serving
                self.results.append(JobResult(j.job_id, j.spec.name, None, j.arrival, now, now, 0,
                                              error=f"start failed: {exc}"))
                continue
            j.admitted = now
            self.used += j.footprint
            self.active.append(j)


def latency_stats(results: List[JobResult]) -> dict:
    ok = [r for r in results if not r.error]
    lat = np.array([r.latency for r in ok])
    if len(lat) == 0:
        return {"n_jobs": 0}
    span = max(r.finished for r in ok) - min(r.arrival for r in ok)
    return {
        "n_jobs": len(ok), "n_rejected": len(results) - len(ok),
        "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
        "mean_s": float(lat.mean()), "max_s": float(lat.max()),
        "makespan_s": float(span),
        "walker_steps_per_s": float(sum(r.walker_steps for r in ok) / span) if span > 0 else None,
    }


class SimBackend:
    """Host-only stand-in for the device: footprints from a formula, work
    completes after a modelled time.  Lets the scheduler run without a GPU."""

    def __init__(self, clock: Callable[[], float], bytes_per_walker: int = 100,
                 walker_steps_per_s: float = 1e9, sleep_until: Optional[Callable[[float], None]] = None):
        self.clock = clock
        self.sleep_until = sleep_until
        self.bpw = bytes_per_walker
        self.rate = walker_steps_per_s
        self.busy_until = 0.0
        self.log: List[list] = []
        self.started: List[int] = []

    def footprint(self, spec: JobSpec) -> int:
        return spec.n_traj * self.bpw

    def start(self, spec: JobSpec):
        self.started.append(id(spec))
        return {"spec": spec, "steps": 0}

    def advance(self, work):
        t = max(self.clock(), self.busy_until)
        cost = sum(s.n_traj * n for _, s, n in work) / self.rate
        self.busy_until = t + cost
        for h, s, n in work:
            h["steps"] += n
        self.log.append([(s.name, n) for _, s, n in work])

    def finish(self, handle, spec):
        return _SimFuture(self, self.busy_until, handle)

    def release(self, handle):
        pass

    def barrier(self):
        return self.busy_until

    def wait(self, token):
        if self.sleep_until is not None:
            self.sleep_until(token)
            return
        while self.clock() < token:
            time.sleep(1e-4)


class _SimFuture:
    def __init__(self, be, t, handle):
        self.be, self.t, self.handle = be, t, handle

    def ready(self):
        return self.be.clock() >= self.t

    def result(self):
        return np.array([self.handle["steps"]], dtype=np.float64)

    def excluded(self):
        return 0
