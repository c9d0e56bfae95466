"""Scheduling logic of the job server (admission by memory footprint, slot
limit, quanta, backfill, rejection), driven on the host with a modelled
device and a manual clock."""
import types

import pytest

from paper_2608_14544_amd.serve import JobSpec, Server, SimBackend, latency_stats


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def until(self, t):
        self.t = max(self.t, t)


def spec(name, n_traj, n_steps):
    run = types.SimpleNamespace(n_traj=n_traj, n_steps=n_steps, dt=0.1, cadence=10, seed=0)
    return JobSpec(types.SimpleNamespace(run=run), name=name)


def drive(server, clock, dt=1e-3, limit=100000):
    peak_used, peak_active = 0, 0
    for _ in range(limit):
        if server.idle():
            break
        server.step()
        peak_used = max(peak_used, server.used)
        peak_active = max(peak_active, len(server.active))
        assert server.used <= server.budget
        # a retired job keeps its buffers until its result has been copied
        # out: its footprint counts until then
        assert server.used == sum(j.footprint for j in server.active + server.draining)
        clock.t += dt
    assert server.idle()
    return peak_used, peak_active


def make(budget=1000, slots=8, quantum=10, rate=1e6, wait=1.0):
    clock = Clock()
    be = SimBackend(clock, bytes_per_walker=1, walker_steps_per_s=rate, sleep_until=clock.until)
    srv = Server(be, memory_budget=budget, max_slots=slots, quantum_steps=quantum,
                 max_backfill_wait=wait, clock=clock)
    return srv, be, clock


def test_footprint_admission_and_completion():
    srv, be, clock = make(budget=1000)
    for name, T in (("a", 600), ("b", 300), ("c", 500)):
        srv.submit(spec(name, T, 40))
    srv.step()
    assert sorted(j.spec.name for j in srv.active) == ["a", "b"]  # c does not fit yet
    peak, _ = drive(srv, clock)
    assert peak <= 1000
    res = {r.name: r for r in srv.results}
    assert set(res) == {"a", "b", "c"} and all(not r.error for r in res.values())
    # memory is given back once a retired job's result is ready, so c
    # starts after a's result (a frees 600 of the 1000 bytes c needs 500 of)
    rounds_with = lambda n: [i for i, rnd in enumerate(be.log) if any(x == n for x, _ in rnd)]
    assert min(rounds_with("c")) > max(rounds_with("a"))
    assert res["c"].admitted >= res["a"].finished
    for r in res.values():  # every step was run, in quanta
        assert r.out[0] == 40


def test_quanta_cover_every_step():
    srv, be, clock = make(quantum=7)
    srv.submit(spec("x", 10, 95))
    drive(srv, clock)
    steps = [n for rnd in be.log for name, n in rnd if name == "x"]
    assert sum(steps) == 95 and max(steps) == 7 and len(steps) == 14


def test_slot_limit():
    srv, be, clock = make(budget=10 ** 9, slots=2)
    for i in range(5):
        srv.submit(spec(f"j{i}", 10, 30))
    _, peak_active = drive(srv, clock)
    assert peak_active == 2 and len(srv.results) == 5


def test_oversized_job_rejected():
    srv, be, clock = make(budget=100)
    srv.submit(spec("big", 1000, 10))
    srv.submit(spec("ok", 50, 10))
    drive(srv, clock)
    res = {r.name: r for r in srv.results}
    assert res["big"].error and res["big"].out is None
    assert not res["ok"].error


def test_backfill_then_head_protection():
    srv, be, clock = make(budget=1000, wait=0.05, rate=1e5)
    srv.submit(spec("long", 600, 2000))     # holds 600 B for a while
    srv.step()
    srv.submit(spec("head", 700, 10))       # cannot fit until "long" ends
    srv.submit(spec("small", 300, 100))     # fits now: backfilled
    srv.step()
    names = [j.spec.name for j in srv.active]
    assert "small" in names and "head" not in names
    clock.t += 0.1                          # head has waited past the limit
    srv.submit(spec("late", 50, 10))        # would fit, but must not overtake the head
    srv.step()
    assert "late" not in [j.spec.name for j in srv.active]
    drive(srv, clock)
    res = {r.name: r for r in srv.results}
    assert res["late"].admitted >= res["head"].admitted


def test_latency_stats():
    srv, be, clock = make()
    for i in range(4):
        srv.submit(spec(f"j{i}", 10, 20), arrival=0.0)
    drive(srv, clock)
    st = latency_stats(srv.results)
    assert st["n_jobs"] == 4 and st["p99_s"] >= st["p50_s"] > 0


def test_tuning_classes_and_table_roundtrip(tmp_path):
    from paper_2608_14544_amd.tune import TuningTable, kernel_class, padded_modes, rank_bucket
    assert padded_modes(1) == 4 and padded_modes(5) == 8 and padded_modes(9) == 16 and padded_modes(33) == 64
    assert padded_modes(100) == 128
    assert rank_bucket(0, 3) == 1 and rank_bucket(2, 3) == 3 and rank_bucket(4, 3) == 6
    assert kernel_class(2, 8, 3, "fp32") is None           # closed-form two-state kernels
    assert kernel_class(3, 40, 1, "fp32") == (3, 64, 1, "fp32")  # two-wave budget at 64 modes
    assert kernel_class(3, 100, 1, "fp32") is None         # no budget build above 64 modes
    assert kernel_class(4, 20, 1, "fp64") is None          # binary32 only
    assert kernel_class(4, 20, 2, "fp32") is None          # no budget build for four states at 32 modes
    assert kernel_class(4, 12, 2, "fp32") == (4, 16, 4, "fp32")
    assert kernel_class(3, 20, 2, "fp32") == (3, 32, 3, "fp32")
    t = TuningTable()
    t.choice[(4, 16, 4, "fp32")] = 3
    t.choice[(3, 16, 1, "fp32")] = 0
    t.choice[(2, 64, 1, "fp32")] = 2
    t.wpc[(4, 64, 1, 0, 0, "fp32")] = 2
    t.wpc[(2, 3, 0, 0, 0, "fp32")] = 0
    t.serving["quantum_work"] = 8e8
    t.serving["min_steps"] = 16.0
    path = str(tmp_path / "tuning.json")
    t.save(path)
    u = TuningTable(path)
    assert u.choice == t.choice and u.wpc == t.wpc and u.quantum_work() == 8e8 and u.min_steps() == 16


def test_quantum_tuning_keeps_the_lowest_p99_pair():
    from paper_2608_14544_amd.tune import QUANTUM_CANDIDATES, TuningTable
    t = TuningTable()
    seen = []

    def run(q, ms):
        seen.append((q, ms))
        return {"p99_s": abs(q - 2e8) / 1e8 + (0.0 if ms == 16 else 0.5)}
    assert t.tune_quantum(run) == (2e8, 16)
    assert seen == [(float(q), int(m)) for q, m in QUANTUM_CANDIDATES]
    assert t.quantum_work() == 2e8 and t.min_steps() == 16


def test_failing_jobs_are_answered_not_fatal():
    srv, be, clock = make(budget=10 ** 6)

    class Flaky(SimBackend):
        def footprint(self, spec):
            if spec.name == "bad":
                raise ValueError("invalid model")
            return super().footprint(spec)

        def start(self, spec):
            if spec.name == "oom":
                raise MemoryError("device out of memory")
            return super().start(spec)

    fb = Flaky(clock, bytes_per_walker=1, walker_steps_per_s=1e6, sleep_until=clock.until)
    srv.backend = fb
    for name in ("bad", "oom", "good"):
        srv.submit(spec(name, 100, 20))
    drive(srv, clock)
    res = {r.name: r for r in srv.results}
    assert "invalid model" in res["bad"].error and "out of memory" in res["oom"].error
    assert not res["good"].error and srv.used == 0


def test_work_based_quanta():
    clock = Clock()
    be = SimBackend(clock, bytes_per_walker=1, walker_steps_per_s=1e6, sleep_until=clock.until)
    srv = Server(be, memory_budget=10 ** 9, quantum_steps=1000, quantum_work=10_000, clock=clock, min_steps=1)
    srv.submit(spec("small", 100, 300))     # 100 steps per round: done in 3 rounds
    srv.submit(spec("large", 10_000, 20))   # 1 step per round
    drive(srv, clock)
    steps = {}
    for rnd in be.log:
        for name, n in rnd:
            steps.setdefault(name, []).append(n)
    assert steps["small"] == [100, 100, 100] and steps["large"] == [1] * 20
    res = {r.name: r for r in srv.results}
    assert res["small"].finished < res["large"].finished


def test_work_based_quanta_step_floor():
    """A job whose share of a round is fewer than min_steps steps still
    advances min_steps (its state round trip is amortised), and never past
    its end or the per-round cap."""
    clock = Clock()
    be = SimBackend(clock, bytes_per_walker=1, walker_steps_per_s=1e6, sleep_until=clock.until)
    srv = Server(be, memory_budget=10 ** 9, quantum_steps=12, quantum_work=10_000, clock=clock, min_steps=8)
    srv.submit(spec("small", 100, 30))      # 100 steps by work, capped at 12: 12, 12, 6
    srv.submit(spec("large", 10_000, 20))   # 1 step by work, floored at 8: 8, 8, 4
    drive(srv, clock)
    steps = {}
    for rnd in be.log:
        for name, n in rnd:
            steps.setdefault(name, []).append(n)
    assert steps["small"] == [12, 12, 6] and steps["large"] == [8, 8, 4]
    assert all(not r.error for r in srv.results) and srv.used == 0
