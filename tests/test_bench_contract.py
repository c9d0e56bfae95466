"""Host-side parts of bench.py: the multi-GPU refusal and the guarded
lookup of counter-derived HBM traffic."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_traffic_only_for_the_profiled_build(tmp_path, monkeypatch):
    import bench
    good = bench.kernel_sources_sha256()
    prof = tmp_path / "p.md"
    prof.write_text("x\n    traffic_bytes_per_launch: 123\n    n_traj: 1000\n    precision: fp32\n"
                    f"    kernel_sources_sha256: {good}\n")
    monkeypatch.setattr(bench, "HBM_PROFILE", str(prof))
    assert bench.measured_traffic(1000, "fp32") == 123
    assert bench.measured_traffic(2000, "fp32") is None
    assert bench.measured_traffic(1000, "fp64") is None
    prof.write_text(prof.read_text().replace(good, "0" * 64))
    assert bench.measured_traffic(1000, "fp32") is None


def test_committed_counters_match_the_current_kernel_sources():
    """The headline's HBM counter profile was taken on the kernel sources as
    they stand, so the bench line carries roofline.traffic."""
    import bench
    assert bench.measured_traffic(10_000_000, "fp32") is not None


def test_oracle_beside_the_other_legs():
    import bench
    legs = bench._oracle_other_legs()
    assert set(legs) == {"spin_boson_1mode_full", "spin_boson_ohmic_kT0.2", "pyrazine_bilinear", "resample"}
    for v in legs.values():
        assert v["value"] > 0 and v["cores"] >= 1 and v["sample"]


def test_oracle_accuracy_against_the_stored_oracle_run():
    """The bench's accuracy block compares a full-size result with the
    oracle's stored run: the stored result itself has no error, a result
    off by 2e-3 in one bin's population is reported as such."""
    import json
    import numpy as np
    import bench
    import workloads as W
    wl = W.pyrazine_ci()
    ref = np.array(json.load(open(bench.GOLDEN))["out"])
    acc = bench.oracle_accuracy(ref, wl, wl.run.n_traj, "fp32")
    assert acc["max_abs_upper_population_diff"] == 0.0 and acc["bins_within_1e-3"] == acc["bins"] == 101
    off = ref.copy()
    off[3, 0, 1, 1, 0] += 2e-3
    acc = bench.oracle_accuracy(off, wl, wl.run.n_traj, "fp32")
    assert abs(acc["max_abs_upper_population_diff"] - 2e-3) < 1e-12 and acc["bins_within_1e-3"] == 100
    assert bench.oracle_accuracy(ref, wl, 12345, "fp32") is None
    assert abs(bench.flops_per_traj_step(2, 3, bench.coupling_slots(wl.model)) - 124.0) < 1e-9
