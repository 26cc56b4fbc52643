"""bench.py's output contract: the JSON line with its fields, the roofline
and CPU-baseline objects, and the one-GPU guard. The CPU tests run the guard
and the oracle baseline; the GPU test runs a short bench."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_cpu_baseline_times_the_oracle():
    sys.path.insert(0, ROOT)
    import bench
    out, (steps, u_ref) = bench.cpu_baseline(seconds_target=0.5, large=False)
    assert out["kind"] == "oracle" and out["unit"] == "MLUPS" and out["value"] > 0
    assert steps >= 4 and u_ref.shape == (3, 64, 64, 64)
    assert out["cores"] == len(os.sched_getaffinity(0)) and out["single_core_MLUPS"] > 0
    assert "64^3" in out["sample"] and isinstance(out["cpu_model"], str) and out["tgv32_f64_100_steps_MLUPS"] > 0


@pytest.mark.gpu
def test_short_bench_line(monkeypatch, capsys):
    """In the test process itself (no second program on the GPU)."""
    sys.path.insert(0, ROOT)
    import bench
    monkeypatch.setattr(sys, "argv", ["bench.py", "--steps", "50", "--warmup", "2", "--no-autotune", "--no-extra",
                                      "--no-cpu-baseline", "--skip-fp64", "--copy-gib", "0.25", "--roofline-ticks", "4"])
    bench.main()
    lines = [ln for ln in capsys.readouterr().out.splitlines() if ln.startswith("{")]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
                "vs_baseline", "dtype", "data", "config", "roofline"):
        assert key in d, key
    assert d["n_gpus"] == 1 and d["steps"] == 50 and d["warmup"] == 2 and d["unit"] == "MLUPS"
    assert d["value"] > 1000 and d["higher_is_better"] is True and d["vs_baseline"] is None
    assert d["config"]["workload"] == "rtgv64x64_f32" and d["dtype"] == "f32" and d["data"] == "synthetic"
    rf = d["roofline"]
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    assert 0 < rf["frac"] < 1 and abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-3
    assert rf["algorithmic_bytes_per_launch"] == 216 * 64 * 64 ** 3
    assert rf["traffic"] is None or abs(rf["traffic"] / rf["algorithmic_bytes_per_launch"] - 1) < 0.01


@pytest.mark.gpu
def test_bench_measures_the_velocity_error_against_the_oracle():
    """The error field of the bench line: the GPU's sample 0 after the CPU
    baseline's number of steps against the oracle's field of that run."""
    sys.path.insert(0, ROOT)
    import bench
    import mc_inputs
    import paper_2608_23786_amd as mc
    import torch
    _, (steps, u_ref) = bench.cpu_baseline(seconds_target=0.5, large=False)
    wl = mc_inputs.WORKLOADS["rtgv64x64_f32"]
    err = bench.measured_error(mc, torch, wl, (256, 0, 1, 1), steps, u_ref)
    print(err)
    assert err["steps"] == steps and 0 < err["rel_l2_u_vs_oracle"] < 1e-5
