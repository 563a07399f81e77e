"""bench.py end to end at a reduced size: one JSON line with the fields its
contract names, a clean status word, and the roofline and CPU-baseline objects."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_reduced_run_prints_one_valid_json_line():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("\n[case] bench.py reduced", flush=True)
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--n", "512", "--steps", "3",
           "--warmup", "1", "--cpu-n", "64", "--cpu-strip", "16", "--cpu-c2-steps", "3",
           "--adjoint-steps", "4", "--no-batched"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=280, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-3000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1, r.stdout[-2000:]
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
              "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 3 and d["warmup"] == 1 and d["dtype"] == "f64"
    assert d["value"] > 0 and d["status_word"] == 0 and "workload" in d["config"]
    assert d["metric"].startswith("2D Euler HWENO cell-stage updates/s")
    assert 0 < d["roofline"]["hbm_frac"] < 1 and d["adjoint"]["backward_over_forward"] > 0
    rf = d["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in rf, k
    assert 0 < rf["frac"] < 1 and rf["traffic"] is None    # traffic is measured at 4096^2 only
    assert rf["flop_per_cell_stage"] == 3800.0 and rf["derived"]["flop_per_cell_stage"] == 4130.0
    assert rf["hbm_bytes_per_cell_stage"] == 256
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["value"] > 0 and cb["cores"] >= 1
    assert cb["single_thread"]["value"] > 0 and cb["euler1d_4000"]["value"] > 0
    for dt_name in ("f64", "f32"):
        assert d["c3_1024"][dt_name]["value"] > 0 and d["c3_1024"][dt_name]["status"] == 0
    # the headline adjoint figure is the configured checkpointed rollout
    assert d["adjoint"]["checkpoint_every"] == 20 and "meets_target" in d["adjoint"]
    assert d["adjoint"]["every_step_kept"]["grad_finite"]
    assert d["adjoint"]["grad_finite"] and d["small_grid"]["status"] == 0
    # the adjoint kernel against its roofline: 20 taped steps' adjoints, 60 timed launches
    ar = d["adjoint"]["roofline"]
    assert ar["launches"] == 60 and ar["launch_ms"] > 0 and ar["finite"], ar
    assert ar["frac"] is None or 0 < ar["frac"] < 1, ar
    # time-to-solution runs of Examples 3.11 and 3.12: reached T with a clean status word
    for leg, T in (("double_mach", 0.2), ("forward_step", 4.0)):
        r_ = d[leg]
        assert r_["status"] == 0 and r_["steps"] > 0 and r_["value"] > 0, (leg, r_)
        assert abs(r_["t"] - T) <= 1e-12 * T, (leg, r_["t"])


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2 and "one GPU" in r.stderr
