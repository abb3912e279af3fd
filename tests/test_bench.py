"""The benchmark's command-line contract: one JSON line with the fields the
throughput report needs, and a clear refusal of more than one GPU."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_bench(*args, timeout=600):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                          capture_output=True, text=True, timeout=timeout)


def test_more_than_one_gpu_is_refused():
    r = run_bench("--gpus", "2", timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


@pytest.mark.gpu
def test_bench_line_fields():
    """A short run of the default workload, with a short oracle sample: every
    field of the report, with the roofline of the dominant pass and the CPU
    baseline."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    r = run_bench("--steps", "20", "--warmup", "5", "--cpu-cell-updates", "3e7")
    assert r.returncode == 0, r.stderr[-2000:]
    d = json.loads(r.stdout.strip().splitlines()[-1])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
              "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 20 and d["warmup"] == 5
    assert d["value"] > 0 and d["ms_per_step"] > 0 and d["higher_is_better"] is True
    assert d["unit"] == "GCUPS" and d["dtype"] == "f32" and d["vs_baseline"] is None
    assert d["config"]["workload"].startswith("coupled_256_fp32")
    assert d["config"]["cells"] == 256 ** 3
    # exactly the requested attempts are issued in the timed region, as whole
    # graphs of a poll interval that divides them
    assert d["detail"]["attempts_timed"] == 20 and 20 % d["detail"]["steps_per_poll"] == 0
    roof = d["roofline"]
    assert roof["bound"] == "hbm" and roof["unit"] == "GB/s" and roof["peak"] == 8000.0
    assert 0 < roof["frac"] < 1 and abs(roof["frac"] - roof["achieved"] / roof["peak"]) < 1e-3
    assert "S4" in roof["kernel"]
    cpu = d["cpu_baseline"]
    assert cpu["kind"] == "oracle" and cpu["value"] > 0 and cpu["cores"] >= 1
    assert cpu["unit"] == "GCUPS" and "attempts" in cpu["sample"]
    assert "(256, 256, 256)" in cpu["sample"]


def test_poll_interval_divides_the_timed_attempts():
    sys.path.insert(0, ROOT)
    import bench
    assert bench.poll_interval(20, 5, 16) == 5
    assert bench.poll_interval(1000, 50, 16) == 10
    assert bench.poll_interval(64, 0, 16) == 16
    for steps, warm in ((20, 5), (1000, 50), (7, 3), (13, 0), (200, 20)):
        assert steps % bench.poll_interval(steps, warm, 16) == 0
