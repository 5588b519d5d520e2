"""The benchmark's command-line contract: one JSON line with the measured metric,
its roofline and the CPU oracle baseline; a request for more than one GPU is
refused with a message."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_bench(*args, timeout=600):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                          capture_output=True, text=True, timeout=timeout)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = run_bench("--gpus", "2", timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


@pytest.mark.gpu
def test_json_line_carries_metric_roofline_and_cpu_baseline():
    print("[case] bench.py --workload small --steps 20 --warmup 2", flush=True)
    r = run_bench("--workload", "small", "--steps", "20", "--warmup", "2", "--cpu-seconds", "1")
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.strip()]
    assert len(lines) == 1, r.stdout
    d = json.loads(lines[0])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert key in d, key
    assert d["n_gpus"] == 1 and d["steps"] == 20 and d["warmup"] == 2
    assert d["unit"] == "mod-p GMAC/s" and d["higher_is_better"] is True and d["data"] == "synthetic"
    assert d["value"] > 0 and d["ms_per_step"] > 0
    # the headline is the paper's arithmetic (FP64 Q-adic words); the library's own
    # choice rides along with its speed-up over it
    assert d["dtype"] == "f64" and d["config"]["path"] == "fp64_qadic"
    assert d["paths"]["chosen"]["speedup_vs_headline"] > 0
    # value is m n k over the step time
    c = d["config"]
    assert "workload" in c
    assert abs(d["value"] - c["m"] * c["n"] * c["k"] / (d["ms_per_step"] * 1e-3) / 1e9) <= 1e-6 * d["value"]
    roof = d["roofline"]
    for key in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert key in roof, key
    assert roof["bound"] in ("mfma", "hbm", "alu")
    assert abs(roof["frac"] - roof["achieved"] / roof["peak"]) <= 1e-9 * max(1.0, roof["frac"])
    cpu = d["cpu_baseline"]
    for key in ("value", "unit", "cores", "kind", "sample"):
        assert key in cpu, key
    assert cpu["kind"] == "oracle" and cpu["cores"] >= 1 and cpu["value"] > 0
