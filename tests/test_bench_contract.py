"""bench.py's output contract: one JSON line with the metric, the roofline of the
dominant kernel and the comparison path; multi-GPU runs are refused."""
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
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


@pytest.mark.gpu
def test_json_line_at_the_small_workload():
    r = run_bench("--workload", "fzp2mm", "--steps", "1", "--warmup", "0", "--no-batch", "--no-multilevel",
                  "--no-cpu-baseline", "--no-configs", "--no-surrogate", "--no-sa", "--fp64-steps", "1", "--fp64-warmup", "0")
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for key, kind in (("metric", str), ("value", float), ("unit", str), ("n_gpus", int), ("steps", int),
                      ("warmup", int), ("ms_per_step", float), ("higher_is_better", bool), ("scaling", str),
                      ("dtype", str), ("data", str), ("config", dict), ("roofline", dict)):
        assert isinstance(d[key], kind), key
    assert d["n_gpus"] == 1 and d["steps"] == 1 and d["value"] > 0 and d["higher_is_better"] is True
    assert d["vs_baseline"] is None
    assert d["config"]["workload"] and "model" not in d["config"]
    ro = d["roofline"]
    assert ro["bound"] == "mfma" and ro["unit"] == "TFLOP/s" and ro["peak"] == 2500.0
    assert 0 < ro["achieved"] < ro["peak"] and abs(ro["frac"] - ro["achieved"] / ro["peak"]) < 1e-3
    assert ro["traffic"] is None            # the committed counters cover the 1 m workload only
    assert ro["mfma_busy"] is None
    assert d["valid_rel_l2_le_1e-4"] is True and d["rel_l2_split_vs_fp64"] <= 1e-4
    assert d["fp64_bluestein"]["roofline"]["bound"] == "alu"
    i8 = d["split_int8"]
    assert i8["gsamples_s"] > 0 and i8["valid_rel_l2_le_1e-4"] is True
    assert i8["roofline"]["unit"] == "TOP/s" and i8["roofline"]["peak"] == 5000.0
    assert 0 < i8["roofline"]["frac"] < 1
