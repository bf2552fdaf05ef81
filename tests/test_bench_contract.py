"""The measurement script's command-line contract: one JSON line with the
metric, throughput, roofline and CPU-baseline fields; more than one GPU is
refused with a message."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(args, timeout):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=timeout, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _run(["--gpus", "2"], 120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


@pytest.mark.gpu
def test_default_line_fields():
    r = _run(["--steps", "1", "--warmup", "0"], 300)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.strip().splitlines() if l.startswith("{")]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
              "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 1 and d["value"] > 0
    assert d["config"]["workload"] and d["config"]["evals_per_step"] == 64 * 100 * 14000
    rf = d["roofline"]
    assert rf["bound"] in ("alu", "hbm", "mfma") and 0 < rf["frac"] < 1
    assert abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-9
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["cores"] >= 1 and cb["value"] > 0 and cb["sample"]
    ac = cb["all_cores"]   # the oracle on a pool of one-thread worker processes
    assert ac["cores"] >= 1 and ac["value"] > 0 and ac["sample"]
    d = d["d100"]   # the D = 100 half of the metric, both precisions, with its oracle baseline
    assert d["evals_per_step"] == 128 * 256 * 500
    for prec in ("fp32", "bf16"):
        v = d[prec]
        assert v["value"] > 0 and v["ms_per_step"] > 0
        rf = v["roofline"]
        assert rf["bound"] == "mfma" and 0 < rf["frac"] < 1
        assert abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-9
    assert d["bf16"]["refine_rate"] is not None and 0 <= d["bf16"]["refine_rate"] <= 1
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["cores"] == 1 and cb["value"] > 0 and cb["sample"]
    assert cb["all_cores"]["cores"] >= 1 and cb["all_cores"]["value"] > 0
