"""The benchmark's output contract on a small channel: one JSON line last on
stdout with the fields the benchmark promises (metric, value, unit, counts,
dtype, workload, roofline of the dominant kernel, the three legs), run as its
own process the way it is launched."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_json_line_on_a_small_channel():
    args = ["--n", "32", "--steps", "2", "--warmup", "1", "--tank-n", "0", "--incline-n", "0", "--learned-n", "0",
            "--cg-n", "0", "--kernel-n", "0", "--fp32-n", "0", "--cpu-sample", "0"]
    print(f"[bench] {' '.join(args)}", flush=True)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                       timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    line = r.stdout.strip().splitlines()[-1]
    d = json.loads(line)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline", "sequence", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 2 and d["warmup"] == 1
    assert d["unit"] == "particle-iters/s" and d["higher_is_better"] is True and d["data"] == "synthetic"
    assert d["dtype"] == "f32" and d["vs_baseline"] is None and d["cpu_baseline"] is None
    assert d["value"] > 0 and d["ms_per_step"] > 0
    assert "workload" in d["config"] and d["config"]["n_particles"] > 32 ** 3
    seq = d["sequence"]
    assert set(seq) == {"learned_f32op", "plain_f32op", "plain_f64"}
    for leg in seq.values():
        assert len(leg["iterations"]) == 2 and leg["true_rel_res_max"] < 1e-6
    rf = d["roofline"]
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    assert abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-3 and 0.0 < rf["frac"] < 1.0
    # measured traffic belongs to the 320^3 channel's counters only
    assert rf["traffic"] is None
