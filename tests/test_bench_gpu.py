"""The benchmark's own bookkeeping on a small mesh: one JSON line with the
fields of its contract, consistent numbers, and an FP32-form error that
matches what the FP32 tests bound (a reference state advanced past the
compared step, for instance, shows up as a large error here)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.gpu
def test_bench_line_on_a_small_mesh():
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--size", "64", "--steps", "6",
           "--warmup", "2", "--forms", "f32", "--no-cpu-baseline"]
    print("case: bench.py --size 64 --steps 6 --forms f32", flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    line = json.loads(r.stdout.strip().splitlines()[-1])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
                "higher_is_better", "scaling", "dtype", "data", "config", "roofline"):
        assert key in line, key
    assert line["n_gpus"] == 1 and line["steps"] == 6 and line["warmup"] == 2
    cells = 64 ** 3
    assert line["value"] == pytest.approx(cells / (line["ms_per_step"] / 1e3), rel=1e-9)
    roof = line["roofline"]
    assert 0 < roof["frac"] < 1 and roof["achieved"] == pytest.approx(roof["frac"] * roof["peak"], rel=1e-3)
    assert line["repeats"]["blocks"] == 5 and line["host_dt"]["steps"] == 20
    assert line["hbm_copy_ceiling_gbs"] > 0
    f32 = line["forms"]["f32"]
    # 8 steps of the FP32 form against the FP64 solution of the same input
    # and time steps: a few FP32 units in the last place
    assert max(f32["linf_rel_err"]) < 1e-5, f32
    assert max(f32["l1_rel_err"]) < 1e-6, f32


def test_bench_refuses_several_gpus():
    # exits before touching the GPU: runs anywhere
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
