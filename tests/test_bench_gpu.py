"""The benchmark's own bookkeeping on a small mesh: one JSON line with the
fields of its contract, consistent numbers, an FP32-form error that
matches what the FP32 tests bound (a reference state advanced past the
compared step, for instance, shows up as a large error here), and the
batched form's figures."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.gpu
def test_bench_line_on_a_small_mesh():
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--size", "64", "--steps", "6",
           "--warmup", "2", "--forms", "f32,batch", "--no-cpu-baseline", "--case-sizes", "48,64"]
    print("case: bench.py --size 64 --steps 6 --forms f32,batch --case-sizes 48,64", flush=True)
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
    assert line["host_dt_last"]["steps"] == 20 and line["host_dt_last"]["value"] > 0
    ceil = line["hbm_ceiling_gbs"]
    for key in ("copy_1to1", "copy_1to1_nt", "add_2to1", "add_2to1_nt", "torch_copy"):
        assert ceil[key] > 0, key
    assert roof["frac_of_ceiling"] == pytest.approx(roof["achieved"] / roof["ceiling_gbs"], rel=1e-3)
    assert line["step_frac_of_hbm_peak"] == pytest.approx(line["hbm_gbs_algorithmic"] / 8000.0,
                                                          rel=1e-3)
    # the other cases: the Riemann case at both sizes, the smooth case at the
    # size that is not the headline's; FP64 and FP32 each
    cases = line["cases"]
    assert sorted(cases) == sorted(["plane_48_f64", "plane_48_f32", "sine_48_f64", "sine_48_f32",
                                    "plane_64_f64", "plane_64_f32"]), sorted(cases)
    for key, c in cases.items():
        n = int(key.split("_")[1])
        assert c["value"] == pytest.approx(n ** 3 / (c["ms_per_step"] / 1e3), rel=1e-3), key
        assert 0 < c["roofline"]["frac"] < 1, key
    assert max(cases["plane_64_f32"]["linf_rel_err"]) < 1e-5
    assert max(cases["plane_64_f32"]["l1_rel_err"]) < 1e-6
    f32 = line["forms"]["f32"]
    # 8 steps of the FP32 form against the FP64 solution of the same input
    # and time steps: a few FP32 units in the last place
    assert max(f32["linf_rel_err"]) < 1e-5, f32
    assert max(f32["l1_rel_err"]) < 1e-6, f32
    # the batched form: 64 uneven problems, whole-batch rate against the same
    # problems one at a time; the batch fills the chip, one small problem
    # does not
    for key in ("batch_f64", "batch_f32"):
        b = line["forms"][key]
        assert b["value"] > 0 and b["sequential_value"] > 0, b
        assert b["value"] == pytest.approx(b["speedup_vs_one_at_a_time"] * b["sequential_value"],
                                           rel=1e-2), b
        assert b["speedup_vs_one_at_a_time"] > 1.0, b
        assert b["launch"]["tile_y"] in (8, 16) and b["launch"]["chunk_z"] in (16, 32, 64), b


def test_bench_refuses_several_gpus():
    # exits before touching the GPU: runs anywhere
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
