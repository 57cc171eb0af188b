"""The benchmark's command-line contract: one GPU only, and one JSON line
with the fields a reader of the results relies on."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_cpu_baseline_sample_and_gate_values():
    sys.path.insert(0, ROOT)
    import bench
    from oracle import oracle as orc
    from paper_2509_19294_amd import ics

    pos, vel, mass = ics.plummer(600, seed=3)
    cb, gate, refs = bench.cpu_baseline(pos, mass, 0.01, 0.2)
    assert cb["kind"] == "oracle" and cb["unit"] == "G pair-interactions/s" and cb["cores"] >= 1
    assert cb["value"] > 0 and "full evaluations" in cb["sample"]
    ra, rp = orc.accel_pot(pos, mass, 0.01)
    assert orc.rel_rms(refs[0], ra[gate]) < 1e-13 and orc.rel_rms(refs[1], rp[gate]) < 1e-13
    cb, gate, refs = bench.cpu_baseline(pos, mass, 0.01, 0.2, vel=vel)
    _, rj, _ = orc.accel_jerk(pos, vel, mass, 0.01)
    assert "jerks" in cb["sample"] and orc.rel_rms(refs[2], rj[gate]) < 1e-13


@pytest.mark.gpu
@pytest.mark.parametrize("extra", [[], ["--hermite"]])
def test_bench_json_line(extra):
    r = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--steps", "3", "--warmup", "1",
                        "--cpu-seconds", "1", *extra], capture_output=True, text=True, timeout=240, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    line = json.loads(r.stdout.strip().splitlines()[-1])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline", "accuracy"):
        assert key in line, key
    assert line["n_gpus"] == 1 and line["steps"] == 3 and line["warmup"] == 1
    assert line["value"] > 0 and line["accuracy"]["gate_rel_rms_1e-5"]
    assert "workload" in line["config"]
    rl = line["roofline"]
    assert rl["bound"] == "alu" and rl["unit"] == "TFLOP/s" and rl["peak"] == 157.3
    assert np.isclose(rl["frac"], rl["achieved"] / rl["peak"], atol=1e-4)
    ck = line["clock"]
    print("clock", ck, "frac", rl["frac"], "at measured clock", rl["frac_at_measured_clock"], flush=True)
    if ck["gfx_mhz_median"] is not None:
        assert 300 < ck["gfx_mhz_median"] < 3000 and ck["samples"] > 0
        assert np.isclose(rl["frac_at_measured_clock"],
                          rl["achieved"] / (rl["peak"] * ck["gfx_mhz_median"] / 2400.0), atol=1e-3)
    else:
        assert rl["frac_at_measured_clock"] is None and ck["notes"]
    cb = line["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["cores"] >= 1 and cb["value"] > 0
