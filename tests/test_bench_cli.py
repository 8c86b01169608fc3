"""bench.py's command line on the host (nothing here touches a GPU)."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, cwd=ROOT)


def test_more_than_one_gpu_exits_with_a_message():
    r = _run("--gpus", "2")
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_unknown_workload_is_rejected():
    r = _run("--workload", "c9")
    assert r.returncode != 0
    assert "invalid choice" in r.stderr


def test_cpu_baseline_reports_all_core_and_single_thread():
    import numpy as np
    import bench
    from synth import make_config
    sc = make_config(2, small=True)
    frames = sc.frames(range(6))
    targets = [sc.target(t) for t in range(6)]
    r = bench.cpu_baseline(sc, frames, targets, 300, 40, reps=2)
    assert r["kind"] == "oracle" and r["unit"] == "frames/s" and r["cores"] >= 1
    assert r["value"] > 0 and r["single_thread"]["value"] > 0 and r["single_thread"]["cores"] == 1
    assert np.isfinite(list(r["seconds_per_frame_median"].values())).all()
