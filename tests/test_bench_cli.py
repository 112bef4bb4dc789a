"""bench.py and the binding on the host: more than one GPU is refused with a
message (the measured path runs on one GPU); stored HBM byte counts are
reported only for the kernel sources, precision and launch size they were
taken for; without the built library every entry point raises."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_stored_traffic_is_guarded(tmp_path):
    sys.path.insert(0, ROOT)
    import bench
    rec = {"precision": "fp32", "paths_per_step": 62500, "source_sha256": bench.kernel_source_hash(),
           "bytes_per_launch": 123.0}
    path = str(tmp_path / "t.json")
    with open(path, "w") as f:
        json.dump(rec, f)
    assert bench.stored_traffic(path, "fp32", 62500) == 123.0
    assert bench.stored_traffic(path, "fp64", 62500) is None
    assert bench.stored_traffic(path, "fp32", 6250) is None
    with open(path, "w") as f:
        json.dump(dict(rec, source_sha256="0" * 64), f)
    assert bench.stored_traffic(path, "fp32", 62500) is None   # counters of another kernel version
    assert bench.stored_traffic(str(tmp_path / "missing.json"), "fp32", 62500) is None
    # the committed profile names its summary file
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
        t = json.load(f)
    assert os.path.exists(os.path.join(ROOT, "profiles", t["summary"]))


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without the built HIP library every entry point raises; nothing falls
    back to a CPU computation."""
    import numpy as np

    from paper_1512_02818_amd import pdd
    monkeypatch.setattr(pdd, "LIB_PATH", str(tmp_path / "libpdd.so"))
    monkeypatch.setattr(pdd, "_lib", None)
    for call in (lambda: pdd.lib(),
                 lambda: pdd.glm_fit(np.arange(3.0), np.arange(3.0)),
                 lambda: pdd.plan_paths(np.zeros(1, dtype=pdd.STATS_DTYPE), 1e-3, 100)):
        with pytest.raises(RuntimeError, match="no CPU fallback"):
            call()


def test_serving_knee():
    """The knee of a rate sweep: the highest rate up to which every rate
    completed everything (and, with a busy limit, left the device idle part
    of the time); unordered input is sorted by rate first."""
    sys.path.insert(0, ROOT)
    import bench

    def r(rate, offered, completed, busy=0.5):
        return {"rate_per_s": rate, "offered": offered, "completed": completed,
                "cancelled": offered - completed, "busy_frac": busy}
    sweep = [r(5.0, 10, 10), r(0.5, 6, 6), r(1.0, 8, 7), r(2.0, 9, 9)]
    assert bench.knee_rate(sweep) == 0.5  # 1 request/s lost one: the higher rates do not count
    assert bench.knee_rate([r(1.0, 3, 2)]) is None
    light = [r(10.0, 46, 46, 0.32), r(25.0, 109, 109, 0.84), r(50.0, 191, 191, 0.94), r(100.0, 413, 413, 1.0)]
    assert bench.knee_rate(light, busy_limit=0.95) == 50.0
    assert bench.knee_rate(light) == 100.0
