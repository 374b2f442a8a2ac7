"""Host-side parts of bench.py (no GPU): the one-GPU refusal, the seeded serving trace and the
batching workload, and the CPU description that goes into cpu_baseline."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode != 0
    assert "one GPU" in (p.stdout + p.stderr)


def test_serving_trace_is_seeded_and_shaped():
    a, b = bench.make_trace(0.5), bench.make_trace(0.5)
    assert len(a) == len(b) == 99                     # Poisson arrivals at 200/s over the first 0.5 s
    t = np.array([r["t"] for r in a])
    assert np.all(np.diff(t) >= 0) and t[-1] <= 0.5
    for r, s in zip(a, b):
        assert r["t"] == s["t"] and r["q"] == s["q"] and np.array_equal(r["X"], s["X"])
        n, d = r["X"].shape
        assert 1000 <= n <= 500_000 and 6 <= d <= 24 and r["q"] in (4, 5, 6)
        assert np.allclose(r["f"], np.sin(r["X"].sum(1)))
        assert np.all(r["X"] >= 0) and np.all(r["X"] <= r["b"][None, :])
    # the slice is the start of the 60 s trace
    full = bench.make_trace(1.0)
    assert [r["t"] for r in full[:len(a)]] == list(t)


def test_batching_workload_is_seeded_and_shaped():
    p = bench.make_batch_problems(16)
    q = bench.make_batch_problems(16)
    for (n, d, X, b), (n2, d2, X2, b2) in zip(p, q):
        assert (n, d) == (n2, d2) and np.array_equal(X, X2)
        assert 2000 <= n <= 200_000 and 8 <= d <= 16 and X.shape == (n, d)


def test_cpu_model_names_the_processor():
    m = bench.cpu_model()
    assert isinstance(m, str) and m and m != "unknown"
