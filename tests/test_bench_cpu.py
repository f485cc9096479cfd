"""CPU checks of the benchmark's host-side pieces: the all-cores oracle
timing splits the rollout over particle ranges, which must give the
single-threaded oracle's costs and controls exactly; --gpus above 1 exits
with a message."""
import os
import subprocess
import sys

import numpy as np

from paper_2104_13542_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_chunked_oracle_rollout_equals_whole(oracle_lib):
    sys.path.insert(0, ROOT)
    import bench

    prob = inputs.config2(3, n_particles=40, horizon=12, n_obs_spheres=4, n_obs_cuboids=4)
    prob.params.n_halton = 17
    prob.params.n_null = 3
    p = prob.params
    o = oracle_lib.Oracle(prob)
    eps = o.noise(2)
    mean = np.random.default_rng(1).normal(scale=0.2, size=(p.horizon, 7))
    sig = np.full(7, 0.3)
    whole = o.rollout(mean, sig, eps, want_terms=False)
    parts = [bench._oracle_chunk((prob, a, b, mean, sig, eps[a:b])) for a, b in ((0, 9), (9, 23), (23, 38), (38, 40))]
    np.testing.assert_array_equal(np.concatenate([c for c, _ in parts]), whole["C"])
    np.testing.assert_array_equal(np.concatenate([u for _, u in parts]), whole["u"])


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
