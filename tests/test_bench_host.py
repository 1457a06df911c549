"""Host-side logic of bench.py (no GPU): the one-GPU guard, the estimator that
combines measurement records over chain groups, and the traffic summary check."""
import os
import subprocess
import sys

import numpy as np

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_weighted_mean_with_unit_sign_is_the_binned_mean():
    # with every sign +1, <s E>/<s> is the plain mean, and the delete-one-bin
    # jackknife of a ratio with constant denominator is the standard error of
    # the bin means
    rng = np.random.default_rng(7)
    n = 200
    rec = np.stack([np.ones(n), rng.normal(-1.0, 0.3, n), rng.uniform(0, 0.2, n)], axis=1)
    bins = rec[:, 1].reshape(20, 10).mean(axis=1)
    m, e = bench.weighted_mean(rec, 1)
    assert abs(m - rec[:, 1].mean()) < 1e-14
    assert abs(e - bins.std(ddof=1) / np.sqrt(20)) < 1e-14
    s, se = bench.weighted_mean(rec, 0)
    assert s == 1.0 and se == 0.0


def test_weighted_mean_is_sign_weighted():
    # two bins: signs (+1 x 10) with E = 1, then (-1 x 3, +1 x 7) with E = 3:
    # <s E> / <s> = (10 * 1 + 4 * 3) / (10 + 4) = 22 / 14
    rec = np.zeros((20, 3))
    rec[:, 0] = 1.0
    rec[10:13, 0] = -1.0
    rec[:10, 1] = 1.0
    rec[10:, 1] = 3.0
    m, _ = bench.weighted_mean(rec, 1)
    assert abs(m - 22.0 / 14.0) < 1e-15
    assert bench.weighted_mean(rec[:19], 1) is None       # fewer than two bins


def test_traffic_summary_is_used_only_for_the_same_kernel_and_launch(tmp_path, monkeypatch):
    f = tmp_path / "traffic.txt"
    f.write_text(f"kernel_source_sha: {bench.kernel_sha()}\nchains: 2048\nchains_per_launch: 512\n"
                 "precision: mixed\nhbm_bytes_per_launch: 12345\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.read_traffic(512, "mixed") == 12345.0
    assert bench.read_traffic(2048, "mixed") is None
    assert bench.read_traffic(512, "fp64") is None
    f.write_text(f.read_text().replace(bench.kernel_sha(), "0" * 16))
    assert bench.read_traffic(512, "mixed") is None
