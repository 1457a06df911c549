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
    assert bench.read_traffic(512, "mixed", "12x12") is None
    f.write_text(f.read_text().replace(bench.kernel_sha(), "0" * 16))
    assert bench.read_traffic(512, "mixed") is None


def test_library_estimator_equals_the_oracle_estimator():
    """The binned sign-weighted jackknife of the product side (the estimator
    of gpqmc_measure_*) equals the oracle's stats.sign_weighted on the same
    records, signs included."""
    from oracle import stats

    rng = np.random.default_rng(11)
    n = 230
    rec = np.stack([rng.choice([-1.0, 1.0], n, p=[0.2, 0.8]), rng.normal(-1.0, 0.4, n),
                    rng.uniform(0, 0.2, n), rng.uniform(0, 0.05, n)], axis=1)
    for col in (1, 2, 3):
        m, e = bench.weighted_mean(rec, col)
        mo, eo = stats.sign_weighted(rec[:, 0], rec[:, col], bin_size=10)
        assert abs(m - mo) < 1e-14 and abs(e - eo) < 1e-14


def test_pooled_over_chains_reduces_to_the_standard_error_of_chain_means():
    """Delete-one-chain jackknife: with every sign +1 and chains of equal
    length, the pooled mean is the grand mean and its error the standard error
    of the chain means; the average sign with all signs +1 is exactly 1 with
    zero error; sign weighting counts negative records negatively."""
    from paper_2303_13403_amd.estimators import pooled_over_chains

    rng = np.random.default_rng(5)
    recs = [np.stack([np.ones(6), rng.normal(-1.0, 0.3, 6), np.zeros(6), np.zeros(6)], axis=1)
            for _ in range(40)]
    m, e = pooled_over_chains(recs, 1)
    cm = np.array([r[:, 1].mean() for r in recs])
    assert abs(m - cm.mean()) < 1e-14
    assert abs(e - cm.std(ddof=1) / np.sqrt(len(cm))) < 1e-14
    assert pooled_over_chains(recs, 0) == (1.0, 0.0)
    two = [np.array([[1.0, 2.0, 0, 0], [1.0, 2.0, 0, 0]]), np.array([[-1.0, 5.0, 0, 0], [1.0, 3.0, 0, 0]])]
    # sum(s E) = 2 + 2 - 5 + 3 = 2, sum(s) = 2
    assert abs(pooled_over_chains(two, 1)[0] - 1.0) < 1e-15
    assert abs(pooled_over_chains(two, 0)[0] - 0.5) < 1e-15
    assert pooled_over_chains(recs[:1], 1) is None


def test_cpu_baseline_runs_one_chain_per_core():
    """The oracle leg on the 4x4 workload with two cores: fresh processes, one
    chain each, the aggregate rate, the CPU model and the core count."""
    import argparse

    a = argparse.Namespace(workload="4x4", ns=5, k=16, cpu_cores=2, chains=2)
    out = bench.cpu_baseline(a)
    assert out["kind"] == "oracle" and out["cores"] == min(2, len(os.sched_getaffinity(0)))
    assert out["value"] > 0 and out["per_core"] > 0 and out["cpu_model"]
