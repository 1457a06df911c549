"""Binning and jackknife for sign-weighted Monte Carlo averages.

TEST INFRASTRUCTURE ONLY (see the package header).

<O> = sum_k s_k O_k / sum_k s_k (the sign-reweighted estimate of the projector
expectation value when configurations are sampled with |W|); its error is the
delete-one-bin jackknife over bins of consecutive measurements.
"""
from __future__ import annotations

import numpy as np


def binned(values, bin_size):
    v = np.asarray(values, dtype=np.float64)
    nb = len(v) // bin_size
    if nb < 2:
        raise ValueError("need at least two bins")
    return v[: nb * bin_size].reshape(nb, bin_size).mean(axis=1)


def sign_weighted(signs, obs, bin_size=10):
    """(mean, jackknife error) of sum(s O) / sum(s)."""
    s = binned(signs, bin_size)
    so = binned(np.asarray(signs, np.float64) * np.asarray(obs, np.float64), bin_size)
    nb = len(s)
    mean = so.sum() / s.sum()
    jk = (so.sum() - so) / (s.sum() - s)
    err = np.sqrt((nb - 1) / nb * np.sum((jk - jk.mean()) ** 2))
    return float(mean), float(err)


def mean_error(values, bin_size=10):
    b = binned(values, bin_size)
    return float(b.mean()), float(b.std(ddof=1) / np.sqrt(len(b)))
