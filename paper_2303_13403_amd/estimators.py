"""Estimators over measurement records (host side).

A record is one measurement of a chain at tau = Theta: (sign, E/N, D, S_AFM)
with D the double occupancy per site and S_AFM the staggered spin structure
factor (records with fewer columns are accepted: only the columns asked for
are read).  Sign-weighted averages <s O>/<s> over the
records of several chains, with a delete-one-bin jackknife error over bins of
ten consecutive records, the same estimator the library applies to one
context (gpqmc_measure_*).
"""
from __future__ import annotations

from typing import Optional, Tuple

import numpy as np

BIN = 10


def weighted_mean(rec: np.ndarray, which: int) -> Optional[Tuple[float, float]]:
    """<s O>/<s> over measurement records (rows: sign, E/N, D, S_AFM) with a
    delete-one-bin jackknife over bins of 10 records (which = 0: the sign
    itself, binned mean); the estimator the library applies to one context."""
    nb = len(rec) // BIN
    if nb < 2:
        return None
    rec = np.asarray(rec, np.float64)
    r = rec[: nb * BIN].reshape(nb, BIN, rec.shape[1])
    s = r[:, :, 0].mean(axis=1)
    if which == 0:
        return float(s.mean()), float(s.std(ddof=1) / np.sqrt(nb))
    so = (r[:, :, 0] * r[:, :, which]).mean(axis=1)
    S, SO = s.sum(), so.sum()
    jk = (SO - so) / (S - s)
    return float(SO / S), float(np.sqrt((nb - 1) / nb * ((jk - jk.mean()) ** 2).sum()))
