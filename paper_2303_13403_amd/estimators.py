"""Estimators over measurement records (host side).

A record is one measurement of a chain at tau = Theta: (sign, E/N, D, S_AFM)
with D the double occupancy per site and S_AFM the staggered spin structure
factor.  Sign-weighted averages <s O>/<s> (the reweighting of configurations
sampled with |W|; the paper's average-sign figures are <s>):

* ``weighted_mean``: the records of one or more chains concatenated, with a
  delete-one-bin jackknife over bins of ten consecutive records (the
  estimator the library applies, gpqmc_measure_*);
* ``pooled_over_chains``: many independent chains with few records each (a
  batch), with a delete-one-chain jackknife, so that no bin straddles two
  chains and the error reflects the chain-to-chain spread.
"""
from __future__ import annotations

from typing import Optional, Sequence, Tuple

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


def pooled_over_chains(recs: Sequence[np.ndarray], which: int) -> Optional[Tuple[float, float]]:
    """Pooled sum(s O) / sum(s) over the records of independent chains, error
    by delete-one-chain jackknife (which = 0: the average sign sum(s) / count,
    same jackknife).  Chains without records are skipped; at least two are
    needed."""
    so, s, n = [], [], []
    for r in recs:
        r = np.asarray(r, np.float64)
        if len(r) == 0:
            continue
        s.append(r[:, 0].sum())
        so.append((r[:, 0] * r[:, which]).sum() if which else r[:, 0].sum())
        n.append(float(len(r)))
    nc = len(s)
    if nc < 2:
        return None
    s, so, n = np.array(s), np.array(so), np.array(n)
    den = n if which == 0 else s
    S, SO = den.sum(), so.sum()
    jk = (SO - so) / (S - den)
    return float(SO / S), float(np.sqrt((nc - 1) / nc * ((jk - jk.mean()) ** 2).sum()))
