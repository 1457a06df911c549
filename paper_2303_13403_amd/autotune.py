"""Autotuner for the delay rank k and the stabilisation interval n_s of a batch.

Both parameters trade speed against work or accuracy:

* k (sites per delayed segment) sets how often the whole Green's function is
  streamed by a flush (N / k times per slice) against the size of the
  submatrix merge inside the scan (quadratic in the accepted count);
* n_s (slices between re-stabilisations) sets how often the FP64 checkpoint
  (Cholesky-QR, (L R)^{-1}, fresh G) runs, against the drift the wrapped
  Green's function accumulates in between.

For every candidate pair the tuner builds a context for the caller's batch,
runs warm-up sweeps, times sweeps with HIP events on the context's stream and
reads every chain's largest relative checkpoint drift (|G_wrapped - G_fresh|
over |G_fresh|, largest elements).  A pair qualifies when the 90th percentile
of those drifts over the batch stays below the precision's limit (FP64: 1e-6;
with an FP32 Green's function: 1e-5, the mixed path's stated accuracy; these
are the library's default flag thresholds) and no chain went non-finite or
singular.  It returns the fastest qualifying pair and raises NoQualifyingPair
(carrying the table) if none qualifies.
Everything runs through the C ABI; nothing here computes any part of the
method.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import Iterable, List, Optional, Sequence

from . import gpqmc
from .workloads import Workload

__all__ = ["Trial", "autotune", "qualifies", "DRIFT_LIMIT", "NoQualifyingPair"]

DRIFT_LIMIT = {gpqmc.FP64: 1e-6, gpqmc.FP64_WRAP: 1e-6, gpqmc.MIXED: 1e-5,
               gpqmc.MIXED_FP32_BASIS: 1e-5}


class NoQualifyingPair(RuntimeError):
    """No (k, n_s) candidate met the drift limit; ``trials`` holds the table."""

    def __init__(self, trials, limit):
        super().__init__(f"no (k, n_s) candidate keeps the 90th-percentile relative drift "
                         f"within {limit:g}")
        self.trials = trials


@dataclasses.dataclass
class Trial:
    delay_rank: int
    stab_interval: int
    ms_per_sweep: float
    updates_per_s: float
    max_rel_drift: float
    p90_rel_drift: float
    flags: int


def _run(ws: Sequence[Workload], precision: int, k: int, n_s: int, warmup: int, sweeps: int,
         device: str) -> Trial:
    import torch

    descs = [gpqmc.chain_desc_arrays(w.replace(delay_rank=k, stab_interval=n_s), c, precision)
             for c, w in enumerate(ws)]
    ctx = gpqmc.Context(descs, device=device, meas_capacity=max(8, warmup + sweeps + 2))
    try:
        ctx.init_trial()
        ctx.sweep(warmup, measure=False)
        ctx.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(ctx.stream)
        ctx.sweep(sweeps, measure=False)
        ev1.record(ctx.stream)
        ev1.synchronize()
        ms = ev0.elapsed_time(ev1) / sweeps
        infos = [ctx.chain_info(c) for c in range(len(ws))]
    finally:
        ctx.close()
    updates = sum((2 * w.l_half + 2) * w.n_sites for w in ws)
    flags = 0
    for i in infos:
        flags |= i["flags"]
    rel = sorted(r if math.isfinite(r) else math.inf for r in (i["max_rel_drift"] for i in infos))
    p90 = rel[min(len(rel) - 1, (9 * len(rel)) // 10)]
    return Trial(k, n_s, ms, updates / (ms / 1e3), rel[-1], p90, flags)


def qualifies(t: Trial, limit: float) -> bool:
    """90th-percentile relative drift within ``limit``, every drift finite and
    no chain with a non-finite Green's function or a singular L R."""
    return t.p90_rel_drift <= limit and math.isfinite(t.max_rel_drift) and (t.flags & 6) == 0


def autotune(workloads: Sequence[Workload], precision: int,
             delay_ranks: Iterable[int] = (16, 32, 64),
             stab_intervals: Iterable[int] = (3, 5, 10),
             warmup: int = 1, sweeps: int = 2, device: str = "cuda:0",
             drift_limit: Optional[float] = None, log=None):
    """Time every (k, n_s) candidate on the batch ``workloads`` and return
    ``(best, trials)``: the chosen :class:`Trial` and the table of all trials.

    Candidates with k above the largest lattice are skipped (they equal
    k = N).  ``drift_limit`` defaults to the library's drift tolerance of the
    precision."""
    limit = DRIFT_LIMIT[precision] if drift_limit is None else drift_limit
    n_max = max(w.n_sites for w in workloads)
    trials: List[Trial] = []
    for k in delay_ranks:
        if k > max(n_max, min(delay_ranks)):
            continue
        for n_s in stab_intervals:
            t0 = time.time()
            tr = _run(workloads, precision, int(k), int(n_s), warmup, sweeps, device)
            trials.append(tr)
            if log is not None:
                log(f"autotune k={k:3d} n_s={n_s:2d}: {tr.ms_per_sweep:9.2f} ms/sweep "
                    f"{tr.updates_per_s:.4g} upd/s  relative drift p90 {tr.p90_rel_drift:.2e} "
                    f"max {tr.max_rel_drift:.2e} "
                    f"({time.time() - t0:.1f} s)")
    ok = [t for t in trials if qualifies(t, limit)]
    if not ok:
        raise NoQualifyingPair(trials, limit)
    return min(ok, key=lambda t: t.ms_per_sweep), trials
