"""Shared helpers of the GPU parity tests (HIP library through the C ABI vs oracle)."""
import math

import numpy as np

from oracle import pqmc
from paper_2303_13403_amd import gpqmc

# "fp64": the factored FP64 engine (G = 1 - A B^T); "fp64wrap": FP64 with G
# wrapped as an N x N matrix; "mixed": FP32 Green's function of the wrap engine
PREC = {"fp64": gpqmc.FP64, "fp64wrap": gpqmc.FP64_WRAP, "mixed": gpqmc.MIXED,
        "mixed32b": gpqmc.MIXED_FP32_BASIS}
# G and ratio tolerance, max|x - x_ref| / max|x_ref|: FP64 paths 1e-10, mixed
# path 1e-5; the FP32-basis variant is bounded by eps_fp32 cond(L R), stated as 1e-4
TOL = {"fp64": 1e-10, "fp64wrap": 1e-10, "mixed": 1e-5, "mixed32b": 1e-4}
# acceptance draws this close to their threshold (relative) may decide differently
TIE = {"fp64": 1e-9, "fp64wrap": 1e-9, "mixed": 1e-4, "mixed32b": 1e-3}


def is_fp64(prec):
    return prec in ("fp64", "fp64wrap")


def rel_err(x, ref):
    x, ref = np.asarray(x), np.asarray(ref)
    return float(np.max(np.abs(x - ref)) / max(np.max(np.abs(ref)), 1e-300))


def make_context(workloads, prec, trace=False, chain_ids=None, **kw):
    chains = []
    for c, w in enumerate(workloads):
        cid = c if chain_ids is None else chain_ids[c]
        chains.append(gpqmc.chain_desc_arrays(w, cid, PREC[prec], trace=trace))
    return gpqmc.Context(chains, **kw)


def oracle_chain(w, chain_id, field=None):
    return pqmc.Chain(pqmc.Model.from_workload(w), seed=w.seed, chain_id=chain_id, field=field)


def oracle_fixed_pass(ch):
    """One oracle pass with every proposal rejected; records ratios and the
    fresh Green's functions at the checkpoints."""
    ch.record_ratios = True
    ch.record_greens = True
    ch.ratios.clear()
    ch.checkpoint_greens.clear()
    ch.checkpoint_logdets.clear()
    ch.follow = ch.field.copy()
    ch.follow_tol = math.inf
    try:
        ch.sweep(1, measure=False)
    finally:
        ch.follow = None
    return ch


def ratio_array(ch, sweep, n_slices, N):
    r = np.zeros((n_slices, N, 2))
    for (sw, l, i), v in ch.ratios.items():
        if sw == sweep:
            r[l, i, 0], r[l, i, 1] = v[0], v[1]
    return r
