"""Throughput benchmark of the Gutzwiller-projection PQMC sweep on one MI355X.

Workload (the configuration the headline metric is quoted on): 16x16 periodic
Hubbard model, t = 1, U = 3.5, 112 + 112 electrons (<n> = 0.875), dtau = 0.1,
Theta = 10 (l_half = 100 slices per side, M + 2 = 202 slices), Neel trial
M_N = 0.07 with Gutzwiller g = 0.55 and the trial-only shell-closing ramp, a
batch of independent chains.

The timed path is GPQMC_FP64: every step in FP64 with the Green's function
kept as G = 1 - A B^T.  Two comparison legs are timed on the same batch: the
FP64 path that wraps G as an N x N matrix (GPQMC_FP64_WRAP) and the mixed path
with an FP32 Green's function (GPQMC_MIXED); each leg reports its checkpoint
drift and whether it holds the 1e-5 relative G error bound while sampling.

One step = one sweep (one pass over all 202 slices) of every chain of the
batch; value = HS-field updates (proposals) per second over the timed steps,
inputs resident in HBM.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--chains B] [--gpus 1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2303_13403_amd.estimators import pooled_over_chains, weighted_mean  # noqa: E402,F401

METRIC = "HS-field updates/sec at 16×16, L=100; mixed vs FP64 GPU at 1e-5 rel G error"
UNIT = "HS-field updates/s"
G_BOUND = 1e-5              # relative G error bound of the metric (mixed path)
PEAK_FP32_MFMA = 157.3e12   # MI355X dense FP32 matrix, FLOP/s
PEAK_FP64_MFMA = 78.6e12
PEAK_HBM = 8.0e12           # MI355X HBM3E, B/s
KERNEL_SRC = os.path.join(ROOT, "paper_2303_13403_amd", "csrc", "gpqmc_scan.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_segment_update_16x16_b2048.txt")
FLAGGED = 2 | 4 | 8         # NaN, singular L R, sign mismatch (chains left out of the estimates)

# in-sweep timed kernel classes (gpqmc_set_kernel_timing) of each engine
CLASSES = {
    "fp64": ("propagation", "segment_update", "scan"),
    "wrap": ("wrap", "propagation", "slice_update"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_sha() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def read_traffic(chains_per_launch: int, precision: str, workload: str = "16x16"):
    """HBM bytes per launch of the segment update from the committed PMC
    summary, if it was taken on the current kernel source, workload, launch
    size and precision."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if (kv.get("kernel_source_sha") != kernel_sha()
            or int(kv.get("chains_per_launch", -1)) != chains_per_launch
            or kv.get("precision") != precision
            or kv.get("workload", "16x16") != workload):
        return None
    return float(kv["hbm_bytes_per_launch"])


def finite_or_none(x):
    return x if (x is not None and math.isfinite(x)) else None


DEFAULT_CHAINS = {"16x16": 2048, "12x12": 2048, "honeycomb12x12": 2048, "24x24": 512,
                  "uneven": 256, "tv15_V1.6": 512, "tv15_V1.35": 512, "tv6": 2048}


def is_tv(w) -> bool:
    """A spinless t-V workload (bond fields, one species)."""
    return hasattr(w, "V")


def n_props(w) -> int:
    """HS fields per slice: sites (Hubbard) or bonds (t-V)."""
    return len(w.lattice()[2]) if is_tv(w) else w.n_sites


def n_occ(w) -> int:
    """Particles of one propagated species."""
    return w.n_particles if is_tv(w) else w.n_up


def batch(args, ns=None):
    """The workload of every chain of the batch (uneven: lattices drawn from
    {6, 8, 10, 12}^2 and U from [2, 6], half filling, Theta = 5)."""
    from paper_2303_13403_amd.workloads import TV_WORKLOADS, WORKLOADS, batch_uneven

    ns = args.ns if ns is None else ns
    if args.workload in TV_WORKLOADS:
        return [TV_WORKLOADS[args.workload].replace(stab_interval=ns, delay_rank=args.k)] * args.chains
    if args.workload == "uneven":
        return batch_uneven(args.chains, precision="fp64", stab_interval=ns, delay_rank=args.k)
    return [WORKLOADS[args.workload].replace(stab_interval=ns, delay_rank=args.k)] * args.chains


def describe(args, ws):
    w = ws[0]
    M = 2 * w.l_half
    if args.workload == "16x16":
        return (f"16x16 periodic Hubbard, U=3.5, 112+112 electrons, dtau=0.1, Theta=10 "
                f"(l_half=100, {M + 2} slices), Neel M_N=0.07 + Gutzwiller g=0.55, batch of "
                f"{len(ws)} chains")
    if args.workload == "uneven":
        sizes = sorted({x.lx for x in ws})
        return (f"batch of {len(ws)} independent half-filled chains, lattices L x L with L drawn "
                f"from {sizes}, U uniform in [2, 6], dtau={w.dtau}, Theta={w.dtau * w.l_half:g} "
                f"({M + 2} slices), Neel M_N={w.m_neel} + Gutzwiller g={w.g}")
    if is_tv(w):
        return (f"{w.name}, spinless, {w.n_particles} particles, {n_props(w)} bond fields per "
                f"slice, dtau={w.dtau}, {M + 2} slices, CDW trial Delta_C={w.delta_c} + bond "
                f"Gutzwiller g={w.g}, batch of {len(ws)} chains")
    return (f"{w.name}, {w.n_up}+{w.n_dn} electrons, dtau={w.dtau}, {M + 2} slices, Neel "
            f"M_N={w.m_neel} + Gutzwiller g={w.g}, batch of {len(ws)} chains")


def drift_stats(infos):
    rel = sorted(i["max_rel_drift"] if math.isfinite(i["max_rel_drift"]) else math.inf
                 for i in infos)
    n = len(rel)
    return {"max": finite_or_none(rel[-1]), "median": finite_or_none(rel[n // 2]),
            "p90": finite_or_none(rel[min(n - 1, (9 * n) // 10)]),
            "non_finite": sum(not math.isfinite(r) for r in rel),
            "frac_above_1e-5": sum(r > G_BOUND for r in rel) / n}


def run_gpu(args, precision_name, steps, warmup, ns=None):
    """Time `steps` sweeps of every chain after `warmup` unmeasured sweeps.
    The chains are split into args.groups contiguous groups, one context (and
    HIP stream) each, swept concurrently."""
    import numpy as np
    import torch

    from paper_2303_13403_amd import gpqmc

    prec = {"fp64": gpqmc.FP64, "fp64wrap": gpqmc.FP64_WRAP, "mixed": gpqmc.MIXED,
            "mixed32b": gpqmc.MIXED_FP32_BASIS}[precision_name]
    classes = CLASSES["fp64" if precision_name == "fp64" else "wrap"]
    ws = batch(args, ns)
    w = ws[0]
    G = args.groups
    if G < 1 or args.chains % G:
        raise SystemExit(f"--groups {G} must divide --chains {args.chains}")
    per = args.chains // G
    t0 = time.time()
    ctxs = []
    ph = args.particle_hole and precision_name == "fp64"
    for g in range(G):
        chains = [gpqmc.chain_desc_arrays(ws[g * per + c], g * per + c, prec) for c in range(per)]
        ctxs.append(gpqmc.Context(chains, device="cuda:0", meas_capacity=max(8, steps + 2),
                                  particle_hole=ph))
    for ctx in ctxs:
        ctx.init_trial()
    log(f"[{precision_name}] {G} context(s) + init_trial: {time.time() - t0:.1f} s, "
        f"workspace {sum(c.workspace_bytes for c in ctxs) / 2**30:.2f} GiB")
    # warm-up sweeps record nothing: the estimates below use the timed sweeps only
    for ctx in ctxs:
        ctx.sweep(warmup, measure=False)
    torch.cuda.synchronize()

    def all_infos():
        return [ctx.chain_info(c) for ctx in ctxs for c in range(per)]

    infos0 = all_infos()
    acc0 = sum(i["accepted"] for i in infos0)
    prop0 = sum(i["proposed"] for i in infos0)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = [torch.cuda.Event(enable_timing=True) for _ in ctxs]
    # HIP events around every launch of the timed kernel classes inside the
    # timed sweeps, on each context's stream
    for ctx in ctxs:
        ctx.set_kernel_timing(0 if args.no_kernel_timing else 7)
    torch.cuda.synchronize()

    def timed(n):
        torch.cuda.synchronize()
        ev0.record(ctxs[0].stream)
        for ctx in ctxs[1:]:
            ctx.stream.wait_event(ev0)
        w0 = time.time()
        for _ in range(n):                 # one sweep of every group at a time
            for ctx in ctxs:
                ctx.sweep(1, measure=True)
        for ctx, e in zip(ctxs, ev1):
            e.record(ctx.stream)
        torch.cuda.synchronize()
        return max(ev0.elapsed_time(e) for e in ev1), time.time() - w0

    ms, wall = timed(steps)
    kt = {}
    for k, name in enumerate(classes):
        parts = [ctx.kernel_timing(k) for ctx in ctxs]
        tot, n = sum(t for t, _ in parts), sum(n for _, n in parts)
        kt[name] = {"ms_per_launch": tot / max(n, 1), "launches": n, "ms_total": tot}
    for ctx in ctxs:
        ctx.set_kernel_timing(0)
    infos = all_infos()
    acc = sum(i["accepted"] for i in infos) - acc0
    prop = sum(i["proposed"] for i in infos) - prop0
    n_updates = (2 * w.l_half + 2) * sum(n_props(x) for x in ws) * steps
    assert prop == n_updates, (prop, n_updates)
    # estimates from the timed sweeps' records, pooled with a delete-one-chain
    # jackknife over the chains without a NaN, singular or sign-mismatch flag
    # (the drift flag alone is reported, not excluded)
    recs, n_flagged = [], 0
    for ctx in ctxs:
        for c in range(per):
            if ctx.chain_info(c)["flags"] & FLAGGED:
                n_flagged += 1
                continue
            recs.append(ctx.measurements(c))
    est = {}
    for name, col in (("sign", 0), ("energy_per_site", 1), ("double_occupancy", 2),
                      ("structure_factor", 3)):
        e = pooled_over_chains(recs, col) if recs else None
        est[name] = None if e is None else [e[0], e[1]]
    res = dict(ms=ms, wall=wall, updates=n_updates, accept=acc / max(prop, 1),
               rel_drift=drift_stats(infos), flags=sorted({i["flags"] for i in infos}),
               n_flagged=n_flagged, sign_mismatch=sum(i["sign_mismatch"] for i in infos),
               kernels=kt, estimates=est, stab_interval=w.stab_interval, delay_rank=w.delay_rank,
               spins=[1 if (i["particle_hole"] or is_tv(w)) else 2 for i in infos],
               n_particle_hole=sum(i["particle_hole"] for i in infos))
    log(f"[{precision_name}] {steps} sweeps: {ms:.1f} ms (wall {wall * 1e3:.1f} ms), "
        f"{n_updates / (ms / 1e3):.4g} updates/s, acceptance {res['accept']:.3f}, "
        f"kernels {json.dumps({k: round(v['ms_per_launch'], 4) for k, v in kt.items()})} ms/launch, "
        f"relative drift {res['rel_drift']}, flags {res['flags']}, flagged chains {n_flagged}")
    for ctx in ctxs:
        ctx.close()
    del ctxs
    torch.cuda.empty_cache()
    return res


# --------------------------------------------------------------------------- #
# the oracle on the host cores
# --------------------------------------------------------------------------- #
def _oracle_worker(job):
    """One oracle chain of the workload: time one sweep after initialisation
    (BLAS on one thread).  Runs in a fresh process."""
    w, chain_id = job
    from threadpoolctl import threadpool_limits

    from oracle import pqmc, tv

    with threadpool_limits(limits=1):
        if is_tv(w):
            ch = tv.TVChain(tv.TVModel.from_workload(w), seed=w.seed, chain_id=chain_id)
        else:
            ch = pqmc.Chain(pqmc.Model.from_workload(w), seed=w.seed, chain_id=chain_id)
        t0 = time.time()
        ch.sweep(1, measure=True)
        dt = time.time() - t0
    return (2 * w.l_half + 2) * n_props(w), dt


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(args):
    """The oracle (serial FP64 NumPy) on the host: one independent chain per
    core, one sweep each, run concurrently in fresh processes; the aggregate
    rate is the sum of the per-chain rates (wall time per process)."""
    import multiprocessing as mp

    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    cores = max(1, min(avail, args.cpu_cores))
    ws = batch(args)
    w = ws[0]
    jobs = [(ws[c % len(ws)], c) for c in range(cores)]
    t0 = time.time()
    with mp.get_context("spawn").Pool(cores) as pool:
        out = pool.map(_oracle_worker, jobs)
    wall = time.time() - t0
    rates = [u / dt for u, dt in out]
    return {"value": sum(rates), "unit": UNIT, "cores": cores, "kind": "oracle",
            "per_core": sum(rates) / len(rates),
            "cpu_model": cpu_model(), "host_cpus_visible": avail,
            "sample": f"{cores} independent chains of the {describe(args, ws)} workload "
                      f"(chain ids 0..{cores - 1}), one sweep each ({2 * w.l_half + 2} slices x "
                      f"the chain's sites) after "
                      f"initialisation, one process per core, serial FP64 NumPy with BLAS threads = 1; "
                      f"{wall:.1f} s wall"}


def copy_calibration(mib: int, reps: int = 5):
    """Device-to-device copies of a known size: the FETCH_SIZE / WRITE_SIZE
    counters of these dispatches give the scale of the counters in bytes."""
    import torch

    n = mib * 2 ** 20 // 4
    src = torch.rand(n, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": n * 4, "reps": reps}), flush=True)


def leg_summary(res):
    value = res["updates"] / (res["ms"] / 1e3)
    rd = res["rel_drift"]
    return {"value": value, "unit": UNIT, "ms_per_step": res["ms"] / res.get("steps", 1),
            "stab_interval": res["stab_interval"], "delay_rank": res["delay_rank"],
            "acceptance": round(res["accept"], 4), "rel_drift": rd,
            "holds_1e-5": rd["frac_above_1e-5"] == 0.0 and rd["non_finite"] == 0,
            "flags": res["flags"], "n_flagged": res["n_flagged"],
            "kernels_ms_per_launch": {k: v["ms_per_launch"] for k, v in res["kernels"].items()},
            **res["estimates"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=6)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--chains", type=int, default=None,
                    help="chains in the batch (default 2048; 512 at 24x24; 256 for uneven)")
    ap.add_argument("--workload", default="16x16",
                    choices=["16x16", "honeycomb12x12", "12x12", "24x24", "uneven", "tv15_V1.6",
                             "tv15_V1.35", "tv6"],
                    help="16x16: the headline configuration; 12x12: the half-filled 12x12 "
                         "lattice; 24x24: N = 576 at dtau = 0.05, Theta = 10; uneven: 256 chains "
                         "on 6x6 .. 12x12 with U in [2, 6]; honeycomb12x12: the paper's lattice "
                         "at 288 sites; tv15_V1.6 / tv15_V1.35: the spinless t-V model on the "
                         "15x15-cell honeycomb lattice (450 sites)")
    ap.add_argument("--no-kernel-timing", action="store_true",
                    help="time the sweeps as captured HIP graphs, without the in-sweep kernel "
                         "events (no roofline block)")
    ap.add_argument("--particle-hole", action="store_true",
                    help="the half-filling particle-hole shortcut (spin up only) wherever exact")
    ap.add_argument("--groups", type=int, default=1,
                    help="chain groups, one context and HIP stream each, swept concurrently")
    ap.add_argument("--ns", type=int, default=None,
                    help="stabilisation interval (default 10; 5 for the t-V workloads, whose drift "
                         "at 10 passes the 1e-5 bound)")
    ap.add_argument("--k", type=int, default=32)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp64wrap", "mixed", "mixed32b"])
    ap.add_argument("--leg-steps", type=int, default=2,
                    help="sweeps of each comparison leg (FP64 wrap, mixed); 0 = skip the legs")
    ap.add_argument("--wrap-ns", type=int, default=10,
                    help="stabilisation interval of the FP64 wrap leg")
    ap.add_argument("--mixed-ns", type=int, default=5,
                    help="stabilisation interval of the mixed leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-cores", type=int, default=16,
                    help="host cores for the oracle leg (one chain each; capped by the visible CPUs)")
    ap.add_argument("--autotune", action="store_true",
                    help="choose --k and --ns with the autotuner on this batch first (table on stderr)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run device-to-device copies of MIB MiB (the reference kernel for "
                         "scaling the HBM traffic counters) and exit")
    args = ap.parse_args()
    if args.chains is None:
        args.chains = DEFAULT_CHAINS[args.workload]
    if args.ns is None:
        args.ns = 5 if args.workload.startswith("tv") else 10
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (--gpus {args.gpus} requested): the chains of a "
              "multi-GPU run are independent, so a node's throughput is N times one GPU's.",
              file=sys.stderr)
        sys.exit(2)
    # the oracle leg runs first, in fresh processes, before this process
    # touches the GPU
    cpu = None
    if not args.no_cpu_baseline and not args.copy_calibration:
        cpu = cpu_baseline(args)
        log(f"[cpu] oracle on {cpu['cores']} cores ({cpu['cpu_model']}): {cpu['value']:.4g} updates/s")
    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)

    if args.copy_calibration > 0:
        copy_calibration(args.copy_calibration)
        return
    if args.autotune:
        from paper_2303_13403_amd import gpqmc
        from paper_2303_13403_amd.autotune import autotune

        prec = {"mixed": gpqmc.MIXED, "fp64": gpqmc.FP64, "fp64wrap": gpqmc.FP64_WRAP,
                "mixed32b": gpqmc.MIXED_FP32_BASIS}[args.precision]
        best, _ = autotune(batch(args), prec, delay_ranks=(8, 16, 32),
                           stab_intervals=(5, 10, 20), log=log)
        args.k, args.ns = best.delay_rank, best.stab_interval
        log(f"autotune: k={args.k} n_s={args.ns}")
    ws = batch(args)
    w = ws[0]
    M = 2 * w.l_half
    main_res = run_gpu(args, args.precision, args.steps, args.warmup)
    main_res["steps"] = args.steps
    legs = {}
    if args.leg_steps > 0 and not is_tv(w):      # the t-V model runs on the factored engine only
        for name, prec, ns in (("fp64_wrap_gpu", "fp64wrap", args.wrap_ns),
                               ("mixed_gpu", "mixed", args.mixed_ns)):
            if prec == args.precision:
                continue
            r = run_gpu(args, prec, args.leg_steps, 1, ns=ns)
            r["steps"] = args.leg_steps
            legs[name] = leg_summary(r)

    value = main_res["updates"] / (main_res["ms"] / 1e3)
    per_launch = args.chains // args.groups
    kt = main_res["kernels"]
    rooflines = []
    spins = main_res["spins"]
    grp = ws[:per_launch]                  # the chains one launch covers
    if args.precision == "fp64" and not args.no_kernel_timing:
        # segment update Q <- Q - (Q Mf^T) Wf, bound by HBM: algorithmic bytes
        # per chain and spin = Q read and written (2 N n doubles) + Mf and Wf
        # read (2 f n doubles), f = the mean accepted flips of a segment; the
        # same launch forms the next segment's block (all but the last segment
        # of a slice): its k rows of both factors read (2 k n doubles) and the
        # k x k block written.  A chain takes part in ceil(N / k) of the
        # ceil(N_max / k) launches of a slice (spin up only with the
        # particle-hole shortcut)
        f_mean = main_res["accept"] * args.k
        def segs(x):   # scan segments per slice: k sites, or k / 2 bonds (t-V)
            return math.ceil(n_props(x) / (args.k // 2)) if is_tv(x) else math.ceil(x.n_sites / args.k)
        n_seg = max(segs(x) for x in grp)
        seg_bytes = sum(spins[c] * 8.0 *
                        (segs(x) * (2 * x.n_sites * n_occ(x) + 2 * f_mean * n_occ(x))
                         + (segs(x) - 1) * (2 * args.k * n_occ(x) + args.k ** 2))
                        for c, x in enumerate(grp)) / n_seg
        seg_ms = kt["segment_update"]["ms_per_launch"]
        seg_ach = seg_bytes / (seg_ms / 1e3)
        rooflines.append({"bound": "hbm", "achieved": seg_ach / 1e9, "peak": PEAK_HBM / 1e9,
                          "unit": "GB/s", "frac": seg_ach / PEAK_HBM,
                          "traffic": None if args.particle_hole else
                          read_traffic(per_launch, args.precision, args.workload),
                          "kernel": "k_segupd_f (Q <- Q - (Q Mf^T) Wf and the next segment's "
                                    "block, every chain and spin)"
                                    if max(n_occ(x) for x in ws) <= 128 else
                                    "k_gemm SEGP + SEGF (Q Mf^T, then Q - (Q Mf^T) Wf)",
                          "bytes_per_launch": seg_bytes, "ms_per_launch": seg_ms,
                          "ms_total": kt["segment_update"]["ms_total"],
                          "timing": f"HIP events on the context's stream around each of the "
                                    f"{kt['segment_update']['launches']} launches in the timed sweeps"})
        # propagation of both factors, FP64 MFMA: 2 N^2 n flops per factor,
        # chain and spin
        prop_flops = sum(spins[c] * 2 * 2.0 * x.n_sites ** 2 * n_occ(x) for c, x in enumerate(grp))
        prop_ms = kt["propagation"]["ms_per_launch"]
        prop_ach = prop_flops / (prop_ms / 1e3)
        rooflines.append({"bound": "mfma", "achieved": prop_ach / 1e12, "peak": PEAK_FP64_MFMA / 1e12,
                          "unit": "TFLOP/s", "frac": prop_ach / PEAK_FP64_MFMA, "traffic": None,
                          "kernel": "k_prop (A <- D e^{-+dtau K} A, B likewise; "
                                    "every chain and spin x 2 factors)",
                          "flops_per_launch": prop_flops, "ms_per_launch": prop_ms,
                          "ms_total": kt["propagation"]["ms_total"],
                          "timing": f"HIP events around each of the {kt['propagation']['launches']} "
                                    f"launches in the timed sweeps"})
        rooflines.sort(key=lambda r: -r["ms_total"])
    out = {
        "metric": METRIC if args.workload == "16x16" else f"HS-field updates/sec, {describe(args, ws)}",
        "value": value, "unit": UNIT, "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": main_res["ms"] / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision in ("fp64", "fp64wrap") else "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": describe(args, ws),
            "chains": args.chains, "chain_groups": args.groups,
            "particle_hole_chains": main_res["n_particle_hole"],
            "precision": {"fp64": "fp64, factored G = 1 - A B^T",
                          "fp64wrap": "fp64, G wrapped as N x N",
                          "mixed": "FP32 G, FP64 bases and checkpoints",
                          "mixed32b": "FP32 G and bases"}[args.precision],
            "stab_interval": args.ns, "delay_rank": args.k,
            "acceptance": round(main_res["accept"], 4),
            "rel_drift": main_res["rel_drift"],
            "holds_1e-5": main_res["rel_drift"]["frac_above_1e-5"] == 0.0
                          and main_res["rel_drift"]["non_finite"] == 0,
            "flags": main_res["flags"], "n_flagged": main_res["n_flagged"],
            "estimates_from": f"the {args.steps} timed sweeps (warm-up sweeps record nothing), "
                              f"pooled over the chains without a NaN, singular or sign-mismatch "
                              f"flag, delete-one-chain jackknife",
            **main_res["estimates"],
        },
        "kernels_ms_per_launch": {k: v["ms_per_launch"] for k, v in kt.items()},
        "kernel_launches": {k: v["launches"] for k, v in kt.items()},
        "launch": (f"{args.groups} chain groups of {args.chains // args.groups}, one context and "
                   f"HIP stream each, swept concurrently; " if args.groups > 1 else
                   "one context; ") + ("each pass replayed as a captured HIP graph"
                                       if args.no_kernel_timing else
                                       "direct launches (kernel events in the timed sweeps)"),
    }
    if rooflines:
        out["roofline"] = rooflines[0]
        out["roofline_2"] = rooflines[1]
    out.update(legs)
    if "fp64_wrap_gpu" in legs:
        out["speedup_over_fp64_wrap"] = value / legs["fp64_wrap_gpu"]["value"]
    if "mixed_gpu" in legs:
        out["mixed_over_this"] = legs["mixed_gpu"]["value"] / value
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
