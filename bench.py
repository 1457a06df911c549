"""Throughput benchmark of the Gutzwiller-projection PQMC sweep on one MI355X.

Workload (the configuration the headline metric is quoted on): 16x16 periodic
Hubbard model, t = 1, U = 3.5, 112 + 112 electrons (<n> = 0.875), dtau = 0.1,
Theta = 10 (l_half = 100 slices per side, M + 2 = 202 slices), Neel trial
M_N = 0.07 with Gutzwiller g = 0.55 and the trial-only shell-closing ramp,
mixed precision (FP32-MFMA Green's-function work, FP64 bases and
stabilisation), a batch of independent chains.

One step = one sweep (one pass over all 202 slices) of every chain of the
batch; value = HS-field updates (proposals) per second over the timed steps,
inputs resident in HBM.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--chains B] [--gpus 1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2303_13403_amd.estimators import weighted_mean  # noqa: E402

METRIC = "HS-field updates/sec at 16×16, L=100; mixed vs FP64 GPU at 1e-5 rel G error"
UNIT = "HS-field updates/s"
PEAK_FP32_MFMA = 157.3e12   # MI355X dense FP32 matrix, FLOP/s
PEAK_FP64_MFMA = 78.6e12
PEAK_HBM = 8.0e12           # MI355X HBM3E, B/s
# the dominant kernel (largest share of the sweep): the large-tile MFMA GEMM of
# the kinetic wrap and the slice update; the roofline is taken on its wrap launch
KERNEL_SRC = os.path.join(ROOT, "paper_2303_13403_amd", "csrc", "gpqmc_gemm.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_wrap_gemm_16x16_b2048.txt")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_sha() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def read_traffic(chains_per_launch: int, precision: str):
    """HBM bytes per launch of the wrap GEMM from the committed PMC summary, if
    it was taken on the current kernel source, launch size and precision."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if (kv.get("kernel_source_sha") != kernel_sha()
            or int(kv.get("chains_per_launch", -1)) != chains_per_launch
            or kv.get("precision") != precision):
        return None
    return float(kv["hbm_bytes_per_launch"])


def workload(args, ns=None):
    from paper_2303_13403_amd.workloads import WORKLOADS

    return WORKLOADS[args.workload].replace(stab_interval=args.ns if ns is None else ns,
                                      delay_rank=args.k)


def run_gpu(args, precision_name, steps, warmup, ns=None):
    """Time `steps` sweeps of every chain.  The chains are split into
    args.groups contiguous groups, one context (and HIP stream) each, swept
    concurrently: the latency-bound scan and append launches of one group
    overlap the MFMA GEMMs of another."""
    import numpy as np
    import torch

    from paper_2303_13403_amd import gpqmc

    prec = {"mixed": gpqmc.MIXED, "fp64": gpqmc.FP64, "mixed32b": gpqmc.MIXED_FP32_BASIS}[precision_name]
    w = workload(args, ns)
    G = args.groups
    if G < 1 or args.chains % G:
        raise SystemExit(f"--groups {G} must divide --chains {args.chains}")
    per = args.chains // G
    t0 = time.time()
    ctxs = []
    for g in range(G):
        chains = [gpqmc.chain_desc_arrays(w, g * per + c, prec) for c in range(per)]
        ctxs.append(gpqmc.Context(chains, device="cuda:0", meas_capacity=max(64, steps + warmup + 4)))
    for ctx in ctxs:
        ctx.init_trial()
    log(f"[{precision_name}] {G} context(s) + init_trial: {time.time() - t0:.1f} s, "
        f"workspace {sum(c.workspace_bytes for c in ctxs) / 2**30:.2f} GiB")
    for ctx in ctxs:
        ctx.sweep(warmup, measure=True)
    torch.cuda.synchronize()
    log(f"[{precision_name}] warmup {warmup} sweeps done")

    def all_infos():
        return [ctx.chain_info(c) for ctx in ctxs for c in range(per)]

    infos0 = all_infos()
    acc0 = sum(i["accepted"] for i in infos0)
    prop0 = sum(i["proposed"] for i in infos0)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = [torch.cuda.Event(enable_timing=True) for _ in ctxs]
    # HIP events around every launch of the wrap, propagation and slice-update
    # GEMMs inside the timed sweeps (on each context's stream)
    for ctx in ctxs:
        ctx.set_kernel_timing(7)
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
    kt = []
    for k in range(3):
        parts = [ctx.kernel_timing(k) for ctx in ctxs]
        kt.append((sum(t for t, _ in parts), sum(n for _, n in parts)))
    for ctx in ctxs:
        ctx.set_kernel_timing(0)
    infos = all_infos()
    graph_ms = timed(steps)[0] if args.graph_check else None
    acc = sum(i["accepted"] for i in infos) - acc0
    prop = sum(i["proposed"] for i in infos) - prop0
    n_updates = (2 * w.l_half + 2) * w.n_sites * args.chains * steps
    assert prop == n_updates, (prop, n_updates)
    wrap_ms, prop_ms, flush_ms = (t / max(n, 1) for t, n in kt)
    launches = {"wrap": kt[0][1], "prop": kt[1][1], "slice_update": kt[2][1]}
    rel = sorted(i["max_rel_drift"] for i in infos)
    energy = sign = saf = None
    if args.chains * (steps + warmup) >= 20:
        rec = np.concatenate([ctx.measurements(c) for ctx in ctxs for c in range(per)])
        energy, sign = weighted_mean(rec, 1), weighted_mean(rec, 0)
        saf = weighted_mean(rec, 3)
    res = dict(ms=ms, wall=wall, updates=n_updates, accept=acc / max(prop, 1),
               max_drift=max(i["max_drift"] for i in infos),
               rel_drift={"max": rel[-1], "median": rel[len(rel) // 2],
                          "p90": rel[min(len(rel) - 1, (9 * len(rel)) // 10)],
                          "frac_above_1e-5": sum(r > 1e-5 for r in rel) / len(rel)},
               flags=sorted({i["flags"] for i in infos}),
               sign_mismatch=sum(i["sign_mismatch"] for i in infos),
               wrap_ms=wrap_ms, prop_ms=prop_ms, flush_ms=flush_ms, launches=launches,
               graph_ms=graph_ms, sign=sign, energy=energy, structure_factor=saf)
    log(f"[{precision_name}] {steps} sweeps: {ms:.1f} ms (wall {wall * 1e3:.1f} ms), "
        f"{n_updates / (ms / 1e3):.4g} updates/s, acceptance {res['accept']:.3f}, "
        f"slice update {flush_ms:.3f} ms/launch, wrap GEMM {wrap_ms:.3f} ms/launch, "
        f"max drift {res['max_drift']:.2e}, relative drift over chains {res['rel_drift']}, "
        f"flags {res['flags']}")
    for ctx in ctxs:
        ctx.close()
    del ctxs
    torch.cuda.empty_cache()
    return res


def cpu_baseline(args, budget_s=30.0):
    """The oracle on the host: one chain of the same workload, BLAS on one
    thread, timed over whole sweeps after its initialisation."""
    from threadpoolctl import threadpool_limits

    from oracle import pqmc

    w = workload(args)
    with threadpool_limits(limits=1):
        ch = pqmc.Chain(pqmc.Model.from_workload(w), seed=w.seed, chain_id=0)
        t0 = time.time()
        n = 0
        while True:
            ch.sweep(1, measure=True)
            n += 1
            if time.time() - t0 > budget_s / 3 or n >= 3:
                break
        dt = time.time() - t0
    upd = (2 * w.l_half + 2) * w.n_sites * n
    return {"value": upd / dt, "unit": UNIT, "cores": 1, "kind": "oracle",
            "sample": f"{n} sweep(s) of one {w.name} chain ({2 * w.l_half + 2} slices x "
                      f"{w.n_sites} sites), serial FP64 NumPy, BLAS threads = 1, {dt:.1f} s"}


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=6)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--chains", type=int, default=2048)
    ap.add_argument("--workload", default="16x16", choices=["16x16", "honeycomb12x12"],
                    help="16x16: the headline configuration; honeycomb12x12: the paper's "
                         "lattice at 288 sites")
    ap.add_argument("--groups", type=int, default=1,
                    help="chain groups, one context and HIP stream each, swept concurrently "
                         "(the roofline kernel's launches then overlap other groups' work)")
    ap.add_argument("--ns", type=int, default=5)
    ap.add_argument("--k", type=int, default=32)
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64", "mixed32b"])
    ap.add_argument("--fp64-steps", type=int, default=2,
                    help="sweeps of the plain FP64 GPU path timed for comparison (0 = skip)")
    ap.add_argument("--fp64-ns", type=int, default=10,
                    help="stabilisation interval of the FP64 comparison (its relative drift "
                         "stays below 1e-6 at 10 on this workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--graph-check", action="store_true",
                    help="also time the same number of sweeps launched as HIP graphs")
    ap.add_argument("--autotune", action="store_true",
                    help="choose --k and --ns with the autotuner on this batch first (table on stderr)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run device-to-device copies of MIB MiB (the reference kernel for "
                         "scaling the HBM traffic counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (--gpus {args.gpus} requested): the chains of a "
              "multi-GPU run are independent, so a node's throughput is N times one GPU's.",
              file=sys.stderr)
        sys.exit(2)
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

        prec = {"mixed": gpqmc.MIXED, "fp64": gpqmc.FP64, "mixed32b": gpqmc.MIXED_FP32_BASIS}[args.precision]
        best, _ = autotune([workload(args)] * args.chains, prec, delay_ranks=(16, 32, 64),
                           stab_intervals=(5, 10, 20), log=log)
        args.k, args.ns = best.delay_rank, best.stab_interval
        log(f"autotune: k={args.k} n_s={args.ns}")
    w = workload(args)
    N, M = w.n_sites, 2 * w.l_half
    main_res = run_gpu(args, args.precision, args.steps, args.warmup)
    fp64_res = None
    if args.fp64_steps > 0 and args.precision != "fp64":
        fp64_res = run_gpu(args, "fp64", args.fp64_steps, 1, ns=args.fp64_ns)

    value = main_res["updates"] / (main_res["ms"] / 1e3)
    # dominant kernel: the kinetic-wrap GEMM Gtmp = e^{-dtau K} G, MFMA-bound;
    # algorithmic flops per launch = every chain of the group x 2 spins x 2 N^3
    per_launch = args.chains // args.groups
    wrap_flops = 2.0 * per_launch * 2.0 * N ** 3
    peak = PEAK_FP32_MFMA if args.precision != "fp64" else PEAK_FP64_MFMA
    achieved = wrap_flops / (main_res["wrap_ms"] / 1e3)
    traffic = read_traffic(per_launch, args.precision)
    out = {
        "metric": METRIC if args.workload == "16x16" else f"HS-field updates/sec, {w.name}",
        "value": value, "unit": UNIT, "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": main_res["ms"] / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": (f"16x16 periodic Hubbard, U=3.5, 112+112 electrons, dtau=0.1, "
                         f"Theta=10 (l_half=100, {M + 2} slices), Neel M_N=0.07 + Gutzwiller "
                         f"g=0.55, batch of {args.chains} chains" if args.workload == "16x16" else
                         f"{w.name}, {w.n_up}+{w.n_dn} electrons, dtau={w.dtau}, "
                         f"{M + 2} slices, Neel M_N={w.m_neel} + Gutzwiller g={w.g}, "
                         f"batch of {args.chains} chains"),
            "chains": args.chains, "chain_groups": args.groups,
            "precision": args.precision, "stab_interval": args.ns,
            "delay_rank": args.k, "acceptance": round(main_res["accept"], 4),
            "max_drift": main_res["max_drift"], "rel_drift": main_res["rel_drift"],
            "flags": main_res["flags"], "energy_per_site": main_res["energy"],
            "structure_factor": main_res["structure_factor"], "sign": main_res["sign"],
        },
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": peak / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / peak, "traffic": traffic,
                     "kernel": ("k_gemm_l STORE (e^{-dtau K} G, " if args.precision != "fp64" else
                                "k_gemm<double> STORE (e^{-dtau K} G, ") +
                               ("every chain x 2 spins" if args.groups == 1 else
                                "every chain of a group x 2 spins") +
                               ("; 128x128 MFMA tiles)" if args.precision != "fp64" else ")"),
                     "flops_per_launch": wrap_flops, "ms_per_launch": main_res["wrap_ms"],
                     "timing": f"HIP events on the context's stream around each of the "
                               f"{main_res['launches']['wrap']} launches in the timed sweeps" +
                               (f" ({args.groups} chain groups running concurrently)"
                                if args.groups > 1 else "")},
        "slice_update_gemm_ms": main_res["flush_ms"],
        "propagation_gemm_ms": main_res["prop_ms"],
        "launch": (f"{args.groups} chain groups of {args.chains // args.groups}, one context and "
                   f"HIP stream each, swept concurrently; " if args.groups > 1 else
                   "one context; ") + "direct launches (kernel events in the timed sweeps)",
    }
    if main_res["graph_ms"] is not None:
        out["graph_ms_per_step"] = main_res["graph_ms"] / args.steps
    if fp64_res is not None:
        out["fp64_gpu"] = {"value": fp64_res["updates"] / (fp64_res["ms"] / 1e3), "unit": UNIT,
                           "steps": args.fp64_steps, "stab_interval": args.fp64_ns,
                           "wrap_gemm_ms_per_launch": fp64_res["wrap_ms"],
                           "rel_drift": fp64_res["rel_drift"], "energy_per_site": fp64_res["energy"]}
        out["mixed_over_fp64"] = value / out["fp64_gpu"]["value"]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
