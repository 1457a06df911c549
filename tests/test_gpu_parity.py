"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

* MFMA tile GEMM against a float64 CPU product (ragged shapes, transposed A);
* initial field (Philox) bit-exact; Green's function after init_trial;
* fixed field (every proposal rejected): ratios of every proposal and the
  fresh Green's functions at every checkpoint of an upward and a downward pass;
* Markov trajectories with shared Philox streams: fields bit-exact except for
  draws within the tie tolerance of their threshold (follow mode), and the
  measured (sign, E/N, D) of every pass;
* uneven batch, determinism, and a sampled chain of the 16x16 benchmark batch.
Tolerances: max|x - x_ref| / max|x_ref| <= 1e-10 (FP64) or 1e-5 (mixed).
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from gpu_helpers import (TIE, TOL, is_fp64, make_context, oracle_chain, oracle_fixed_pass, ratio_array,
                         rel_err)
from oracle import philox, pqmc
from paper_2303_13403_amd import gpqmc
from paper_2303_13403_amd.workloads import WORKLOADS, Workload, batch_uneven


def small(prec="fp64", L=4, l_half=6, n_s=3, k=8, U=4.0, n=None, **kw):
    n = L * L // 2 if n is None else n
    return Workload(f"{L}x{L} test", L, L, U, n, n, 0.1, l_half, 0.21, 0.6, n_s, k, prec, 10, **kw)


# --------------------------------------------------------------------------- #
# MFMA GEMM tile kernel
# --------------------------------------------------------------------------- #
@pytest.mark.parametrize("prec", [gpqmc.FP64, gpqmc.MIXED])
@pytest.mark.parametrize("shape", [(64, 64, 64), (100, 70, 37), (1, 129, 5), (144, 72, 144)])
@pytest.mark.parametrize("trans", [False, True])
def test_mfma_gemm_matches_cpu(prec, shape, trans):
    M, N, K = shape
    g = torch.Generator().manual_seed(M * 7 + N * 3 + K)
    A = torch.randn((K, M) if trans else (M, K), generator=g, dtype=torch.float64)
    B = torch.randn((K, N), generator=g, dtype=torch.float64)
    dt = torch.float64 if prec == gpqmc.FP64 else torch.float32
    A, B = A.to(dt).to(torch.float64), B.to(dt).to(torch.float64)
    ref = (A.T if trans else A) @ B
    C = gpqmc.debug_gemm(A.cuda(), B.cuda(), trans_a=trans, precision=prec).cpu().to(torch.float64)
    tol = 1e-13 if prec == gpqmc.FP64 else 2e-6
    assert rel_err(C.numpy(), ref.numpy()) < tol


@pytest.mark.parametrize("shape", [(256, 256, 256), (128, 128, 1), (144, 72, 144),
                                   (300, 130, 37), (257, 255, 33), (36, 36, 36)])
def test_large_tile_fp32_gemm_matches_cpu(shape):
    """The kinetic wrap's 128 x 128 FP32 kernel: whole, ragged and thin tiles,
    k not a multiple of its k-tile."""
    M, N, K = shape
    g = torch.Generator().manual_seed(M * 5 + N * 11 + K)
    A = torch.randn((M, K), generator=g, dtype=torch.float64).to(torch.float32).to(torch.float64)
    B = torch.randn((K, N), generator=g, dtype=torch.float64).to(torch.float32).to(torch.float64)
    C = gpqmc.debug_gemm(A.cuda(), B.cuda(), precision=gpqmc.MIXED, large_tile=True).cpu()
    assert rel_err(C.to(torch.float64).numpy(), (A @ B).numpy()) < 2e-6


@pytest.mark.parametrize("shape", [(256, 256, 256), (128, 128, 1), (144, 72, 144),
                                   (300, 130, 37), (257, 255, 33), (256, 112, 256)])
def test_large_tile_fp64_gemm_matches_cpu(shape):
    """The 128 x 128 FP64 kernel of the FP64 wrap, slice update and basis
    propagation: whole, ragged and thin tiles, odd leading dimensions (the
    unaligned load path) and k not a multiple of its k-tile."""
    M, N, K = shape
    g = torch.Generator().manual_seed(M * 13 + N * 5 + K)
    A = torch.randn((M, K), generator=g, dtype=torch.float64)
    B = torch.randn((K, N), generator=g, dtype=torch.float64)
    C = gpqmc.debug_gemm(A.cuda(), B.cuda(), precision=gpqmc.FP64, large_tile=True).cpu()
    assert rel_err(C.numpy(), (A @ B).numpy()) < 1e-13


# --------------------------------------------------------------------------- #
# initialisation
# --------------------------------------------------------------------------- #
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("L,l_half,n_s", [(4, 6, 3), (6, 5, 4)])
def test_init_field_and_green(prec, L, l_half, n_s):
    w = small(prec, L=L, l_half=l_half, n_s=n_s)
    ctx = make_context([w], prec).init_trial()
    ch = oracle_chain(w, 0)
    assert np.array_equal(ctx.get_field(0), ch.field)
    for s, sp in ((1, 0), (-1, 1)):
        assert rel_err(ctx.get_green(0, sp), ch.G[s]) < TOL[prec]
    info = ctx.chain_info(0)
    assert info["sign"] == ch.sign and info["flags"] == 0
    ctx.close()


# --------------------------------------------------------------------------- #
# fixed field: every ratio and every checkpoint Green's function of a pass
# --------------------------------------------------------------------------- #
FIXED = [
    ("fp64", dict(L=4, l_half=6, n_s=3, k=8)),
    ("fp64", dict(L=6, l_half=5, n_s=4, k=16)),            # N = 36: ragged tiles
    ("fp64", dict(L=12, l_half=50, n_s=10, k=32)),         # the 12x12 workload
    ("mixed", dict(L=4, l_half=6, n_s=3, k=8)),
    ("mixed", dict(L=6, l_half=5, n_s=4, k=16)),
    ("mixed", dict(L=12, l_half=50, n_s=4, k=32)),      # FP32 wrap needs n_s ~ 4 at dtau 0.1
    ("mixed32b", dict(L=4, l_half=6, n_s=3, k=8)),
    ("mixed32b", dict(L=12, l_half=50, n_s=3, k=32)),
    ("fp64", dict(L=4, l_half=5, n_s=3, k=5, U=3.0, n=5, ramp=0.05)),   # doped
    ("fp64", dict(L=6, l_half=4, n_s=2, k=40)),                          # two scan blocks per segment
    ("fp64", dict(L=4, l_half=0, n_s=1, k=8)),                          # boundary slices only
    ("fp64wrap", dict(L=4, l_half=6, n_s=3, k=8)),
    ("fp64wrap", dict(L=12, l_half=50, n_s=10, k=32)),
    ("fp64wrap", dict(L=4, l_half=5, n_s=3, k=5, U=3.0, n=5, ramp=0.05)),
]


LOGDET_TOL = {"fp64": 1e-10, "fp64wrap": 1e-10, "mixed": 1e-7, "mixed32b": 1e-5}


def check_fixed_field(w, prec, **ctx_kw):
    ctx = make_context([w], prec, trace=True, **ctx_kw).init_trial()
    ctx.set_debug(True)
    if ctx_kw.get("particle_hole"):
        assert ctx.chain_info(0)["particle_hole"] == 1
    ch = oracle_chain(w, 0)
    N = w.n_sites
    for sweep in range(2):                     # one upward and one downward pass
        ctx.sweep(1, measure=False)
        oracle_fixed_pass(ch)
        r_gpu, g_gpu, d_gpu = ctx.trace(0)
        ld_gpu = ctx.trace_logdet(0)
        r_ref = ratio_array(ch, sweep, ch.m.n_slices, N)
        assert rel_err(r_gpu, r_ref) < TOL[prec], f"ratios, sweep {sweep}"
        assert len(ch.checkpoint_greens) == g_gpu.shape[0]
        for k, (sw, p, gu, gd, drift, field) in enumerate(ch.checkpoint_greens):
            assert rel_err(g_gpu[k, 0], gu) < TOL[prec], f"G_up at p={p}, sweep {sweep}"
            assert rel_err(g_gpu[k, 1], gd) < TOL[prec], f"G_dn at p={p}, sweep {sweep}"
        # log|W_sigma| and its sign at every checkpoint: FP64 bookkeeping in
        # every precision (relative to max(1, |log W|)); the FP32-basis variant
        # factorises FP32-propagated bases, whose rounding enters log|det T|
        assert len(ch.checkpoint_logdets) == ld_gpu.shape[0]
        for k, (sw, p, ld) in enumerate(ch.checkpoint_logdets):
            for sp, s in ((0, 1), (1, -1)):
                la, sg = ld[s]
                assert ld_gpu[k, sp, 1] == sg, f"sign of W at p={p}"
                assert abs(ld_gpu[k, sp, 0] - la) < LOGDET_TOL[prec] * max(1.0, abs(la)), \
                    f"log|W| at p={p}: {ld_gpu[k, sp, 0]} vs {la}"
        assert np.max(d_gpu) < (1e-8 if is_fp64(prec) else 1e-3)
        print(f"{prec} {w.name}: sweep {sweep}: max ratio err {rel_err(r_gpu, r_ref):.2e}, "
              f"max G err {max(rel_err(g_gpu[k, s], g[2 + s]) for k, g in enumerate(ch.checkpoint_greens) for s in (0, 1)):.2e}, "
              f"max drift {np.max(d_gpu):.2e}")
    assert np.array_equal(ctx.get_field(0), ch.field)
    ctx.close()


@pytest.mark.parametrize("prec,kw", FIXED)
def test_fixed_field_pass_matches_oracle(prec, kw):
    check_fixed_field(small(prec, **kw), prec)


# the 16x16 benchmark workload (N = 256, 112 + 112 electrons, shell-closing
# ramp) at a short projection time: every tile, segment and factorisation size
# of the benchmark
BENCH = WORKLOADS["16x16"].replace(stab_interval=5, delay_rank=32)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_fixed_field_pass_16x16(prec):
    check_fixed_field(BENCH.replace(l_half=5, precision=prec), prec)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_fixed_field_pass_16x16_full_projection(prec):
    """The 16x16 benchmark workload at its full projection time (Theta = 10,
    l_half = 100, 202 slices, n_s = 5, k = 32): every checkpoint Green's
    function and every ratio of an upward and a downward pass at a fixed field
    against the oracle, 1e-10 (FP64) or 1e-5 (mixed) relative."""
    check_fixed_field(BENCH.replace(precision=prec), prec)


def _pooled_energy(ctx, n_chains):
    """Per-chain sums of the sign and the sign-weighted energy per site."""
    s = np.zeros(n_chains)
    se = np.zeros(n_chains)
    for c in range(n_chains):
        m = ctx.measurements(c)
        s[c] = m[:, 0].sum()
        se[c] = (m[:, 0] * m[:, 1]).sum()
    return s, se


def _jackknife_over_chains(f, *cols):
    n = len(cols[0])
    full = f(*(c.sum() for c in cols))
    loo = np.array([f(*(c.sum() - c[i] for c in cols)) for i in range(n)])
    return full, float(np.sqrt((n - 1) / n * np.sum((loo - loo.mean()) ** 2)))


def test_energy_mixed_matches_fp64_16x16():
    """Mixed against FP64 on the same batch of 16x16 chains at the full
    projection time (same seeds, so the same random streams): the
    sign-weighted energy per site agrees within one standard error of the
    FP64 estimate (error by jackknife over chains), and so does the
    difference within its own paired error bar."""
    n_chains, sweeps = 128, 6
    res = {}
    for prec in ("fp64", "mixed"):
        ctx = make_context([BENCH] * n_chains, prec, meas_capacity=sweeps + 2).init_trial()
        ctx.sweep(sweeps, measure=True)
        res[prec] = _pooled_energy(ctx, n_chains) + ([ctx.get_field(c) for c in range(n_chains)],)
        info = [ctx.chain_info(c) for c in range(n_chains)]
        # no NaN and no singular L R; the FP32 Green's function of the mixed
        # path may drift past its flag threshold between checkpoints (and a
        # tracked sign may then disagree with the recomputed one), but every
        # measurement is taken on the fresh FP64 G and sign of a checkpoint
        assert all((i["flags"] & (2 | 4)) == 0 for i in info), info
        if prec == "fp64":
            assert all(i["flags"] & ~16 == 0 and i["sign_mismatch"] == 0 for i in info), info
        print(f"{prec}: relative drift median {np.median([i['max_rel_drift'] for i in info]):.2e}, "
              f"max {max(i['max_rel_drift'] for i in info):.2e}; chains with a sign mismatch "
              f"{sum(i['sign_mismatch'] > 0 for i in info)}/{n_chains}")
        ctx.close()
    (s64, se64, f64), (s32, se32, f32) = res["fp64"], res["mixed"]
    e64, err64 = _jackknife_over_chains(lambda s, se: se / s, s64, se64)
    e32, err32 = _jackknife_over_chains(lambda s, se: se / s, s32, se32)
    d, derr = _jackknife_over_chains(lambda a, b, c, e: b / a - e / c, s32, se32, s64, se64)
    same = sum(np.array_equal(a, b) for a, b in zip(f32, f64))
    print(f"E/N fp64 {e64:.6f} +- {err64:.6f}, mixed {e32:.6f} +- {err32:.6f}, "
          f"difference {d:.2e} +- {derr:.2e}; chains with identical fields {same}/{n_chains}")
    assert abs(e32 - e64) <= err64
    assert abs(d) <= 3 * derr + 1e-6


# --------------------------------------------------------------------------- #
# Markov trajectories with shared random streams
# --------------------------------------------------------------------------- #
def follow_and_compare(ctx, chains, prec, n_sweeps, indep=None):
    """Advance GPU and oracle chains pass by pass; the oracle follows the GPU's
    decisions and every disagreement must be a near-threshold draw."""
    n_meas0 = [len(ch.measurements) for ch in chains]
    for sweep in range(n_sweeps):
        ctx.sweep(1, measure=True)
        for c, ch in enumerate(chains):
            f_gpu = ctx.get_field(c)
            bad = ch.sweep_following(f_gpu, TIE[prec])
            assert not bad, f"chain {c} sweep {sweep}: decisions differ beyond the tie band: {bad[:3]}"
            assert np.array_equal(ch.field, f_gpu)
            if indep is not None:
                indep[c].sweep(1)
    for c, ch in enumerate(chains):
        m_gpu = ctx.measurements(c)
        m_ref = np.array(ch.measurements[n_meas0[c]:])
        assert m_gpu.shape == m_ref.shape
        assert np.array_equal(m_gpu[:, 0], m_ref[:, 0])          # signs
        tol = {"fp64": 1e-10, "fp64wrap": 1e-10, "mixed": 1e-4, "mixed32b": 1e-3}[prec]
        assert np.max(np.abs(m_gpu[:, 1:] - m_ref[:, 1:])) < tol
        info = ctx.chain_info(c)
        # FP64 paths raise no flag; an FP32 Green's function may pass the
        # mixed path's 1e-5 drift threshold between checkpoints (flag 1),
        # while its decisions and measurements above still follow the oracle
        allowed = 16 if is_fp64(prec) else (16 | 1)
        assert info["sign_mismatch"] == 0 and (info["flags"] & ~allowed) == 0, info
        print(f"{prec} chain {c}: max relative drift {info['max_rel_drift']:.2e}")
        # log|W_sigma| and sgn W_sigma at the last checkpoint of the last pass
        la, sg = ctx.logdet(c)
        ref = ch.checkpoint_logdets[-1][2]
        for sp, s in ((0, 1), (1, -1)):
            assert sg[sp] == ref[s][1]
            assert abs(la[sp] - ref[s][0]) < LOGDET_TOL[prec] * max(1.0, abs(ref[s][0]))


@pytest.mark.parametrize("prec,kw,n_sweeps", [
    ("fp64", dict(L=4, l_half=6, n_s=3, k=8), 6),
    ("fp64wrap", dict(L=4, l_half=6, n_s=3, k=8), 6),
    ("fp64", dict(L=6, l_half=4, n_s=2, k=40), 4),                         # two scan blocks per segment
    ("fp64wrap", dict(L=4, l_half=5, n_s=3, k=5, U=3.0, n=5, ramp=0.05), 6),
    ("mixed", dict(L=4, l_half=6, n_s=3, k=8), 6),
    ("fp64", dict(L=6, l_half=5, n_s=4, k=7), 4),
    ("mixed", dict(L=8, l_half=10, n_s=4, k=16), 4),
    ("mixed32b", dict(L=6, l_half=5, n_s=3, k=16), 4),
    ("fp64", dict(L=4, l_half=5, n_s=3, k=5, U=3.0, n=5, ramp=0.05), 6),   # doped: signs
])
def test_trajectory_follows_oracle(prec, kw, n_sweeps):
    w = small(prec, **kw)
    ctx = make_context([w], prec).init_trial()
    ch = oracle_chain(w, 0)
    indep = [oracle_chain(w, 0)]
    follow_and_compare(ctx, [ch], prec, n_sweeps, indep)
    if is_fp64(prec):   # independent oracle run reaches the same field exactly
        assert np.array_equal(indep[0].field, ctx.get_field(0))
    ctx.close()


def rect(prec, lx, ly, n, l_half, n_s, k, U=4.0):
    return Workload(f"{lx}x{ly} test", lx, ly, U, n, n, 0.1, l_half, 0.21, 0.6, n_s, k, prec, 10)


# odd site counts: every row of G, X_a, Y_a and the bases is misaligned for
# vector loads, so the append, scan and GEMM kernels take their partial paths
ODD = [
    ("fp64", dict(lx=3, ly=5, n=7, l_half=5, n_s=3, k=8)),
    ("mixed", dict(lx=3, ly=5, n=7, l_half=5, n_s=3, k=8)),
    ("fp64", dict(lx=5, ly=5, n=12, l_half=4, n_s=3, k=16)),
    ("mixed", dict(lx=5, ly=5, n=12, l_half=4, n_s=3, k=16)),
]


@pytest.mark.parametrize("prec,kw", ODD)
def test_fixed_field_pass_odd_lattice(prec, kw):
    check_fixed_field(rect(prec, **kw), prec)


# doped lattices whose particle numbers per spin fall in the register-tile
# widths of the checkpoint factorisations (16 x 16 threads, ceil(n / 16)
# columns each) that no other case meets: 33-48, 81-96 and 113-128.  At
# n = 128, the largest width, the fused segment update and the propagation
# also span all eight 16-column blocks.  The ramp closes the trial's shell.
WIDTHS = [dict(L=8, n=40), dict(L=12, n=90), dict(L=12, n=128)]


@pytest.mark.parametrize("kw", WIDTHS)
def test_fixed_field_pass_every_factorisation_width(kw):
    w = small("fp64", l_half=3, n_s=2, k=32, U=3.0, ramp=0.1, **kw)
    check_fixed_field(w, "fp64")


def honey(prec, l1, l2, U=4.0, l_half=5, n_s=3, k=8):
    """Half-filled l1 x l2 honeycomb lattice (2 l1 l2 sites), the paper's
    Hubbard lattice (Eq. 2)."""
    n = l1 * l2
    return Workload(f"honeycomb {l1}x{l2}", l1, l2, U, n, n, 0.1, l_half, 0.21, 0.6, n_s, k, prec,
                    10, lattice_kind="honeycomb")


@pytest.mark.parametrize("prec,l1,l2", [("fp64", 3, 3), ("mixed", 3, 3), ("fp64", 8, 8),
                                        ("mixed", 8, 8)])
def test_fixed_field_pass_honeycomb(prec, l1, l2):
    """18 sites, and 128 sites (the large-tile GEMM path)."""
    check_fixed_field(honey(prec, l1, l2), prec)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_trajectory_honeycomb(prec):
    w = honey(prec, 3, 4, l_half=4, n_s=3, k=8)
    ctx = make_context([w], prec).init_trial()
    follow_and_compare(ctx, [oracle_chain(w, 0)], prec, 4)
    ctx.close()


def test_mixed_batch_of_honeycomb_and_square_follows_oracle():
    ws = [honey("mixed", 3, 3, l_half=4, n_s=2, k=8), small("mixed", L=4, l_half=4, n_s=2, k=8),
          honey("mixed", 4, 3, l_half=4, n_s=2, k=8)]
    ctx = make_context(ws, "mixed").init_trial()
    follow_and_compare(ctx, [oracle_chain(w, c) for c, w in enumerate(ws)], "mixed", 3)
    ctx.close()


def test_trajectory_odd_lattice_fp64():
    w = rect("fp64", 3, 7, 10, l_half=4, n_s=3, k=8)
    ctx = make_context([w], "fp64").init_trial()
    indep = [oracle_chain(w, 0)]
    follow_and_compare(ctx, [oracle_chain(w, 0)], "fp64", 4, indep)
    assert np.array_equal(indep[0].field, ctx.get_field(0))
    ctx.close()


def test_mixed_batch_of_odd_and_even_lattices_follows_oracle():
    """One context over 3x5, 4x4 and 5x5 chains (15, 16 and 25 sites)."""
    ws = [rect("mixed", 3, 5, 7, l_half=4, n_s=3, k=8), small("mixed", L=4, l_half=4, n_s=3, k=8),
          rect("mixed", 5, 5, 12, l_half=4, n_s=3, k=8)]
    ctx = make_context(ws, "mixed").init_trial()
    chains = [oracle_chain(w, c) for c, w in enumerate(ws)]
    follow_and_compare(ctx, chains, "mixed", 3)
    ctx.close()


@pytest.mark.parametrize("ph", [False, True])
def test_fixed_field_pass_18x18_wide_segment_update(ph):
    """18x18 at half filling (N = 324, 162 + 162 electrons, k = 32): more than
    128 particles per spin, so the one-wave scan feeds the Woodbury rows and
    the two segment GEMMs, and the propagation takes the general GEMM; with
    and without the particle-hole shortcut."""
    w = small("fp64", L=18, l_half=3, n_s=2, k=32)
    check_fixed_field(w, "fp64", **({"particle_hole": True} if ph else {}))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_fixed_field_pass_24x24(prec):
    """The large workload (N = 576, 288 + 288 electrons, dtau = 0.05, k = 64):
    factorisations beyond the register-tile size (n = 288) and 64-site
    segments, at a short projection time."""
    check_fixed_field(WORKLOADS["24x24"].replace(l_half=3, stab_interval=3, precision=prec), prec)


def test_uneven_batch_configuration_sampled_chains():
    """The uneven-batch configuration at its full size (256 chains, lattices
    6x6 .. 12x12, U in [2, 6], l_half = 50, k = 32, n_s = 5, FP64), one
    sweep; a 12x12 and a 6x6 chain are followed through the whole pass by the
    oracle, and no chain of the batch raises a flag."""
    ws = [w.replace(delay_rank=32) for w in batch_uneven(256)]
    ctx = make_context(ws, "fp64", meas_capacity=4).init_trial()
    ctx.sweep(1, measure=True)
    picks = [next(c for c, w in enumerate(ws) if w.lx == 12), next(c for c, w in enumerate(ws) if w.lx == 6)]
    for c in picks:
        ch = oracle_chain(ws[c], c)
        f_gpu = ctx.get_field(c)
        bad = ch.sweep_following(f_gpu, TIE["fp64"])
        assert not bad, f"chain {c}: decisions differ beyond the tie band: {bad[:3]}"
        assert np.array_equal(ch.field, f_gpu)
        m_gpu, m_ref = ctx.measurements(c), np.array(ch.measurements)
        assert m_gpu.shape == m_ref.shape
        assert np.array_equal(m_gpu[:, 0], m_ref[:, 0])
        assert np.max(np.abs(m_gpu[:, 1:] - m_ref[:, 1:])) < 1e-10
    drifts = []
    for c in range(len(ws)):
        info = ctx.chain_info(c)
        assert info["sign_mismatch"] == 0 and (info["flags"] & ~16) == 0, (c, info)
        drifts.append(info["max_rel_drift"])
    print(f"uneven batch: relative drift median {np.median(drifts):.2e}, max {max(drifts):.2e}")
    ctx.close()


def test_trajectory_16x16_fp64():
    w = BENCH.replace(l_half=5, precision="fp64")
    ctx = make_context([w], "fp64").init_trial()
    follow_and_compare(ctx, [oracle_chain(w, 0)], "fp64", 2)
    ctx.close()


@pytest.mark.parametrize("groups", [1, 4])
def test_bench_configuration_sampled_chains_fp64(groups):
    """The benchmark's launch configuration (2048 chains of the 16x16 workload
    at l_half = 100, k = 32, n_s = 5: one context, or 4 groups of 512 chains,
    one context and stream each, swept concurrently), one FP64 sweep; two
    sampled chains are followed through the whole pass by the oracle: fields
    (tie band aside) and the measured (sign, E/N, D)."""
    n_chains = 2048
    per = n_chains // groups
    ctxs = [make_context([BENCH] * per, "fp64", meas_capacity=4,
                         chain_ids=list(range(g * per, (g + 1) * per))).init_trial()
            for g in range(groups)]
    for ctx in ctxs:
        ctx.sweep(1, measure=True)
    for ctx in ctxs:
        ctx.synchronize()
    for c in (0, 1733):
        ctx, lc = ctxs[c // per], c % per
        ch = oracle_chain(BENCH, c)
        f_gpu = ctx.get_field(lc)
        bad = ch.sweep_following(f_gpu, TIE["fp64"])
        assert not bad, f"chain {c}: decisions differ beyond the tie band: {bad[:3]}"
        assert np.array_equal(ch.field, f_gpu)
        m_gpu, m_ref = ctx.measurements(lc), np.array(ch.measurements)
        assert m_gpu.shape == m_ref.shape
        assert np.array_equal(m_gpu[:, 0], m_ref[:, 0])
        assert np.max(np.abs(m_gpu[:, 1:] - m_ref[:, 1:])) < 1e-10
        info = ctx.chain_info(lc)
        assert info["sign_mismatch"] == 0 and (info["flags"] & ~16) == 0, info
    for ctx in ctxs:
        ctx.close()


def test_config_4x4_trajectory_fp64():
    w = WORKLOADS["4x4"]
    ctx = make_context([w, w], "fp64", chain_ids=[0, 1]).init_trial()
    chains = [oracle_chain(w, 0), oracle_chain(w, 1)]
    follow_and_compare(ctx, chains, "fp64", 4)
    ctx.close()


def test_uneven_batch_follows_oracle():
    ws = [w.replace(l_half=5, stab_interval=4) for w in batch_uneven(6, l_half=5)]
    ctx = make_context(ws, "mixed").init_trial()
    chains = [oracle_chain(w, c) for c, w in enumerate(ws)]
    follow_and_compare(ctx, chains, "mixed", 2)
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_determinism_same_seed_twice(prec):
    w = small(prec, L=8, l_half=8, n_s=4, k=16)
    out = []
    for _ in range(2):
        ctx = make_context([w, w], prec, chain_ids=[0, 1]).init_trial().sweep(3)
        out.append((ctx.get_field(0), ctx.get_field(1), ctx.get_green(0, 0), ctx.measurements(1)))
        ctx.close()
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_graph_and_direct_launch_agree(prec):
    w = small(prec, L=6, l_half=5, n_s=4, k=16)
    res = []
    for g in (True, False):
        ctx = make_context([w], prec, use_graph=g).init_trial().sweep(4)
        res.append((ctx.get_field(0), ctx.measurements(0)))
        ctx.close()
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_in_sweep_kernel_timing_counts_every_launch(prec):
    """Event timing inside sweeps, and the same chain as without timing.  Wrap
    engine: one wrap GEMM per bulk slice and one slice update per slice of
    each pass.  Factored engine: one propagation per bulk slice, one segment
    update and one scan per delay segment of every slice."""
    w = small(prec, L=6, l_half=5, n_s=4, k=16)
    res = []
    for timed in (True, False):
        ctx = make_context([w], prec).init_trial()
        if timed:
            ctx.set_kernel_timing(7)
        ctx.sweep(2)
        if timed:
            (t0, n0), (t1, n1), (t2, n2) = (ctx.kernel_timing(k) for k in range(3))
            M = 2 * w.l_half
            if prec == "fp64":
                nseg = 2 * (M + 2) * math.ceil(w.n_sites / w.delay_rank)
                assert n0 == 2 * M and n1 == nseg and n2 == nseg, (n0, n1, n2)
            else:
                assert n0 == 2 * M and n2 == 2 * (M + 2) and n1 > 0, (n0, n1, n2)
            assert t0 > 0 and t1 > 0 and t2 > 0
            ctx.set_kernel_timing(0)
            assert ctx.kernel_timing(0) == (0.0, 0)
        res.append((ctx.get_field(0), ctx.measurements(0)))
        ctx.close()
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])


def test_autotune_times_every_candidate_and_picks_a_valid_one():
    from paper_2303_13403_amd.autotune import DRIFT_LIMIT, autotune, qualifies

    ws = [w.replace(l_half=5) for w in batch_uneven(8, l_half=5)]
    best, trials = autotune(ws, gpqmc.FP64, delay_ranks=(8, 16), stab_intervals=(2, 4), sweeps=1)
    assert sorted((t.delay_rank, t.stab_interval) for t in trials) == [(8, 2), (8, 4), (16, 2), (16, 4)]
    assert all(t.ms_per_sweep > 0 and t.updates_per_s > 0 for t in trials)
    lim = DRIFT_LIMIT[gpqmc.FP64]
    assert best in trials and qualifies(best, lim)
    assert best.ms_per_sweep == min(t.ms_per_sweep for t in trials if qualifies(t, lim))


# --------------------------------------------------------------------------- #
# edge cases and the full-size configurations
# --------------------------------------------------------------------------- #
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_workspace_contents_do_not_matter(prec):
    """A read of device memory the library never wrote would make results
    depend on what the workspace held before: 64 chains of the 16x16 workload
    (l_half = 5) swept three times from a NaN-filled and from a zero-filled
    workspace give bit-identical fields, records and flags."""
    w = BENCH.replace(l_half=5)
    out = []
    for fill in (float("nan"), 0.0):
        ctx = make_context([w] * 64, prec, meas_capacity=8, workspace_fill=fill).init_trial()
        ctx.sweep(3, measure=True)
        out.append(([ctx.get_field(c) for c in range(64)], [ctx.measurements(c) for c in range(64)],
                    [ctx.chain_info(c)["flags"] for c in range(64)]))
        ctx.close()
    (fa, ma, ga), (fb, mb, gb) = out
    assert all(np.array_equal(a, b) for a, b in zip(fa, fb))
    assert all(np.array_equal(a, b) for a, b in zip(ma, mb))
    assert ga == gb
    assert all(np.all(np.isfinite(m)) for m in ma)


@pytest.mark.parametrize("prec", ["fp64", "fp64wrap", "mixed"])
def test_free_fermions_every_record_is_the_closed_form(prec):
    """U = 0 and g = 0: every flip factor is zero (the scans' zero-Delta path
    on bulk and boundary slices), every proposal is accepted without changing
    G, and every record's energy equals the closed-form free-fermion value
    sum_sigma -tr(K G_sigma) with R = e^{-Theta K} P (no Trotter error at U = 0)."""
    w = small(prec, L=4, l_half=6, n_s=3, k=8, U=0.0).replace(g=0.0)
    ctx = make_context([w, w], prec, chain_ids=[0, 1]).init_trial()
    ctx.sweep(4, measure=True)
    m = pqmc.Model.from_workload(w)
    e_ref = pqmc.free_energy_closed_form(m.K, m.P[1], m.P[-1], w.theta) / m.N
    for c in range(2):
        rec = ctx.measurements(c)
        assert rec.shape[0] == 4 and np.all(rec[:, 0] == 1)
        tol = 1e-10 if is_fp64(prec) else 1e-6
        assert np.max(np.abs(rec[:, 1] - e_ref)) < tol * abs(e_ref), (rec[:, 1], e_ref)
        info = ctx.chain_info(c)
        assert info["accepted"] == info["proposed"] and (info["flags"] & ~16) == 0, info
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_trajectory_slater_trial_g0_follows_oracle(prec):
    """The plain Slater-determinant trial SD(AFM) (g = 0, M_N > 0): the
    boundary slices carry no flip factor (the scans' zero-Delta path on them)
    while the bulk slices sample; doped 4x4 and half-filled 6x6."""
    for kw in (dict(L=4, l_half=5, n_s=3, k=5, U=3.0, n=5, ramp=0.05), dict(L=6, l_half=5, n_s=4, k=16)):
        w = small(prec, **kw).replace(g=0.0)
        ctx = make_context([w], prec).init_trial()
        follow_and_compare(ctx, [oracle_chain(w, 0)], prec, 4)
        ctx.close()


def _sampled_full_projection(w, prec, positions):
    """One fixed-field upward pass of one chain on the GPU with every
    checkpoint recorded; the oracle computes the fresh G at the sampled
    positions independently (QR after every slice), and the ratios of the
    slice after each from its diagonal."""
    ctx = make_context([w], prec, trace=True).init_trial()
    ctx.set_debug(True)
    ctx.sweep(1, measure=False)
    r_gpu, g_gpu, d_gpu = ctx.trace(0)
    m = pqmc.Model.from_workload(w)
    f = ctx.get_field(0)
    assert np.array_equal(f, oracle_chain(w, 0).field)
    ck = [p for p in m.checkpoints if p >= 0]      # the upward pass's checkpoints, in order
    errs = []
    for p in positions:
        k = ck.index(p)
        for sp, s in ((0, 1), (1, -1)):
            G = pqmc.green_stable(m, f, p, s)
            errs.append(rel_err(g_gpu[k, sp], G))
            if p + 1 <= m.M + 1:                 # ratios of slice p + 1 from diag G_p
                l = p + 1
                r_ref = np.array([1.0 + m.flip_delta(int(f[l, i]), l, s) * (1.0 - G[i, i])
                                  for i in range(m.N)])
                errs.append(rel_err(r_gpu[l, :, sp], r_ref))
    ctx.close()
    return max(errs), float(np.max(d_gpu))


def test_fixed_field_24x24_full_projection_sampled():
    """The 24x24 configuration at its full size (N = 576, 288 + 288 electrons,
    dtau = 0.05, l_half = 200: 402 slices, n_s = 10, k = 32, FP64): the fresh G
    at sampled checkpoints of an upward fixed-field pass (both spins) and the
    ratios of the following slices against the oracle's independent
    stabilised products."""
    w = WORKLOADS["24x24"].replace(stab_interval=10, delay_rank=32, precision="fp64")
    err, drift = _sampled_full_projection(w, "fp64", [200, 401])
    print(f"24x24 full projection, fp64: max error {err:.2e}, max drift {drift:.2e}")
    assert err < 1e-10 and drift < 1e-8


def test_fixed_field_12x12_mixed_at_its_configured_interval():
    """The 12x12 configuration compares FP64 with the mixed path at QR every
    10 slices.  At a fixed field the mixed path's fresh checkpoint G (FP64)
    holds 1e-5, but its FP32 Green's function drifts between checkpoints: the
    error of the ratios of a whole upward and downward pass is stated here and
    bounded by what was measured (FP64 at the same interval: 1e-10)."""
    res = {}
    for prec in ("mixed", "fp64"):
        w = small(prec, L=12, l_half=50, n_s=10, k=32)
        ctx = make_context([w], prec, trace=True).init_trial()
        ctx.set_debug(True)
        ch = oracle_chain(w, 0)
        r_err = g_err = drift = 0.0
        for sweep in range(2):
            ctx.sweep(1, measure=False)
            oracle_fixed_pass(ch)
            r_gpu, g_gpu, d_gpu = ctx.trace(0)
            r_err = max(r_err, rel_err(r_gpu, ratio_array(ch, sweep, ch.m.n_slices, w.n_sites)))
            for k, (sw, p, gu, gd, _, _) in enumerate(ch.checkpoint_greens):
                g_err = max(g_err, rel_err(g_gpu[k, 0], gu), rel_err(g_gpu[k, 1], gd))
            drift = max(drift, float(np.max(d_gpu)))
        res[prec] = (r_err, g_err, drift)
        print(f"12x12 {prec}, n_s = 10: ratio error {r_err:.2e}, checkpoint G error {g_err:.2e}, "
              f"max drift {drift:.2e}")
        ctx.close()
    assert res["fp64"][0] < 1e-10 and res["fp64"][1] < 1e-10
    assert res["mixed"][1] < 1e-5          # the fresh FP64 G at the checkpoints
    assert res["mixed"][0] < 1e-1          # the FP32 ratios: the stated error (see the printout)


# --------------------------------------------------------------------------- #
# particle-hole shortcut at half filling: spin up only, spin down derived; the
# oracle runs both spins independently
# --------------------------------------------------------------------------- #
PH_FIXED = [
    dict(L=4, l_half=6, n_s=3, k=8),
    dict(L=4, l_half=0, n_s=1, k=8),                  # boundary slices only
    dict(L=6, l_half=5, n_s=4, k=7),                  # ragged segments
    dict(L=12, l_half=50, n_s=10, k=32),              # the 12x12 workload
    dict(L=24, l_half=3, n_s=2, k=32),                # N_sigma = 288: general segment update
    dict(L=4, l_half=6, n_s=3, k=8, g=0.0),          # no boundary coupling
]


@pytest.mark.parametrize("kw", PH_FIXED)
def test_particle_hole_fixed_field_matches_two_spin_oracle(kw):
    """Every ratio (both spins), every checkpoint G (spin down mirrored from
    spin up) and every log|W_sigma| (spin down from the field sum) of an upward
    and a downward pass against the oracle's independent two-spin run."""
    g = kw.pop("g", None)
    w = small("fp64", **kw)
    if g is not None:
        w = w.replace(g=g)
    check_fixed_field(w, "fp64", particle_hole=True)


@pytest.mark.parametrize("l1,l2", [(3, 3), (8, 8)])
def test_particle_hole_fixed_field_honeycomb(l1, l2):
    check_fixed_field(honey("fp64", l1, l2), "fp64", particle_hole=True)


@pytest.mark.parametrize("kw,n_sweeps", [
    (dict(L=4, l_half=6, n_s=3, k=8), 6),
    (dict(L=6, l_half=5, n_s=4, k=7), 4),
    (dict(L=8, l_half=10, n_s=5, k=32), 3),
])
def test_particle_hole_trajectory_follows_two_spin_oracle(kw, n_sweeps):
    w = small("fp64", **kw)
    ctx = make_context([w], "fp64", particle_hole=True).init_trial()
    assert ctx.chain_info(0)["particle_hole"] == 1
    ch = oracle_chain(w, 0)
    indep = [oracle_chain(w, 0)]
    follow_and_compare(ctx, [ch], "fp64", n_sweeps, indep)
    assert np.array_equal(indep[0].field, ctx.get_field(0))
    # the last fresh G (spin down mirrored on the host) at the pass's end
    p_end = ch.m.M + 1 if n_sweeps % 2 else -1
    f = ctx.get_field(0)
    for sp, s in ((0, 1), (1, -1)):
        assert rel_err(ctx.get_green(0, sp), pqmc.green_stable(ch.m, f, p_end, s)) < 1e-10
    ctx.close()


def test_particle_hole_only_where_exact():
    """A batch of half-filled square and honeycomb chains, a doped chain and
    a half-filled chain with a trial potential: the shortcut applies to the
    first two only, and every chain follows the oracle."""
    ws = [small("fp64", L=4, l_half=5, n_s=3, k=8),
          honey("fp64", 3, 3, l_half=5, n_s=3, k=8),
          small("fp64", L=4, l_half=5, n_s=3, k=8, U=3.0, n=5),
          small("fp64", L=4, l_half=5, n_s=3, k=8, ramp=0.05)]
    ctx = make_context(ws, "fp64", particle_hole=True).init_trial()
    assert [ctx.chain_info(c)["particle_hole"] for c in range(4)] == [1, 1, 0, 0]
    chains = [oracle_chain(w, c) for c, w in enumerate(ws)]
    follow_and_compare(ctx, chains, "fp64", 3)
    ctx.close()
    # without the option no chain uses it
    ctx = make_context(ws[:1], "fp64").init_trial()
    assert ctx.chain_info(0)["particle_hole"] == 0
    ctx.close()
