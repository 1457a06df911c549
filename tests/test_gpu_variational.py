"""Theta = 0 (variational) scans over the trial parameters (g, M_N) on the
HIP path, against the oracle: the Markov trajectory with only the two
projector slices, and the sampled variational energy and staggered structure
factor against the exact Fock-space values of tiny clusters."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from gpu_helpers import TIE, make_context, oracle_chain
from oracle import ed, pqmc
from paper_2303_13403_amd import gpqmc
from paper_2303_13403_amd.variational import optimum, variational_scan
from paper_2303_13403_amd.workloads import Workload


def _w(L=4, g=0.6, m=0.21, U=4.0, k=8, lx=None, ly=None):
    lx = L if lx is None else lx
    ly = L if ly is None else ly
    n = lx * ly // 2
    return Workload(f"{lx}x{ly} theta0", lx, ly, U, n, n, 0.1, 0, m, g, 1, k, "fp64", 10)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_zero_projection_trajectory_follows_oracle(prec):
    """l_half = 0: both passes cover only the two projector slices; fields
    bit-exact except near-threshold draws, and the measured (sign, E/N, D)."""
    ws = [_w(4, g=0.6, m=0.21), _w(4, g=0.3, m=0.5)]
    ctx = make_context(ws, prec, chain_ids=[0, 1]).init_trial()
    chains = [oracle_chain(w, c) for c, w in enumerate(ws)]
    n_meas0 = [len(ch.measurements) for ch in chains]
    for sweep in range(6):
        ctx.sweep(1, measure=True)
        for c, ch in enumerate(chains):
            f_gpu = ctx.get_field(c)
            bad = ch.sweep_following(f_gpu, TIE[prec])
            assert not bad, f"chain {c} sweep {sweep}: {bad[:3]}"
            assert np.array_equal(ch.field, f_gpu)
    tol = {"fp64": 1e-10, "mixed": 1e-4}[prec]
    for c, ch in enumerate(chains):
        m_gpu, m_ref = ctx.measurements(c), np.array(ch.measurements[n_meas0[c]:])
        assert m_gpu.shape == m_ref.shape and len(m_gpu) == 6      # one record per sweep
        assert np.array_equal(m_gpu[:, 0], m_ref[:, 0])
        assert np.max(np.abs(m_gpu[:, 1:] - m_ref[:, 1:])) < tol
    ctx.close()


def test_variational_scan_matches_exact_energies_2x2():
    """2x2 half filling, U = 4: the sampled Theta = 0 energy of every grid
    point agrees with the exact variational energy of the Gutzwiller state
    within four standard errors, and the scan's optimum is the exact one
    (exact energies of this grid: optimum -1.3739 at g = 0.3, M_N = 0.3,
    the next -1.3505)."""
    gs, ms = [0.1, 0.3, 0.7], [0.3, 1.0]
    base = _w(lx=2, ly=2, k=4)
    pts, st = variational_scan(base, gs, ms, chains_per_point=512, sweeps=100, warmup=10)
    assert st["chains"] == 6 * 512
    exact = {}
    for p in pts:
        m = pqmc.Model.from_workload(base.replace(g=p["g"], m_neel=p["m_neel"], l_half=0,
                                                  stab_interval=1))
        exact[(p["g"], p["m_neel"])] = ed.trotter_energy_ed_projector(m)
        e, err = p["energy"]
        assert p["records"] == 512 * 100
        assert 0 < err < 0.01
        assert abs(e - exact[(p["g"], p["m_neel"])]) < 4 * err + 1e-12, (p, exact)
        # the staggered structure factor of the same state, exact in Fock space
        s, serr = p["structure_factor"]
        s_ex = ed.trotter_saf_ed(m)
        assert 0 < serr < 0.01 and abs(s - s_ex) < 4 * serr + 1e-12, (p, s_ex)
    best = optimum(pts)
    ex_best = min(exact, key=exact.get)
    # the best exact energy is several standard errors clear of the next
    gap = sorted(exact.values())[1] - sorted(exact.values())[0]
    assert gap > 6 * max(p["energy"][1] for p in pts)
    assert (best["g"], best["m_neel"]) == ex_best


def test_variational_scan_single_point_equals_its_chains():
    """A grid of one point: the scan's estimate is the library's own
    estimator over that context's chains."""
    w = _w(4, k=8)
    pts, _ = variational_scan(w, [0.6], [0.21], chains_per_point=8, sweeps=20, warmup=2)
    assert len(pts) == 1 and pts[0]["records"] == 8 * 20
    ctx = make_context([w.replace(l_half=0, stab_interval=1)] * 8, "fp64",
                       chain_ids=list(range(8)), meas_capacity=64).init_trial()
    ctx.sweep(2, measure=True)
    ctx.reset_measurements()
    ctx.sweep(20, measure=True)
    e_lib = ctx.measure_energy(-1)
    ctx.close()
    assert abs(pts[0]["energy"][0] - e_lib[0]) < 1e-12
    assert abs(pts[0]["energy"][1] - e_lib[1]) < 1e-12


def test_variational_scan_matches_exact_honeycomb_3x1():
    """The paper's lattice: 3 x 1 honeycomb cells (6 sites) at half filling,
    U = 4.  Energies and staggered structure factors of a 2 x 2 grid agree
    with the exact Fock-space values within four standard errors, and the
    scan's optimum is the exact one (-1.3080 at g = 0.6, M_N = 0.3; the next
    is -1.2790)."""
    base = Workload("honeycomb 3x1 theta0", 3, 1, 4.0, 3, 3, 0.1, 0, 0.3, 0.6, 1, 6, "fp64", 10,
                    lattice_kind="honeycomb")
    pts, st = variational_scan(base, [0.2, 0.6], [0.3, 0.8], chains_per_point=512, sweeps=100,
                               warmup=10)
    exact = {}
    for p in pts:
        m = pqmc.Model.from_workload(base.replace(g=p["g"], m_neel=p["m_neel"]))
        e_ex, s_ex = ed.trotter_energy_ed_projector(m), ed.trotter_saf_ed(m)
        exact[(p["g"], p["m_neel"])] = e_ex
        (e, de), (s, ds) = p["energy"], p["structure_factor"]
        assert abs(e - e_ex) < 4 * de + 1e-12, (p, e_ex)
        assert abs(s - s_ex) < 4 * ds + 1e-12, (p, s_ex)
    gap = sorted(exact.values())[1] - sorted(exact.values())[0]
    assert gap > 6 * max(p["energy"][1] for p in pts)
    best = optimum(pts)
    assert (best["g"], best["m_neel"]) == min(exact, key=exact.get)
