"""Pins of the whole estimator chain (decoupling, boundary slices, Trotter order,
Wick estimates): exact enumeration of every auxiliary-field configuration
against Fock-space linear algebra on tiny clusters, and the Markov chain against
the same exact values within statistical errors (no GPU)."""
import math

import numpy as np
import pytest

from oracle import ed, pqmc, stats
from paper_2303_13403_amd.workloads import square_lattice


def _ring(n, t=1.0):
    K = np.zeros((n, n))
    for i in range(n):
        K[i, (i + 1) % n] -= t
        K[(i + 1) % n, i] -= t
    return K, np.array([(-1) ** i for i in range(n)])


CASES = {
    "2x2 half filling": lambda: pqmc.Model(*square_lattice(2, 2)[:2], U=4.0, n_up=2, n_dn=2,
                                           dtau=0.1, l_half=1, m_neel=0.21, g=0.6,
                                           stab_interval=1),
    "4-ring half filling": lambda: pqmc.Model(*_ring(4), U=3.0, n_up=2, n_dn=2, dtau=0.2,
                                              l_half=1, m_neel=0.3, g=0.55, stab_interval=1),
    "4-ring doped 1+2": lambda: pqmc.Model(*_ring(4), U=5.0, n_up=1, n_dn=2, dtau=0.3,
                                           l_half=1, m_neel=0.4, g=0.8, stab_interval=1,
                                           potential=[0.0, 0.05, 0.1, 0.15]),
    "3-site random hopping": lambda: pqmc.Model(
        (lambda A: A + A.T)(np.random.default_rng(1).normal(size=(3, 3))),
        [1, -1, 1], U=3.0, n_up=1, n_dn=2, dtau=0.2, l_half=1, m_neel=0.3, g=0.5,
        stab_interval=1),
    "3-site two slices per side": lambda: pqmc.Model(
        (lambda A: A + A.T)(np.random.default_rng(2).normal(size=(3, 3))),
        [1, -1, 1], U=2.0, n_up=1, n_dn=1, dtau=0.25, l_half=2, m_neel=0.2, g=0.7,
        stab_interval=2),
}


@pytest.mark.parametrize("name", list(CASES))
def test_enumeration_equals_fock_space(name):
    m = CASES[name]()
    e_ed, d_ed = ed.trotter_energy_ed(m)
    e_en, d_en, _ = ed.enumerate_energy(m)
    assert math.isclose(e_en, e_ed, rel_tol=1e-12, abs_tol=1e-12)
    assert math.isclose(d_en, d_ed, rel_tol=1e-12, abs_tol=1e-12)


def test_variational_energy_at_zero_projection():
    """Theta = 0 (only the two projector slices): the estimate is the
    variational energy of the Gutzwiller state (Method section)."""
    K, eps, _ = square_lattice(2, 2)
    m = pqmc.Model(K, eps, U=4.0, n_up=2, n_dn=2, dtau=0.1, l_half=0, m_neel=0.21,
                   g=0.6, stab_interval=1)
    e_en, _, _ = ed.enumerate_energy(m)
    assert math.isclose(e_en, ed.trotter_energy_ed_projector(m), rel_tol=1e-12)
    # g = 0 gives the plain Slater-determinant energy: the projector matters
    m0 = pqmc.Model(K, eps, U=4.0, n_up=2, n_dn=2, dtau=0.1, l_half=0, m_neel=0.21,
                    g=0.0, stab_interval=1)
    assert ed.trotter_energy_ed_projector(m0) > ed.trotter_energy_ed_projector(m) + 1e-3


def test_gutzwiller_only_fields_u0():
    """U = 0, g > 0: only the 2N boundary fields matter."""
    K, eps = _ring(4)
    m = pqmc.Model(K, eps, U=0.0, n_up=2, n_dn=2, dtau=0.3, l_half=1, m_neel=0.3,
                   g=0.9, stab_interval=1)
    e_en, d_en, _ = ed.enumerate_energy(m)
    e_ed, d_ed = ed.trotter_energy_ed(m)
    assert math.isclose(e_en, e_ed, rel_tol=1e-12)
    assert math.isclose(d_en, d_ed, rel_tol=1e-12)


@pytest.mark.parametrize("name", ["2x2 half filling", "4-ring doped 1+2"])
def test_markov_chain_agrees_with_exact(name):
    m = CASES[name]()
    e_ex, d_ex, _ = ed.enumerate_energy(m)
    ch = pqmc.Chain(m, seed=21).sweep(1600)
    meas = np.array(ch.measurements[200:])
    e, de = stats.sign_weighted(meas[:, 0], meas[:, 1], 20)
    d, dd = stats.sign_weighted(meas[:, 0], meas[:, 2], 20)
    assert abs(e - e_ex) < 3.5 * de + 1e-12, (e, de, e_ex)
    assert abs(d - d_ex) < 3.5 * dd + 1e-12, (d, dd, d_ex)
    assert ch.sign_mismatches == 0


@pytest.mark.parametrize("name", list(CASES))
def test_structure_factor_enumeration_equals_fock_space(name):
    """S_AFM: the Wick estimator summed over every field configuration
    against the spin operators in Fock space (pins every term of the Wick
    expansion, including the spin-flip part)."""
    m = CASES[name]()
    _, _, s_en, _ = ed.enumerate_energy(m, with_saf=True)
    s_ed = ed.trotter_saf_ed(m)
    assert math.isclose(s_en, s_ed, rel_tol=1e-11, abs_tol=1e-12)


def test_structure_factor_of_a_neel_product_state():
    """A classical Neel state (one up spin on every A site, one down on every
    B site) has <S^z_i S^z_j> = eps_i eps_j / 4 and no spin-flip correlation
    off the diagonal: S_AFM = 1/4 + (3/4 - 1/4) / N, from the Wick estimator
    with the Green's functions of that Slater determinant."""
    N = 6
    eps = np.array([1, -1] * 3)
    occ_up = np.diag((eps > 0).astype(float))
    occ_dn = np.diag((eps < 0).astype(float))
    Gup, Gdn = np.eye(N) - occ_up, np.eye(N) - occ_dn       # G_ij = <c_i c_j^dag>
    s = pqmc.structure_factor(eps, Gup, Gdn)
    # S^z part: (sum_i eps_i S^z_i)^2 / N^2 = (N/2)^2 / N^2 = 1/4; flip part on
    # the diagonal: <S^+_i S^-_i + S^-_i S^+_i>/2 = 1/2 per site
    assert math.isclose(s, 0.25 + 0.5 / N, rel_tol=1e-14)
