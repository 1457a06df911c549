"""Pins of the oracle's building blocks against published values, closed forms,
library routines and exhaustive checks (no GPU)."""
import itertools
import math
import os

import numpy as np
import pytest
import scipy.linalg

from oracle import philox, pqmc
from paper_2303_13403_amd.workloads import WORKLOADS, shell_ramp, square_lattice

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------- #
# Philox4x32-10: published known-answer vectors
# --------------------------------------------------------------------------- #
def _kat():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((v[:4], v[4:6], v[6:]))
    return rows


@pytest.mark.parametrize("ctr,key,out", _kat())
def test_philox_known_answers(ctr, key, out):
    got = philox.philox4x32_10(np.array(ctr), key)
    assert [int(x) for x in got] == out


def test_philox_uniform_range_and_moments():
    u = philox.accept_uniforms(13403, 3, 7, 11, 200000)
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 4 * math.sqrt(1 / 12 / len(u))
    assert abs(u.var() - 1 / 12) < 0.002
    # 53-bit resolution: values are multiples of 2^-53 and not of 2^-32 only
    assert np.all(np.floor(u * 2.0**53) == u * 2.0**53)
    assert np.any(np.floor(u * 2.0**32) != u * 2.0**32)


def test_philox_streams_are_distinct():
    a = philox.accept_uniforms(1, 0, 0, 0, 64)
    b = philox.accept_uniforms(1, 1, 0, 0, 64)
    c = philox.accept_uniforms(1, 0, 1, 0, 64)
    d = philox.accept_uniforms(1, 0, 0, 1, 64)
    assert len({tuple(x) for x in (a, b, c, d)}) == 4
    f = philox.initial_field(13403, 0, 5, 16)
    assert set(np.unique(f)) == {-1, 1}
    assert np.array_equal(f, philox.initial_field(13403, 0, 5, 16))


# --------------------------------------------------------------------------- #
# Eq. 1: the discrete decoupling of the Gutzwiller / Hubbard factor
# --------------------------------------------------------------------------- #
@pytest.mark.parametrize("x", [0.0, 0.2, 0.35, 0.4, 0.55, 0.6, 1.7])
def test_decoupling_identity_all_occupations(x):
    c = pqmc.hs_coupling(x)
    assert math.isclose(math.cosh(c), math.exp(x / 2), rel_tol=1e-14)
    for nu, nd in itertools.product((0, 1), repeat=2):
        lhs = math.exp(-x * (nu - 0.5) * (nd - 0.5))
        rhs = 0.5 * math.exp(-x / 4) * sum(math.exp(c * s * (nu - nd)) for s in (1, -1))
        assert math.isclose(lhs, rhs, rel_tol=1e-14)
        # the shifted form differs from exp(-x n_up n_dn) by exp(-x (n_up + n_dn)/2 + x/4),
        # a constant at fixed particle number
        assert math.isclose(math.exp(-x * nu * nd),
                            lhs * math.exp(-x * (nu + nd) / 2 + x / 4), rel_tol=1e-14)


def test_decoupling_as_printed_is_not_an_identity():
    """Eq. 1 as printed (density channel, no shift) fails on every occupation;
    this is why the spin-channel reading is used."""
    g = 0.6
    lam = math.acosh(math.exp(g / 2))
    bad = 0
    for nu, nd in itertools.product((0, 1), repeat=2):
        lhs = math.exp(-g * nu * nd)
        rhs = 0.5 * math.exp(-g / 4) * sum(math.exp(lam * s * (nu + nd)) for s in (1, -1))
        bad += not math.isclose(lhs, rhs, rel_tol=1e-6)
    assert bad == 4


# --------------------------------------------------------------------------- #
# lattice, e^{-dtau K}, Neel trial (Hubbard section)
# --------------------------------------------------------------------------- #
@pytest.mark.parametrize("L", [2, 3, 4, 6, 12])
def test_square_lattice_spectrum_closed_form(L):
    K, eps, xy = square_lattice(L, L)
    assert np.allclose(K, K.T)
    k = 2 * np.pi * np.arange(L) / L
    ref = np.sort((-2 * (np.cos(k)[:, None] + np.cos(k)[None, :])).ravel())
    # (L = 2: both wrap bonds land on the same pair and accumulate, which is
    # exactly what the plane-wave formula counts)
    assert np.allclose(np.linalg.eigvalsh(K), ref, atol=1e-12)
    if L % 2 == 0:   # bipartite: eps K eps = -K
        S = np.diag(eps.astype(float))
        assert np.allclose(S @ K @ S, -K)


def test_hopping_exponentials_match_expm():
    K, _, _ = square_lattice(4, 4)
    Km, Kp = pqmc.hopping_exponentials(K, 0.1)
    assert np.allclose(Km, scipy.linalg.expm(-0.1 * K), atol=1e-13)
    assert np.allclose(Kp, scipy.linalg.expm(0.1 * K), atol=1e-13)
    assert np.allclose(Km @ Kp, np.eye(16), atol=1e-13)


@pytest.mark.parametrize("L,m", [(4, 0.21), (6, 0.07), (12, 0.21)])
def test_neel_trial_spectrum_closed_form(L, m):
    K, eps, _ = square_lattice(L, L)
    k = 2 * np.pi * np.arange(L) / L
    ek = (-2 * (np.cos(k)[:, None] + np.cos(k)[None, :])).ravel()
    # k and k + (pi, pi) fold onto one pair of bands +-sqrt(e_k^2 + M^2): every
    # value of the doubled list below appears twice
    ref = np.sort(np.concatenate([-np.sqrt(ek**2 + m**2), np.sqrt(ek**2 + m**2)]))[::2]
    for s in (1, -1):
        P, w, gap = pqmc.neel_trial(K, eps, m, L * L // 2, s)
        assert np.allclose(np.sort(w), ref, atol=1e-12)
        assert math.isclose(gap, 2 * m, rel_tol=1e-9)     # half filling
        assert np.allclose(P.T @ P, np.eye(L * L // 2), atol=1e-12)


def test_doped_16x16_trial_needs_the_ramp():
    w = WORKLOADS["16x16"]
    K, eps, _ = w.lattice()
    _, _, gap0 = pqmc.neel_trial(K, eps, w.m_neel, w.n_up, 1)
    assert gap0 < 1e-10           # four-fold degenerate Fermi level
    _, _, gap = pqmc.neel_trial(K, eps, w.m_neel, w.n_up, 1, shell_ramp(16, 16, 0.1))
    assert gap > 1e-3
    with pytest.raises(ValueError):
        pqmc.Model.from_workload(w.replace(ramp=0.0, l_half=1))


# --------------------------------------------------------------------------- #
# free fermions: closed forms (U = 0, g = 0)
# --------------------------------------------------------------------------- #
def _free_ground(L, n):
    k = 2 * np.pi * np.arange(L) / L
    ek = np.sort((-2 * (np.cos(k)[:, None] + np.cos(k)[None, :])).ravel())
    return 2 * ek[:n].sum()


def test_free_ground_state_values():
    # independent closed-form values, quoted to 10 digits
    assert math.isclose(_free_ground(4, 8), -24.0, abs_tol=1e-12)
    assert math.isclose(_free_ground(12, 72), -230.8512516844, abs_tol=1e-9)
    assert math.isclose(_free_ground(16, 112), -412.0817960355, abs_tol=1e-9)


@pytest.mark.parametrize("l_half", [0, 3, 10])
def test_free_fermion_energy_matches_closed_form(l_half):
    """U = 0 and g = 0: every field weight is equal, no Trotter error; the
    chain's measured energy equals the single-particle closed form exactly."""
    K, eps, _ = square_lattice(4, 4)
    # M_N > 0 gives a non-degenerate trial that is not the ground state of K
    m = pqmc.Model(K, eps, U=0.0, n_up=8, n_dn=8, dtau=0.1, l_half=l_half,
                   m_neel=0.5, g=0.0, stab_interval=3)
    ch = pqmc.Chain(m, seed=1).sweep(2)
    ref = pqmc.free_energy_closed_form(K, m.P[1], m.P[-1], l_half * 0.1) / 16
    for sgn, e, *_ in ch.measurements:
        assert sgn == 1
        assert math.isclose(e, ref, abs_tol=1e-12)


def test_free_fermion_long_projection_reaches_ground_state():
    K, eps, _ = square_lattice(4, 4)
    _, _, gap = pqmc.neel_trial(K, eps, 0.5, 8, 1)
    m = pqmc.Model(K, eps, U=0.0, n_up=8, n_dn=8, dtau=0.25, l_half=40,
                   m_neel=0.5, g=0.0, stab_interval=4)
    ch = pqmc.Chain(m, seed=2).sweep(1)
    assert math.isclose(ch.measurements[0][1] * 16, -24.0, abs_tol=1e-8)


def test_jackknife_reduces_to_binned_standard_error_without_sign():
    """With every sign +1 the jackknife of sum(s O)/sum(s) is the standard
    error of the bin means (delete-one estimates of a plain mean are the mean
    shifted by (m - b_k)/(nb - 1)); a constant observable has zero error."""
    from oracle import stats
    rng = np.random.default_rng(3)
    obs = rng.normal(size=200)
    m1, e1 = stats.sign_weighted(np.ones(200), obs, bin_size=10)
    bins = obs.reshape(20, 10).mean(axis=1)
    assert m1 == pytest.approx(obs.mean(), rel=1e-13)
    assert e1 == pytest.approx(bins.std(ddof=1) / np.sqrt(20), rel=1e-12)
    m2, e2 = stats.mean_error(obs, bin_size=10)
    assert (m2, e2) == pytest.approx((m1, e1), rel=1e-12)
    signs = rng.choice([-1.0, 1.0], size=200, p=[0.3, 0.7])
    m3, e3 = stats.sign_weighted(signs, np.full(200, 2.5), bin_size=10)
    assert m3 == pytest.approx(2.5, rel=1e-14) and e3 < 1e-13

