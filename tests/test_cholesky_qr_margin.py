"""Margin of the single-pass Cholesky-QR used at the checkpoints (re-stabilisation
every n_s slices, Method section).

A checkpoint orthonormalises the propagated basis U (N x N_sigma) as
W = U^T U = R^T R, Q = U R^{-1}.  In floating point Q loses orthogonality by
about eps cond(U)^2, and W stops being positive definite once eps cond(U)^2
reaches order one.  Starting from an orthonormal basis, the oracle's slice
products B_l = e^{-dtau K} D_l (random Ising field of the chain's Philox
stream) are applied n times to the 16x16 and 12x12 workloads' trial bases:

* at the configured interval n_s = 10, eps cond^2 < 1e-8 and Q^T Q = 1 to
  1e-10 (FP64);
* eps cond^2 grows by orders of magnitude per five slices and passes 1e-3
  before 30 slices, so the interval has a ceiling about three times above
  the one used, which the library flags (a Gram matrix that is not positive
  definite sets the singular flag) rather than repairs.

The checkpoint kernel forms R and R^{-1} in one elimination pass (W = L U
without pivoting, L^{-1} built in the eliminated slots); the identities it
relies on are checked here step by step against numpy's Cholesky factor.
"""
import numpy as np
import pytest

from oracle import philox, pqmc
from paper_2303_13403_amd.workloads import WORKLOADS

EPS = np.finfo(np.float64).eps


def _cholesky_qr(U):
    R = np.linalg.cholesky(U.T @ U).T
    return U @ np.linalg.inv(R)


def _propagated(name, sigma, n_max):
    """cond(U_n) and U_n for n = 1 .. n_max slices from an orthonormal basis."""
    w = WORKLOADS[name]
    m = pqmc.Model.from_workload(w)
    field = philox.initial_field(w.seed, 0, m.n_slices, m.N)
    U = np.linalg.qr(m.P[sigma])[0]
    out = []
    for n in range(1, n_max + 1):
        U = pqmc.apply_slice(m, field, n, sigma, U)
        out.append((np.linalg.cond(U), U.copy()))
    return out


@pytest.mark.parametrize("name", ["16x16", "12x12"])
@pytest.mark.parametrize("sigma", [1, -1])
def test_cholesky_qr_holds_at_the_configured_interval(name, sigma):
    steps = _propagated(name, sigma, 30)
    c10, U10 = steps[9]
    assert EPS * c10 ** 2 < 1e-8, f"{name}: cond {c10:.3g} after 10 slices"
    Q = _cholesky_qr(U10)
    orth = np.abs(Q.T @ Q - np.eye(Q.shape[1])).max()
    assert orth < 1e-10, f"{name}: |Q^T Q - 1| = {orth:.2g}"
    # the loss of orthogonality tracks eps cond^2 (within a small factor)
    assert orth < 100 * EPS * c10 ** 2
    # the margin closes a few tens of slices later
    c30 = steps[29][0]
    assert EPS * c30 ** 2 > 1e-3, f"{name}: cond {c30:.3g} after 30 slices"
    conds = [c for c, _ in steps]
    assert all(b > a for a, b in zip(conds[4::5], conds[9::5])), "cond grows along the pass"


def _eliminate_in_place(W):
    """The checkpoint kernel's single pass over the Gram matrix, step by step:
    below each pivot, row r -= l_rj row j over every column (the trailing block
    and the L^{-1} columns already formed), then slot (r, j) <- -l_rj; the
    multipliers come from row j (the trailing block is symmetric).  Returns
    the tile and the pivots U_jj (1 where a pivot is not positive)."""
    m = np.array(W, dtype=np.float64)
    n = len(m)
    piv = np.ones(n)
    for j in range(n):
        row = m[j].copy()
        u = row[j]
        ok = u > 0.0
        piv[j] = u if ok else 1.0
        below = np.arange(n) > j
        rl = np.where(below, row * (1.0 / u if ok else 0.0), 0.0)
        m -= np.outer(rl, row)
        m[below, j] = -rl[below]
    return m, piv


@pytest.mark.parametrize("n", [1, 2, 7, 40, 112, 128])
def test_single_pass_cholesky_inverse_identity(n):
    """W = L U without pivoting, with L^{-1} kept in the eliminated slots:
    R = diag(U)^{-1/2} U is the Cholesky factor (W = R^T R) and
    R^{-1} = (L^{-1})^T diag(U)^{-1/2}; log det R = (1/2) sum log U_jj."""
    rng = np.random.default_rng(n)
    M = rng.standard_normal((2 * n + 3, n))
    W = M.T @ M
    m, piv = _eliminate_in_place(W)
    Linv = np.tril(m, -1) + np.eye(n)
    U = np.triu(m)
    R = U / np.sqrt(piv)[:, None]
    Rinv = Linv.T / np.sqrt(piv)[None, :]
    R_ref = np.linalg.cholesky(W).T
    assert np.allclose(R, R_ref, rtol=0, atol=1e-12 * np.abs(R_ref).max())
    Rinv_ref = np.linalg.inv(R_ref)
    assert np.abs(Rinv - Rinv_ref).max() < 1e-12 * np.abs(Rinv_ref).max()
    assert np.abs(Rinv @ R - np.eye(n)).max() < 1e-12
    assert abs(0.5 * np.log(piv).sum() - np.log(np.diag(R_ref)).sum()) < 1e-12 * max(1.0, n)


def test_single_pass_cholesky_stays_finite_without_definiteness():
    """A finite symmetric matrix that is not positive definite (the second
    pivot is 1 - 4 = -3): the pass takes no multipliers at that step and
    reports the pivot as 1, so every entry stays finite (the kernel flags
    the chain)."""
    W = np.array([[1.0, 2.0, 0.5],
                  [2.0, 1.0, 0.3],
                  [0.5, 0.3, 2.0]])
    m, piv = _eliminate_in_place(W)
    assert piv[0] == 1.0 and piv[1] == 1.0 and piv[2] > 0.0
    assert np.isfinite(m).all()
