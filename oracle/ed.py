"""Fock-space exact diagonalisation and exact field enumeration (tiny clusters).

TEST INFRASTRUCTURE ONLY (see the package header).

These two routes compute the same Trotterised projector estimate

  E_Trot = <psi_N| P_g B^L H B^L P_g |psi_N> / <psi_N| P_g B^{2L} P_g |psi_N>,
  B = e^{-dtau K} e^{-dtau U sum_i n_i_up n_i_dn},  P_g = e^{-g sum_i n_i_up n_i_dn},

(Method section; H of Eq. 2) in two independent ways:

* ``trotter_energy_ed`` works in the many-body Fock space with the projector and
  the interaction written exactly as the paper writes them (n_up n_dn, no
  decoupling, no auxiliary field);
* ``enumerate_energy`` sums the determinant weights and Wick estimates of the
  auxiliary-field formulation over every field configuration, with no Monte
  Carlo.

Their agreement pins the decoupling (the spin-channel reading of Eq. 1), the
boundary slices, the Trotter order and the Wick estimators of ``pqmc``.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.linalg

from . import pqmc


def _states(n_sites, n_particles):
    return [sum(1 << i for i in occ)
            for occ in itertools.combinations(range(n_sites), n_particles)]


def _one_body(A, states):
    """Matrix of sum_ij A_ij c_i^dag c_j for one fermion species.

    Basis |b> = c^dag_{o1} c^dag_{o2} ... |0> with o1 < o2 < ... (bits of b)."""
    index = {b: k for k, b in enumerate(states)}
    n = A.shape[0]
    out = np.zeros((len(states), len(states)))
    for k, b in enumerate(states):
        for j in range(n):
            if not (b >> j) & 1:
                continue
            sj = (-1) ** bin(b & ((1 << j) - 1)).count("1")
            b1 = b ^ (1 << j)
            for i in range(n):
                if A[i, j] == 0.0 or (b1 >> i) & 1:
                    continue
                si = (-1) ** bin(b1 & ((1 << i) - 1)).count("1")
                out[index[b1 | (1 << i)], k] += A[i, j] * sj * si
    return out


def _slater(P, states):
    """Amplitudes of prod_n (sum_i P[i, n] c_i^dag)|0> on the occupation basis."""
    n = P.shape[0]
    amp = np.empty(len(states))
    for k, b in enumerate(states):
        rows = [i for i in range(n) if (b >> i) & 1]
        amp[k] = np.linalg.det(P[rows, :])
    return amp


def fock_operators(K, n_up, n_dn):
    """(Kinetic, double-occupancy count) as dense matrices on the
    (n_up, n_dn) sector; basis index = i_up * dim_dn + i_dn."""
    n = K.shape[0]
    su, sd = _states(n, n_up), _states(n, n_dn)
    Ku, Kd = _one_body(K, su), _one_body(K, sd)
    kin = np.kron(Ku, np.eye(len(sd))) + np.kron(np.eye(len(su)), Kd)
    dbl = np.array([bin(bu & bd).count("1") for bu in su for bd in sd], dtype=np.float64)
    return kin, dbl, su, sd


def fock_spin_afm(eps, su, sd, n):
    """sum_ij eps_i eps_j S_i . S_j as a dense matrix on the (n_up, n_dn)
    sector (basis index = i_up * dim_dn + i_dn), from the spin operators:

      S^z_i = (n_i,up - n_i,dn) / 2, diagonal;
      S^+_i S^-_j = c_i,up^dag c_j,up  c_i,dn c_j,dn^dag
                  = T^up_ij (x) (delta_ij - T^dn_ji),
      S^-_i S^+_j = (delta_ij - T^up_ji) (x) T^dn_ij,

    with T^s_ij the matrix of c_i,s^dag c_j,s on the species' occupation
    basis (every up operator is ordered before every down operator, and the
    pairs moved past each other are even, so no sign arises between species).
    """
    du, dd = len(su), len(sd)
    e = np.asarray(eps, dtype=np.float64)
    nu = np.array([[(b >> i) & 1 for i in range(n)] for b in su], dtype=np.float64)
    nd = np.array([[(b >> i) & 1 for i in range(n)] for b in sd], dtype=np.float64)
    mz = 0.5 * ((nu @ e)[:, None] - (nd @ e)[None, :]).ravel()     # sum_i eps_i S^z_i
    out = np.diag(mz * mz)
    Iu, Id = np.eye(du), np.eye(dd)
    for i in range(n):
        for j in range(n):
            Eij = np.zeros((n, n))
            Eij[i, j] = 1.0
            Eji = Eij.T.copy()
            Tu_ij, Tu_ji = _one_body(Eij, su), _one_body(Eji, su)
            Td_ij, Td_ji = _one_body(Eij, sd), _one_body(Eji, sd)
            dij = 1.0 if i == j else 0.0
            pm = np.kron(Tu_ij, dij * Id - Td_ji)
            mp = np.kron(dij * Iu - Tu_ji, Td_ij)
            out += e[i] * e[j] * 0.5 * (pm + mp)
    return out


def trotter_saf_ed(model: "pqmc.Model"):
    """S_AFM = <sum_ij eps_i eps_j S_i . S_j> / N^2 of the Trotterised projector
    estimate, by Fock-space linear algebra (the bra and ket of
    ``trotter_energy_ed``; l_half = 0 gives the Gutzwiller state's value)."""
    m = model
    kin, dbl, su, sd = fock_operators(m.K, m.n[1], m.n[-1])
    psi = np.kron(_slater(m.P[1], su), _slater(m.P[-1], sd))
    pg = np.exp(-m.g * dbl)
    eK = scipy.linalg.expm(-m.dtau * kin)
    eV = np.exp(-m.dtau * m.U * dbl)
    ket = pg * psi
    bra = pg * psi
    for _ in range(m.l_half):
        ket = eK @ (eV * ket)
        bra = eV * (eK.T @ bra)
    S = fock_spin_afm(m.eps, su, sd, m.N)
    return float(bra @ S @ ket / (bra @ ket)) / (m.N * m.N)


def trotter_energy_ed(model: "pqmc.Model"):
    """(E_Trot / N, D_Trot) by Fock-space linear algebra (no auxiliary field)."""
    m = model
    kin, dbl, su, sd = fock_operators(m.K, m.n[1], m.n[-1])
    psi = np.kron(_slater(m.P[1], su), _slater(m.P[-1], sd))
    pg = np.exp(-m.g * dbl)
    eK = scipy.linalg.expm(-m.dtau * kin)
    eV = np.exp(-m.dtau * m.U * dbl)
    ket = pg * psi
    bra = pg * psi
    for _ in range(m.l_half):
        ket = eK @ (eV * ket)
        bra = eV * (eK.T @ bra)          # bra B = (B^T bra^T)^T
    H = kin + m.U * np.diag(dbl)
    norm = bra @ ket
    return float(bra @ H @ ket / norm) / m.N, float(bra @ (dbl * ket) / norm) / m.N


def trotter_energy_ed_projector(model: "pqmc.Model"):
    """Variational energy of the Gutzwiller state at Theta = 0 (l_half = 0):
    <psi_G|H|psi_G>/<psi_G|psi_G> with psi_G = P_g psi_N (Method section)."""
    m = model
    kin, dbl, su, sd = fock_operators(m.K, m.n[1], m.n[-1])
    psi = np.exp(-m.g * dbl) * np.kron(_slater(m.P[1], su), _slater(m.P[-1], sd))
    H = kin + m.U * np.diag(dbl)
    return float(psi @ H @ psi / (psi @ psi)) / m.N


def enumerate_energy(model: "pqmc.Model", chunk: int = 1 << 14, with_saf: bool = False):
    """(E/N, D, <sign>) summed exactly over all 2^{(M+2) N} field configurations
    ((E/N, D, S_AFM, <sign>) with ``with_saf``, S_AFM from the oracle's Wick
    estimator ``pqmc.structure_factor``).

    Weight W(s) = W_up(s) W_dn(s), W_sigma = det(P^T S_{M+1} ... S_0 P); the
    decoupling prefactors are the same for every configuration and cancel."""
    m = model
    n_f = m.n_slices * m.N
    if n_f > 24:
        raise ValueError("too many fields to enumerate")
    total = 1 << n_f
    num_e = num_d = num_s = den = asum = 0.0
    for start in range(0, total, chunk):
        idx = np.arange(start, min(total, start + chunk), dtype=np.int64)
        bits = ((idx[:, None] >> np.arange(n_f)) & 1).astype(np.int8)
        fields = (2 * bits - 1).reshape(-1, m.n_slices, m.N)
        W = np.ones(len(idx))
        G = {}
        for s in pqmc.SPINS:
            R = np.broadcast_to(m.P[s], (len(idx),) + m.P[s].shape).copy()
            Lt = R.copy()
            for l in range(0, m.l_half + 1):
                d = np.exp(s * m.coupling(l) * fields[:, l, :].astype(np.float64))
                R = d[:, :, None] * R
                if m.is_bulk(l):
                    R = m.Km @ R
            for l in range(m.M + 1, m.l_half, -1):
                if m.is_bulk(l):
                    Lt = m.Km @ Lt
                d = np.exp(s * m.coupling(l) * fields[:, l, :].astype(np.float64))
                Lt = d[:, :, None] * Lt
            X = np.swapaxes(Lt, 1, 2) @ R
            W = W * np.linalg.det(X)
            G[s] = np.eye(m.N) - R @ np.linalg.solve(X, np.swapaxes(Lt, 1, 2))
        ekin = sum(np.einsum("ij,bji->b", m.K, np.eye(m.N) - G[s]) for s in pqmc.SPINS)
        docc = (1.0 - np.diagonal(G[1], axis1=1, axis2=2)) * \
               (1.0 - np.diagonal(G[-1], axis1=1, axis2=2))
        e = (ekin + m.U * docc.sum(axis=1)) / m.N
        num_e += float(np.sum(W * e))
        num_d += float(np.sum(W * docc.mean(axis=1)))
        if with_saf:
            saf = np.array([pqmc.structure_factor(m.eps, G[1][b], G[-1][b])
                            for b in range(len(idx))])
            num_s += float(np.sum(W * saf))
        den += float(np.sum(W))
        asum += float(np.sum(np.abs(W)))
    if with_saf:
        return num_e / den, num_d / den, num_s / den, den / asum
    return num_e / den, num_d / den, den / asum


# --------------------------------------------------------------------------- #
# spinless t-V model ("Repulsive spinless honeycomb model", Eq. 3)
# --------------------------------------------------------------------------- #
def tv_fock(model):
    """(kinetic matrix, occupations, states) on the N/2-particle sector of one
    species."""
    states = _states(model.N, model.n[1])
    occ = np.array([[(b >> i) & 1 for i in range(model.N)] for b in states], dtype=np.float64)
    return _one_body(model.K, states), occ, states


def tv_trotter_ed(model):
    """(E/N, NN density correlation, S_CDW) of the Trotterised projector
    estimate with the operators as the paper writes them: the interaction
    V sum_b (n_i - 1/2)(n_j - 1/2) and the projector exp(-g sum_b n_i n_j),
    no decoupling."""
    m = model
    kin, occ, states = tv_fock(m)
    i, j = m.bonds[:, 0], m.bonds[:, 1]
    hv = ((occ[:, i] - 0.5) * (occ[:, j] - 0.5)).sum(axis=1)
    nn = (occ[:, i] * occ[:, j]).sum(axis=1)
    cdw = ((occ - 0.5) @ m.eps) ** 2
    psi = np.exp(-m.g * nn) * _slater(m.P[1], states)
    eK = scipy.linalg.expm(-m.dtau * kin)
    eV = np.exp(-m.dtau * m.V * hv)
    ket, bra = psi.copy(), psi.copy()
    for _ in range(m.l_half):
        ket = eK @ (eV * ket)
        bra = eV * (eK.T @ bra)
    norm = bra @ ket
    H = kin + m.V * np.diag(hv)
    return (float(bra @ H @ ket / norm) / m.N, float(bra @ (nn * ket) / norm) / m.n_bonds,
            float(bra @ (cdw * ket) / norm) / (m.N * m.N))


def tv_enumerate(model, chunk: int = 1 << 12):
    """(E/N, NN density correlation, S_CDW, <sign>) summed exactly over all
    2^{(M+2) N_b} bond-field configurations with the oracle's Wick estimators
    (``tv.estimators``); the decoupling prefactors are equal for every
    configuration and cancel."""
    from . import tv

    m = model
    n_f = m.n_slices * m.n_bonds
    if n_f > 20:
        raise ValueError("too many fields to enumerate")
    total = 1 << n_f
    num = np.zeros(3)
    den = asum = 0.0
    for start in range(0, total, chunk):
        idx = np.arange(start, min(total, start + chunk), dtype=np.int64)
        bits = ((idx[:, None] >> np.arange(n_f)) & 1).astype(np.int8)
        fields = (2 * bits - 1).reshape(-1, m.n_slices, m.n_bonds)
        for f in fields:
            R = m.P[1].copy()
            for l in range(0, m.l_half + 1):
                R = m.diag(f[l], l)[:, None] * R
                if m.is_bulk(l):
                    R = m.Km @ R
            Lt = m.P[1].copy()
            for l in range(m.M + 1, m.l_half, -1):
                if m.is_bulk(l):
                    Lt = m.Km @ Lt
                Lt = m.diag(f[l], l)[:, None] * Lt
            X = Lt.T @ R
            W = float(np.linalg.det(X))
            G = np.eye(m.N) - R @ np.linalg.solve(X, Lt.T)
            num += W * np.array(tv.estimators(m, G))
            den += W
            asum += abs(W)
    return tuple(float(x) for x in num / den) + (den / asum,)
