"""Serial FP64 projector determinant QMC of the spinless t-V model.

TEST INFRASTRUCTURE ONLY (see the package header).

What is computed (arXiv:2303.13403, "Repulsive spinless honeycomb model",
Eq. 3 and the trial state that follows it):

* H = K + V sum_<ij> (n_i - 1/2)(n_j - 1/2), K_ij = -t on nearest-neighbour
  bonds, one fermion species at half filling (N/2 particles);
* trial |psi_T> = exp(-g sum_<ij> n_i n_j) |psi_C>, |psi_C> the N/2 lowest
  orbitals of K + Delta_C diag(eps) (CDW mean field, eps = +1 on A, -1 on B);
* estimand as for the Hubbard model: <psi_T| e^{-Theta H} O e^{-Theta H} |psi_T>
  / <psi_T| e^{-2 Theta H} |psi_T>, L_half slices of dtau per side,
  B = e^{-dtau K} e^{-dtau H_V}.

Readings (the paper names the density channel but prints no decoupling):

* per bond b = (i, j), i on sublattice A: since (n_i - n_j)^2 = n_i + n_j -
  2 n_i n_j for occupation numbers,
    exp(-x (n_i - 1/2)(n_j - 1/2)) = 1/2 e^{-x/4} sum_{s=+-1} e^{c s (n_i - n_j)},
    cosh c = e^{x/2},
  with x = dtau V on the M = 2 L_half bulk slices (coupling alpha) and x = g on
  the boundary slices 0 and M+1 (coupling lambda).  exp(-g n_i n_j) differs
  from exp(-g (n_i - 1/2)(n_j - 1/2)) by exp(-g (n_i + n_j)/2 + g/4), whose
  product over bonds is a constant at fixed particle number when every site has
  the same number of bonds (true on the periodic honeycomb lattice and the
  ring), so it is dropped;
* D_l = diag(exp(c_l m_{l,k})), m_{l,k} = sum over the bonds b of site k of
  +s_{l,b} (k the A end) or -s_{l,b} (k the B end); S_l = K_l D_l as for the
  Hubbard model (K_l = e^{-dtau K} in the bulk, 1 on the boundary slices);
* flipping s_{l,b} multiplies D_l at i by 1 + Delta_i, Delta_i = e^{-2 c s} - 1,
  and at j by 1 + Delta_j, Delta_j = e^{+2 c s} - 1.  With X = 1 - G in the
  frame where D_l acts, the ratio is det(1 + Delta_F X[F, F]) over F = {i, j}
  (matrix determinant lemma) and the update is the Woodbury form
  G' = G - G[:, F] (1 + Delta_F X[F, F])^{-1} Delta_F X[F, :];
* the weight can be negative (the density channel is not sign-free, as the
  paper states): Metropolis on |r|, the sign multiplied by sgn r;
* bonds are proposed in the order of the bond list within a slice (an input);
  otherwise sweeps, checkpoints and stabilisation follow ``pqmc``;
* estimators per field (Wick, one species, Gb_ij = <c_i^dag c_j> = delta_ij -
  G_ji): <n_i n_j> = Gb_ii Gb_jj + Gb_ij G_ij (i != j), <n_i n_i> = Gb_ii;
  E/N = [sum_ij K_ij Gb_ij + V sum_b <(n_i - 1/2)(n_j - 1/2)>] / N, the
  nearest-neighbour density correlation (1/N_b) sum_b <n_i n_j>, and the CDW
  structure factor S_CDW = (1/N^2) sum_ij eps_i eps_j <(n_i - 1/2)(n_j - 1/2)>
  (the paper defers its definitions to supplementary material that is not
  available; this is the standard staggered density correlation).
"""
from __future__ import annotations

import math

import numpy as np

from . import philox
from .pqmc import (Chain, apply_slice, apply_slice_left, hopping_exponentials, hs_coupling,
                   neel_trial)


class TVModel:
    """All inputs of one spinless t-V chain.  Offers the interface of
    ``pqmc.Model`` that the slice-product functions use (``diag``, ``Km``,
    ``is_bulk``, ``P``, ``M``) with the single species labelled sigma = +1."""

    def __init__(self, K, eps, bonds, V, dtau, l_half, delta_c, g, stab_interval,
                 n_particles=None, gap_tol=1e-6):
        self.K = np.array(K, dtype=np.float64)
        self.N = self.K.shape[0]
        self.eps = np.asarray(eps, dtype=np.float64)
        self.bonds = np.asarray(bonds, dtype=np.int64).reshape(-1, 2)
        self.n_bonds = len(self.bonds)
        self.V, self.dtau, self.g, self.delta_c = float(V), float(dtau), float(g), float(delta_c)
        n_p = self.N // 2 if n_particles is None else int(n_particles)
        self.n = {1: n_p}
        self.l_half = int(l_half)
        self.M = 2 * self.l_half
        self.n_slices = self.M + 2
        self.n_s = int(stab_interval)
        self.alpha = hs_coupling(self.dtau * self.V)
        self.lam = hs_coupling(self.g)
        self.Km, self.Kp = hopping_exponentials(self.K, self.dtau)
        P, _, gap = neel_trial(self.K, self.eps, self.delta_c, n_p, 1)
        if gap < gap_tol:
            raise ValueError(f"degenerate CDW trial state: gap {gap:.3e}")
        self.P = {1: P}
        # incidence: +1 at a bond's A end, -1 at its B end
        self.inc = np.zeros((self.N, self.n_bonds))
        for b, (i, j) in enumerate(self.bonds):
            self.inc[i, b] += 1.0
            self.inc[j, b] -= 1.0
        ck = {-1, self.l_half, self.M + 1}
        if self.n_s > 0:
            ck |= {j * self.n_s for j in range(1, self.M // self.n_s + 1)}
        self.checkpoints = sorted(ck)

    @classmethod
    def from_workload(cls, w, **over):
        K, eps, bonds = w.lattice()
        kw = dict(K=K, eps=eps, bonds=bonds, V=w.V, dtau=w.dtau, l_half=w.l_half,
                  delta_c=w.delta_c, g=w.g, stab_interval=w.stab_interval)
        kw.update(over)
        return cls(**kw)

    def coupling(self, l: int) -> float:
        return self.lam if l in (0, self.M + 1) else self.alpha

    def is_bulk(self, l: int) -> bool:
        return 1 <= l <= self.M

    def site_exponent(self, field_row):
        """m_k = sum_b inc[k, b] s_b for one slice's bond fields."""
        return self.inc @ np.asarray(field_row, dtype=np.float64)

    def diag(self, field_row, l, sigma=1):
        """Diagonal of D_l: exp(c_l m_k)."""
        return np.exp(self.coupling(l) * self.site_exponent(field_row))

    def flip_deltas(self, s_lb, l):
        """(Delta_i, Delta_j) of flipping the field s_lb of bond (i, j)."""
        c = self.coupling(l)
        return math.exp(-2.0 * c * s_lb) - 1.0, math.exp(2.0 * c * s_lb) - 1.0


def green_at(model, field, p):
    """G_p with both products orthonormalised after every slice."""
    R = model.P[1].copy()
    for l in range(0, p + 1):
        R, _ = np.linalg.qr(apply_slice(model, field, l, 1, R))
    Lt = model.P[1].copy()
    for l in range(model.M + 1, p, -1):
        Lt, _ = np.linalg.qr(apply_slice_left(model, field, l, 1, Lt))
    X = Lt.T @ R
    return np.eye(model.N) - R @ np.linalg.solve(X, Lt.T)


def weight(model, field):
    """W = det(P^T S_{M+1} ... S_0 P) (plain product: small cases only)."""
    R = model.P[1].copy()
    for l in range(0, model.M + 2):
        R = apply_slice(model, field, l, 1, R)
    return float(np.linalg.det(model.P[1].T @ R))


def estimators(model, G):
    """(E/N, NN density correlation, S_CDW) at one field configuration."""
    N = model.N
    I = np.eye(N)
    Gb = I - G.T
    n = np.diag(Gb).copy()
    C = np.outer(n, n) + Gb * G          # <n_i n_j> for i != j
    np.fill_diagonal(C, n)               # <n_i n_i> = <n_i>
    ekin = float(np.sum(model.K * Gb))
    i, j = model.bonds[:, 0], model.bonds[:, 1]
    nn = C[i, j]
    ev = float(np.sum(nn - 0.5 * (n[i] + n[j]) + 0.25))
    Cc = C - 0.5 * (n[:, None] + n[None, :]) + 0.25
    e = model.eps
    s_cdw = float(e @ Cc @ e) / (N * N)
    return (ekin + model.V * ev) / N, float(nn.mean()), s_cdw


class TVChain:
    """One Markov chain of the spinless t-V model: bond field, Green's
    function, checkpoint stack, sign (single species)."""

    def __init__(self, model: TVModel, seed: int = 13403, chain_id: int = 0, field=None):
        self.m = model
        self.seed, self.chain_id = int(seed), int(chain_id)
        if field is None:
            field = philox.initial_field(seed, chain_id, model.n_slices, model.n_bonds)
        self.field = np.array(field, dtype=np.int8).reshape(model.n_slices, model.n_bonds).copy()
        self.sweep_index = 0
        self.measurements = []          # (sign, E/N, NN density correlation, S_CDW)
        self.ratios = {}                # (sweep, l, b) -> (r, u, accepted)
        self.checkpoint_greens = []     # (sweep, p, G, drift, field snapshot)
        self.checkpoint_logdets = []    # (sweep, p, (log|W|, sign))
        self.sign_mismatches = 0
        self.max_drift = 0.0
        self.record_ratios = False
        self.record_greens = False
        self.follow = None
        self.follow_tol = 0.0
        self.follow_violations = []
        self.init_trial()

    def init_trial(self):
        m = self.m
        self.stack = {(m.M + 1): (m.P[1].copy(), 0.0, 1)}
        run = (m.P[1].copy(), 0.0, 1)
        for l in range(m.M + 1, -1, -1):
            Lt, lg, sg = run
            run = (apply_slice_left(m, self.field, l, 1, Lt), lg, sg)
            p = l - 1
            if p in m.checkpoints:
                run = Chain._orthonormalise(*run)
                self.stack[p] = run
        QL, _, sgL = self.stack[-1]
        X = QL.T @ m.P[1]
        sgX, _ = np.linalg.slogdet(X)
        self.G = np.eye(m.N) - m.P[1] @ np.linalg.solve(X, QL.T)
        self.sign = int(sgL * np.sign(sgX))
        self.sweep_index = 0

    def _flips(self, l):
        m = self.m
        u_all = philox.accept_uniforms(self.seed, self.chain_id, self.sweep_index, l, m.n_bonds)
        for b in range(m.n_bonds):
            i, j = int(m.bonds[b, 0]), int(m.bonds[b, 1])
            F = [i, j]
            s_lb = int(self.field[l, b])
            d = np.array(m.flip_deltas(s_lb, l))
            G = self.G
            XF = -G[np.ix_(F, F)] + np.eye(2)          # X[F, F] = 1 - G[F, F]
            A = np.eye(2) + d[:, None] * XF
            r = float(np.linalg.det(A))
            u = float(u_all[b])
            accept = u < abs(r)
            if self.follow is not None:
                forced = bool(self.follow[l, b] != self.field[l, b])
                if forced != accept:
                    if abs(u - abs(r)) > self.follow_tol * max(abs(r), 1.0):
                        self.follow_violations.append((self.sweep_index, l, b, u, abs(r)))
                    accept = forced
            if self.record_ratios:
                self.ratios[(self.sweep_index, l, b)] = (r, u, accept)
            if accept:
                XrowF = -G[F, :].copy()
                XrowF[0, i] += 1.0
                XrowF[1, j] += 1.0
                self.G = G - G[:, F] @ np.linalg.solve(A, d[:, None] * XrowF)
                self.field[l, b] = -s_lb
                self.sign *= 1 if r > 0 else -1

    def _checkpoint(self, p, run, up):
        m = self.m
        Q, lg, sg = Chain._orthonormalise(*run)
        Qo, lgo, sgo = self.stack[p]
        R, Lt = (Q, Qo) if up else (Qo, Q)
        X = Lt.T @ R
        sgX, lgX = np.linalg.slogdet(X)
        Gf = np.eye(m.N) - R @ np.linalg.solve(X, Lt.T)
        drift = float(np.max(np.abs(self.G - Gf)))
        self.G = Gf
        self.stack[p] = (Q, lg, sg)
        logdet = (lg + lgo + float(lgX), int(sg * sgo * np.sign(sgX)))
        self.checkpoint_logdets.append((self.sweep_index, p, logdet))
        self.max_drift = max(self.max_drift, drift)
        if logdet[1] != self.sign:
            self.sign_mismatches += 1
            self.sign = logdet[1]
        if self.record_greens:
            self.checkpoint_greens.append((self.sweep_index, p, Gf.copy(), drift, self.field.copy()))
        return (Q, lg, sg)

    def _measure(self):
        e, nn, s = estimators(self.m, self.G)
        self.measurements.append((self.sign, e, nn, s))

    def _up_pass(self, measure):
        m = self.m
        self.stack[-1] = (m.P[1].copy(), 0.0, 1)
        run = (m.P[1].copy(), 0.0, 1)
        for l in range(0, m.M + 2):
            d = m.diag(self.field[l], l)
            self.G = d[:, None] * self.G / d[None, :]
            self._flips(l)
            if m.is_bulk(l):
                self.G = m.Km @ self.G @ m.Kp
            B, lg, sg = run
            run = (apply_slice(m, self.field, l, 1, B), lg, sg)
            if l in m.checkpoints:
                run = self._checkpoint(l, run, up=True)
            if l == m.l_half and measure:
                self._measure()

    def _down_pass(self, measure):
        m = self.m
        self.stack[m.M + 1] = (m.P[1].copy(), 0.0, 1)
        run = (m.P[1].copy(), 0.0, 1)
        for l in range(m.M + 1, -1, -1):
            if m.is_bulk(l):
                self.G = m.Kp @ self.G @ m.Km
            self._flips(l)
            d = m.diag(self.field[l], l)
            self.G = self.G * d[None, :] / d[:, None]
            B, lg, sg = run
            run = (apply_slice_left(m, self.field, l, 1, B), lg, sg)
            p = l - 1
            if p in m.checkpoints:
                run = self._checkpoint(p, run, up=False)
            if p == m.l_half and measure:
                self._measure()

    def sweep(self, n: int = 1, measure: bool = True):
        for _ in range(n):
            if self.sweep_index % 2 == 0:
                self._up_pass(measure)
            else:
                self._down_pass(measure)
            self.sweep_index += 1
        return self

    def sweep_following(self, field_after, tol):
        """One pass that takes each acceptance from ``field_after``, recording
        every decision that disagrees by more than ``tol`` relative to its
        threshold."""
        self.follow = np.asarray(field_after, dtype=np.int8).reshape(self.field.shape)
        self.follow_tol = float(tol)
        try:
            self.sweep(1)
        finally:
            self.follow = None
        return self.follow_violations


def free_energy_closed_form(model: TVModel, theta: float) -> float:
    """V = 0, g = 0: E/N = sum_ij K_ij <c_i^dag c_j> / N with R = e^{-Theta K} P,
    L = P^T e^{-Theta K} (no Trotter error without interaction)."""
    w, Vv = np.linalg.eigh(model.K)
    E = (Vv * np.exp(-theta * w)) @ Vv.T
    R = E @ model.P[1]
    G = np.eye(model.N) - R @ np.linalg.solve(R.T @ R, R.T)
    return float(np.sum(model.K * (np.eye(model.N) - G.T))) / model.N
