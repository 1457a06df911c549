"""Serial FP64 projector determinant QMC with a Gutzwiller-projected Neel trial.

TEST INFRASTRUCTURE ONLY (see the package header).

What is computed (arXiv:2303.13403, Method section and the Hubbard section):

* estimand: <psi_T| e^{-Theta H} O e^{-Theta H} |psi_T> / <psi_T| e^{-2 Theta H} |psi_T>
  with |psi_T> = exp(-g sum_i n_i_up n_i_dn) |psi_N> (Method section; the
  denominator's trial state is read as psi_T), Trotterised with L_half slices
  of dtau on each side, B = e^{-dtau K} e^{-dtau V};
* the Gutzwiller factor is decoupled with a discrete field per site.  Eq. 1 as
  printed does not hold for any occupation; the exact identity used here is
  exp(-x (n_up - 1/2)(n_dn - 1/2)) = 1/2 e^{-x/4} sum_{s=+-1} e^{c s (n_up - n_dn)},
  cosh c = e^{x/2}, which differs from exp(-g n_up n_dn) only by a constant at
  fixed particle number.  With x = g it gives the two boundary slices (ket slice
  0 and bra slice M+1); with x = dtau*U it is Hirsch's spin-channel
  decoupling of the Hubbard term on the M = 2 L_half bulk slices;
* the Neel trial |psi_N> (Hubbard section): for spin sigma = +1 (up), -1 (down)
  the lowest N_sigma orbitals of h_sigma = K + sigma M_N diag(eps) (+ an
  optional trial-only potential), eps_i = +1 on sublattice A and -1 on B.

Conventions (written out because the paper defers them to standard PQMC):

* slice matrices S_l = K_l D_l, D_l = diag(exp(sigma c_l s_{l,i})), K_l = e^{-dtau K}
  for 1 <= l <= M and the identity on the boundary slices 0 and M+1; c_l is the
  projector coupling lambda on the boundary slices and alpha on the bulk ones;
* position p in {-1, ..., M+1} means "after slice p":
  R_p = S_p ... S_0 P,  L_p = P^T S_{M+1} ... S_{p+1},
  G_p = 1 - R_p (L_p R_p)^{-1} L_p  (G_ij = <c_i c_j^dagger>);
* flipping s_{l,i} multiplies D_l by (1 + Delta e_i e_i^T), Delta = e^{-2 sigma c_l s} - 1;
  with G in the frame where D_l acts, the weight ratio is 1 + Delta (1 - G_ii)
  (matrix determinant lemma) and G' = G - Delta/r G e_i (e_i^T - G[i, :])
  (Sherman-Morrison);
* Metropolis on the absolute weight: accept iff u < |r_up r_dn|; the sign of the
  weight is multiplied by sgn(r_up r_dn) on acceptance;
* a sweep is one pass over the slices, upward (0 .. M+1) on even sweep indices
  and downward (M+1 .. 0) on odd ones; sites ascend within a slice;
* checkpoints C = {-1, L_half, M+1} U {j n_s : 1 <= j n_s <= M}: the propagated
  basis is QR-orthonormalised and G recomputed from the stored opposite-side
  basis; measurement at position L_half (tau = Theta) once per pass;
* energy per site E/N = [sum_sigma sum_ij K_ij <c_i^dag c_j> + U sum_i <n_up n_dn>]/N
  (Eq. 2 with U n_up n_dn), double occupancy D = sum_i <n_up n_dn> / N, by Wick.
"""
from __future__ import annotations

import math

import numpy as np

from . import philox

SPINS = (1, -1)


# --------------------------------------------------------------------------- #
# model setup (Method section; Hubbard section, Eq. 2 and the Neel trial)
# --------------------------------------------------------------------------- #
def hs_coupling(x: float) -> float:
    """Coupling c of the discrete decoupling, cosh c = exp(x/2) (x >= 0)."""
    if x < 0:
        raise ValueError("decoupling needs x >= 0 (repulsive U, g >= 0)")
    return float(np.arccosh(np.exp(0.5 * x)))


def hopping_exponentials(K: np.ndarray, dtau: float):
    """(e^{-dtau K}, e^{+dtau K}) from the eigendecomposition of symmetric K."""
    w, V = np.linalg.eigh(K)
    return (V * np.exp(-dtau * w)) @ V.T, (V * np.exp(dtau * w)) @ V.T


def neel_trial(K, eps, m_neel, n_sigma, sigma, potential=None):
    """Lowest n_sigma orbitals of h = K + sigma M_N diag(eps) (+ diag(potential)).

    Returns (P, energies, gap) with gap = e_{n_sigma} - e_{n_sigma - 1}
    (0-based; +inf when the band is full).
    """
    h = np.array(K, dtype=np.float64) + sigma * m_neel * np.diag(np.asarray(eps, np.float64))
    if potential is not None:
        h = h + np.diag(np.asarray(potential, np.float64))
    w, V = np.linalg.eigh(h)
    gap = w[n_sigma] - w[n_sigma - 1] if n_sigma < len(w) else math.inf
    return V[:, :n_sigma].copy(), w, gap


class Model:
    """All inputs of one chain (the Hamiltonian, the trial state and the
    Trotter/stabilisation parameters)."""

    def __init__(self, K, eps, U, n_up, n_dn, dtau, l_half, m_neel, g,
                 stab_interval, potential=None, gap_tol=1e-6):
        self.K = np.array(K, dtype=np.float64)
        self.N = self.K.shape[0]
        self.eps = np.asarray(eps, dtype=np.float64)
        self.U, self.dtau, self.g, self.m_neel = float(U), float(dtau), float(g), float(m_neel)
        self.n = {1: int(n_up), -1: int(n_dn)}
        self.l_half = int(l_half)
        self.M = 2 * self.l_half
        self.n_slices = self.M + 2
        self.n_s = int(stab_interval)
        self.alpha = hs_coupling(self.dtau * self.U)
        self.lam = hs_coupling(self.g)
        self.Km, self.Kp = hopping_exponentials(self.K, self.dtau)
        self.P = {}
        self.gap = {}
        for s in SPINS:
            P, _, gap = neel_trial(self.K, self.eps, self.m_neel, self.n[s], s, potential)
            if gap < gap_tol:
                raise ValueError(f"degenerate trial state for spin {s}: gap {gap:.3e}")
            self.P[s], self.gap[s] = P, gap
        ck = {-1, self.l_half, self.M + 1}
        if self.n_s > 0:
            ck |= {j * self.n_s for j in range(1, self.M // self.n_s + 1)}
        self.checkpoints = sorted(ck)

    @classmethod
    def from_workload(cls, w, **over):
        K, eps, _ = w.lattice()
        kw = dict(K=K, eps=eps, U=w.U, n_up=w.n_up, n_dn=w.n_dn, dtau=w.dtau,
                  l_half=w.l_half, m_neel=w.m_neel, g=w.g,
                  stab_interval=w.stab_interval, potential=w.trial_potential())
        kw.update(over)
        return cls(**kw)

    def coupling(self, l: int) -> float:
        return self.lam if l in (0, self.M + 1) else self.alpha

    def is_bulk(self, l: int) -> bool:
        return 1 <= l <= self.M

    def diag(self, field_row, l, sigma):
        """Diagonal of D_l for spin sigma: exp(sigma c_l s_{l,i})."""
        return np.exp(sigma * self.coupling(l) * field_row.astype(np.float64))

    def flip_delta(self, s_li, l, sigma):
        """Delta such that flipping s_{l,i} multiplies D_l[i,i] by 1 + Delta."""
        return math.exp(-2.0 * sigma * self.coupling(l) * s_li) - 1.0


# --------------------------------------------------------------------------- #
# fixed-field quantities (no Monte Carlo): used by the chain and as pins
# --------------------------------------------------------------------------- #
def apply_slice(model, field, l, sigma, X):
    """S_l X = K_l D_l X."""
    Y = model.diag(field[l], l, sigma)[:, None] * X
    return model.Km @ Y if model.is_bulk(l) else Y


def apply_slice_left(model, field, l, sigma, Lt):
    """(L S_l)^T = D_l K_l L^T for a basis stored as L^T (K symmetric)."""
    Y = model.Km @ Lt if model.is_bulk(l) else Lt
    return model.diag(field[l], l, sigma)[:, None] * Y


def right_basis(model, field, p, sigma):
    """R_p = S_p ... S_0 P (plain product, no stabilisation: small cases only)."""
    R = model.P[sigma].copy()
    for l in range(0, p + 1):
        R = apply_slice(model, field, l, sigma, R)
    return R


def left_basis_T(model, field, p, sigma):
    """L_p^T with L_p = P^T S_{M+1} ... S_{p+1} (plain product)."""
    Lt = model.P[sigma].copy()
    for l in range(model.M + 1, p, -1):
        Lt = apply_slice_left(model, field, l, sigma, Lt)
    return Lt


def green_from_bases(R, Lt):
    """G = 1 - R (L R)^{-1} L for L = Lt^T."""
    X = Lt.T @ R
    return np.eye(R.shape[0]) - R @ np.linalg.solve(X, Lt.T)


def green_stable(model, field, p, sigma):
    """G_p with both products orthonormalised after every slice (exact mode)."""
    R = model.P[sigma].copy()
    for l in range(0, p + 1):
        R, _ = np.linalg.qr(apply_slice(model, field, l, sigma, R))
    Lt = model.P[sigma].copy()
    for l in range(model.M + 1, p, -1):
        Lt, _ = np.linalg.qr(apply_slice_left(model, field, l, sigma, Lt))
    return green_from_bases(R, Lt)


def weight(model, field, sigma):
    """W_sigma = det(P^T S_{M+1} ... S_0 P) (plain product: small cases only)."""
    R = right_basis(model, field, model.M + 1, sigma)
    return float(np.linalg.det(model.P[sigma].T @ R))


def estimators(model, Gup, Gdn):
    """(E/N, D) at one field configuration, from Wick's theorem.

    <c_i^dag c_j> = delta_ij - G_ji;  <n_up n_dn>_i = (1 - Gup_ii)(1 - Gdn_ii).
    """
    N = model.N
    ekin = 0.0
    for G in (Gup, Gdn):
        ekin += float(np.sum(model.K * (np.eye(N) - G.T)))
    docc = (1.0 - np.diag(Gup)) * (1.0 - np.diag(Gdn))
    return (ekin + model.U * float(docc.sum())) / N, float(docc.mean())


def structure_factor(eps, Gup, Gdn):
    """Staggered spin structure factor S_AFM = (1/N^2) sum_ij eps_i eps_j
    <S_i . S_j> at one field configuration, written out term by term with
    Wick's theorem (the spin sectors do not mix: the field couples to n_up -
    n_dn).  With Gb_ij = <c_i^dag c_j> = delta_ij - G_ji and G_ij = <c_i c_j^dag>
    for each spin:

      <S^z_i S^z_j> = 1/4 sum_{s,s'} s s' <n_is n_js'>,
        <n_is n_js>  = Gb^s_ii Gb^s_jj + Gb^s_ij G^s_ij,
        <n_is n_j-s> = Gb^s_ii Gb^-s_jj;
      <S^+_i S^-_j> = <c_i,up^dag c_j,up> <c_i,dn c_j,dn^dag> = Gb^up_ij G^dn_ij,
      <S^-_i S^+_j> = Gb^dn_ij G^up_ij;
      S_i . S_j = S^z_i S^z_j + (S^+_i S^-_j + S^-_i S^+_j) / 2.
    """
    N = len(eps)
    e = np.asarray(eps, dtype=np.float64)
    I = np.eye(N)
    Gbu, Gbd = I - Gup.T, I - Gdn.T
    nu, nd = np.diag(Gbu), np.diag(Gbd)
    total = 0.0
    for i in range(N):
        for j in range(N):
            uu = nu[i] * nu[j] + Gbu[i, j] * Gup[i, j]
            dd = nd[i] * nd[j] + Gbd[i, j] * Gdn[i, j]
            ud = nu[i] * nd[j]
            du = nd[i] * nu[j]
            szsz = 0.25 * (uu + dd - ud - du)
            flip = 0.5 * (Gbu[i, j] * Gdn[i, j] + Gbd[i, j] * Gup[i, j])
            total += e[i] * e[j] * (szsz + flip)
    return total / (N * N)


# --------------------------------------------------------------------------- #
# the Markov chain
# --------------------------------------------------------------------------- #
class Chain:
    """One Markov chain: field, Green's functions, checkpoint stack, sign.

    ``exact=True`` recomputes G from scratch (orthonormalised products) at every
    slice instead of wrapping it; used as a pin of the wrapped sweep.
    """

    def __init__(self, model: Model, seed: int = 13403, chain_id: int = 0,
                 field=None, exact: bool = False):
        self.m = model
        self.seed, self.chain_id = int(seed), int(chain_id)
        self.exact = exact
        if field is None:
            field = philox.initial_field(seed, chain_id, model.n_slices, model.N)
        self.field = np.array(field, dtype=np.int8).reshape(model.n_slices, model.N).copy()
        self.sweep_index = 0
        self.measurements = []          # (sign, E/N, D, S_AFM) per measurement
        self.ratios = {}                # (sweep, l, i) -> (r_up, r_dn, u, accepted)
        self.checkpoint_greens = []     # (sweep, p, G_up, G_dn, drift, field snapshot)
        self.checkpoint_logdets = []    # (sweep, p, {spin: (log|det(L_p R_p)|, sign)})
        self.sign_mismatches = 0
        self.max_drift = 0.0
        self.record_ratios = False
        self.record_greens = False
        self.follow = None              # externally decided acceptances (follow mode)
        self.follow_tol = 0.0
        self.follow_violations = []
        self.init_trial()

    # -- initialisation: build the L stack from the top, G at position -1 -----
    def init_trial(self):
        m = self.m
        self.stack = {}
        for s in SPINS:
            self.stack[(m.M + 1, s)] = (m.P[s].copy(), 0.0, 1)
        run = {s: (m.P[s].copy(), 0.0, 1) for s in SPINS}
        for l in range(m.M + 1, -1, -1):
            for s in SPINS:
                Lt, lg, sg = run[s]
                run[s] = (apply_slice_left(m, self.field, l, s, Lt), lg, sg)
            p = l - 1
            if p in m.checkpoints:
                for s in SPINS:
                    Q, lg, sg = self._orthonormalise(*run[s])
                    self.stack[(p, s)] = (Q, lg, sg)
                    run[s] = (Q, lg, sg)
        self.G = {}
        wsign = 1
        for s in SPINS:
            QL, lgL, sgL = self.stack[(-1, s)]
            X = QL.T @ m.P[s]
            sgX, _ = np.linalg.slogdet(X)
            self.G[s] = np.eye(m.N) - m.P[s] @ np.linalg.solve(X, QL.T)
            wsign *= int(sgL * np.sign(sgX))
        self.sign = wsign
        self.sweep_index = 0

    @staticmethod
    def _orthonormalise(B, logabs, sgn):
        """QR of the propagated basis; returns Q and the updated log|det|, sign."""
        Q, T = np.linalg.qr(B)
        d = np.diag(T)
        return Q, logabs + float(np.sum(np.log(np.abs(d)))), sgn * int(np.prod(np.sign(d)))

    # -- one Metropolis pass over the sites of slice l -------------------------
    def _flips(self, l):
        m = self.m
        u_all = philox.accept_uniforms(self.seed, self.chain_id, self.sweep_index, l, m.N)
        if self.exact:
            self._exact_green_at_slice(l)
        for i in range(m.N):
            s_li = int(self.field[l, i])
            delta, r = {}, {}
            for s in SPINS:
                delta[s] = m.flip_delta(s_li, l, s)
                r[s] = 1.0 + delta[s] * (1.0 - self.G[s][i, i])
            u = float(u_all[i])
            prob = abs(r[1] * r[-1])
            accept = u < prob
            if self.follow is not None:
                forced = bool(self.follow[l, i] != self.field[l, i])
                if forced != accept:
                    if abs(u - prob) > self.follow_tol * max(prob, 1.0):
                        self.follow_violations.append((self.sweep_index, l, i, u, prob))
                    accept = forced
            if self.record_ratios:
                self.ratios[(self.sweep_index, l, i)] = (r[1], r[-1], u, accept)
            if accept:
                for s in SPINS:
                    G = self.G[s]
                    col = G[:, i].copy()
                    row = -G[i, :].copy()
                    row[i] += 1.0
                    G -= (delta[s] / r[s]) * np.outer(col, row)
                self.field[l, i] = -s_li
                self.sign *= 1 if r[1] * r[-1] > 0 else -1
                if self.exact:
                    self._exact_green_at_slice(l)

    def _exact_green_at_slice(self, l):
        """G in the frame where D_l acts: R = D_l R_{l-1}, L = L_l K_l (fresh)."""
        m = self.m
        for s in SPINS:
            R = m.P[s].copy()
            for ll in range(0, l):
                R, _ = np.linalg.qr(apply_slice(m, self.field, ll, s, R))
            R = m.diag(self.field[l], l, s)[:, None] * R
            Lt = m.P[s].copy()
            for ll in range(m.M + 1, l, -1):
                Lt, _ = np.linalg.qr(apply_slice_left(m, self.field, ll, s, Lt))
            if m.is_bulk(l):
                Lt = m.Km @ Lt
            self.G[s] = green_from_bases(R, Lt)

    # -- checkpoints -----------------------------------------------------------
    def _checkpoint(self, p, run, up):
        """Orthonormalise the active basis, recompute G at position p from the
        stored opposite-side basis, check the sign, store the new basis."""
        m = self.m
        wsign = 1
        fresh = {}
        logdet = {}
        drift = 0.0
        for s in SPINS:
            Q, lg, sg = self._orthonormalise(*run[s])
            run[s] = (Q, lg, sg)
            Qo, lgo, sgo = self.stack[(p, s)]
            R, Lt = (Q, Qo) if up else (Qo, Q)
            X = Lt.T @ R
            sgX, lgX = np.linalg.slogdet(X)
            Gf = np.eye(m.N) - R @ np.linalg.solve(X, Lt.T)
            drift = max(drift, float(np.max(np.abs(self.G[s] - Gf))))
            fresh[s] = Gf
            self.G[s] = Gf
            self.stack[(p, s)] = (Q, lg, sg)
            # W_sigma = det(L_p R_p) = det(T_L) det(T_R) det(Q_L^T Q_R): the
            # accumulated triangular factors of both sides and the overlap
            logdet[s] = (lg + lgo + float(lgX), int(sg * sgo * np.sign(sgX)))
            wsign *= logdet[s][1]
        self.checkpoint_logdets.append((self.sweep_index, p, logdet))
        self.max_drift = max(self.max_drift, drift)
        if wsign != self.sign:
            self.sign_mismatches += 1
            self.sign = wsign
        if self.record_greens:
            self.checkpoint_greens.append((self.sweep_index, p, fresh[1].copy(),
                                           fresh[-1].copy(), drift, self.field.copy()))

    def _measure(self):
        e, d = estimators(self.m, self.G[1], self.G[-1])
        saf = structure_factor(self.m.eps, self.G[1], self.G[-1])
        self.measurements.append((self.sign, e, d, saf))

    # -- passes ----------------------------------------------------------------
    def _up_pass(self, measure):
        m = self.m
        run = {}
        for s in SPINS:
            self.stack[(-1, s)] = (m.P[s].copy(), 0.0, 1)
            run[s] = (m.P[s].copy(), 0.0, 1)
        for l in range(0, m.M + 2):
            for s in SPINS:
                d = m.diag(self.field[l], l, s)
                self.G[s] = d[:, None] * self.G[s] / d[None, :]
            self._flips(l)
            if m.is_bulk(l):
                for s in SPINS:
                    self.G[s] = m.Km @ self.G[s] @ m.Kp
            for s in SPINS:
                B, lg, sg = run[s]
                run[s] = (apply_slice(m, self.field, l, s, B), lg, sg)
            if l in m.checkpoints:
                self._checkpoint(l, run, up=True)
            if l == m.l_half and measure:
                self._measure()

    def _down_pass(self, measure):
        m = self.m
        run = {}
        for s in SPINS:
            self.stack[(m.M + 1, s)] = (m.P[s].copy(), 0.0, 1)
            run[s] = (m.P[s].copy(), 0.0, 1)
        for l in range(m.M + 1, -1, -1):
            if m.is_bulk(l):
                for s in SPINS:
                    self.G[s] = m.Kp @ self.G[s] @ m.Km
            self._flips(l)
            for s in SPINS:
                d = m.diag(self.field[l], l, s)
                self.G[s] = self.G[s] * d[None, :] / d[:, None]
                B, lg, sg = run[s]
                run[s] = (apply_slice_left(m, self.field, l, s, B), lg, sg)
            p = l - 1
            if p in m.checkpoints:
                self._checkpoint(p, run, up=False)
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
        """One pass that takes each acceptance from ``field_after`` (the field
        another implementation reached after the same pass), recording every
        decision that disagrees with this oracle by more than ``tol`` relative
        to its threshold."""
        self.follow = np.asarray(field_after, dtype=np.int8).reshape(self.field.shape)
        self.follow_tol = float(tol)
        try:
            self.sweep(1)
        finally:
            self.follow = None
        return self.follow_violations


def free_energy_closed_form(K, P_up, P_dn, theta):
    """U = 0, g = 0: E = sum_sigma sum_ij K_ij <c_i^dag c_j> with
    R = e^{-Theta K} P, L = P^T e^{-Theta K} (no Trotter error without V)."""
    w, V = np.linalg.eigh(K)
    E = (V * np.exp(-theta * w)) @ V.T
    tot = 0.0
    for P in (P_up, P_dn):
        G = green_from_bases(E @ P, E @ P)
        tot += float(np.sum(K * (np.eye(K.shape[0]) - G.T)))
    return tot
