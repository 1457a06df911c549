"""Seeded synthetic workloads for the Gutzwiller-projection PQMC sweep.

This module only *describes inputs*: lattices (hopping matrix and sublattice
signs of the Hubbard model, Eq. 2), model parameters, the trial-only on-site
potential used to close the shell of a doped lattice, and the random draws that
define a batch of uneven chains.  It contains none of the method's arithmetic
(no propagation, no Green's function, no Monte Carlo) and is imported both by
the tests that drive the oracle and by the code that drives the HIP library.

The headline workloads are the square lattice with periodic boundaries and
nearest-neighbour hopping -t, which has the same two-sublattice (Neel)
structure used by the trial state (Method section, Neel mean-field Hamiltonian
after Eq. 2).  The paper's own Hubbard lattice, the honeycomb lattice (Eq. 2),
is available as ``Workload(..., lattice_kind="honeycomb")``.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

__all__ = [
    "square_lattice",
    "honeycomb_lattice",
    "honeycomb_bonds",
    "ring_lattice",
    "shell_ramp",
    "Workload",
    "WORKLOADS",
    "TVWorkload",
    "TV_WORKLOADS",
    "batch_uneven",
]


def square_lattice(lx: int, ly: int, t: float = 1.0):
    """Hopping matrix of an lx x ly periodic square lattice.

    Returns ``(K, eps, xy)``: ``K`` is the N x N real symmetric matrix with
    ``K[i, j] = -t`` for every nearest-neighbour bond (bonds that wrap onto the
    same pair twice, as on a 2-site-wide torus, accumulate), ``eps`` the
    sublattice sign (+1 on A, -1 on B: (-1)^(x+y)) and ``xy`` the site
    coordinates.  Site index is ``i = x + lx * y``.
    """
    n = lx * ly
    K = np.zeros((n, n), dtype=np.float64)
    xy = np.zeros((n, 2), dtype=np.int64)
    for y in range(ly):
        for x in range(lx):
            i = x + lx * y
            xy[i] = (x, y)
            for dx, dy in ((1, 0), (0, 1)):
                if (dx == 1 and lx == 1) or (dy == 1 and ly == 1):
                    continue
                j = (x + dx) % lx + lx * ((y + dy) % ly)
                K[i, j] -= t
                K[j, i] -= t
    eps = np.where((xy[:, 0] + xy[:, 1]) % 2 == 0, 1, -1).astype(np.int8)
    return K, eps, xy


def honeycomb_lattice(l1: int, l2: int, t: float = 1.0):
    """Hopping matrix of an l1 x l2 periodic honeycomb lattice (Eq. 2).

    Unit cell (x, y) holds site A = 2 (x + l1 y) and site B = A + 1.  With
    primitive vectors a1, a2, every A site is bonded to the B site of its own
    cell and to the B sites of cells (x - 1, y) and (x, y - 1); each bond
    carries -t (bonds that wrap onto the same pair twice accumulate).  Returns
    ``(K, eps, cells)``: ``eps`` is +1 on A and -1 on B, ``cells`` the unit
    cell of every site.
    """
    n = 2 * l1 * l2
    K = np.zeros((n, n), dtype=np.float64)
    cells = np.zeros((n, 2), dtype=np.int64)
    for y in range(l2):
        for x in range(l1):
            a = 2 * (x + l1 * y)
            cells[a] = cells[a + 1] = (x, y)
            for dx, dy in ((0, 0), (-1, 0), (0, -1)):
                b = 2 * ((x + dx) % l1 + l1 * ((y + dy) % l2)) + 1
                K[a, b] -= t
                K[b, a] -= t
    eps = np.where(np.arange(n) % 2 == 0, 1, -1).astype(np.int8)
    return K, eps, cells


def honeycomb_bonds(l1: int, l2: int) -> np.ndarray:
    """Nearest-neighbour bonds (A, B) of the l1 x l2 periodic honeycomb lattice
    of ``honeycomb_lattice``, grouped by direction: first every A site's bond
    to the B site of its own cell, then to the B site of cell (x - 1, y), then
    of cell (x, y - 1).  Each group is a perfect matching (no two bonds of a
    group share a site), so any run of consecutive bonds inside a group is
    site-disjoint.  Needs l1, l2 >= 2 (no doubled bonds)."""
    if l1 < 2 or l2 < 2:
        raise ValueError("honeycomb bonds need l1, l2 >= 2")
    out = []
    for dx, dy in ((0, 0), (-1, 0), (0, -1)):
        for y in range(l2):
            for x in range(l1):
                a = 2 * (x + l1 * y)
                b = 2 * ((x + dx) % l1 + l1 * ((y + dy) % l2)) + 1
                out.append((a, b))
    return np.array(out, dtype=np.int32)


def ring_lattice(n: int, t: float = 1.0):
    """Periodic ring of an even number n >= 4 of sites: ``(K, eps, bonds)``
    with bonds (even site, odd site) grouped as (0,1), (2,3), ... then
    (2,1), (4,3), ..., (0, n-1): two perfect matchings."""
    if n < 4 or n % 2:
        raise ValueError("the ring needs an even n >= 4")
    K = np.zeros((n, n))
    bonds = [(i, i + 1) for i in range(0, n, 2)] + [((i + 1) % n, i) for i in range(1, n, 2)]
    for a, b in bonds:
        K[a, b] -= t
        K[b, a] -= t
    eps = np.where(np.arange(n) % 2 == 0, 1, -1).astype(np.int8)
    return K, eps, np.array(bonds, dtype=np.int32)


def shell_ramp(lx: int, ly: int, delta: float = 0.1, tilt: float = 0.37):
    """Trial-only on-site potential delta*(x/lx + tilt*y/ly).

    A doped square lattice (e.g. 16x16 with 112 electrons per spin) has a
    degenerate Fermi level, so the mean-field trial determinant is not unique.
    This small potential enters only the trial Hamiltonian (never the
    Hamiltonian that is simulated), splits the degeneracy and makes the trial
    state well defined.  The projector estimate is unbiased for any trial state
    with non-zero overlap with the ground state.
    """
    _, _, xy = square_lattice(lx, ly)
    return delta * (xy[:, 0] / lx + tilt * xy[:, 1] / ly)


@dataclasses.dataclass
class Workload:
    name: str
    lx: int
    ly: int
    U: float
    n_up: int
    n_dn: int
    dtau: float
    l_half: int            # slices per side: Theta / dtau
    m_neel: float
    g: float
    stab_interval: int     # slices between QR re-stabilisations
    delay_rank: int        # delay rank: sites per scan segment (one delayed flush each)
    precision: str         # "fp64" or "mixed"
    sweeps: int
    t: float = 1.0
    ramp: float = 0.0      # trial-only shell-closing ramp amplitude (0 = none)
    seed: int = 13403
    lattice_kind: str = "square"   # "square" (lx x ly sites) or "honeycomb" (lx x ly cells of 2)

    @property
    def n_sites(self) -> int:
        return self.lx * self.ly * (2 if self.lattice_kind == "honeycomb" else 1)

    @property
    def theta(self) -> float:
        return self.l_half * self.dtau

    def lattice(self):
        if self.lattice_kind == "honeycomb":
            return honeycomb_lattice(self.lx, self.ly, self.t)
        if self.lattice_kind != "square":
            raise ValueError(f"unknown lattice kind {self.lattice_kind!r}")
        return square_lattice(self.lx, self.ly, self.t)

    def trial_potential(self) -> Optional[np.ndarray]:
        if self.ramp == 0.0:
            return None
        if self.lattice_kind != "square":
            raise ValueError("the shell-closing ramp is defined on the square lattice")
        return shell_ramp(self.lx, self.ly, self.ramp)

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


# The synthetic workloads: a small 4x4 case, a 12x12 half-filled case, the
# 16x16 doped case whose throughput is the headline figure, a batch of uneven
# lattices, a 24x24 large case and the half-filled honeycomb lattice of the
# paper's Hubbard study at 288 sites.  Model parameters follow the Gutzwiller
# optima the paper prints for the Hubbard model (Fig. 1 caption: g=0.55,
# M_N=0.07 at U=3.5; g=0.6, M_N=0.21 at U=4).
WORKLOADS = {
    "4x4": Workload("4x4 U=4 half filling Theta=2", 4, 4, 4.0, 8, 8, 0.1, 20,
                    0.21, 0.6, 5, 16, "fp64", 200),
    "12x12": Workload("12x12 U=4 half filling Theta=5", 12, 12, 4.0, 72, 72, 0.1, 50,
                      0.21, 0.6, 10, 64, "mixed", 500),
    "16x16": Workload("16x16 U=3.5 n=0.875 Theta=10", 16, 16, 3.5, 112, 112, 0.1, 100,
                      0.07, 0.55, 5, 32, "mixed", 1000, ramp=0.1),
    "24x24": Workload("24x24 U=4 half filling Theta=10 dtau=0.05", 24, 24, 4.0, 288, 288,
                      0.05, 200, 0.21, 0.6, 10, 64, "mixed", 100),
    "honeycomb12x12": Workload("honeycomb 12x12 cells (288 sites) U=4 half filling Theta=5",
                               12, 12, 4.0, 144, 144, 0.1, 50, 0.21, 0.6, 5, 32, "mixed", 100,
                               lattice_kind="honeycomb"),
}


@dataclasses.dataclass
class TVWorkload:
    """Spinless t-V model (Eq. 3) at half filling: H = -t sum c^dag c +
    V sum_<ij> (n_i - 1/2)(n_j - 1/2) on the honeycomb lattice (or a ring for
    the smallest checks), trial e^{-g sum_<ij> n_i n_j} |psi_C> with |psi_C>
    the ground state of K + Delta_C sum_i eps_i n_i (CDW mean field)."""
    name: str
    l1: int                # honeycomb cells per direction (ring: number of sites)
    l2: int
    V: float
    dtau: float
    l_half: int
    delta_c: float         # CDW order parameter of the trial
    g: float               # bond Gutzwiller parameter
    stab_interval: int
    delay_rank: int        # sites per scan segment: delay_rank / 2 bonds of one direction
    sweeps: int
    t: float = 1.0
    seed: int = 13403
    lattice_kind: str = "honeycomb"   # or "ring"

    @property
    def n_sites(self) -> int:
        return 2 * self.l1 * self.l2 if self.lattice_kind == "honeycomb" else self.l1

    @property
    def n_particles(self) -> int:
        return self.n_sites // 2

    @property
    def theta(self) -> float:
        return self.l_half * self.dtau

    def lattice(self):
        """(K, eps, bonds)."""
        if self.lattice_kind == "ring":
            return ring_lattice(self.l1, self.t)
        if self.lattice_kind != "honeycomb":
            raise ValueError(f"unknown lattice kind {self.lattice_kind!r}")
        K, eps, _ = honeycomb_lattice(self.l1, self.l2, self.t)
        return K, eps, honeycomb_bonds(self.l1, self.l2)

    def replace(self, **kw) -> "TVWorkload":
        return dataclasses.replace(self, **kw)


# The spinless t-V workloads: the paper's L = 15 honeycomb lattice (450 sites)
# in the CDW phase (V = 1.6) and near the transition (V = 1.35), Theta = 5;
# a 6x6-cell lattice for parity tests.  The paper does not print its trial
# parameters for this model: Delta_C = 0.3 and g = 0.3 are a fixed choice.
TV_WORKLOADS = {
    "tv15_V1.6": TVWorkload("t-V honeycomb 15x15 (450 sites) V=1.6 half filling Theta=5",
                            15, 15, 1.6, 0.1, 50, 0.3, 0.3, 5, 32, 100),
    "tv15_V1.35": TVWorkload("t-V honeycomb 15x15 (450 sites) V=1.35 half filling Theta=5",
                             15, 15, 1.35, 0.1, 50, 0.3, 0.3, 5, 32, 100),
    "tv6": TVWorkload("t-V honeycomb 6x6 (72 sites) V=1.6 half filling Theta=2",
                      6, 6, 1.6, 0.1, 20, 0.3, 0.3, 5, 32, 100),
}


def batch_uneven(n_chains: int = 256, seed: int = 13403, l_half: int = 50,
                 dtau: float = 0.1, precision: str = "mixed", stab_interval: int = 5,
                 delay_rank: int = 64):
    """Batch of independent half-filled chains on uneven lattices.

    Each chain draws its linear size uniformly from {6, 8, 10, 12} and U
    uniformly from [2, 6] (numpy PCG64 stream seeded with ``seed``); every
    chain uses M_N = 0.21, g = 0.6, Theta = l_half * dtau.
    """
    rng = np.random.default_rng(seed)
    sizes = np.array([6, 8, 10, 12])
    pick = rng.integers(0, 4, size=n_chains)
    us = rng.uniform(2.0, 6.0, size=n_chains)
    out = []
    for c in range(n_chains):
        L = int(sizes[pick[c]])
        out.append(Workload(f"batch chain {c}: {L}x{L} U={us[c]:.3f}", L, L, float(us[c]),
                            L * L // 2, L * L // 2, dtau, l_half, 0.21, 0.6,
                            stab_interval, delay_rank, precision, 500, seed=seed))
    return out
