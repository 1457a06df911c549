"""Lattice generators (the inputs shared by the oracle and the HIP path),
pinned to closed forms: the tight-binding spectra of the periodic square and
honeycomb lattices."""
import numpy as np
import pytest

from paper_2303_13403_amd.workloads import Workload, honeycomb_lattice, square_lattice


@pytest.mark.parametrize("l1,l2", [(3, 3), (4, 2), (6, 6), (5, 4)])
def test_honeycomb_spectrum_is_the_graphene_band_structure(l1, l2):
    # eigenvalues +-t |1 + e^{i k1} + e^{i k2}|, k_a = 2 pi m_a / l_a
    t = 1.3
    K, eps, _ = honeycomb_lattice(l1, l2, t)
    k1 = 2 * np.pi * np.arange(l1)[:, None] / l1
    k2 = 2 * np.pi * np.arange(l2)[None, :] / l2
    e = t * np.abs(1 + np.exp(1j * k1) + np.exp(1j * k2)).ravel()
    ref = np.sort(np.concatenate([e, -e]))
    assert np.allclose(np.sort(np.linalg.eigvalsh(K)), ref, atol=1e-12)


def test_honeycomb_is_bipartite_with_three_bonds_per_site():
    K, eps, cells = honeycomb_lattice(4, 3)
    assert K.shape == (24, 24) and np.array_equal(K, K.T)
    assert np.all((K != 0).sum(axis=1) == 3)
    i, j = np.nonzero(K)
    assert np.all(eps[i] != eps[j])                  # bonds join A and B only
    assert eps.sum() == 0 and np.all(cells[0::2] == cells[1::2])


@pytest.mark.parametrize("lx,ly", [(4, 4), (6, 4), (5, 3)])
def test_square_spectrum_is_the_cosine_band(lx, ly):
    K, _, _ = square_lattice(lx, ly)
    kx = 2 * np.pi * np.arange(lx)[:, None] / lx
    ky = 2 * np.pi * np.arange(ly)[None, :] / ly
    ref = np.sort((-2 * np.cos(kx) - 2 * np.cos(ky)).ravel())
    assert np.allclose(np.sort(np.linalg.eigvalsh(K)), ref, atol=1e-12)


def test_workload_lattice_kind():
    w = Workload("hc", 3, 3, 4.0, 9, 9, 0.1, 4, 0.21, 0.6, 2, 8, "fp64", 10,
                 lattice_kind="honeycomb")
    assert w.n_sites == 18
    K, eps, _ = w.lattice()
    assert K.shape == (18, 18)
    with pytest.raises(ValueError):
        w.replace(lattice_kind="kagome").lattice()
