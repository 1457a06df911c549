"""Serial FP64 CPU oracle for the Gutzwiller-projection PQMC sweep.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) may import, call or link anything in this package.  Only the
tests, the smoke check and the CPU-baseline leg of the benchmark use it.

The oracle is a plain, slow, obviously correct NumPy implementation of what the
sweep computes (Chang & Li, "Boosting quantum Monte Carlo and alleviating sign
problem by Gutzwiller projection", arXiv:2303.13403):

* ``philox``  -- Philox4x32-10 counter-based generator (Salmon et al., SC'11),
  written from its published definition; the HIP side has its own.
* ``pqmc``    -- the projector determinant QMC chain with the Gutzwiller trial
  state (Method section, Eq. 1 read in the spin channel; the Neel trial after
  Eq. 2), rank-1 Sherman-Morrison updates, QR re-stabilisation, measurement.
* ``tv``      -- the same chain for the spinless t-V model ("Repulsive
  spinless honeycomb model", Eq. 3): bond fields decoupled in the density
  channel, CDW trial with the bond Gutzwiller factor, rank-2 Woodbury updates,
  a signful weight.
* ``ed``      -- Fock-space exact diagonalisation of tiny clusters, and exact
  enumeration of every auxiliary-field configuration (both models); used as
  pins.
* ``stats``   -- binning / jackknife for sign-weighted averages.

Every function pinned by ``tests/test_oracle_*.py`` against closed forms,
brute force, library routines or symmetries; see each module's header.
"""
