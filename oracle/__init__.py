"""FP64 CPU oracle for the DD-alpha-AMG hot path (arXiv:1307.6101).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
numpy implementation of what the GPU library computes.  Only the test-suite,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import it; the product path never does, and the two share no code (the only
common module is ``workloads``, which draws seeded random inputs).

Layout: a field on a level is a complex128 array of shape (T, Z, Y, X, d);
direction mu = 0..3 is x, y, z, t and lives on array axis 3 - mu.

Modules
  lattice     geometry: shifts, block / aggregate reshapes, parity
  dirac       gamma matrices, clover leaves, the Wilson-clover operator
  stencil     generic nearest-neighbour block stencil (coarse operators)
  sap         minimal residual and the red-black Schwarz smoother
  aggregation block-spin interpolation P (chirality-preserving aggregation)
  galerkin    D_c = P^H D P
  krylov      FGMRES, GMRES, odd-even (Schur) coarsest solve
  multigrid   hierarchy, K-cycle / V-cycle, setup phases, outer solve

Parity pins: every function is checked in tests/test_oracle_*.py against a
closed form, an invariant or a dense brute-force computation.  The setup
phases (``multigrid.initial_setup``, ``multigrid.iterative_setup``) and the
three-level K-, V- and W-cycles are pinned by dense closed forms with exact
block solves in place of MR (the smoother is then linear) and an exact
coarsest solve (tests/test_oracle_setup.py).  The test-vector values of a
setup with MR block solves have no unique value; the GPU library is compared
with the oracle there through exported and imported interpolation bases.
"""
