"""FP64 CPU oracle for the two-stage preconditioned FGMRES solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library or its Python binding
imports, calls or links this package; only the tests, the smoke check and the
benchmark's CPU-baseline leg do.  It shares no code with the HIP path.

It is a plain, slow, obviously-checkable implementation of what the solver
computes, written from the paper:
  * fgmres.py   -- right-preconditioned flexible GMRES(m) with classical
                   Gram-Schmidt applied twice and Givens rotations (Sec. 4).
  * precond.py  -- Algorithm 1 (application of the block preconditioner) and the
                   setup of its operators: fixed-stress Schur approximation
                   (eq. Schur_1_FS), quasi-IMPES reduction (Sec. 5.3), separate
                   displacement component approximation (Sec. 5.2).
  * amg.py      -- classical AMG for the two scalar sub-problems: strength of
                   connection, PMIS coarsening, direct interpolation, Galerkin
                   coarse operators, V(1,1)-cycle, dense coarsest solve.
  * local.py    -- second-stage local preconditioners on the interleaved flow
                   system: block ILU(0) and block Jacobi (Sec. 5.3).
  * rng.py      -- the counter-based SplitMix64 generator used for PMIS tie
                   breaking and power-iteration start vectors.
Where the paper is silent the oracle takes one stated reading; each module lists
its readings.  Functions without an independent pin say "parity unpinned".
"""
from .precond import Options, setup, apply_precond, system_matrices
from .fgmres import fgmres, solve

__all__ = ["Options", "setup", "apply_precond", "system_matrices", "fgmres", "solve"]
