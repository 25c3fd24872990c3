"""CPU oracle of IBMI (Iterative Block Matrix Inversion) -- TEST INFRASTRUCTURE ONLY.

A plain, slow, FP64 CPU implementation of what the GPU library computes, written from the
paper (Paterson, Pestana, Dolean, "An Iterative Block Matrix Inversion (IBMI) Algorithm for
Symmetric Positive Definite Matrices with Applications to Covariance Matrices"):

* ``partition``  -- contiguous, optionally overlapping index sets I_k (section on the
  multi-block overlapping case; the cost section fixes end blocks of m+h rows and interior
  blocks of m+2h rows);
* ``ibmi``       -- the block update of eq. (IBMI), Algorithm 1 (sweeps over k = 1..K using
  the most recent approximation), the residual ||I - A H||_F, the paper's error estimate of
  eq. (error), a certified bound on the relative error of H from ||H (I - A H)||_F, and a
  correction (defect) form of the same update with emulated low-precision products;
* ``cholinv``    -- the Cholesky-based direct inverse of the introduction, written out with
  loops (A = L L^T, then L z_i = e_i and L^T h_i = z_i);
* ``exact``      -- IBMI in exact rational arithmetic for tiny matrices.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import this package.  It shares no code with the HIP library and never imports it; the
product path never imports this package.

Pinning status of each function is stated in its docstring; nothing here is "parity
unpinned" except where a docstring says so.
"""
from .partition import partition, validate_blocks, complement
from .ibmi import (
    IbmiError, plan, block_factors, initial_h, block_update, sweep, residual_fro, paper_error,
    ibmi_solve, correction_sweep, emulate_product, hr_error_bound,
)
from .cholinv import cholesky_inverse_loops
from .exact import exact_ibmi, exact_residual_sq

__all__ = [
    "partition", "validate_blocks", "complement", "IbmiError", "plan", "block_factors",
    "initial_h",
    "block_update", "sweep", "residual_fro", "paper_error", "ibmi_solve",
    "correction_sweep", "emulate_product", "hr_error_bound", "cholesky_inverse_loops",
    "exact_ibmi", "exact_residual_sq",
]
