"""Cholesky-based direct inverse written out with loops -- oracle side (test infrastructure).

The paper's introduction describes the direct method IBMI is compared with: factor
A = L L^T, then for every unit vector e_i solve L z_i = e_i and L^T h_i = z_i; the h_i are
the columns of A^{-1}.  This routine does exactly that with explicit loops (no LAPACK),
so that it is an independent check of the K = 1 case of IBMI and of converged iterates.
Meant for p <= a few hundred.  Pinned by A @ inverse = I on random SPD matrices and by the
closed-form inverse of 2x2 and tridiagonal test matrices.
"""
from __future__ import annotations

import math

import numpy as np


def cholesky_loops(a: np.ndarray) -> np.ndarray:
    """Lower-triangular L with A = L L^T, column by column (Cholesky-Banachiewicz order)."""
    n = a.shape[0]
    l = np.zeros((n, n))
    for j in range(n):
        s = a[j, j] - float(np.dot(l[j, :j], l[j, :j]))
        if not s > 0.0:
            raise ValueError(f"non-positive pivot at column {j}")
        l[j, j] = math.sqrt(s)
        for i in range(j + 1, n):
            l[i, j] = (a[i, j] - float(np.dot(l[i, :j], l[j, :j]))) / l[j, j]
    return l


def cholesky_inverse_loops(a: np.ndarray) -> np.ndarray:
    """A^{-1} column by column: forward substitution with L, back substitution with L^T."""
    n = a.shape[0]
    l = cholesky_loops(np.asarray(a, dtype=np.float64))
    inv = np.zeros((n, n))
    for col in range(n):
        z = np.zeros(n)
        for i in range(n):
            rhs = (1.0 if i == col else 0.0) - float(np.dot(l[i, :i], z[:i]))
            z[i] = rhs / l[i, i]
        x = np.zeros(n)
        for i in range(n - 1, -1, -1):
            rhs = z[i] - float(np.dot(l[i + 1:, i], x[i + 1:]))
            x[i] = rhs / l[i, i]
        inv[:, col] = x
    return inv
