"""IBMI in exact rational arithmetic for tiny matrices -- oracle side (test infrastructure).

Applies eq. (IBMI) literally with Python ``fractions.Fraction``: A_I^{-1} by Gauss-Jordan
elimination, then the four blocks of the update, then the next set (Algorithm 1).  With no
rounding at all, it fixes the iterates of small examples exactly; the FP64 oracle must
agree with it to rounding level.  Independent pins: the p = 2 closed form derived by hand
from eq. (IBMI) and the Lemma's scalar contraction (c^2 / (a d))^2 per sweep.
"""
from __future__ import annotations

from fractions import Fraction


def _inverse(m):
    n = len(m)
    aug = [[Fraction(x) for x in row] + [Fraction(int(i == j)) for j in range(n)]
           for i, row in enumerate(m)]
    for col in range(n):
        piv = next(r for r in range(col, n) if aug[r][col] != 0)
        aug[col], aug[piv] = aug[piv], aug[col]
        pv = aug[col][col]
        aug[col] = [x / pv for x in aug[col]]
        for r in range(n):
            if r != col and aug[r][col] != 0:
                f = aug[r][col]
                aug[r] = [x - f * y for x, y in zip(aug[r], aug[col])]
    return [row[n:] for row in aug]


def _mul(x, y):
    return [[sum((x[i][t] * y[t][j] for t in range(len(y))), Fraction(0))
             for j in range(len(y[0]))] for i in range(len(x))]


def exact_ibmi(a, sets, sweeps: int, h0=None):
    """Return the list of iterates H^{(r,K)}, r = 1..sweeps, as lists of Fractions.

    ``a`` is a small integer or Fraction matrix, ``sets`` a list of index lists, ``h0`` the
    initial H (identity when None).
    """
    p = len(a)
    a = [[Fraction(x) for x in row] for row in a]
    h = [[Fraction(int(i == j)) for j in range(p)] for i in range(p)] if h0 is None else \
        [[Fraction(x) for x in row] for row in h0]
    out = []
    for _ in range(sweeps):
        for idx in sets:
            comp = [j for j in range(p) if j not in idx]
            a_i = [[a[r][c] for c in idx] for r in idx]
            ainv = _inverse(a_i)
            if not comp:
                for x, r in enumerate(idx):
                    for y, c in enumerate(idx):
                        h[r][c] = ainv[x][y]
                continue
            a_ic = [[a[r][c] for c in comp] for r in idx]
            w = _mul(ainv, a_ic)
            h_ic = [[h[r][c] for c in comp] for r in comp]
            v = _mul(w, h_ic)
            wt = [list(col) for col in zip(*w)]
            x_blk = _mul(v, wt)
            for x, r in enumerate(idx):
                for y, c in enumerate(comp):
                    h[r][c] = -v[x][y]
                    h[c][r] = -v[x][y]
                for y, c in enumerate(idx):
                    h[r][c] = ainv[x][y] + x_blk[x][y]
        out.append([row[:] for row in h])
    return out


def exact_residual_sq(a, h) -> Fraction:
    """||I - A H||_F^2 exactly."""
    p = len(a)
    ah = _mul([[Fraction(x) for x in row] for row in a], h)
    return sum(((Fraction(int(i == j)) - ah[i][j]) ** 2 for i in range(p) for j in range(p)),
               Fraction(0))
