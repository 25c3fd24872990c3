"""IBMI in plain FP64 NumPy -- oracle side (test infrastructure only).

Notation follows the paper: A (the paper's Q) is SPD and p x p, H approximates A^{-1}
(the paper's Sigma-tilde), I is the current index set and I^c its complement.  Library
primitives used as single steps: numpy's Cholesky, SciPy's triangular solve, matmul and
the Frobenius / spectral norm.  There is no blocking, fusion or reordering beyond what the
paper's equations state.

Pins (tests/test_oracle_pins.py): the Lemma and Theorem of the convergence section
(two non-overlapping sets), the Corollary (exact Schur-complement inverse gives A^{-1} in
one step), the K = 1 case against the loop-written Cholesky inverse, exact rational
iterates at p <= 4, the multiplicative-Schwarz error propagator for overlapping sets,
fixed point, invariants after each block step, and convergence on random SPD matrices.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy.linalg import solve_triangular

from .partition import complement, validate_blocks


class IbmiError(Exception):
    """Error with a status name matching the C library's codes (INVALID_ARG, NOT_SPD, NONFINITE)."""

    def __init__(self, code: str, msg: str, block: int = -1):
        super().__init__(f"{code}: {msg}")
        self.code = code
        self.block = block


@dataclass
class BlockPlan:
    """Per-set quantities that depend on A only (computed once, reused every sweep)."""
    idx: np.ndarray      # I_k
    comp: np.ndarray     # I_k^c
    chol: np.ndarray     # L with A_I = L L^T
    ainv: np.ndarray     # A_I^{-1}, symmetrised
    w: np.ndarray        # A_I^{-1} A_{I, I^c}   (|I| x |I^c|)


def _index_sets(p: int, blocks) -> list:
    """Accept half-open ranges (s, e) or explicit index arrays; return index arrays."""
    sets = []
    if all(isinstance(b, tuple) and len(b) == 2 for b in blocks):
        try:
            validate_blocks(p, blocks)
        except ValueError as exc:
            raise IbmiError("INVALID_ARG", str(exc)) from None
        return [np.arange(s, e) for s, e in blocks]
    covered = np.zeros(p, dtype=bool)
    for b in blocks:
        idx = np.asarray(b, dtype=np.int64)
        if idx.size == 0 or idx.min() < 0 or idx.max() >= p or np.unique(idx).size != idx.size:
            raise IbmiError("INVALID_ARG", "index set empty, out of range or repeated")
        covered[idx] = True
        sets.append(idx)
    if not covered.all():
        raise IbmiError("INVALID_ARG", "index sets do not cover {0..p-1}")
    return sets


def plan(a: np.ndarray, blocks) -> list:
    """Factor every diagonal block once: L_k, A_{I_k}^{-1} and W_k = A_{I_k}^{-1} A_{I_k, I_k^c}.

    These depend on A only, so they are computed once per solve although the paper's cost
    section counts them every iteration.  A_I^{-1} = L^{-T} L^{-1} with L^{-1} from a
    triangular solve against the identity, then symmetrised as (X + X^T)/2.
    A non-positive or non-finite pivot in set k raises NOT_SPD with ``block = k``.
    """
    a = np.asarray(a, dtype=np.float64)
    if a.ndim != 2 or a.shape[0] != a.shape[1] or a.shape[0] < 1:
        raise IbmiError("INVALID_ARG", "A must be square and non-empty")
    if not np.isfinite(a).all():
        raise IbmiError("INVALID_ARG", "A has non-finite entries")
    if not np.array_equal(a, a.T):
        raise IbmiError("INVALID_ARG", "A must be exactly symmetric")
    p = a.shape[0]
    return [plan_one(a, idx, k) for k, idx in enumerate(_index_sets(p, blocks))]


def block_factors(a: np.ndarray, s: int, e: int) -> BlockPlan:
    """The factors of one contiguous set [s, e) alone (same steps as ``plan``), for checking
    single block steps on matrices too large for a full CPU sweep."""
    return plan_one(np.asarray(a, dtype=np.float64), np.arange(s, e), 0)


def plan_one(a: np.ndarray, idx: np.ndarray, k: int) -> BlockPlan:
    comp = complement(a.shape[0], idx)
    a_i = a[np.ix_(idx, idx)]
    try:
        chol = np.linalg.cholesky(a_i)
    except np.linalg.LinAlgError:
        raise IbmiError("NOT_SPD", f"diagonal block {k} is not positive definite", k) from None
    d = np.diag(chol)
    if not (np.isfinite(d).all() and (d > 0).all()):
        raise IbmiError("NOT_SPD", f"diagonal block {k} has a bad pivot", k)
    linv = solve_triangular(chol, np.eye(idx.size), lower=True)
    ainv = linv.T @ linv
    ainv = 0.5 * (ainv + ainv.T)
    w = ainv @ a[np.ix_(idx, comp)]
    return BlockPlan(idx, comp, chol, ainv, w)


def initial_h(a: np.ndarray, blocks_plan: list, kind: str = "identity", h0=None) -> np.ndarray:
    """Initial approximation (Algorithm 1 input; only H0[I_1^c, I_1^c] is ever read).

    ``identity``: H0 = I, the paper's default.  ``blockdiag_inv``: H0 = blockdiag(A_{I_k}^{-1})
    for non-overlapping sets (the A_{I^c}^{-1} guess of the initial-guess study).
    ``given``: a copy of ``h0`` (resume from a saved iterate).
    """
    p = a.shape[0]
    if kind == "identity":
        return np.eye(p)
    if kind == "blockdiag_inv":
        seen = np.zeros(p, dtype=np.int64)
        for bp in blocks_plan:
            seen[bp.idx] += 1
        if (seen != 1).any():
            raise IbmiError("INVALID_ARG", "block-diagonal initial guess needs disjoint sets")
        h = np.zeros((p, p))
        for bp in blocks_plan:
            h[np.ix_(bp.idx, bp.idx)] = bp.ainv
        return h
    if kind == "given":
        h = np.array(h0, dtype=np.float64, copy=True)
        if h.shape != (p, p):
            raise IbmiError("INVALID_ARG", "given H0 has the wrong shape")
        return h
    raise IbmiError("INVALID_ARG", f"unknown initial guess {kind!r}")


def block_update(h: np.ndarray, bp: BlockPlan) -> None:
    """One application of eq. (IBMI) for set I, in place, using the current H[I^c, I^c].

    With W = A_I^{-1} A_{I,I^c} and the current approximation H_{I^c} of the inverse Schur
    complement:  H[I,I^c] = -W H_{I^c},  H[I^c,I] = -H_{I^c} W^T (written as the transpose
    of the same product, so H stays exactly symmetric), and
    H[I,I] = A_I^{-1} + W H_{I^c} W^T, symmetrised as (X + X^T)/2.  H[I^c,I^c] is unchanged.
    """
    i, ic = bp.idx, bp.comp
    if ic.size == 0:
        h[np.ix_(i, i)] = bp.ainv
        return
    h_ic = h[np.ix_(ic, ic)]
    v = bp.w @ h_ic
    h[np.ix_(i, ic)] = -v
    h[np.ix_(ic, i)] = -v.T
    x = bp.ainv + v @ bp.w.T
    h[np.ix_(i, i)] = 0.5 * (x + x.T)


def sweep(h: np.ndarray, blocks_plan: list) -> None:
    """One iteration r of Algorithm 1: k = 1..K in order, each using the latest H."""
    for bp in blocks_plan:
        block_update(h, bp)


def residual_fro(a: np.ndarray, h: np.ndarray) -> float:
    """||I - A H||_F in FP64."""
    r = np.eye(a.shape[0]) - a @ h
    return float(np.sqrt(np.sum(r * r)))


def paper_error(a: np.ndarray, h: np.ndarray, idx: np.ndarray, norm: str = "2") -> float:
    """The paper's stopping estimate, eq. (error): ||H_I A_{I,I^c} + H_{I,I^c} A_{I^c}||,
    the (1,2) block of H A for set I, in the spectral norm (``norm="2"``, the paper's) or the
    Frobenius norm (``"fro"``, an upper bound of it, the run-time stop test)."""
    ic = complement(a.shape[0], idx)
    if ic.size == 0:
        return 0.0
    e = h[np.ix_(idx, idx)] @ a[np.ix_(idx, ic)] + h[np.ix_(idx, ic)] @ a[np.ix_(ic, ic)]
    return float(np.linalg.norm(e, 2 if norm == "2" else "fro"))


def hr_error_bound(a: np.ndarray, h: np.ndarray) -> tuple:
    """Certified bound on the relative Frobenius error of H as an inverse of A, from R = I - A H.

    With E = H - A^{-1}: A^{-1} R = A^{-1} - H = -E and A^{-1} = H - E, so E (R - I) = H R and,
    when ||R||_2 <= ||R||_F < 1, ||E||_F <= ||H R||_F / (1 - ||R||_F) =: x ||H||_F.  Since
    ||A^{-1}||_F >= ||H||_F - ||E||_F, the relative error is at most x / (1 - x).  Returns
    (bound, ||R||_F); the bound is inf when ||R||_F >= 1 or x >= 1.  Exact-arithmetic bound:
    the FP64 evaluation of R limits it near the FP64 floor.
    """
    r = np.eye(a.shape[0]) - a @ h
    rho = float(np.sqrt(np.sum(r * r)))
    if rho >= 1.0:
        return float("inf"), rho
    hr = h @ r
    x = float(np.sqrt(np.sum(hr * hr))) / ((1.0 - rho) * float(np.sqrt(np.sum(h * h))))
    return (x / (1.0 - x) if x < 1.0 else float("inf")), rho


@dataclass
class SolveResult:
    h: np.ndarray
    sweeps: int
    history: list = field(default_factory=list)
    converged: bool = False
    floor_limited: bool = False
    stop_value: float = float("inf")  # after the last sweep
    evaluations: int = 0              # sweeps at which the rel_hr bound was evaluated


def _stop_value(a, h, rho, stop, lam_min):
    if stop == "fro":
        return rho
    if stop == "rel_bound":
        # ||H - A^{-1}||_F <= ||A^{-1}||_2 ||A H - I||_F <= rho / lambda_min(A); relative to ||H||_F.
        return rho / (lam_min * float(np.sqrt(np.sum(h * h))))
    raise IbmiError("INVALID_ARG", f"unknown stop test {stop!r}")


GUARD_SWEEPS = 16  # sweeps without a 1% improvement that end a solve at its floor


def ibmi_solve(a, blocks, init: str = "identity", h0=None, tol: float = 1e-10,
               max_sweeps: int = 500, stagnation_guard: bool = True, stop: str = "fro",
               lam_min: float = 0.0, fixed_sweeps: int = 0) -> SolveResult:
    """Algorithm 1 with the residual checked after every full sweep.

    ``stop="fro"`` stops once ||I - A H||_F < tol; ``stop="rel_bound"`` once
    ||I - A H||_F / (lam_min ||H||_F) < tol (a certified bound on the relative error of H
    when lam_min is a lower bound on A's smallest eigenvalue); ``stop="rel_hr"`` once the
    bound of hr_error_bound (from ||H R||_F, tight to first order) is below tol.  That bound
    costs a second p^3 product, so it is evaluated only at some sweeps: when ||R||_F < 1 for
    the first time, when ||R||_F has fallen tenfold since the last evaluation, and when the
    last evaluation's ratio bound/||R||_F times the current ||R||_F is below tol; at other
    sweeps the stop value is that prediction (inf before the first evaluation).
    ``stop="paper"`` stops once the Frobenius form of the paper's eq. (error) estimate for the
    last set, ||(H A)[I_K, I_K^c]||_F, is below tol.  The loop always runs at
    least one sweep, and returns H after ``max_sweeps`` with converged=False when the test
    never passes.  Stagnation guard (the FP64 floor of ||I - A H||_F can lie above tol):
    stop with floor_limited=True once the best stop value so far (the quantity compared with
    tol) is below 100 tol and no sweep has improved on it by at least 1% for sixteen sweeps
    in a row (a window long enough that the sweep-to-sweep noise of a slowly converging
    iteration, about 1% per sweep at p = 16384, does not end it early).
    ``fixed_sweeps > 0`` runs exactly that many sweeps (parity at equal sweep counts).
    """
    if tol <= 0 or max_sweeps < 1:
        raise IbmiError("INVALID_ARG", "tol must be > 0 and max_sweeps >= 1")
    bp = plan(a, blocks)
    h = initial_h(a, bp, init, h0)
    res = SolveResult(h, 0)
    limit = fixed_sweeps if fixed_sweeps > 0 else max_sweeps
    best, since_best = float("inf"), 0
    ratio, rho_eval = None, None
    while True:
        res.sweeps += 1
        sweep(h, bp)
        rho = residual_fro(a, h)
        if not np.isfinite(rho):
            raise IbmiError("NONFINITE", f"residual is not finite after sweep {res.sweeps}")
        res.history.append(rho)
        if stop == "rel_hr":
            last = fixed_sweeps > 0 and res.sweeps >= limit
            due = rho < 1.0 and (ratio is None or ratio * rho < tol or rho < 0.1 * rho_eval)
            if due or last:
                sv, _ = hr_error_bound(a, h)
                ratio, rho_eval = (sv / rho if rho > 0.0 else 0.0), rho
                res.evaluations += 1
            else:
                sv = ratio * rho if ratio is not None else float("inf")
        else:
            sv = (paper_error(a, h, bp[-1].idx, "fro") if stop == "paper"
                  else _stop_value(a, h, rho, stop, lam_min))
        res.stop_value = sv
        if sv < 0.99 * best:
            best, since_best = sv, 0
        else:
            since_best += 1
        if fixed_sweeps > 0:
            if res.sweeps >= limit:
                res.converged = sv < tol
                break
            continue
        if sv < tol:
            res.converged = True
            break
        if res.sweeps >= limit:
            break
        if stagnation_guard and best < 100.0 * tol and since_best >= GUARD_SWEEPS:
            res.floor_limited = True
            break
    return res


# --------------------------------------------------------------------------------------
# Correction (defect) form of the same block update, for the mixed-precision form.
# --------------------------------------------------------------------------------------

def _round_bf16(x32: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (round to nearest, ties to even), kept as float32."""
    u = x32.astype(np.float32).view(np.uint32).astype(np.uint64)
    bias = 0x7FFF + ((u >> 16) & 1)
    return ((u + bias) & 0xFFFF0000).astype(np.uint32).view(np.float32)


def emulate_product(x: np.ndarray, y: np.ndarray, kind: str) -> np.ndarray:
    """x @ y as a low-precision GEMM with FP32 accumulation would compute it, returned in FP64.

    ``fp64``: plain FP64.  ``fp32``: operands rounded to FP32, FP32 products and sums.
    ``bf16x3``: each operand split as hi + lo with hi = bf16(v), lo = bf16(v - hi); the
    product keeps hi*hi + hi*lo + lo*hi (the split-bfloat16 method of Henry, Tang and
    Heinecke, ARITH 2019).  ``bf16x6``: three-term split hi + mid + lo, keeping the six
    products whose term indices sum to at most 2.  Each bf16 x bf16 product is exact in
    FP32, so the FP32 GEMM over the split terms models the hardware's accumulation.

    Pinned by hand-computed products whose dropped and kept pairs are known exactly, by the
    split's error bound on random operands (with every result an FP32 number), and, for the
    bfloat16 rounding, by a brute-force rational round-to-nearest-even and the library's own
    float32 -> bfloat16 conversion.
    """
    if kind == "fp64":
        return x @ y
    x32, y32 = x.astype(np.float32), y.astype(np.float32)
    if kind == "fp32":
        return (x32 @ y32).astype(np.float64)

    def split(v64, terms):
        parts, rest = [], v64.astype(np.float32)
        for _ in range(terms):
            t = _round_bf16(rest)
            parts.append(t)
            rest = (rest - t).astype(np.float32)
        return parts

    if kind == "bf16x3":
        xs, ys = split(x, 2), split(y, 2)
        pairs = [(0, 0), (0, 1), (1, 0)]
    elif kind == "bf16x6":
        xs, ys = split(x, 3), split(y, 3)
        pairs = [(0, 0), (0, 1), (1, 0), (0, 2), (1, 1), (2, 0)]
    else:
        raise IbmiError("INVALID_ARG", f"unknown product kind {kind!r}")
    acc = np.zeros((x.shape[0], y.shape[1]), dtype=np.float32)
    for i, j in pairs:
        acc += xs[i] @ ys[j]
    return acc.astype(np.float64)


def correction_sweep(a: np.ndarray, h: np.ndarray, blocks_plan: list, product: str = "fp64") -> None:
    """One sweep of eq. (IBMI) written as corrections driven by the residual R = I - H A.

    At the start of the sweep R_s = I - H_s A is formed in FP64.  Before set k the current
    residual columns are R[:, I] = R_s[:, I] - D A[:, I], where D = H - H_s is the change made
    so far in this sweep; only this product uses the ``product`` precision.  Then, in FP64:
    Delta = R[I^c, I] A_I^{-1};  H[I^c, I] += Delta;  H[I, I^c] = H[I^c, I]^T;
    H[I, I] += (R[I, I] - Delta^T A[I^c, I]) A_I^{-1}, symmetrised.  In exact arithmetic this
    equals eq. (IBMI) (the new H makes (I - H A)[:, I] vanish); with an inexact product the
    error made is proportional to D, which shrinks as the iteration converges.
    """
    p = a.shape[0]
    h_start = h.copy()
    r_start = np.eye(p) - h_start @ a
    for bp in blocks_plan:
        i, ic = bp.idx, bp.comp
        d = h - h_start
        r_cols = r_start[:, i] - emulate_product(d, a[:, i], product)
        if ic.size == 0:
            h[np.ix_(i, i)] = bp.ainv
            continue
        delta = r_cols[ic, :] @ bp.ainv
        new_ic_i = h[np.ix_(ic, i)] + delta
        h[np.ix_(ic, i)] = new_ic_i
        h[np.ix_(i, ic)] = new_ic_i.T
        x = h[np.ix_(i, i)] + (r_cols[i, :] - delta.T @ a[np.ix_(ic, i)]) @ bp.ainv
        h[np.ix_(i, i)] = 0.5 * (x + x.T)
