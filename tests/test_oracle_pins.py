"""Pins of the CPU oracle against what the paper and the mathematics fix (no GPU needed).

Each test checks the oracle against something other than itself: a closed form derived by
hand from eq. (IBMI), the Lemma / Theorem / Corollary of the convergence section, a library
inverse, the loop-written Cholesky inverse, exact rational arithmetic, or the
multiplicative-Schwarz error propagator.  A dropped term, a sign error, a wrong index set
or a transposed operand in the oracle's block update fails at least one of them.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rel(x, y):
    return float(np.linalg.norm(x - y) / np.linalg.norm(y))


def _spd(p, seed, shift=0.1):
    return workloads.wishart_spd(p, np.random.default_rng(seed), shift=shift)


# ---------------------------------------------------------------- p = 2 closed form

def test_p2_closed_form_matches_hand_derivation():
    """p=2, sets {0},{1}: from eq. (IBMI) with scalars, after set 1
    H11 = 1/a + c^2 h/a^2, H12 = -c h/a (h = current H22); after set 2
    H22 = 1/d + c^2 H11/d^2, H21 = -c H11/d."""
    rng = np.random.default_rng(11)
    for _ in range(5):
        a_, d_ = rng.uniform(1, 3, 2)
        c_ = rng.uniform(-0.9, 0.9) * math.sqrt(a_ * d_)
        A = np.array([[a_, c_], [c_, d_]])
        h22 = 1.0
        res = oracle.ibmi_solve(A, [(0, 1), (1, 2)], tol=1e-300, fixed_sweeps=4)
        H = np.eye(2)
        P = oracle.plan(A, [(0, 1), (1, 2)])
        for _r in range(4):
            h11 = 1 / a_ + c_ * c_ * h22 / a_ ** 2
            h22 = 1 / d_ + c_ * c_ * h11 / d_ ** 2
            h21 = -c_ * h11 / d_
            oracle.sweep(H, P)
            assert H[0, 0] == pytest.approx(h11, rel=1e-14)
            assert H[1, 1] == pytest.approx(h22, rel=1e-14)
            assert H[1, 0] == pytest.approx(h21, rel=1e-14)
            assert H[0, 1] == H[1, 0]
        np.testing.assert_allclose(res.h, H, rtol=1e-14)


def test_p2_worked_example_exact_values():
    """A = [[2,1],[1,2]], H0 = I: sweep 1 gives [[3/4,-3/8],[-3/8,11/16]] and ||I-AH||_F^2 = 5/256;
    sweep 2 gives diagonal 43/64, 171/256 (hand-derived from the closed form above);
    the H22 error contracts by (c^2/(a d))^2 = 1/16 per sweep (Lemma with scalar T = 1/4)."""
    A = [[2, 1], [1, 2]]
    its = oracle.exact_ibmi(A, [[0], [1]], sweeps=3)
    F = Fraction
    assert its[0] == [[F(3, 4), F(-3, 8)], [F(-3, 8), F(11, 16)]]
    assert its[1][0][0] == F(43, 64) and its[1][1][1] == F(171, 256)
    assert its[1][0][1] == F(-43, 128)
    assert oracle.exact_residual_sq(A, its[0]) == F(5, 256)
    assert oracle.exact_residual_sq(A, its[1]) == F(5, 65536)
    for r in range(1, 3):
        assert its[r][1][1] - F(2, 3) == (its[r - 1][1][1] - F(2, 3)) / 16
    res = oracle.ibmi_solve(np.array(A, float), [(0, 1), (1, 2)], tol=1e-300, fixed_sweeps=2)
    assert res.h[0, 0] == pytest.approx(43 / 64, rel=1e-15)
    assert res.h[1, 1] == pytest.approx(171 / 256, rel=1e-15)
    assert res.history[0] ** 2 == pytest.approx(5 / 256, rel=1e-15)


# ---------------------------------------------------------------- exact rational iterates

def _golden():
    with open(os.path.join(GOLDEN, "exact_iterates.json")) as f:
        return json.load(f)


def test_exact_iterates_satisfy_block_identities():
    """Exact iterates from the golden file: after the last set I_K of a sweep,
    (I - H A)[:, I_K] = 0 exactly and H is exactly symmetric (consequences of eq. (IBMI))."""
    for case in _golden()["cases"]:
        A = [[Fraction(x) for x in row] for row in case["A"]]
        p = len(A)
        last = case["sets"][-1]
        for it in case["iterates"]:
            H = [[Fraction(x) for x in row] for row in it]
            for i in range(p):
                for j in range(p):
                    assert H[i][j] == H[j][i]
            for i in range(p):
                for j in last:
                    ha = sum((H[i][t] * A[t][j] for t in range(p)), Fraction(0))
                    assert ha == (1 if i == j else 0)


def test_float_oracle_matches_exact_iterates():
    for case in _golden()["cases"]:
        A = np.array([[float(Fraction(x)) for x in row] for row in case["A"]])
        sets = [np.array(s) for s in case["sets"]]
        P = oracle.plan(A, sets)
        H = np.eye(A.shape[0])
        for it in case["iterates"]:
            oracle.sweep(H, P)
            ref = np.array([[float(Fraction(x)) for x in row] for row in it])
            assert _rel(H, ref) < 1e-14


def test_golden_matches_exact_oracle():
    """The stored exact values are what the committed generator script produces."""
    for case in _golden()["cases"]:
        its = oracle.exact_ibmi(case["A"], case["sets"], sweeps=len(case["iterates"]))
        for got, want in zip(its, case["iterates"]):
            assert [[str(x) for x in row] for row in got] == want


# ---------------------------------------------------------------- convergence theory

def _two_block_T(A, i1, i2):
    inv = np.linalg.inv
    return inv(A[np.ix_(i2, i2)]) @ A[np.ix_(i2, i1)] @ inv(A[np.ix_(i1, i1)]) @ A[np.ix_(i1, i2)]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_lemma_error_recurrence(seed):
    """Lemma (convergence section): E_r = T^r E_0 (T^T)^r for the I_2 block, two disjoint sets,
    with T = A_{I2}^{-1} A_{I2,I1} A_{I1}^{-1} A_{I1,I2}."""
    rng = np.random.default_rng(100 + seed)
    p = 14
    A = _spd(p, seed, shift=0.3)
    perm = rng.permutation(p)
    i1, i2 = np.sort(perm[:6]), np.sort(perm[6:])
    sigma = np.linalg.inv(A)
    T = _two_block_T(A, i1, i2)
    H0 = np.eye(p)
    E0 = H0[np.ix_(i2, i2)] - sigma[np.ix_(i2, i2)]
    P = oracle.plan(A, [i1, i2])
    H = H0.copy()
    for r in range(1, 7):
        oracle.sweep(H, P)
        Tr = np.linalg.matrix_power(T, r)
        pred = Tr @ E0 @ Tr.T
        got = H[np.ix_(i2, i2)] - sigma[np.ix_(i2, i2)]
        assert np.linalg.norm(got - pred) <= 1e-11 * max(1.0, np.linalg.norm(E0))
        # Theorem: ||E_r||_2 <= ||T||_2^{2r} ||E_0||_2
        assert np.linalg.norm(got, 2) <= np.linalg.norm(T, 2) ** (2 * r) * np.linalg.norm(E0, 2) * (1 + 1e-9)


def test_corollary_exact_schur_guess_gives_inverse_in_one_step():
    """Corollary: with H0[I2,I2] equal to the exact inverse Schur complement (A^{-1})[I2,I2],
    the update for I_1 returns A^{-1}."""
    p = 12
    A = _spd(p, 5)
    sigma = np.linalg.inv(A)
    i1, i2 = np.arange(0, 5), np.arange(5, p)
    H = np.eye(p)
    H[np.ix_(i2, i2)] = sigma[np.ix_(i2, i2)]
    P = oracle.plan(A, [i1, i2])
    oracle.block_update(H, P[0])
    assert _rel(H, sigma) < 1e-12


def _schwarz_M(A, sets):
    """Multiplicative-Schwarz error propagator M = M_{I_K} ... M_{I_1},
    M_I = I - R_I^T A_I^{-1} R_I A (library inverse)."""
    p = A.shape[0]
    M = np.eye(p)
    for idx in sets:
        R = np.zeros((idx.size, p))
        R[np.arange(idx.size), idx] = 1.0
        Mi = np.eye(p) - R.T @ np.linalg.inv(A[np.ix_(idx, idx)]) @ R @ A
        M = Mi @ M
    return M


def test_overlapping_sweeps_follow_schwarz_propagator():
    """For any sets (overlapping, K > 2), H - A^{-1} maps to M (H - A^{-1}) M^T per sweep."""
    p = 20
    A = _spd(p, 7, shift=0.2)
    ranges = [(0, 8), (6, 14), (12, 20)]
    sets = [np.arange(s, e) for s, e in ranges]
    sigma = np.linalg.inv(A)
    M = _schwarz_M(A, sets)
    P = oracle.plan(A, ranges)
    H = np.eye(p)
    E = H - sigma
    for _ in range(4):
        oracle.sweep(H, P)
        E = M @ E @ M.T
        assert np.linalg.norm((H - sigma) - E) <= 1e-11 * np.linalg.norm(sigma)


def test_residual_rate_tends_to_schwarz_spectral_radius_squared():
    """Workload 1 (two sets of 128, no overlap, block-diagonal start): residual ratio -> rho(M)^2."""
    A = workloads.config1_matrix()
    ranges = oracle.partition(256, 128, 0)
    M = _schwarz_M(A, [np.arange(s, e) for s, e in ranges])
    rho = max(abs(np.linalg.eigvals(M)))
    res = oracle.ibmi_solve(A, ranges, init="blockdiag_inv", tol=1e-10, max_sweeps=200)
    assert res.sweeps == 200 and not res.converged
    ratio = res.history[-1] / res.history[-2]
    assert ratio == pytest.approx(rho ** 2, rel=2e-3)
    assert 5e-9 < res.history[-1] < 1.5e-8


# ---------------------------------------------------------------- special cases

def test_single_block_is_cholesky_inverse():
    """K = 1 (I^c empty): one update returns A_I^{-1}, i.e. the Cholesky-based inverse."""
    A = _spd(40, 3)
    res = oracle.ibmi_solve(A, [(0, 40)], tol=1e-8)
    ref = oracle.cholesky_inverse_loops(A)
    assert res.sweeps == 1 and res.converged
    assert _rel(res.h, ref) < 1e-13


def test_loop_cholesky_inverse_against_closed_forms():
    A = np.array([[4.0, 2.0], [2.0, 3.0]])
    np.testing.assert_allclose(oracle.cholesky_inverse_loops(A), np.array([[3, -2], [-2, 4]]) / 8.0,
                               rtol=1e-15)
    n = 30  # tridiag(-1, 2, -1) has inverse min(i,j)(n+1-max(i,j))/(n+1), 1-based
    T = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    i = np.arange(1, n + 1)
    ref = np.minimum.outer(i, i) * (n + 1 - np.maximum.outer(i, i)) / (n + 1)
    np.testing.assert_allclose(oracle.cholesky_inverse_loops(T), ref, rtol=1e-12, atol=1e-13)
    with pytest.raises(ValueError):
        oracle.cholesky_inverse_loops(np.array([[1.0, 2.0], [2.0, 1.0]]))


def test_block_diagonal_matrix_converges_in_one_sweep():
    A = np.zeros((12, 12))
    A[:5, :5] = _spd(5, 1)
    A[5:, 5:] = _spd(7, 2)
    res = oracle.ibmi_solve(A, [(0, 5), (5, 12)], tol=1e-12)
    assert res.sweeps == 1 and res.converged
    assert _rel(res.h, np.linalg.inv(A)) < 1e-13


def test_initial_guesses():
    """Identity is I; the block-diagonal guess holds each disjoint set's inverse (LAPACK's
    LU-based inverse, not the oracle's Cholesky route) and zeros elsewhere, and needs disjoint
    sets; a given H0 is copied, not aliased."""
    A = _spd(13, 4)
    sets = [(0, 4), (4, 9), (9, 13)]
    P = oracle.plan(A, sets)
    assert np.array_equal(oracle.initial_h(A, P, "identity"), np.eye(13))
    H = oracle.initial_h(A, P, "blockdiag_inv")
    want = np.zeros((13, 13))
    for s, e in sets:
        want[s:e, s:e] = np.linalg.inv(A[s:e, s:e])
    assert np.abs(H - want).max() < 1e-12 * np.abs(want).max()
    assert np.array_equal(H, H.T)
    h0 = _spd(13, 5)
    G = oracle.initial_h(A, P, "given", h0)
    assert np.array_equal(G, h0) and G is not h0
    with pytest.raises(oracle.IbmiError):
        oracle.initial_h(A, oracle.plan(A, [(0, 6), (4, 13)]), "blockdiag_inv")


def test_fixed_point():
    A = _spd(16, 9)
    sigma = np.linalg.inv(A)
    sigma = 0.5 * (sigma + sigma.T)
    P = oracle.plan(A, [(0, 7), (5, 12), (10, 16)])
    H = sigma.copy()
    oracle.sweep(H, P)
    assert _rel(H, sigma) < 1e-13


def test_invariants_after_every_block_step():
    """After updating set I: H exactly symmetric, H[I^c,I^c] bit-for-bit unchanged,
    (I - H A)[:, I] = 0 to rounding."""
    p = 30
    A = _spd(p, 4)
    P = oracle.plan(A, oracle.partition(p, 10, 4))
    H = np.eye(p)
    for _ in range(2):
        for bp in P:
            before = H[np.ix_(bp.comp, bp.comp)].copy()
            oracle.block_update(H, bp)
            assert np.array_equal(H, H.T)
            assert np.array_equal(H[np.ix_(bp.comp, bp.comp)], before)
            R = np.eye(p) - H @ A
            assert np.abs(R[:, bp.idx]).max() < 1e-12 * np.abs(H).max() * np.abs(A).max() * p


def test_paper_error_estimate_identity():
    """Right after updating set I, the (1,2) block of H A equals W (I - H_{I^c} S) with
    S = A_{I^c} - A_{I^c,I} A_I^{-1} A_{I,I^c} (motivation of eq. (error), sign as derived)."""
    p = 18
    A = _spd(p, 12)
    ranges = [(0, 9), (9, 18)]
    P = oracle.plan(A, ranges)
    H = np.eye(p)
    oracle.sweep(H, P)
    i, ic = np.arange(9, 18), np.arange(0, 9)
    inv = np.linalg.inv
    S = A[np.ix_(ic, ic)] - A[np.ix_(ic, i)] @ inv(A[np.ix_(i, i)]) @ A[np.ix_(i, ic)]
    W = inv(A[np.ix_(i, i)]) @ A[np.ix_(i, ic)]
    pred = np.linalg.norm(W @ (np.eye(9) - H[np.ix_(ic, ic)] @ S), 2)
    assert oracle.paper_error(A, H, i) == pytest.approx(pred, rel=1e-10)


@pytest.mark.parametrize("seed", range(4))
def test_random_spd_random_partitions_converge(seed):
    """Theorem: two disjoint sets converge for any SPD A; overlapping K=4 converges too."""
    rng = np.random.default_rng(seed)
    p = 24
    A = _spd(p, 50 + seed, shift=0.5)
    perm = rng.permutation(p)
    res = oracle.ibmi_solve(A, [perm[:10], perm[10:]], tol=1e-11, max_sweeps=3000)
    assert res.converged
    assert _rel(res.h, np.linalg.inv(A)) < 1e-9
    res = oracle.ibmi_solve(A, oracle.partition(p, 8, 2), tol=1e-11, max_sweeps=3000)
    assert res.converged


# ---------------------------------------------------------------- partition

@pytest.mark.parametrize("p,b,ovl,k_sets,sizes", [
    (256, 128, 0, 2, {128}),
    (4096, 576, 64, 8, {544, 576}),
    (16384, 576, 64, 32, {544, 576}),
    (100, 128, 16, 1, {100}),
    (128, 128, 16, 1, {128}),
])
def test_partition_workload_shapes(p, b, ovl, k_sets, sizes):
    ranges = oracle.partition(p, b, ovl)
    assert len(ranges) == k_sets
    assert {e - s for s, e in ranges} == sizes
    oracle.validate_blocks(p, ranges)
    for (s0, e0), (s1, e1) in zip(ranges, ranges[1:]):
        assert e0 - s1 == ovl


def test_partition_merges_short_last_core():
    ranges = oracle.partition(230, 128, 16)  # m = 112: cores 112, 112, 6 -> last merged
    assert ranges == [(0, 120), (104, 230)]
    for p in range(1, 3000, 7):
        r = oracle.partition(p, 128, 16)
        oracle.validate_blocks(p, r)
        assert all(e - s <= 128 + 16 for s, e in r)


# ---------------------------------------------------------------- errors

@pytest.mark.filterwarnings("ignore:invalid value encountered:RuntimeWarning")
def test_error_paths():
    A = _spd(10, 1)
    bad = A.copy()
    bad[6, 6] = -5.0
    with pytest.raises(oracle.IbmiError) as ei:
        oracle.ibmi_solve(bad, [(0, 5), (5, 10)])
    assert ei.value.code == "NOT_SPD" and ei.value.block == 1
    nan = A.copy()
    nan[0, 0] = np.nan
    with pytest.raises(oracle.IbmiError) as ei:
        oracle.ibmi_solve(nan, [(0, 5), (5, 10)])
    assert ei.value.code == "INVALID_ARG"
    unsym = A.copy()
    unsym[0, 1] += 1e-9
    with pytest.raises(oracle.IbmiError):
        oracle.ibmi_solve(unsym, [(0, 5), (5, 10)])
    with pytest.raises(oracle.IbmiError):
        oracle.ibmi_solve(A, [(0, 5), (6, 10)])
    with pytest.raises(oracle.IbmiError):
        oracle.ibmi_solve(A, [(0, 6), (4, 10)], init="blockdiag_inv")
    h0 = np.eye(10)
    h0[7, 7] = np.inf
    with pytest.raises(oracle.IbmiError) as ei:
        oracle.ibmi_solve(A, [(0, 5), (5, 10)], init="given", h0=h0)
    assert ei.value.code == "NONFINITE"


# ---------------------------------------------------------------- correction form

def test_correction_form_equals_direct_form():
    p = 40
    A = _spd(p, 21)
    P = oracle.plan(A, oracle.partition(p, 12, 4))
    H1, H2 = np.eye(p), np.eye(p)
    for _ in range(3):
        oracle.sweep(H1, P)
        oracle.correction_sweep(A, H2, P, "fp64")
        assert _rel(H2, H1) < 1e-13
        assert np.array_equal(H2, H2.T)


def test_fp32_correction_form_refines_to_fp64_accuracy():
    """With only the D A[:, I] product in FP32 the correction form still reaches the FP64
    answer (its injected error scales with the shrinking change D)."""
    A = workloads.config2_matrix(p=512)
    ranges = oracle.partition(512, 160, 32)
    P = oracle.plan(A, ranges)
    H = np.eye(512)
    for _ in range(60):
        oracle.correction_sweep(A, H, P, "fp32")
    ref = np.linalg.inv(A)
    assert _rel(H, ref) < 1e-10


def _bf16_nearest_even(v: float) -> float:
    """Brute force: the two bfloat16 neighbours of a finite float32 v (8 significant bits)
    by exact rational arithmetic, the nearer one, ties to the even significand."""
    from fractions import Fraction
    if v == 0.0:
        return v
    f = Fraction(v)
    e = math.floor(math.log2(abs(v)))
    while Fraction(2) ** e > abs(f):
        e -= 1
    while Fraction(2) ** (e + 1) <= abs(f):
        e += 1
    ulp = Fraction(2) ** (e - 7)
    lo = (abs(f) // ulp) * ulp
    hi = lo + ulp
    d_lo, d_hi = abs(f) - lo, hi - abs(f)
    if d_lo < d_hi or (d_lo == d_hi and (lo / ulp) % 2 == 0):
        r = lo
    else:
        r = hi
    return float(r if f > 0 else -r)


def test_bf16_rounding_nearest_even():
    """The oracle's float32 -> bfloat16 rounding is round to nearest, ties to even: against
    a brute-force rational rounding and the library conversion on random and tie cases."""
    import torch
    from oracle.ibmi import _round_bf16
    rng = np.random.default_rng(30)
    x = (rng.standard_normal(2000) * np.exp2(rng.integers(-30, 30, 2000))).astype(np.float32)
    # exact ties: 8 significant bits plus a half unit in the last place
    ties = np.array([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -(1 + 2.0 ** -8), 3 * 2.0 ** -9 + 2.0 ** -16,
                     1 + 2.0 ** -8 + 2.0 ** -20, 1.0, 1.5, 2.0 ** -10], dtype=np.float32)
    x = np.concatenate([x, ties])
    got = _round_bf16(x)
    want = np.array([_bf16_nearest_even(float(v)) for v in x], dtype=np.float32)
    assert np.array_equal(got, want)
    assert np.array_equal(got, torch.from_numpy(x).to(torch.bfloat16).float().numpy())
    assert got[-8] == 1.0 and got[-7] == 1 + 2.0 ** -6 and got[-4] == 1 + 2.0 ** -7


def test_split_products_closed_forms():
    """Hand-computed cases of the emulated low-precision products.  x = 1 + 2^-10 splits as
    hi = 1, lo = 2^-10: bf16x3 keeps hi*hi + 2 hi*lo = 1 + 2^-9 and drops lo*lo = 2^-20;
    bf16x6 keeps it (three terms, pair (1,1)), so it returns x^2 exactly; FP32 rounds x^2 =
    1 + 2^-9 + 2^-20 exactly too (21 bits).  Sums run in FP32: 1 + 2^-30 accumulates to 1."""
    x = np.array([[1 + 2.0 ** -10]])
    assert oracle.emulate_product(x, x, "bf16x3")[0, 0] == 1 + 2.0 ** -9
    assert oracle.emulate_product(x, x, "bf16x6")[0, 0] == (1 + 2.0 ** -10) ** 2
    assert oracle.emulate_product(x, x, "fp32")[0, 0] == (1 + 2.0 ** -10) ** 2
    row, col = np.array([[1.0, 2.0 ** -30]]), np.array([[1.0], [1.0]])
    for kind in ("fp32", "bf16x3", "bf16x6"):
        assert oracle.emulate_product(row, col, kind)[0, 0] == 1.0
    assert oracle.emulate_product(row, col, "fp64")[0, 0] == 1 + 2.0 ** -30
    # a second term that needs the third split term: hi = 1, mid = 2^-9, lo = 2^-17
    y = np.array([[1 + 2.0 ** -9 + 2.0 ** -17]])
    one = np.array([[1.0]])
    assert oracle.emulate_product(y, one, "bf16x3")[0, 0] == 1 + 2.0 ** -9
    assert oracle.emulate_product(y, one, "bf16x6")[0, 0] == 1 + 2.0 ** -9 + 2.0 ** -17


@pytest.mark.parametrize("kind,u", [("bf16x3", 2.0 ** -16), ("bf16x6", 2.0 ** -23)])
def test_split_products_within_their_error_bound(kind, u):
    """On random operands each emulated entry lies within the split's bound of the FP64
    product: per term the dropped pairs are below 3u |x||y| (two operands, each term split
    to relative 2^-8 per term), and the FP32 sum over n terms adds at most n 2^-24 |x||y|."""
    rng = np.random.default_rng(31)
    n = 200
    x, y = rng.standard_normal((30, n)), rng.standard_normal((n, 20))
    got = oracle.emulate_product(x, y, kind)
    scale = np.abs(x) @ np.abs(y)
    assert np.all(np.abs(got - x @ y) <= (3 * u + n * 2.0 ** -24) * scale)
    # FP32 accumulation: every entry is an FP32 number
    assert np.array_equal(got.astype(np.float32).astype(np.float64), got)
    # the kept pairs matter: the leading bfloat16 terms alone are far off
    from oracle.ibmi import _round_bf16
    hx = _round_bf16(x.astype(np.float32)).astype(np.float64)
    hy = _round_bf16(y.astype(np.float32)).astype(np.float64)
    assert np.abs(got - x @ y).max() < 0.01 * np.abs(hx @ hy - x @ y).max()


def test_stagnation_guard_stops_at_the_floor():
    """A tolerance below the FP64 floor of ||I - A H||_F ends with floor_limited, not at the
    cap; the same matrix with a reachable tolerance converges."""
    A = workloads.config2_matrix(p=1500)
    ranges = oracle.partition(1500, 576, 64)
    res = oracle.ibmi_solve(A, ranges, tol=1e-11, max_sweeps=500)  # floor here: 2.9e-10
    assert res.floor_limited and not res.converged and res.sweeps < 30
    best = min(res.history)
    assert best < 100 * 1e-11 and all(h > 0.99 * best for h in res.history[-16:])
    res2 = oracle.ibmi_solve(A, ranges, tol=1e-8, max_sweeps=500)
    assert res2.converged and not res2.floor_limited


def test_stagnation_guard_works_in_the_stop_test_units():
    """With the relative-error bound as stop test the guard compares that bound (not the
    residual, which sits near 3e-10 here) with 100 tol: a bound tolerance below the floor the
    bound reaches (about 1.3e-11) ends with floor_limited."""
    A = workloads.config2_matrix(p=1500)
    ranges = oracle.partition(1500, 576, 64)
    res = oracle.ibmi_solve(A, ranges, tol=1e-12, stop="rel_bound", lam_min=1e-2,
                            max_sweeps=500)
    bound = res.history[-1] / (1e-2 * np.linalg.norm(res.h))
    assert res.floor_limited and not res.converged and res.sweeps < 40
    assert 1e-12 < bound < 100 * 1e-12


def test_hr_bound_closed_form_scaled_inverse():
    """H = (1 - d) A^{-1} for diagonal A: R = d I, H R = d (1 - d) A^{-1}, so the bound is
    x / (1 - x) with x = d / (1 - d sqrt(p)), and the true relative error is d <= bound."""
    p, d = 50, 1e-3
    A = np.diag(np.arange(1.0, p + 1.0))
    H = (1.0 - d) * np.diag(1.0 / np.arange(1.0, p + 1.0))
    bound, rho = oracle.hr_error_bound(A, H)
    x = d / (1.0 - d * np.sqrt(p))
    assert rho == pytest.approx(d * np.sqrt(p), rel=1e-12)
    assert bound == pytest.approx(x / (1.0 - x), rel=1e-10)
    assert bound >= d
    assert oracle.hr_error_bound(A, 0.5 * np.linalg.inv(A))[0] == float("inf")  # ||R||_F >= 1


def test_hr_bound_is_certified_and_tight_along_iteration():
    """Along an IBMI iteration the bound is never below the true relative error (computed
    from LAPACK's inverse) and is tight to first order in ||R||_F: once ||R||_F < 0.1 it
    exceeds the true error by less than a factor 1 + 1.5 ||R||_F."""
    A = workloads.wishart_spd(400, np.random.default_rng(11), shift=0.05)
    ranges = oracle.partition(400, 120, 16)
    P = oracle.plan(A, ranges)
    H = np.eye(400)
    inv = np.linalg.inv(A)
    seen = 0
    for r in range(40):
        oracle.sweep(H, P)
        bound, rho = oracle.hr_error_bound(A, H)
        true = _rel(H, inv)
        if np.isfinite(bound):
            assert bound >= true * (1 - 1e-9)
            if rho < 0.1:
                assert bound <= (1.0 + 1.5 * rho) * true
                seen += 1
    assert seen >= 5


def test_rel_hr_stop_ends_at_the_true_error():
    """The rel_hr stop converges once the certified bound is below tol, evaluating the
    bound at a few sweeps only; the true error of the returned H is below tol while one
    sweep earlier it was not."""
    A = workloads.config2_matrix(p=1200)
    ranges = oracle.partition(1200, 300, 40)
    tol = 1e-9
    res = oracle.ibmi_solve(A, ranges, tol=tol, stop="rel_hr", max_sweeps=300)
    inv = np.linalg.inv(A)
    assert res.converged and res.stop_value < tol
    assert _rel(res.h, inv) < tol
    assert 1 <= res.evaluations <= 10 and res.evaluations < res.sweeps
    prev = oracle.ibmi_solve(A, ranges, tol=1e-300, fixed_sweeps=res.sweeps - 1)
    assert _rel(prev.h, inv) > 0.5 * tol


def test_paper_estimate_frobenius_form():
    """The Frobenius form of eq. (error) is the Frobenius norm of the (1,2) block of H A (the
    two-term expression is that block split over I and I^c), bounds the paper's spectral
    form from above, and vanishes at A^{-1}; the "paper" stop test ends a solve on it."""
    A = workloads.wishart_spd(300, np.random.default_rng(4), shift=0.3)
    ranges = oracle.partition(300, 100, 20)
    res = oracle.ibmi_solve(A, ranges, tol=1e-300, fixed_sweeps=3)
    idx = np.arange(*ranges[-1])
    ic = np.setdiff1d(np.arange(300), idx)
    fro = oracle.paper_error(A, res.h, idx, "fro")
    assert fro == pytest.approx(np.linalg.norm((res.h @ A)[np.ix_(idx, ic)]), rel=1e-10)
    assert fro >= oracle.paper_error(A, res.h, idx) * (1 - 1e-12)
    assert oracle.paper_error(A, np.linalg.inv(A), idx, "fro") < 1e-10
    sol = oracle.ibmi_solve(A, ranges, tol=1e-8, stop="paper", max_sweeps=200)
    assert sol.converged and sol.stop_value < 1e-8
    assert oracle.paper_error(A, sol.h, idx, "fro") == pytest.approx(sol.stop_value, rel=1e-12)
