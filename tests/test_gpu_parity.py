"""Parity of the HIP path (through the C ABI) with the CPU oracle, on seeded inputs.

Bar (FP64 path): relative Frobenius error of H <= 1e-10 against the oracle at the SAME sweep
count; residual histories agree to the same relative level.  Integer work (the partition) is
bit-exact.  Sizes span several 64/128 tiles with ragged tails; the full 16384 workload is
checked on outputs the oracle can compute one set at a time and on properties that hold at
any size.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu
TOL = 1e-10


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def ib():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2502_06377_amd as m
    return m


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _rel(x, y):
    return float(np.linalg.norm(x - y) / np.linalg.norm(y))


def _gpu_solve(ib, A, **kw):
    plan = ib.Plan(_dev(A), **kw)
    out = plan.solve()
    torch.cuda.synchronize()
    H = out.H.cpu().numpy()
    plan.close()
    return out, H


def _resid_atol(A, H):
    """Rounding level of ||I - A H||_F in FP64: each entry of A H carries an error of about
    sqrt(p) u sum_k |A_ik||H_kj| (random-walk bound on p terms), so two correct evaluations
    of the residual norm may differ by up to about sqrt(p) u || |A| |H| ||_F."""
    p = A.shape[0]
    return 4.0 * np.sqrt(p) * np.finfo(float).eps * np.linalg.norm(np.abs(A) @ np.abs(H))


def _compare(ib, A, ranges, sweeps, init="identity", **kw):
    p = A.shape[0]
    ref = oracle.ibmi_solve(A, ranges, init=init, tol=1e-300, fixed_sweeps=sweeps)
    out, H = _gpu_solve(ib, A, bounds=ranges, init=init, fixed_sweeps=sweeps, tol=1e-300, **kw)
    assert out.sweeps == ref.sweeps == sweeps
    assert np.array_equal(H, H.T), "H must be bitwise symmetric"
    err = _rel(H, ref.h)
    assert err <= TOL, f"relative Frobenius error {err:.3e}"
    np.testing.assert_allclose(out.history, ref.history, rtol=1e-10, atol=_resid_atol(A, ref.h))
    return out, H, ref


def test_workload1_two_blocks_200_sweeps(ib):
    _say("workload 1: p=256, two sets of 128, blockdiag init, 200 sweeps")
    A = workloads.config1_matrix()
    ranges = oracle.partition(256, 128, 0)
    out, H, ref = _compare(ib, A, ranges, 200, init="blockdiag_inv")
    assert 5e-9 < out.history[-1] < 1.5e-8


@pytest.mark.parametrize("p,b,ovl,seed", [(300, 100, 20, 0), (517, 96, 32, 1), (130, 64, 8, 2),
                                          (1000, 256, 40, 3)])
def test_ragged_random_spd(ib, p, b, ovl, seed):
    _say(f"ragged wishart p={p} b={b} ovl={ovl}")
    A = workloads.wishart_spd(p, np.random.default_rng(seed), shift=0.3)
    _compare(ib, A, oracle.partition(p, b, ovl), 3)


@pytest.mark.parametrize("precision", ["fp64", "bf16x3"])
def test_branch_free_path_with_edge_tiles(ib, precision):
    """Sets of 272 rows at p = 1040: every K range (c = 768, p = 1040) is a whole number of
    stages, so the products take the branch-free loop, while 272 rows and 1040 columns leave
    partial edge tiles that load the last valid columns in place of missing ones."""
    _say(f"branch-free path with edge tiles p=1040 b=272 ({precision})")
    A = workloads.wishart_spd(1040, np.random.default_rng(21), shift=0.3)
    ranges = [(0, 272), (256, 528), (512, 784), (768, 1040)]
    if precision == "fp64":
        _compare(ib, A, ranges, 3)
        return
    bp = oracle.plan(A, ranges)
    h_emul, h64 = np.eye(1040), np.eye(1040)
    for _ in range(2):
        oracle.correction_sweep(A, h_emul, bp, precision)
        oracle.correction_sweep(A, h64, bp, "fp64")
    out, H = _gpu_solve(ib, A, bounds=ranges, precision=precision, tol=1e-300, fixed_sweeps=2)
    assert np.array_equal(H, H.T)
    # A wrong edge load corrupts outputs at O(1); the split rounding itself is ~1e-6 here and
    # FP32 accumulation order moves the result by about a third of that (CPU emulation).
    assert _rel(H, h_emul) < 2.0 * _rel(h_emul, h64)


def test_odd_explicit_bounds(ib):
    _say("explicit odd bounds p=151")
    A = workloads.wishart_spd(151, np.random.default_rng(9), shift=0.3)
    ranges = [(0, 37), (30, 101), (95, 151)]
    _compare(ib, A, ranges, 4)


def test_single_block_is_inverse(ib):
    _say("single set p=200")
    A = workloads.config2_matrix(p=200)
    out, H, ref = _compare(ib, A, [(0, 200)], 1)
    assert _rel(H, oracle.cholesky_inverse_loops(A)) < 1e-12


def test_workload2_fixed_sweeps(ib):
    _say("workload 2: p=4096 Matern-3/2, 8 sets of 576/544, 4 sweeps")
    A = workloads.config2_matrix()
    _compare(ib, A, oracle.partition(4096, 576, 64), 4)


def test_block_step_invariants(ib):
    _say("block step invariants p=700")
    p = 700
    A = workloads.config2_matrix(p=p)
    plan = ib.Plan(_dev(A), block_rows=200, overlap=24)
    H = torch.empty((p, p), dtype=torch.float64, device="cuda")
    ib.ibmi_init_h(plan.handle, H)
    Hn = H.cpu().numpy()
    for k, (s, e) in enumerate(plan.blocks):
        before = Hn.copy()
        ib.ibmi_block_step(plan.handle, H, k)
        torch.cuda.synchronize()
        Hn = H.cpu().numpy()
        idx = np.arange(s, e)
        ic = oracle.complement(p, idx)
        assert np.array_equal(Hn, Hn.T)
        assert np.array_equal(Hn[np.ix_(ic, ic)], before[np.ix_(ic, ic)])
        R = np.eye(p) - Hn @ A
        assert np.abs(R[:, idx]).max() < 1e-12 * np.abs(Hn).max() * np.abs(A).max() * p
    plan.close()


def test_residual_matches_numpy(ib):
    _say("residual p=333")
    rng = np.random.default_rng(4)
    A = workloads.wishart_spd(333, rng)
    H = rng.standard_normal((333, 333)) * 0.01
    plan = ib.Plan(_dev(A), block_rows=128, overlap=16)
    got = plan.residual(_dev(H))
    want = np.linalg.norm(np.eye(333) - A @ H)
    assert got == pytest.approx(want, rel=1e-13)
    plan.close()


def test_not_spd_reports_block(ib):
    _say("not SPD")
    A = workloads.wishart_spd(300, np.random.default_rng(5))
    A[150, 150] = -1.0
    with pytest.raises(ib.IbmiError) as ei:
        ib.Plan(_dev(A), block_rows=100, overlap=0)
    assert ei.value.status == ib.IBMI_ERR_NOT_SPD and ei.value.block == 1


@pytest.mark.filterwarnings("ignore:invalid value encountered:RuntimeWarning")
def test_nonfinite_inputs_are_reported(ib):
    """NaN inside a diagonal block fails its Cholesky pivot (NOT_SPD with that block); NaN only
    in an off-diagonal block surfaces as a NaN residual after the first sweep (NONFINITE): the
    library does not scan A (the oracle rejects a non-finite A up front).  An Inf in the part
    of a given initial H that the first set reads gives NONFINITE in both; one in rows the
    first set overwrites is never read, and both solve normally."""
    _say("nonfinite inputs p=300")
    base = workloads.wishart_spd(300, np.random.default_rng(5))
    ranges = [(0, 100), (100, 200), (200, 300)]
    A = base.copy()
    A[150, 151] = A[151, 150] = np.nan
    with pytest.raises(ib.IbmiError) as ei:
        ib.Plan(_dev(A), bounds=ranges)
    assert ei.value.status == ib.IBMI_ERR_NOT_SPD and ei.value.block == 1
    A = base.copy()
    A[0, 299] = A[299, 0] = np.nan
    plan = ib.Plan(_dev(A), bounds=ranges, max_sweeps=5)
    with pytest.raises(ib.IbmiError) as ei:
        plan.solve()
    assert ei.value.status == ib.IBMI_ERR_NONFINITE
    plan.close()
    for (i, j), bad in (((150, 250), True), ((10, 250), False)):
        h0 = np.eye(300)
        h0[i, j] = h0[j, i] = np.inf
        plan = ib.Plan(_dev(base), bounds=ranges, max_sweeps=5, tol=1e-300, init="given")
        if bad:
            with pytest.raises(oracle.IbmiError) as eo:
                oracle.ibmi_solve(base, ranges, init="given", h0=h0, tol=1e-300, max_sweeps=5)
            assert eo.value.code == "NONFINITE"
            with pytest.raises(ib.IbmiError) as ei:
                plan.solve(_dev(h0))
            assert ei.value.status == ib.IBMI_ERR_NONFINITE
        else:
            ref = oracle.ibmi_solve(base, ranges, init="given", h0=h0, tol=1e-300, max_sweeps=5)
            out = plan.solve(_dev(h0))
            assert out.sweeps == ref.sweeps == 5
            assert _rel(out.H.cpu().numpy(), ref.h) <= TOL
        plan.close()


def test_deterministic_and_resume(ib):
    _say("determinism and resume p=400")
    A = workloads.config2_matrix(p=400)
    plan = ib.Plan(_dev(A), block_rows=128, overlap=16, fixed_sweeps=5, tol=1e-300)
    h1 = plan.solve().H.clone()
    h2 = plan.solve().H.clone()
    assert torch.equal(h1, h2)
    plan.close()
    p3 = ib.Plan(_dev(A), block_rows=128, overlap=16, fixed_sweeps=3, tol=1e-300)
    h3 = p3.solve().H
    p2 = ib.Plan(_dev(A), block_rows=128, overlap=16, fixed_sweeps=2, tol=1e-300, init="given")
    h5 = p2.solve(h3).H
    assert torch.equal(h5, h1)
    p3.close()
    p2.close()


def test_stop_tests_converge(ib):
    """Both stop tests on a well-conditioned matrix (shift 0.3 bounds lambda_min below), with
    tolerances far from the FP64 floor so that the crossing sweep is unambiguous."""
    _say("stop tests p=1200")
    A = workloads.wishart_spd(1200, np.random.default_rng(8), shift=0.3)
    ranges = oracle.partition(1200, 256, 32)
    out, H = _gpu_solve(ib, A, block_rows=256, overlap=32, tol=1e-8, max_sweeps=500)
    ref = oracle.ibmi_solve(A, ranges, tol=1e-8, max_sweeps=500)
    assert out.converged and ref.converged and out.sweeps == ref.sweeps
    assert _rel(H, ref.h) <= TOL
    out2, H2 = _gpu_solve(ib, A, block_rows=256, overlap=32, stop="rel_bound", lambda_min=0.3,
                          tol=1e-11, max_sweeps=500)
    assert out2.converged and out2.stop_value < 1e-11
    assert _rel(H2, np.linalg.inv(A)) < 1e-11
    out3, _ = _gpu_solve(ib, A, block_rows=256, overlap=32, tol=1e-300, max_sweeps=3)
    assert out3.sweeps == 3 and not out3.converged


def test_full_size_16384_first_block_and_properties(ib):
    """Workload 3 at full size: after one block step from H = I the rows of set 0 are
    H[I,I^c] = -W and H[I,I] = A_I^{-1} + W W^T (eq. (IBMI) with H_{I^c} = I), which the oracle
    computes for that set alone; after a full sweep (I - H A)[:, I_K] = 0 on sampled columns."""
    _say("workload 3 full size p=16384: block 0 and sweep properties")
    A = workloads.config3_matrix()
    p = A.shape[0]
    plan = ib.Plan(_dev(A), block_rows=576, overlap=64)
    assert plan.blocks == oracle.partition(p, 576, 64)
    H = torch.empty((p, p), dtype=torch.float64, device="cuda")
    ib.ibmi_init_h(plan.handle, H)
    ib.ibmi_block_step(plan.handle, H, 0)
    torch.cuda.synchronize()
    s, e = plan.blocks[0]
    bp = oracle.block_factors(A, s, e)
    rows = H[s:e].cpu().numpy()
    want_off = -bp.w
    want_diag = bp.ainv + bp.w @ bp.w.T
    assert _rel(rows[:, bp.comp], want_off) <= TOL
    assert _rel(rows[:, bp.idx], want_diag) <= TOL
    for k in range(1, len(plan.blocks)):
        ib.ibmi_block_step(plan.handle, H, k)
    torch.cuda.synchronize()
    s, e = plan.blocks[-1]
    cols = np.arange(s, e, 61)
    Hh = H.cpu().numpy()
    assert np.array_equal(Hh[::97], Hh[:, ::97].T)
    R = np.eye(p)[:, cols] - Hh @ A[:, cols]
    assert np.abs(R).max() < 1e-12 * np.abs(Hh).max() * np.abs(A).max() * p
    res = plan.residual(H)
    assert np.isfinite(res) and res > 0
    plan.close()


def test_max_size_past_int32_element_count(ib):
    """p = 46400, so p^2 exceeds 2^31 - 1 and every flat index of A, H and the workspace must
    be 64-bit (the largest benchmark matrix has p^2 = 2.7e8).  Matern-3/2 (workload 2's
    kernel) on seeded points, built in row chunks straight into device memory.  After block
    step 0 from H = I the rows of set 0 match the oracle's (eq. (IBMI) with H_{I^c} = I);
    after the full sweep H is bitwise symmetric on sampled rows, (I - H A)[:, I_K] = 0 on
    sampled columns of the last set, and the residual is finite."""
    p = 46400
    assert p * p > 2 ** 31 - 1
    _say(f"max size p={p}: block 0 vs oracle, sweep properties")
    pts = workloads.sorted_points(p, 2, np.random.default_rng(2))
    A = torch.empty((p, p), dtype=torch.float64, device="cuda")
    ranges = oracle.partition(p, 576, 64)
    s0, e0 = ranges[0]
    a_host = np.empty((p, p))  # only rows of set 0 are filled (pages of the rest untouched)
    for r0, r1, rows in workloads.covariance_row_chunks(pts, "matern32", 0.1, 1e-2):
        A[r0:r1].copy_(torch.from_numpy(rows))
        if r0 < e0:
            a_host[r0:min(r1, e0)] = rows[:min(r1, e0) - r0]
    plan = ib.Plan(A, block_rows=576, overlap=64)
    assert plan.blocks == ranges
    H = torch.empty((p, p), dtype=torch.float64, device="cuda")
    ib.ibmi_init_h(plan.handle, H)
    ib.ibmi_block_step(plan.handle, H, 0)
    torch.cuda.synchronize()
    bp = oracle.block_factors(a_host, s0, e0)
    del a_host
    rows = H[s0:e0].cpu().numpy()
    assert _rel(rows[:, bp.comp], -bp.w) <= TOL
    assert _rel(rows[:, bp.idx], bp.ainv + bp.w @ bp.w.T) <= TOL
    for k in range(1, len(ranges)):
        ib.ibmi_block_step(plan.handle, H, k)
    torch.cuda.synchronize()
    assert torch.equal(H[::997], H[:, ::997].T)
    s, e = ranges[-1]
    cols = torch.arange(s, e, 61, device="cuda")
    eye = torch.zeros((p, cols.numel()), dtype=torch.float64, device="cuda")
    eye[cols, torch.arange(cols.numel(), device="cuda")] = 1.0
    R = eye - H @ A[:, cols].contiguous()
    bound = 1e-12 * H.abs().max().item() * A.abs().max().item() * p
    assert R.abs().max().item() < bound
    res = plan.residual(H)
    assert np.isfinite(res) and res > 0
    plan.close()


# ------------------------------------------------------------ low-precision update forms

MIXED = ["fp32", "bf16x3", "bf16x6"]
# Unit roundoff of the update product: FP32, a two-term bfloat16 split (16 significant bits,
# the dropped lo*lo term is of the same order), a three-term split (about FP32's).
U_LOW = {"fp32": 2.0 ** -24, "bf16x3": 2.0 ** -16, "bf16x6": 2.0 ** -23}


# Largest ratio of the low-precision form's residual to the FP64 form's over the first four
# sweeps of workload 3 (measured on MI355X: fp32 1.024, bf16x3 1.72; deterministic kernels).
FULL_SIZE_RATIO = {"fp32": 1.05, "bf16x3": 2.0}


@pytest.mark.parametrize("form", ["fp32", "bf16x3"])
def test_full_size_16384_mixed_sweeps_track_fp64(ib, form):
    """Workload 3 at full size in a low-precision update form, with the tiles and K chunks the
    benchmark times, against the FP64 form (checked at this size above).  From H = I the
    first sweeps change H by far more than H itself will later move, so the low-precision
    product D A of the correction form rounds against |D||A| ~ 1e4 while D A ~ 1: the
    residual runs above the FP64 one (bf16x3 most), but stays within a small factor of it.
    A lost K chunk, tile or term would leave entries of D A itself in R and stall the sweep.
    H stays bitwise symmetric."""
    _say(f"workload 3 full size p=16384, {form} vs fp64: residuals of 4 sweeps")
    A = _dev(workloads.config3_matrix())
    p = A.shape[0]
    hist = {}
    for f in ("fp64", form):
        plan = ib.Plan(A, block_rows=576, overlap=64, precision=f, tol=1e-300, fixed_sweeps=4)
        out = plan.solve()
        torch.cuda.synchronize()
        assert out.sweeps == 4
        hist[f] = np.asarray(out.history[:4])
        if f == form:
            Hs = out.H[::97].cpu().numpy()
            Hc = out.H[:, ::97].cpu().numpy()
            assert np.array_equal(Hs, Hc.T)
        plan.close()
    ratio = hist[form] / hist["fp64"]
    _say(f"residual ratios {np.array2string(ratio, precision=4)}")
    assert np.all(np.isfinite(ratio))
    assert np.all(ratio >= 0.99) and np.all(ratio <= FULL_SIZE_RATIO[form])


@pytest.mark.parametrize("form", MIXED)
def test_mixed_form_refines_to_fp64_oracle(ib, form):
    """Low-precision matrix-core products in the correction form, FP64 factors and residual:
    the converged H matches the FP64 oracle's converged H to the FP64 bar."""
    _say(f"{form} form p=2048 Matern-3/2 to rel bound 1e-10")
    A = workloads.config2_matrix(p=2048)
    ranges = oracle.partition(2048, 576, 64)
    ref = oracle.ibmi_solve(A, ranges, tol=1e-10, stop="rel_bound", lam_min=1e-2, max_sweeps=500)
    assert ref.converged
    out, H = _gpu_solve(ib, A, block_rows=576, overlap=64, precision=form, stop="rel_bound",
                        lambda_min=1e-2, tol=1e-10, max_sweeps=500)
    assert out.converged and np.array_equal(H, H.T)
    assert abs(out.sweeps - ref.sweeps) <= (2 if form != "bf16x3" else 4)
    assert _rel(H, ref.h) <= TOL


@pytest.mark.parametrize("form", MIXED)
def test_mixed_form_ragged_against_inverse(ib, form):
    _say(f"{form} form ragged wishart p=1000 b=256 ovl=40")
    A = workloads.wishart_spd(1000, np.random.default_rng(3), shift=0.3)
    out, H = _gpu_solve(ib, A, block_rows=256, overlap=40, precision=form, stop="rel_bound",
                        lambda_min=0.3, tol=1e-12, max_sweeps=500)
    assert out.converged
    assert _rel(H, np.linalg.inv(A)) <= TOL
    ref = oracle.ibmi_solve(A, oracle.partition(1000, 256, 40), tol=1e-12, stop="rel_bound",
                            lam_min=0.3)
    assert _rel(H, ref.h) <= TOL


@pytest.mark.parametrize("form", MIXED)
def test_mixed_first_sweeps_close_to_fp64(ib, form):
    """Two low-precision sweeps differ from the FP64 sweeps only by the rounding of the
    product D A[:,I]; D is bounded by |H| there, so the difference is a small multiple of
    u_low * kappa.  p = 777 leaves a ragged row stride for the FP32 copies."""
    _say(f"{form} vs fp64 two sweeps p=777")
    A = workloads.wishart_spd(777, np.random.default_rng(6), shift=0.5)
    ranges = oracle.partition(777, 200, 24)
    ref = oracle.ibmi_solve(A, ranges, tol=1e-300, fixed_sweeps=2)
    out, H = _gpu_solve(ib, A, bounds=ranges, precision=form, tol=1e-300, fixed_sweeps=2)
    kappa = np.linalg.cond(A)
    assert _rel(H, ref.h) < 100 * U_LOW[form] * kappa


@pytest.mark.parametrize("form", ["bf16x3", "bf16x6"])
def test_split_products_match_emulation(ib, form):
    """The matrix-core split-bfloat16 product is the oracle's emulated one (same terms, same
    dropped pairs, round to nearest even) up to FP32 accumulation order.  Measured on the CPU
    for this case (bf16x3): emulation vs FP64 1.2e-5, two FP32 accumulation orders 3.2e-6,
    truncating instead of rounding 3.9e-5 away, keeping only hi*hi 6.7e-2 away.  So the GPU
    H must sit nearer the emulation than half the emulation's distance from FP64.  For
    bf16x6 the split error is at the accumulation-order level (4e-7), so only a lost or
    extra term (1.2e-5 for the bf16x3 pairs) is detectable: within 3x of that distance."""
    _say(f"{form} vs emulated {form} two sweeps p=900")
    A = workloads.config2_matrix(p=900)
    ranges = oracle.partition(900, 256, 32)
    bp = oracle.plan(A, ranges)
    h_emul, h64 = np.eye(900), np.eye(900)
    for _ in range(2):
        oracle.correction_sweep(A, h_emul, bp, form)
        oracle.correction_sweep(A, h64, bp, "fp64")
    out, H = _gpu_solve(ib, A, bounds=ranges, precision=form, tol=1e-300, fixed_sweeps=2)
    gap_low = _rel(h_emul, h64)
    assert gap_low > 0
    limit = 0.5 if form == "bf16x3" else 3.0
    assert _rel(H, h_emul) < limit * gap_low, (_rel(H, h_emul), gap_low)


@pytest.mark.parametrize("form", ["fp64", "fp32", "bf16x3"])
def test_rel_hr_stop_matches_oracle(ib, form):
    """The H R relative-error stop: same stopping sweep as the oracle (FP64 form: same
    evaluations too, and the same H to the FP64 bar), and the returned H is within tol of
    LAPACK's inverse."""
    _say(f"rel_hr stop, {form} form, p=1200 Matern-3/2, tol 1e-9")
    A = workloads.config2_matrix(p=1200)
    ranges = oracle.partition(1200, 300, 40)
    ref = oracle.ibmi_solve(A, ranges, tol=1e-9, stop="rel_hr", max_sweeps=300)
    assert ref.converged
    out, H = _gpu_solve(ib, A, bounds=ranges, precision=form, tol=1e-9, stop="rel_hr",
                        max_sweeps=300)
    assert out.converged and out.stop_value < 1e-9
    assert _rel(H, np.linalg.inv(A)) < 1e-9
    if form == "fp64":
        assert out.sweeps == ref.sweeps and out.evaluations == ref.evaluations
        assert out.stop_value == pytest.approx(ref.stop_value, rel=0.02)  # R rounding noise
        assert _rel(H, ref.h) <= TOL
    else:
        assert abs(out.sweeps - ref.sweeps) <= 2


def test_paper_stop_matches_oracle(ib):
    """Stop on the Frobenius form of the paper's eq. (error) estimate for the last set: same
    stopping sweep and stop value as the oracle, and the same H."""
    _say("paper estimate stop p=700, tol 1e-8")
    A = workloads.wishart_spd(700, np.random.default_rng(14), shift=0.3)
    ranges = oracle.partition(700, 200, 24)
    ref = oracle.ibmi_solve(A, ranges, tol=1e-8, stop="paper", max_sweeps=300)
    out, H = _gpu_solve(ib, A, bounds=ranges, tol=1e-8, stop="paper", max_sweeps=300)
    assert ref.converged and out.converged and out.sweeps == ref.sweeps
    # both sides evaluate the block with FP64 rounding of their own order
    assert out.stop_value == pytest.approx(ref.stop_value, rel=1e-4)
    assert _rel(H, ref.h) <= TOL


def test_stagnation_guard_matches_oracle(ib):
    """A tolerance below the FP64 floor: both sides stop with floor_limited within a few
    sweeps of each other.  The floor itself is the rounding level of evaluating I - A H and
    depends on the summation order: the oracle's blocked BLAS sums reach about 2.9e-10 here,
    the matrix cores' sequential sums over k about 1.1e-9, so tol = 1e-10 lies below both
    floors while 100 tol lies above both."""
    _say("stagnation guard p=1500 Matern-3/2, tol 1e-10")
    A = workloads.config2_matrix(p=1500)
    ranges = oracle.partition(1500, 576, 64)
    ref = oracle.ibmi_solve(A, ranges, tol=1e-10, max_sweeps=500)
    out, H = _gpu_solve(ib, A, bounds=ranges, tol=1e-10, max_sweeps=500)
    assert ref.floor_limited and out.floor_limited and not out.converged
    assert abs(out.sweeps - ref.sweeps) <= 4, (out.sweeps, ref.sweeps)
    assert min(out.history) < max(10 * min(ref.history), _resid_atol(A, ref.h))


def test_sweep_entry_point_matches_solve(ib):
    _say("ibmi_sweep vs ibmi_solve p=640")
    A = workloads.config2_matrix(p=640)
    for prec in ("fp64", "fp32", "bf16x3"):
        plan = ib.Plan(_dev(A), block_rows=200, overlap=24, precision=prec, fixed_sweeps=3,
                       tol=1e-300)
        h_solve = plan.solve().H.clone()
        H = torch.empty_like(h_solve)
        ib.ibmi_init_h(plan.handle, H)
        res = [ib.ibmi_sweep(plan.handle, H, r == 0) for r in range(3)]
        torch.cuda.synchronize()
        assert torch.equal(H, h_solve), prec
        assert res[-1] == pytest.approx(plan.residual(H), rel=1e-12)
        plan.close()


def test_progress_callback_can_stop(ib):
    _say("progress callback cancels after 3 sweeps")
    A = workloads.config2_matrix(p=700)
    plan = ib.Plan(_dev(A), block_rows=200, overlap=24, tol=1e-14, max_sweeps=50)
    seen = []
    out = plan.solve(progress=lambda r, res, sv: seen.append((r, res)) or r >= 3)
    assert out.sweeps == 3 and out.cancelled and not out.converged
    assert [r for r, _ in seen] == [1, 2, 3]
    assert seen[-1][1] == out.residual
    plan.close()
