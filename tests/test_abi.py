"""The C-ABI library loads and exports every entry point include/ibmi.h declares; host-only
entry points (partitioner, workspace sizing, status strings) agree with the oracle.
No device work is launched here."""
import ctypes
import os
import re

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ibmi.h")
LIB = os.path.join(ROOT, "paper_2502_06377_amd", "libibmi.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ibmi_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def binding():
    if not os.path.exists(LIB):
        pytest.fail("libibmi.so is not built (run python paper_2502_06377_amd/build.py)")
    import paper_2502_06377_amd as m
    return m


def test_every_declared_symbol_is_exported(binding):
    lib = ctypes.CDLL(LIB)
    names = _declared()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(binding.EXPORTED)


@pytest.mark.parametrize("p,b,ovl", [(256, 128, 0), (4096, 576, 64), (16384, 576, 64), (100, 128, 16),
                                     (230, 128, 16), (1000, 128, 16), (7, 3, 1), (8192, 576, 64)])
def test_partition_matches_oracle(binding, p, b, ovl):
    assert binding.ibmi_partition(p, b, ovl) == oracle.partition(p, b, ovl)


def test_partition_sweep_matches_oracle(binding):
    for p in range(1, 2100, 13):
        for b, ovl in [(128, 16), (64, 0), (96, 31)]:
            assert binding.ibmi_partition(p, b, ovl) == oracle.partition(p, b, ovl)


def test_partition_rejects_bad_arguments(binding):
    for args in [(0, 10, 0), (10, 0, 0), (10, 5, 5), (10, 5, -1)]:
        with pytest.raises(binding.IbmiError):
            binding.ibmi_partition(*args)


def test_workspace_bytes(binding):
    m = binding
    ok = m.make_options(4096, 576, 64)
    n = m.ibmi_workspace_bytes(ok)
    # at least W^T (sum b c) and the three b x b factor blocks, in FP64
    sets = oracle.partition(4096, 576, 64)
    floor = sum(8 * ((e - s) * (4096 - (e - s)) + 3 * (e - s) ** 2) for s, e in sets)
    assert n >= floor and n % 256 == 0
    assert m.ibmi_workspace_bytes(m.make_options(4096, 576, 64, tol=-1.0)) == 0
    assert m.ibmi_workspace_bytes(m.make_options(4096, 2048, 64)) == 0          # sets > 1024 rows
    assert m.ibmi_workspace_bytes(m.make_options(100, bounds=[(0, 50), (60, 100)])) == 0  # gap
    assert m.ibmi_workspace_bytes(m.make_options(100, bounds=[(50, 100), (0, 60)])) == 0  # unsorted
    assert m.ibmi_workspace_bytes(m.make_options(100, bounds=[(0, 60), (50, 100)],
                                                 init="blockdiag_inv")) == 0
    assert m.ibmi_workspace_bytes(m.make_options(100, bounds=[(0, 60), (50, 100)])) > 0


def test_status_strings(binding):
    assert binding.ibmi_status_str(0) == "IBMI_OK"
    assert binding.ibmi_status_str(2) == "IBMI_ERR_NOT_SPD"
    assert binding.ibmi_status_str(99) == "IBMI_UNKNOWN_STATUS"


def test_workspace_bytes_per_form_and_stop(binding):
    """The low-precision forms add their FP32 copies of A and D (p x ld32, ld32 = p rounded
    up to 4) and R (p x p FP64); the split forms also their K-chunk partials; the REL_HR stop
    adds R to the FP64 form; precisions and stop tests outside the enums are rejected."""
    m = binding
    p = 1001
    base = m.ibmi_workspace_bytes(m.make_options(p, 256, 32))
    ld32 = (p + 3) // 4 * 4
    for form in ("fp32", "bf16x3", "bf16x6"):
        n = m.ibmi_workspace_bytes(m.make_options(p, 256, 32, precision=form))
        assert n >= base + 2 * p * ld32 * 4 + p * p * 8, form
    assert m.ibmi_workspace_bytes(m.make_options(p, 256, 32, stop="rel_hr")) >= base + p * p * 8
    assert m.ibmi_workspace_bytes(m.make_options(p, 256, 32, stop="paper")) == base
    o = m.make_options(p, 256, 32)
    o.precision = 4
    assert m.ibmi_workspace_bytes(o) == 0
    o = m.make_options(p, 256, 32)
    o.stop = 4
    assert m.ibmi_workspace_bytes(o) == 0


def test_bench_refuses_several_gpus():
    """bench.py measures one GPU: asked for more it exits with status 2 and says why."""
    import subprocess
    import sys
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_covariance_row_chunks_same_bits():
    """The chunked covariance generator (used where the matrix is too large to build on the
    host at once) yields exactly the rows of the full matrix, nugget included."""
    import numpy as np
    import workloads
    pts = workloads.sorted_points(1500, 2, np.random.default_rng(2))
    full = workloads.covariance(pts, "matern32", 0.1, 1e-2)
    out = np.full_like(full, np.nan)
    for r0, r1, rows in workloads.covariance_row_chunks(pts, "matern32", 0.1, 1e-2,
                                                         row_chunk=333):
        out[r0:r1] = rows
    assert np.array_equal(out, full)


def test_oracle_only_where_allowed():
    """The product package never imports the oracle, and bench.py touches it only in its
    CPU-baseline leg (the GPU figures use the package's own flop counts)."""
    import ast
    import glob
    for path in glob.glob(os.path.join(ROOT, "paper_2502_06377_amd", "*.py")):
        tree = ast.parse(open(path).read())
        for node in ast.walk(tree):
            if isinstance(node, ast.Import):
                assert all(a.name.split(".")[0] != "oracle" for a in node.names), path
            if isinstance(node, ast.ImportFrom):
                assert (node.module or "").split(".")[0] != "oracle", path
    tree = ast.parse(open(os.path.join(ROOT, "bench.py")).read())
    allowed = set()
    for node in ast.walk(tree):
        if isinstance(node, ast.FunctionDef) and node.name == "cpu_baseline":
            allowed |= {id(n) for n in ast.walk(node)}
    for node in ast.walk(tree):
        uses = (isinstance(node, ast.Name) and node.id == "oracle") or (
            isinstance(node, ast.Import) and any(a.name == "oracle" for a in node.names))
        if uses:
            assert id(node) in allowed, f"bench.py line {node.lineno} uses the oracle"


def test_sweep_flops_of_the_benchmark_workload():
    """Per set 2bc^2 + 2b^2c plus 2p^3: 1.83e13 flops per sweep at p = 16384 (32 sets)."""
    from paper_2502_06377_amd.flops import plan_flops, sweep_flops
    ranges = oracle.partition(16384, 576, 64)
    f = sweep_flops(16384, ranges)
    assert abs(f / 1.83e13 - 1) < 0.005
    b, c = 576, 16384 - 576
    assert sweep_flops(16384, [(0, 576)], with_residual=False) == 2 * b * c * c + 2 * b * b * c
    assert plan_flops(16384, [(0, 576)]) == b ** 3 + 2 * b * b * c


def test_entry_points_reject_bad_arguments_before_device_work(binding):
    """Argument checks of the C ABI run on the host before any device call, so they are
    exercised here with stand-in addresses that are never dereferenced: null pointers, bad
    options, lda < p, a misaligned or too small workspace, A overlapping the workspace, and
    calls on a null plan."""
    m = binding
    lib = m._lib
    INV, OOM = m.IBMI_ERR_INVALID_ARG, m.IBMI_ERR_OUT_OF_MEMORY
    p = 1000
    o = m.make_options(p, 256, 32)
    need = m.ibmi_workspace_bytes(o)
    a_fake, w_fake = 1 << 40, 1 << 44  # far apart, 256-byte aligned, never touched
    h = ctypes.c_void_p()

    def plan(opts, a=a_fake, lda=p, w=w_fake, nbytes=need, out=True):
        return lib.ibmi_plan(ctypes.byref(h) if out else None, ctypes.byref(opts) if opts else None,
                             a, lda, w, nbytes, None)

    assert plan(o, out=False) == INV
    assert plan(None) == INV
    assert plan(o, a=None) == INV
    assert plan(o, w=None) == INV
    assert plan(o, lda=p - 1) == INV
    assert plan(o, w=w_fake + 8) == INV                     # workspace not 256-byte aligned
    assert plan(o, nbytes=need - 1) == OOM
    assert plan(o, w=a_fake + 8 * p) == INV                 # workspace inside A
    for field, bad in (("tol", 0.0), ("max_sweeps", 0), ("precision", 4), ("init", 3),
                       ("stop", 4), ("fixed_sweeps", -1)):
        ob = m.make_options(p, 256, 32)
        setattr(ob, field, bad)
        assert plan(ob) == INV, field
    ob = m.make_options(p, 256, 32, stop="rel_bound", lambda_min=0.0)
    assert plan(ob) == INV
    for pp, b, ov in ((0, 256, 32), (-5, 256, 32), (p, 0, 0), (p, 64, 64)):
        assert plan(m.make_options(pp, b, ov), lda=max(pp, 1)) == INV, (pp, b, ov)
    ob = m.make_options(p, bounds=[(0, 600), (700, 1000)])   # sets leave a gap
    assert plan(ob) == INV
    info = m.IbmiInfo()
    r = ctypes.c_double()
    assert lib.ibmi_solve(None, a_fake, p, ctypes.byref(info), None) == INV
    assert lib.ibmi_sweep(None, a_fake, p, 0, ctypes.byref(r)) == INV
    assert lib.ibmi_block_step(None, a_fake, p, 0) == INV
    assert lib.ibmi_init_h(None, a_fake, p) == INV
    assert lib.ibmi_residual(None, a_fake, p, ctypes.byref(r)) == INV
    assert lib.ibmi_plan_destroy(None) == INV
    bo = m.make_options(300, 128, 16)
    ps = (ctypes.c_int64 * 1)(300)
    ptrs = (ctypes.c_void_p * 1)(a_fake)
    lds = (ctypes.c_int64 * 1)(300)
    bh = ctypes.c_void_p()
    assert lib.ibmi_batch_plan(ctypes.byref(bh), 0, ps, ptrs, lds, ctypes.byref(bo), w_fake,
                               1 << 30, None) == INV
    bo.precision = 1
    assert lib.ibmi_batch_plan(ctypes.byref(bh), 1, ps, ptrs, lds, ctypes.byref(bo), w_fake,
                               1 << 30, None) == INV


def test_serving_footprint_and_summary(binding):
    """Admission footprint = A + H (rows padded to 8 elements) + the plan's workspace; it grows
    with p and the low-precision forms need more than FP64.  The summary's percentiles are
    those of the recorded latencies."""
    from paper_2502_06377_amd import serve
    m = binding
    for p in (512, 1000, 8192):
        ld = (p + 7) // 8 * 8
        ws = m.ibmi_workspace_bytes(m.make_options(p, 576, 64, tol=1e-10))
        assert serve.footprint_bytes(p, "fp64", 576, 64, 1e-10) == 2 * p * ld * 8 + ws
        assert serve.footprint_bytes(p, serve.LOW_FORM, 576, 64, 1e-6) > ws + 2 * p * ld * 8
    sizes = [serve.footprint_bytes(p, "fp64", 576, 64, 1e-10) for p in (512, 1024, 4096, 8192)]
    assert sizes == sorted(sizes)
    st = serve.ServeStats(wall=2.0)
    for i in range(100):
        st.results.append(serve.Result(rid=i, p=512, tol=1e-10, form="fp64", arrival=0.0,
                                       start=0.0, end=0.01 * (i + 1), sweeps=3, converged=True,
                                       residual=0.0, footprint=0))
    s = st.summary(120, 1 << 30)
    assert s["requests_done"] == 100 and s["solves_per_s"] == 50.0
    assert abs(s["latency_p50_s"] - 0.505) < 1e-9 and abs(s["latency_p99_s"] - 0.9901) < 1e-9
    assert s["converged"] == 100 and s["capped_or_failed"] == 0


def test_autotune_cache_round_trip(binding, monkeypatch):
    """The batched form's tile cache: a miss runs the autotuner once and stores its choice; the
    next lookup of the same key applies the stored choice without tuning."""
    from paper_2502_06377_amd import tuning

    class FakeBatch:
        def __init__(self):
            self.applied, self.tunes = None, 0

        def autotune(self, reps):
            self.tunes += 1
            return (4, 1, 2), 12.5

        def set_tuning(self, *cfg):
            self.applied = cfg

    monkeypatch.setattr(tuning, "batch_key", lambda b: "gfx950/batch/test")
    os.makedirs(os.path.join(ROOT, "_build"), exist_ok=True)
    path = os.path.join(ROOT, "_build", "test_tune_cache.json")
    if os.path.exists(path):
        os.remove(path)
    b1 = FakeBatch()
    r1 = tuning.tuned(b1, path=path)
    assert not r1["cached"] and b1.tunes == 1 and r1["cfg"] == (4, 1, 2)
    b2 = FakeBatch()
    r2 = tuning.tuned(b2, path=path)
    assert r2["cached"] and b2.tunes == 0 and b2.applied == (4, 1, 2)
    assert r2["ms_per_sweep"] == 12.5


def test_bench_traffic_only_for_the_profiled_kernel():
    """The bench's roofline `traffic` comes from the committed PMC summary and only while that
    summary names the panel kernel instantiation the bench runs; any other name gives None."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    t = bench.measured_traffic(bench.PANEL_KERNEL)
    assert t is not None and 1e9 < t < 1e11
    assert bench.measured_traffic(bench.PANEL_KERNEL.replace("96, 64", "64, 64")) is None
    profile = open(os.path.join(ROOT, "profiles", "ibmi_sweep_p16384_kernel_stats.md")).read()
    assert bench.PANEL_KERNEL in profile
