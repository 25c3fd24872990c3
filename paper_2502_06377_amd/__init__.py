"""Python binding of libibmi (MI355X / gfx950 IBMI), argument marshalling only.

Every function named ``ibmi_*`` here calls the C entry point of the same name in
``libibmi.so`` (declared in ``include/ibmi.h``); all arithmetic runs in the library's HIP
kernels.  PyTorch provides device memory and streams.  There is no CPU fallback: importing
this package without the built library raises ``ImportError``.

``Plan`` and ``solve`` are thin conveniences that allocate A's workspace and H as torch
tensors on the current device and stream.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch  # loads the HIP runtime that libibmi then shares (same SONAME)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libibmi.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2502_06377_amd/build.py`")
_lib = ctypes.CDLL(LIB_PATH)

# ------------------------------------------------------------------ constants (ibmi.h)
IBMI_OK, IBMI_ERR_INVALID_ARG, IBMI_ERR_NOT_SPD, IBMI_ERR_OUT_OF_MEMORY, IBMI_ERR_HIP, \
    IBMI_ERR_NONFINITE = range(6)
IBMI_PREC_FP64, IBMI_PREC_FP32_UPDATE, IBMI_PREC_BF16X3_UPDATE, IBMI_PREC_BF16X6_UPDATE = 0, 1, 2, 3
IBMI_INIT_IDENTITY, IBMI_INIT_BLOCKDIAG_INV, IBMI_INIT_GIVEN = 0, 1, 2
IBMI_STOP_FRO, IBMI_STOP_REL_BOUND, IBMI_STOP_REL_HR, IBMI_STOP_PAPER = 0, 1, 2, 3

_INIT = {"identity": IBMI_INIT_IDENTITY, "blockdiag_inv": IBMI_INIT_BLOCKDIAG_INV,
         "given": IBMI_INIT_GIVEN}
_STOP = {"fro": IBMI_STOP_FRO, "rel_bound": IBMI_STOP_REL_BOUND, "rel_hr": IBMI_STOP_REL_HR,
         "paper": IBMI_STOP_PAPER}
_PREC = {"fp64": IBMI_PREC_FP64, "fp32": IBMI_PREC_FP32_UPDATE, "bf16x3": IBMI_PREC_BF16X3_UPDATE,
         "bf16x6": IBMI_PREC_BF16X6_UPDATE}


class IbmiOptions(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int64), ("block_rows", ctypes.c_int32), ("overlap", ctypes.c_int32),
                ("bounds", ctypes.POINTER(ctypes.c_int64)), ("n_blocks", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("init", ctypes.c_int32), ("stop", ctypes.c_int32),
                ("tol", ctypes.c_double), ("lambda_min", ctypes.c_double),
                ("max_sweeps", ctypes.c_int32), ("stagnation_guard", ctypes.c_int32),
                ("fixed_sweeps", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class IbmiInfo(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("failed_block", ctypes.c_int32), ("floor_limited", ctypes.c_int32),
                ("residual", ctypes.c_double), ("stop_value", ctypes.c_double),
                ("cancelled", ctypes.c_int32), ("evaluations", ctypes.c_int32)]


PROGRESS_FN = ctypes.CFUNCTYPE(ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                               ctypes.c_void_p)


_vp, _i64, _i32, _dp = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
_SIGS = {
    "ibmi_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "ibmi_partition": (ctypes.c_int, [_i64, _i32, _i32, ctypes.POINTER(ctypes.c_int64), _i32,
                                      ctypes.POINTER(ctypes.c_int32)]),
    "ibmi_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(IbmiOptions)]),
    "ibmi_plan": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.POINTER(IbmiOptions), _dp, _i64, _vp,
                                 ctypes.c_size_t, _vp]),
    "ibmi_plan_failed_block": (ctypes.c_int32, []),
    "ibmi_plan_blocks": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_int64)]),
    "ibmi_solve": (ctypes.c_int, [_vp, _dp, _i64, ctypes.POINTER(IbmiInfo),
                                  ctypes.POINTER(ctypes.c_double)]),
    "ibmi_sweep": (ctypes.c_int, [_vp, _dp, _i64, _i32, ctypes.POINTER(ctypes.c_double)]),
    "ibmi_block_step": (ctypes.c_int, [_vp, _dp, _i64, _i32]),
    "ibmi_init_h": (ctypes.c_int, [_vp, _dp, _i64]),
    "ibmi_residual": (ctypes.c_int, [_vp, _dp, _i64, ctypes.POINTER(ctypes.c_double)]),
    "ibmi_set_profiling": (ctypes.c_int, [_vp, _i32]),
    "ibmi_set_progress": (ctypes.c_int, [_vp, PROGRESS_FN, _vp]),
    "ibmi_kernel_times": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(ctypes.c_double)]),
    "ibmi_plan_destroy": (ctypes.c_int, [_vp]),
    "ibmi_batch_workspace_bytes": (ctypes.c_size_t, [_i32, ctypes.POINTER(ctypes.c_int64),
                                                     ctypes.POINTER(IbmiOptions)]),
    "ibmi_batch_plan": (ctypes.c_int, [ctypes.POINTER(_vp), _i32, ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(ctypes.c_void_p),
                                       ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(IbmiOptions), _vp, ctypes.c_size_t, _vp]),
    "ibmi_batch_solve": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_void_p),
                                        ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(IbmiInfo)]),
    "ibmi_batch_set_tuning": (ctypes.c_int, [_vp, _i32, _i32, _i32]),
    "ibmi_batch_get_tuning": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int32)]),
    "ibmi_batch_autotune": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_void_p),
                                           ctypes.POINTER(ctypes.c_int64), _i32,
                                           ctypes.POINTER(ctypes.c_int32),
                                           ctypes.POINTER(ctypes.c_double)]),
    "ibmi_batch_destroy": (ctypes.c_int, [_vp]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype, _f.argtypes = _res, _args

EXPORTED = tuple(_SIGS)


class IbmiError(RuntimeError):
    def __init__(self, status: int, where: str, block: int = -1):
        self.status = status
        self.block = block
        name = _lib.ibmi_status_str(status).decode()
        super().__init__(f"{where}: {name}" + (f" (block {block})" if block >= 0 else ""))


def _check(status: int, where: str, block: int = -1):
    if status != IBMI_OK:
        raise IbmiError(status, where, block)


# ------------------------------------------------------------------ same-name wrappers

def ibmi_status_str(status: int) -> str:
    return _lib.ibmi_status_str(status).decode()


def ibmi_partition(p: int, block_rows: int, overlap: int) -> list:
    n = ctypes.c_int32(0)
    _check(_lib.ibmi_partition(p, block_rows, overlap, None, 0, ctypes.byref(n)), "ibmi_partition")
    buf = (ctypes.c_int64 * (2 * n.value))()
    _check(_lib.ibmi_partition(p, block_rows, overlap, buf, n.value, ctypes.byref(n)),
           "ibmi_partition")
    return [(buf[2 * k], buf[2 * k + 1]) for k in range(n.value)]


def make_options(p: int, block_rows: int = 576, overlap: int = 64, bounds=None,
                 precision: str = "fp64", init: str = "identity", stop: str = "fro",
                 tol: float = 1e-10, lambda_min: float = 0.0, max_sweeps: int = 500,
                 stagnation_guard: bool = True, fixed_sweeps: int = 0) -> IbmiOptions:
    o = IbmiOptions()
    o.p, o.block_rows, o.overlap = p, block_rows, overlap
    if bounds is not None:
        flat = (ctypes.c_int64 * (2 * len(bounds)))(*[int(v) for se in bounds for v in se])
        o._bounds_keepalive = flat
        o.bounds = ctypes.cast(flat, ctypes.POINTER(ctypes.c_int64))
        o.n_blocks = len(bounds)
    o.precision, o.init, o.stop = _PREC[precision], _INIT[init], _STOP[stop]
    o.tol, o.lambda_min = tol, lambda_min
    o.max_sweeps, o.stagnation_guard, o.fixed_sweeps = max_sweeps, int(stagnation_guard), fixed_sweeps
    return o


def ibmi_workspace_bytes(opts: IbmiOptions) -> int:
    return int(_lib.ibmi_workspace_bytes(ctypes.byref(opts)))


def _dptr(t: torch.Tensor) -> int:
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    return t.data_ptr()


def _stream_handle(stream) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def ibmi_plan(opts: IbmiOptions, A: torch.Tensor, work: torch.Tensor, stream=None) -> int:
    """Returns the opaque plan handle (int).  A: p x p float64 device tensor (row stride = lda)."""
    if A.dtype != torch.float64 or A.dim() != 2 or A.stride(1) != 1:
        raise ValueError("A must be a 2-D float64 tensor with unit column stride")
    h = _vp()
    st = _lib.ibmi_plan(ctypes.byref(h), ctypes.byref(opts), _dptr(A), A.stride(0), _dptr(work),
                        work.numel() * work.element_size(), _stream_handle(stream))
    _check(st, "ibmi_plan", _lib.ibmi_plan_failed_block() if st == IBMI_ERR_NOT_SPD else -1)
    return h.value


def ibmi_plan_blocks(plan: int) -> list:
    n = ctypes.c_int32(0)
    _check(_lib.ibmi_plan_blocks(plan, ctypes.byref(n), None), "ibmi_plan_blocks")
    buf = (ctypes.c_int64 * (2 * n.value))()
    _check(_lib.ibmi_plan_blocks(plan, ctypes.byref(n), buf), "ibmi_plan_blocks")
    return [(buf[2 * k], buf[2 * k + 1]) for k in range(n.value)]


def ibmi_solve(plan: int, H: torch.Tensor, history_len: int = 0):
    info = IbmiInfo()
    hist = (ctypes.c_double * history_len)() if history_len > 0 else None
    _check(_lib.ibmi_solve(plan, _dptr(H), H.stride(0), ctypes.byref(info), hist), "ibmi_solve")
    return info, ([hist[i] for i in range(info.sweeps)] if hist is not None else [])


def ibmi_sweep(plan: int, H: torch.Tensor, restart: bool) -> float:
    out = ctypes.c_double(0.0)
    _check(_lib.ibmi_sweep(plan, _dptr(H), H.stride(0), int(restart), ctypes.byref(out)),
           "ibmi_sweep")
    return out.value


def ibmi_block_step(plan: int, H: torch.Tensor, k: int) -> None:
    _check(_lib.ibmi_block_step(plan, _dptr(H), H.stride(0), k), "ibmi_block_step")


def ibmi_init_h(plan: int, H: torch.Tensor) -> None:
    _check(_lib.ibmi_init_h(plan, _dptr(H), H.stride(0)), "ibmi_init_h")


def ibmi_residual(plan: int, H: torch.Tensor) -> float:
    out = ctypes.c_double(0.0)
    _check(_lib.ibmi_residual(plan, _dptr(H), H.stride(0), ctypes.byref(out)), "ibmi_residual")
    return out.value


def ibmi_set_profiling(plan: int, on: bool) -> None:
    _check(_lib.ibmi_set_profiling(plan, int(on)), "ibmi_set_profiling")


KERNEL_CATEGORIES = ("panel", "diag", "resid")


def ibmi_kernel_times(plan: int) -> dict:
    """{category: (milliseconds, launches, algorithmic flops)} since the last call."""
    ms = (ctypes.c_double * 3)()
    n = (ctypes.c_int64 * 3)()
    fl = (ctypes.c_double * 3)()
    _check(_lib.ibmi_kernel_times(plan, ms, n, fl), "ibmi_kernel_times")
    return {c: (ms[i], n[i], fl[i]) for i, c in enumerate(KERNEL_CATEGORIES)}


def ibmi_plan_destroy(plan: int) -> None:
    _check(_lib.ibmi_plan_destroy(plan), "ibmi_plan_destroy")


# ------------------------------------------------------------------ conveniences

@dataclass
class SolveOutput:
    H: torch.Tensor
    sweeps: int
    converged: bool
    floor_limited: bool
    residual: float
    stop_value: float
    history: list
    cancelled: bool = False
    evaluations: int = 0  # sweeps at which the rel_hr bound was evaluated


class Plan:
    """Owns the workspace tensor and the plan handle; A is borrowed (kept referenced)."""

    def __init__(self, A: torch.Tensor, stream=None, **opt_kwargs):
        self.A = A
        self.p = A.shape[0]
        self.opts = make_options(self.p, **opt_kwargs)
        nbytes = ibmi_workspace_bytes(self.opts)
        if nbytes == 0:
            raise IbmiError(IBMI_ERR_INVALID_ARG, "ibmi_workspace_bytes")
        self.work = torch.empty(nbytes, dtype=torch.uint8, device=A.device)
        self.stream = stream
        self.handle = ibmi_plan(self.opts, A, self.work, stream)
        self.blocks = ibmi_plan_blocks(self.handle)

    def solve(self, H: torch.Tensor | None = None, progress=None) -> SolveOutput:
        """progress(sweep, residual, stop_value) -> truthy to stop early (optional)."""
        if H is None:
            H = torch.empty((self.p, self.p), dtype=torch.float64, device=self.A.device)
        n = self.opts.fixed_sweeps if self.opts.fixed_sweeps > 0 else self.opts.max_sweeps
        cb = None
        if progress is not None:
            cb = PROGRESS_FN(lambda r, res, sv, _u: 1 if progress(r, res, sv) else 0)
            _check(_lib.ibmi_set_progress(self.handle, cb, None), "ibmi_set_progress")
        try:
            info, hist = ibmi_solve(self.handle, H, n)
        finally:
            if cb is not None:
                _lib.ibmi_set_progress(self.handle, PROGRESS_FN(), None)
        return SolveOutput(H, info.sweeps, bool(info.converged), bool(info.floor_limited),
                           info.residual, info.stop_value, hist, bool(info.cancelled),
                           info.evaluations)

    def residual(self, H: torch.Tensor) -> float:
        return ibmi_residual(self.handle, H)

    def close(self):
        if self.handle:
            ibmi_plan_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve(A: torch.Tensor, **kwargs) -> SolveOutput:
    """Plan + solve in one call on the current stream."""
    plan = Plan(A, **kwargs)
    try:
        return plan.solve()
    finally:
        plan.close()


# ------------------------------------------------------------------ batched form

class BatchPlan:
    """n independent SPD matrices solved together (grouped launches in one captured graph).

    ``As`` is a list of square float64 device tensors with unit column stride; they are
    borrowed (kept referenced).  H buffers are allocated with a leading dimension rounded up
    to a multiple of 8 elements so that the 16-byte load path applies."""

    def __init__(self, As, stream=None, **opt_kwargs):
        self.As = list(As)
        self.n = len(self.As)
        self.p = [int(a.shape[0]) for a in self.As]
        for a in self.As:
            if a.dtype != torch.float64 or a.dim() != 2 or a.stride(1) != 1:
                raise ValueError("each A must be a 2-D float64 tensor with unit column stride")
        self.opts = make_options(max(self.p), **opt_kwargs)
        self._p = (ctypes.c_int64 * self.n)(*self.p)
        nbytes = _lib.ibmi_batch_workspace_bytes(self.n, self._p, ctypes.byref(self.opts))
        if nbytes == 0:
            raise IbmiError(IBMI_ERR_INVALID_ARG, "ibmi_batch_workspace_bytes")
        dev = self.As[0].device
        self.work = torch.empty(int(nbytes), dtype=torch.uint8, device=dev)
        ptrs = (ctypes.c_void_p * self.n)(*[_dptr(a) for a in self.As])
        ldas = (ctypes.c_int64 * self.n)(*[a.stride(0) for a in self.As])
        # graph capture needs a stream of its own (not the legacy default stream)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=dev)
        self.stream.wait_stream(torch.cuda.current_stream(dev))
        h = _vp()
        _check(_lib.ibmi_batch_plan(ctypes.byref(h), self.n, self._p, ptrs, ldas,
                                    ctypes.byref(self.opts), _dptr(self.work), int(nbytes),
                                    self.stream.cuda_stream), "ibmi_batch_plan")
        self.handle = h.value
        self.H = []
        for p in self.p:
            ld = (p + 7) // 8 * 8
            self.H.append(torch.empty((p, ld), dtype=torch.float64, device=dev)[:, :p])
        self._hp = (ctypes.c_void_p * self.n)(*[h.data_ptr() for h in self.H])
        self._hld = (ctypes.c_int64 * self.n)(*[h.stride(0) for h in self.H])

    def solve(self):
        infos = (IbmiInfo * self.n)()
        self.stream.wait_stream(torch.cuda.current_stream(self.As[0].device))
        st = _lib.ibmi_batch_solve(self.handle, self._hp, self._hld, infos)
        out = [SolveOutput(self.H[i], infos[i].sweeps, bool(infos[i].converged),
                           bool(infos[i].floor_limited), infos[i].residual, infos[i].stop_value, [])
               for i in range(self.n)]
        _check(st, "ibmi_batch_solve")
        return out

    def set_tuning(self, panel: int, diag: int, resid: int) -> None:
        _check(_lib.ibmi_batch_set_tuning(self.handle, panel, diag, resid), "ibmi_batch_set_tuning")

    def get_tuning(self) -> tuple:
        c = (ctypes.c_int32 * 3)()
        _check(_lib.ibmi_batch_get_tuning(self.handle, c), "ibmi_batch_get_tuning")
        return tuple(c)

    def autotune(self, reps: int = 2):
        self.stream.wait_stream(torch.cuda.current_stream(self.As[0].device))
        c = (ctypes.c_int32 * 3)()
        ms = ctypes.c_double(0.0)
        _check(_lib.ibmi_batch_autotune(self.handle, self._hp, self._hld, reps, c,
                                        ctypes.byref(ms)), "ibmi_batch_autotune")
        return tuple(c), ms.value

    def close(self):
        if getattr(self, "handle", 0):
            _check(_lib.ibmi_batch_destroy(self.handle), "ibmi_batch_destroy")
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
