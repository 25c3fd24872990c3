"""Serving form: a continuous-batching request loop over the IBMI library on one GPU.

Requests (a covariance matrix to invert, with a tolerance) arrive on a seeded Poisson
schedule.  A fixed number of worker slots, each with its own HIP stream, run requests
concurrently; a request is admitted when a slot is free and its device footprint (A + H +
the plan's workspace, from ``ibmi_workspace_bytes``) fits the free part of an HBM budget, so
work from several requests overlaps on the device while later arrivals wait in the queue.
A request asking for 1e-6 runs the split-bfloat16 (bf16x3) update form, the fastest
correction form per sweep, one asking for 1e-10 the FP64 form.
Latency is measured from arrival to completion.

The matrix of a request is built on the device from its seeded points (input generation,
not part of the IBMI path); every IBMI step runs in the library's kernels.
"""
from __future__ import annotations

import argparse
import json
import math
import queue
import sys
import threading
import time
from dataclasses import dataclass, field

import numpy as np
import torch

import paper_2502_06377_amd as ib


LOW_FORM = "bf16x3"  # update form of the requests that ask for 1e-6


@dataclass
class Result:
    rid: int
    p: int
    tol: float
    form: str
    arrival: float
    start: float
    end: float
    sweeps: int
    converged: bool
    residual: float
    footprint: int
    H: torch.Tensor | None = None
    error: str | None = None
    floor_limited: bool = False

    @property
    def latency(self) -> float:
        return self.end - self.arrival


def matern32_on_device(pts: np.ndarray, ell: float, nugget: float, device) -> torch.Tensor:
    """Matern-3/2 covariance (variance 1) of the points plus ``nugget * I``, built on the GPU.
    Row stride rounded up to 8 elements (16-byte aligned rows)."""
    p = pts.shape[0]
    x = torch.from_numpy(pts).to(device)
    d2 = torch.zeros((p, p), dtype=torch.float64, device=device)
    for c in range(x.shape[1]):
        diff = x[:, c][:, None] - x[:, c][None, :]
        d2 += diff * diff
    z = math.sqrt(3.0) / ell * torch.sqrt(d2)
    a = (1.0 + z) * torch.exp(-z)
    a.diagonal().add_(nugget)
    ld = (p + 7) // 8 * 8
    out = torch.empty((p, ld), dtype=torch.float64, device=device)[:, :p]
    out.copy_(a)
    return out


def request_points(req) -> np.ndarray:
    """The seeded, x-sorted points of a request (same recipe as workloads.request_matrix)."""
    import workloads
    rng = np.random.default_rng(req.seed)
    return workloads.sorted_points(req.p, 2, rng)


def footprint_bytes(p: int, form: str, block_rows: int, overlap: int, tol: float) -> int:
    ld = (p + 7) // 8 * 8
    opts = ib.make_options(p, block_rows=block_rows, overlap=overlap, precision=form, tol=tol)
    return 2 * p * ld * 8 + ib.ibmi_workspace_bytes(opts)


@dataclass
class ServeStats:
    results: list = field(default_factory=list)
    max_in_use: int = 0
    max_queue: int = 0
    wall: float = 0.0

    def summary(self, offered: int, budget: int) -> dict:
        lat = np.array([r.latency for r in self.results]) if self.results else np.array([0.0])
        done = len(self.results)
        return {"requests_offered": offered, "requests_done": done,
                "wall_s": round(self.wall, 3), "solves_per_s": round(done / self.wall, 3),
                "latency_p50_s": round(float(np.percentile(lat, 50)), 4),
                "latency_p99_s": round(float(np.percentile(lat, 99)), 4),
                "latency_max_s": round(float(lat.max()), 4),
                "converged": sum(r.converged for r in self.results),
                "floor_limited": sum(r.floor_limited for r in self.results),
                "capped_or_failed": sum(not (r.converged or r.floor_limited)
                                        for r in self.results),
                "errors": [r.error for r in self.results if r.error][:5],
                "max_hbm_in_use_bytes": self.max_in_use, "hbm_budget_bytes": budget,
                "max_queue_depth": self.max_queue}


class ServeLoop:
    """Continuous-batching server over `slots` concurrent streams within `hbm_budget` bytes."""

    def __init__(self, slots: int = 4, hbm_budget: int = 64 << 30, block_rows: int = 576,
                 overlap: int = 64, max_sweeps: int = 500, keep_h: bool = False,
                 device="cuda:0", progress: bool = False):
        self.progress = progress
        self.slots = slots
        self.budget = hbm_budget
        self.block_rows = block_rows
        self.overlap = overlap
        self.max_sweeps = max_sweeps
        self.keep_h = keep_h
        self.device = torch.device(device)
        self.lock = threading.Condition()
        self.in_use = 0
        self.free_slots = slots
        self.stats = ServeStats()

    def _form(self, tol: float) -> str:
        return LOW_FORM if tol >= 1e-6 else "fp64"

    def _run(self, req, arrival_abs: float, fp: int, stream: torch.cuda.Stream) -> Result:
        form = self._form(req.tol)
        start = time.perf_counter()
        with torch.cuda.stream(stream):
            A = matern32_on_device(request_points(req), 0.1, 1e-2, self.device)
            ld = (req.p + 7) // 8 * 8
            H = torch.empty((req.p, ld), dtype=torch.float64, device=self.device)[:, :req.p]
            plan = ib.Plan(A, stream=stream, block_rows=self.block_rows, overlap=self.overlap,
                           precision=form, tol=req.tol, max_sweeps=self.max_sweeps)
            out = plan.solve(H)
            plan.close()
            stream.synchronize()
        end = time.perf_counter()
        return Result(req.rid, req.p, req.tol, form, arrival_abs, start, end, out.sweeps,
                      out.converged, out.residual, fp, H if self.keep_h else None,
                      floor_limited=out.floor_limited)

    def run(self, requests, time_scale: float = 1.0, max_wall: float | None = None) -> ServeStats:
        """Replay ``requests`` (with arrival_s fields) in real time scaled by ``time_scale``."""
        pending: queue.Queue = queue.Queue()
        t0 = time.perf_counter()
        streams = [torch.cuda.Stream(device=self.device) for _ in range(self.slots)]
        free_streams = list(range(self.slots))
        stop = threading.Event()

        def arrivals():
            for r in requests:
                due = t0 + r.arrival_s * time_scale
                while not stop.is_set():
                    now = time.perf_counter()
                    if now >= due:
                        break
                    time.sleep(min(0.005, due - now))
                if stop.is_set():
                    return
                pending.put((r, time.perf_counter()))
            pending.put(None)

        workers = []

        def worker(req, arrival_abs, fp, sidx):
            try:
                res = self._run(req, arrival_abs, fp, streams[sidx])
            except Exception as exc:  # a failed request must not disturb the others
                res = Result(req.rid, req.p, req.tol, self._form(req.tol), arrival_abs,
                             arrival_abs, time.perf_counter(), 0, False, float("nan"), fp)
                res.error = repr(exc)
            with self.lock:
                self.in_use -= fp
                free_streams.append(sidx)
                self.stats.results.append(res)
                self.lock.notify_all()

        feeder = threading.Thread(target=arrivals, daemon=True)
        feeder.start()
        waiting = []
        done_feeding = False
        next_report = t0 + 10.0
        while True:
            if self.progress and time.perf_counter() >= next_report:
                next_report += 10.0
                print(f"[serve] t={time.perf_counter() - t0:.0f}s done={len(self.stats.results)} "
                      f"queued={len(waiting)} running={self.slots - len(free_streams)}",
                      file=sys.stderr, flush=True)
            # drain arrivals into the waiting list
            try:
                while True:
                    item = pending.get(timeout=0.002)
                    if item is None:
                        done_feeding = True
                        break
                    waiting.append(item)
            except queue.Empty:
                pass
            self.stats.max_queue = max(self.stats.max_queue, len(waiting))
            if max_wall is not None and time.perf_counter() - t0 > max_wall:
                stop.set()
                waiting.clear()
                done_feeding = True
            # admit in arrival order while a slot and memory are free
            with self.lock:
                while waiting and free_streams:
                    req, arr = waiting[0]
                    fp = footprint_bytes(req.p, self._form(req.tol), self.block_rows,
                                         self.overlap, req.tol)
                    if fp > self.budget:
                        waiting.pop(0)  # can never fit: reject
                        continue
                    if self.in_use + fp > self.budget:
                        break
                    waiting.pop(0)
                    self.in_use += fp
                    self.stats.max_in_use = max(self.stats.max_in_use, self.in_use)
                    sidx = free_streams.pop()
                    th = threading.Thread(target=worker, args=(req, arr, fp, sidx), daemon=True)
                    workers.append(th)
                    th.start()
                busy = len(free_streams) < self.slots
                if done_feeding and not waiting and not busy:
                    break
                if not waiting and not done_feeding:
                    pass
                else:
                    self.lock.wait(timeout=0.005)
        for th in workers:
            th.join()
        self.stats.wall = time.perf_counter() - t0
        return self.stats


def main():
    import workloads
    ap = argparse.ArgumentParser(description="IBMI serving loop on one GPU")
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--duration", type=float, default=60.0)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--budget-gib", type=float, default=64.0)
    ap.add_argument("--max-wall", type=float, default=None)
    ap.add_argument("--p-lo", type=int, default=512)
    ap.add_argument("--p-hi", type=int, default=8192)
    args = ap.parse_args()
    reqs = workloads.config5_arrivals(rate_hz=args.rate, duration_s=args.duration, lo=args.p_lo,
                                      hi=args.p_hi)
    loop = ServeLoop(slots=args.slots, hbm_budget=int(args.budget_gib * (1 << 30)), progress=True)
    stats = loop.run(reqs, max_wall=args.max_wall)
    out = stats.summary(len(reqs), loop.budget)
    out.update({"rate_hz": args.rate, "duration_s": args.duration, "slots": args.slots})
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
