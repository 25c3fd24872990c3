"""Serving form: requests solved concurrently on several streams under an HBM budget give the
same result as the same request solved alone (bitwise: the kernels and tile choices are the
same, only the interleaving on the device differs), and admission never exceeds the budget."""
import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def srv():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2502_06377_amd as ib
    from paper_2502_06377_amd import serve
    return ib, serve


def test_serve_mix_equals_alone(srv):
    ib, serve = srv
    _say("serving: 14 requests, 3 slots, budget-limited admission")
    rng = np.random.default_rng(51)
    reqs = []
    for rid in range(14):
        p = int(rng.integers(200, 1400))
        tol = 1e-6 if rid % 2 else 1e-10
        reqs.append(workloads.Request(rid, 0.0005 * rid, p, tol, int(rng.integers(0, 2**31 - 1))))
    budgets = [serve.footprint_bytes(r.p, "fp64" if r.tol < 1e-6 else serve.LOW_FORM, 256, 32,
                                     r.tol)
               for r in reqs]
    budget = int(2.2 * max(budgets))
    loop = serve.ServeLoop(slots=3, hbm_budget=budget, block_rows=256, overlap=32, keep_h=True)
    stats = loop.run(reqs)
    assert len(stats.results) == len(reqs)
    assert stats.max_in_use <= budget
    # a request either meets its tolerance or stops at its FP64 floor (stagnation guard)
    bad = [(r.rid, r.p, r.form, r.sweeps, r.residual, r.error)
           for r in stats.results if not (r.converged or r.floor_limited)]
    assert not bad, bad
    by_id = {r.rid: r for r in stats.results}
    for rid in (0, 3, 8, 13):
        req, res = reqs[rid], by_id[rid]
        A = serve.matern32_on_device(serve.request_points(req), 0.1, 1e-2, torch.device("cuda:0"))
        ld = (req.p + 7) // 8 * 8
        H = torch.empty((req.p, ld), dtype=torch.float64, device="cuda:0")[:, :req.p]
        plan = ib.Plan(A, block_rows=256, overlap=32, precision=res.form, tol=req.tol,
                       max_sweeps=500)
        out = plan.solve(H)
        plan.close()
        torch.cuda.synchronize()
        assert out.sweeps == res.sweeps
        diff = float(torch.linalg.norm(out.H - res.H) / torch.linalg.norm(out.H))
        assert diff <= 1e-12, (rid, diff)
        inv = torch.linalg.inv(A.cpu()).numpy()
        rel = np.linalg.norm(res.H.cpu().numpy() - inv) / np.linalg.norm(inv)
        assert rel < (1e-8 if req.tol < 1e-6 else 1e-4), (rid, rel)
    s = stats.summary(len(reqs), budget)
    assert s["latency_p99_s"] >= s["latency_p50_s"] > 0
