"""The serving loop on the GPU: every request's result in the mix equals, bit for bit,
the same product run alone (same plan, operands, seed), in every execution mode; results
are within the fp8 leaves' error of the float64 product."""

import sys

import numpy as np
import pytest
import torch

from paper_1905_07439_amd import serve

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("mode,engine", [("batch", "persistent"), ("batch", "levels"), ("direct", "levels")])
def test_served_results_equal_alone(mode, engine):
    reqs = serve.make_requests(4000, 0.03, 11, lo=128, hi=640)
    keep = {r.rid: None for r in reqs}
    ex = serve.GpuExecutor(prec="fp8c", mode=mode, keep=keep, engine=engine)
    sch = serve.Scheduler(200e9, max_batch=32)
    stats = serve.serve(reqs, ex, sch, slots=4)
    _say(mode, engine, {k: stats[k] for k in ("requests", "batches", "mean_batch", "latency_ms")})
    assert stats["requests"] == len(reqs) and sch.in_use == 0
    assert all(np.isfinite(r.done) and r.done >= r.arrival for r in reqs)
    if mode == "batch":
        assert stats["mean_batch"] > 1.0  # arrivals overlapped and were batched
    for r in reqs:
        A, B, C = keep[r.rid]
        alone = ex.plan(r).matmul(A, B, seed=r.seed, mode="full")
        assert torch.equal(C, alone), (r.rid, r.n, r.scheme)
    for r in reqs[::9]:
        A, B, C = keep[r.rid]
        ref = A.double() @ B.double()
        err = float(torch.linalg.norm(C.double() - ref) / torch.linalg.norm(ref))
        assert err < 3e-2, (r.rid, r.n, r.scheme, err)
