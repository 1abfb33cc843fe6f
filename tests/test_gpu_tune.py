"""The autotuner on the GPU: it times every candidate, keeps the fastest, and the plan it
returns computes exactly what the same plan built by hand computes."""

import pytest
import torch

import paper_1905_07439_amd as rbc
from paper_1905_07439_amd.tune import Tuner

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.mark.parametrize("prec,name,n", [("f16s", "strassen", 384), ("fp8c", "laderman", 288), ("f32", "strassen", 512)])
def test_tuned_plan_is_the_hand_built_plan(prec, name, n):
    t = Tuner(reps=2, min_leaf=32)
    sch = rbc.Scheme.builtin(name)
    c = t.choose(n, n, n, sch, prec, name)
    tried = t.trials[t.key(n, n, n, name, prec)]
    print(prec, name, n, c, tried, flush=True)
    assert len(tried) >= 2 and all(x["ms"] > 0 for x in tried)
    assert c["ms"] == min(x["ms"] for x in tried)
    g = torch.Generator(device=DEV)
    g.manual_seed(5)
    A = torch.randn(n, n, device=DEV, generator=g)
    B = torch.randn(n, n, device=DEV, generator=g)
    C1 = t.plan(n, n, n, sch, prec, name).matmul(A, B, seed=3)
    C2 = rbc.Plan(n, n, n, [sch] * c["levels"], prec=prec, leaf_tile=c["tile"]).matmul(A, B, seed=3)
    torch.cuda.synchronize()
    assert torch.equal(C1, C2)
    ref = A.double() @ B.double()
    assert float(torch.linalg.norm(C1.double() - ref) / torch.linalg.norm(ref)) < 3e-2
