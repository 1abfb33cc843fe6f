"""Products captured in a HIP graph (torch.cuda.CUDAGraph) and replayed.

A product's launches take their draws and parameters by value, and the
product path records no memset or allocation, so a captured product replays
to the bits of the eager call.  The graph is replayed several times with other
work of the program in between (another product into the same workspace, and a
fill of the output), and every replay is compared with the eager result.  The
allocation-free entry point is captured the same way (the caller it is meant
for: code under stream capture).
"""

import sys

import pytest
import torch

import paper_1905_07439_amd as rbc

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def setup_module(module):
    assert torch.cuda.is_available(), "GPU tests need a GPU"


CASES = [
    ("f32", ["strassen"] * 3, 2048),     # the leaf gather is on at this size
    ("f32", ["strassen"] * 3, 4096),     # and the scatter is one pass over the three levels (k_scatter3)
    ("f32", ["laderman", "strassen"], 600),
    ("f64", ["strassen"] * 2, 64),
    ("f16s", ["strassen"] * 2, 1024),
    ("fp8c", ["laderman", "strassen"], 768),
    ("bf16x3", ["apa322:0.001"], 768),
]


def _plan(prec, names, n):
    return rbc.Plan(n, n, n, [rbc.Scheme.builtin(x) for x in names], prec=prec)


@pytest.mark.parametrize("prec,names,n", CASES)
def test_captured_product_replays_bitwise(prec, names, n):
    print("graph", prec, names, n, flush=True)
    sys.stdout.flush()
    plan = _plan(prec, names, n)
    dt = torch.float64 if prec == "f64" else torch.float32
    g = torch.Generator(device=DEV)
    g.manual_seed(n + len(names))
    A = torch.randn(n, n, device=DEV, generator=g, dtype=dt)
    B = torch.randn(n, n, device=DEV, generator=g, dtype=dt)
    ws = plan.workspace(DEV)
    ref = plan.matmul(A, B, seed=7, mode="full", workspace=ws).clone()  # also uploads the tables
    other = plan.matmul(A, B, seed=8, mode="full", workspace=ws).clone()
    C = torch.empty_like(ref)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        plan.matmul(A, B, C=C, seed=7, mode="full", workspace=ws, stream=s)
    torch.cuda.synchronize()
    for rep in range(3):
        C.fill_(float("nan"))
        D = plan.matmul(A, B, seed=8, mode="full", workspace=ws)  # other work on the same workspace
        torch.cuda.synchronize()
        assert torch.equal(D, other)
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(C, ref), (prec, rep)


def test_captured_noalloc_product_replays_bitwise():
    plan = _plan("f32", ["strassen"] * 2, 1000)
    g = torch.Generator(device=DEV)
    g.manual_seed(5)
    A = torch.randn(1000, 1000, device=DEV, generator=g)
    B = torch.randn(1000, 1000, device=DEV, generator=g)
    ref = plan.matmul(A, B, seed=11, mode="signs").clone()
    C = torch.empty_like(ref)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        plan.matmul_noalloc(A, B, C, seed=11, mode="signs", stream=s)
    torch.cuda.synchronize()
    for rep in range(3):
        C.fill_(float("nan"))
        plan.matmul_noalloc(A, B, torch.empty_like(ref), seed=12, mode="full")  # shares the library's array
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(C, ref), rep
