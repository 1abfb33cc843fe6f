"""The deepest level's scatter folded into the f32 leaf product (leaf scatter).

The workgroup that stores the last of a parent's R leaf tiles over a 64 x 64
region combines that region through the deepest level's folded W into the
parent's product block, with the same arithmetic in the same order as the
deepest scatter pass.  C must therefore be bitwise equal to the path with the
separate scatter pass (leaf gather on, leaf scatter off), which the stage tests
pin bit for bit to the oracle's combination (eq. recursive-random-formula), and
to the path with neither fusion.  The workspace is filled with NaN bytes before
the calls, so that a region combined before all of its tiles were visible, or
a counter left over from an earlier call, shows up as a mismatch.
"""

import sys

import numpy as np
import pytest
import torch

import paper_1905_07439_amd as rbc
from oracle import schemes as osch

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def setup_module(module):
    assert torch.cuda.is_available(), "GPU tests need a GPU"


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _scheme(name):
    if name.startswith("scaled:"):  # Strassen with U times u, V times v (approximate)
        _, u, v = name.split(":")
        U, V, W = osch.strassen()
        return rbc.Scheme.from_tensors(np.asarray(U) * float(u), np.asarray(V) * float(v), np.asarray(W),
                                       residual_tol=float("inf"))
    if name.startswith("wscaled:"):  # Strassen with W times w: non-unit coefficients in the folded scatter
        w = float(name.split(":")[1])
        U, V, W = osch.strassen()
        return rbc.Scheme.from_tensors(np.asarray(U), np.asarray(V), np.asarray(W) * w, residual_tol=float("inf"))
    return rbc.Scheme.builtin(name)


CASES = [
    # (schemes, M, K, N, leaf tile)
    (["strassen"] * 3, 4096, 4096, 4096, 0),     # 343 leaves of 512^3, 128-tiles with a 64-tile last round
    (["strassen"] * 3, 1000, 600, 777, 64),
    (["strassen"] * 2, 300, 192, 500, 128),      # 128-tiles whose tail tiles take 16-k slabs
    (["strassen"] * 2, 300, 200, 500, 64),
    (["laderman", "strassen"], 700, 500, 900, 64),
    (["strassen"] * 4, 1024, 1024, 1024, 0),
    (["strassen", "naive:2,3,2"], 260, 300, 170, 64),  # deepest level <2,3,2>, one term per product
    (["naive:3,2,2", "naive:2,2,2"], 1000, 1000, 1000, 0),
    (["strassen", "scaled:0.75:1.25"], 1024, 1024, 1024, 128),
    (["strassen", "wscaled:0.7"], 1000, 1000, 1000, 128),
]


@pytest.mark.parametrize("names,M,K,N,tile", CASES)
def test_leaf_scatter_same_bits(names, M, K, N, tile):
    _say("leaf scatter", names, M, K, N, tile)
    plan = rbc.Plan(M, K, N, [_scheme(n) for n in names], prec="f32", leaf_tile=tile)
    assert plan.leaf_gather[1] and plan.leaf_scatter[1]
    g = torch.Generator(device=DEV)
    g.manual_seed(M + 3 * K + 7 * N)
    A = torch.randn(M, K, device=DEV, generator=g)
    B = torch.randn(K, N, device=DEV, generator=g)
    before = plan.workspace_bytes
    plan.set_leaf_gather(True)
    plan.set_leaf_scatter(True)  # lays out its regions: the workspace grows once
    assert plan.workspace_bytes > before
    ws = plan.workspace(DEV)
    for seed, mode, ks in [(0, "full", True), (5, "full", False), (1, "signs", True), (3, "none", False),
                           (2, "perms", True)]:
        plan.set_leaf_gather(False)
        C0 = plan.matmul(A, B, seed=seed, mode=mode, kappa_scale=ks, workspace=ws)
        plan.set_leaf_gather(True)
        plan.set_leaf_scatter(False)
        C1 = plan.matmul(A, B, seed=seed, mode=mode, kappa_scale=ks, workspace=ws)
        plan.set_leaf_scatter(True)
        ws.fill_(0xFF)  # NaN in every f32 slot, and counters of -1
        C2 = plan.matmul(A, B, seed=seed, mode=mode, kappa_scale=ks, workspace=ws)
        torch.cuda.synchronize()
        assert torch.equal(C1, C0), (seed, mode, float((C1 - C0).abs().max()))
        assert torch.equal(C2, C1), (seed, mode, float((C2 - C1).abs().nan_to_num(float("inf")).max()))
    assert plan.leaf_scatter == (True, True)
    plan.set_leaf_gather(False)
    assert plan.leaf_scatter == (False, True)


def test_leaf_scatter_back_to_back_calls():
    # Many products on one workspace without synchronisation between them: every call
    # clears its counters on the stream before its leaf launch, and each result equals
    # the unfused path's for the same seed.
    N = 2048
    plan = rbc.Plan(N, N, N, [rbc.Scheme.builtin("strassen")] * 3, prec="f32", leaf_tile=128)
    plan.set_leaf_gather(True)
    plan.set_leaf_scatter(True)
    g = torch.Generator(device=DEV)
    g.manual_seed(77)
    A = torch.randn(N, N, device=DEV, generator=g)
    B = torch.randn(N, N, device=DEV, generator=g)
    ws = plan.workspace(DEV)
    ws.fill_(0xFF)
    outs = [plan.matmul(A, B, seed=s, mode="full", workspace=ws) for s in range(12)]
    plan.set_leaf_scatter(False)
    for s, C in enumerate(outs):
        ref = plan.matmul(A, B, seed=s, mode="full")
        torch.cuda.synchronize()
        assert torch.equal(C, ref), s


def test_leaf_scatter_integers_exact():
    # Small integers: every intermediate is an integer below 2^24, so C = A B exactly.
    M, K, N = 1024, 768, 640
    plan = rbc.Plan(M, K, N, [rbc.Scheme.builtin("strassen")] * 3, prec="f32", leaf_tile=64)
    plan.set_leaf_gather(True)
    plan.set_leaf_scatter(True)
    rng = np.random.default_rng(11)
    A = rng.integers(-4, 5, size=(M, K)).astype(np.float32)
    B = rng.integers(-4, 5, size=(K, N)).astype(np.float32)
    C = plan.matmul(torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV), seed=9, mode="full").cpu().numpy()
    assert np.array_equal(C.astype(np.float64), A.astype(np.float64) @ B.astype(np.float64))


def test_leaf_scatter_switches():
    plan = rbc.Plan(512, 512, 512, [rbc.Scheme.builtin("laderman")] * 2, prec="f32")
    assert plan.leaf_scatter == (False, False)
    with pytest.raises(rbc.RbcError):
        plan.set_leaf_scatter(True)
    plan = rbc.Plan(1024, 1024, 1024, [rbc.Scheme.builtin("strassen")] * 2, prec="f32")
    plan.set_leaf_gather(False)
    with pytest.raises(rbc.RbcError):
        plan.set_leaf_scatter(True)
    plan.set_leaf_gather(True)
    plan.set_leaf_scatter(True)
    assert plan.leaf_scatter == (True, True)
