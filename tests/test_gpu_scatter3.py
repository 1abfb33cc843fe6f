"""Three Strassen-shaped levels in one scatter pass (k_scatter3).

The pass must compute every output with the same roundings in the same order
as the oracle's combination (eq. recursive-random-formula, the W side; sums
over ascending r, zero coefficients skipped, the first term alone), so the
stage scatter is compared with the oracle bit for bit -- as bit patterns, so
that the sign of an exact zero counts too.  The products are small integers
with exact zeros of both signs, so that many sums cancel exactly.  Levels whose
W table has Strassen's zero pattern take a walk specialized to it; perturbed
schemes (dense W) take the general walk.
"""

import os
import sys

import numpy as np
import pytest
import torch

import paper_1905_07439_amd as rbc
from oracle import recursion

from test_gpu_parity import _level_draws, _schemes

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def setup_module(module):
    assert torch.cuda.is_available(), "GPU tests need a GPU"


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _plan(M, K, N, lib_s, prec, tile, fuse):
    """A plan made with RBC_MAX_FUSED_LEVELS = fuse (None: the default rule)."""
    old = os.environ.get("RBC_MAX_FUSED_LEVELS")
    if fuse is None:
        os.environ.pop("RBC_MAX_FUSED_LEVELS", None)
    else:
        os.environ["RBC_MAX_FUSED_LEVELS"] = str(fuse)
    try:
        return rbc.Plan(M, K, N, lib_s, prec=prec, leaf_tile=tile)
    finally:
        if old is None:
            os.environ.pop("RBC_MAX_FUSED_LEVELS", None)
        else:
            os.environ["RBC_MAX_FUSED_LEVELS"] = old


CASES = [
    # (schemes, M, K, N, prec, leaf tile, scatter passes)
    (["strassen"] * 3, 512, 256, 512, "f32", 64, 1),
    (["strassen"] * 3, 300, 200, 260, "f32", 64, 1),     # ragged: cropped stores, partial position blocks
    (["strassen"] * 4, 512, 512, 512, "f32", 64, 2),     # levels [1, 4) in one pass, then level 0
    (["laderman"] + ["strassen"] * 3, 200, 150, 230, "f32", 64, 2),
    (["strassen"] * 3, 64, 64, 64, "f64", 16, 1),
    (["strassen"] * 3, 100, 90, 70, "f64", 16, 1),
    (["pert:1e-2:5"] * 3, 260, 200, 240, "f32", 64, 1),  # dense W: the general walk
    (["strassen", "pert:1e-3:7", "strassen"], 256, 256, 256, "f32", 64, 1),  # one level general
]


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("mode", ["full", "none", "signs", "perms"])
def test_three_level_scatter_bit_exact(case, mode):
    names, M, K, N, prec, tile, passes = CASES[case]
    _say("three-level scatter", names, M, K, N, prec, mode)
    lib_s, ref_s = _schemes(names)
    plan = _plan(M, K, N, lib_s, prec, tile, 3)
    info = plan.info
    assert info["n_scatter_groups"] == passes
    tdt = torch.float64 if prec == "f64" else torch.float32
    ndt = np.float64 if prec == "f64" else np.float32
    udt = np.uint64 if prec == "f64" else np.uint32
    arith = "f64" if prec == "f64" else "f32"
    L, mM, mK, mN = info["n_leaves"], info["mM"], info["mK"], info["mN"]
    g = np.random.default_rng(100 + case)
    P = g.integers(-2, 3, size=(L, mM, mN)).astype(ndt)
    P[g.random(P.shape) < 0.05] = -0.0
    s, p, dr = _level_draws(plan, ref_s, 500 + case, mode)
    ws = torch.zeros(info["workspace_bytes"], dtype=torch.uint8, device=DEV)
    ws[info["off_P"]:info["off_P"] + info["bytes_P"]].copy_(torch.from_numpy(P.view(np.uint8).reshape(-1)))
    for ks in (True, False):
        C = torch.full((M, N), float("nan"), dtype=tdt, device=DEV)
        plan.stage_scatter(s, p, C, ws, kappa_scale=ks)
        ref = recursion.combine(list(P), M, N, K, ref_s, dr, kappa_scale=ks, arith=arith, leaf_dims=(mM, mK, mN))
        got = C.cpu().numpy()
        assert np.isfinite(got).all()
        np.testing.assert_array_equal(got.view(udt), np.asarray(ref, dtype=ndt).view(udt))


@pytest.mark.parametrize("prec", ["f32", "f64", "f16s", "fp8c", "bf16x3"])
def test_three_level_scatter_same_bits_as_two_passes(prec):
    # The whole product with the default plan (one scatter pass over the three
    # levels) against a plan whose scatters take at most two levels per pass.
    N = 2048
    _say("three-level vs two-pass", prec, N)
    S = rbc.Scheme.builtin("strassen")
    p3 = _plan(N, N, N, [S] * 3, prec, 0, 3)
    p2 = _plan(N, N, N, [S] * 3, prec, 0, 2)
    assert p3.info["n_scatter_groups"] == 1 and p2.info["n_scatter_groups"] == 2
    dt = torch.float64 if prec == "f64" else torch.float32
    g = torch.Generator(device=DEV)
    g.manual_seed(4242)
    A = torch.randn(N, N, device=DEV, generator=g, dtype=dt)
    B = torch.randn(N, N, device=DEV, generator=g, dtype=dt)
    for seed, mode in [(0, "full"), (1, "signs"), (2, "perms"), (3, "none")]:
        C3 = p3.matmul(A, B, seed=seed, mode=mode)
        C2 = p2.matmul(A, B, seed=seed, mode=mode)
        torch.cuda.synchronize()
        assert torch.equal(C3.view(torch.int64 if dt == torch.float64 else torch.int32),
                           C2.view(torch.int64 if dt == torch.float64 else torch.int32)), (seed, mode)
