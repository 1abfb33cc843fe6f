"""Seeded sweep over product shapes and level stacks (exact schemes, small-integer inputs, where
every intermediate is an integer below 2^24): C must equal the exact product bit for bit, for
f32 and f64, whatever grouping, leaf gather, tile and pairing of launches the plan picks.  The
cases are drawn once from a fixed seed, so the sweep is the same on every run."""

import numpy as np
import pytest
import torch

import paper_1905_07439_amd as rbc
import workloads

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _cases(count=24, seed=20240607):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        q = int(rng.integers(1, 4))
        names = [str(rng.choice(["strassen", "strassen", "laderman", "naive:2,3,2"])) for _ in range(q)]
        M, K, N = (int(x) for x in rng.integers(1, 700, size=3))
        # f32 stays exact for Strassen and naive stacks at these sizes (|S|, |T| <= 2 * 2^Q,
        # every partial sum below 2^24); Laderman's seven-term sums take f64
        prec = "f64" if "laderman" in names else ("f32" if rng.random() < 0.8 else "f64")
        fusion = str(rng.choice(["auto", "max"]))
        out.append((names, M, K, N, prec, fusion, int(rng.integers(0, 1000))))
    return out


@pytest.mark.parametrize("case", range(24))
def test_exact_on_integers(case):
    names, M, K, N, prec, fusion, seed = _cases()[case]
    print("sweep", case, names, M, K, N, prec, fusion, seed, flush=True)
    plan = rbc.Plan(M, K, N, [rbc.Scheme.builtin(n) for n in names], prec=prec, fusion=fusion)
    # small integers keep every intermediate exact: |entries| <= 2, K <= 700, scheme sums small
    A = workloads.integers((M, K), 100 + case, lo=-2, hi=2)
    B = workloads.integers((K, N), 200 + case, lo=-2, hi=2)
    ref = A.astype(np.int64) @ B.astype(np.int64)
    dt = torch.float64 if prec == "f64" else torch.float32
    Ad = torch.from_numpy(A.astype(np.float64)).to(DEV, dt)
    Bd = torch.from_numpy(B.astype(np.float64)).to(DEV, dt)
    for mode in ("full", "none"):
        C = plan.matmul(Ad, Bd, seed=seed, mode=mode).cpu().numpy()
        np.testing.assert_array_equal(C.astype(np.int64), ref, err_msg=str((names, M, K, N, prec, fusion, mode)))
