"""The approximate-to-exact combination on the GPU (Section 1, eq. APA-to-EBC)
against the oracle's, element by element, and against the standard product."""
import sys

import numpy as np
import pytest
import torch

import paper_1905_07439_amd as rbc
import workloads
from oracle import recursion, schemes as osch

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
EPS7 = [0.1 * k for k in range(1, 8)]


def _say(*a):
    print("[apa_ebc]", *a, file=sys.stderr, flush=True)


def _oracle_levels(names):
    def at(e):
        out = []
        for n in names:
            out.append(getattr(osch, n)(e) if n.startswith("apa") else getattr(osch, n)())
        return out
    return at


@pytest.mark.parametrize("names,M,K,N,seed,mode", [
    (["apa322", "apa223", "apa232"], 120, 120, 120, 0, "none"),
    (["apa322", "apa223", "apa232"], 130, 100, 110, 4, "full"),
    (["apa322", "strassen"], 90, 64, 70, 2, "signs"),
])
def test_ebc_f64_matches_oracle_and_is_exact(names, M, K, N, seed, mode):
    _say(names, M, K, N, seed, mode)
    for kind in ("ints", "gauss"):
        if kind == "ints":
            A = workloads.integers((M, K), 21, -3, 3).astype(np.float64)
            B = workloads.integers((K, N), 22, -3, 3).astype(np.float64)
        else:
            A = workloads.gaussian((M, K), 23)
            B = workloads.gaussian((K, N), 24)
        C = rbc.matmul_apa_ebc(torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV), names, EPS7,
                               prec="f64", seed=seed, mode=mode)
        torch.cuda.synchronize()
        C = C.cpu().numpy()
        p = rbc.Plan(M, K, N, [rbc.Scheme.builtin(n) for n in rbc.apa_scheme_levels(names, 0.1)], prec="f64")
        dims = (p.info["mM"], p.info["mK"], p.info["mN"])
        ref = recursion.apa_ebc(A, B, _oracle_levels(names), EPS7, seed=seed, mode=mode, leaf_dims=dims)
        e_or = recursion.rel_err(C, ref)
        e_ab = recursion.rel_err(C, A @ B)
        _say(kind, "rel err vs oracle %.3g vs A B %.3g" % (e_or, e_ab))
        assert e_or <= 1e-12
        assert e_ab <= 1e-10


def test_ebc_f32_products_beat_a_single_lambda():
    # f32 products combined in f64: rounding grows with 1/eps^3 and the weights (up to
    # 35), yet the combination is far closer to A B than one approximate product.
    names = ["apa322", "apa223", "apa232"]
    A = workloads.gaussian((240, 240), 41)
    B = workloads.gaussian((240, 240), 42)
    Ad = torch.from_numpy(A.astype(np.float32)).to(DEV)
    Bd = torch.from_numpy(B.astype(np.float32)).to(DEV)
    C = rbc.matmul_apa_ebc(Ad, Bd, names, EPS7, prec="f32").cpu().numpy()
    one = rbc.Plan(240, 240, 240, [rbc.Scheme.builtin(n) for n in rbc.apa_scheme_levels(names, 0.1)], prec="f32")
    C1 = one.matmul(Ad, Bd, mode="none").cpu().numpy()
    e, e1 = recursion.rel_err(C, A @ B), recursion.rel_err(C1, A @ B)
    _say("f32 ebc %.3g single lambda=0.1 %.3g" % (e, e1))
    assert e < 1e-3 and e < e1 / 100


def test_ebc_rejects_mismatched_input():
    A = torch.zeros((32, 32), dtype=torch.float64, device=DEV)
    with pytest.raises(Exception):
        rbc.matmul_apa_ebc(A, A, ["apa322"], [0.1, 0.1])
    with pytest.raises(Exception):
        rbc.matmul_apa_ebc(A.float(), A.float(), ["apa322"], [0.1, 0.2], prec="f64")
