"""Approximate schemes at N = 3072 on bf16 hi+lo leaves (the approximate-scheme
workload), against the oracle.

Inputs: A, B i.i.d. N(0, 1) (data seeds 3001/3002) rounded to f32; the rank-10
<3,2,2> APA at one level (10 leaves of 1024 x 1536 x 1536) and perturbed
Strassen (Section 3.1 recipe, sigma = lambda) at three levels (343 leaves of
384^3), lambda in {1e-1, 1e-2, 1e-3, 1e-4}, modes none and full.  The plans
pick the 128-tile bf16 hi+lo leaf kernel, whose grid here does not fill whole
rounds, so its last round runs as 64-tiles.

The library's gathers and scatters are bit-identical to the oracle's (f32 block
combinations, f64 recombination; tests/test_gpu_parity.py), so C_gpu differs from
the oracle's emulation only through the leaf products.  The emulation: the same
f32 leaf operands split hi + lo in bf16 (oracle.precision.split_hi_lo), the three
products S_hi T_hi + S_hi T_lo + S_lo T_hi in f64, rounded to f32, then the f64
recombination and the final rounding to f32.  Every row g of C depends only on row
g mod m of every leaf product (m the leaf height), so the oracle computes the leaf
products on a sample of local rows and C is compared on every row that maps to
them.  Bound per element: the f32 accumulation of the 3K products of a leaf entry
(gamma_{3K} (|S_hi| + |S_lo|)(|T_hi| + |T_lo|), u = 2^-24) plus both sides'
roundings of P to f32, carried through |W-hat| (times |(1 - kappa)^-1| per level),
plus the f64 scatter's own roundings and the final rounding to f32.  In norm the
GPU's error against A B (f64 product of the same f32 inputs) must stay within 4x
the emulation's.
"""

import sys

import numpy as np
import pytest
import torch

import paper_1905_07439_amd as rbc
import workloads
from oracle import precision, recursion, schemes as osch, tensors as oten

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
N = 3072
U24 = 2.0 ** -24


def setup_module(module):
    assert torch.cuda.is_available(), "GPU tests need a GPU"


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


_DATA = {}


def _inputs():
    if not _DATA:
        A = workloads.gaussian((N, N), 3001).astype(np.float32)
        B = workloads.gaussian((N, N), 3002).astype(np.float32)
        _DATA.update(A=A, B=B, Ad=torch.from_numpy(A).to(DEV), Bd=torch.from_numpy(B).to(DEV))
    return _DATA


def _case(kind, lam):
    if kind == "apa322":
        return [rbc.Scheme.builtin("apa322", lam)], [osch.apa322(lam)]
    lib = rbc.Scheme.builtin("perturbed_strassen", lam, 42)
    ref = osch.perturbed(*osch.strassen(), lam, 42)
    return [lib] * 3, [ref] * 3


def _abs_levels(ref_s, dr):
    """|U|, |V|, |W| with the same permutations and all signs +1: combining with these
    gives |U-hat| etc. (folding only permutes and flips signs)."""
    absS = [tuple(np.abs(np.asarray(T, np.float64)) for T in s) for s in ref_s]
    adr = [(np.ones_like(a), np.ones_like(b), np.ones_like(c), p1, p2, p3) for a, b, c, p1, p2, p3 in dr]
    return absS, adr


def _sample_rows(m, seed):
    g = np.random.default_rng(seed)
    rows = {0, 1, 2, m // 2, m - 2, m - 1} | set(g.integers(0, m, size=10).tolist())
    return np.array(sorted(rows))


@pytest.mark.parametrize("mode", ["none", "full"])
@pytest.mark.parametrize("lam", [1e-1, 1e-2, 1e-3, 1e-4])
@pytest.mark.parametrize("kind", ["apa322", "perturbed_strassen"])
def test_cfg3_bf16x3_n3072_matches_oracle(kind, lam, mode):
    d = _inputs()
    A, B = d["A"], d["B"]
    lib_s, ref_s = _case(kind, lam)
    plan = rbc.Plan(N, N, N, lib_s, prec="bf16x3")
    info = plan.info
    assert info["tile_m"] == 128
    dims = (info["mM"], info["mK"], info["mN"])
    _say("cfg3", kind, lam, mode, "leaves", info["n_leaves"], "leaf", dims)
    seed = 3
    kscale = mode != "none"
    dr = recursion.seeded_draws(ref_s, seed, mode)
    C = plan.matmul(d["Ad"], d["Bd"], seed=seed, mode=mode).cpu().numpy()

    m, K = dims[0], dims[1]
    X = _sample_rows(m, int(lam * 1e4) + (mode == "full"))
    ops = recursion.leaf_operands(A, B, ref_s, dr, kappa_scale=kscale, arith="f32", leaf_dims=dims)
    g3k = 3 * K * U24 / (1 - 3 * K * U24)
    P_emu, P_err, P_abs = [], [], []
    for S, T in ops:
        sh, sl = [x.astype(np.float64) for x in precision.split_hi_lo(S[X], "bf16")]
        th, tl = [x.astype(np.float64) for x in precision.split_hi_lo(T, "bf16")]
        p = (sh @ th + sh @ tl + sl @ th).astype(np.float32).astype(np.float64)
        mag = (np.abs(sh) + np.abs(sl)) @ (np.abs(th) + np.abs(tl))
        full = np.zeros((m, dims[2]))
        err = np.zeros((m, dims[2]))
        pab = np.zeros((m, dims[2]))
        full[X] = p
        err[X] = g3k * mag + 2 * U24 * np.abs(p)
        pab[X] = np.abs(p)
        P_emu.append(full)
        P_err.append(err)
        P_abs.append(pab)
    del ops
    emu = recursion.combine(P_emu, N, N, N, ref_s, dr, kappa_scale=kscale, arith="f64", leaf_dims=dims)
    absS, adr = _abs_levels(ref_s, dr)
    fac = 1.0
    if kscale:
        for s in ref_s:
            fac *= abs(1.0 / (1.0 - float(oten.kappa(*s))))
    bound = fac * recursion.combine(P_err, N, N, N, absS, adr, kappa_scale=False, leaf_dims=dims)
    pmag = fac * recursion.combine(P_abs, N, N, N, absS, adr, kappa_scale=False, leaf_dims=dims)
    del P_emu, P_err, P_abs
    G = np.flatnonzero(np.isin(np.arange(N) % m, X))
    emu32 = emu[G].astype(np.float32).astype(np.float64)
    bound = bound[G] + 64 * 2.0 ** -53 * pmag[G] + 2 * U24 * np.abs(emu[G]) + 1e-30
    diff = np.abs(C[G].astype(np.float64) - emu32)
    worst = float(np.max(diff / bound))
    _say("cfg3 %s lam %g %s: max |C - emulation| / bound = %.3g over %d rows" % (kind, lam, mode, worst, G.size))
    assert np.all(diff <= bound), worst

    # norms on the sampled rows: the GPU's error against A B within 4x the emulation's;
    # the algorithmic error of the f64 recursion (exact arithmetic up to f64) beside them
    AB = A[G].astype(np.float64) @ B.astype(np.float64)
    e_gpu = recursion.rel_err(C[G], AB)
    e_emu = recursion.rel_err(emu[G], AB)
    ops64 = recursion.leaf_operands(A, B, ref_s, dr, kappa_scale=kscale, arith="f64", leaf_dims=dims)
    P64 = []
    for S, T in ops64:
        full = np.zeros((m, dims[2]))
        full[X] = S[X] @ T
        P64.append(full)
    del ops64
    f64 = recursion.combine(P64, N, N, N, ref_s, dr, kappa_scale=kscale, arith="f64", leaf_dims=dims)[G]
    e_alg = recursion.rel_err(f64, AB)
    e_num = recursion.rel_err(C[G], f64)
    _say("cfg3 %s lam %g %s: rel err vs AB %.3g (emulation %.3g); algorithmic %.3g, numerical %.3g"
         % (kind, lam, mode, e_gpu, e_emu, e_alg, e_num))
    assert e_gpu <= 4 * e_emu + 1e-7


def test_apa_ebc_bf16x3_matches_oracle_emulation():
    # The exact combination of the 12 x 12 step over seven lambda (eq. APA-to-EBC) on
    # bf16 hi+lo leaves: element-wise against the weighted sum of the oracle's bf16x3
    # emulations of the seven products (same draws), and close to A B.
    n = 240
    names = ["apa322", "apa223", "apa232"]
    eps = [0.1 * k for k in range(1, 8)]
    A = workloads.gaussian((n, n), 31).astype(np.float32)
    B = workloads.gaussian((n, n), 32).astype(np.float32)
    Ad, Bd = torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV)
    plans = rbc.apa_ebc_plans(n, n, n, names, eps, prec="bf16x3")
    dims = (plans[0].info["mM"], plans[0].info["mK"], plans[0].info["mN"])
    alpha = osch.apa_ebc_weights(eps)
    for seed, mode in ((0, "none"), (5, "full")):
        C = rbc.matmul_apa_ebc(Ad, Bd, names, eps, prec="bf16x3", seed=seed, mode=mode, plans=plans).cpu().numpy()
        total = np.zeros((n, n))
        bound = np.zeros((n, n))
        K = dims[1]
        g3k = 3 * K * U24 / (1 - 3 * K * U24)
        for a, e in zip(alpha, eps):
            lv = [osch.apa322(e), osch.apa223(e), osch.apa232(e)]
            dr = recursion.seeded_draws(lv, seed, mode)
            ops = recursion.leaf_operands(A, B, lv, dr, kappa_scale=False, arith="f32", leaf_dims=dims)
            prods, errs, pabs = [], [], []
            for S, T in ops:
                sh, sl = [x.astype(np.float64) for x in precision.split_hi_lo(S, "bf16")]
                th, tl = [x.astype(np.float64) for x in precision.split_hi_lo(T, "bf16")]
                p = (sh @ th + sh @ tl + sl @ th).astype(np.float32).astype(np.float64)
                prods.append(p)
                errs.append(g3k * ((np.abs(sh) + np.abs(sl)) @ (np.abs(th) + np.abs(tl))) + 2 * U24 * np.abs(p))
                pabs.append(np.abs(p))
            Ce = recursion.combine(prods, n, n, n, lv, dr, kappa_scale=False, arith="f64", leaf_dims=dims)
            absS, adr = _abs_levels(lv, dr)
            be = recursion.combine(errs, n, n, n, absS, adr, kappa_scale=False, leaf_dims=dims)
            pm = recursion.combine(pabs, n, n, n, absS, adr, kappa_scale=False, leaf_dims=dims)
            # each product is rounded to f32 before its weighted f64 accumulation
            Ce32 = Ce.astype(np.float32).astype(np.float64)
            total = total + a * Ce32
            # (the library's weights come from its own formula: allow 1e-12 relative in alpha)
            bound = bound + abs(a) * (be + 64 * 2.0 ** -53 * pm + 2 * U24 * np.abs(Ce) + 1e-12 * np.abs(Ce))
        diff = np.abs(C - total)
        worst = float(np.max(diff / (bound + 1e-30)))
        AB = A.astype(np.float64) @ B.astype(np.float64)
        _say("apa-ebc bf16x3 %s: max |C - emulation| / bound = %.3g; rel err vs AB %.3g (emulation %.3g)"
             % (mode, worst, recursion.rel_err(C, AB), recursion.rel_err(total, AB)))
        assert np.all(diff <= bound + 1e-30), worst
        assert recursion.rel_err(C, AB) <= 4 * recursion.rel_err(total, AB) + 1e-6
