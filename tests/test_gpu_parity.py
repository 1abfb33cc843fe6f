"""GPU parity of the HIP path against the oracle (run on an MI355X).

Stages: the gathers and the scatter are compared with the oracle's recursion
element by element and must be bit-identical (same folded coefficients, same
summation order, one rounding per operation).  The leaf products are compared
with a float64 matmul within the format's rounding.  End to end: exact schemes
on small integers are exact (every intermediate stays below 2^24 here), and
real inputs are held to the tolerances written in each test.
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
AUX_EXPS = 8192  # byte offset of the per-leaf exponents in the auxiliary region (include/rbc.h)


def setup_module(module):
    assert torch.cuda.is_available(), "GPU tests need a GPU"


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


BASE = {"strassen": osch.strassen, "laderman": osch.laderman}


def _schemes(names):
    """(library schemes, oracle tensors) for a list of names ("strassen", "laderman",
    "naive:b1,b2,b3", "pert:<sigma>:<seed>", "apa322:<lambda>" for the rank-10 <3,2,2> APA, "apa223:", "apa232:" for its rotations)."""
    lib, ref = [], []
    for n in names:
        if n.startswith("naive:"):
            b = tuple(int(x) for x in n[6:].split(","))
            lib.append(rbc.Scheme.builtin(n))
            ref.append(osch.naive(*b))
        elif n.startswith("apa"):  # apa322:<lambda>, apa223:<lambda>, apa232:<lambda>
            kind, lam = n.split(":")
            lib.append(rbc.Scheme.builtin("%s:%r" % (kind, float(lam))))
            ref.append(getattr(osch, kind)(float(lam)))
        elif n.startswith("scaled:"):  # scaled:<u>:<v>: Strassen with U times u, V times v (approximate)
            _, u, v = n.split(":")
            U, V, W = osch.strassen()
            U, V = np.asarray(U) * float(u), np.asarray(V) * float(v)
            lib.append(rbc.Scheme.from_tensors(U, V, W, residual_tol=float("inf")))
            ref.append((U, V, np.asarray(W)))
        elif n.startswith("pert:"):
            _, sigma, seed = n.split(":")
            base = osch.strassen()
            lib.append(rbc.Scheme.builtin("perturbed_strassen", float(sigma), int(seed)))
            ref.append(osch.perturbed(*base, float(sigma), int(seed)))
        else:
            lib.append(rbc.Scheme.builtin(n))
            ref.append(BASE[n]())
    return lib, ref


def _level_draws(plan, ref, seed, mode):
    s, p = plan.draws(seed, mode)
    out, o = [], 0
    for U, V, W in ref:
        b1, b2, b3, _ = oten.dims(U, V, W)
        n = b1 + b2 + b3
        ss, pp = s[o:o + n], p[o:o + n]
        out.append((ss[:b1], ss[b1:b1 + b2], ss[b1 + b2:], pp[:b1], pp[b1:b1 + b2], pp[b1 + b2:]))
        o += n
    return s, p, out


def _region(ws, off, nbytes, dtype, shape):
    return ws[off:off + nbytes].view(dtype).reshape(shape).cpu().numpy()


GATHER_CASES = [
    # (schemes, M, K, N, prec, tile)
    (["strassen"], 64, 64, 64, "f32", 64),
    (["strassen", "strassen"], 130, 70, 90, "f32", 64),
    (["strassen"] * 3, 512, 256, 512, "f32", 64),
    (["laderman"], 200, 150, 100, "f32", 64),
    (["laderman", "strassen"], 300, 200, 260, "f32", 64),
    (["naive:2,3,2", "strassen"], 100, 130, 70, "f32", 64),
    (["strassen"] * 4, 512, 512, 512, "f32", 64),
    (["pert:1e-2:5", "pert:1e-3:6"], 150, 150, 150, "f32", 64),
    (["strassen", "strassen"], 64, 64, 64, "f64", 16),
    (["laderman", "pert:1e-2:1"], 90, 60, 120, "f64", 16),
    ([], 100, 60, 50, "f32", 64),
    (["apa322:0.0625", "strassen"], 150, 100, 90, "f32", 64),
    (["apa322:0.001", "apa322:0.01"], 90, 60, 50, "f64", 16),
    (["apa322:0.015", "apa223:0.015", "apa232:0.015"], 130, 100, 120, "f32", 64),
    # exact blocks (leaf tile -1): the unpadded problem's block structure, leaves of any size
    (["strassen"] * 3, 80, 80, 80, "f32", -1),
    (["strassen"] * 2, 321, 130, 99, "f32", -1),
    (["laderman", "strassen"], 100, 90, 110, "f64", -1),
    (["pert:1e-3:42"] * 3, 80, 80, 80, "f64", -1),
]


@pytest.mark.parametrize("case", range(len(GATHER_CASES)))
@pytest.mark.parametrize("mode", ["full", "none", "signs", "perms"])
def test_gather_and_scatter_bit_exact(case, mode):
    names, M, K, N, prec, tile = GATHER_CASES[case]
    _say("gather/scatter case", names, M, K, N, prec, mode)
    lib_s, ref_s = _schemes(names)
    plan = rbc.Plan(M, K, N, lib_s, prec=prec, leaf_tile=tile)
    info = plan.info
    arith = "f64" if prec == "f64" else "f32"
    tdt = torch.float64 if prec == "f64" else torch.float32
    ndt = np.float64 if prec == "f64" else np.float32
    A = workloads.gaussian((M, K), 10 + case).astype(ndt)
    B = workloads.gaussian((K, N), 20 + case).astype(ndt)
    seed = 1000 + case
    s, p, dr = _level_draws(plan, ref_s, seed, mode)
    ws = torch.zeros(info["workspace_bytes"], dtype=torch.uint8, device=DEV)
    Ad = torch.from_numpy(A).to(DEV)
    Bd = torch.from_numpy(B).to(DEV)
    plan.stage_gather(0, Ad, s, p, ws)
    plan.stage_gather(1, Bd, s, p, ws)
    torch.cuda.synchronize()
    L, mM, mK, mN = info["n_leaves"], info["mM"], info["mK"], info["mN"]
    Sg = _region(ws, info["off_S"], info["bytes_S"], tdt, (L, mM, mK))
    Tg = _region(ws, info["off_T"], info["bytes_T"], tdt, (L, mK, mN))
    ops = recursion.leaf_operands(A, B, ref_s, dr, kappa_scale=(mode != "none"), arith=arith,
                                  leaf_dims=(mM, mK, mN))
    assert len(ops) == L
    for l, (S, T) in enumerate(ops):
        np.testing.assert_array_equal(Sg[l], S, err_msg="S leaf %d" % l)
        np.testing.assert_array_equal(Tg[l], T, err_msg="T leaf %d" % l)
    # scatter of random products
    g = np.random.default_rng(case)
    P = g.standard_normal((L, mM, mN)).astype(ndt)
    ws[info["off_P"]:info["off_P"] + info["bytes_P"]].copy_(torch.from_numpy(P.view(np.uint8).reshape(-1)))
    for ks in (True, False):
        C = torch.full((M, N), float("nan"), dtype=tdt, device=DEV)
        plan.stage_scatter(s, p, C, ws, kappa_scale=ks)
        ref = recursion.combine(list(P), M, N, K, ref_s, dr, kappa_scale=ks, arith=arith,
                                leaf_dims=(mM, mK, mN))
        np.testing.assert_array_equal(C.cpu().numpy(), ref)


@pytest.mark.parametrize("prec,names,N", [("f32", ["strassen"] * 5, 320), ("f64", ["strassen"] * 3, 80),
                                          ("f32", ["laderman", "strassen"], 102), ("f64", ["strassen"] * 2, 77)])
def test_exact_blocks_end_to_end(prec, names, N):
    # Exact-block plans split the matrices as the unpadded problem does (N = 320 with five
    # Strassen levels: leaves of 10 x 10) -- the oracle's default padding.  Integers are exact;
    # f64 Gaussian products match the oracle's recursion to rounding.
    _say("exact blocks", prec, names, N)
    lib_s, ref_s = _schemes(names)
    plan = rbc.Plan(N, N, N, lib_s, prec=prec, leaf_tile=-1)
    P1 = int(np.prod([osch_dims(r)[0] for r in ref_s]))
    assert plan.info["Mp"] == -(-N // P1) * P1 and plan.info["mM"] == -(-N // P1)
    tdt = torch.float64 if prec == "f64" else torch.float32
    ndt = np.float64 if prec == "f64" else np.float32
    Ai = workloads.integers((N, N), 31).astype(ndt)
    Bi = workloads.integers((N, N), 32).astype(ndt)
    for seed, mode in [(0, "full"), (3, "signs"), (4, "none")]:
        C = plan.matmul(torch.from_numpy(Ai).to(DEV), torch.from_numpy(Bi).to(DEV), seed=seed, mode=mode)
        torch.cuda.synchronize()
        assert np.array_equal(C.cpu().numpy(), (Ai.astype(np.float64) @ Bi.astype(np.float64)).astype(ndt))
    if prec == "f64":
        A = workloads.gaussian((N, N), 33)
        B = workloads.gaussian((N, N), 34)
        C = plan.matmul(torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV), seed=7).cpu().numpy()
        ref = recursion.rbc_seeded(A, B, ref_s, 7)
        assert recursion.rel_err(C, ref) <= 1e-13


def osch_dims(t):
    return oten.dims(*t)


@pytest.mark.parametrize("names,M,K,N", [(["strassen", "strassen"], 256, 192, 320),
                                         (["laderman"], 192, 96, 288),
                                         (["apa322:0.001", "strassen"], 288, 160, 192),
                                         (["apa322:0.03", "apa223:0.03", "apa232:0.03"], 240, 240, 240)])
def test_bf16x3_gather_split_and_f64_scatter_bit_exact(names, M, K, N):
    _say("bf16x3 stages", names, M, K, N)
    lib_s, ref_s = _schemes(names)
    plan = rbc.Plan(M, K, N, lib_s, prec="bf16x3", leaf_tile=64)
    info = plan.info
    A = workloads.gaussian((M, K), 1).astype(np.float32)
    B = workloads.gaussian((K, N), 2).astype(np.float32)
    s, p, dr = _level_draws(plan, ref_s, 3, "full")
    ws = torch.zeros(info["workspace_bytes"], dtype=torch.uint8, device=DEV)
    plan.stage_gather(0, torch.from_numpy(A).to(DEV), s, p, ws)
    plan.stage_gather(1, torch.from_numpy(B).to(DEV), s, p, ws)
    torch.cuda.synchronize()
    L, mM, mK, mN = info["n_leaves"], info["mM"], info["mK"], info["mN"]
    Sg = _region(ws, info["off_S"], info["bytes_S"], torch.int16, (2, L, mM, mK)).view(np.uint16)
    Tg = _region(ws, info["off_T"], info["bytes_T"], torch.int16, (2, L, mK, mN)).view(np.uint16)
    ops = recursion.leaf_operands(A, B, ref_s, dr, arith="f32", leaf_dims=(mM, mK, mN))
    for l, (S, T) in enumerate(ops):
        for X, G in ((S, Sg), (T, Tg)):
            hi, lo = precision.split_hi_lo(X, "bf16")
            np.testing.assert_array_equal(G[0, l], (hi.view(np.uint32) >> 16).astype(np.uint16))
            np.testing.assert_array_equal(G[1, l], (lo.view(np.uint32) >> 16).astype(np.uint16))
    P = np.random.default_rng(0).standard_normal((L, mM, mN)).astype(np.float32)
    ws[info["off_P"]:info["off_P"] + info["bytes_P"]].copy_(torch.from_numpy(P.view(np.uint8).reshape(-1)))
    C = torch.empty((M, N), dtype=torch.float32, device=DEV)
    plan.stage_scatter(s, p, C, ws)
    ref = recursion.combine(list(P.astype(np.float64)), M, N, K, ref_s, dr, arith="f64",
                            leaf_dims=(mM, mK, mN)).astype(np.float32)
    np.testing.assert_array_equal(C.cpu().numpy(), ref)


@pytest.mark.parametrize("prec,m,n,k,tile,batch", [("f32", 128, 256, 64, 128, 3), ("f32", 64, 128, 48, 64, 4),
                                                   ("f64", 16, 48, 20, 16, 3), ("f32", 512, 512, 512, 128, 2)])
def test_leaf_products(prec, m, n, k, tile, batch):
    # A zero-level plan is one leaf; use the stage API on a plan with the given leaf count.
    _say("leaf", prec, m, n, k, tile, batch)
    S = rbc.Scheme.builtin("naive:1,1,%d" % batch) if batch > 1 else None
    plan = rbc.Plan(m, k, n * batch, [S] if S else [], prec=prec, leaf_tile=tile)
    info = plan.info
    assert info["n_leaves"] == batch and (info["mM"], info["mK"], info["mN"]) == (m, k, n)
    tdt = torch.float64 if prec == "f64" else torch.float32
    g = torch.Generator(device="cpu").manual_seed(0)
    ws = torch.zeros(info["workspace_bytes"], dtype=torch.uint8, device=DEV)
    Sx = torch.randn(batch, m, k, generator=g, dtype=tdt)
    Tx = torch.randn(batch, k, n, generator=g, dtype=tdt)
    ws[info["off_S"]:info["off_S"] + info["bytes_S"]].copy_(Sx.view(torch.uint8).reshape(-1))
    ws[info["off_T"]:info["off_T"] + info["bytes_T"]].copy_(Tx.view(torch.uint8).reshape(-1))
    plan.stage_leaf(ws)
    torch.cuda.synchronize()
    P = _region(ws, info["off_P"], info["bytes_P"], tdt, (batch, m, n))
    ref = np.matmul(Sx.double().numpy(), Tx.double().numpy())
    eps = 2.0 ** -53 if prec == "f64" else 2.0 ** -24
    bound = 2 * k * eps * np.matmul(np.abs(Sx.double().numpy()), np.abs(Tx.double().numpy()))
    assert np.all(np.abs(P - ref) <= bound + 1e-300)


def test_cfg1_fp64_n64_strassen_two_levels():
    # Strassen, Q = 2, N = 64 -> 49 leaves of 16x16, f64; seed 0; data seeds 1001..1003.
    _say("cfg1 f64 n=64")
    lib_s, ref_s = _schemes(["strassen", "strassen"])
    plan = rbc.Plan(64, 64, 64, lib_s, prec="f64")
    Ai = workloads.integers((64, 64), 1003)
    Bi = workloads.integers((64, 64), 1004)
    for mode in ("full", "signs", "perms", "none"):
        C = plan.matmul(torch.from_numpy(Ai.astype(np.float64)).to(DEV),
                        torch.from_numpy(Bi.astype(np.float64)).to(DEV), seed=0, mode=mode)
        np.testing.assert_array_equal(C.cpu().numpy(), (Ai @ Bi).astype(np.float64))
    A = workloads.gaussian((64, 64), 1001)
    B = workloads.gaussian((64, 64), 1002)
    C = plan.matmul(torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV), seed=0).cpu().numpy()
    ref = recursion.rbc_seeded(A, B, ref_s, 0)
    assert recursion.rel_err(C, ref) <= 1e-13
    assert recursion.rel_err(C, A @ B) <= 1e-13


@pytest.mark.parametrize("names,M,K,N,tile", [
    (["strassen"] * 3, 4096, 4096, 4096, 0),
    (["strassen"] * 3, 1000, 600, 777, 64),
    (["laderman", "strassen"], 700, 500, 900, 64),
    (["strassen"] * 5, 2048, 2048, 2048, 64),
    (["naive:2,3,2"], 130, 90, 200, 64),
    ([], 300, 200, 100, 64),
])
def test_f32_integers_exact(names, M, K, N, tile):
    _say("f32 integers exact", names, M, K, N)
    lib_s, _ = _schemes(names)
    plan = rbc.Plan(M, K, N, lib_s, prec="f32", leaf_tile=tile)
    A = workloads.integers((M, K), 7)
    B = workloads.integers((K, N), 8)
    # float64 product of the integer matrices: exact here (|entries| < 2^53), and fast
    ref = (A.astype(np.float64) @ B.astype(np.float64)).astype(np.float32)
    Ad = torch.from_numpy(A.astype(np.float32)).to(DEV)
    Bd = torch.from_numpy(B.astype(np.float32)).to(DEV)
    for seed, mode in [(0, "full"), (1, "signs"), (2, "perms"), (3, "none")]:
        C = plan.matmul(Ad, Bd, seed=seed, mode=mode)
        np.testing.assert_array_equal(C.cpu().numpy(), ref, err_msg="seed %d %s" % (seed, mode))


def _abs_draws(dr):
    """Same permutations, all signs +1: folding |U|, |V|, |W| with these gives |U-hat| etc."""
    return [(np.ones_like(a), np.ones_like(b), np.ones_like(c), p1, p2, p3) for a, b, c, p1, p2, p3 in dr]


def test_cfg2_f32_n4096_uniform_matches_oracle():
    # Strassen Q = 3, N = 4096, 512^3 leaves on f32 MFMA; U[-1,1], data seeds 2001/2002.
    # The gathers and the scatter are bit-identical to the oracle's float32 recursion, so
    # C_gpu - C_oracle comes from the leaf products alone: |P_gpu - P| <= g_K |S||T| with
    # g_K = K u / (1 - K u) (f32 accumulation over K = 512, u = 2^-24), carried up through
    # |W-hat|, plus the scatter's own roundings of the perturbed sums (<= 8u |W-hat||P| here).
    _say("cfg2 f32 n=4096 vs oracle")
    lib_s, ref_s = _schemes(["strassen"] * 3)
    plan = rbc.Plan(4096, 4096, 4096, lib_s, prec="f32")
    A = workloads.uniform((4096, 4096), 2001, -1, 1)
    B = workloads.uniform((4096, 4096), 2002, -1, 1)
    A32, B32 = A.astype(np.float32), B.astype(np.float32)
    AB = A32.astype(np.float64) @ B32.astype(np.float64)
    Ad = torch.from_numpy(A32).to(DEV)
    Bd = torch.from_numpy(B32).to(DEV)
    dr = recursion.seeded_draws(ref_s, 0)
    emu = recursion.rbc(A32, B32, ref_s, dr, arith="f32")
    ops = recursion.leaf_operands(A32, B32, ref_s, dr, arith="f32")
    u, K = 2.0 ** -24, 512
    gK = K * u / (1 - K * u)
    absS = [tuple(np.abs(T.astype(np.float64)) for T in sch) for sch in ref_s]
    leaf_err = [gK * (np.abs(S.astype(np.float64)) @ np.abs(T.astype(np.float64))) for S, T in ops]
    leaf_abs = [np.abs(S.astype(np.float64) @ T.astype(np.float64)) for S, T in ops]
    del ops
    adr = _abs_draws(dr)
    bound = recursion.combine(leaf_err, 4096, 4096, 4096, absS, adr, kappa_scale=False) + \
        8 * u * recursion.combine(leaf_abs, 4096, 4096, 4096, absS, adr, kappa_scale=False)
    errs = []
    for seed in range(16):
        C = plan.matmul(Ad, Bd, seed=seed).cpu().numpy()
        e = recursion.rel_err(C, AB)
        errs.append(e)
        assert e <= 1e-5, (seed, e)
        if seed == 0:
            diff = np.abs(C.astype(np.float64) - emu.astype(np.float64))
            assert np.all(diff <= bound), float(np.max(diff / np.maximum(bound, 1e-300)))
            _say("cfg2 max |C - oracle| / bound = %.3g" % float(np.max(diff / bound)))
    _say("cfg2 rel err per seed", ["%.3g" % e for e in errs],
         "oracle f32 (exactly rounded leaves) %.3g" % recursion.rel_err(emu, AB))


def test_perturbed_f64_matches_oracle_and_expectation_direction():
    _say("perturbed f64")
    lib_s, ref_s = _schemes(["pert:1e-2:3", "pert:1e-2:4"])
    plan = rbc.Plan(96, 96, 96, lib_s, prec="f64")
    A = workloads.gaussian((96, 96), 5)
    B = workloads.gaussian((96, 96), 6)
    Ad, Bd = torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV)
    for seed in range(4):
        for mode in ("full", "none"):
            C = plan.matmul(Ad, Bd, seed=seed, mode=mode).cpu().numpy()
            # an approximate scheme's result depends on the block partition: use the plan's padding
            ref = recursion.rbc_seeded(A, B, ref_s, seed, mode,
                                       leaf_dims=(plan.info["mM"], plan.info["mK"], plan.info["mN"]))
            assert recursion.rel_err(C, ref) <= 1e-13


def test_apa_f64_matches_oracle_and_error_is_order_lambda():
    # The rank-10 <3,2,2> APA at two levels, f64: the library against the oracle's
    # recursion on the same draws (1/lambda = 16 amplifies the leaf products' rounding
    # differences only 16^2-fold), and the approximation error against A B shrinking
    # with lambda.
    _say("apa f64")
    A = workloads.gaussian((150, 100), 7)
    B = workloads.gaussian((100, 90), 8)
    AB = A @ B
    Ad, Bd = torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV)
    errs = []
    for lam in (2.0 ** -4, 2.0 ** -8, 2.0 ** -12):
        lib_s, ref_s = _schemes(["apa322:%r" % lam] * 2)
        plan = rbc.Plan(150, 100, 90, lib_s, prec="f64")
        for seed, mode in ((0, "full"), (1, "none")):
            C = plan.matmul(Ad, Bd, seed=seed, mode=mode).cpu().numpy()
            ref = recursion.rbc_seeded(A, B, ref_s, seed, mode,
                                       leaf_dims=(plan.info["mM"], plan.info["mK"], plan.info["mN"]))
            assert recursion.rel_err(C, ref) <= 1e-12 / lam ** 2, (lam, seed, mode)
        errs.append(recursion.rel_err(C, AB))
    _say("apa f64 rel err vs A B", errs)
    assert errs[1] < errs[0] / 8 and errs[2] < errs[1] / 8


def test_bini12_step_f64_and_f32_match_oracle():
    # One step of the rank-1000 12 x 12 approximate scheme (three levels <3,2,2>,
    # <2,2,3>, <2,3,2>) at N = 240: f64 against the oracle's recursion on the same
    # draws, and f32 within the f32 emulation's error, which grows like u / lambda^3.
    _say("bini12 f64/f32")
    A = workloads.gaussian((240, 240), 31)
    B = workloads.gaussian((240, 240), 32)
    AB = A @ B
    lam = 2.0 ** -5
    lib_s, ref_s = _schemes(["apa322:%r" % lam, "apa223:%r" % lam, "apa232:%r" % lam])
    plan = rbc.Plan(240, 240, 240, lib_s, prec="f64")
    dims = (plan.info["mM"], plan.info["mK"], plan.info["mN"])
    for seed, mode in ((0, "full"), (2, "none")):
        C = plan.matmul(torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV), seed=seed, mode=mode)
        ref = recursion.rbc_seeded(A, B, ref_s, seed, mode, leaf_dims=dims)
        assert recursion.rel_err(C.cpu().numpy(), ref) <= 1e-11
    e64 = recursion.rel_err(C.cpu().numpy(), AB)
    p32 = rbc.Plan(240, 240, 240, lib_s, prec="f32")
    C32 = p32.matmul(torch.from_numpy(A.astype(np.float32)).to(DEV),
                     torch.from_numpy(B.astype(np.float32)).to(DEV), seed=2, mode="none").cpu().numpy()
    e32 = recursion.rel_err(C32, AB)
    _say("bini12 rel err f64 %.3g f32 %.3g" % (e64, e32))
    assert e64 < 0.2 and e32 < e64 + 2.0 ** -23 / lam ** 3 * 64


def test_bf16x3_end_to_end():
    _say("bf16x3 end to end")
    lib_s, ref_s = _schemes(["strassen"] * 3)
    plan = rbc.Plan(768, 768, 768, lib_s, prec="bf16x3", leaf_tile=0)
    A = workloads.gaussian((768, 768), 3001)
    B = workloads.gaussian((768, 768), 3002)
    AB = A @ B
    C = plan.matmul(torch.from_numpy(A.astype(np.float32)).to(DEV),
                    torch.from_numpy(B.astype(np.float32)).to(DEV), seed=0).cpu().numpy()

    def leaf(S, T):
        sh, sl = precision.split_hi_lo(S.astype(np.float32), "bf16")
        th, tl = precision.split_hi_lo(T.astype(np.float32), "bf16")
        sh, sl, th, tl = [x.astype(np.float64) for x in (sh, sl, th, tl)]
        return (sh @ th + sh @ tl + sl @ th).astype(np.float32).astype(np.float64)

    # emulation: f32 combinations, split leaves, f64 recombination
    ops = recursion.leaf_operands(A.astype(np.float32), B.astype(np.float32), ref_s,
                                  recursion.seeded_draws(ref_s, 0), arith="f32")
    prods = [leaf(S, T) for S, T in ops]
    emu = recursion.combine(prods, 768, 768, 768, ref_s, recursion.seeded_draws(ref_s, 0), arith="f64")
    e_emu = recursion.rel_err(emu, AB)
    e = recursion.rel_err(C, AB)
    _say("bf16x3 rel err %.3g, emulation %.3g" % (e, e_emu))
    assert e <= 1.5 * e_emu + 2e-7 and e <= 1e-4


F16S_CASES = [(["laderman", "strassen"], 480, 480, 480, 0), (["laderman"], 192, 192, 192, 0),
              (["strassen", "strassen"], 300, 260, 200, 32), (["laderman", "strassen", "strassen"], 1152, 1152, 1152, 0),
              (["strassen"], 200, 190, 180, 96)]


@pytest.mark.parametrize("case", range(len(F16S_CASES)))
def test_f16s_scaled_leaves(case):
    # f16 leaves with per-leaf power-of-two scales: exponents and scaled operands are
    # bit-identical to the oracle's; the product is within the f16 emulation's error.
    names, M, K, N, tile = F16S_CASES[case]
    _say("f16s", names, M, K, N)
    lib_s, ref_s = _schemes(names)
    plan = rbc.Plan(M, K, N, lib_s, prec="f16s", leaf_tile=tile)
    info = plan.info
    A = workloads.scaled_gaussian((M, K), 4000 + case).astype(np.float32)
    B = workloads.scaled_gaussian((K, N), 4100 + case).astype(np.float32)
    s, p, dr = _level_draws(plan, ref_s, 7, "full")
    ws = torch.zeros(info["workspace_bytes"], dtype=torch.uint8, device=DEV)
    Ad, Bd = torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV)
    plan.stage_gather(0, Ad, s, p, ws)
    plan.stage_gather(1, Bd, s, p, ws)
    torch.cuda.synchronize()
    L, mM, mK, mN = info["n_leaves"], info["mM"], info["mK"], info["mN"]
    Sg = _region(ws, info["off_S"], info["bytes_S"], torch.int16, (L, mM, mK)).view(np.float16)
    Tg = _region(ws, info["off_T"], info["bytes_T"], torch.int16, (L, mK, mN)).view(np.float16)
    ex = _region(ws, info["off_aux"] + AUX_EXPS, 2 * L * 4, torch.int32, (2, L))
    dims = (mM, mK, mN)
    ops = recursion.leaf_operands(A, B, ref_s, dr, arith="f32", leaf_dims=dims)
    gA, gB = precision.path_norms(ref_s, "A"), precision.path_norms(ref_s, "B")
    mA, mB = float(np.max(np.abs(A))), float(np.max(np.abs(B)))
    prods = []
    for l, (S, T) in enumerate(ops):
        eA, eB = precision.leaf_exponent(mA, gA[l]), precision.leaf_exponent(mB, gB[l])
        assert (ex[0, l], ex[1, l]) == (eA, eB), l
        S16 = np.ldexp(S, eA).astype(np.float16)
        T16 = np.ldexp(T, eB).astype(np.float16)
        np.testing.assert_array_equal(Sg[l].view(np.uint16), S16.view(np.uint16))
        np.testing.assert_array_equal(Tg[l].view(np.uint16), T16.view(np.uint16))
        prods.append(np.ldexp(S16.astype(np.float64) @ T16.astype(np.float64), -(eA + eB)).astype(np.float32))
    emu = recursion.combine(prods, M, N, K, ref_s, dr, arith="f32", leaf_dims=dims)
    C = plan.matmul(Ad, Bd, seed=7).cpu().numpy()
    AB = A.astype(np.float64) @ B.astype(np.float64)
    e, e_emu = recursion.rel_err(C, AB), recursion.rel_err(emu, AB)
    _say("f16s rel err %.3g, emulation %.3g" % (e, e_emu))
    assert e <= 1.1 * e_emu + 1e-6 and e < 2e-2


FP8C_CASES = [(["strassen", "strassen"], 256, 256, 256, 0), (["laderman"], 192, 192, 192, 0),
              (["laderman", "strassen"], 480, 480, 480, 0), (["strassen"], 200, 190, 180, 96),
              (["pert:0.001:42", "pert:0.001:42"], 512, 512, 512, 0), (["strassen"] * 3, 1024, 1024, 1024, 128)]


@pytest.mark.parametrize("case", range(len(FP8C_CASES)))
def test_fp8c_split_leaves(case):
    # fp8 leaves: exponents and both e4m3 planes are bit-identical to the oracle's scaled
    # split; the product is within the emulation's error (the device accumulates in f32).
    names, M, K, N, tile = FP8C_CASES[case]
    _say("fp8c", names, M, K, N)
    lib_s, ref_s = _schemes(names)
    plan = rbc.Plan(M, K, N, lib_s, prec="fp8c", leaf_tile=tile)
    info = plan.info
    A = workloads.scaled_gaussian((M, K), 4200 + case).astype(np.float32)
    B = workloads.scaled_gaussian((K, N), 4300 + case).astype(np.float32)
    s, p, dr = _level_draws(plan, ref_s, 11, "full")
    ws = torch.zeros(info["workspace_bytes"], dtype=torch.uint8, device=DEV)
    Ad, Bd = torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV)
    plan.stage_gather(0, Ad, s, p, ws)
    plan.stage_gather(1, Bd, s, p, ws)
    torch.cuda.synchronize()
    L, mM, mK, mN = info["n_leaves"], info["mM"], info["mK"], info["mN"]
    Sg = _region(ws, info["off_S"], info["bytes_S"], torch.uint8, (2, L, mM, mK))
    Tg = _region(ws, info["off_T"], info["bytes_T"], torch.uint8, (2, L, mK, mN))
    ex = _region(ws, info["off_aux"] + AUX_EXPS, 2 * L * 4, torch.int32, (2, L))
    dims = (mM, mK, mN)
    ops = recursion.leaf_operands(A, B, ref_s, dr, arith="f32", leaf_dims=dims)
    gA, gB = precision.path_norms(ref_s, "A"), precision.path_norms(ref_s, "B")
    mA, mB = float(np.max(np.abs(A))), float(np.max(np.abs(B)))
    prods = []
    for l, (S, T) in enumerate(ops):
        eA = precision.leaf_exponent(mA, gA[l], target=448.0)
        eB = precision.leaf_exponent(mB, gB[l], target=448.0)
        assert (ex[0, l], ex[1, l]) == (eA, eB), l
        sh, sl = precision.split_e4m3_scaled(np.ldexp(S.astype(np.float64), eA))
        th, tl = precision.split_e4m3_scaled(np.ldexp(T.astype(np.float64), eB))
        np.testing.assert_array_equal(precision.decode_e4m3(Sg[0, l]), sh)
        np.testing.assert_array_equal(precision.decode_e4m3(Sg[1, l]), sl)
        np.testing.assert_array_equal(precision.decode_e4m3(Tg[0, l]), th)
        np.testing.assert_array_equal(precision.decode_e4m3(Tg[1, l]), tl)
        prods.append(np.ldexp(sh @ th + (sh @ tl + sl @ th) / 16.0, -(eA + eB)).astype(np.float32))
    plan.stage_leaf(ws)
    Pg = _region(ws, info["off_P"], info["bytes_P"], torch.float32, (L, mM, mN))
    for l in range(0, L, max(1, L // 7)):
        # The fp8 MFMA's internal accumulation is not the sequential f32 sum (its errors reach
        # about 2^-18 of the sum of |terms| at K = 64); a wrong lane layout or byte order would
        # give errors of the order of the values themselves.
        eA, eB = ex[0, l], ex[1, l]
        sh, sl = precision.split_e4m3_scaled(np.ldexp(ops[l][0].astype(np.float64), eA))
        th, tl = precision.split_e4m3_scaled(np.ldexp(ops[l][1].astype(np.float64), eB))
        bound = np.ldexp(np.abs(sh) @ np.abs(th) + (np.abs(sh) @ np.abs(tl) + np.abs(sl) @ np.abs(th)) / 16.0,
                         -(eA + eB)) * (mK + 2) * 2.0 ** -20
        assert (np.abs(Pg[l] - prods[l]) <= bound + 1e-30).all(), l
    emu = recursion.combine(prods, M, N, K, ref_s, dr, arith="f32", leaf_dims=dims)
    C = plan.matmul(Ad, Bd, seed=11).cpu().numpy()
    AB = A.astype(np.float64) @ B.astype(np.float64)
    e, e_emu = recursion.rel_err(C, AB), recursion.rel_err(emu, AB)
    _say("fp8c rel err %.3g, emulation %.3g" % (e, e_emu))
    assert e <= 1.1 * e_emu + 1e-6 and e < 5e-2


def test_results_are_deterministic_and_stream_ordered():
    _say("determinism")
    lib_s, _ = _schemes(["strassen"] * 3)
    plan = rbc.Plan(1024, 1024, 1024, lib_s, prec="f32")
    A = torch.randn(1024, 1024, device=DEV)
    B = torch.randn(1024, 1024, device=DEV)
    C1 = plan.matmul(A, B, seed=5).clone()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        C2 = plan.matmul(A, B, seed=5, workspace=torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=DEV))
    s.synchronize()
    assert torch.equal(C1, C2)
    C3 = plan.matmul(A, B, seed=6)
    assert not torch.equal(C1, C3)


@pytest.mark.parametrize("prec", ["f32", "f16s", "fp8c", "bf16x3"])
def test_tail_split_tiles_give_the_same_bits(prec):
    # N = 2048, Q = 2: 49 leaves of 512^2, 784 tiles of 128 -- more than one round of the resident
    # grid and not a whole number of rounds, so the last round runs as 64-tiles; the products must
    # be bitwise those of the same plan on 64-tiles only (same instruction, same k order).
    _say("tail split", prec)
    n = 2048
    lib_s, _ = _schemes(["strassen"] * 2)
    big = rbc.Plan(n, n, n, lib_s, prec=prec, leaf_tile=128)
    small = rbc.Plan(n, n, n, lib_s, prec=prec, leaf_tile=64)
    assert big.info["tile_m"] == 128 and small.info["tile_m"] == 64
    g = torch.Generator(device=DEV)
    g.manual_seed(9)
    A = torch.randn(n, n, device=DEV, generator=g)
    B = torch.randn(n, n, device=DEV, generator=g)
    C1 = big.matmul(A, B, seed=2)
    C2 = small.matmul(A, B, seed=2)
    torch.cuda.synchronize()
    assert torch.equal(C1, C2)


@pytest.mark.parametrize("names,M,K,N,tile", [
    (["strassen"] * 3, 4096, 4096, 4096, 0),
    (["strassen"] * 3, 1000, 600, 777, 64),
    (["strassen"] * 2, 300, 192, 500, 64),     # leaf K = 48: 64-tiles with K slabs of 16
    (["strassen"] * 2, 300, 200, 500, 128),
    (["laderman", "strassen"], 700, 500, 900, 64),
    (["strassen"] * 4, 1024, 1024, 1024, 0),
    (["strassen"] * 2, 300, 192, 500, 128),    # 128-tiles whose tail tiles take 16-k slabs
    (["strassen", "naive:2,3,2"], 260, 300, 170, 64),  # non-square deepest level, one term each
    (["naive:3,2,2", "naive:2,2,2"], 1000, 1000, 1000, 0),
    # coefficients other than +-1 at the deepest level: both terms rounded apart (U), and
    # a +-1 second coefficient after a scaled first one (V scaled by 1 keeps +-1)
    (["strassen", "scaled:0.75:1.25"], 1024, 1024, 1024, 128),
    (["strassen", "scaled:0.5:1"], 1000, 1000, 1000, 128),
])
def test_leaf_gather_same_bits(names, M, K, N, tile):
    # The leaf product that forms its operands while loading them (deepest level's gather
    # inside the leaf tile) must give C bitwise equal to the separate gather of every level.
    _say("leaf gather", names, M, K, N, tile)
    lib_s, _ = _schemes(names)
    plan = rbc.Plan(M, K, N, lib_s, prec="f32", leaf_tile=tile)
    assert plan.leaf_gather[1]  # available (whether it is on by default is the cost model's call)
    g = torch.Generator(device=DEV)
    g.manual_seed(M + K + N)
    A = torch.randn(M, K, device=DEV, generator=g)
    B = torch.randn(K, N, device=DEV, generator=g)
    for seed, mode in [(0, "full"), (5, "full"), (1, "signs"), (3, "none")]:
        plan.set_leaf_gather(True)
        C1 = plan.matmul(A, B, seed=seed, mode=mode)
        plan.set_leaf_gather(False)
        C2 = plan.matmul(A, B, seed=seed, mode=mode)
        torch.cuda.synchronize()
        assert torch.equal(C1, C2), (seed, mode, float((C1 - C2).abs().max()))
    assert plan.leaf_gather == (False, True)


@pytest.mark.parametrize("prec,names,M,K,N", [
    ("f32", ["strassen"] * 2, 300, 200, 500),
    ("f32", ["laderman", "strassen"], 700, 500, 900),
    ("f64", ["strassen"] * 2, 64, 64, 64),
    ("f16s", ["strassen"] * 2, 520, 260, 1030),
    ("fp8c", ["laderman"], 390, 700, 200),
    ("bf16x3", ["strassen"] * 2, 256, 192, 320),
])
def test_paired_gathers_same_bits(prec, names, M, K, N):
    # Without stage timing the A and B gathers of each level group share one launch (the grid
    # spans the larger side; the other side's extra blocks do nothing); with timing they run
    # apart.  C must be the same bits.
    _say("paired gathers", prec, names, M, K, N)
    lib_s, _ = _schemes(names)
    plan = rbc.Plan(M, K, N, lib_s, prec=prec)
    dt = torch.float64 if prec == "f64" else torch.float32
    g = torch.Generator(device=DEV)
    g.manual_seed(77)
    A = torch.randn(M, K, device=DEV, generator=g, dtype=dt)
    B = torch.randn(K, N, device=DEV, generator=g, dtype=dt)
    for seed in (0, 3):
        C1 = plan.matmul(A, B, seed=seed)
        plan.set_timing(True)
        C2 = plan.matmul(A, B, seed=seed)
        plan.set_timing(False)
        plan.timing_collect()
        torch.cuda.synchronize()
        assert torch.equal(C1, C2), (seed, float((C1 - C2).abs().max()))


@pytest.mark.parametrize("prec,n,q", [("f64", 64, 2), ("fp8c", 1024, 3), ("f16s", 512, 2), ("f32", 1024, 3)])
def test_fusion_choice_same_bits(prec, n, q):
    # One pass per level (the default for small products) or fused passes: the same
    # arithmetic per level, so the same bits.
    _say("fusion choice", prec, n, q)
    S = rbc.Scheme.builtin("strassen")
    a = rbc.Plan(n, n, n, [S] * q, prec=prec)
    m = rbc.Plan(n, n, n, [S] * q, prec=prec, fusion="max")
    dt = torch.float64 if prec == "f64" else torch.float32
    g = torch.Generator(device=DEV)
    g.manual_seed(n + q)
    A = torch.randn(n, n, device=DEV, generator=g, dtype=dt)
    B = torch.randn(n, n, device=DEV, generator=g, dtype=dt)
    for seed in (0, 9):
        C1 = a.matmul(A, B, seed=seed)
        C2 = m.matmul(A, B, seed=seed)
        torch.cuda.synchronize()
        assert torch.equal(C1, C2), (seed, float((C1 - C2).abs().max()))


# Leaf products of the 16-bit formats, element by element.  The plans only lay out the
# workspace: the test writes its own leaf operands (bf16 hi and lo planes from a split of
# f32 values; f16 values and per-leaf exponents), runs the leaf stage alone and compares
# every product (or every product on sampled rows) with the f64 product of the same bits.
# Tile counts: 161 leaves x 16 (128-tiles) = 2576 and x 64 (64-tiles) = 10304 are no
# whole number of rounds of any resident grid of 256 x (1..8) workgroups and exceed one
# round, so those launches run their last round as tiles of half the side.
LOWP_LEAF_CASES = [
    # (prec, schemes, M, K, N, tile, sampled rows or 0 for all)
    ("bf16x3", ["laderman", "strassen"], 3072, 384, 3072, 128, 0),
    ("bf16x3", ["laderman", "strassen"], 3072, 384, 3072, 64, 0),
    ("bf16x3", ["apa322:0.001"], 3072, 3072, 3072, 128, 24),   # the approximate-scheme leaves, 1024 x 1536 x 1536
    ("f16s", ["laderman", "strassen"], 3072, 384, 3072, 128, 0),
    ("f16s", ["laderman", "strassen"], 3072, 384, 3072, 64, 0),
    ("f16s", ["laderman", "strassen"], 1728, 192, 1728, 96, 0),
    ("f16s", ["laderman", "strassen"], 384, 384, 384, 32, 0),
]


@pytest.mark.parametrize("case", range(len(LOWP_LEAF_CASES)))
def test_lowp_leaf_products_elementwise(case):
    prec, names, M, K, N, tile, nrows = LOWP_LEAF_CASES[case]
    lib_s, _ = _schemes(names)
    plan = rbc.Plan(M, K, N, lib_s, prec=prec, leaf_tile=tile)
    info = plan.info
    L, m, k, n = info["n_leaves"], info["mM"], info["mK"], info["mN"]
    assert info["tile_m"] == tile
    _say("lowp leaf", prec, tile, "leaves", L, "leaf", (m, k, n), "tiles", L * (m // tile) * (n // tile))
    g = np.random.default_rng(100 + case)
    ws = torch.zeros(info["workspace_bytes"], dtype=torch.uint8, device=DEV)
    if prec == "bf16x3":
        S = g.standard_normal((L, m, k)).astype(np.float32)
        T = g.standard_normal((L, k, n)).astype(np.float32) * np.float32(3.0)
        planes = []
        for X in (S, T):
            hi, lo = precision.split_hi_lo(X, "bf16")
            planes.append((hi, lo))
            bits = np.stack([(hi.view(np.uint32) >> 16).astype(np.uint16), (lo.view(np.uint32) >> 16).astype(np.uint16)])
            off = info["off_S"] if X is S else info["off_T"]
            ws[off:off + bits.nbytes].copy_(torch.from_numpy(bits.view(np.uint8).reshape(-1)))
        (sh, sl), (th, tl) = planes
        passes = 3
    else:
        S16 = (g.standard_normal((L, m, k)) * 100.0).astype(np.float16)
        T16 = (g.standard_normal((L, k, n)) * 0.01).astype(np.float16)
        ex = g.integers(-6, 7, size=(2, L)).astype(np.int32)
        for X, off in ((S16, info["off_S"]), (T16, info["off_T"])):
            ws[off:off + X.nbytes].copy_(torch.from_numpy(X.view(np.uint8).reshape(-1)))
        a = info["off_aux"] + AUX_EXPS
        ws[a:a + ex.nbytes].copy_(torch.from_numpy(ex.view(np.uint8).reshape(-1)))
        passes = 1
    plan.stage_leaf(ws)
    torch.cuda.synchronize()
    P = _region(ws, info["off_P"], info["bytes_P"], torch.float32, (L, m, n))
    rows = np.arange(m) if not nrows else np.unique(np.concatenate(
        [[0, 1, m // 2, m - 1], g.integers(0, m, size=nrows)]))
    gK = passes * k * 2.0 ** -24 / (1 - passes * k * 2.0 ** -24)
    worst = 0.0
    for l in range(L):
        if prec == "bf16x3":
            a_h, a_l = sh[l][rows].astype(np.float64), sl[l][rows].astype(np.float64)
            b_h, b_l = th[l].astype(np.float64), tl[l].astype(np.float64)
            ref = a_h @ b_h + a_h @ b_l + a_l @ b_h
            mag = np.abs(a_h) @ np.abs(b_h) + np.abs(a_h) @ np.abs(b_l) + np.abs(a_l) @ np.abs(b_h)
        else:
            sc = -(int(ex[0, l]) + int(ex[1, l]))
            a16, b16 = S16[l][rows].astype(np.float64), T16[l].astype(np.float64)
            ref = np.ldexp(a16 @ b16, sc)
            mag = np.ldexp(np.abs(a16) @ np.abs(b16), sc)
        bound = gK * mag + 2.0 ** -24 * np.abs(ref) + 1e-38
        d = np.abs(P[l][rows].astype(np.float64) - ref)
        worst = max(worst, float(np.max(d / bound)))
        assert np.all(d <= bound), (l, float(np.max(d / bound)))
    _say("lowp leaf %s tile %d: max |P - ref| / bound = %.3g" % (prec, tile, worst))
