"""GPU checks of the batch engine (one persistent launch for many products).

Every product of a batch must equal, bit for bit, the same product run alone
by Plan.matmul (the stand-alone path, itself checked against the oracle in
test_gpu_parity): the batch runs the same arithmetic in the same order.
Exact schemes on small integers must also give the exact product, which
checks the batch against the plain definition independently of the
stand-alone path, and the reduced-precision products stay within the stated
multiple of the oracle's emulation error.
"""

import sys

import numpy as np
import pytest
import torch

import paper_1905_07439_amd as rbc
import workloads
from oracle import precision, recursion

from test_gpu_parity import _level_draws, _schemes as _oracle_schemes

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def setup_module(module):
    assert torch.cuda.is_available(), "GPU tests need a GPU"


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


_PLANS = {}


def _scheme(name):
    if name.startswith("pert:"):  # perturbed Strassen, pert:<sigma>:<seed>
        _, sigma, seed = name.split(":")
        return rbc.Scheme.builtin("perturbed_strassen", float(sigma), int(seed))
    return rbc.Scheme.builtin(name)


def _plan(n, names, prec):
    key = (n, tuple(names), prec)
    if key not in _PLANS:
        _PLANS[key] = rbc.Plan(n, n, n, [_scheme(s) for s in names], prec)
    return _PLANS[key]


def _operands(n, seed, kind):
    if kind == "int":
        A = workloads.integers((n, n), 4000 + seed)
        B = workloads.integers((n, n), 5000 + seed)
    else:  # entries N(0,1) times 10^U(-3,3) per matrix
        A = workloads.scaled_gaussian((n, n), 4000 + seed)
        B = workloads.scaled_gaussian((n, n), 5000 + seed)
    return (torch.from_numpy(np.ascontiguousarray(A, np.float32)).to(DEV),
            torch.from_numpy(np.ascontiguousarray(B, np.float32)).to(DEV))


F32_SPECS = [(("strassen", "strassen"), 256), (("laderman",), 192), (("laderman", "strassen"), 384),
             (("strassen", "strassen", "strassen"), 512), (("strassen",), 320)]
F16S_SPECS = [(("laderman",), 192), (("laderman",), 288), (("laderman", "strassen"), 480),
              (("laderman", "strassen", "strassen"), 768), (("laderman", "strassen", "strassen"), 864),
              (("laderman", "strassen", "strassen", "strassen"), 1536)]
FP8C_SPECS = [(("strassen",), 128), (("laderman",), 192), (("pert:0.001:42", "pert:0.001:42"), 512),
              (("laderman", "strassen"), 480), (("strassen", "strassen", "strassen"), 1024),
              (("strassen", "strassen"), 320)]
MODES = ["full", "signs", "perms", "none"]


def _build(prec, specs, kind, reps=1, **opt):
    items = []
    b = rbc.Batch(**opt)
    for r in range(reps):
        for i, (names, n) in enumerate(specs):
            seed = r * len(specs) + i
            plan = _plan(n, names, prec)
            A, B = _operands(n, seed, kind)
            mode = MODES[seed % len(MODES)]
            _, C = b.add(plan, A, B, seed=seed, mode=mode)
            items.append((plan, A, B, seed, mode, C))
    return b, items


def _alone(items):
    out = []
    for plan, A, B, seed, mode, _ in items:
        out.append(plan.matmul(A, B, seed=seed, mode=mode).clone())
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("engine", ["persistent", "persistent-depth", "levels"])
@pytest.mark.parametrize("prec,specs", [("f32", F32_SPECS), ("f16s", F16S_SPECS), ("fp8c", FP8C_SPECS)])
def test_batch_equals_alone_bitwise(prec, specs, engine):
    opt = {"persistent": {}, "persistent-depth": {"order": "depth"}, "levels": {"mode": "levels"}}[engine]
    b, items = _build(prec, specs, "gauss", **opt)
    _say("batch", prec, b.info())
    b.prepare()
    b.launch()
    b.check()
    ref = _alone(items)
    for (plan, A, B, seed, mode, C), R in zip(items, ref):
        _say("  n=%d seed=%d mode=%s" % (A.shape[0], seed, mode))
        assert torch.isfinite(C).all()
        assert torch.equal(C, R), (A.shape[0], seed, mode, (C - R).abs().max().item())


def _emulation(prec, A, B, ref_s, dr, dims, kappa_scale):
    """The oracle's emulation of one reduced-precision product: f32 combinations, the
    per-leaf power-of-two scales, f16 leaves (f16s) or e4m3 hi + lo leaves with one
    correction product (fp8c) multiplied exactly, then the f32 recombination."""
    M, N, K = A.shape[0], B.shape[1], A.shape[1]
    ops = recursion.leaf_operands(A, B, ref_s, dr, kappa_scale=kappa_scale, arith="f32", leaf_dims=dims)
    gA, gB = precision.path_norms(ref_s, "A"), precision.path_norms(ref_s, "B")
    mA, mB = float(np.max(np.abs(A))), float(np.max(np.abs(B)))
    prods = []
    for l, (S, T) in enumerate(ops):
        if prec == "f16s":
            eA, eB = precision.leaf_exponent(mA, gA[l]), precision.leaf_exponent(mB, gB[l])
            S16 = np.ldexp(S, eA).astype(np.float16).astype(np.float64)
            T16 = np.ldexp(T, eB).astype(np.float16).astype(np.float64)
            prods.append(np.ldexp(S16 @ T16, -(eA + eB)).astype(np.float32))
        else:
            eA = precision.leaf_exponent(mA, gA[l], target=448.0)
            eB = precision.leaf_exponent(mB, gB[l], target=448.0)
            sh, sl = precision.split_e4m3_scaled(np.ldexp(S.astype(np.float64), eA))
            th, tl = precision.split_e4m3_scaled(np.ldexp(T.astype(np.float64), eB))
            prods.append(np.ldexp(sh @ th + (sh @ tl + sl @ th) / 16.0, -(eA + eB)).astype(np.float32))
    return recursion.combine(prods, M, N, K, ref_s, dr, kappa_scale=kappa_scale, arith="f32", leaf_dims=dims)


@pytest.mark.parametrize("prec,specs", [("f16s", F16S_SPECS[:3]), ("fp8c", FP8C_SPECS[:4])])
def test_batch_errors_within_emulation(prec, specs):
    # The stated gates of the batched (f16 leaves) and served (e4m3 leaves) configurations:
    # each product's relative Frobenius error against A B at most 4x that of the oracle's
    # emulation of the same precision, on the same draws, for inputs of the batched
    # configuration's recipe (N(0,1) times 10^U(-3,3) per matrix).
    b, items = _build(prec, specs, "gauss")
    b.prepare()
    b.launch()
    b.check()
    for (plan, A, B, seed, mode, C), (names, n) in zip(items, specs):
        _, ref_s = _oracle_schemes(list(names))
        _, _, dr = _level_draws(plan, ref_s, seed, mode)
        info = plan.info
        An, Bn = A.cpu().numpy(), B.cpu().numpy()
        emu = _emulation(prec, An, Bn, ref_s, dr, (info["mM"], info["mK"], info["mN"]), mode != "none")
        AB = An.astype(np.float64) @ Bn.astype(np.float64)
        e, e_emu = recursion.rel_err(C.cpu().numpy(), AB), recursion.rel_err(emu, AB)
        _say("  %s n=%d %s seed=%d mode=%s: rel err %.3g, emulation %.3g" % (prec, n, names, seed, mode, e, e_emu))
        assert e <= 4 * e_emu, (n, names, seed, mode, e, e_emu)


def test_batch_f32_integers_exact():
    b, items = _build("f32", F32_SPECS, "int")
    b.prepare()
    b.launch()
    b.check()
    for plan, A, B, seed, mode, C in items:
        exact = (A.double().cpu() @ B.double().cpu())
        assert torch.equal(C.double().cpu(), exact), (A.shape[0], seed)


def test_batch_options_ring_and_graph_replays():
    """Window, task size and a workspace ring change the schedule, not one bit of any result;
    graph replays, with other work between them, repeat the eager result."""
    base, items = _build("f16s", F16S_SPECS, "gauss", reps=2)
    base.prepare()
    base.launch()
    base.check()
    want = [it[5].clone() for it in items]
    biggest = max(it[0].workspace_bytes for it in items)
    for opt in (dict(window=1), dict(window=8, task_bytes=1 << 16),
                dict(item_budget=int(biggest * 1.6), window=3), dict(mode="levels"),
                dict(mode="levels", item_budget=int(biggest * 1.6)),
                dict(order="depth", item_budget=int(biggest * 1.6), task_bytes=1 << 18)):
        b, its = _build("f16s", F16S_SPECS, "gauss", reps=2, **opt)
        _say("options", opt, b.info())
        b.prepare()
        b.launch()
        b.check()
        for it, w in zip(its, want):
            assert torch.equal(it[5], w), opt
    s = torch.cuda.Stream()
    for engine in ("persistent", "levels"):
        b, its = _build("f16s", F16S_SPECS, "gauss", reps=1, item_budget=int(biggest * 1.6), mode=engine)
        with torch.cuda.stream(s):
            b.prepare(stream=s)
        for rep in range(3):
            for it in its:
                it[5].fill_(float("nan"))
            x = torch.randn(1024, 1024, device=DEV)
            (x @ x).sum().item()  # unrelated eager work between replays
            torch.cuda.synchronize()
            b.launch(graph=True, stream=s)
            b.check(stream=s)
            for it, w in zip(its, want):
                assert torch.equal(it[5], w), (engine, rep)


@pytest.mark.parametrize("prec,specs", [("f32", F32_SPECS), ("f16s", F16S_SPECS)])
def test_batch_signals_publish_written_data(prec, specs):
    """A counter moves only once its task's writes have left the producer's L2: with the stage
    buffers filled with NaN bytes before every run, the smallest tasks (the most signals, the
    most consumers on other XCDs) still give the bits of the products run alone."""
    b, items = _build(prec, specs, "gauss", task_bytes=1 << 16, window=8)
    ws = b.prepare()
    ctl = b.info()["control_bytes"]
    _say("signals", prec, b.info())
    ref = _alone(items)
    for rep in range(3):
        ws[ctl:].fill_(0xFF)
        for it in items:
            it[5].fill_(float("nan"))
        b.launch()
        b.check()
        for (plan, A, B, seed, mode, C), R in zip(items, ref):
            assert torch.equal(C, R), (prec, rep, A.shape[0], seed, mode)


def test_batch_reruns_and_check():
    b, items = _build("f32", F32_SPECS[:2], "gauss")
    b.prepare()
    for _ in range(3):
        b.launch()
    b.check()
    ref = _alone(items)
    for it, R in zip(items, ref):
        assert torch.equal(it[5], R)
