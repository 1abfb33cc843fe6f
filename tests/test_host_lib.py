"""Host-side checks of librbc on the CPU: symbols, schemes, draws, fold, plans, errors.

No device compute is issued here.  The oracle is the reference for every value.
"""

import ctypes
import math
import os
import re

import numpy as np
import pytest

import paper_1905_07439_amd as rbc
from paper_1905_07439_amd import _lib
from oracle import draws as odraws
from oracle import recursion
from oracle import schemes as oschemes
from oracle import tensors as otensors

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    text = open(os.path.join(ROOT, "include", "rbc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rbc_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    L = rbc.lib()
    names = _header_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
        assert n in _lib.SIGNATURES, n
    assert L.rbc_abi_version() == 2


@pytest.mark.parametrize("name,builder", [("strassen", oschemes.strassen), ("laderman", oschemes.laderman)])
def test_builtin_schemes_match_oracle(name, builder):
    s = rbc.Scheme.builtin(name)
    U, V, W = builder()
    Ul, Vl, Wl = s.tensors()
    np.testing.assert_array_equal(Ul, U)
    np.testing.assert_array_equal(Vl, V)
    np.testing.assert_array_equal(Wl, W)
    i = s.info()
    assert i["tau"] == 0.0 and i["kappa"] == 0.0
    assert i["q"] == pytest.approx(otensors.q_uvw(U, V, W), rel=1e-14)
    assert i["ynorm"] == pytest.approx(otensors.ynorm(U, V, W), rel=1e-14)


@pytest.mark.parametrize("lam", [1.0, 0.1, 1e-3, 2.0 ** -20])
@pytest.mark.parametrize("name,dims", [("apa322", (3, 2, 2)), ("apa223", (2, 2, 3)), ("apa232", (2, 3, 2))])
def test_apa_builtins_match_oracle(name, dims, lam):
    s = rbc.Scheme.builtin("%s:%r" % (name, lam))
    for got, want in zip(s.tensors(), getattr(oschemes, name)(lam)):
        np.testing.assert_array_equal(got, want)
    i = s.info()
    assert (i["b1"], i["b2"], i["b3"], i["R"]) == dims + (10,)
    U, V, W = getattr(oschemes, name)(lam)
    assert i["tau"] == pytest.approx(otensors.tau(U, V, W), rel=1e-12)
    assert i["kappa"] == pytest.approx(otensors.kappa(U, V, W), abs=1e-12)
    for bad in (0.0, -0.1, 1.5, float("nan"), float("inf")):
        with pytest.raises(rbc.RbcError) as e:
            rbc.Scheme.builtin(name, bad)
        assert e.value.status == _lib.RBC_EINVAL
    for bad in ("", "1e-3x"):  # the binding's name parsing
        with pytest.raises(ValueError):
            rbc.Scheme.builtin("%s:%s" % (name, bad))
    # three levels at N = 3072: b^3 blocks per dimension, zero padding to whole leaves
    p = rbc.Plan(3072, 3072, 3072, [s] * 3, prec="bf16x3")
    assert p.info["n_leaves"] == 1000
    b1, b2, b3 = dims
    assert p.info["mM"] * b1 ** 3 >= 3072 and p.info["mK"] * b2 ** 3 >= 3072 and p.info["mN"] * b3 ** 3 >= 3072


def test_naive_builtin_and_rank_one_scheme():
    s = rbc.Scheme.builtin("naive:2,3,2")
    U, V, W = oschemes.naive(2, 3, 2)
    np.testing.assert_array_equal(s.tensors()[0], U)
    one = rbc.Scheme.from_tensors(*oschemes.rank_one_all_ones(2), residual_tol=math.inf)
    assert one.info()["kappa"] == 0.0
    assert one.info()["tau"] == pytest.approx(math.sqrt(56.0), rel=1e-15)


@pytest.mark.parametrize("base", ["strassen", "laderman"])
def test_perturbed_scheme_matches_oracle_recipe_and_kappa(base):
    # The library's seeded perturbation (Philox words, Box-Muller normals, partial
    # Fisher-Yates picks) and the oracle's, written separately, agree to the bit.
    for sigma, seed in [(1e-3, 0), (1e-1, 7), (1e-4, 42), (0.5, 2 ** 64 - 1), (1e-2, 12345)]:
        s = rbc.Scheme.builtin("perturbed_" + base, sigma, seed)
        ref = oschemes.perturbed(*getattr(oschemes, base)(), sigma, seed)
        for a, b in zip(s.tensors(), ref):
            np.testing.assert_array_equal(a, b)
        i = s.info()
        assert i["tau"] == pytest.approx(otensors.tau(*ref), rel=1e-12)
        assert i["kappa"] == pytest.approx(otensors.kappa(*ref), rel=1e-12, abs=1e-18)


def test_scheme_validation_errors():
    U, V, W = oschemes.strassen()
    W2 = W.copy()
    W2[0, 0, 0] = 0
    with pytest.raises(rbc.RbcError) as e:
        rbc.Scheme.from_tensors(U, V, W2)
    assert e.value.status == _lib.RBC_ESCHEME
    # kappa = 1 is rejected (Definition 2 needs kappa != 1)
    with pytest.raises(rbc.RbcError) as e:
        rbc.Scheme.from_tensors(U * 0.0, V, W, residual_tol=math.inf)
    assert e.value.status == _lib.RBC_ESCHEME
    with pytest.raises(rbc.RbcError) as e:
        rbc.Scheme.from_tensors(np.zeros((5, 2, 1)), np.zeros((2, 2, 1)), np.zeros((5, 2, 1)))
    assert e.value.status == _lib.RBC_EINVAL
    with pytest.raises(rbc.RbcError):
        rbc.Scheme.builtin("winograd")
    # exact schemes take no lambda or aux seed; the approximate ones need lambda in range
    for name, lam, seed in [("strassen", 0.1, 0), ("laderman", 0.0, 3), ("apa322", 0.0, 0), ("apa223", 2.0, 0),
                            ("perturbed_strassen", -1e-3, 0), ("perturbed_strassen", float("nan"), 0),
                            ("perturbed_winograd", 1e-3, 0)]:
        with pytest.raises(rbc.RbcError) as e:
            rbc.Scheme.builtin(name, lam, seed)
        assert e.value.status == _lib.RBC_EINVAL, (name, lam, seed)


@pytest.mark.parametrize("b", [(2, 2, 2), (3, 3, 3), (3, 2, 2), (1, 4, 2)])
@pytest.mark.parametrize("mode", ["full", "signs", "perms", "none"])
def test_draws_match_oracle(b, mode):
    for seed in list(range(40)) + [2 ** 63 + 5, 2 ** 64 - 1]:
        for depth in range(4):
            s, p = rbc.draw(seed, depth, *b, mode=mode)
            ref = odraws.draw(seed, depth, *b, mode=mode)
            np.testing.assert_array_equal(s, np.concatenate(ref[:3]))
            np.testing.assert_array_equal(p, np.concatenate(ref[3:]))


def test_fold_matches_oracle_bitwise():
    base = oschemes.perturbed(*oschemes.laderman(), 1e-2, 3)
    s = rbc.Scheme.from_tensors(*base, residual_tol=math.inf)
    for seed in range(10):
        sg, pm = rbc.draw(seed, 1, 3, 3, 3)
        ref_draw = odraws.draw(seed, 1, 3, 3, 3)
        for ks in (True, False):
            c = 1.0 / (1.0 - float(otensors.kappa(*base))) if ks else 1.0
            ref = odraws.fold(*base, ref_draw, c)
            got = rbc.fold(s, sg, pm, kappa_scale=ks)
            for a, r in zip(got, ref):
                np.testing.assert_array_equal(a, r)


def test_plan_geometry():
    S = rbc.Scheme.builtin("strassen")
    p = rbc.Plan(4096, 4096, 4096, [S, S, S], prec="f32")
    i = p.info
    assert (i["mM"], i["mK"], i["mN"]) == (512, 512, 512)
    assert i["n_leaves"] == 343 and i["tile_m"] == 128
    # fused groups of at most two levels by default, formed from the bottom: [0] [1, 2]
    assert i["n_groups"] == (1 if os.environ.get("RBC_MAX_FUSED_LEVELS") == "3" else 2)
    assert i["bytes_S"] == 343 * 512 * 512 * 4
    assert i["workspace_bytes"] >= 3 * 343 * 512 * 512 * 4
    q = rbc.Plan(64, 64, 64, [S, S], prec="f64")
    assert (q.info["mM"], q.info["n_leaves"], q.info["tile_m"]) == (16, 49, 16)
    # ragged sizes pad up to the leaf tile; Laderman then Strassen is two groups
    L = rbc.Scheme.builtin("laderman")
    r = rbc.Plan(1000, 777, 333, [L, S], prec="f32", leaf_tile=64)
    i = r.info
    assert i["n_groups"] == 2 and i["n_leaves"] == 23 * 7
    assert i["mM"] == 192 and i["Mp"] == 192 * 6 >= 1000
    assert i["mK"] % 16 == 0 and i["mK"] * 6 >= 777
    assert i["mN"] == 64 and i["Np"] >= 333
    # five Strassen levels: [0] [1, 2] [3, 4]
    f = rbc.Plan(2048, 2048, 2048, [S] * 5, prec="f32", leaf_tile=64)
    assert f.info["n_leaves"] == 7 ** 5
    assert f.info["n_groups"] == (2 if os.environ.get("RBC_MAX_FUSED_LEVELS") == "3" else 3)
    z = rbc.Plan(100, 50, 30, [], prec="f32")
    assert z.info["n_leaves"] == 1 and z.info["mM"] == 128 and z.info["n_groups"] == 1
    # the plain product's one group copies A in and C out: its bytes are counted
    tz = z.traffic()
    assert tz["gather_A"] == 100 * 50 * 4 + 128 * 64 * 4 and tz["scatter"] == 128 * 64 * 4 + 100 * 30 * 4


def test_exact_block_plans():
    # leaf tile -1: padding only to a multiple of the block counts (the oracle's default
    # padding), leaves of any size; f32 and f64 only
    S = rbc.Scheme.builtin("strassen")
    L = rbc.Scheme.builtin("laderman")
    p = rbc.Plan(320, 320, 320, [S] * 5, prec="f32", leaf_tile=-1)
    i = p.info
    assert (i["Mp"], i["mM"], i["mK"], i["mN"], i["tile_m"]) == (320, 10, 10, 10, 1)
    assert p.leaf_gather == (False, False)
    q = rbc.Plan(100, 90, 110, [L, S], prec="f64", leaf_tile=-1)
    assert (q.info["mM"], q.info["mK"], q.info["mN"]) == (17, 15, 19)
    assert (q.info["Mp"], q.info["Kp"], q.info["Np"]) == (102, 90, 114)
    assert (q.info["mM"], q.info["mK"], q.info["mN"]) == tuple(
        d // b for d, b in zip(recursion.padded_dims(100, 90, 110, [oschemes.laderman(), oschemes.strassen()]), (6, 6, 6)))
    for prec in ("bf16x3", "f16s", "fp8c"):
        with pytest.raises(rbc.RbcError):
            rbc.Plan(64, 64, 64, [S], prec=prec, leaf_tile=-1)


def test_fusion_needs_parallel_work():
    # Two levels share one combination pass only when the pass has at least 2^18 elements of
    # parallel work (top blocks entering it x bottom-block elements); smaller products take one
    # pass per level.
    if os.environ.get("RBC_MAX_FUSED_LEVELS"):
        pytest.skip("the environment fixes the fusion depth")
    S = rbc.Scheme.builtin("strassen")
    cases = [("f64", 64, 2, 2), ("f32", 1024, 2, 2), ("f32", 1024, 3, 3), ("fp8c", 1024, 2, 2),
             ("f32", 2048, 2, 1), ("fp8c", 2048, 2, 1), ("f32", 2048, 3, 2), ("f32", 4096, 3, 2), ("f32", 4096, 2, 1)]
    for prec, n, q, groups in cases:
        assert rbc.Plan(n, n, n, [S] * q, prec=prec).info["n_groups"] == groups, (prec, n, q)


def test_scatter_passes_take_three_levels():
    # Scatters fuse up to three Strassen-shaped levels per pass under the same
    # parallel-work rule; the gathers (and the batch engine) keep two.
    if os.environ.get("RBC_MAX_FUSED_LEVELS"):
        pytest.skip("the environment fixes the fusion depth")
    S = rbc.Scheme.builtin("strassen")
    cases = [("f32", 4096, 3, 2, 1), ("f64", 4096, 3, 2, 1), ("f32", 4096, 4, 2, 2), ("f32", 2048, 3, 2, 2),
             ("f32", 1024, 3, 3, 3), ("f32", 8192, 3, 2, 1), ("fp8c", 4096, 4, 2, 2), ("f32", 4096, 2, 1, 1)]
    for prec, n, q, groups, sgroups in cases:
        i = rbc.Plan(n, n, n, [S] * q, prec=prec).info
        assert (i["n_groups"], i["n_scatter_groups"]) == (groups, sgroups), (prec, n, q)
    L = rbc.Scheme.builtin("laderman")
    i = rbc.Plan(4096, 4096, 4096, [L, S, S, S], prec="f32").info
    assert i["n_scatter_groups"] == 2
    # the workspace does not grow: boundary buffers are shared with the gathers' groups
    os.environ["RBC_MAX_FUSED_LEVELS"] = "2"
    try:
        two = rbc.Plan(4096, 4096, 4096, [S] * 4, prec="f32").info
    finally:
        del os.environ["RBC_MAX_FUSED_LEVELS"]
    assert rbc.Plan(4096, 4096, 4096, [S] * 4, prec="f32").info["workspace_bytes"] == two["workspace_bytes"]


def test_fusion_max_option():
    if os.environ.get("RBC_MAX_FUSED_LEVELS"):
        pytest.skip("the environment fixes the fusion depth")
    S = rbc.Scheme.builtin("strassen")
    a = rbc.Plan(1024, 1024, 1024, [S] * 3, prec="fp8c")
    m = rbc.Plan(1024, 1024, 1024, [S] * 3, prec="fp8c", fusion="max")
    assert a.info["n_groups"] == 3 and m.info["n_groups"] == 2
    assert m.info["n_leaves"] == a.info["n_leaves"] and m.info["mM"] == a.info["mM"]
    # fewer group boundaries: fewer intermediate bytes
    assert m.traffic()["gather_A"] < a.traffic()["gather_A"]
    with pytest.raises(ValueError):
        rbc.Plan(64, 64, 64, [S], fusion="some")
    L = rbc.lib()
    assert L.rbc_plan_set_fusion(a._h, 1) == 0 and L.rbc_plan_set_fusion(a._h, 0) == 0


def test_f16s_plan_geometry():
    L = rbc.Scheme.builtin("laderman")
    S = rbc.Scheme.builtin("strassen")
    p = rbc.Plan(480, 480, 480, [L, S], prec="f16s")
    i = p.info
    # leaf 80: pads to 96 with the least padded area (tiles 96 and 32 tie; the larger
    # wins), K to a multiple of 32
    assert (i["mM"], i["mK"], i["mN"], i["tile_m"]) == (96, 96, 96, 96)
    assert rbc.Plan(480, 480, 480, [L, S], prec="f16s", leaf_tile=32).info["mM"] == 96
    with pytest.raises(rbc.RbcError):
        rbc.Plan(480, 480, 480, [L, S], prec="f16s", leaf_tile=48)
    assert i["bytes_S"] == 161 * 96 * 96 * 2
    assert i["bytes_aux"] == 2 * 1024 * 4 + 2 * 161 * 4 and i["off_aux"] >= i["off_P"] + i["bytes_P"]
    q = rbc.Plan(768, 768, 768, [L, S], prec="f16s")
    assert q.info["tile_m"] == 128 and q.info["mM"] == 128


def test_fp8c_plan_geometry():
    S = rbc.Scheme.builtin("strassen")
    p = rbc.Plan(300, 260, 200, [S, S], prec="fp8c")
    i = p.info
    # leaves 75 x 65 x 50: M, N to the tile with the least padded area (32), K to the
    # 64-byte slab; two one-byte planes per operand element
    assert (i["mM"], i["mK"], i["mN"], i["tile_m"], i["tile_k"]) == (96, 128, 64, 32, 64)
    assert i["bytes_S"] == 49 * 96 * 128 * 2 and i["bytes_T"] == 49 * 128 * 64 * 2
    assert i["bytes_aux"] == 2 * 1024 * 4 + 2 * 49 * 4
    t = p.traffic()
    assert t["leaf"] == 49 * (96 * 128 * 2 + 128 * 64 * 2 + 96 * 64 * 4)


def test_leaf_gather_availability_and_traffic():
    # Available for f32 plans of two or more levels whose deepest scheme has at most two
    # nonzero coefficients per product in U and in V (Strassen, not Laderman), on by default.
    S = rbc.Scheme.builtin("strassen")
    L = rbc.Scheme.builtin("laderman")
    env = os.environ.get("RBC_LEAF_GATHER")
    p = rbc.Plan(4096, 4096, 4096, [S, S, S], prec="f32")
    assert p.leaf_gather == (env != "0", True)
    # the cost model: off for two Strassen levels at N = 4096 (the gathers save little)
    assert rbc.Plan(4096, 4096, 4096, [S, S], prec="f32").leaf_gather == (env == "1", True)
    assert rbc.Plan(4096, 4096, 4096, [S] * 4, prec="f32").leaf_gather == (env != "0", True)
    assert rbc.Plan(700, 500, 900, [L, S], prec="f32").leaf_gather[1]
    for q in (rbc.Plan(4096, 4096, 4096, [S], prec="f32"), rbc.Plan(900, 900, 900, [S, L], prec="f32"),
              rbc.Plan(1024, 1024, 1024, [S, S], prec="f16s"), rbc.Plan(1024, 1024, 1024, [S, S], prec="fp8c"),
              rbc.Plan(256, 256, 256, [S, S], prec="f64"), rbc.Plan(256, 256, 256, [S, S], prec="bf16x3")):
        assert q.leaf_gather == (False, False)
        with pytest.raises(rbc.RbcError) as e:
            q.set_leaf_gather(True)
        assert e.value.status == _lib.RBC_EUNSUPPORTED
        q.set_leaf_gather(False)
    # Traffic: with the leaf gather the gathers stop at the 49 parents of 1024^2 and the
    # leaf stage reads each parent once; the scatter is unchanged.
    p.set_leaf_gather(False)
    t0 = p.traffic()
    p.set_leaf_gather(True)
    t1 = p.traffic()
    n, e = 4096, 4
    assert t0["gather_A"] == n * n * e + 7 * 2048 * 2048 * e + 7 * 2048 * 2048 * e + 343 * 512 * 512 * e
    assert t1["gather_A"] == n * n * e + 49 * 1024 * 1024 * e
    assert t1["leaf"] == 2 * 49 * 1024 * 1024 * e + 343 * 512 * 512 * e
    assert t0["scatter"] == t1["scatter"]
    assert p.workspace_bytes == rbc.Plan(4096, 4096, 4096, [S, S, S], prec="f32").workspace_bytes


def test_plan_errors():
    S = rbc.Scheme.builtin("strassen")
    with pytest.raises(rbc.RbcError) as e:
        rbc.Plan(0, 4, 4, [S])
    assert e.value.status == _lib.RBC_EINVAL
    with pytest.raises(rbc.RbcError) as e:
        rbc.Plan(64, 64, 64, [S], prec="f32", leaf_tile=96)
    assert e.value.status == _lib.RBC_EUNSUPPORTED
    with pytest.raises(rbc.RbcError):
        rbc.Plan(64, 64, 64, [S] * 9)


def test_matmul_argument_errors_are_synchronous():
    # Argument checks fire before any device call, so they run without a GPU.
    S = rbc.Scheme.builtin("strassen")
    p = rbc.Plan(64, 64, 64, [S], prec="f32")
    L = rbc.lib()
    null = ctypes.c_void_p()
    st = L.rbc_matmul(p._h, null, 64, null, 64, null, 64, 0, 0, 1, null, 0, null)
    assert st == _lib.RBC_EINVAL
    fake = ctypes.c_void_p(0x1000)
    st = L.rbc_matmul(p._h, fake, 64, fake, 64, fake, 64, 0, 0, 1, ctypes.c_void_p(0x1010), 10, null)
    assert st == _lib.RBC_EINVAL  # workspace not 256-byte aligned
    st = L.rbc_matmul(p._h, fake, 64, fake, 64, fake, 64, 0, 0, 1, ctypes.c_void_p(0x100000), 10, null)
    assert st == _lib.RBC_ENOMEM
    st = L.rbc_matmul(p._h, fake, 32, fake, 64, fake, 64, 0, 0, 1, ctypes.c_void_p(0x100000), 1 << 30, null)
    assert st == _lib.RBC_EINVAL
    st = L.rbc_matmul(p._h, fake, 64, fake, 64, fake, 64, 0, 7, 1, ctypes.c_void_p(0x100000), 1 << 30, null)
    assert st == _lib.RBC_EINVAL
    bad_s = (ctypes.c_int32 * 6)(1, 1, 2, 1, 1, 1)
    ok_p = (ctypes.c_int32 * 6)(0, 1, 0, 1, 0, 1)
    st = L.rbc_matmul_draws(p._h, fake, 64, fake, 64, fake, 64, bad_s, ok_p, 1, ctypes.c_void_p(0x100000),
                            1 << 30, null)
    assert st == _lib.RBC_EINVAL
    assert b"draw" in L.rbc_last_error()


def test_peak_argument_errors_are_synchronous():
    # Argument checks of the measured-ceiling calls fire before any device call.
    L = rbc.lib()
    null = ctypes.c_void_p()
    assert L.rbc_peak_copy(null, null, 16, null) == _lib.RBC_EINVAL
    fake = ctypes.c_void_p(0x1000)
    assert L.rbc_peak_copy(fake, ctypes.c_void_p(0x1008), 16, null) == _lib.RBC_EINVAL
    assert L.rbc_peak_copy(fake, fake, 15, null) == _lib.RBC_EINVAL
    fl = ctypes.c_double()
    assert L.rbc_peak_mfma(0, 0, 10, fake, ctypes.byref(fl), null) == _lib.RBC_EINVAL
    assert L.rbc_peak_mfma(99, 1, 10, fake, ctypes.byref(fl), null) == _lib.RBC_EINVAL
    assert b"kind" in L.rbc_last_error()


def test_apa_ebc_weights_match_the_oracle():
    # The library takes the Lagrange route, the oracle solves the Vandermonde system.
    from oracle import schemes as osch
    for eps in ([0.1 * k for k in range(1, 8)], [0.5], [0.03, 0.2], [2.0 ** -5, 0.3, 0.11, 0.7]):
        np.testing.assert_allclose(rbc.apa_ebc_weights(eps), osch.apa_ebc_weights(eps), rtol=1e-10, atol=1e-10)
    for bad in ([0.1, 0.1], [], [0.0, 0.2], [float("nan")], [0.01] * 40):
        with pytest.raises(Exception):
            rbc.apa_ebc_weights(bad)
