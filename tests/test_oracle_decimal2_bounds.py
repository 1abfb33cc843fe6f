"""Example 7 (2-digit arithmetic) and the bound helpers (Props. 8-9, Example 13)."""

import json
import os

import numpy as np
import pytest

from oracle import bounds, decimal2, draws, expectation, recursion, schemes, tensors
import workloads


def _example7(golden_dir):
    with open(os.path.join(golden_dir, "example7.json")) as f:
        return json.load(f)


def test_example7_deterministic_errors(golden_dir):
    g = _example7(golden_dir)
    A = np.array(g["A"])
    B = np.array(g["B"])
    U, V, W = [T.astype(np.float64) for T in schemes.strassen()]
    err = np.linalg.norm(decimal2.bc_2digit(U, V, W, A, B) - A @ B)
    assert err == pytest.approx(g["printed"]["g_error"], rel=0.02)
    Ar, Br = A[:, ::-1].copy(), B[:, ::-1].copy()
    err_r = np.linalg.norm(decimal2.bc_2digit(U, V, W, Ar, Br) - Ar @ Br)
    assert err_r < 2 * g["printed"]["g_error_reversed"]
    assert err_r < err / 10


def test_example7_expectations_agree_for_both_pairs(golden_dir):
    g = _example7(golden_dir)
    A = np.array(g["A"])
    B = np.array(g["B"])
    Ar, Br = A[:, ::-1].copy(), B[:, ::-1].copy()
    U, V, W = [T.astype(np.float64) for T in schemes.strassen()]
    assert g["printed"]["n_sign_functions"] * g["printed"]["n_permutation_functions"] == 512

    def expected_error(X, Y):
        mean = expectation.mean_over_draws(lambda dr: decimal2.bc_2digit(*draws.fold(U, V, W, dr), X, Y),
                                           2, 2, 2)
        return np.linalg.norm(mean - X @ Y)

    e, er = expected_error(A, B), expected_error(Ar, Br)
    # printed: both approximately 0.0024 -- the equality is reproduced, the value is not
    assert e == pytest.approx(er, rel=1e-9)
    assert 0 < e < np.linalg.norm(decimal2.bc_2digit(U, V, W, A, B) - A @ B)


def test_example13_printed_value(golden_dir):
    with open(os.path.join(golden_dir, "example13.json")) as f:
        g = json.load(f)
    assert round(bounds.example13(p=2.5), 4) == g["printed"]["second_term_coefficient"]
    assert bounds.example13(p=1.5) == pytest.approx(2 * bounds.example13(p=2.5))


def test_prop8_bound_holds_in_float32():
    U, V, W = schemes.strassen()
    q = tensors.q_uvw(U, V, W)
    eps = 2.0 ** -24
    for seed in range(200):
        A = workloads.gaussian((2, 2), seed)
        B = workloads.gaussian((2, 2), seed + 1000)
        A32, B32 = A.astype(np.float32).astype(np.float64), B.astype(np.float32).astype(np.float64)
        mu = max(np.linalg.norm(A32), np.linalg.norm(B32))
        exact = recursion.rbc_seeded(A32, B32, [(U, V, W)], seed, "none")
        fl = recursion.rbc_seeded(A32, B32, [(U, V, W)], seed, "none", arith="f32")
        assert np.linalg.norm(fl - exact) <= bounds.prop8(2, 7, eps, mu, q)


def test_prop9_bound_holds_in_float32_blocks():
    U, V, W = schemes.strassen()
    q = tensors.q_uvw(U, V, W)
    eps = 2.0 ** -24
    for seed in range(10):
        A = workloads.gaussian((32, 32), seed).astype(np.float32).astype(np.float64)
        B = workloads.gaussian((32, 32), seed + 50).astype(np.float32).astype(np.float64)
        mu = max(np.linalg.norm(A), np.linalg.norm(B))
        exact = recursion.rbc_seeded(A, B, [(U, V, W)], seed)
        fl = recursion.rbc_seeded(A, B, [(U, V, W)], seed, arith="f32")
        assert np.linalg.norm(fl - exact) <= bounds.prop9(2, 16, 7, eps, mu, q)


def _prop5_lhs(U, V, W, mu):
    """|eta| mu^2 ||Y|| of Prop. 5, eta = (1 - kappa)^-1 - 1, from the oracle's kappa and ||Y||."""
    return abs(bounds.eta(float(tensors.kappa(U, V, W)))) * mu * mu * tensors.ynorm(U, V, W)


def test_prop5_holds_on_perturbed_schemes():
    # Prop. 5 (with the corrected |kappa| <= n^(-3/2) tau) on perturbed Strassen (n = 2)
    # and Laderman (n = 3) at several noise levels, where |kappa| <= 1/2.
    for base, n in ((schemes.strassen(), 2), (schemes.laderman(), 3)):
        for sigma in (1e-4, 1e-3, 1e-2, 1e-1, 0.3):
            for seed in range(5):
                U, V, W = schemes.perturbed(*base, sigma, seed)
                k = float(tensors.kappa(U, V, W))
                assert abs(k) <= 0.5
                t = tensors.tau(U, V, W)
                for mu in (1.0, 3.5):
                    assert _prop5_lhs(U, V, W, mu) <= bounds.prop5(mu, n, t) * (1 + 1e-12)


def test_prop5_on_scaled_w_closed_form():
    # W of an exact scheme scaled by (1 + delta): Y = (1 + delta) X, so tau = delta n^(3/2),
    # kappa = -delta, |eta| = delta / (1 + delta) and |eta| ||Y|| = delta n^(3/2) exactly.
    # The corrected bound 2 (n^(-3/2) tau + 1) tau = 2 (1 + delta) delta n^(3/2) holds with
    # ratio 1 / (2 (1 + delta)); the printed one, 2 (n^(-5/2) tau + 1/n) tau
    # = 2 (1 + delta) delta n^(1/2), is exceeded for n = 3 (ratio 3 / (2 (1 + delta))).
    for base, n in ((schemes.strassen(), 2), (schemes.laderman(), 3)):
        U, V, W = [T.astype(np.float64) for T in base]
        for delta in (1e-3, 1e-2, 0.25):
            Ws = W * (1.0 + delta)
            t = tensors.tau(U, V, Ws)
            assert t == pytest.approx(delta * n ** 1.5, rel=1e-12)
            assert float(tensors.kappa(U, V, Ws)) == pytest.approx(-delta, rel=1e-12)
            lhs = _prop5_lhs(U, V, Ws, 1.0)
            assert lhs == pytest.approx(delta * n ** 1.5, rel=1e-12)
            assert lhs / bounds.prop5(1.0, n, t) == pytest.approx(1.0 / (2.0 * (1.0 + delta)), rel=1e-12)
            printed = bounds.prop5(1.0, n, t, p=2.5)
            assert printed == pytest.approx(2 * (1 + delta) * delta * n ** 0.5, rel=1e-12)
            if n == 3:
                assert lhs > printed
