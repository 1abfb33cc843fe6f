"""Pins for tau, kappa, ||Y|| and q (Definition 1, eq. epsilon-def, Props. 4-5, Example 13)."""

import json
import os

import numpy as np
import pytest

from oracle import bounds, schemes, tensors


def test_rank_one_all_ones_remark():
    # Remark after Prop. 5: R = 1 and all ones gives kappa = 0 but a large tau.
    U, V, W = schemes.rank_one_all_ones(2)
    assert tensors.kappa(U, V, W) == 0
    assert tensors.tau_squared_exact(U, V, W) == 64 - 8
    assert tensors.tau(U, V, W) == pytest.approx(np.sqrt(56.0), rel=1e-15)


@pytest.mark.parametrize("n", [2, 3, 4])
def test_x_norm(n):
    X = tensors.brent_X(n, n, n)
    assert np.sum(X) == n ** 3
    assert np.sqrt(np.sum(X * X)) == pytest.approx(n ** 1.5)


def test_strassen_q_is_sqrt_32(golden_dir):
    with open(os.path.join(golden_dir, "example13.json")) as f:
        printed = json.load(f)["printed"]["strassen_q"]
    assert "6" in printed
    q = tensors.q_uvw(*schemes.strassen())
    assert q == pytest.approx(np.sqrt(32.0), rel=1e-15)
    assert round(q) == 6


def test_y_norm_bound_and_corrected_kappa_bound():
    rng = np.random.default_rng(11)
    base = schemes.strassen()
    for trial in range(20):
        P = schemes.perturbed(*base, 10 ** rng.uniform(-4, -1), 100 + trial)
        t = tensors.tau(*P)
        k = tensors.kappa(*P)
        assert tensors.ynorm(*P) <= t + 2 ** 1.5 + 1e-12          # eq. Ye-bound
        assert abs(k) <= bounds.kappa_bound(2, t, p=1.5) + 1e-15  # corrected eq. epsilon-bound


def test_printed_kappa_bound_fails_on_scaled_w():
    # W scaled by (1 + delta): every "X = 1" entry of Y becomes 1 + delta.
    U, V, W = schemes.strassen()
    delta = 1e-3
    W2 = W * (1 + delta)
    k = tensors.kappa(U, V, W2)
    t = tensors.tau(U, V, W2)
    assert k == pytest.approx(-delta, rel=1e-9)
    assert abs(k) > bounds.kappa_bound(2, t, p=2.5)              # the printed n^-5/2 bound fails
    assert abs(k) <= bounds.kappa_bound(2, t, p=1.5) * (1 + 1e-9)  # the corrected bound is tight


def test_kappa_closed_form_for_scaled_exact_scheme():
    # U*a, V*b, W*c of an exact scheme: every "X = 1" entry of Y is abc, so kappa = 1 - abc
    # and tau = |abc - 1| n^(3/2) (Y = abc X).
    for name, n in [("strassen", 2), ("laderman", 3)]:
        U, V, W = [T.astype(np.float64) for T in getattr(schemes, name)()]
        a, b, c = 1.25, 0.5, 1.5
        k = tensors.kappa(U * a, V * b, W * c)
        assert k == pytest.approx(1 - a * b * c, abs=1e-14)
        assert tensors.tau(U * a, V * b, W * c) == pytest.approx(abs(a * b * c - 1) * n ** 1.5, rel=1e-12)
