"""Pins for the oracle's scheme tensors (eq. requirement, Section 3.1)."""

import numpy as np
import pytest

from oracle import schemes, tensors
import workloads


@pytest.mark.parametrize("name", ["strassen", "laderman"])
def test_exact_schemes_satisfy_brent_equations_in_int64(name):
    U, V, W = getattr(schemes, name)()
    assert U.dtype == np.int64
    assert tensors.tau_squared_exact(U, V, W) == 0
    assert tensors.kappa(U, V, W) == 0


@pytest.mark.parametrize("name,R", [("strassen", 7), ("laderman", 23)])
def test_exact_schemes_reproduce_matmul(name, R):
    # Independent of the Brent tensor: evaluate the BC of eq. bilinear-computation-block
    # on integer matrices and compare with a library matrix product.
    U, V, W = getattr(schemes, name)()
    assert U.shape[2] == R
    b = U.shape[0]
    for m, seed in [(1, 1), (3, 2), (4, 3)]:
        A = workloads.integers((b * m, b * m), seed)
        B = workloads.integers((b * m, b * m), seed + 100)
        assert np.array_equal(tensors.bc_evaluate(U, V, W, A, B), A @ B)


@pytest.mark.parametrize("b1,b2,b3", [(2, 3, 2), (3, 2, 2), (1, 2, 3)])
def test_naive_rectangular_scheme_is_exact(b1, b2, b3):
    U, V, W = schemes.naive(b1, b2, b3)
    assert tensors.tau_squared_exact(U, V, W) == 0
    A = workloads.integers((b1 * 2, b2 * 3), 7)
    B = workloads.integers((b2 * 3, b3 * 5), 8)
    assert np.array_equal(tensors.bc_evaluate(U, V, W, A, B), A @ B)


def test_strassen_nonzero_counts():
    U, V, W = schemes.strassen()
    assert (np.count_nonzero(U), np.count_nonzero(V), np.count_nonzero(W)) == (12, 12, 12)


def test_perturbed_scheme_tau_scales_with_sigma():
    base = schemes.strassen()
    ratios = []
    for sigma in [1e-1, 1e-2, 1e-3, 1e-4]:
        P = schemes.perturbed(*base, sigma, np.random.default_rng(5))
        t = tensors.tau(*P)
        assert t > 0
        ratios.append(t / sigma)
    # same noise pattern scaled by sigma: tau/sigma converges (first-order in sigma)
    assert max(ratios) / min(ratios) < 1.3


def test_perturbed_scheme_touches_ones_and_five_zeros():
    base = schemes.strassen()
    P = schemes.perturbed(*base, 1e-3, np.random.default_rng(0))
    for T0, T in zip(base, P):
        changed = T != T0
        assert np.all(changed[T0 == 1])
        assert np.sum(changed[T0 == 0]) == 5
        assert not np.any(changed[T0 == -1])
