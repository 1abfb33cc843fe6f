"""Oracle pins for the approximate-to-exact combination (Section 1, eq. APA-to-EBC)."""
from fractions import Fraction

import numpy as np
import pytest

import workloads
from oracle import recursion, schemes, tensors


def _lagrange_at_zero(eps):
    """alpha_i = prod_{j != i} eps_j / (eps_j - eps_i) in exact rationals: the weights
    of Lagrange interpolation evaluated at 0, which reproduce p(0) for any polynomial
    p of degree < len(eps)."""
    e = [Fraction(x) for x in eps]
    out = []
    for i, ei in enumerate(e):
        a = Fraction(1)
        for j, ej in enumerate(e):
            if j != i:
                a *= ej / (ej - ei)
        out.append(a)
    return out


def test_weights_for_the_papers_seven_values_are_binomial():
    # eps = 0.1, ..., 0.7: alpha_i = (-1)^(i+1) C(7, i), i = 1..7 (closed form of the
    # Lagrange weights at 0 for equispaced nodes k h).
    eps = [Fraction(k, 10) for k in range(1, 8)]
    alpha = schemes.apa_ebc_weights([float(e) for e in eps])
    exact = _lagrange_at_zero(eps)
    assert exact == [7, -21, 35, -35, 21, -7, 1]
    np.testing.assert_allclose(alpha, [float(a) for a in exact], rtol=0, atol=1e-9)


@pytest.mark.parametrize("eps", [[0.5], [0.1, 0.3], [2.0 ** -4, 2.0 ** -3, 0.75], [0.05, 0.9, 0.4, 0.2]])
def test_weights_match_lagrange_in_rationals(eps):
    alpha = schemes.apa_ebc_weights(eps)
    np.testing.assert_allclose(alpha, [float(a) for a in _lagrange_at_zero(eps)], rtol=1e-10, atol=1e-10)


def test_weights_reject_repeated_or_empty_eps():
    with pytest.raises(ValueError):
        schemes.apa_ebc_weights([0.1, 0.1])
    with pytest.raises(ValueError):
        schemes.apa_ebc_weights([])


@pytest.mark.parametrize("name", ["apa322", "apa223", "apa232"])
def test_two_values_make_the_rank10_tensor_exact(name):
    # The rank-10 schemes' error is a degree-1 polynomial in lambda: two distinct
    # values already give the exact <b1,b2,b3> tensor, one does not.
    build = getattr(schemes, name)
    b1, b2, b3, _ = tensors.dims(*build(0.5))
    X = tensors.brent_X(b1, b2, b3).astype(np.float64)
    for eps in ([0.1, 0.2], [0.25, 0.5], [0.1 * k for k in range(1, 8)]):
        alpha = schemes.apa_ebc_weights(eps)
        Y = sum(a * tensors.brent_Y(*build(e)) for a, e in zip(alpha, eps))
        np.testing.assert_allclose(Y, X, rtol=0, atol=1e-9)
    assert np.abs(tensors.brent_Y(*build(0.1)) - X).max() > 0.05


def _bini12(e):
    return schemes.bini12(e)


@pytest.mark.parametrize("seed,mode", [(0, "none"), (3, "full"), (5, "signs")])
def test_ebc_of_the_12x12_step_is_exact_on_integers(seed, mode):
    # One step of the 12 x 12 scheme (error of degree 3 in lambda) combined over the
    # seven values 0.1..0.7: the standard product of small integer matrices up to
    # f64 rounding, while a single lambda = 0.1 is off by O(lambda).
    A = workloads.integers((24, 24), 11, -3, 3)
    B = workloads.integers((24, 24), 12, -3, 3)
    AB = A @ B
    eps = [0.1 * k for k in range(1, 8)]
    C = recursion.apa_ebc(A, B, _bini12, eps, seed=seed, mode=mode)
    assert np.abs(C - AB).max() < 1e-8
    one = recursion.rbc_seeded(A, B, _bini12(0.1), seed, mode)
    assert np.abs(one - AB).max() > 0.1
    # Three values do not reach degree 3: the combination is still approximate.
    C3 = recursion.apa_ebc(A, B, _bini12, eps[:3], seed=seed, mode=mode)
    assert np.abs(C3 - AB).max() > 1e-6
