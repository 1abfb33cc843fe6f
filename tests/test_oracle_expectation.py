"""Exact enumeration pins of Propositions 3 and 6 (E[f-hat] = A B)."""

import numpy as np

from oracle import draws, expectation, recursion, schemes, tensors
import workloads


def test_expectation_exact_for_approximate_scheme():
    # Prop. 3: for an ABC with kappa != 0, the mean over all 2^6 * 2^3 draws is A B.
    base = schemes.perturbed(*schemes.strassen(), 3e-2, 7)
    k = float(tensors.kappa(*base))
    assert abs(k) > 1e-4
    A = workloads.gaussian((4, 6), 1)
    B = workloads.gaussian((6, 2), 2)
    mean = expectation.mean_over_draws(lambda dr: recursion.rbc(A, B, [base], [dr]), 2, 2, 2)
    np.testing.assert_allclose(mean, A @ B, rtol=1e-12, atol=1e-13)
    # without the (1 - kappa)^-1 factor the mean is (1 - kappa) A B
    mean_u = expectation.mean_over_draws(lambda dr: recursion.rbc(A, B, [base], [dr], kappa_scale=False),
                                         2, 2, 2)
    np.testing.assert_allclose(mean_u, (1 - k) * (A @ B), rtol=1e-12, atol=1e-13)
    # a single realisation is not exact
    one = recursion.rbc(A, B, [base], [draws.draw(0, 0, 2, 2, 2)])
    assert np.linalg.norm(one - A @ B) > 1e-3 * np.linalg.norm(A @ B)


def test_expectation_exact_rectangular_blocks():
    base = schemes.perturbed(*schemes.naive(2, 3, 2), 5e-2, 1)
    A = workloads.gaussian((4, 6), 3)
    B = workloads.gaussian((6, 4), 4)
    mean = expectation.mean_over_draws(lambda dr: recursion.rbc(A, B, [base], [dr]), 2, 3, 2)
    np.testing.assert_allclose(mean, A @ B, rtol=1e-12, atol=1e-13)


def test_sign_only_expectation_of_exact_scheme():
    # Proof of Prop. 3: averaging over signs alone keeps only the i=k, l=k', j=l' terms.
    A = workloads.gaussian((6, 6), 5)
    B = workloads.gaussian((6, 6), 6)
    L = schemes.laderman()
    mean = expectation.mean_over_draws(lambda dr: recursion.rbc(A, B, [L], [dr]), 3, 3, 3, mode="signs")
    np.testing.assert_allclose(mean, A @ B, rtol=1e-12, atol=1e-12)


def test_enumeration_count_matches_example_7():
    assert sum(1 for _ in expectation.all_draws(2, 2, 2)) == 64 * 8
