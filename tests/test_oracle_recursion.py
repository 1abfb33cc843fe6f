"""Pins for the oracle's recursion F-hat^(Q) (Section 2.1.1)."""

import numpy as np
import pytest

from oracle import bounds, draws, recursion, schemes, tensors
import workloads

S = schemes.strassen()
L = schemes.laderman()

EXACT_PLANS = {
    "strassen_q1": [S],
    "strassen_q2": [S, S],
    "strassen_q3": [S, S, S],
    "laderman_q1": [L],
    "laderman_strassen": [L, S],
    "naive_232_then_strassen": [schemes.naive(2, 3, 2), S],
}


@pytest.mark.parametrize("plan", list(EXACT_PLANS))
@pytest.mark.parametrize("mode", ["full", "signs", "perms", "none"])
def test_exact_scheme_is_exact_on_integers_for_every_draw(plan, mode):
    # Remark after Definition 2: for an EBC, f-hat(A, B) = A B for every draw.
    levels = EXACT_PLANS[plan]
    for seed, (M, K, N) in [(0, (24, 24, 24)), (1, (23, 17, 29)), (2, (7, 30, 12))]:
        A = workloads.integers((M, K), 100 + seed)
        B = workloads.integers((K, N), 200 + seed)
        C = recursion.rbc_seeded(A, B, levels, seed, mode)
        assert np.array_equal(C, A @ B), (plan, mode, seed)
        C32 = recursion.rbc_seeded(A, B, levels, seed, mode, arith="f32")
        assert np.array_equal(C32, A @ B), (plan, mode, seed)


def test_float64_error_of_exact_scheme_is_rounding_level():
    A = workloads.gaussian((64, 64), 1001)
    B = workloads.gaussian((64, 64), 1002)
    C = recursion.rbc_seeded(A, B, [S, S], 0)
    assert recursion.rel_err(C, A @ B) < 1e-14


def test_prop4_ii_bound_single_level():
    base = schemes.perturbed(*S, 1e-2, 4)
    A = workloads.gaussian((8, 8), 5)
    B = workloads.gaussian((8, 8), 6)
    bound = bounds.prop4_ii(np.linalg.norm(A), np.linalg.norm(B), *base)
    tight = 0.0
    for seed in range(40):
        err = np.linalg.norm(recursion.rbc_seeded(A, B, [base], seed) - A @ B)
        assert err <= bound * (1 + 1e-12)
        tight = max(tight, err / bound)
    assert tight > 1e-3   # the bound is not vacuous for this case


def test_prop4_i_bound_deterministic():
    base = schemes.perturbed(*L, 1e-2, 8)
    A = workloads.gaussian((9, 9), 7)
    B = workloads.gaussian((9, 9), 8)
    err = np.linalg.norm(recursion.rbc_seeded(A, B, [base], 0, "none") - A @ B)
    assert err <= bounds.prop4_i(np.linalg.norm(A), np.linalg.norm(B), tensors.tau(*base))


def test_approximate_scheme_error_is_first_order_in_lambda():
    A = workloads.gaussian((32, 32), 3001)
    B = workloads.gaussian((32, 32), 3002)
    lams = [1e-1, 1e-2, 1e-3, 1e-4]
    for Q in (1, 2):
        errs = []
        for lam in lams:
            base = schemes.perturbed(*S, lam, 42)
            errs.append(recursion.rel_err(recursion.rbc_seeded(A, B, [base] * Q, 3), A @ B))
        slope = np.polyfit(np.log10(lams), np.log10(errs), 1)[0]
        assert 0.9 < slope < 1.1, (Q, errs)


def test_f32_working_precision_close_to_f64():
    A = workloads.uniform((64, 64), 2001, -1, 1)
    B = workloads.uniform((64, 64), 2002, -1, 1)
    c64 = recursion.rbc_seeded(A, B, [S, S, S], 0)
    c32 = recursion.rbc_seeded(A, B, [S, S, S], 0, arith="f32")
    assert c32.dtype == np.float32
    e = recursion.rel_err(c32, A @ B)
    assert 1e-8 < e < 1e-5
    assert recursion.rel_err(c64, A @ B) < 1e-14


def test_leaf_operands_and_combine_reassemble_the_product():
    levels = [S, S]
    dr = recursion.seeded_draws(levels, 9)
    A = workloads.gaussian((20, 12), 1)
    B = workloads.gaussian((12, 28), 2)
    ops = recursion.leaf_operands(A, B, levels, dr)
    assert len(ops) == 49
    assert ops[0][0].shape == (5, 3) and ops[0][1].shape == (3, 7)
    prods = [s @ t for s, t in ops]
    C = recursion.combine(prods, 20, 28, 12, levels, dr)
    np.testing.assert_array_equal(C, recursion.rbc(A, B, levels, dr))


def test_deterministic_is_mode_none_without_kappa_scale():
    base = schemes.perturbed(*S, 1e-2, 1)
    A = workloads.gaussian((8, 8), 1)
    B = workloads.gaussian((8, 8), 2)
    det = tensors.bc_evaluate(*base, A, B)
    C = recursion.rbc_seeded(A, B, [base], 123, "none")
    np.testing.assert_allclose(C, det, rtol=1e-13, atol=1e-13)


def test_monte_carlo_mean_two_levels():
    # Prop. 6 for Q = 2: the sample mean over seeds approaches A B for an ABC.
    base = schemes.perturbed(*S, 5e-2, 2)
    A = workloads.gaussian((4, 4), 11)
    B = workloads.gaussian((4, 4), 12)
    samples = np.array([recursion.rbc_seeded(A, B, [base, base], s) for s in range(3000)])
    mean = samples.mean(axis=0)
    se = samples.std(axis=0) / np.sqrt(len(samples))
    assert np.all(np.abs(mean - A @ B) <= 5 * se + 1e-12)
    det = recursion.rbc_seeded(A, B, [base, base], 0, "none")
    assert np.linalg.norm(mean - A @ B) < np.linalg.norm(det - A @ B)
