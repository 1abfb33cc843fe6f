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
        P = schemes.perturbed(*base, sigma, 5)
        t = tensors.tau(*P)
        assert t > 0
        ratios.append(t / sigma)
    # same noise pattern scaled by sigma: tau/sigma converges (first-order in sigma)
    assert max(ratios) / min(ratios) < 1.3


def test_perturbed_scheme_touches_ones_and_five_zeros():
    base = schemes.strassen()
    P = schemes.perturbed(*base, 1e-3, 0)
    for T0, T in zip(base, P):
        changed = T != T0
        assert np.all(changed[T0 == 1])
        assert np.sum(changed[T0 == 0]) == 5
        assert not np.any(changed[T0 == -1])


def test_perturbation_uniforms_are_exact_and_open():
    # u = (floor(w / 2^12) + 1/2) 2^-52: the extreme words map strictly inside (0, 1)
    assert schemes.open_unit(0) == 2.0 ** -53
    assert schemes.open_unit(2 ** 64 - 1) == 1.0 - 2.0 ** -53
    assert schemes.open_unit(2 ** 63) == 0.5 + 2.0 ** -53
    from fractions import Fraction
    for w in (1, 4095, 4096, 2 ** 40 + 12345, 2 ** 64 - 4097):
        assert Fraction(schemes.open_unit(w)) == (Fraction(w >> 12) + Fraction(1, 2)) / 2 ** 52


def test_perturbation_words_are_numpys_philox_with_key_word_one():
    w = schemes.aux_words(9)
    got = [next(w) for _ in range(10)]
    g = np.random.Philox(key=np.array([9, 1], np.uint64), counter=np.zeros(4, np.uint64))
    assert got == [int(x) for x in g.random_raw(10)]
    # a different key word than the level draws (key (seed, 0))
    g0 = np.random.Philox(key=np.array([9, 0], np.uint64), counter=np.zeros(4, np.uint64))
    assert got != [int(x) for x in g0.random_raw(10)]


def test_box_muller_normals():
    # Against numpy's own (vectorised) log / cos / sqrt on the same uniforms, and the
    # first four moments of N(0, 1) over 40000 draws.
    w = schemes.aux_words(123)
    z = np.array([schemes.box_muller(w) for _ in range(40000)])
    w = schemes.aux_words(123)
    words = np.array([next(w) for _ in range(80000)], dtype=np.uint64)
    u = ((words >> np.uint64(12)).astype(np.float64) + 0.5) * 2.0 ** -52
    ref = np.sqrt(-2.0 * np.log(u[0::2])) * np.cos(2.0 * np.pi * u[1::2])
    assert np.max(np.abs(z - ref)) <= 8 * 2.0 ** -52 * np.max(np.abs(ref))
    n = z.size
    assert abs(z.mean()) < 5 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 5 * np.sqrt(2.0 / n)
    assert abs(np.mean(z ** 3)) < 5 * np.sqrt(15.0 / n)
    assert abs(np.mean(z ** 4) - 3.0) < 5 * np.sqrt(96.0 / n)
    from scipy import stats
    assert stats.kstest(z, "norm").pvalue > 1e-4


def test_perturbation_picks_zeros_uniformly():
    # 5 of Strassen's 16 zeros of U picked without replacement: each with probability 5/16
    base = schemes.strassen()
    zeros = np.flatnonzero(base[0].reshape(-1) == 0)
    assert zeros.size == 16
    n = 3000
    hits = np.zeros(zeros.size)
    for seed in range(n):
        P = schemes.perturbed(*base, 1e-3, seed)
        changed = P[0].reshape(-1)[zeros] != 0
        assert changed.sum() == 5
        hits += changed
    p = 5 / 16
    assert np.all(np.abs(hits / n - p) < 6 * np.sqrt(p * (1 - p) / n))


def test_perturbation_zero_sigma_and_seed_dependence():
    base = schemes.laderman()
    for T0, T in zip(base, schemes.perturbed(*base, 0.0, 5)):
        np.testing.assert_array_equal(T, T0)
    a = schemes.perturbed(*base, 1e-2, 5)
    b = schemes.perturbed(*base, 1e-2, 6)
    assert not np.array_equal(a[0], b[0])
    # the noise scales with sigma: same draws, sigma 1e-2 vs 1e-4
    c = schemes.perturbed(*base, 1e-4, 5)
    for T0, Ta, Tc in zip(base, a, c):
        d = Ta - T0
        np.testing.assert_allclose((Tc - T0) * 100.0, d, rtol=1e-9, atol=1e-15)


def _residual_exact(U, V, W):
    """Brent residual Y - X (eq. requirement) in exact rationals: every float entry is
    an exact binary fraction, so Fraction(x) loses nothing."""
    from fractions import Fraction
    b1, b2, R = U.shape
    b3 = V.shape[1]
    E = {}
    for i, j, jj, k, ii, kk in np.ndindex(b1, b2, b2, b3, b1, b3):
        y = sum(Fraction(float(U[i, j, r])) * Fraction(float(V[jj, k, r])) * Fraction(float(W[ii, kk, r]))
                for r in range(R))
        E[(i, j, jj, k, ii, kk)] = y - (1 if (i == ii and j == jj and k == kk) else 0)
    return E


def _solve_exact(M, y):
    """Solve the square system M x = y over Fractions (Gauss-Jordan)."""
    n = len(y)
    A = [list(row) + [v] for row, v in zip(M, y)]
    for c in range(n):
        p = next(r for r in range(c, n) if A[r][c] != 0)
        A[c], A[p] = A[p], A[c]
        A[c] = [x / A[c][c] for x in A[c]]
        for r in range(n):
            if r != c and A[r][c] != 0:
                A[r] = [a - A[r][c] * b for a, b in zip(A[r], A[c])]
    return [A[r][n] for r in range(n)]


@pytest.mark.parametrize("name", ["apa322", "apa223", "apa232"])
def test_apa_residual_is_order_lambda_in_exact_arithmetic(name):
    # U and V are affine in lam and W is (1/lam) times constants, so every entry of
    # Y(lam) - X is c_{-1}/lam + c_0 + c_1 lam + c_2 lam^2.  Recover the four
    # coefficients exactly from lam = 2^-1 .. 2^-4, require c_{-1} = c_0 = 0 (no
    # blow-up, no constant term: Y(lam) -> X), some c_1 != 0 (a real approximation),
    # and check the Laurent polynomial against the exact residual at lam = 2^-5 .. 2^-30.
    from fractions import Fraction
    lams = [Fraction(1, 2 ** k) for k in range(1, 31)]
    build = getattr(schemes, name)
    res = [_residual_exact(*build(float(l))) for l in lams]
    M = [[1 / l, Fraction(1), l, l * l] for l in lams[:4]]
    nonzero_c1 = 0
    for key in res[0]:
        c = _solve_exact(M, [r[key] for r in res[:4]])
        assert c[0] == 0 and c[1] == 0, key
        nonzero_c1 += c[2] != 0
        for l, r in zip(lams[4:], res[4:]):
            assert c[2] * l + c[3] * l * l == r[key], key
    assert nonzero_c1 > 0
    # tau(lam) = Theta(lam): halving lam halves tau in the limit
    t = [tensors.tau(*build(2.0 ** -k)) for k in (20, 21)]
    assert abs(t[0] / t[1] - 2.0) < 1e-6


def test_apa322_approximates_matmul_on_integers():
    # The scheme as a plain bilinear computation (eq. bilinear-computation-block) on
    # 3m x 2m times 2m x 2m integer matrices, lam = 2^-20 (every partial sum exact in
    # float64): blocks C11 and C31 exact, the others within O(lam).
    lam = 2.0 ** -20
    U, V, W = schemes.apa322(lam)
    for m, seed in [(1, 5), (3, 6)]:
        A = workloads.integers((3 * m, 2 * m), seed).astype(np.float64)
        B = workloads.integers((2 * m, 2 * m), seed + 100).astype(np.float64)
        C = tensors.bc_evaluate(U, V, W, A, B)
        ref = A @ B
        # at most four O(lam) block products in an entry, each entry of one at most m |A| |B|
        assert np.abs(C - ref).max() <= 4 * lam * m * np.abs(A).max() * np.abs(B).max()
        assert np.array_equal(C[:m, :m], ref[:m, :m])          # C11: no lam term
        assert np.array_equal(C[2 * m:, :m], ref[2 * m:, :m])  # C31: no lam term


@pytest.mark.parametrize("name", ["strassen", "laderman", "naive:2,3,4"])
def test_rotation_keeps_exact_schemes_exact(name):
    if name.startswith("naive:"):
        base = schemes.naive(*(int(x) for x in name[6:].split(",")))
    else:
        base = getattr(schemes, name)()
    b1, b2, b3 = base[0].shape[0], base[0].shape[1], base[1].shape[1]
    U, V, W = schemes.rotate(*base)
    assert (U.shape[0], U.shape[1], V.shape[1]) == (b2, b3, b1)
    assert tensors.tau_squared_exact(U, V, W) == 0
    A = workloads.integers((b2 * 2, b3 * 3), 11)
    B = workloads.integers((b3 * 3, b1 * 2), 12)
    assert np.array_equal(tensors.bc_evaluate(U, V, W, A, B), A @ B)
    # three rotations give the scheme back
    for got, want in zip(schemes.rotate(*schemes.rotate(U, V, W)), base):
        assert np.array_equal(got, want)


def test_bini12_levels_approximate_matmul():
    # One step of the 12 x 12 scheme is the three-level recursion over <3,2,2>,
    # <2,2,3>, <2,3,2> (no randomization): within O(lam) of A B on N = 24, and the
    # error halves with lam while lam dominates the float64 rounding (amplified 1/lam^3).
    from oracle import recursion
    A = workloads.gaussian((24, 24), 21)
    B = workloads.gaussian((24, 24), 22)
    AB = A @ B
    errs = []
    for k in (8, 9):
        lam = 2.0 ** -k
        C = recursion.rbc_seeded(A, B, schemes.bini12(lam), 0, "none")
        errs.append(recursion.rel_err(C, AB))
    assert errs[0] < 0.05
    assert 1.8 < errs[0] / errs[1] < 2.2
