"""Pins for the per-level draws and the fold (Section 2.1, Definition 2, Prop. 10)."""

import numpy as np
import pytest

from oracle import draws, schemes, tensors
import workloads


@pytest.mark.parametrize("b1,b2,b3", [(2, 2, 2), (3, 3, 3), (3, 2, 2)])
def test_draws_are_signed_permutations(b1, b2, b3):
    for seed in range(50):
        for d in range(3):
            s1, s2, s3, p1, p2, p3 = draws.draw(seed, d, b1, b2, b3, "full")
            for s, b in ((s1, b1), (s2, b2), (s3, b3)):
                assert len(s) == b and set(np.unique(s)) <= {-1, 1}
            for p, b in ((p1, b1), (p2, b2), (p3, b3)):
                assert sorted(p.tolist()) == list(range(b))


def test_word_count_and_numpy_stream():
    assert draws.words_needed(2, 2, 2) == 9
    assert draws.words_needed(3, 3, 3) == 15
    # the words are numpy's Philox raw stream at counter (0, d, 0, 0), key (seed, 0)
    g = np.random.Philox(key=np.array([7, 0], np.uint64), counter=np.array([0, 2, 0, 0], np.uint64))
    assert draws.philox_words(7, 2, 9) == [int(x) for x in g.random_raw(9)]
    assert draws.philox_words(7, 2, 9) != draws.philox_words(7, 1, 9)
    assert draws.philox_words(7, 2, 9) != draws.philox_words(8, 2, 9)


def test_mode_semantics_share_the_stream():
    full = draws.draw(3, 0, 3, 3, 3, "full")
    sg = draws.draw(3, 0, 3, 3, 3, "signs")
    pm = draws.draw(3, 0, 3, 3, 3, "perms")
    no = draws.draw(3, 0, 3, 3, 3, "none")
    for i in range(3):
        assert np.array_equal(sg[i], full[i]) and np.array_equal(pm[3 + i], full[3 + i])
        assert np.array_equal(sg[3 + i], np.arange(3)) and np.array_equal(pm[i], np.ones(3))
        assert np.array_equal(no[i], np.ones(3)) and np.array_equal(no[3 + i], np.arange(3))


def test_draw_statistics():
    # P[pi(j) = k] = 1/n and P[s = +1] = 1/2 (Section 2.1); loose 6-sigma checks.
    n_seeds = 6000
    counts = np.zeros((3, 3))
    plus = 0
    for seed in range(n_seeds):
        s1, s2, s3, p1, p2, p3 = draws.draw(seed, 0, 3, 3, 3)
        for j in range(3):
            counts[j, p1[j]] += 1
        plus += int(np.sum(s1 == 1))
    p = counts / n_seeds
    sd = np.sqrt((1 / 3) * (2 / 3) / n_seeds)
    assert np.all(np.abs(p - 1 / 3) < 6 * sd)
    assert abs(plus / (3 * n_seeds) - 0.5) < 6 * np.sqrt(0.25 / (3 * n_seeds))


def test_fold_preserves_slice_norms():
    # Proof of Prop. 10: ||Uh_r|| = ||U_r||, ||Vh_r|| = ||V_r||, ||Wh_r|| = c ||W_r||.
    base = schemes.perturbed(*schemes.laderman(), 1e-2, 3)
    dr = draws.draw(5, 1, 3, 3, 3)
    c = 1.0 / (1.0 - tensors.kappa(*base))
    Uh, Vh, Wh = draws.fold(*base, dr, c)
    for T, Th, f in ((base[0], Uh, 1.0), (base[1], Vh, 1.0), (base[2], Wh, c)):
        np.testing.assert_allclose(np.linalg.norm(Th, axis=(0, 1)), f * np.linalg.norm(T, axis=(0, 1)),
                                   rtol=1e-14)


def _block_matrix(perm, signs, m):
    """M_i = P_i S_i of Section 2.1: P_i has identity blocks at (pi(j), j), S_i = diag(s(j) I)."""
    n = len(perm)
    M = np.zeros((n * m, n * m))
    for j in range(n):
        M[perm[j] * m:(perm[j] + 1) * m, j * m:(j + 1) * m] = signs[j] * np.eye(m)
    return M


@pytest.mark.parametrize("name", ["strassen", "laderman"])
def test_fold_equals_definition_2_with_explicit_matrices(name):
    # eq. f-hat-def computed with explicit orthogonal matrices M_i, against the folded
    # tensors of eq. randomized-algorithm; both evaluated as a plain BC in float64.
    base = schemes.perturbed(*getattr(schemes, name)(), 1e-2, 9)
    n = base[0].shape[0]
    m = 3
    A = workloads.gaussian((n * m, n * m), 1)
    B = workloads.gaussian((n * m, n * m), 2)
    k = float(tensors.kappa(*base))
    for seed in range(5):
        dr = draws.draw(seed, 0, n, n, n)
        s1, s2, s3, p1, p2, p3 = dr
        M1, M2, M3 = (_block_matrix(p1, s1, m), _block_matrix(p2, s2, m), _block_matrix(p3, s3, m))
        assert np.allclose(M1.T @ M1, np.eye(n * m))
        ref = M1.T @ tensors.bc_evaluate(*base, M1 @ A @ M2.T, M2 @ B @ M3.T) @ M3 / (1 - k)
        Uh, Vh, Wh = draws.fold(*base, dr, 1.0 / (1 - k))
        got = tensors.bc_evaluate(Uh, Vh, Wh, A, B)
        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)
