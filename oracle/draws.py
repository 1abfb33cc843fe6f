"""Random signed block permutations, one draw per recursion level, and the fold.

Section 2.1 (before Definition 2): s_i(j) are i.i.d. Rademacher signs and pi_i
are random permutations with P[pi_i(j) = k] = 1/n, for i in {1, 2, 3}; in the
recursive algorithm (Section 2.1.1) each level q has its own independent set.

Reading of the paper where it is silent (the RNG, the word-to-draw mapping and
the level index):
  * generator: Philox4x64-10 (Salmon et al., SC'11) with key (seed, 0); the
    words for depth d (0 = outermost level) are the raw output of numpy's Philox
    bit generator started at counter (0, d, 0, 0), i.e. blocks (1,d,0,0),
    (2,d,0,0), ... four words each, in order;
  * signs s1[0..b1), s2[0..b2), s3[0..b3) take one word each, +1 when the top
    bit is 0 and -1 otherwise;
  * then pi1, pi2, pi3 by Fisher-Yates from the identity: for i = b-1 down to 1,
    j = floor(word * (i + 1) / 2^64), swap p[i] and p[j] (one word per step);
    every permutation of [b] is then equally likely up to a bias <= b / 2^64;
  * modes: "full" keeps both, "signs" sets pi = id, "perms" sets s = 1,
    "none" sets both (the deterministic F^(Q) of Section 3); every word is
    consumed in every mode so the streams of the modes stay aligned.

Fold (proof of Proposition 10, eq. randomized-algorithm):
  Uh[k,l,r]   = U[pi1(k), pi2(l), r] s1(k) s2(l)
  Vh[k',l',r] = V[pi2(k'), pi3(l'), r] s2(k') s3(l')
  Wh[i,j,r]   = c s1(i) s3(j) W[pi1(i), pi3(j), r],   c = (1 - kappa)^-1 or 1.

Pins: the generator is numpy's (an independent library); tests check that each
draw is a valid signed permutation, the statistics of the mapping, that the
fold preserves ||U_r||, ||V_r|| and scales ||W_r|| by c (Proposition 10), and
that for an exact scheme every draw gives A B exactly on integer inputs.
"""

import numpy as np

MODES = ("full", "signs", "perms", "none")


def philox_words(seed, depth, count):
    """``count`` raw 64-bit words of Philox4x64-10, key (seed, 0), stream ``depth``."""
    key = np.array([seed & 0xFFFFFFFFFFFFFFFF, 0], dtype=np.uint64)
    ctr = np.array([0, depth, 0, 0], dtype=np.uint64)
    g = np.random.Philox(key=key, counter=ctr)
    return [int(w) for w in g.random_raw(count)]


def words_needed(b1, b2, b3):
    return (b1 + b2 + b3) + (b1 - 1) + (b2 - 1) + (b3 - 1)


def draw_from_words(words, b1, b2, b3, mode="full"):
    """Map words to (s1, s2, s3, p1, p2, p3) as described in the module docstring."""
    if mode not in MODES:
        raise ValueError(mode)
    it = iter(words)
    signs = []
    for b in (b1, b2, b3):
        signs.append(np.array([1 if (next(it) >> 63) == 0 else -1 for _ in range(b)], dtype=np.int64))
    perms = []
    for b in (b1, b2, b3):
        p = list(range(b))
        for i in range(b - 1, 0, -1):
            j = (next(it) * (i + 1)) >> 64
            p[i], p[j] = p[j], p[i]
        perms.append(np.array(p, dtype=np.int64))
    if mode in ("perms", "none"):
        signs = [np.ones(b, dtype=np.int64) for b in (b1, b2, b3)]
    if mode in ("signs", "none"):
        perms = [np.arange(b, dtype=np.int64) for b in (b1, b2, b3)]
    return tuple(signs) + tuple(perms)


def draw(seed, depth, b1, b2, b3, mode="full"):
    return draw_from_words(philox_words(seed, depth, words_needed(b1, b2, b3)), b1, b2, b3, mode)


def fold(U, V, W, dr, c=1.0):
    """Folded tensors (Uh, Vh, Wh) for one draw ``dr`` = (s1, s2, s3, p1, p2, p3)."""
    s1, s2, s3, p1, p2, p3 = dr
    U = np.asarray(U, np.float64)
    V = np.asarray(V, np.float64)
    W = np.asarray(W, np.float64)
    b1, b2, R = U.shape
    b3 = V.shape[1]
    Uh = np.empty_like(U)
    Vh = np.empty_like(V)
    Wh = np.empty_like(W)
    for k in range(b1):
        for l in range(b2):
            Uh[k, l, :] = U[p1[k], p2[l], :] * (s1[k] * s2[l])
    for k in range(b2):
        for l in range(b3):
            Vh[k, l, :] = V[p2[k], p3[l], :] * (s2[k] * s3[l])
    for i in range(b1):
        for j in range(b3):
            Wh[i, j, :] = c * (s1[i] * s3[j]) * W[p1[i], p3[j], :]
    return Uh, Vh, Wh
