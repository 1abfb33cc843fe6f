"""Exact enumeration of the expectation over every draw of one level.

Propositions 3 and 6: E[F-hat^(Q)(A, B)] = A B.  With b x b blocks there are
2^(b1+b2+b3) sign vectors and b1! b2! b3! permutation triples, all equally
likely (the fold is uniform over them), so the expectation is the plain mean
over that finite set.  For Q = 1 the mean is taken over all draws of the single
level (512 for 2x2 schemes, as counted in Example 7).
"""

import itertools

import numpy as np


def all_draws(b1, b2, b3, mode="full"):
    sign_sets = [list(itertools.product((1, -1), repeat=b)) for b in (b1, b2, b3)]
    perm_sets = [list(itertools.permutations(range(b))) for b in (b1, b2, b3)]
    if mode in ("perms", "none"):
        sign_sets = [[tuple([1] * b)] for b in (b1, b2, b3)]
    if mode in ("signs", "none"):
        perm_sets = [[tuple(range(b))] for b in (b1, b2, b3)]
    for s1 in sign_sets[0]:
        for s2 in sign_sets[1]:
            for s3 in sign_sets[2]:
                for p1 in perm_sets[0]:
                    for p2 in perm_sets[1]:
                        for p3 in perm_sets[2]:
                            yield tuple(np.array(x, dtype=np.int64) for x in (s1, s2, s3, p1, p2, p3))


def mean_over_draws(fn, b1, b2, b3, mode="full"):
    """Mean of fn(draw) over every draw of one level (float64 accumulation)."""
    total = None
    count = 0
    for dr in all_draws(b1, b2, b3, mode):
        v = np.asarray(fn(dr), dtype=np.float64)
        total = v.copy() if total is None else total + v
        count += 1
    return total / count
