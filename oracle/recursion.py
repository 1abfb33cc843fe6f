"""F-hat^(Q): the recursive randomized bilinear computation (Section 2.1.1).

eq. recursive-random-formula, written with the folded tensors of
eq. randomized-algorithm (Proposition 10) at every level:

  rec(A, B, d):                           d = depth from the top, 0 = outermost
    if d == Q: return A B                 standard product at the leaves
    split A into b1 x b2 blocks A_kl and B into b2 x b3 blocks B_k'l'
    for r = 1..R:
      S_r = sum_{k,l}   Uh[k,l,r]   A_kl   (the paper's A^(q) for this r)
      T_r = sum_{k',l'} Vh[k',l',r] B_k'l' (the paper's B^(q) for this r)
      P_r = rec(S_r, T_r, d + 1)
    C_ij = sum_r Wh[i,j,r] P_r

Readings (the paper is silent on these; they fix the rounding order so that a
float32 evaluation is reproducible bit for bit):
  * sums run sequentially (the fl model of Section 2.2): S_r over (k, l) in
    row-major order and C_ij over ascending r, each skipping zero
    coefficients; the first term is fl(coef * block), then
    acc = fl(acc + fl(coef * block)); a sum with no term is a zero block;
  * one draw per level, shared by every subproblem of that level (the paper
    builds F-hat^(q-1) on one set of random variables per level);
  * the (1 - kappa)^-1 factor appears at every level when ``kappa_scale`` is
    on (it is in eq. recursive-random-formula); the deterministic F^(Q) of
    Section 3 is the same recursion with s = 1, pi = id;
  * inputs whose sizes are not m * prod(b) are zero padded (end of
    Section 2.1.1); padding never changes the cropped result in exact
    arithmetic.  Rectangular A (M x K) and B (K x N) are allowed.

``arith`` selects the working precision of the block combinations: "f64"
(default) or "f32" (inputs, coefficients and every sum rounded to float32;
numpy evaluates each elementwise product and sum with one IEEE rounding and
never fuses them).  The leaf product is computed in float64 and, for "f32",
rounded once to float32.  ``leaf`` may replace the leaf product (tests use it
to read the leaf operands or to inject given leaf products).

Pins: exact A B on integer inputs for exact schemes and every draw/mode/depth
(the remark after Definition 2); E[F-hat] = A B by exact enumeration
(Propositions 3 and 6, tests/test_oracle_expectation.py); the bound of
Proposition 4(ii); the O(lambda) error slope of approximate schemes.
"""

import numpy as np

from . import tensors
from .draws import draw, fold


def standard(A, B):
    """The standard O(n^3) product used as truth: float64, or int64 for integer inputs."""
    if np.issubdtype(A.dtype, np.integer) and np.issubdtype(B.dtype, np.integer):
        return A.astype(np.int64) @ B.astype(np.int64)
    return A.astype(np.float64) @ B.astype(np.float64)


def _seq_sum(terms, shape, dt):
    acc = None
    for coef, blk in terms:
        t = coef * blk
        acc = t if acc is None else acc + t
    if acc is None:
        return np.zeros(shape, dtype=dt)
    return acc


def padded_dims(M, K, N, schemes, leaf_dims=None):
    """Smallest zero-padded sizes M_p = m_M prod(b1), K_p = m_K prod(b2), N_p = m_N prod(b3)."""
    p1 = int(np.prod([tensors.dims(*s)[0] for s in schemes])) if schemes else 1
    p2 = int(np.prod([tensors.dims(*s)[1] for s in schemes])) if schemes else 1
    p3 = int(np.prod([tensors.dims(*s)[2] for s in schemes])) if schemes else 1
    if leaf_dims is None:
        leaf_dims = (-(-M // p1), -(-K // p2), -(-N // p3))
    mM, mK, mN = leaf_dims
    if mM * p1 < M or mK * p2 < K or mN * p3 < N:
        raise ValueError("leaf dims too small")
    return mM * p1, mK * p2, mN * p3


def rbc(A, B, schemes, level_draws, kappa_scale=True, arith="f64", leaf=None, leaf_dims=None):
    """C = F-hat^(Q)(A, B) for Q = len(schemes), one draw per level (top first).

    schemes:     list of (U, V, W), top level first.
    level_draws: list of (s1, s2, s3, p1, p2, p3), one per level.
    """
    if len(schemes) != len(level_draws):
        raise ValueError("one draw per level")
    dt = np.float32 if arith == "f32" else np.float64
    M, K = A.shape
    K2, N = B.shape
    if K != K2:
        raise ValueError("inner dimensions differ")
    Mp, Kp, Np = padded_dims(M, K, N, schemes, leaf_dims)
    Ap = np.zeros((Mp, Kp), dtype=dt)
    Bp = np.zeros((Kp, Np), dtype=dt)
    Ap[:M, :K] = A.astype(dt)
    Bp[:K, :N] = B.astype(dt)

    folded = []
    for (U, V, W), dr in zip(schemes, level_draws):
        c = 1.0
        if kappa_scale:
            c = 1.0 / (1.0 - float(tensors.kappa(U, V, W)))
        Uh, Vh, Wh = fold(U, V, W, dr, c)
        folded.append((Uh.astype(dt), Vh.astype(dt), Wh.astype(dt)))

    if leaf is None:
        if dt == np.float32:
            def leaf(S, T):
                return (S.astype(np.float64) @ T.astype(np.float64)).astype(np.float32)
        else:
            def leaf(S, T):
                return S @ T

    def rec(X, Y, d):
        if d == len(folded):
            return leaf(X, Y)
        Uh, Vh, Wh = folded[d]
        b1, b2, R = Uh.shape
        b3 = Vh.shape[1]
        h, w = X.shape[0] // b1, X.shape[1] // b2
        z = Y.shape[1] // b3
        Xb = [[X[k * h:(k + 1) * h, l * w:(l + 1) * w] for l in range(b2)] for k in range(b1)]
        Yb = [[Y[k * w:(k + 1) * w, l * z:(l + 1) * z] for l in range(b3)] for k in range(b2)]
        P = []
        for r in range(R):
            S = _seq_sum([(Uh[k, l, r], Xb[k][l]) for k in range(b1) for l in range(b2)
                          if Uh[k, l, r] != 0], (h, w), dt)
            T = _seq_sum([(Vh[k, l, r], Yb[k][l]) for k in range(b2) for l in range(b3)
                          if Vh[k, l, r] != 0], (w, z), dt)
            P.append(rec(S, T, d + 1))
        C = np.empty((b1 * h, b3 * z), dtype=dt)
        for i in range(b1):
            for j in range(b3):
                C[i * h:(i + 1) * h, j * z:(j + 1) * z] = _seq_sum(
                    [(Wh[i, j, r], P[r]) for r in range(R) if Wh[i, j, r] != 0], (h, z), dt)
        return C

    return rec(Ap, Bp, 0)[:M, :N]


def seeded_draws(schemes, seed, mode="full"):
    out = []
    for d, s in enumerate(schemes):
        b1, b2, b3, _ = tensors.dims(*s)
        out.append(draw(seed, d, b1, b2, b3, mode))
    return out


def rbc_seeded(A, B, schemes, seed, mode="full", kappa_scale=None, arith="f64", leaf=None, leaf_dims=None):
    """F-hat^(Q) with the draws of ``seed`` (kappa_scale defaults to on unless mode is "none")."""
    if kappa_scale is None:
        kappa_scale = mode != "none"
    return rbc(A, B, schemes, seeded_draws(schemes, seed, mode), kappa_scale, arith, leaf, leaf_dims)


def leaf_operands(A, B, schemes, level_draws, kappa_scale=True, arith="f64", leaf_dims=None):
    """The leaf operands (S, T) in visiting order (r_0 slowest, r_{Q-1} fastest)."""
    seen = []

    def rec_leaf(S, T):
        seen.append((S.copy(), T.copy()))
        return np.zeros((S.shape[0], T.shape[1]), dtype=S.dtype)

    rbc(A, B, schemes, level_draws, kappa_scale, arith, rec_leaf, leaf_dims)
    return seen


def combine(products, M, N, K, schemes, level_draws, kappa_scale=True, arith="f64", leaf_dims=None):
    """C from given leaf products (same order as ``leaf_operands``), i.e. the W side alone."""
    dt = np.float32 if arith == "f32" else np.float64
    it = iter(products)

    def give(S, T):
        return np.asarray(next(it), dtype=dt)

    A = np.zeros((M, K), dtype=dt)
    B = np.zeros((K, N), dtype=dt)
    return rbc(A, B, schemes, level_draws, kappa_scale, arith, give, leaf_dims)


def rel_err(C, ref):
    C = np.asarray(C, np.float64)
    ref = np.asarray(ref, np.float64)
    return float(np.linalg.norm(C - ref) / np.linalg.norm(ref))


def apa_ebc(A, B, levels_at, eps, seed=0, mode="none", kappa_scale=None, leaf_dims=None):
    """The exact product from an approximate scheme (Section 1, eq. APA-to-EBC):
    sum_i alpha_i F(A, B; eps_i), F the recursion over the level tensors
    levels_at(eps_i) with the draws of (seed, mode), which depend only on the levels'
    block shapes and so are the same for every eps_i.  alpha from
    schemes.apa_ebc_weights; the terms are added in the order of eps, in f64."""
    from . import schemes
    alpha = schemes.apa_ebc_weights(eps)
    out = None
    for a, e in zip(alpha, eps):
        Y = rbc_seeded(A, B, levels_at(e), seed, mode, kappa_scale=kappa_scale, leaf_dims=leaf_dims)
        out = a * Y if out is None else out + a * Y
    return out
