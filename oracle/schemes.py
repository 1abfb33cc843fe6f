"""Bilinear-computation tensors (U, V, W) used by the oracle.

Convention (Section 1, eq. bilinear-computation): for a scheme with block
partition <b1, b2, b3> and R products,
  U[k, l, r]   multiplies block A_kl   (k < b1, l < b2),
  V[k', l', r] multiplies block B_k'l' (k' < b2, l' < b3),
  W[i, j, r]   weights product r in block C_ij (i < b1, j < b3).
The paper states the square case b1 = b2 = b3 = n; the rectangular case is the
natural extension the paper's footnote to Section 2.1 anticipates.

Pins (tests/test_oracle_schemes.py): Strassen and Laderman satisfy the Brent
equations (eq. requirement) exactly in int64 AND, independently, reproduce
np.matmul on random integer matrices when evaluated as a plain bilinear
computation; the perturbed scheme has tau = Theta(sigma); the rank-10 <3,2,2>
approximate scheme has, in exact rational arithmetic, a Brent residual with no
constant term that halves with lam.
"""

import math

import numpy as np


def strassen():
    """Strassen's rank-7 scheme for 2x2 blocks (cited in Section 1).

    The form is the one in Strassen (1969) as written in Golub & Van Loan,
    Section 1.3.11 (the paper's Example 7 follows that book's setup):
      P1 = (A11 + A22)(B11 + B22)   P5 = (A11 + A12) B22
      P2 = (A21 + A22) B11          P6 = (A21 - A11)(B11 + B12)
      P3 = A11 (B12 - B22)          P7 = (A12 - A22)(B21 + B22)
      P4 = A22 (B21 - B11)
      C11 = P1 + P4 - P5 + P7,  C12 = P3 + P5,
      C21 = P2 + P4,            C22 = P1 - P2 + P3 + P6.
    Returns int64 arrays of shapes (2,2,7), (2,2,7), (2,2,7).
    """
    # (coef, row, col), 1-based, per product
    a = [[(1, 1, 1), (1, 2, 2)], [(1, 2, 1), (1, 2, 2)], [(1, 1, 1)], [(1, 2, 2)],
         [(1, 1, 1), (1, 1, 2)], [(1, 2, 1), (-1, 1, 1)], [(1, 1, 2), (-1, 2, 2)]]
    b = [[(1, 1, 1), (1, 2, 2)], [(1, 1, 1)], [(1, 1, 2), (-1, 2, 2)], [(1, 2, 1), (-1, 1, 1)],
         [(1, 2, 2)], [(1, 1, 1), (1, 1, 2)], [(1, 2, 1), (1, 2, 2)]]
    c = {(1, 1): [(1, 1), (1, 4), (-1, 5), (1, 7)], (1, 2): [(1, 3), (1, 5)],
         (2, 1): [(1, 2), (1, 4)], (2, 2): [(1, 1), (-1, 2), (1, 3), (1, 6)]}
    return _assemble(2, 2, 2, 7, a, b, c)


def laderman():
    """Laderman's rank-23 scheme for 3x3 blocks (Laderman 1976, cited in Section 1).

    Products m1..m23 and outputs as published:
      m1 = (a11+a12+a13-a21-a22-a32-a33) b22
      m2 = (a11-a21)(-b12+b22)
      m3 = a22 (-b11+b12+b21-b22-b23-b31+b33)
      m4 = (-a11+a21+a22)(b11-b12+b22)
      m5 = (a21+a22)(-b11+b12)
      m6 = a11 b11
      m7 = (-a11+a31+a32)(b11-b13+b23)
      m8 = (-a11+a31)(b13-b23)
      m9 = (a31+a32)(-b11+b13)
      m10 = (a11+a12+a13-a22-a23-a31-a32) b23
      m11 = a32 (-b11+b13+b21-b22-b23-b31+b32)
      m12 = (-a13+a32+a33)(b22+b31-b32)
      m13 = (a13-a33)(b22-b32)
      m14 = a13 b31
      m15 = (a32+a33)(-b31+b32)
      m16 = (-a13+a22+a23)(b23+b31-b33)
      m17 = (a13-a23)(b23-b33)
      m18 = (a22+a23)(-b31+b33)
      m19 = a12 b21,  m20 = a23 b32,  m21 = a21 b13,  m22 = a31 b12,  m23 = a33 b33
      c11 = m6+m14+m19             c12 = m1+m4+m5+m6+m12+m14+m15
      c13 = m6+m7+m9+m10+m14+m16+m18
      c21 = m2+m3+m4+m6+m14+m16+m17  c22 = m2+m4+m5+m6+m20
      c23 = m14+m16+m17+m18+m21     c31 = m6+m7+m8+m11+m12+m13+m14
      c32 = m12+m13+m14+m15+m22     c33 = m6+m7+m8+m9+m23
    """
    A = [
        "+11 +12 +13 -21 -22 -32 -33", "+11 -21", "+22", "-11 +21 +22", "+21 +22", "+11",
        "-11 +31 +32", "-11 +31", "+31 +32", "+11 +12 +13 -22 -23 -31 -32", "+32",
        "-13 +32 +33", "+13 -33", "+13", "+32 +33", "-13 +22 +23", "+13 -23", "+22 +23",
        "+12", "+23", "+21", "+31", "+33"]
    B = [
        "+22", "-12 +22", "-11 +12 +21 -22 -23 -31 +33", "+11 -12 +22", "-11 +12", "+11",
        "+11 -13 +23", "+13 -23", "-11 +13", "+23", "-11 +13 +21 -22 -23 -31 +32",
        "+22 +31 -32", "+22 -32", "+31", "-31 +32", "+23 +31 -33", "+23 -33", "-31 +33",
        "+21", "+32", "+13", "+12", "+33"]
    Cmap = {
        (1, 1): [6, 14, 19], (1, 2): [1, 4, 5, 6, 12, 14, 15], (1, 3): [6, 7, 9, 10, 14, 16, 18],
        (2, 1): [2, 3, 4, 6, 14, 16, 17], (2, 2): [2, 4, 5, 6, 20], (2, 3): [14, 16, 17, 18, 21],
        (3, 1): [6, 7, 8, 11, 12, 13, 14], (3, 2): [12, 13, 14, 15, 22], (3, 3): [6, 7, 8, 9, 23]}

    def parse(s):
        out = []
        for tok in s.split():
            out.append((1 if tok[0] == "+" else -1, int(tok[1]), int(tok[2])))
        return out

    a = [parse(s) for s in A]
    b = [parse(s) for s in B]
    c = {ij: [(1, r) for r in rs] for ij, rs in Cmap.items()}
    return _assemble(3, 3, 3, 23, a, b, c)


def naive(b1, b2, b3):
    """The standard algorithm written as a BC: one product a_il b_lj per (i, l, j).

    R = b1 b2 b3; exact by construction (c_ij = sum_l a_il b_lj, eq. bilinear-computation).
    Product index r = (i * b2 + l) * b3 + j.
    """
    R = b1 * b2 * b3
    U = np.zeros((b1, b2, R), dtype=np.int64)
    V = np.zeros((b2, b3, R), dtype=np.int64)
    W = np.zeros((b1, b3, R), dtype=np.int64)
    for i in range(b1):
        for l in range(b2):
            for j in range(b3):
                r = (i * b2 + l) * b3 + j
                U[i, l, r] = 1
                V[l, j, r] = 1
                W[i, j, r] = 1
    return U, V, W


def rank_one_all_ones(n=2):
    """The R = 1, all-ones scheme of the remark after Proposition 5 (kappa = 0, large tau)."""
    one = np.ones((n, n, 1), dtype=np.int64)
    return one.copy(), one.copy(), one.copy()


def aux_words(aux_seed):
    """Endless raw 64-bit words of Philox4x64-10 with key (aux_seed, 1), blocks at
    counters (1,0,0,0), (2,0,0,0), ... (numpy's Philox started at counter 0)."""
    key = np.array([int(aux_seed) & 0xFFFFFFFFFFFFFFFF, 1], dtype=np.uint64)
    g = np.random.Philox(key=key, counter=np.zeros(4, dtype=np.uint64))
    while True:
        for w in g.random_raw(64):
            yield int(w)


def open_unit(word):
    """u = (floor(word / 2^12) + 1/2) 2^-52, a double in (0, 1) (exact)."""
    return (float(word >> 12) + 0.5) * 2.0 ** -52


def box_muller(words):
    """One standard normal from two words: sqrt(-2 ln u1) cos(2 pi u2) (Box and Muller 1958)."""
    u1 = open_unit(next(words))
    u2 = open_unit(next(words))
    return math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * u2)


def perturbed(U, V, W, sigma, aux_seed, n_zero=5):
    """Approximate scheme of Section 3.1: perturb an exact scheme.

    For each of the three tensors independently: add i.i.d. N(0, sigma^2) noise
    to every entry equal to 1, and to n_zero entries equal to 0 chosen uniformly
    without replacement.  The paper uses sigma = 1e-3 and n_zero = 5.  Entries
    equal to -1 are left unchanged (the paper names entries equal to 1).

    Random numbers (a reading: the paper does not say how they are drawn): the
    words of ``aux_words(aux_seed)`` in order; per tensor (U, V, W): one normal
    (``box_muller``) per entry equal to 1 in row-major order; then the picks:
    the row-major list of zero positions, shuffled partially by Fisher-Yates
    (for i < n_zero: j = i + floor(word * (nz - i) / 2^64), swap items i and j),
    the first n_zero items picked; then one normal per pick in pick order.  An
    entry x becomes x + sigma * z, each operation rounded to double.
    """
    words = aux_words(aux_seed)
    out = []
    for T in (U, V, W):
        T = np.asarray(T, dtype=np.float64).copy()
        flat = T.reshape(-1)
        zeros = [i for i in range(flat.size) if flat[i] == 0.0]
        for i in range(flat.size):
            if flat[i] == 1.0:
                noise = sigma * box_muller(words)
                flat[i] = float(flat[i]) + noise
        picks = min(n_zero, len(zeros))
        for i in range(picks):
            j = i + ((next(words) * (len(zeros) - i)) >> 64)
            zeros[i], zeros[j] = zeros[j], zeros[i]
        for i in range(picks):
            noise = sigma * box_muller(words)
            flat[zeros[i]] = float(flat[zeros[i]]) + noise
        out.append(T)
    return tuple(out)


def apa322(lam):
    """Rank-10 approximate scheme for <3,2,2> blocks (the APA family of Section 1,
    eq. APA-y: Y(lam) = X + O(lam), coefficients 1/lam in W).

    The paper names such a scheme (Bini et al. 1979) without printing it.  This one
    follows that construction: the 3x2 A is split into two 2x2 problems that each
    miss one block (rows 1, 2 without A22, and rows 3, 2 without A21), each
    computed approximately with five products, and the two share C's middle row:
      P1  = (A12 + lam A11)(B12 + lam B22)   P6  = (A31 + lam A32)(B22 + lam B12)
      P2  = (A21 + lam A11) B11              P7  = (A22 + lam A32) B21
      P3  = A12 B12                          P8  = A31 B22
      P4  = A21 (B11 + B12 + lam B21)        P9  = A22 (B21 + B22 + lam B11)
      P5  = (A12 + A21)(B12 + lam B21)       P10 = (A31 + A22)(B22 + lam B11)
      C11 = (P2 - P3 - P4 + P5) / lam        C12 = (P1 - P3) / lam
      C21 = P2 + P7                          C22 = P5 - P3 + P10 - P8
      C31 = (P7 - P8 - P9 + P10) / lam       C32 = (P6 - P8) / lam
    C11 and C31 are exact; the other four carry an O(lam) error.  Returns float64
    arrays of shapes (3,2,10), (2,2,10), (3,2,10).
    """
    lam = float(lam)
    if not lam > 0.0:
        raise ValueError("lam must be positive")
    a = [[(1.0, 1, 2), (lam, 1, 1)], [(1.0, 2, 1), (lam, 1, 1)], [(1.0, 1, 2)], [(1.0, 2, 1)],
         [(1.0, 1, 2), (1.0, 2, 1)],
         [(1.0, 3, 1), (lam, 3, 2)], [(1.0, 2, 2), (lam, 3, 2)], [(1.0, 3, 1)], [(1.0, 2, 2)],
         [(1.0, 3, 1), (1.0, 2, 2)]]
    b = [[(1.0, 1, 2), (lam, 2, 2)], [(1.0, 1, 1)], [(1.0, 1, 2)], [(1.0, 1, 1), (1.0, 1, 2), (lam, 2, 1)],
         [(1.0, 1, 2), (lam, 2, 1)],
         [(1.0, 2, 2), (lam, 1, 2)], [(1.0, 2, 1)], [(1.0, 2, 2)], [(1.0, 2, 1), (1.0, 2, 2), (lam, 1, 1)],
         [(1.0, 2, 2), (lam, 1, 1)]]
    il = 1.0 / lam
    c = {(1, 1): [(il, 2), (-il, 3), (-il, 4), (il, 5)], (1, 2): [(il, 1), (-il, 3)],
         (2, 1): [(1.0, 2), (1.0, 7)], (2, 2): [(1.0, 5), (-1.0, 3), (1.0, 10), (-1.0, 8)],
         (3, 1): [(il, 7), (-il, 8), (-il, 9), (il, 10)], (3, 2): [(il, 6), (-il, 8)]}
    return _assemble(3, 2, 2, 10, a, b, c, dtype=np.float64)


def rotate(U, V, W):
    """The cyclic rotation of a scheme for <b1,b2,b3> into one for <b2,b3,b1>.

    The Brent equations (eq. requirement) are invariant under the cyclic shift
    A -> B, B -> C^T, C -> A^T of the three matrix roles, so U' = V, V'[k,i] = W[i,k],
    W'[j,i] = U[i,j] satisfy them whenever (U, V, W) does, with the same residual norm.
    """
    return (np.array(V, copy=True), np.ascontiguousarray(np.transpose(W, (1, 0, 2))),
            np.ascontiguousarray(np.transpose(U, (1, 0, 2))))


def apa223(lam):
    """apa322 rotated once: a rank-10 approximate scheme for <2,2,3>."""
    return rotate(*apa322(lam))


def apa232(lam):
    """apa322 rotated twice: a rank-10 approximate scheme for <2,3,2>."""
    return rotate(*apa223(lam))


def bini12(lam):
    """The three levels whose recursion is one step of a rank-1000 approximate scheme
    for 12 x 12 blocks (<3,2,2> x <2,2,3> x <2,3,2> = <12,12,12>, the Bini et al.
    construction): the list of per-level tensors, outermost first."""
    return [apa322(lam), apa223(lam), apa232(lam)]


def _assemble(b1, b2, b3, R, a, b, c, dtype=np.int64):
    U = np.zeros((b1, b2, R), dtype=dtype)
    V = np.zeros((b2, b3, R), dtype=dtype)
    W = np.zeros((b1, b3, R), dtype=dtype)
    for r in range(R):
        for coef, i, j in a[r]:
            U[i - 1, j - 1, r] = coef
        for coef, i, j in b[r]:
            V[i - 1, j - 1, r] = coef
    for (i, j), lst in c.items():
        for coef, r in lst:
            W[i - 1, j - 1, r - 1] = coef
    return U, V, W


def apa_ebc_weights(eps):
    """Weights alpha_1..alpha_{d+1} that turn an approximate scheme into an exact one
    (Section 1, eq. APA-to-EBC): sum_i alpha_i Y(eps_i) = X.

    Every entry of the error E(eps) = Y(eps) - X is a polynomial in eps with zero
    constant term and degree at most d, so the combination is exact for every such
    E exactly when sum_i alpha_i = 1 and sum_i alpha_i eps_i^k = 0 for k = 1..d:
    the (d+1) x (d+1) Vandermonde system solved here.  The eps_i must be distinct;
    d = len(eps) - 1 may exceed the scheme's own degree (the combination stays exact).
    """
    e = np.asarray(eps, dtype=np.float64)
    if e.ndim != 1 or e.size < 1:
        raise ValueError("eps must be a non-empty 1-D sequence")
    if np.unique(e).size != e.size:
        raise ValueError("eps values must be distinct")
    powers = np.vander(e, increasing=True).T  # powers[k, i] = eps_i ** k
    rhs = np.zeros(e.size)
    rhs[0] = 1.0
    return np.linalg.solve(powers, rhs)
