"""The 6-way tensors X and Y and the scalar quantities built from them.

  Y[k,l,k',l',i,j] = sum_r U[k,l,r] V[k',l',r] W[i,j,r]        (eq. def-y)
  X[k,l,k',l',i,j] = delta(k,i) delta(l',j) delta(l,k')          (eq. def-x)
  tau   = ||Y - X||_F                                            (Definition 1)
  kappa = (b1 b2 b3)^-1 sum_{i,l,j} (1 - sum_r U[i,l,r] V[l,j,r] W[i,j,r])
                                                                 (eq. epsilon-def)
  q     = sqrt(sum_r ||U_r||^2 ||V_r||^2 ||W_r||^2)              (eq. square-root-of-sum)

Y is formed by brute force over every index 6-tuple (a plain einsum).  Integer
tensors are evaluated in int64, which is exact.  The rectangular kappa divides
by b1*b2*b3, the number of (i,l,j) triples; for b1 = b2 = b3 = n this is n^3.

Pins: Brent residual 0 for Strassen/Laderman (also checked through plain
matrix products), the R=1 all-ones remark (kappa = 0, tau = sqrt(56) for
n = 2), ||X|| = n^(3/2), Strassen q = sqrt(32) ("approximately 6" in
Example 13), and the corrected |kappa| <= n^(-3/2) tau (tests/test_oracle_tensors.py).
"""

import numpy as np


def _dtype(*Ts):
    return np.int64 if all(np.issubdtype(np.asarray(T).dtype, np.integer) for T in Ts) else np.float64


def brent_Y(U, V, W):
    dt = _dtype(U, V, W)
    return np.einsum("klr,mnr,ijr->klmnij", np.asarray(U, dt), np.asarray(V, dt), np.asarray(W, dt))


def brent_X(b1, b2, b3, dtype=np.int64):
    X = np.zeros((b1, b2, b2, b3, b1, b3), dtype=dtype)
    for i in range(b1):
        for l in range(b2):
            for j in range(b3):
                X[i, l, l, j, i, j] = 1
    return X


def dims(U, V, W):
    b1, b2, R = np.shape(U)
    b2v, b3, Rv = np.shape(V)
    b1w, b3w, Rw = np.shape(W)
    if not (b2 == b2v and b1 == b1w and b3 == b3w and R == Rv == Rw):
        raise ValueError("inconsistent scheme shapes")
    return b1, b2, b3, R


def residual_tensor(U, V, W):
    b1, b2, b3, _ = dims(U, V, W)
    Y = brent_Y(U, V, W)
    return Y - brent_X(b1, b2, b3, Y.dtype)


def tau(U, V, W):
    D = residual_tensor(U, V, W)
    if D.dtype == np.int64:
        return float(np.sqrt(float(np.sum(D * D))))
    return float(np.sqrt(np.sum(D * D)))


def tau_squared_exact(U, V, W):
    """||Y - X||^2 as an exact Python integer (integer schemes only)."""
    D = residual_tensor(U, V, W)
    if D.dtype != np.int64:
        raise TypeError("exact residual needs integer tensors")
    return int(np.sum(D * D))


def kappa(U, V, W):
    """kappa of eq. epsilon-def; exact (a Fraction) for integer tensors."""
    b1, b2, b3, _ = dims(U, V, W)
    dt = _dtype(U, V, W)
    U = np.asarray(U, dt)
    V = np.asarray(V, dt)
    W = np.asarray(W, dt)
    total = 0
    for i in range(b1):
        for l in range(b2):
            for j in range(b3):
                total += 1 - np.sum(U[i, l, :] * V[l, j, :] * W[i, j, :])
    if dt == np.int64:
        from fractions import Fraction
        return Fraction(int(total), b1 * b2 * b3)
    return float(total) / (b1 * b2 * b3)


def ynorm(U, V, W):
    Y = brent_Y(U, V, W).astype(np.float64)
    return float(np.sqrt(np.sum(Y * Y)))


def q_uvw(U, V, W):
    U = np.asarray(U, np.float64)
    V = np.asarray(V, np.float64)
    W = np.asarray(W, np.float64)
    nu = np.sum(U * U, axis=(0, 1))
    nv = np.sum(V * V, axis=(0, 1))
    nw = np.sum(W * W, axis=(0, 1))
    return float(np.sqrt(np.sum(nu * nv * nw)))


def bc_evaluate(U, V, W, A, B):
    """Plain bilinear computation of eq. bilinear-computation-block (no randomization).

    Used by the tests as an independent check of a scheme: for an exact scheme
    it must equal A @ B.  A is (b1*m) x (b2*p), B is (b2*p) x (b3*q).
    """
    b1, b2, b3, R = dims(U, V, W)
    h, w = A.shape[0] // b1, A.shape[1] // b2
    w2, z = B.shape[0] // b2, B.shape[1] // b3
    assert w == w2
    Ab = [[A[k * h:(k + 1) * h, l * w:(l + 1) * w] for l in range(b2)] for k in range(b1)]
    Bb = [[B[k * w:(k + 1) * w, l * z:(l + 1) * z] for l in range(b3)] for k in range(b2)]
    C = np.zeros((b1 * h, b3 * z), dtype=np.result_type(A, B, U))
    for r in range(R):
        S = sum(U[k, l, r] * Ab[k][l] for k in range(b1) for l in range(b2))
        T = sum(V[k, l, r] * Bb[k][l] for k in range(b2) for l in range(b3))
        P = S @ T
        for i in range(b1):
            for j in range(b3):
                C[i * h:(i + 1) * h, j * z:(j + 1) * z] += W[i, j, r] * P
    return C
