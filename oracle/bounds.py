"""Error bounds of Section 2 as plain formulas.

  prop4_i     ||f(A,B) - AB||      <= ||A|| ||B|| tau                       (Prop. 4(i))
  prop4_ii    ||f-hat(A,B) - AB||  <= ||A|| ||B|| ||(1-kappa)^-1 Y - X||   (Prop. 4(ii), middle form)
  prop5       |eta| mu^2 ||Y||     <= 2 mu^2 (n^-p tau + n^(3/2-p)) tau     (Prop. 5)
  prop8       1.01 (4n + R - 1) sqrt(R) eps mu^2 q                          (Prop. 8)
  prop9/10    1.01 (4n + m + R - 2) sqrt(R) eps mu^2 q [(1-kappa)^-1]       (Props. 9, 10)
  example13   10 * 1.01 * (4*2 + 50000 + 7 - 2) * sqrt(7) * 2^-p * 1e-8     (Example 13)

Reading: the proof of Prop. 5 bounds ||z||_1 by sqrt(n) ||z|| although z has
n^3 entries; the valid step is ||z||_1 <= n^(3/2) ||z||, so
|kappa| <= n^(-3/2) tau and Prop. 5 holds with p = 3/2 (the printed p = 5/2 is
too small: scaling W of an exact scheme by (1 + delta) gives |kappa| = delta
while n^(-5/2) tau = delta / 2 for n = 2).  ``p`` defaults to the corrected
3/2; p = 5/2 reproduces the paper's printed numbers (Example 13: 0.0024).
The hypotheses "(4n + m + R - 2) eps <= 1.01" of Props. 9-12 are read as
"<= 0.01", the precondition of Prop. 8 and of Golub & Van Loan Lemma 2.7.1.

Pins (tests/test_oracle_decimal2_bounds.py, tests/test_oracle_tensors.py):
Prop. 4(ii) and the corrected kappa bound hold on every tested draw;
example13(p=2.5) reproduces the printed 0.0024; prop5 holds on perturbed
Strassen and Laderman schemes and equals its closed form on the scaled-W
family, where the printed constant (p = 5/2) fails for n = 3.
"""

import numpy as np

from . import tensors


def eta(kappa):
    return 1.0 / (1.0 - float(kappa)) - 1.0


def prop4_i(normA, normB, tau):
    return normA * normB * tau


def prop4_ii(normA, normB, U, V, W):
    b1, b2, b3, _ = tensors.dims(U, V, W)
    k = float(tensors.kappa(U, V, W))
    Y = tensors.brent_Y(U, V, W).astype(np.float64)
    X = tensors.brent_X(b1, b2, b3, np.float64)
    return normA * normB * float(np.linalg.norm((Y / (1.0 - k) - X).ravel()))


def kappa_bound(n, tau, p=1.5):
    return n ** (-p) * tau


def prop5(mu, n, tau, p=1.5):
    return 2.0 * mu * mu * (n ** (-p) * tau + n ** (1.5 - p)) * tau


def prop8(n, R, eps, mu, q):
    return 1.01 * (4 * n + R - 1) * np.sqrt(R) * eps * mu * mu * q


def prop9(n, m, R, eps, mu, q, kappa=0.0):
    return 1.01 * (4 * n + m + R - 2) * np.sqrt(R) * eps * mu * mu * q / (1.0 - float(kappa))


def example13(p=2.5):
    return 10 * 1.01 * (4 * 2 + 50000 + 7 - 2) * np.sqrt(7) / 2 ** p * 1e-8
