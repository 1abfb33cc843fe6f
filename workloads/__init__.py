"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module holds no arithmetic of the method: it only draws matrices with the
shapes and distributions of the paper's experiments (Section 3: Gaussian,
uniform, the adversarial pairs of Definition 14, the Hilbert matrix) and of the
benchmark configurations.  Every generator takes an explicit integer seed and
uses numpy's PCG64.  Results are float64 (or int64 for integer matrices);
callers cast to the working precision.
"""

import numpy as np


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def gaussian(shape, seed):
    return _rng(seed).standard_normal(shape)


def uniform(shape, seed, lo=0.0, hi=1.0):
    return _rng(seed).uniform(lo, hi, size=shape)


def integers(shape, seed, lo=-4, hi=4):
    """Integers uniform on {lo, ..., hi} (inclusive)."""
    return _rng(seed).integers(lo, hi + 1, size=shape, dtype=np.int64)


def scaled_gaussian(shape, seed, decades=3.0):
    """N(0,1) entries times one factor 10^U(-decades, decades) for the whole matrix."""
    g = _rng(seed)
    f = 10.0 ** g.uniform(-decades, decades)
    return g.standard_normal(shape) * f


def hilbert(n):
    i = np.arange(1, n + 1, dtype=np.float64)
    return 1.0 / (i[:, None] + i[None, :] - 1.0)


def adversarial(kind, n, seed):
    """A pair (A, B) of the adversarial types 1-3 (Definition 14), 1-based i, j."""
    g = _rng(seed)
    i = np.arange(1, n + 1)[:, None] * np.ones((1, n), dtype=np.int64)
    j = np.ones((n, 1), dtype=np.int64) * np.arange(1, n + 1)[None, :]
    small = 1.0 / n ** 2

    def draw(mask_small, big=None):
        X = g.uniform(0.0, 1.0, size=(n, n))
        X = np.where(mask_small, g.uniform(0.0, small, size=(n, n)), X)
        if big is not None:
            X = np.where(big, g.uniform(0.0, float(n ** 2), size=(n, n)), X)
        return X

    if kind == 1:
        A = draw(j > n / 2)
        B = draw(i < n / 2)
    elif kind == 2:
        A = draw(np.zeros((n, n), bool), big=(i < n / 2) & (j > n / 2))
        B = draw(j < n / 2)
    elif kind == 3:
        m = ((i < n / 2) & (j > n / 2)) | ((i >= n / 2) & (j <= n / 2))
        A = draw(m)
        B = draw(m)
    else:
        raise ValueError(kind)
    return A, B


def batch_sizes(count, seed, unit=96, kmin=2, kmax=24):
    """Sizes N_i = unit * k_i with k_i uniform on {kmin..kmax} (batched workload)."""
    return (unit * _rng(seed).integers(kmin, kmax + 1, size=count)).tolist()


def poisson_arrivals(rate, duration, seed):
    """Arrival times of a Poisson process of ``rate`` per second over ``duration`` seconds."""
    g = _rng(seed)
    t, out = 0.0, []
    while True:
        t += g.exponential(1.0 / rate)
        if t >= duration:
            return np.array(out)
        out.append(t)


def log_uniform_sizes(count, seed, lo=128, hi=4096):
    g = _rng(seed)
    return np.round(np.exp(g.uniform(np.log(lo), np.log(hi), size=count))).astype(np.int64).tolist()
