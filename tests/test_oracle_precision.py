"""Reduced-precision rounding helpers against torch's CPU casts (an independent implementation)."""

import numpy as np
import torch

from oracle import precision


def _values():
    g = np.random.default_rng(0)
    x = np.concatenate([g.standard_normal(20000) * 10.0 ** g.uniform(-6, 3, 20000),
                        [0.0, 1.0, -1.0, 1.00390625, 1.0078125 + 2 ** -9, 3.1e-5, 448.0, -300.0]])
    return x.astype(np.float32)


def test_bf16_matches_torch():
    x = _values()
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(precision.round_bf16(x), ref)


def test_f16_matches_torch():
    x = _values()
    x = x[np.abs(x) < 60000]
    ref = torch.from_numpy(x).to(torch.float16).to(torch.float32).numpy()
    np.testing.assert_array_equal(precision.round_f16(x), ref)


def test_e4m3_matches_torch():
    x = _values()
    x = x[np.abs(x) <= 448]
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).to(torch.float32).numpy()
    np.testing.assert_array_equal(precision.round_e4m3(x), ref)


def test_split_hi_lo_bf16_recovers_16_bits():
    x = _values()
    x = x[(np.abs(x) > 1e-30) & (np.abs(x) < 1e30)]
    hi, lo = precision.split_hi_lo(x, "bf16")
    rel = np.abs((hi.astype(np.float64) + lo) - x) / np.abs(x)
    assert rel.max() <= 2.0 ** -16


def test_leaf_exponent_keeps_scaled_values_in_range():
    rng = np.random.default_rng(1)
    for _ in range(2000):
        mx = float(np.float32(10 ** rng.uniform(-8, 8)))
        G = float(rng.integers(1, 400))
        e = precision.leaf_exponent(mx, G)
        assert G * mx * 2.0 ** e <= 32768.0 * (1 + 2.0 ** -20)  # not above 2^15 (float32 rounding)
        assert G * mx * 2.0 ** (e + 1) > 32768.0 * (1 - 1e-6)  # and the largest such power
    assert precision.leaf_exponent(0.0, 5.0) == 0


def test_path_norms_strassen_laderman():
    from oracle import schemes
    S, L = schemes.strassen(), schemes.laderman()
    gA = precision.path_norms([L, S], "A")
    assert gA.shape == (23 * 7,)
    # Laderman product 1 uses 7 blocks of A, Strassen product 1 uses 2
    assert gA[0] == 7 * 2
    assert precision.path_norms([S], "B").tolist() == [2, 1, 2, 2, 1, 2, 2]


def test_decode_e4m3_matches_torch_for_every_code():
    codes = np.arange(256, dtype=np.uint8)
    ref = torch.from_numpy(codes).view(torch.float8_e4m3fn).to(torch.float64).numpy()
    got = precision.decode_e4m3(codes)
    np.testing.assert_array_equal(np.isnan(got), np.isnan(ref))
    ok = ~np.isnan(ref)
    np.testing.assert_array_equal(got[ok], ref[ok])


def test_round_e4m3_lands_on_codes_and_is_nearest():
    vals = precision.decode_e4m3(np.arange(256, dtype=np.uint8))
    grid = np.unique(vals[~np.isnan(vals)])
    x = _values().astype(np.float64)
    x = x[np.abs(x) <= 448]
    r = precision.round_e4m3(x).astype(np.float64)
    assert np.isin(r, grid).all()
    # nearest: no grid value strictly closer than the rounded one
    idx = np.searchsorted(grid, x)
    lo = grid[np.clip(idx - 1, 0, len(grid) - 1)]
    hi = grid[np.clip(idx, 0, len(grid) - 1)]
    best = np.minimum(np.abs(x - lo), np.abs(x - hi))
    assert (np.abs(x - r) <= best).all()


def test_fp8_split_recovers_about_eight_bits():
    g = np.random.default_rng(5)
    y = (g.standard_normal(50000) * 10.0 ** g.uniform(-1.5, 2.4, 50000)).astype(np.float32)
    y = y[np.abs(y) <= 448]
    hi, lo = precision.split_e4m3_scaled(y)
    err = np.abs(hi + lo / 16.0 - y)
    normal = np.abs(y) >= 2.0 ** -6
    # hi leaves |y - hi| <= 2^-4 |y|; lo holds 16 (y - hi) to 3 fraction bits
    assert (err[normal] <= 2.0 ** -8 * np.abs(y[normal]) * (1 + 1e-12)).all()
    assert (err[~normal] <= 2.0 ** -14).all()
    assert precision.split_e4m3_scaled(np.array([448.0]))[0][0] == 448.0
