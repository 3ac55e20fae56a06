"""Pins of the FP8 (E4M3) arithmetic of the oracle against the format's
definition: every finite code round-trips, ties go to the even code, the
per-tensor / per-row exponents are the smallest that keep values finite,
rounding error stays within half a unit in the last place, and products of
values exact in E4M3 are exact."""
import numpy as np
import pytest

from oracle import fp8


def decode(b):
    """Value of E4M3 code b from the bit fields (bias 7, 3 mantissa bits)."""
    s, e, m = (b >> 7) & 1, (b >> 3) & 15, b & 7
    if e == 15 and m == 7:
        return None                       # NaN code
    v = m * 2.0 ** -9 if e == 0 else (1 + m / 8.0) * 2.0 ** (e - 7)
    return -v if s else v


CODES = [b for b in range(256) if decode(b) is not None]


def test_every_finite_code_round_trips():
    vals = np.array([decode(b) for b in CODES])
    assert np.array_equal(fp8.e4m3(vals), vals)
    assert max(vals) == 448.0 and min(v for v in vals if v > 0) == 2.0 ** -9


def test_ties_round_to_even_codes():
    pos = sorted({decode(b) for b in range(128) if decode(b) is not None})
    code = {decode(b): b for b in range(128) if decode(b) is not None}
    for lo, hi in zip(pos[:-1], pos[1:]):
        mid = 0.5 * (lo + hi)
        want = lo if code[lo] % 2 == 0 else hi
        assert fp8.e4m3(mid) == want, (lo, hi)
        assert fp8.e4m3(-mid) == -want


def test_scale_exponent_is_smallest_that_fits():
    assert fp8.scale_exp(0.0) == 0
    assert fp8.scale_exp(448.0) == 0
    assert fp8.scale_exp(np.nextafter(448.0, 1e9)) == 1
    assert fp8.scale_exp(1.0) == -8
    assert fp8.scale_exp(1.75) == -8
    assert fp8.scale_exp(np.nextafter(1.75, 9.0)) == -7
    rng = np.random.default_rng(3)
    for m in np.exp(rng.uniform(-30, 30, 500)):
        e = fp8.scale_exp(m)
        assert m * 2.0 ** -e <= 448.0 < m * 2.0 ** -(e - 1)


def test_rounding_error_within_half_ulp():
    rng = np.random.default_rng(4)
    x = rng.uniform(-448, 448, 20000) * 2.0 ** rng.integers(-12, 1, 20000)
    q = fp8.e4m3(x)
    a = np.abs(x)
    ulp = np.where(a >= 2.0 ** -6, 2.0 ** (np.floor(np.log2(np.maximum(a, 1e-300))) - 3), 2.0 ** -9)
    assert np.all(np.abs(q - x) <= 0.5 * ulp * (1 + 1e-12))


def test_fp8_matmul_exact_on_representable_inputs():
    rng = np.random.default_rng(5)
    a = rng.integers(-8, 9, (7, 64)).astype(np.float64)     # small integers: exact in E4M3
    w = rng.integers(-8, 9, (16, 64)).astype(np.float64)
    got = fp8.matmul_t(a, w)
    assert np.array_equal(got, a @ w.T)


def test_fp8_matmul_close_to_exact():
    rng = np.random.default_rng(6)
    a = rng.standard_normal((5, 256))
    w = rng.standard_normal((32, 256)) * 0.05
    got, ref = fp8.matmul_t(a, w), a @ w.T
    # each operand carries at most 2^-4 relative rounding error
    bound = (np.abs(a) @ np.abs(w).T) * (2 * 2.0 ** -4 + 2.0 ** -8)
    assert np.all(np.abs(got - ref) <= bound)
