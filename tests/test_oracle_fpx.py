"""Pins of the FPX storage-format oracle (Section V-A: X-bit byte-aligned floats with
FP32's 8-bit exponent and bias, X - 9 significand bits, IEEE round-to-nearest-even;
FP32 itself for X = 32).  Fixed by numpy's IEEE FP32 conversion (X = 32), torch's
bfloat16 conversion (X = 16 has bfloat16's layout), an exact rational
nearest-representable search for every X, and the round-trip error bound."""
from fractions import Fraction

import numpy as np
import pytest

import oracle

M_MAX = {b: b - 9 for b in oracle.FPX_BITS}


def edge_values(rng, n=4000):
    """Random magnitudes over the whole FP32 range and beyond, plus specials."""
    x = rng.standard_normal(n) * 10.0 ** rng.integers(-48, 41, n)
    special = [0.0, -0.0, np.inf, -np.inf, 2.0 ** -126, 2.0 ** -149, 2.0 ** -150, 3 * 2.0 ** -151,
               2.0 ** 128, (2 - 2.0 ** -24) * 2.0 ** 127, (2 - 2.0 ** -25) * 2.0 ** 127, 1e-320, -5e-324,
               1.0 + 2.0 ** -24, 1.0 + 3 * 2.0 ** -24, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8]
    return np.concatenate([x, special])


def test_fpx32_is_ieee_fp32():
    x = edge_values(np.random.default_rng(0))
    with np.errstate(over="ignore"):
        ref = x.astype(np.float32)
    got = oracle.fpx_round(x, 32)
    assert np.array_equal(got, ref.astype(np.float64))
    assert np.array_equal(oracle.fpx_encode(x, 32).view(np.uint32), ref.view(np.uint32))
    n = np.array([np.nan, -np.nan])
    assert np.all(np.isnan(oracle.fpx_round(n, 32)))


def test_fpx16_is_bfloat16():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    x32 = (rng.standard_normal(20000) * 10.0 ** rng.integers(-40, 38, 20000)).astype(np.float32)
    x32 = np.concatenate([x32, np.float32([0, 2.0 ** -126, 2.0 ** -133, 3.3e38, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8])])
    ref = torch.from_numpy(x32).to(torch.bfloat16)
    got = oracle.fpx_encode(x32.astype(np.float64), 16).view(np.uint16)
    assert np.array_equal(got, ref.view(torch.int16).numpy().view(np.uint16))


def nearest_fpx(x: float, bits: int) -> float:
    """Exact search: the FPX value nearest to x, ties to the even significand;
    values at or past max + ulp/2 become infinite."""
    if x != x or x in (np.inf, -np.inf) or x == 0:
        return x
    m = bits - 9
    a = Fraction(abs(x))
    e = a.numerator.bit_length() - a.denominator.bit_length()
    while Fraction(2) ** e > a:
        e -= 1
    while Fraction(2) ** (e + 1) <= a:
        e += 1
    e = max(e, -126)
    ulp = Fraction(2) ** (e - m)
    k = a // ulp
    lo, hi = k * ulp, (k + 1) * ulp
    d_lo, d_hi = a - lo, hi - a
    pick = lo if (d_lo < d_hi or (d_lo == d_hi and k % 2 == 0)) else hi
    if pick >= Fraction(2) ** 128:
        return float(np.copysign(np.inf, x))
    return float(np.copysign(float(pick), x))


@pytest.mark.parametrize("bits", oracle.FPX_BITS)
def test_fpx_matches_exact_nearest(bits):
    rng = np.random.default_rng(bits)
    x = edge_values(rng, 600)
    # exact ties of this format: halfway points between neighbours
    m = bits - 9
    ties = [1.0 + 2.0 ** -(m + 1), 1.0 + 3 * 2.0 ** -(m + 1), (1 + 2.0 ** -m) * 2.0 ** -126 / 2,
            2.0 ** (-126 - m - 1), 3 * 2.0 ** (-126 - m - 1), (2 - 2.0 ** -(m + 1)) * 2.0 ** 127]
    x = np.concatenate([x, ties, -np.array(ties)])
    got = oracle.fpx_round(x, bits)
    ref = np.array([nearest_fpx(float(v), bits) for v in x])
    assert np.array_equal(got, ref), [(v, g, r) for v, g, r in zip(x, got, ref) if g != r][:5]


@pytest.mark.parametrize("bits", oracle.FPX_BITS)
def test_fpx_roundtrip_bound_and_monotone(bits):
    rng = np.random.default_rng(100 + bits)
    x = rng.standard_normal(20000) * 10.0 ** rng.integers(-30, 30, 20000)
    enc = oracle.fpx_encode(x, bits)
    assert enc.size == x.size * bits // 8
    y = oracle.fpx_decode(enc, bits, x.size)
    assert np.array_equal(y, oracle.fpx_round(x, bits))
    assert np.all(np.abs(y - x) <= 2.0 ** -(bits - 8) * np.abs(x))     # half an ulp: 2^-(m+1)
    s = np.sort(x)
    assert np.all(np.diff(oracle.fpx_round(s, bits)) >= 0)
