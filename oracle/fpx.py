"""FP64 oracle of the FPX storage formats (Section V-A).

TEST INFRASTRUCTURE ONLY (see the package docstring): not used by the product.

FPX, X in {56, 48, 40, 32, 24, 16}, is a byte-aligned floating-point format of X
bits: 1 sign bit, an 8-bit exponent with FP32's bias (127) and X - 9 significand
bits, rounded by IEEE-754 round-to-nearest-even; with X = 32 it is IEEE FP32.  The
format keeps FP32's range: normal magnitudes 2^-126 ... (2 - 2^-m) 2^127 with
subnormals below (m = X - 9), infinities and NaN as in IEEE-754.  Values of a
larger magnitude than the largest finite one rounds to become infinite.

Element i of an array is stored in bytes [i X/8, (i+1) X/8), little-endian.
Written from the definition on the 64-bit pattern of each FP64 value: an integer
significand M (53 bits with the hidden one), shifted right to the target precision
with round-to-nearest-even on the dropped bits.
"""
from __future__ import annotations

import numpy as np

FPX_BITS = (16, 24, 32, 40, 48, 56)


def _rshift_rne(M, sh):
    """M >> sh (uint64 arrays, 0 <= sh, sh may exceed 63), rounded to nearest even."""
    M = M.astype(np.uint64)
    sh = np.asarray(sh, dtype=np.int64)
    big = sh >= 64
    s = np.where(big, 0, sh).astype(np.uint64)
    q = np.where(big, np.uint64(0), M >> s)
    rem = np.where(big, M, M & ((np.uint64(1) << s) - np.uint64(1)))
    half = np.where(sh == 0, np.uint64(0), np.where(big, np.uint64(1) << np.uint64(63),
                                                     np.uint64(1) << (s - np.uint64(1)).clip(0)))
    # with sh >= 64 the whole of M is dropped: M < 2^53 < half, so q stays 0
    up = (sh > 0) & ((rem > half) | ((rem == half) & ((q & np.uint64(1)) == np.uint64(1))))
    up &= ~(big & (M <= half))
    return q + up.astype(np.uint64)


def fpx_codes(x, bits):
    """The X-bit codes (as uint64) of the FP64 values x."""
    assert bits in FPX_BITS
    m = bits - 9
    x = np.ascontiguousarray(x, dtype=np.float64).ravel()
    u = x.view(np.uint64)
    sign = (u >> np.uint64(63)).astype(np.uint64)
    e64 = ((u >> np.uint64(52)) & np.uint64(0x7FF)).astype(np.int64)
    f52 = u & np.uint64((1 << 52) - 1)
    M = np.where(e64 == 0, f52, f52 | np.uint64(1 << 52))
    E = np.where(e64 == 0, -1022, e64 - 1023)          # |x| = M 2^(E - 52)
    # normal target (E >= -126): keep m fraction bits; code = ((E + 126) << m) + q
    # subnormal target: q counts units of 2^(-126 - m) and is itself the code
    sh = np.where(E >= -126, 52 - m, 52 - m + (-126 - E))
    q = _rshift_rne(M, sh)
    base = np.where(E >= -126, (E + 126).clip(0), 0).astype(np.uint64)
    code = (base << np.uint64(m)) + q
    inf_code = np.uint64(255) << np.uint64(m)
    code = np.where(code >= inf_code, inf_code, code)                       # overflow -> inf
    code = np.where(M == 0, np.uint64(0), code)                             # +-0
    code = np.where(e64 == 0x7FF, np.where(f52 == 0, inf_code,               # inf, NaN
                                            inf_code | (np.uint64(1) << np.uint64(m - 1))), code)
    return code | (sign << np.uint64(bits - 1))


def fpx_values(codes, bits):
    """FP64 values of X-bit codes (exact: every FPX value is an FP64 value)."""
    m = bits - 9
    c = np.asarray(codes, dtype=np.uint64)
    s = np.where((c >> np.uint64(bits - 1)) & np.uint64(1), -1.0, 1.0)
    be = ((c >> np.uint64(m)) & np.uint64(0xFF)).astype(np.int64)
    f = (c & np.uint64((1 << m) - 1)).astype(np.float64)
    val = np.where(be == 0, np.ldexp(f, -126 - m), np.ldexp(f + 2.0 ** m, be - 127 - m))
    val = np.where(be == 255, np.where(f == 0, np.inf, np.nan), val)
    return s * val


def fpx_round(x, bits):
    """x rounded to FPX (returned as FP64)."""
    return fpx_values(fpx_codes(x, bits), bits).reshape(np.shape(x))


def fpx_encode(x, bits):
    """Byte array of the codes: element i in bytes [i X/8, (i+1) X/8), little-endian."""
    c = fpx_codes(x, bits)
    nb = bits // 8
    out = np.empty((c.size, nb), np.uint8)
    for k in range(nb):
        out[:, k] = ((c >> np.uint64(8 * k)) & np.uint64(0xFF)).astype(np.uint8)
    return out.ravel()


def fpx_decode(data, bits, n):
    nb = bits // 8
    d = np.asarray(data, dtype=np.uint8)[: n * nb].reshape(n, nb).astype(np.uint64)
    c = np.zeros(n, np.uint64)
    for k in range(nb):
        c |= d[:, k] << np.uint64(8 * k)
    return fpx_values(c, bits)
