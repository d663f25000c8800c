"""Host-side parameters of the INT8 modular (Ozaki II) product scheme.

The library chooses, for p moduli and contraction length K, the moduli and the
operand integer width kbits.  Pinned here with exact integer arithmetic:
  * the moduli are odd (symmetric residues fit int8 and negation stays in range),
    at most 255 and pairwise coprime (the CRT needs it);
  * kbits is the largest width with 8 K 4^kbits < M = prod m_i, so the exact
    sums |sum_k Ar'Br' - Ai'Bi'| <= 2 K 4^kbits stay below M / 4 (no wrap modulo
    M, and the CRT's final rounding to the nearest integer has a 1/4 margin);
  * the moduli count is clipped to the largest whose kbits is at most 47
    (residues from FP64 stay exact, and M stays within 16x of the largest sum);
  * the CRT identity the kernels fold with, C / M = sum_i ((C mod m_i) u_i mod m_i)
    / m_i (mod 1) with u_i = (M / m_i)^-1 mod m_i, recovers C for |C| < M / 2.
"""
import math
import random
from fractions import Fraction

import pytest

from paper_2606_25595_amd import qtx


def _lib_or_skip():
    try:
        qtx.load_library()
    except ImportError:
        pytest.skip("library not built")


ALL_MODULI = [255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 217, 211, 199, 197, 193, 191]


def test_moduli_odd_coprime():
    assert all(m % 2 == 1 and 3 <= m <= 255 for m in ALL_MODULI)
    for i in range(len(ALL_MODULI)):
        for j in range(i + 1, len(ALL_MODULI)):
            assert math.gcd(ALL_MODULI[i], ALL_MODULI[j]) == 1, (ALL_MODULI[i], ALL_MODULI[j])


@pytest.mark.parametrize("p", list(range(2, 17)))
def test_library_uses_a_prefix(p):
    _lib_or_skip()
    mods, _ = qtx.ozaki2_bits(p, 65536 if p > 2 else 16)
    assert 2 <= len(mods) <= p and mods == ALL_MODULI[:len(mods)]


@pytest.mark.parametrize("p", [2, 4, 8, 10, 11, 12, 16])
@pytest.mark.parametrize("K", [1, 16, 100, 416, 512, 1024, 65536])
def test_kbits_largest_safe(p, K):
    _lib_or_skip()
    all_mods = ALL_MODULI

    def kbits(q):
        M = math.prod(all_mods[:q])
        k = 0
        while 8 * K * 4 ** (k + 1) < M:
            k += 1
        return k if 8 * K * 4 ** k < M else -1

    q = p
    while kbits(q) > 47 and q > 2:
        q -= 1
    if not 1 <= kbits(q) <= 47:
        with pytest.raises(qtx.QtxError):
            qtx.ozaki2_bits(p, K)
        return
    mods, kb = qtx.ozaki2_bits(p, K)
    assert mods == all_mods[:q]
    M = math.prod(mods)
    assert 1 <= kb <= 47
    assert 8 * K * 4 ** kb < M <= 8 * K * 4 ** (kb + 1)
    assert q == p or kbits(q + 1) > 47


def test_out_of_range_rejected():
    _lib_or_skip()
    for p, K in [(1, 16), (17, 16), (11, 0), (11, 65537), (2, 65536), (2, 4096)]:
        with pytest.raises(qtx.QtxError):
            qtx.ozaki2_bits(p, K)


@pytest.mark.parametrize("p", [2, 5, 11, 16])
def test_crt_identity(p):
    """Exact rational check of the reconstruction on random and extreme C."""
    _lib_or_skip()
    mods, _ = qtx.ozaki2_bits(p, 16)
    M = math.prod(mods)
    u = [pow(M // m, -1, m) for m in mods]
    rng = random.Random(p)
    cases = [0, 1, -1, (M - 1) // 2, -((M - 1) // 2)] + [rng.randrange(-(M // 2) + 1, M // 2) for _ in range(200)]
    for C in cases:
        S = sum(Fraction((C % m) * ui % m, m) for m, ui in zip(mods, u))
        S -= round(S)                      # into [-1/2, 1/2]
        assert S * M == C
