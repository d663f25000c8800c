"""Pins of the error metric every parity test compares with.

The per-block relative Frobenius error ||X - X*||_F / ||X*||_F (absolute where
||X*||_F = 0) is checked against values computed by hand, so that a mistake in
it (a dropped square root, a missing modulus, the wrong reduced axes, a swapped
reference) cannot hide behind the tolerances of the other tests.
"""
import math

import numpy as np

import oracle


def test_rel_fro_err_hand_values():
    # X* = 3 I_2 (||X*||_F = sqrt(18)); X - X* has one entry 1 (||.||_F = 1)
    ref = 3.0 * np.eye(2, dtype=np.complex128)
    x = ref.copy()
    x[0, 1] += 1.0
    e = oracle.rel_fro_err(x[None], ref[None])
    assert e.shape == (1,)
    assert e[0] == 1.0 / math.sqrt(18.0)


def test_rel_fro_err_complex_entries_and_modulus():
    # difference 3 + 4i in one entry: |.| = 5, so ||X - X*||_F = 5 (a real-part-only
    # or squared metric would give 3, 9 or 25); X* = diag(1, 2i, 2): ||X*||_F = 3
    ref = np.diag([1.0, 2.0j, 2.0]).astype(np.complex128)
    x = ref.copy()
    x[2, 0] += 3.0 + 4.0j
    e = oracle.rel_fro_err(x, ref)          # a single 2-D block: a 0-d result
    assert np.ndim(e) == 0
    assert float(e) == 5.0 / 3.0
    # the reference is the second argument (swapping them changes the value)
    e_sw = float(oracle.rel_fro_err(ref, x))
    assert abs(e_sw - 5.0 / math.sqrt(9.0 + 25.0)) < 1e-15


def test_rel_fro_err_reduces_the_last_two_axes_per_leading_index():
    # [n_e = 2][n_b = 3][2][2]: one value per (energy, block)
    ref = np.zeros((2, 3, 2, 2), dtype=np.complex128)
    x = np.zeros_like(ref)
    expect = np.zeros((2, 3))
    for e in range(2):
        for i in range(3):
            scale = float(1 + e + 2 * i)            # ||X*||_F = 2 * scale (entries +-scale)
            ref[e, i] = scale * np.array([[1, -1], [1j, 1]])
            d = float(e + 1) * (i + 1)              # one entry off by d: ||X - X*||_F = d
            x[e, i] = ref[e, i]
            x[e, i, 1, 0] += d
            expect[e, i] = d / (2.0 * scale)
    got = oracle.rel_fro_err(x, ref)
    assert got.shape == (2, 3)
    np.testing.assert_allclose(got, expect, rtol=1e-15, atol=0)
    # errors in one block never leak into another
    x2 = ref.copy()
    x2[1, 2, 0, 0] += 2.0
    got2 = oracle.rel_fro_err(x2, ref)
    assert np.count_nonzero(got2) == 1 and got2[1, 2] == 2.0 / (2.0 * 6.0)


def test_rel_fro_err_zero_reference_is_absolute():
    ref = np.zeros((2, 2, 2), dtype=np.complex128)
    x = np.zeros_like(ref)
    x[0, 0, 0] = 3.0
    x[0, 1, 1] = 4.0j                             # ||X||_F = 5 in block 0
    got = oracle.rel_fro_err(x, ref)
    assert got[0] == 5.0 and got[1] == 0.0
    # a reference that is zero in one block only: that block absolute, the other relative
    ref2 = np.zeros((2, 2, 2), dtype=np.complex128)
    ref2[1] = 2.0 * np.eye(2)                     # ||.||_F = 2 sqrt(2)
    x3 = ref2.copy()
    x3[0, 0, 1] = 1.5
    x3[1, 1, 0] = 1.0
    got3 = oracle.rel_fro_err(x3, ref2)
    assert got3[0] == 1.5
    assert abs(got3[1] - 1.0 / (2.0 * math.sqrt(2.0))) < 1e-16


def test_rel_fro_err_exact_match_and_scale_invariance():
    rng = np.random.default_rng(3)
    ref = rng.standard_normal((4, 5, 5)) + 1j * rng.standard_normal((4, 5, 5))
    assert np.all(oracle.rel_fro_err(ref.copy(), ref) == 0.0)
    x = ref + 1e-3 * (rng.standard_normal(ref.shape) + 1j * rng.standard_normal(ref.shape))
    e1 = oracle.rel_fro_err(x, ref)
    e2 = oracle.rel_fro_err(4.0 * x, 4.0 * ref)   # relative: power-of-two scaling is exact
    np.testing.assert_array_equal(e1, e2)
    # and it is the plain definition, written out with loops over the entries
    for k in range(4):
        num = math.sqrt(sum(abs(x[k, r, c] - ref[k, r, c]) ** 2 for r in range(5) for c in range(5)))
        den = math.sqrt(sum(abs(ref[k, r, c]) ** 2 for r in range(5) for c in range(5)))
        assert abs(e1[k] - num / den) <= 1e-14 * e1[k]
