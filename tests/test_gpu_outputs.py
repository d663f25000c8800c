"""Compact input and output forms of the solve (through the C ABI).

QTX_SIGMA_DIAG: the diagonal self-energy blocks (contact and broadening terms, which
are diagonal matrices in the paper's devices) travel as b-vectors instead of b x b
blocks.  The results equal those of the same solve with the dense blocks: the
epilogue adds the vector on the diagonal, where the dense form adds the same values
plus exact zeros.

out_bits < 64: the off-diagonal outputs G^R_{i,i+1}, G^R_{i+1,i}, G^<_{i,i+1} (and
G^>_{i,i+1}) are written in the FPX storage format of Section V-A, encoded on the GPU
from the FP64 blocks of each backward step.  The recurrences stay FP64, so the bytes
equal the oracle's FPX encoding of the complex128 solve's blocks, and the diagonal
outputs are unchanged.
"""
import numpy as np
import pytest

import oracle
from paper_2606_25595_amd import inputs

pytestmark = pytest.mark.gpu

OFF = ("GR_u", "GR_l", "GL_u")
DIAG = ("GR_d", "GL_d")


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_25595_amd import qtx
    c = qtx.Context(0)
    yield c
    c.close()


def varied_problem(n_b, b, n_e, seed, greater=False, bt_sigma=0.0):
    """random_bt_problem with a different value at every diagonal position of the
    diagonal self-energy blocks (so that a wrong element index shows), keeping
    Sigma^R's anti-Hermitian part negative definite and Sigma^<, Sigma^> skew-Hermitian."""
    E = np.linspace(-1.6, 1.7, n_e)
    p = inputs.random_bt_problem(n_b, b, E, seed=seed, with_greater=greater, bt_sigma=bt_sigma)
    rng = np.random.default_rng(seed + 100)
    ii = np.arange(b)
    dr = 0.05 * rng.standard_normal((n_e, n_b, b)) - 0.02j * rng.random((n_e, n_b, b))
    dl = 0.03j * rng.random((n_e, n_b, b))
    p.SR_d = p.SR_d.copy()
    p.SL_d = p.SL_d.copy()
    p.SR_d[:, :, ii, ii] += dr
    p.SL_d[:, :, ii, ii] += dl
    if greater:
        p.SG_d = p.SG_d.copy()
        p.SG_d[:, :, ii, ii] -= dl
    return p


def run(ctx, p, split=False, **kw):
    import torch
    from paper_2606_25595_amd import qtx
    scheme = dict(kw)
    dev_kw = {k: scheme.pop(k) for k in ("sigma_diag", "out_bits") if k in scheme}
    dp = qtx.to_device(p, **dev_kw)
    dp.split = split
    for k in OFF + DIAG:
        getattr(dp, k).fill_(0)   # no stale values can pass
    ctx.solve(dp, **scheme)
    torch.cuda.synchronize()
    return dp, dp.outputs()


SCHEMES = [dict(prec="fp64"),
           dict(prec="int8", n_slices=10),
           dict(prec="fp64", prec_lesser="bf16", n_slices_lesser=3)]


@pytest.mark.parametrize("scheme", SCHEMES, ids=["fp64", "int8", "bf16-lesser"])
@pytest.mark.parametrize("greater,bt,split", [(False, 0.0, False), (True, 0.0, False), (True, 0.2, False),
                                              (False, 0.0, True)])
def test_sigma_diag_equals_dense(ctx, scheme, greater, bt, split):
    p = varied_problem(6, 40, 7, seed=3, greater=greater, bt_sigma=bt)
    _, ref = run(ctx, p, split=split, **scheme)
    dp, out = run(ctx, p, split=split, sigma_diag=True, **scheme)
    assert tuple(dp.SR_d.shape) == (7, 6, 40)
    assert np.all(out["status"] == 0)
    keys = OFF + DIAG + (("GG_d", "GG_u") if greater else ())
    for k in keys:
        assert np.array_equal(out[k], ref[k]), k


def test_sigma_diag_against_oracle(ctx):
    """The diagonal form of the self-energies against the oracle's dense solve."""
    p = varied_problem(5, 24, 4, seed=8, greater=True)
    _, out = run(ctx, p, sigma_diag=True, prec="fp64")
    ref = oracle.rgf_selected(p)
    for k in OFF + DIAG + ("GG_d", "GG_u"):
        err = oracle.rel_fro_err(out[k], ref[k])
        assert np.max(err) < 1e-11, (k, err)


def expected_fpx(block_array, bits):
    """[n_e][n_b-1][b][b] complex128 -> [n_e][n_b-1][2 b b bits / 8] bytes (oracle encode)."""
    n_e, nu = block_array.shape[:2]
    flat = np.ascontiguousarray(block_array).view(np.float64).reshape(n_e, nu, -1)
    return oracle.fpx_encode(flat, bits).reshape(n_e, nu, -1)


@pytest.mark.parametrize("bits", [16, 24, 32, 48, 56])
@pytest.mark.parametrize("scheme", SCHEMES[:2], ids=["fp64", "int8"])
def test_fpx_outputs_equal_encoded_fp64_solve(ctx, bits, scheme):
    p = varied_problem(5, 40, 6, seed=5, greater=True, bt_sigma=0.1)
    _, ref = run(ctx, p, **scheme)
    dp, out = run(ctx, p, out_bits=bits, **scheme)
    assert np.all(out["status"] == 0)
    for k in OFF + ("GG_u",):
        assert out[k].dtype == np.uint8 and out[k].shape == (6, 4, 40 * 40 * bits // 4), k
        assert np.array_equal(out[k], expected_fpx(ref[k], bits)), (k, bits)
    for k in DIAG + ("GG_d",):
        assert np.array_equal(out[k], ref[k]), k
    # decoded, the blocks are the FP64 ones to within the format's rounding
    dec = oracle.fpx_decode(out["GR_u"].ravel(), bits, 2 * ref["GR_u"].size).view(np.complex128)
    err = np.abs(dec - ref["GR_u"].ravel()) / np.maximum(np.abs(ref["GR_u"].ravel()), 1e-30)
    assert np.max(err[np.abs(ref["GR_u"].ravel()) > 1e-30]) <= 2.0 ** (-(bits - 9)) * 2


def test_fpx_outputs_with_sigma_diag_and_ragged_block(ctx):
    """Both compact forms at once, with b = 37 (2 b^2 X / 8 bytes per block is not a
    multiple of 8 for X = 24: unaligned block starts take the byte path)."""
    p = varied_problem(4, 37, 5, seed=9)
    _, ref = run(ctx, p, prec="fp64")
    _, out = run(ctx, p, prec="fp64", out_bits=24, sigma_diag=True)
    for k in OFF:
        assert np.array_equal(out[k], expected_fpx(ref[k], 24)), k
    for k in DIAG:
        assert np.array_equal(out[k], ref[k]), k


def test_fpx_failed_energy_holds_nan_codes(ctx):
    p = varied_problem(4, 32, 5, seed=2)
    p.SL_d = p.SL_d.copy()
    p.SL_d[3, 1, 4, 4] = np.nan
    _, ref = run(ctx, p, prec="fp64")
    _, out = run(ctx, p, prec="fp64", out_bits=32, sigma_diag=True)
    assert list(out["status"]) == list(ref["status"])
    assert out["status"][3] != 0 and np.all(np.delete(out["status"], 3) == 0)
    for k in OFF:
        n = out[k][3].size // 4
        vals = oracle.fpx_decode(out[k][3].ravel(), 32, n)
        assert np.all(np.isnan(vals)), k
        good = [e for e in range(5) if e != 3]
        assert np.array_equal(out[k][good], expected_fpx(ref[k][good], 32)), k


def test_fpx_outputs_under_graph_replay(ctx):
    """Captured and replayed solves (the FPX encode kernels are part of the graph)."""
    import torch
    from paper_2606_25595_amd import qtx
    p = varied_problem(5, 48, 6, seed=4)
    _, ref = run(ctx, p, prec="int8", n_slices=10)
    ctx.set_graph(True)
    try:
        dp = qtx.to_device(p, out_bits=48, sigma_diag=True)
        for rep in range(3):
            for k in OFF:
                getattr(dp, k).fill_(0)
            torch.cuda.synchronize()
            ctx.solve(dp, prec="int8", n_slices=10)
            torch.cuda.synchronize()
            out = dp.outputs()
            for k in OFF:
                assert np.array_equal(out[k], expected_fpx(ref[k], 48)), (rep, k)
    finally:
        ctx.set_graph(False)


def test_fpx_argument_errors(ctx):
    from paper_2606_25595_amd import qtx
    p = varied_problem(4, 16, 2, seed=6)
    dp = qtx.to_device(p, out_bits=32)
    dp.split = True
    assert ctx.solve(dp, check=False) == qtx.QTX_ERR_UNSUPPORTED
    dp.split = False
    dp.out_bits = 20
    assert ctx.solve(dp, check=False) == qtx.QTX_ERR_ARG
