"""GPU parity of the screened Coulomb (W) system (Table I, W row) against the FP64
oracle: the BT blocks of V P^R and V P^<> V^H (qtx_w_assemble), and the selected
blocks of M^-1 and W^<> = M^-1 B^<> M^-H from qtx_rgf_solve on the assembled
system.  FP64 bar: relative Frobenius error per block <= 1e-12 for the assembly
(a few FP64 block products of O(1) blocks) and <= 1e-10 for the solve (the W
systems here have kappa < 10)."""
import numpy as np
import pytest

import oracle
from paper_2606_25595_amd import inputs

pytestmark = pytest.mark.gpu

KEYS = ("GR_d", "GR_u", "GR_l", "GL_d", "GL_u")


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_25595_amd import qtx
    c = qtx.Context(0)
    yield c
    c.close()


def worst(out, ref, keys):
    return {k: float(oracle.rel_fro_err(out[k], ref[k]).max()) for k in keys if ref[k].size}


@pytest.mark.parametrize("n_b,b,n_e", [(1, 5, 2), (2, 3, 2), (3, 65, 3), (5, 40, 2), (4, 100, 1)])
def test_w_assemble_matches_oracle(ctx, n_b, b, n_e):
    import torch
    from paper_2606_25595_amd import qtx
    w = inputs.random_w_problem(n_b, b, np.linspace(-1.5, 1.2, n_e), seed=n_b * 10 + b, with_greater=True)
    asm = ctx.w_assemble(qtx.w_to_device(w))
    torch.cuda.synchronize()
    ref = oracle.w_assemble(w)
    for k in ("VPR_d", "VPR_u", "VPR_l", "BL_d", "BL_u", "BG_d", "BG_u"):
        if ref[k].size:
            err = oracle.rel_fro_err(asm[k].cpu().numpy(), ref[k]).max()
            assert err <= 1e-12, (k, err)


@pytest.mark.parametrize("n_b,b,n_e", [(2, 3, 2), (3, 65, 3), (6, 48, 2)])
def test_w_solve_matches_oracle(ctx, n_b, b, n_e):
    import torch
    from paper_2606_25595_amd import qtx
    w = inputs.random_w_problem(n_b, b, np.linspace(-1.8, 1.6, n_e), seed=7 + b, with_greater=True)
    dp = ctx.w_solve(qtx.w_to_device(w))
    torch.cuda.synchronize()
    out = dp.outputs()
    assert np.all(out["status"] == 0)
    keys = KEYS + ("GG_d", "GG_u")
    w_rgf = worst(out, oracle.w_selected(w, "rgf"), keys)
    assert max(w_rgf.values()) <= 1e-10, w_rgf
    w_dense = worst(out, oracle.w_selected(w, "dense"), keys)
    assert max(w_dense.values()) <= 1e-10, w_dense


@pytest.mark.parametrize("p,tol", [(6, 1e-4), (8, 1e-6)])
def test_w_solve_int8(ctx, p, tol):
    """The better-conditioned W system takes fewer moduli than G (Section V-B reads
    6 moduli as enough for W): INT8 products in the solve, FP64 assembly."""
    import torch
    from paper_2606_25595_amd import qtx
    w = inputs.random_w_problem(5, 96, np.linspace(-2.0, 2.0, 3), seed=5)
    dp = ctx.w_solve(qtx.w_to_device(w), prec="int8", n_slices=p)
    torch.cuda.synchronize()
    errs = worst(dp.outputs(), oracle.w_selected(w, "rgf"), KEYS)
    assert max(errs.values()) <= tol, errs


def test_w_assemble_energy_chunks_bitwise(ctx):
    """A workspace cap that forces one energy per chunk gives bitwise the same blocks."""
    import torch
    from paper_2606_25595_amd import qtx
    w = inputs.random_w_problem(4, 64, np.linspace(-1.0, 1.0, 5), seed=9, with_greater=True)
    dw = qtx.w_to_device(w)
    a = ctx.w_assemble(dw)
    small = qtx.Context(0, workspace_bytes=5 * 64 * 64 * 16 + 8192)
    try:
        b = small.w_assemble(dw)
        torch.cuda.synchronize()
    finally:
        small.close()
    for k in a:
        assert torch.equal(a[k], b[k]), k


def test_w_assemble_argument_errors(ctx):
    from paper_2606_25595_amd import qtx
    w = inputs.random_w_problem(3, 8, np.array([0.2]), seed=1, with_greater=True)
    dw = qtx.w_to_device(w)
    out = ctx.w_assemble(dw)
    P = qtx._ptr
    lib = ctx.lib
    args = [P(dw.V_d), P(dw.V_u), P(dw.PR_d), P(dw.PR_u), P(dw.PR_l), P(dw.PL_d), P(dw.PL_u), P(dw.PG_d),
            P(dw.PG_u), P(out["VPR_d"]), P(out["VPR_u"]), P(out["VPR_l"]), P(out["BL_d"]), P(out["BL_u"]),
            None, None, None]                                   # P^> given without its outputs
    assert lib.qtx_w_assemble(ctx.handle, 3, 8, 1, 0, 0, *args) == qtx.QTX_ERR_ARG
    args[14], args[15] = P(out["BG_d"]), P(out["BG_u"])
    assert lib.qtx_w_assemble(ctx.handle, 3, 8, 1, 7, 0, *args) == qtx.QTX_ERR_UNSUPPORTED
    assert lib.qtx_w_assemble(ctx.handle, 3, 2000, 1, 0, 0, *args) == qtx.QTX_ERR_ARG
    assert lib.qtx_w_assemble(ctx.handle, 3, 8, 1, 0, 0, *args) == qtx.QTX_OK
