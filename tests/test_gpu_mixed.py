"""Mixed-precision complex block products (FP32 and slice-split FP16/BF16) on the GPU.

Bars (per element, against numpy FP64 products of the same inputs):
  * integer-valued operands that the first digit represents exactly, and sums
    below 2^24, give results bit-identical to FP64 for every split scheme;
  * random operands: |C - C_ref| <= c * u_eff * K * rowmax|A| * colmax|B|, with
    u_eff = 2^-24 (FP32 accumulation of FP32-rounded operands), the digit
    resolution 2^-(W*NS) of the split (W = 8 for BF16, 10 for FP16), or 2^-kbits
    for the INT8 modular scheme (its operands are rounded to integers of kbits
    bits after power-of-two scaling; each product term then errs by at most
    2 * 2^-kbits * rowmax * colmax per real product, two of them per complex
    part), c = 8;
  * INT8 modular scheme on integer operands (no rounding of the operands): only
    the FP64 CRT sum rounds, |C - C_ref| <= M (p + 1) 2^-50 * 2^(eA + eB - 2 kbits
    - 2), M the product of the moduli, eA / eB the row / column exponents.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

SCHEMES = [("fp32", 0), ("bf16", 2), ("bf16", 3), ("bf16", 4), ("bf16", 5), ("fp16", 2), ("fp16", 3),
           ("int8", 6), ("int8", 11), ("int8", 16)]


def u_eff(prec, ns, K=None):
    if prec == "fp32":
        return 2.0 ** -23
    if prec == "int8":
        from paper_2606_25595_amd import qtx
        return 2.0 ** -qtx.ozaki2_bits(ns, K)[1]
    w = 8 if prec == "bf16" else 10
    return max(2.0 ** (-(w * ns) + 1), 2.0 ** -50)


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_25595_amd import qtx
    c = qtx.Context(0)
    yield c
    c.close()


def crand(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def ops(A, B, opA, opB):
    a = A if opA == "N" else np.conj(np.transpose(A, (0, 2, 1)))
    b = B if opB == "N" else np.conj(np.transpose(B, (0, 2, 1)))
    return a, b


@pytest.mark.parametrize("prec,ns", [s for s in SCHEMES if s[0] in ("bf16", "fp16")])
@pytest.mark.parametrize("opA,opB", [("N", "N"), ("N", "C"), ("C", "N"), ("C", "C")])
def test_split_integer_operands_bit_exact(ctx, prec, ns, opA, opB):
    import torch
    rng = np.random.default_rng(ns * 10 + (prec == "fp16"))
    M, N, K, batch = 70, 45, 100, 2
    ints = lambda *s: (rng.integers(-7, 8, size=s) + 1j * rng.integers(-7, 8, size=s)).astype(np.complex128)
    A = ints(batch, *((M, K) if opA == "N" else (K, M)))
    B = ints(batch, *((K, N) if opB == "N" else (N, K)))
    C = torch.zeros(batch, M, N, dtype=torch.complex128, device="cuda")
    ctx.zgemm(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), C, opA=opA, opB=opB, prec=prec, n_slices=ns)
    a, b = ops(A, B, opA, opB)
    assert np.array_equal(C.cpu().numpy(), a @ b)


@pytest.mark.parametrize("prec,ns", SCHEMES)
@pytest.mark.parametrize("opA,opB", [("N", "N"), ("N", "C"), ("C", "N")])
@pytest.mark.parametrize("M,N,K", [(17, 33, 5), (64, 64, 64), (130, 70, 416)])
def test_mixed_random_error_bound(ctx, prec, ns, opA, opB, M, N, K):
    import torch
    rng = np.random.default_rng(M + N + K)
    batch = 2
    A = crand(rng, batch, *((M, K) if opA == "N" else (K, M)))
    B = crand(rng, batch, *((K, N) if opB == "N" else (N, K)))
    C0 = crand(rng, batch, M, N)
    C = torch.from_numpy(C0.copy()).cuda()
    ctx.zgemm(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), C, opA=opA, opB=opB, alpha=-1.0,
              beta=1.0, prec=prec, n_slices=ns)
    a, b = ops(A, B, opA, opB)
    ref = C0 - a @ b
    got = C.cpu().numpy()
    amax = np.max(np.abs(np.stack([a.real, a.imag])), axis=(0, 3))       # [batch][M]
    bmax = np.max(np.abs(np.stack([b.real, b.imag])), axis=(0, 2))       # [batch][N]
    bound = 8 * u_eff(prec, ns, K) * K * amax[:, :, None] * bmax[:, None, :] + 1e-300
    assert np.all(np.abs(got - ref) <= bound), np.max(np.abs(got - ref) / bound)


@pytest.mark.parametrize("prec,ns,tol", [("bf16", 5, 1e-7), ("bf16", 4, 3e-5), ("fp16", 3, 1e-4),
                                         ("int8", 11, 1e-7), ("int8", 8, 3e-4)])
def test_mixed_solve_tiny_workload(ctx, prec, ns, tol):
    """End-to-end error of the mixed solve against the FP64 oracle.  Eq. 6 puts
    the error near kappa * u_eff.  Measured amplifications of product errors
    into G^< on these inputs are up to ~5e4 (G^R ~30x less), so the bar is
    5e4 * u_eff with u_eff = 2^-(W*NS+1)."""
    import oracle
    from paper_2606_25595_amd import inputs, qtx
    p = inputs.config_problem("tiny")
    dp = qtx.to_device(p)
    ctx.solve(dp, prec=prec, n_slices=ns)
    out = dp.outputs()
    ref = oracle.dense_selected(p)
    assert np.all(out["status"] == 0)
    for k in ("GR_d", "GR_u", "GR_l", "GL_d", "GL_u"):
        err = oracle.rel_fro_err(out[k], ref[k]).max()
        assert err <= tol, (k, err)


def test_mixed_per_chain_schemes(ctx):
    """Retarded and lesser chains with different schemes: the lesser products
    carry the G^< error (the retarded FP64 run keeps G^R at FP64 accuracy)."""
    import oracle
    from paper_2606_25595_amd import inputs, qtx
    p = inputs.config_problem("tiny", energy_index=list(range(0, 32, 3)))
    dp = qtx.to_device(p)
    ctx.solve(dp, prec="fp64", prec_lesser="bf16", n_slices_lesser=4)
    out = dp.outputs()
    ref = oracle.dense_selected(p)
    for k in ("GR_d", "GR_u", "GR_l"):
        assert oracle.rel_fro_err(out[k], ref[k]).max() <= 1e-10
    for k in ("GL_d", "GL_u"):
        assert oracle.rel_fro_err(out[k], ref[k]).max() <= 3e-5


@pytest.mark.parametrize("p", [4, 11, 16])
@pytest.mark.parametrize("opA,opB", [("N", "N"), ("C", "N"), ("N", "C")])
def test_int8_integer_operands_crt_only(ctx, p, opA, opB):
    """Integer operands are scaled without rounding, so the only error left is
    the FP64 rounding of the CRT sum."""
    import math
    import torch
    from paper_2606_25595_amd import qtx
    rng = np.random.default_rng(p)
    M_, N_, K, batch = 70, 45, 100, 2
    ints = lambda *s: (rng.integers(-7, 8, size=s) + 1j * rng.integers(-7, 8, size=s)).astype(np.complex128)
    A = ints(batch, *((M_, K) if opA == "N" else (K, M_)))
    B = ints(batch, *((K, N_) if opB == "N" else (N_, K)))
    C = torch.zeros(batch, M_, N_, dtype=torch.complex128, device="cuda")
    ctx.zgemm(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), C, opA=opA, opB=opB, prec="int8", n_slices=p)
    a, b = ops(A, B, opA, opB)
    ref = a @ b
    mods, kb = qtx.ozaki2_bits(p, K)
    Mp = float(math.prod(mods))
    amax = np.max(np.abs(np.stack([a.real, a.imag])), axis=(0, 3))
    bmax = np.max(np.abs(np.stack([b.real, b.imag])), axis=(0, 2))
    ea = np.where(amax > 0, np.floor(np.log2(np.where(amax > 0, amax, 1))) + 2, 0)
    eb = np.where(bmax > 0, np.floor(np.log2(np.where(bmax > 0, bmax, 1))) + 2, 0)
    tol = Mp * (p + 1) * 2.0 ** -50 * 2.0 ** (ea[:, :, None] + eb[:, None, :] - 2 * kb - 2)
    err = np.abs(C.cpu().numpy() - ref)
    assert np.all(err <= tol), np.max(err / tol)


def test_int8_accuracy_improves_with_moduli(ctx):
    """More moduli -> wider integers -> smaller error (until the CRT rounding)."""
    import torch
    rng = np.random.default_rng(7)
    A = crand(rng, 2, 96, 96)
    B = crand(rng, 2, 96, 96)
    ref = A @ B
    errs = []
    for p in (6, 8, 10, 12):
        C = torch.zeros(2, 96, 96, dtype=torch.complex128, device="cuda")
        ctx.zgemm(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), C, prec="int8", n_slices=p)
        errs.append(np.max(np.abs(C.cpu().numpy() - ref)))
    assert all(errs[i + 1] < errs[i] / 16 for i in range(len(errs) - 1)), errs


@pytest.mark.parametrize("K", [512, 700])
@pytest.mark.parametrize("opA,opB", [("N", "N"), ("C", "C")])
def test_int8_long_contraction(ctx, K, opA, opB):
    """K = 512 is the longest contraction of the single-pass operand conversion;
    longer ones take the two-pass conversion.  Same error bar as above."""
    import torch
    rng = np.random.default_rng(K)
    M_, N_, batch, p = 40, 50, 2, 11
    A = crand(rng, batch, *((M_, K) if opA == "N" else (K, M_)))
    B = crand(rng, batch, *((K, N_) if opB == "N" else (N_, K)))
    C = torch.zeros(batch, M_, N_, dtype=torch.complex128, device="cuda")
    ctx.zgemm(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), C, opA=opA, opB=opB, prec="int8", n_slices=p)
    a, b = ops(A, B, opA, opB)
    amax = np.max(np.abs(np.stack([a.real, a.imag])), axis=(0, 3))
    bmax = np.max(np.abs(np.stack([b.real, b.imag])), axis=(0, 2))
    bound = 8 * u_eff("int8", p, K) * K * amax[:, :, None] * bmax[:, None, :]
    assert np.all(np.abs(C.cpu().numpy() - a @ b) <= bound)
