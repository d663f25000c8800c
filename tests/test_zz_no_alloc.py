"""qtx_zgemm_noalloc: the block product for callers that cannot allocate, with its
converted operands in a fixed per-GPU scratch buffer (through the C ABI).

Each call is checked against qtx_zgemm on the same inputs (the same kernels, so
the same bits), twice in a row with the second call smaller than the first (the
scratch keeps the first call's bytes beyond what the second converts); calls too
large for the scratch are refused with nothing enqueued.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("prec,ns", [("int8", 10), ("int8", 6), ("bf16", 4), ("fp16", 3), ("fp64", 0), ("fp32", 0)])
def test_noalloc_equals_zgemm_two_calls_shrinking(ctx, prec, ns):
    import torch
    rng = np.random.default_rng(11 + ns)
    # (M, N, K, batch, opA, opB, shared A): the second call is smaller than the first
    calls = [(416, 416, 416, 4, "N", "C", False), (100, 72, 130, 3, "C", "N", True)]
    for M, N, K, batch, opA, opB, shared in calls:
        A = crand(rng, 1 if shared else batch, *((M, K) if opA == "N" else (K, M)))
        B = crand(rng, batch, *((K, N) if opB == "N" else (N, K)))
        C0 = crand(rng, batch, M, N)
        dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
        ref = torch.from_numpy(C0).cuda()
        got = torch.from_numpy(C0).cuda()
        ctx.zgemm(dA, dB, ref, opA=opA, opB=opB, alpha=0.5 - 1j, beta=-1.0, prec=prec, n_slices=ns)
        ctx.zgemm(dA, dB, got, opA=opA, opB=opB, alpha=0.5 - 1j, beta=-1.0, prec=prec, n_slices=ns, noalloc=True)
        torch.cuda.synchronize()
        r, g = ref.cpu().numpy(), got.cpu().numpy()
        assert np.all(np.isfinite(g))
        assert np.array_equal(g.view(np.float64), r.view(np.float64)), (M, N, K, batch)
        # and it is the product, to the scheme's accuracy
        opa = A if opA == "N" else np.conj(np.swapaxes(A, 1, 2))
        opb = B if opB == "N" else np.conj(np.swapaxes(B, 1, 2))
        exact = (0.5 - 1j) * (opa @ opb) - C0
        if prec == "int8":
            from paper_2606_25595_amd import qtx
            kbits = qtx.ozaki2_bits(ns, K)[1]
            bound = 8 * 2.0 ** -kbits * K * np.abs(opa).max() * np.abs(opb).max() * abs(0.5 - 1j) + 1e-12
            assert np.abs(g - exact).max() <= bound
        else:
            scale = np.abs(opa) @ np.abs(opb) + np.abs(C0)
            tol = {"bf16": 1e-6, "fp16": 1e-6, "fp64": 1e-13, "fp32": 1e-5}[prec]
            assert np.max(np.abs(g - exact) / scale) <= tol


def test_noalloc_refuses_more_than_the_scratch(ctx):
    import torch
    from paper_2606_25595_amd import qtx
    # 1024 x 1024 x 1024, batch 4, 10 moduli: about 2 * 10 * 2048 * 1024 * 4 bytes > 64 MiB
    A = torch.zeros((4, 1024, 1024), dtype=torch.complex128, device="cuda")
    C = torch.full((4, 1024, 1024), 3.0 + 0j, dtype=torch.complex128, device="cuda")
    rc = ctx.zgemm(A, A, C, prec="int8", n_slices=10, noalloc=True, check=False)
    assert rc == qtx.QTX_ERR_ARG
    torch.cuda.synchronize()
    assert bool((C == 3.0).all())           # nothing was enqueued
    # the FP64 product of the same size needs no scratch
    assert ctx.zgemm(A, A, C, prec="fp64", noalloc=True, check=False) == qtx.QTX_OK
    torch.cuda.synchronize()
    assert bool((C == 0.0).all())
