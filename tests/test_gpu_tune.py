"""INT8 product tile variants and the autotuner: every variant gives bitwise the
same product (the same exact INT32 sums and the same CRT fold order), the tuner
records a choice per shape, writes and re-reads its cache file, and a solve after
tuning equals the solve before it."""
import numpy as np
import pytest

import oracle
from paper_2606_25595_amd import inputs

pytestmark = pytest.mark.gpu
N_VARIANTS = 14     # tile variants of the INT8 product kernel


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_25595_amd import qtx
    c = qtx.Context(0)
    yield c
    c.close()


def rand_c(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize("M,N,K,batch", [(416, 416, 416, 3), (200, 150, 300, 2), (33, 97, 70, 4), (64, 64, 64, 1),
                                         (130, 70, 600, 1)])
@pytest.mark.parametrize("ops", ["NN", "NC", "CN", "CC"])
@pytest.mark.parametrize("p", [6, 11])
def test_variants_bitwise_equal(ctx, M, N, K, batch, ops, p):
    import torch
    rng = np.random.default_rng(M * 7 + N * 3 + K + p)
    A = rand_c(rng, batch, *((M, K) if ops[0] == "N" else (K, M)))
    B = rand_c(rng, batch, *((K, N) if ops[1] == "N" else (N, K)))
    C0 = rand_c(rng, batch, M, N)
    At, Bt = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    outs = []
    try:
        for v in range(N_VARIANTS):
            ctx.set_int8_tile_variant(v)
            C = torch.from_numpy(C0).cuda()
            ctx.zgemm(At, Bt, C, opA=ops[0], opB=ops[1], alpha=-1.0, beta=1.0, prec="int8", n_slices=p)
            torch.cuda.synchronize()
            outs.append(C.cpu().numpy())
    finally:
        ctx.set_int8_tile_variant(-1)
    for v in range(1, N_VARIANTS):
        assert np.array_equal(outs[v].view(np.float64), outs[0].view(np.float64)), v
    # and the common result is the product to the scheme's accuracy
    opa = A if ops[0] == "N" else np.conj(np.swapaxes(A, 1, 2))
    opb = B if ops[1] == "N" else np.conj(np.swapaxes(B, 1, 2))
    ref = C0 - opa @ opb
    from paper_2606_25595_amd import qtx
    kbits = qtx.ozaki2_bits(p, K)[1]
    bound = 8 * 2.0 ** -kbits * K * np.abs(opa).max() * np.abs(opb).max()
    assert np.abs(outs[0] - ref).max() <= bound


def test_tune_records_and_cache(tmp_path):
    import torch
    from paper_2606_25595_amd import qtx
    path = str(tmp_path / "tune.txt")
    c = qtx.Context(0, tune_cache=path)
    try:
        assert c.stat(qtx.QTX_STAT_TUNE_RECORDS) == 0
        v, ms = c.tune(96, "int8", 8, batch=16)
        assert 0 <= v < N_VARIANTS and len(ms) == N_VARIANTS
        assert all(t > 0 for t in ms) and ms[v] == min(ms)
        v2, _ = c.tune(96, "int8", 8, batch=200)          # another batch class: a second record
        assert c.stat(qtx.QTX_STAT_TUNE_RECORDS) == 2
        v, _ = c.tune(96, "int8", 8, batch=16)             # the same key again: replaced, not added
        assert c.stat(qtx.QTX_STAT_TUNE_RECORDS) == 2
        v3, _ = c.tune(96, "int8", 9, batch=16)            # another modulus count: a third record
        assert c.stat(qtx.QTX_STAT_TUNE_RECORDS) == 3
        # FP64 / FP32 / split: two tilings (32 x 32, 64 x 64), one record per scheme
        v4, ms4 = c.tune(96, "fp64", batch=16)
        assert v4 in (0, 1) and len(ms4) == 2 and all(t > 0 for t in ms4) and ms4[v4] == min(ms4)
        v5, _ = c.tune(96, "bf16", 3, batch=16)
        v6, _ = c.tune(96, "fp32", batch=16)
        assert c.stat(qtx.QTX_STAT_TUNE_RECORDS) == 6
    finally:
        c.close()
    lines = open(path).read().splitlines()
    assert lines[0].startswith("qtx-tune 3 ")
    recs = sorted(l.split()[:7] for l in lines[1:])
    assert recs == sorted([["o2", "96", "96", "96", "4", "8", str(v)], ["o2", "96", "96", "96", "8", "8", str(v2)],
                           ["o2", "96", "96", "96", "4", "9", str(v3)], ["tm", "96", "96", "96", "4", "100", str(v4)],
                           ["tm", "96", "96", "96", "4", "123", str(v5)], ["tm", "96", "96", "96", "4", "110", str(v6)]])
    c2 = qtx.Context(0, tune_cache=path)
    try:
        assert c2.stat(qtx.QTX_STAT_TUNE_RECORDS) == 6
    finally:
        c2.close()


def test_bad_cache_file_is_ignored(tmp_path):
    from paper_2606_25595_amd import qtx
    path = tmp_path / "bad.txt"
    path.write_text("qtx-tune 3 some-other-device 7\no2 96 96 96 4 8 1 1.0 2.0 3.0\n")
    c = qtx.Context(0, tune_cache=str(path))
    try:
        assert c.stat(qtx.QTX_STAT_TUNE_RECORDS) == 0
    finally:
        c.close()
    path.write_text("garbage\n\x00\x01 o2 x y\n")
    c = qtx.Context(0, tune_cache=str(path))
    try:
        assert c.stat(qtx.QTX_STAT_TUNE_RECORDS) == 0
    finally:
        c.close()


def test_tune_rejects_bad_arguments(ctx):
    from paper_2606_25595_amd import qtx
    for args in [(0, "int8", 8, 1), (1025, "int8", 8, 1), (64, "int8", 8, 0)]:
        with pytest.raises(qtx.QtxError):
            ctx.tune(*args[:3], batch=args[3])
    with pytest.raises(qtx.QtxError):
        ctx.tune(64, "int8", 1, batch=1)                   # too few moduli
    with pytest.raises(qtx.QtxError):
        ctx.set_int8_tile_variant(N_VARIANTS)


def test_solve_unchanged_by_tuning():
    import torch
    from paper_2606_25595_amd import qtx
    p = inputs.random_bt_problem(4, 72, np.array([-0.5, 0.3, 1.1]), seed=21)
    c = qtx.Context(0)
    try:
        dp = qtx.to_device(p)
        c.solve(dp, prec="int8", n_slices=10, prec_lesser="int8", n_slices_lesser=11)
        torch.cuda.synchronize()
        before = dp.outputs()
        # force each variant, then the tuned choice: the outputs do not move
        for v in list(range(N_VARIANTS)) + [-1]:
            if v < 0:
                c.set_int8_tile_variant(-1)
                c.tune(72, "int8", 10, batch=3)
                c.tune(72, "int8", 11, batch=3)
            else:
                c.set_int8_tile_variant(v)
            dp2 = qtx.to_device(p)
            c.solve(dp2, prec="int8", n_slices=10, prec_lesser="int8", n_slices_lesser=11)
            torch.cuda.synchronize()
            after = dp2.outputs()
            for k in before:
                assert np.array_equal(before[k], after[k]), (v, k)
        ref = oracle.rgf_selected(p)
        for k in ("GR_d", "GR_u", "GR_l", "GL_d", "GL_u"):
            assert oracle.rel_fro_err(before[k], ref[k]).max() <= 1e-6
    finally:
        c.close()


@pytest.mark.parametrize("M,N,K,batch,ops", [(416, 416, 416, 32, "NN"), (416, 416, 416, 32, "NC"),
                                             (128, 128, 128, 256, "NN"), (128, 128, 128, 256, "CC")])
def test_variants_bitwise_equal_persistent_rounds(ctx, M, N, K, batch, ops):
    """Launches with more tiles than the persistent grid holds (416^3 x 32: 1568 64 x 64
    tiles against 768 workgroups of variant 4; 128^3 x 256: 1024), so every persistent
    variant runs several rounds per workgroup and reuses its LDS ring, exponents and
    accumulators between tiles.  All variants give the same bits, within the bound."""
    import torch
    from paper_2606_25595_amd import qtx
    p = 10
    rng = np.random.default_rng(M + batch + (1 if ops == "NC" else 0))
    A = rand_c(rng, batch, *((M, K) if ops[0] == "N" else (K, M)))
    B = rand_c(rng, batch, *((K, N) if ops[1] == "N" else (N, K)))
    At, Bt = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    outs = []
    try:
        for v in range(N_VARIANTS):
            ctx.set_int8_tile_variant(v)
            C = torch.full((batch, M, N), float("nan"), dtype=torch.complex128, device="cuda")
            ctx.zgemm(At, Bt, C, opA=ops[0], opB=ops[1], prec="int8", n_slices=p)
            torch.cuda.synchronize()
            outs.append(C.cpu().numpy())
    finally:
        ctx.set_int8_tile_variant(-1)
    for v in range(1, N_VARIANTS):
        assert np.array_equal(outs[v].view(np.float64), outs[0].view(np.float64)), v
    opa = A if ops[0] == "N" else np.conj(np.swapaxes(A, 1, 2))
    opb = B if ops[1] == "N" else np.conj(np.swapaxes(B, 1, 2))
    ref = opa @ opb
    kbits = qtx.ozaki2_bits(p, K)[1]
    bound = 8 * 2.0 ** -kbits * K * np.abs(opa).max() * np.abs(opb).max()
    assert np.all(np.isfinite(outs[0]))
    assert np.abs(outs[0] - ref).max() <= bound


def test_skew_products_in_persistent_rounds_every_variant(ctx):
    """A solve whose skew-Hermitian INT8 products (G^< blocks) have more upper-triangle
    tiles than the persistent grid holds (b = 416, 40 energies: 28 x 40 = 1120 tiles of
    64 x 64 against 768 workgroups of variant 4; 10 x 40 = 400 tiles of 128 x 128 against
    256), under every forced tile variant: the same bits as the tuned solve, and the
    tuned solve within the scheme's bound of the oracle on two energies."""
    import torch
    from paper_2606_25595_amd import qtx
    p = inputs.random_bt_problem(3, 416, np.linspace(-1.8, 1.7, 40), seed=5)
    keys = ("GR_d", "GR_u", "GR_l", "GL_d", "GL_u")

    def solve():
        dp = qtx.to_device(p)
        ctx.solve(dp, prec="int8", n_slices=10, prec_lesser="int8", n_slices_lesser=11)
        torch.cuda.synchronize()
        assert bool((dp.status == 0).all())
        return dp
    ref_dp = solve()
    try:
        for v in range(N_VARIANTS):
            ctx.set_int8_tile_variant(v)
            dp = solve()
            for k in keys:
                a, b = getattr(dp, k), getattr(ref_dp, k)
                assert torch.equal(torch.view_as_real(a), torch.view_as_real(b)), (v, k)
            del dp
    finally:
        ctx.set_int8_tile_variant(-1)
    sample = [3, 31]
    ref = oracle.rgf_selected(p.subset(sample))
    for k in keys:
        got = getattr(ref_dp, k)[sample].cpu().numpy()
        assert oracle.rel_fro_err(got, ref[k]).max() <= 1e-6, k


@pytest.mark.parametrize("prec,ns", [("fp64", 0), ("fp32", 0), ("bf16", 4), ("fp16", 3)])
def test_tile_tuning_bitwise_and_solve_unchanged(prec, ns):
    """FP64, FP32 and split products with 32 x 32 or 64 x 64 tiles (forced through the
    tuner's records) give the same bits; a solve before and after tuning is unchanged."""
    import torch
    from paper_2606_25595_amd import qtx
    p = inputs.random_bt_problem(4, 100, np.array([-0.7, 0.4]), seed=23)
    c = qtx.Context(0)
    try:
        dp = qtx.to_device(p)
        c.solve(dp, prec=prec, n_slices=ns)
        torch.cuda.synchronize()
        before = dp.outputs()
        rng = np.random.default_rng(5)
        A = torch.from_numpy(rand_c(rng, 6, 100, 100)).cuda()
        B = torch.from_numpy(rand_c(rng, 6, 100, 100)).cuda()
        C1 = torch.empty_like(A)
        C2 = torch.empty_like(A)
        v, ms = c.tune(100, prec, ns, batch=6)      # records one tiling for this shape
        c.zgemm(A, B, C1, opB="C", prec=prec, n_slices=ns)
        # the other tiling: a record with the other variant, through a cache file round trip
        import os, tempfile
        fd, path = tempfile.mkstemp()
        os.close(fd)
        try:
            code = {"fp64": 100, "fp32": 110, "bf16": 120 + ns, "fp16": 130 + ns}[prec]
            from paper_2606_25595_amd import qtx as q
            tag = open(path, "w")
            tag.close()
            c2 = q.Context(0, tune_cache=path)
            c2.tune(100, prec, ns, batch=6)
            c2.close()
            lines = open(path).read().splitlines()
            with open(path, "w") as fh:
                fh.write(lines[0] + "\n")
                fh.write("tm 100 100 100 3 %d %d 1.0 1.0\n" % (code, 1 - v))
            c3 = q.Context(0, tune_cache=path)
            c3.zgemm(A, B, C2, opB="C", prec=prec, n_slices=ns)
            torch.cuda.synchronize()
            c3.close()
        finally:
            os.unlink(path)
        assert torch.equal(torch.view_as_real(C1), torch.view_as_real(C2))
        dp2 = qtx.to_device(p)
        c.solve(dp2, prec=prec, n_slices=ns)
        torch.cuda.synchronize()
        after = dp2.outputs()
        for k in before:
            assert np.array_equal(before[k], after[k]), k
    finally:
        c.close()
