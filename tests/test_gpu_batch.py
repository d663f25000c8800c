"""Batched solves of many problems with uneven block size and block count
(one qtx_rgf_solve call, optionally captured into a hipGraph)."""
import numpy as np
import pytest

import oracle
from paper_2606_25595_amd import inputs

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


KEYS = ("GR_d", "GR_u", "GR_l", "GL_d", "GL_u")


def mixed_problems(seed=0, count=9):
    """Problems with b in {24, 40, 64}, n_b in {2, 3, 5}, one or two energies each."""
    rng = np.random.default_rng(seed)
    probs = []
    for q in range(count):
        b = int(rng.choice([24, 40, 64]))
        n_b = int(rng.choice([2, 3, 5]))
        n_e = int(rng.integers(1, 3))
        E = rng.uniform(-2.0, 2.0, n_e)
        probs.append(inputs.random_bt_problem(n_b, b, E, seed=1000 + q))
    return probs


def test_batch_matches_oracle_and_alone(ctx):
    import torch
    from paper_2606_25595_amd import qtx
    probs = mixed_problems()
    dps = [qtx.to_device(p) for p in probs]
    ctx.solve(dps)
    torch.cuda.synchronize()
    for p, dp in zip(probs, dps):
        out = dp.outputs()
        assert np.all(out["status"] == 0)
        ref = oracle.rgf_selected(p)
        for k in KEYS:
            assert oracle.rel_fro_err(out[k], ref[k]).max() <= 1e-10, k
        # the same problem alone gives bit-identical blocks
        alone = qtx.to_device(p)
        ctx.solve(alone)
        a = alone.outputs()
        for k in KEYS:
            assert np.array_equal(a[k], out[k]), k


def test_batch_graph_replay_equals_eager(ctx):
    import torch
    from paper_2606_25595_amd import qtx
    probs = mixed_problems(seed=3, count=7)
    dps = [qtx.to_device(p) for p in probs]
    ctx.solve(dps)
    torch.cuda.synchronize()
    eager = [dp.outputs() for dp in dps]
    stream = torch.cuda.Stream()
    ctx.set_graph(True)
    try:
        cap0 = ctx.stat(qtx.QTX_STAT_GRAPH_CAPTURES)
        for rep in range(3):
            for dp in dps:
                for k in KEYS:
                    getattr(dp, k).fill_(float("nan"))
            torch.cuda.synchronize()
            with torch.cuda.stream(stream):
                ctx.solve(dps, stream=stream)
            stream.synchronize()
            for dp, ref in zip(dps, eager):
                out = dp.outputs()
                for k in KEYS:
                    assert np.array_equal(out[k], ref[k]), (rep, k)
        assert ctx.stat(qtx.QTX_STAT_GRAPH_CAPTURES) == cap0 + 1      # captured once, replayed after
    finally:
        ctx.set_graph(False)


def test_batch_mixed_precision_per_problem(ctx):
    """Problems with different schemes in one call form separate batches."""
    import torch
    from paper_2606_25595_amd import qtx
    probs = mixed_problems(seed=5, count=4)
    dps = [qtx.to_device(p) for p in probs]
    ctx.solve(dps, prec=["fp64", "bf16", "fp64", "bf16"], n_slices=5)
    torch.cuda.synchronize()
    for q, (p, dp) in enumerate(zip(probs, dps)):
        out = dp.outputs()
        ref = oracle.rgf_selected(p)
        tol = 1e-10 if q % 2 == 0 else 1e-7
        for k in KEYS:
            assert oracle.rel_fro_err(out[k], ref[k]).max() <= tol, (q, k)


def test_batch_per_problem_scheme_lists(ctx):
    """Every scheme field may differ per problem, the lesser-chain scheme included;
    each problem's result equals that of solving it alone with its own scheme."""
    import torch
    from paper_2606_25595_amd import qtx
    probs = mixed_problems(seed=8, count=5)
    sch = [dict(prec="fp64"), dict(prec="int8", n_slices=11), dict(prec="int8", n_slices=10, prec_lesser="int8",
           n_slices_lesser=11), dict(prec="bf16", n_slices=5, prec_lesser="fp64"), dict(prec="int8", n_slices=9)]
    dps = [qtx.to_device(p) for p in probs]
    ctx.solve(dps, prec=[x["prec"] for x in sch], n_slices=[x.get("n_slices", 0) for x in sch],
              prec_lesser=[x.get("prec_lesser") for x in sch],
              n_slices_lesser=[x.get("n_slices_lesser", -1) for x in sch])
    torch.cuda.synchronize()
    tols = [1e-10, 1e-7, 1e-6, 1e-7, 1e-5]
    for q, (p, dp, x) in enumerate(zip(probs, dps, sch)):
        out = dp.outputs()
        ref = oracle.rgf_selected(p)
        for k in KEYS:
            assert oracle.rel_fro_err(out[k], ref[k]).max() <= tols[q], (q, k)
        alone = qtx.to_device(p)
        ctx.solve(alone, **x)
        torch.cuda.synchronize()
        ao = alone.outputs()
        for k in KEYS:
            assert np.array_equal(ao[k], out[k]), (q, k)


@pytest.mark.parametrize("prec,ns", [("fp64", 0), ("int8", 10)])
def test_lane_split_bitwise_equal(ctx, prec, ns):
    """QTX_OPT_LANE_SPLIT runs each group's energies as k batches on k streams; every
    output is bitwise the same as with one lane, also under graph capture."""
    import torch
    from paper_2606_25595_amd import qtx
    probs = mixed_problems(seed=3, count=7)
    ref = [qtx.to_device(p) for p in probs]
    ctx.solve(ref, prec=prec, n_slices=ns)
    torch.cuda.synchronize()
    ref_out = [dp.outputs() for dp in ref]
    try:
        for k, graph in ((2, False), (3, False), (2, True)):
            ctx.set_lane_split(k)
            ctx.set_graph(graph)
            dps = [qtx.to_device(p) for p in probs]
            stream = torch.cuda.Stream()
            with torch.cuda.stream(stream):
                for _ in range(2 if graph else 1):
                    ctx.solve(dps, prec=prec, n_slices=ns, stream=stream)
                stream.synchronize()
            for dp, r in zip(dps, ref_out):
                out = dp.outputs()
                for key in KEYS:
                    assert np.array_equal(out[key], r[key]), (k, graph, key)
    finally:
        ctx.set_lane_split(1)
        ctx.set_graph(False)


@pytest.mark.parametrize("prec,ns,tol", [("fp64", 0, 1e-10), ("int8", 10, 1e-6)])
def test_batch_c3_block_sizes_graph(ctx, prec, ns, tol):
    """Problems at the batching workload's block sizes (b in {128, 256, 384, 512},
    n_b = 16, one energy each) in one call: the 64 x 64 FP64 tiles and the persistent
    INT8 tile variants these sizes select run here.  A captured graph replays to the
    eager bits; a problem alone equals it in the mix; two problems (the smallest and
    the largest block) against the oracle."""
    import torch
    from paper_2606_25595_amd import qtx
    rng = np.random.default_rng(77)
    bs = [128, 256, 384, 512, 256, 128]
    probs = [inputs.random_bt_problem(16, b, rng.uniform(-2.0, 2.0, 1), seed=2000 + q) for q, b in enumerate(bs)]
    dps = [qtx.to_device(p) for p in probs]
    ctx.solve(dps, prec=prec, n_slices=ns)
    torch.cuda.synchronize()
    eager = [dp.outputs() for dp in dps]
    for o in eager:
        assert np.all(o["status"] == 0)
    for q in (0, 3):
        ref = oracle.rgf_selected(probs[q])
        for k in KEYS:
            err = oracle.rel_fro_err(eager[q][k], ref[k]).max()
            assert err <= tol, (q, k, float(err))
    alone = qtx.to_device(probs[1])
    ctx.solve(alone, prec=prec, n_slices=ns)
    torch.cuda.synchronize()
    ao = alone.outputs()
    for k in KEYS:
        assert np.array_equal(ao[k], eager[1][k]), k
    stream = torch.cuda.Stream()
    ctx.set_graph(True)
    try:
        for rep in range(2):
            for dp in dps:
                for k in KEYS:
                    getattr(dp, k).fill_(float("nan"))
            torch.cuda.synchronize()
            with torch.cuda.stream(stream):
                ctx.solve(dps, prec=prec, n_slices=ns, stream=stream)
            stream.synchronize()
            for dp, ref in zip(dps, eager):
                out = dp.outputs()
                for k in KEYS:
                    assert np.array_equal(out[k], ref[k]), (rep, k)
    finally:
        ctx.set_graph(False)
