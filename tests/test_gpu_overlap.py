"""Products overlapped with the forward inversions on a side stream: the outputs
are bitwise those of the single-stream order, for several block-size lanes,
per-chain schemes and the greater recurrence.  The overlap is never captured into
a graph: the two options exclude each other."""
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


def problems(seed, count, greater=False):
    rng = np.random.default_rng(seed)
    out = []
    for q in range(count):
        b = int(rng.choice([24, 40, 72]))          # several lanes
        n_b = int(rng.choice([2, 3, 5, 6]))
        E = rng.uniform(-2.0, 2.0, int(rng.integers(1, 4)))
        out.append(inputs.random_bt_problem(n_b, b, E, seed=300 + q, with_greater=greater))
    return out


def run(ctx, probs, stream=None, **kw):
    import torch
    from paper_2606_25595_amd import qtx
    dps = [qtx.to_device(p) for p in probs]
    if stream is None:
        ctx.solve(dps, **kw)
        torch.cuda.synchronize()
    else:
        with torch.cuda.stream(stream):
            ctx.solve(dps, stream=stream, **kw)
        stream.synchronize()
    return dps, [dp.outputs() for dp in dps]


@pytest.mark.parametrize("scheme", [dict(prec="fp64"), dict(prec="int8", n_slices=10, prec_lesser="int8",
                                                             n_slices_lesser=11), dict(prec="bf16", n_slices=4)])
def test_overlap_bitwise_equal(ctx, scheme):
    probs = problems(1, 7)
    ctx.set_overlap(False)
    _, ref = run(ctx, probs, **scheme)
    ctx.set_overlap(True)
    _, got = run(ctx, probs, **scheme)
    for q, (a, r) in enumerate(zip(got, ref)):
        for k in KEYS:
            assert np.array_equal(a[k], r[k]), (q, k)
    if scheme["prec"] == "fp64":
        for p, a in zip(probs, got):
            refo = oracle.rgf_selected(p)
            for k in KEYS:
                assert oracle.rel_fro_err(a[k], refo[k]).max() <= 1e-10


def test_overlap_with_greater(ctx):
    probs = problems(2, 4, greater=True)
    keys = KEYS + ("GG_d", "GG_u")
    ctx.set_overlap(False)
    _, ref = run(ctx, probs, prec="int8", n_slices=11)
    ctx.set_overlap(True)
    _, got = run(ctx, probs, prec="int8", n_slices=11)
    for a, r in zip(got, ref):
        for k in keys:
            assert np.array_equal(a[k], r[k]), k


def test_overlap_and_graph_are_exclusive(ctx):
    """QTX_OPT_OVERLAP and QTX_OPT_GRAPH cannot both be on (the side stream is never
    captured): turning either on while the other is on is QTX_ERR_UNSUPPORTED and
    leaves the options as they were."""
    from paper_2606_25595_amd import qtx
    ctx.set_overlap(True)
    try:
        with pytest.raises(qtx.QtxError) as ei:
            ctx.set_graph(True)
        assert ei.value.code == qtx.QTX_ERR_UNSUPPORTED
    finally:
        ctx.set_overlap(False)
    ctx.set_graph(True)
    try:
        with pytest.raises(qtx.QtxError) as ei:
            ctx.set_overlap(True)
        assert ei.value.code == qtx.QTX_ERR_UNSUPPORTED
        # the graph path still solves (no side stream involved)
        probs = problems(2, 6)
        _, ref = run(ctx, probs, prec="int8", n_slices=11)
        assert all(np.all(r["status"] == 0) for r in ref)
    finally:
        ctx.set_graph(False)
