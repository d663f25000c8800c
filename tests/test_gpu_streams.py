"""Calls on one context from several streams (through the C ABI).

Every call on a context uses the context's one workspace; a call on another
stream than the previous call's waits on the device for that call, so solves
and products enqueued back to back on different streams give the same bits as
the same calls made one at a time.
"""
import numpy as np
import pytest

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


@pytest.mark.parametrize("prec,ns", [("fp64", 0), ("int8", 10)])
def test_solves_on_two_streams_match_one_at_a_time(ctx, prec, ns):
    import torch
    from paper_2606_25595_amd import qtx
    probs = [inputs.random_bt_problem(6, 192, np.linspace(-1.5, 1.5, 12), seed=40 + q) for q in range(3)]
    # one at a time
    ref = []
    for p in probs:
        dp = qtx.to_device(p)
        ctx.solve(dp, prec=prec, n_slices=ns)
        torch.cuda.synchronize()
        ref.append(dp.outputs())
    # back to back on three streams, no host synchronisation in between
    dps = [qtx.to_device(p) for p in probs]
    for dp in dps:
        for k in KEYS:
            getattr(dp, k).fill_(float("nan"))
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream() for _ in probs]
    for dp, st in zip(dps, streams):
        with torch.cuda.stream(st):
            ctx.solve(dp, prec=prec, n_slices=ns, stream=st)
    for st in streams:
        st.synchronize()
    for dp, r in zip(dps, ref):
        out = dp.outputs()
        assert np.all(out["status"] == 0)
        for k in KEYS:
            assert np.array_equal(out[k], r[k]), k


def test_products_on_two_streams_match_one_at_a_time(ctx):
    import torch
    rng = np.random.default_rng(9)
    n, batch = 256, 24
    mats = [torch.tensor(rng.standard_normal((batch, n, n)) + 1j * rng.standard_normal((batch, n, n)), device="cuda")
            for _ in range(4)]
    ref = []
    for q in range(2):
        C = torch.empty_like(mats[0])
        ctx.zgemm(mats[2 * q], mats[2 * q + 1], C, prec="int8", n_slices=10)
        torch.cuda.synchronize()
        ref.append(C.cpu().numpy())
    outs = [torch.full_like(mats[0], float("nan")) for _ in range(2)]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream() for _ in range(2)]
    for q in range(2):
        with torch.cuda.stream(streams[q]):
            ctx.zgemm(mats[2 * q], mats[2 * q + 1], outs[q], prec="int8", n_slices=10, stream=streams[q])
    for st in streams:
        st.synchronize()
    for q in range(2):
        assert np.array_equal(outs[q].cpu().numpy(), ref[q])
