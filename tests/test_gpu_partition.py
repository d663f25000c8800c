"""P-way partitioned selected solve of each energy (`partitions` = P, through the C ABI)
against the oracle's plain definition (dense inverse, G^< = G Sigma^< G^H) and against
the one-chain GPU solve.

Tolerances.  The separator system is built from fill-in chains over interior segments
cut off from the contacts (at weak broadening their partial inverses reach 1/eta); the
interiors' outputs come from the one-chain recurrences restarted from the exact
left-connected functions of the separators, so they keep the one-chain accuracy up to
the separator system's rounding (the numpy study of the same steps: G^R 6e-13 .. 4e-11,
G^< 4e-12 .. 8e-11 of the energy's largest block at eta = 1e-3, n_b = 64, P = 2 .. 8).
  * devices with strong broadening (BT Sigma of 0.2, eta 0.05): every block at 1e-11;
  * eta = 1e-3 long chains (n_b = 64): every block at 1e-9 (G^< / G^> relative to the
    energy's largest block).
"""
import numpy as np
import pytest

import oracle
from paper_2606_25595_amd import inputs

pytestmark = pytest.mark.gpu

RKEYS = ("GR_d", "GR_u", "GR_l")


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_25595_amd import qtx
    c = qtx.Context(0)
    yield c
    c.close()


def solve(ctx, p, P, sigma_diag=False, **kw):
    import torch
    from paper_2606_25595_amd import qtx
    dp = qtx.to_device(p, sigma_diag=sigma_diag)
    dp.partitions = P
    for k in RKEYS + ("GL_d", "GL_u"):
        getattr(dp, k).fill_(float("nan"))
    ctx.solve(dp, **kw)
    torch.cuda.synchronize()
    return dp.outputs()


def errors(out, ref):
    """G^R: max relative Frobenius error per block; G^< / G^>: max block error over the
    energy's largest reference block."""
    r = {}
    for k in RKEYS:
        r[k] = float(oracle.rel_fro_err(out[k], ref[k]).max())
    for k in ("GL_d", "GL_u", "GG_d", "GG_u"):
        if k not in out or k not in ref:
            continue
        d = np.linalg.norm(out[k] - ref[k], axis=(-1, -2)).max(axis=1)
        n = np.linalg.norm(ref[k], axis=(-1, -2)).max(axis=1)
        r[k] = float((d / np.maximum(n, 1e-300)).max())
    return r


def damped(n_b, b, n_e, seed, **kw):
    kw.setdefault("bt_sigma", 0.2)
    kw.setdefault("eta", 0.05)
    return inputs.random_bt_problem(n_b, b, np.linspace(-1.5, 1.4, n_e), seed=seed, **kw)


@pytest.mark.parametrize("n_b,P", [(7, 2), (9, 3), (17, 5), (16, 4), (13, 7), (24, 8), (12, 2)])
def test_partitions_match_oracle_damped(ctx, n_b, P):
    p = damped(n_b, 24, 3, seed=n_b, with_greater=True)
    out = solve(ctx, p, P)
    assert np.all(out["status"] == 0)
    e = errors(out, oracle.dense_selected(p))
    assert max(e.values()) < 1e-11, e


@pytest.mark.parametrize("feature", ["block_diag_sigma", "general_S", "sigma_diag", "no_greater"])
def test_partition_features(ctx, feature):
    kw = dict(with_greater=feature != "no_greater")
    if feature in ("block_diag_sigma", "sigma_diag"):
        kw.update(bt_sigma=0.0, eta=0.3)
    p = damped(14, 20, 3, seed=7, **kw)
    if feature == "general_S":
        rng = np.random.default_rng(5)
        p.S_u = 0.1 * (rng.standard_normal(p.H_u.shape) + 1j * rng.standard_normal(p.H_u.shape))
        p.S_l = np.conj(np.swapaxes(p.S_u, 1, 2))
        p.S_d = np.stack([np.eye(p.b, dtype=np.complex128)] * p.n_b)
    out = solve(ctx, p, 4, sigma_diag=feature == "sigma_diag")
    assert np.all(out["status"] == 0)
    e = errors(out, oracle.dense_selected(p))
    assert max(e.values()) < 1e-11, (feature, e)


@pytest.mark.parametrize("P", [2, 4, 8])
def test_partitions_long_chain_weak_broadening(ctx, P):
    """n_b = 64 at eta = 1e-3 (the paper's regime): the stated bounds, and the
    one-chain GPU solve of the same energies for comparison."""
    p = inputs.random_bt_problem(64, 24, np.linspace(-1.5, 1.3, 3), seed=1, with_greater=True)
    ref = oracle.dense_selected(p)
    out = solve(ctx, p, P)
    assert np.all(out["status"] == 0)
    e = errors(out, ref)
    assert max(e.values()) < 1e-9, e
    one = solve(ctx, p, 0)
    e1 = errors(one, ref)
    assert max(e1.values()) < 1e-10, e1


@pytest.mark.parametrize("scheme,tol", [(dict(prec="int8", n_slices=11), 1e-6),
                                        (dict(prec="fp64", prec_lesser="bf16", n_slices_lesser=4), 1e-5)])
def test_partitions_mixed_precision(ctx, scheme, tol):
    p = damped(20, 64, 4, seed=3, with_greater=False)
    ref = oracle.dense_selected(p)
    out = solve(ctx, p, 4, **scheme)
    assert np.all(out["status"] == 0)
    e = errors(out, ref)
    assert max(e.values()) < tol, e


def test_partitioned_problems_batch_and_graph_replay(ctx):
    """Several problems in one call (two of one layout share launches, a third has its
    own), eager and captured/replayed, bitwise equal to each other."""
    import torch
    from paper_2606_25595_amd import qtx
    probs = [damped(15, 32, 2, seed=11), damped(15, 32, 3, seed=12), damped(11, 32, 2, seed=13)]
    Ps = [3, 3, 2]
    refs = [oracle.dense_selected(p) for p in probs]

    def run():
        dps = []
        for p, P in zip(probs, Ps):
            dp = qtx.to_device(p)
            dp.partitions = P
            dps.append(dp)
        ctx.solve(dps)
        torch.cuda.synchronize()
        return [dp.outputs() for dp in dps]
    eager = run()
    for o, r in zip(eager, refs):
        assert np.all(o["status"] == 0)
        assert max(errors(o, r).values()) < 1e-11
    ctx.set_graph(True)
    try:
        for rep in range(3):
            outs = run()
            for o, ref_o in zip(outs, eager):
                for k in RKEYS + ("GL_d", "GL_u"):
                    assert np.array_equal(o[k], ref_o[k]), (rep, k)
    finally:
        ctx.set_graph(False)


def test_partition_status_nonfinite(ctx):
    """A NaN in the self-energy of an interior block of a middle partition: that energy
    reports QTX_ERR_NONFINITE with every output NaN; the others are unaffected."""
    p = damped(13, 16, 3, seed=4, with_greater=False)
    p.SL_d = p.SL_d.copy()
    p.SL_d[1, 6, 2, 2] = np.nan
    out = solve(ctx, p, 3)
    assert list(out["status"]) == [0, 6, 0]
    for k in RKEYS + ("GL_d", "GL_u"):
        assert np.all(np.isnan(out[k][1])), k
    ref = oracle.dense_selected(p, energy_index=[0, 2])
    good = {k: v[[0, 2]] for k, v in out.items() if k != "status"}
    assert max(errors(good, ref).values()) < 1e-11


def test_partition_arguments(ctx):
    from paper_2606_25595_amd import qtx
    p = damped(6, 8, 1, seed=2)
    dp = qtx.to_device(p)
    dp.partitions = 4                          # needs n_b >= 7
    assert ctx.solve(dp, check=False) == qtx.QTX_ERR_ARG
    dp.partitions = 2
    dp.split = True
    assert ctx.solve(dp, check=False) == qtx.QTX_ERR_ARG
    dp.split = False
    dp.partitions = 65
    assert ctx.solve(dp, check=False) == qtx.QTX_ERR_ARG
