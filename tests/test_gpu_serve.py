"""Serving loop on the GPU: continuous batching gives each request the same
result as solving it alone, and the FP64 results match the oracle."""
import numpy as np
import pytest

import oracle
from paper_2606_25595_amd import inputs
from paper_2606_25595_amd.serve import GpuExecutor, Request, Server, request_stream

pytestmark = pytest.mark.gpu
KEYS = ("GR_d", "GR_u", "GR_l", "GL_d", "GL_u")


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def small_stream(seed, n_max=12):
    reqs = request_stream(rate=400.0, duration=0.05, seed=seed, b_choices=[32, 48, 64], nb_range=(3, 6),
                          ne_range=(3, 9), mixed_fraction=0.5)[:n_max]
    for r in reqs:
        r.keep_blocks = True
    return reqs


def run_server(reqs, n_slots=3, chunk=4, budget=1 << 31):
    ex = GpuExecutor(n_slots=n_slots, workspace_per_slot=1 << 30)
    try:
        srv = Server(ex, hbm_budget=budget, chunk_energies=chunk)
        rep = srv.run(reqs)
    finally:
        ex.close()
    return srv, rep


def clone(r):
    return Request(rid=r.rid, b=r.b, n_b=r.n_b, n_e=r.n_e, seed=r.seed, precision=r.precision, keep_blocks=True)


def test_mix_equals_alone_and_matches_oracle(gpu):
    reqs = small_stream(seed=4)
    srv, rep = run_server(reqs)
    assert rep["completed"] == len(reqs) and rep["rejected"] == 0
    assert srv.max_chunks_per_launch > 1                         # requests were batched together
    for r in reqs:
        assert np.all(r.status == 0)
        # the same request alone (fresh server, one slot, whole request in one chunk)
        alone = clone(r)
        run_server([alone], n_slots=1, chunk=64)
        for k in KEYS:
            assert np.array_equal(alone.blocks[k], r.blocks[k]), (r.rid, k)
        assert np.array_equal(alone.T_L, r.T_L)
    # FP64 requests against the oracle on the device's own inputs
    for r in [q for q in reqs if q.precision == "fp64"][:3]:
        sr, sl = inputs.random_bt_scalars(r.n_b, r.energies)
        p = inputs.BTProblem(energies=r.energies, H_d=r.blocks["H_d"], H_u=r.blocks["H_u"], H_l=r.blocks["H_l"],
                             SR_d=inputs._diag_blocks(sr, r.b), SL_d=inputs._diag_blocks(sl, r.b))
        ref = oracle.rgf_selected(p)
        for k in KEYS:
            assert oracle.rel_fro_err(r.blocks[k], ref[k]).max() <= 1e-10, (r.rid, k)
        T = oracle.transmission_left(ref["GR_d"][:, 0], 2.0 * 0.5 * np.eye(r.b))
        np.testing.assert_allclose(r.T_L, T, rtol=1e-9, atol=1e-12)
    # mixed-precision requests meet the 1e-6 bar
    mixed = [q for q in reqs if q.precision == "mixed"][:3]
    assert mixed
    for r in mixed:
        sr, sl = inputs.random_bt_scalars(r.n_b, r.energies)
        p = inputs.BTProblem(energies=r.energies, H_d=r.blocks["H_d"], H_u=r.blocks["H_u"], H_l=r.blocks["H_l"],
                             SR_d=inputs._diag_blocks(sr, r.b), SL_d=inputs._diag_blocks(sl, r.b))
        ref = oracle.rgf_selected(p)
        for k in KEYS:
            assert oracle.rel_fro_err(r.blocks[k], ref[k]).max() <= 1e-6, (r.rid, k)


def test_budget_bounds_admission(gpu):
    reqs = small_stream(seed=9, n_max=6)
    one_chunk = max(4 * (7 * r.n_b - 3) * r.b * r.b * 16 + (3 * r.n_b - 2) * r.b * r.b * 16 for r in reqs)
    srv, rep = run_server(reqs, budget=one_chunk)                 # roughly one chunk at a time
    assert rep["completed"] == len(reqs)
    assert srv.peak_used <= one_chunk


def test_split_chains_in_serving_match_oracle(gpu):
    """The executor's split option (two half-chains per energy) serves the same
    requests with FP64 results at the oracle's bar."""
    reqs = [r for r in small_stream(seed=11, n_max=8)]
    ex = GpuExecutor(n_slots=2, workspace_per_slot=1 << 30, split=True)
    try:
        srv = Server(ex, hbm_budget=1 << 31, chunk_energies=4)
        rep = srv.run(reqs)
    finally:
        ex.close()
    assert rep["completed"] == len(reqs)
    for r in reqs:
        assert np.all(r.status == 0)
        sr, sl = inputs.random_bt_scalars(r.n_b, r.energies)
        p = inputs.BTProblem(energies=r.energies, H_d=r.blocks["H_d"], H_u=r.blocks["H_u"], H_l=r.blocks["H_l"],
                             SR_d=inputs._diag_blocks(sr, r.b), SL_d=inputs._diag_blocks(sl, r.b))
        ref = oracle.rgf_selected(p)
        tol = 1e-10 if r.precision == "fp64" else 1e-6
        for k in KEYS:
            assert oracle.rel_fro_err(r.blocks[k], ref[k]).max() <= tol, (r.rid, k)


def wide_stream(seed):
    """Requests of the realistic block size (b = 256) arriving together."""
    reqs = request_stream(rate=2000.0, duration=0.004, seed=seed, b_choices=[256], nb_range=(3, 5),
                          ne_range=(3, 7), mixed_fraction=0.5)
    assert len(reqs) >= 4
    for r in reqs:
        r.keep_blocks = True
    return reqs


def serve_with(reqs, **ex_kw):
    ex = GpuExecutor(n_slots=3, workspace_per_slot=1 << 30, **ex_kw)
    try:
        srv = Server(ex, hbm_budget=1 << 31, chunk_energies=4)
        rep = srv.run(reqs)
    finally:
        ex.close()
    return srv, rep


@pytest.mark.parametrize("out_bits", [32, 48])
def test_compact_executor_at_b256(gpu, out_bits):
    """The executor's compact forms (self-energies as b-vectors, FPX off-diagonal
    outputs) on b = 256 requests: diagonal blocks and observables bitwise equal to the
    dense executor's, FPX bytes equal to the oracle's encoding of the dense executor's
    blocks, and the dense executor's FP64 results at the oracle's bar."""
    dense = wide_stream(seed=21)
    compact = [clone(r) for r in dense]
    _, rep_d = serve_with(dense)
    srv_c, rep_c = serve_with(compact, sigma_diag=True, out_bits=out_bits)
    assert rep_d["completed"] == rep_c["completed"] == len(dense)
    for rd, rc in zip(dense, compact):
        assert np.all(rd.status == 0) and np.all(rc.status == 0)
        for k in ("GR_d", "GL_d"):
            assert np.array_equal(rd.blocks[k], rc.blocks[k]), (rd.rid, k)
        assert np.array_equal(rd.T_L, rc.T_L) and np.array_equal(rd.j_L, rc.j_L)
        for k in ("GR_u", "GR_l", "GL_u"):
            v = rd.blocks[k]
            flat = np.ascontiguousarray(v).view(np.float64).reshape(v.shape[0], v.shape[1], -1)
            want = oracle.fpx_encode(flat, out_bits).reshape(v.shape[0], v.shape[1], -1)
            assert rc.blocks[k].dtype == np.uint8 and np.array_equal(rc.blocks[k], want), (rd.rid, k)
    for r in [q for q in dense if q.precision == "fp64"][:2]:
        sr, sl = inputs.random_bt_scalars(r.n_b, r.energies)
        p = inputs.BTProblem(energies=r.energies, H_d=r.blocks["H_d"], H_u=r.blocks["H_u"], H_l=r.blocks["H_l"],
                             SR_d=inputs._diag_blocks(sr, r.b), SL_d=inputs._diag_blocks(sl, r.b))
        ref = oracle.rgf_selected(p)
        for k in KEYS:
            assert oracle.rel_fro_err(r.blocks[k], ref[k]).max() <= 1e-10, (r.rid, k)
