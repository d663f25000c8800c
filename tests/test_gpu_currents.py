"""Transport observables computed on the GPU from the GPU's own outputs, through the
C ABI: the right-contact transmission and current, and the bond currents
J_i = 2 Re Tr[(H - E S)_{i,i+1} G^<_{i+1,i}] (Section II-B takes the current and its
conservation as the accuracy criterion).

With no broadening inside the device (eta = 0, contacts on the first and last block)
current is conserved: every bond carries the current that enters from the left and
leaves through the right contact (Kirchhoff), and T_L = T_R.
"""
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


def solve(ctx, p, **kw):
    import torch
    from paper_2606_25595_amd import qtx
    dp = qtx.to_device(p)
    ctx.solve(dp, **kw)
    torch.cuda.synchronize()
    return dp


def test_bond_current_kernel_matches_host_formula(ctx):
    """The kernel's J from the GPU's G^< equals the host formula on the same blocks,
    also with a general S (E S_{i,i+1} enters the coupling)."""
    p = inputs.random_bt_problem(5, 40, np.linspace(-1.5, 1.6, 6), seed=31)
    dp = solve(ctx, p)
    J = ctx.bond_currents(dp).cpu().numpy()
    ref = oracle.bond_currents(p, dp.GL_u.cpu().numpy())
    np.testing.assert_allclose(J, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    # general S: the coupling is H_u - E S_u
    rng = np.random.default_rng(4)
    p.S_u = 0.1 * (rng.standard_normal(p.H_u.shape) + 1j * rng.standard_normal(p.H_u.shape))
    p.S_l = np.conj(np.swapaxes(p.S_u, 1, 2))
    p.S_d = np.stack([np.eye(p.b, dtype=np.complex128)] * p.n_b)
    from paper_2606_25595_amd import qtx
    import torch
    dp2 = qtx.to_device(p)
    ctx.solve(dp2)
    torch.cuda.synchronize()
    J2 = ctx.bond_currents(dp2).cpu().numpy()
    ref2 = oracle.bond_currents(p, dp2.GL_u.cpu().numpy())
    np.testing.assert_allclose(J2, ref2, rtol=1e-12, atol=1e-12 * np.abs(ref2).max())


@pytest.mark.parametrize("scheme,tol", [(dict(prec="fp64"), 1e-10),
                                        (dict(prec="fp64", split=True), 1e-10),
                                        (dict(prec="int8", n_slices=10, prec_lesser="int8", n_slices_lesser=10), 1e-6)])
def test_current_conservation_on_gpu_outputs(ctx, scheme, tol):
    """eta = 0: J_i = j_L = -j_R for every bond and energy, T_L = T_R, all computed on
    the GPU from the GPU's blocks; and each agrees with the oracle's value."""
    import torch
    from paper_2606_25595_amd import qtx
    kw = dict(scheme)
    split = kw.pop("split", False)
    E = np.linspace(-1.8, 1.8, 9)
    p = inputs.random_bt_problem(7, 32, E, seed=12, eta=0.0)
    dp = qtx.to_device(p)
    dp.split = split
    ctx.solve(dp, **kw)
    torch.cuda.synchronize()
    assert np.all(dp.status.cpu().numpy() == 0)
    TL, jL = (x.cpu().numpy() for x in ctx.observables(dp, p.gamma_L, p.f_L))
    TR, jR = (x.cpu().numpy() for x in ctx.observables_right(dp, p.gamma_R, p.f_R))
    J = ctx.bond_currents(dp).cpu().numpy()
    scale = np.abs(jL).max()
    assert scale > 1e-3                                      # a current flows (mu_L > mu_R)
    assert np.abs(J - jL[:, None]).max() <= tol * scale
    assert np.abs(jR + jL).max() <= tol * scale
    assert np.abs(TL - TR).max() <= tol * max(np.abs(TL).max(), 1.0)
    # against the oracle's observables
    ref = oracle.rgf_selected(p)
    Jref = oracle.bond_currents(p, ref["GL_u"])
    TRref = oracle.transmission_left(ref["GR_d"][:, -1], p.gamma_R)
    jRref = oracle.contact_current_left(ref["GR_d"][:, -1], ref["GL_d"][:, -1], p.gamma_R, p.f_R)
    assert np.abs(J - Jref).max() <= tol * scale
    assert np.abs(jR - jRref).max() <= tol * scale
    assert np.abs(TR - TRref).max() <= tol * max(np.abs(TRref).max(), 1.0)


def test_bond_currents_rejects_bad_arguments(ctx):
    import torch
    from paper_2606_25595_amd import qtx
    lib = ctx.lib
    J = torch.empty((2, 2), dtype=torch.float64, device="cuda")
    x = torch.zeros((3, 4, 4), dtype=torch.complex128, device="cuda")
    E = torch.zeros(2, dtype=torch.float64, device="cuda")
    p = lambda t: qtx._ptr(t)  # noqa: E731
    assert lib.qtx_rgf_bond_currents(ctx.handle, 4, 1, 2, p(x), None, p(E), p(x), 16, p(J), None) == qtx.QTX_ERR_ARG
    assert lib.qtx_rgf_bond_currents(ctx.handle, 4, 3, 2, None, None, p(E), p(x), 32, p(J), None) == qtx.QTX_ERR_ARG
    assert lib.qtx_rgf_bond_currents(ctx.handle, 4, 3, 2, p(x), None, p(E), p(x), 16, p(J), None) == qtx.QTX_ERR_ARG
    assert lib.qtx_rgf_bond_currents(ctx.handle, 4, 3, 2, p(x), None, p(E), p(x), 32, p(J), None) == qtx.QTX_OK
