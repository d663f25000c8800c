"""Pins of the FP64 oracle against facts fixed independently of it.

Each test fixes the oracle's result by something other than the oracle itself:
exact rational brute force on tiny systems, closed forms of uniform chains
and strips, hand-derived 2x2 values (tests/golden), and structural identities of
retarded/lesser/greater functions.  Problem statement: Eq. 2 with the G row of
Table I (Section II-A).
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import rgf_oracle
from paper_2606_25595_amd import inputs
from tests.exact_rational import qinv, qmat, qmul, qH, to_complex

SOLVERS = {"dense": oracle.dense_selected, "rgf": oracle.rgf_selected}
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- helpers

def gaussian_int_problem(n_b, b, seed, E=0.5, bt_sigma=True, general_S=True, greater=True):
    """Tiny problem with small Gaussian-integer blocks (exactly representable).
    A strong imaginary diagonal shift keeps M diagonally dominant, so every
    leading block submatrix is nonsingular."""
    rng = np.random.default_rng(seed)

    def gi(*shape):
        return (rng.integers(-3, 4, size=shape) + 1j * rng.integers(-3, 4, size=shape)).astype(np.complex128)

    H_d, H_u, H_l = gi(n_b, b, b), gi(n_b - 1, b, b), gi(n_b - 1, b, b)
    SR_d = gi(1, n_b, b, b)
    for i in range(n_b):
        SR_d[0, i] -= 40j * np.eye(b)          # -Sigma^R adds +40i on the diagonal of M
    p = inputs.BTProblem(energies=np.array([E]), H_d=H_d, H_u=H_u, H_l=H_l, SR_d=SR_d,
                         SL_d=gi(1, n_b, b, b))
    if general_S:
        p.S_d = np.stack([np.eye(b) * 2 for _ in range(n_b)]).astype(np.complex128) + gi(n_b, b, b) * 0.5
        p.S_u = gi(n_b - 1, b, b) * 0.5
        p.S_l = gi(n_b - 1, b, b) * 0.5
    if bt_sigma:
        p.SR_u, p.SR_l = gi(1, n_b - 1, b, b), gi(1, n_b - 1, b, b)
        p.SL_u, p.SL_l = gi(1, n_b - 1, b, b), gi(1, n_b - 1, b, b)
    if greater:
        p.SG_d = gi(1, n_b, b, b)
        if bt_sigma:
            p.SG_u, p.SG_l = gi(1, n_b - 1, b, b), gi(1, n_b - 1, b, b)
    return p


def exact_selected(p):
    """Exact G^R, G^<, G^> of a Gaussian-rational problem (energy 0)."""
    M, Bl, Bg = rgf_oracle.assemble_dense(p, 0)   # assembly of small integers/halves is exact
    Mq = qmat(M)
    G = qinv(Mq)
    GH = qH(G)
    Gl = qmul(qmul(G, qmat(Bl)), GH)
    Gg = qmul(qmul(G, qmat(Bg)), GH) if Bg is not None else None
    return to_complex(G), to_complex(Gl), (to_complex(Gg) if Gg is not None else None)


def blocks_of(Mfull, n_b):
    return inputs.bt_from_dense(Mfull, n_b)


def assert_blocks_close(got, ref, rtol, what=""):
    err = oracle.rel_fro_err(got, ref)
    assert np.all(err <= rtol), "%s max rel err %.3e > %.1e" % (what, err.max(), rtol)


# ---------------------------------------------------------------- P1: exact brute force

@pytest.mark.parametrize("solver", ["dense", "rgf"])
@pytest.mark.parametrize("n_b,b,seed", [(1, 3, 0), (2, 2, 1), (3, 2, 2), (4, 1, 3), (3, 3, 4)])
@pytest.mark.parametrize("bt_sigma,general_S", [(True, True), (False, False)])
def test_exact_rational_bruteforce(solver, n_b, b, seed, bt_sigma, general_S):
    p = gaussian_int_problem(n_b, b, seed, bt_sigma=bt_sigma, general_S=general_S)
    G, Gl, Gg = exact_selected(p)
    out = SOLVERS[solver](p)
    d, u, lo = blocks_of(G, n_b)
    assert_blocks_close(out["GR_d"][0], d, 1e-13, "GR_d")
    if n_b > 1:
        assert_blocks_close(out["GR_u"][0], u, 1e-13, "GR_u")
        assert_blocks_close(out["GR_l"][0], lo, 1e-13, "GR_l")
    d, u, _ = blocks_of(Gl, n_b)
    assert_blocks_close(out["GL_d"][0], d, 1e-12, "GL_d")
    if n_b > 1:
        assert_blocks_close(out["GL_u"][0], u, 1e-12, "GL_u")
    d, u, _ = blocks_of(Gg, n_b)
    assert_blocks_close(out["GG_d"][0], d, 1e-12, "GG_d")
    if n_b > 1:
        assert_blocks_close(out["GG_u"][0], u, 1e-12, "GG_u")


def test_golden_scalar_2x2():
    """Hand-derived 2x2 scalar case (n_b = 2, b = 1): G = adj(M)/det(M),
    G^< = G diag(s1, s2) G^H; values in tests/golden/scalar_2x2.json."""
    with open(os.path.join(GOLDEN, "scalar_2x2.json")) as fh:
        g = json.load(fh)
    c = lambda v: complex(v[0], v[1])
    p = inputs.BTProblem(
        energies=np.array([g["E"]]),
        H_d=np.array([[[c(g["H11"])]], [[c(g["H22"])]]]),
        H_u=np.array([[[c(g["H12"])]]]), H_l=np.array([[[c(g["H21"])]]]),
        SR_d=np.array([[[[c(g["SR1"])]], [[c(g["SR2"])]]]]),
        SL_d=np.array([[[[c(g["SL1"])]], [[c(g["SL2"])]]]]))
    for solver in SOLVERS.values():
        out = solver(p)
        for key, ref in g["expect"].items():
            name, i = key.split(":")
            got = out[name][0, int(i), 0, 0]
            assert abs(got - c(ref)) <= 4e-15 * max(1.0, abs(c(ref))), (key, got, ref)


# ---------------------------------------------------------------- P3: uniform 1D chain

CHAIN_E = [-1.7, -0.9, -0.25, 0.0, 0.4, 1.3, 1.85]
CHAIN_E_OUT = [-2.6, 2.4, 3.5]


def chain_closed_form(N, E, t, fL, fR):
    lam = inputs.chain_lead_lambda(E, 0.0, t)
    c = 1.0 / (t * (1.0 / lam - lam))
    gam = inputs.chain_gamma(E, 0.0, t)
    j = np.arange(N)
    G = c * lam ** np.abs(j[:, None] - j[None, :])
    Gl = 1j * gam * c * np.conj(c) * (fL * np.outer(lam ** j, np.conj(lam) ** j)
                                      + fR * np.outer(lam ** (N - 1 - j), np.conj(lam) ** (N - 1 - j)))
    return G, Gl, gam


@pytest.mark.parametrize("solver", ["dense", "rgf"])
@pytest.mark.parametrize("n_b,b", [(1, 6), (6, 1), (4, 3), (3, 5)])
def test_chain_closed_form(solver, n_b, b):
    t = -1.0
    E = np.array(CHAIN_E + CHAIN_E_OUT)
    p = inputs.uniform_chain(n_b, b, E, t=t)
    out = SOLVERS[solver](p)
    N = n_b * b
    for k, En in enumerate(E):
        G, Gl, gam = chain_closed_form(N, En, t, p.f_L[k], p.f_R[k])
        d, u, lo = blocks_of(G, n_b)
        assert_blocks_close(out["GR_d"][k], d, 1e-12, "chain GR_d")
        if n_b > 1:
            assert_blocks_close(out["GR_u"][k], u, 1e-12, "chain GR_u")
            assert_blocks_close(out["GR_l"][k], lo, 1e-12, "chain GR_l")
        d, u, _ = blocks_of(Gl, n_b)
        if gam > 0:
            assert_blocks_close(out["GL_d"][k], d, 1e-11, "chain GL_d")
            if n_b > 1:
                assert_blocks_close(out["GL_u"][k], u, 1e-11, "chain GL_u")
        else:
            assert np.abs(out["GL_d"][k]).max() == 0.0
            assert np.abs(G.imag).max() < 1e-12          # out of band: G^R is real


@pytest.mark.parametrize("solver", ["dense", "rgf"])
def test_chain_transmission_and_currents(solver):
    t = -1.0
    n_b, b = 5, 2
    E = np.array(CHAIN_E + CHAIN_E_OUT)
    p = inputs.uniform_chain(n_b, b, E, t=t)
    out = SOLVERS[solver](p)
    gam = np.array([inputs.chain_gamma(x, 0.0, t) for x in E])
    gL = np.zeros((E.size, b, b), complex)
    gL[:, 0, 0] = gam
    T = oracle.transmission_left(out["GR_d"][:, 0], gL)
    inband = np.abs(E) < 2.0
    np.testing.assert_allclose(T[inband], 1.0, atol=1e-12)
    np.testing.assert_allclose(T[~inband], 0.0, atol=1e-12)
    jL = oracle.contact_current_left(out["GR_d"][:, 0], out["GL_d"][:, 0], gL, p.f_L)
    np.testing.assert_allclose(jL, (p.f_L - p.f_R) * inband, atol=1e-12)
    J = oracle.bond_currents(p, out["GL_u"])
    np.testing.assert_allclose(J, np.repeat(((p.f_L - p.f_R) * inband)[:, None], n_b - 1, 1), atol=1e-12)


# ---------------------------------------------------------------- P4: uniform strip

@pytest.mark.parametrize("n_b,b", [(3, 4), (5, 7), (2, 16)])
def test_strip_closed_form(n_b, b):
    t_x, t_y = -1.0, -0.7
    m = np.arange(1, b + 1)
    eps_m = 2.0 * t_y * np.cos(np.pi * m / (b + 1))
    # keep energies away from every mode threshold eps_m +- 2|t_x|
    cand = np.linspace(-3.2, 3.2, 41)
    thr = np.concatenate([eps_m - 2 * abs(t_x), eps_m + 2 * abs(t_x)])
    E = np.array([x for x in cand if np.min(np.abs(x - thr)) > 2e-2])[:12]
    p = inputs.uniform_strip(n_b, b, E, t_x=t_x, t_y=t_y)
    out = oracle.rgf_selected(p)
    y = np.arange(1, b + 1)
    phi = np.sqrt(2.0 / (b + 1)) * np.sin(np.pi * np.outer(y, m) / (b + 1))
    T = oracle.transmission_left(out["GR_d"][:, 0], p.gamma_L)
    for k, En in enumerate(E):
        lam = np.array([inputs.chain_lead_lambda(En, em, t_x) for em in eps_m])
        c = 1.0 / (t_x * (1.0 / lam - lam))
        Gd = phi @ np.diag(c) @ phi.T
        Gu = phi @ np.diag(c * lam) @ phi.T
        for i in range(n_b):
            assert_blocks_close(out["GR_d"][k, i], Gd, 1e-11, "strip GR_d")
        for i in range(n_b - 1):
            assert_blocks_close(out["GR_u"][k, i], Gu, 1e-11, "strip GR_u")
            assert_blocks_close(out["GR_l"][k, i], Gu, 1e-11, "strip GR_l")
        n_open = int(np.sum(np.abs(En - eps_m) < 2 * abs(t_x)))
        assert abs(T[k] - n_open) < 1e-9, (En, T[k], n_open)


# ---------------------------------------------------------------- invariants P6-P12

@pytest.fixture(scope="module")
def rand_problem():
    E = np.linspace(-2.0, 2.0, 9)
    return inputs.random_bt_problem(5, 6, E, seed=3, with_greater=True)


@pytest.fixture(scope="module")
def rand_out(rand_problem):
    return oracle.rgf_selected(rand_problem)


def test_lesser_skew_hermitian_and_bounded(rand_problem, rand_out):
    o = rand_out
    for k in range(rand_problem.n_e):
        for i in range(rand_problem.n_b):
            Gl = o["GL_d"][k, i]
            scale = np.linalg.norm(Gl)
            assert np.linalg.norm(Gl + Gl.conj().T) <= 1e-12 * scale + 1e-300
            Hm = -1j * Gl
            Hm = 0.5 * (Hm + Hm.conj().T)
            assert np.linalg.eigvalsh(Hm).min() >= -1e-12 * scale
            G = o["GR_d"][k, i]
            A = 1j * (G - G.conj().T)
            A = 0.5 * (A + A.conj().T)
            # 0 <= f <= 1  =>  -iG^< <= A  (occupation bounded by the density of states)
            assert np.linalg.eigvalsh(A - Hm).min() >= -1e-11 * np.linalg.norm(A)


def test_retarded_minus_advanced_equals_greater_minus_lesser(rand_problem, rand_out):
    o = rand_out
    for k in range(rand_problem.n_e):
        for i in range(rand_problem.n_b):
            lhs = o["GR_d"][k, i] - o["GR_d"][k, i].conj().T
            rhs = o["GG_d"][k, i] - o["GL_d"][k, i]
            assert np.linalg.norm(lhs - rhs) <= 1e-11 * np.linalg.norm(lhs)
        for i in range(rand_problem.n_b - 1):
            lhs = o["GR_u"][k, i] - o["GR_l"][k, i].conj().T
            rhs = o["GG_u"][k, i] - o["GL_u"][k, i]
            assert np.linalg.norm(lhs - rhs) <= 1e-11 * np.linalg.norm(lhs)


def test_equilibrium_fluctuation_dissipation():
    E = np.linspace(-1.5, 1.5, 7)
    p = inputs.random_bt_problem(4, 5, E, seed=11, mu_L=0.05, mu_R=0.05)
    o = oracle.rgf_selected(p)
    f = inputs.fermi(E, 0.05, 0.025)
    for k in range(E.size):
        for i in range(p.n_b):
            G = o["GR_d"][k, i]
            ref = -f[k] * (G - G.conj().T)
            assert np.linalg.norm(o["GL_d"][k, i] - ref) <= 1e-11 * np.linalg.norm(G)
        for i in range(p.n_b - 1):
            ref = -f[k] * (o["GR_u"][k, i] - o["GR_l"][k, i].conj().T)
            assert np.linalg.norm(o["GL_u"][k, i] - ref) <= 1e-11 * np.linalg.norm(o["GR_u"][k, i])


def test_power_of_two_scaling_is_bitwise(rand_problem):
    p = rand_problem
    o1 = oracle.rgf_selected(p)
    q = inputs.BTProblem(**{**p.__dict__})
    q.SL_d = p.SL_d * 8.0
    o2 = oracle.rgf_selected(q)
    for key in ("GL_d", "GL_u"):
        assert np.array_equal(o2[key], o1[key] * 8.0)
    for key in ("GR_d", "GR_u", "GR_l"):
        assert np.array_equal(o2[key], o1[key])


def test_block_reversal(rand_problem):
    p = rand_problem
    o = oracle.rgf_selected(p)
    rev = inputs.BTProblem(
        energies=p.energies, H_d=p.H_d[::-1].copy(), H_u=p.H_l[::-1].copy(), H_l=p.H_u[::-1].copy(),
        SR_d=p.SR_d[:, ::-1].copy(), SL_d=p.SL_d[:, ::-1].copy())
    r = oracle.rgf_selected(rev)
    n = p.n_b
    for k in range(p.n_e):
        for i in range(n):
            assert_blocks_close(r["GR_d"][k, i], o["GR_d"][k, n - 1 - i], 1e-11, "rev GR_d")
            assert_blocks_close(r["GL_d"][k, i], o["GL_d"][k, n - 1 - i], 1e-10, "rev GL_d")
        for i in range(n - 1):
            assert_blocks_close(r["GR_u"][k, i], o["GR_l"][k, n - 2 - i], 1e-11, "rev GR_u")
            assert_blocks_close(r["GR_l"][k, i], o["GR_u"][k, n - 2 - i], 1e-11, "rev GR_l")
            # G^<_{i+1,i} = -(G^<_{i,i+1})^H
            assert_blocks_close(r["GL_u"][k, i], -o["GL_u"][k, n - 2 - i].conj().T, 1e-10, "rev GL_u")


def test_reciprocity_real_symmetric():
    E = np.linspace(-1.0, 1.0, 5)
    p = inputs.random_bt_problem(4, 5, E, seed=5)
    p.H_d = p.H_d.real.astype(np.complex128)
    p.H_d = 0.5 * (p.H_d + np.transpose(p.H_d, (0, 2, 1)))
    p.H_u = p.H_u.real.astype(np.complex128)
    p.H_l = np.ascontiguousarray(np.transpose(p.H_u, (0, 2, 1)))
    o = oracle.rgf_selected(p)
    for k in range(p.n_e):
        for i in range(p.n_b):
            assert_blocks_close(o["GR_d"][k, i].T, o["GR_d"][k, i], 1e-12, "recip GR_d")
        for i in range(p.n_b - 1):
            assert_blocks_close(o["GR_l"][k, i], o["GR_u"][k, i].T, 1e-12, "recip GR_l")


def test_current_conservation_without_eta():
    E = np.linspace(-1.8, 1.8, 7)
    p = inputs.random_bt_problem(6, 4, E, seed=8, eta=0.0)
    o = oracle.rgf_selected(p)
    jL = oracle.contact_current_left(o["GR_d"][:, 0], o["GL_d"][:, 0], p.gamma_L, p.f_L)
    J = oracle.bond_currents(p, o["GL_u"])
    scale = np.max(np.abs(jL)) + 1e-300
    assert np.max(np.abs(J - jL[:, None])) <= 1e-10 * scale
    # the right contact sees the same current leaving
    jR = oracle.contact_current_left(o["GR_d"][:, -1], o["GL_d"][:, -1], p.gamma_R, p.f_R)
    assert np.max(np.abs(jR + jL)) <= 1e-10 * scale


def test_dense_and_rgf_agree_on_tiny_workload():
    p = inputs.config_problem("tiny")
    d = oracle.dense_selected(p)
    r = oracle.rgf_selected(p)
    for key in ("GR_d", "GR_u", "GR_l"):
        assert oracle.rel_fro_err(r[key], d[key]).max() < 1e-11
    for key in ("GL_d", "GL_u"):
        assert oracle.rel_fro_err(r[key], d[key]).max() < 1e-10


@pytest.mark.parametrize("bt_sigma", [0.0, 0.05])
def test_schur_complements_are_leading_submatrix_inverses(bt_sigma):
    """Each forward Schur complement S_i inverts to the last diagonal block of the
    inverse of the leading (i+1)-block submatrix of M (dense inverse, LAPACK), so
    the last one inverts to G^R_nn; the first is A_0 itself."""
    p = inputs.random_bt_problem(5, 7, np.array([-0.8, 0.45]), seed=17, bt_sigma=bt_sigma)
    b = p.b
    for e in range(p.n_e):
        M = oracle.assemble_dense(p, e)[0]
        S = oracle.schur_complements(p, e)
        assert len(S) == p.n_b
        np.testing.assert_array_equal(S[0], M[:b, :b])
        for i in range(p.n_b):
            k = (i + 1) * b
            lead_inv = np.linalg.inv(M[:k, :k])
            np.testing.assert_allclose(np.linalg.inv(S[i]), lead_inv[k - b:k, k - b:k], rtol=0, atol=1e-12)
