"""Seeded synthetic inputs for the block-tridiagonal (BT) Green's-function solve.

This module only *builds inputs*: random Hamiltonian blocks, the contact and
broadening self-energies and the energy grid.  It holds none of the solver's
arithmetic, so both the CPU oracle and the GPU library can take their inputs
from it without sharing any of the method.

The system solved per energy is the G row of the paper's Table I applied to
Eq. (2): M(E) = E*S - H - Sigma^R(E) and B = Sigma^<(E) (Section II-A).  The
matrices are quasi-banded and tiled into BT form with n_b diagonal blocks of
size b (Section II-A).  Lesser quantities are skew-Hermitian (Section II-A),
which the generated Sigma^< and Sigma^> respect.

Layout (all numpy, complex128, C-contiguous):
  H_d [n_b][b][b], H_u [n_b-1][b][b] (block (i,i+1)), H_l [n_b-1][b][b] (block (i+1,i))
  S_d/S_u/S_l: same layout, or None for S = I
  SR_d [n_e][n_b][b][b]; SR_u/SR_l [n_e][n_b-1][b][b] or None (block-diagonal)
  SL_* : Sigma^<, same layout;  SG_* : Sigma^> or None
Energies are float64 [n_e].  gamma_L / gamma_R are the b x b contact
broadening matrices (only the contact part, without eta) used for the
transmission; f_L / f_R are the contact occupations per energy.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

__all__ = [
    "BTProblem", "fermi", "random_hamiltonian", "random_bt_problem",
    "config_problem", "uniform_chain", "uniform_strip", "chain_lead_lambda",
    "CONFIGS", "bt_from_dense", "WProblem", "random_w_problem", "w_base_matrices", "w_scalars",
]


@dataclasses.dataclass
class BTProblem:
    energies: np.ndarray
    H_d: np.ndarray
    H_u: np.ndarray
    H_l: np.ndarray
    SR_d: np.ndarray
    SL_d: np.ndarray
    S_d: Optional[np.ndarray] = None
    S_u: Optional[np.ndarray] = None
    S_l: Optional[np.ndarray] = None
    SR_u: Optional[np.ndarray] = None
    SR_l: Optional[np.ndarray] = None
    SL_u: Optional[np.ndarray] = None
    SL_l: Optional[np.ndarray] = None
    SG_d: Optional[np.ndarray] = None
    SG_u: Optional[np.ndarray] = None
    SG_l: Optional[np.ndarray] = None
    gamma_L: Optional[np.ndarray] = None
    gamma_R: Optional[np.ndarray] = None
    f_L: Optional[np.ndarray] = None
    f_R: Optional[np.ndarray] = None

    @property
    def n_b(self) -> int:
        return int(self.H_d.shape[0])

    @property
    def b(self) -> int:
        return int(self.H_d.shape[1])

    @property
    def n_e(self) -> int:
        return int(self.energies.shape[0])

    def subset(self, idx) -> "BTProblem":
        """The same device restricted to the energies `idx` (a list/array)."""
        idx = np.asarray(idx, dtype=np.int64)
        out = dataclasses.replace(self)
        out.energies = self.energies[idx].copy()
        for name in ("SR_d", "SR_u", "SR_l", "SL_d", "SL_u", "SL_l", "SG_d", "SG_u", "SG_l"):
            v = getattr(self, name)
            if v is not None:
                setattr(out, name, np.ascontiguousarray(v[idx]))
        for name in ("f_L", "f_R"):
            v = getattr(self, name)
            if v is not None:
                setattr(out, name, v[idx].copy())
        return out


def fermi(E, mu, kT):
    """Fermi-Dirac occupation 1/(1+exp((E-mu)/kT)), written overflow-free."""
    x = -(np.asarray(E, dtype=np.float64) - mu) / kT
    return np.where(x >= 0, 1.0 / (1.0 + np.exp(-np.abs(x))), np.exp(-np.abs(x)) / (1.0 + np.exp(-np.abs(x))))


def random_hamiltonian(n_b: int, b: int, seed: int, coupling_var: float = 0.5):
    """Random Hermitian BT Hamiltonian.

    Diagonal blocks: H_ii = (X + X^H) / sqrt(2b) with X = (R + iJ)/sqrt(2), R, J iid N(0,1):
    Hermitian, real diagonal ~ N(0,1)/sqrt(b), off-diagonal E|h|^2 = 1/b.
    Couplings: H_{i,i+1} = sqrt(coupling_var/b) * (R + iJ)/sqrt(2) (circular complex normal,
    E|h|^2 = coupling_var/b) and H_{i+1,i} = H_{i,i+1}^H so that H is Hermitian.
    Draw order from numpy PCG64(seed): for each i, R then J of X_i; then for each coupling, R then J.
    """
    rng = np.random.default_rng(seed)
    H_d = np.empty((n_b, b, b), dtype=np.complex128)
    for i in range(n_b):
        R = rng.standard_normal((b, b))
        J = rng.standard_normal((b, b))
        X = (R + 1j * J) / math.sqrt(2.0)
        H_d[i] = (X + X.conj().T) / math.sqrt(2.0 * b)
    H_u = np.empty((max(n_b - 1, 0), b, b), dtype=np.complex128)
    for i in range(n_b - 1):
        R = rng.standard_normal((b, b))
        J = rng.standard_normal((b, b))
        H_u[i] = math.sqrt(coupling_var / b) * (R + 1j * J) / math.sqrt(2.0)
    H_l = np.ascontiguousarray(np.conj(np.transpose(H_u, (0, 2, 1))))
    return H_d, H_u, H_l


def _diag_blocks(scal: np.ndarray, b: int) -> np.ndarray:
    """[n_e][n_b] complex scalars -> [n_e][n_b][b][b] blocks scal*I."""
    n_e, n_b = scal.shape
    out = np.zeros((n_e, n_b, b, b), dtype=np.complex128)
    ii = np.arange(b)
    out[:, :, ii, ii] = scal[:, :, None]
    return out


def random_bt_problem(n_b: int, b: int, energies, seed: int = 0, eta: float = 1e-3,
                      gamma: float = 0.5, mu_L: float = 0.1, mu_R: float = -0.1, kT: float = 0.025,
                      with_greater: bool = False, coupling_var: float = 0.5,
                      bt_sigma: float = 0.0) -> BTProblem:
    """The synthetic device used throughout: random Hermitian BT H, S = I,
    Sigma^R_ii = -i(eta + gamma_i) I with gamma_i = gamma on the first and last block,
    Sigma^< = -f_i(E) (Sigma^R - Sigma^R^H) with f_i the Fermi function at mu_i,
    mu_i linear from mu_L (block 1) to mu_R (block n_b), temperature kT.
    Sigma^> = Sigma^< + Sigma^R - Sigma^A when requested.

    bt_sigma = c > 0 makes every self-energy BT: Sigma^R = -i(eta + gamma_i + K) with K
    the Hermitian BT matrix of diagonal blocks 2c I and upper blocks K_i = c X_i / |X_i|_F
    (X_i circular complex normal, drawn from PCG64([seed, 1])), which is positive
    semidefinite, so the anti-Hermitian part of M stays >= eta.  The off-diagonal
    blocks of Sigma^< take the mean occupation of the two blocks they couple, which
    keeps Sigma^< skew-Hermitian: Sigma^<_{i,i+1} = 2i fbar_i K_i,
    Sigma^<_{i+1,i} = 2i fbar_i K_i^H, Sigma^>_{i,i+1} = 2i (fbar_i - 1) K_i.
    """
    energies = np.atleast_1d(np.asarray(energies, dtype=np.float64))
    H_d, H_u, H_l = random_hamiltonian(n_b, b, seed, coupling_var)
    gam = np.zeros(n_b)
    gam[0] += gamma
    gam[-1] += gamma
    broad = eta + gam                                   # [n_b]
    bt = bt_sigma > 0 and n_b > 1
    if bt:
        broad = broad + 2.0 * bt_sigma
    mu = np.linspace(mu_L, mu_R, n_b)
    f = fermi(energies[:, None], mu[None, :], kT)        # [n_e][n_b]
    sr = np.broadcast_to(-1j * broad[None, :], (energies.size, n_b))
    # Sigma^R - Sigma^A = -2i*broad  ->  Sigma^< = 2i f broad
    sl = 2j * f * broad[None, :]
    prob = BTProblem(
        energies=energies, H_d=H_d, H_u=H_u, H_l=H_l,
        SR_d=_diag_blocks(np.asarray(sr), b), SL_d=_diag_blocks(sl, b),
        gamma_L=2.0 * gamma * np.eye(b, dtype=np.complex128),
        gamma_R=2.0 * gamma * np.eye(b, dtype=np.complex128),
        f_L=fermi(energies, mu_L, kT), f_R=fermi(energies, mu_R, kT))
    if with_greater:
        # Sigma^> = Sigma^< + Sigma^R - Sigma^A = 2i f broad - 2i broad
        prob.SG_d = _diag_blocks(2j * (f - 1.0) * broad[None, :], b)
    if bt:
        rng = np.random.default_rng([seed, 1])
        K = np.empty((n_b - 1, b, b), dtype=np.complex128)
        for i in range(n_b - 1):
            R = rng.standard_normal((b, b))
            J = rng.standard_normal((b, b))
            X = R + 1j * J
            K[i] = bt_sigma * X / np.linalg.norm(X)
        KH = np.conj(np.transpose(K, (0, 2, 1)))
        fbar = 0.5 * (f[:, :-1] + f[:, 1:])               # [n_e][n_b-1]
        n_e = energies.size
        prob.SR_u = np.ascontiguousarray(np.broadcast_to(-1j * K, (n_e,) + K.shape))
        prob.SR_l = np.ascontiguousarray(np.broadcast_to(-1j * KH, (n_e,) + K.shape))
        prob.SL_u = 2j * fbar[:, :, None, None] * K[None]
        prob.SL_l = 2j * fbar[:, :, None, None] * KH[None]
        if with_greater:
            prob.SG_u = 2j * (fbar[:, :, None, None] - 1.0) * K[None]
            prob.SG_l = 2j * (fbar[:, :, None, None] - 1.0) * KH[None]
    return prob


# Shapes of the workloads (tiny, realistic, precision, batching, serving).
CONFIGS = {
    "tiny": dict(n_b=8, b=16, n_e=32),
    "realistic": dict(n_b=32, b=416, n_e=256),
}


def config_problem(name: str, energy_index=None, seed: int = 0, eta: float = 1e-3) -> BTProblem:
    """A named workload with the uniform energy grid linspace(-2, 2, n_e).
    `energy_index` selects a subset of the grid (the device is the same);
    `eta` is the broadening of every block (1e-3 in the named workloads, 1e-6 in
    their ill-conditioned "hard" variants)."""
    c = CONFIGS[name]
    grid = np.linspace(-2.0, 2.0, c["n_e"])
    if energy_index is not None:
        grid = grid[np.asarray(energy_index)]
    return random_bt_problem(c["n_b"], c["b"], grid, seed=seed, eta=eta)


# --------------------------------------------------------------------------
# Closed-form systems (inputs only; the expected values live in the tests)
# --------------------------------------------------------------------------

def chain_lead_lambda(E: float, eps0: float, t: float) -> complex:
    """Root of t*lam^2 - (E-eps0)*lam + t = 0 that is the retarded (E + i0) one:
    |lam| < 1 outside the band; inside the band |lam| = 1 with t*Im(lam) < 0."""
    z = complex(E - eps0, 1e-300)
    disc = np.sqrt(z * z - 4.0 * t * t + 0j)
    r1 = (z + disc) / (2.0 * t)
    r2 = (z - disc) / (2.0 * t)
    if abs(abs(r1) - 1.0) < 1e-12 and abs(abs(r2) - 1.0) < 1e-12:
        return r1 if t * r1.imag < 0 else r2
    return r1 if abs(r1) < abs(r2) else r2


def uniform_chain(n_b: int, b: int, energies, eps0: float = 0.0, t: float = -1.0,
                  mu_L: float = 0.1, mu_R: float = -0.1, kT: float = 0.025) -> BTProblem:
    """Uniform 1D tight-binding chain of N = n_b*b sites, on-site eps0, hopping t,
    cut into n_b blocks of b sites, with exact semi-infinite leads attached to
    site 1 and site N: Sigma^R = t*lam(E) on those sites, and no eta."""
    energies = np.atleast_1d(np.asarray(energies, dtype=np.float64))
    n_e = energies.size
    H_d = np.zeros((n_b, b, b), dtype=np.complex128)
    for i in range(n_b):
        H_d[i] = eps0 * np.eye(b)
        for j in range(b - 1):
            H_d[i, j, j + 1] = t
            H_d[i, j + 1, j] = t
    H_u = np.zeros((max(n_b - 1, 0), b, b), dtype=np.complex128)
    H_u[:, b - 1, 0] = t
    H_l = np.ascontiguousarray(np.transpose(H_u, (0, 2, 1)))
    SR_d = np.zeros((n_e, n_b, b, b), dtype=np.complex128)
    SL_d = np.zeros((n_e, n_b, b, b), dtype=np.complex128)
    fL = fermi(energies, mu_L, kT)
    fR = fermi(energies, mu_R, kT)
    gL = np.zeros((b, b), dtype=np.complex128)
    gR = np.zeros((b, b), dtype=np.complex128)
    for e, E in enumerate(energies):
        sig = t * chain_lead_lambda(E, eps0, t)
        gam = -2.0 * sig.imag
        SR_d[e, 0, 0, 0] += sig
        SR_d[e, n_b - 1, b - 1, b - 1] += sig
        SL_d[e, 0, 0, 0] += 1j * fL[e] * gam
        SL_d[e, n_b - 1, b - 1, b - 1] += 1j * fR[e] * gam
    prob = BTProblem(energies=energies, H_d=H_d, H_u=H_u, H_l=H_l, SR_d=SR_d, SL_d=SL_d,
                     gamma_L=gL, gamma_R=gR, f_L=fL, f_R=fR)
    return prob


def chain_gamma(E: float, eps0: float, t: float) -> float:
    """Lead broadening Gamma = -2 Im(t*lam) of the chain's exact lead (input helper)."""
    return -2.0 * (t * chain_lead_lambda(E, eps0, t)).imag


def uniform_strip(n_b: int, b: int, energies, eps0: float = 0.0, t_x: float = -1.0,
                  t_y: float = -1.0) -> BTProblem:
    """Uniform quasi-1D strip: b transverse sites per slice (open boundaries),
    transverse hopping t_y inside a block, longitudinal hopping t_x*I between
    blocks; exact semi-infinite leads in the transverse-mode basis on the
    first and last block.  Sigma^< = 0 (only the retarded part is of interest)."""
    energies = np.atleast_1d(np.asarray(energies, dtype=np.float64))
    n_e = energies.size
    y = np.arange(1, b + 1)
    m = np.arange(1, b + 1)
    phi = math.sqrt(2.0 / (b + 1)) * np.sin(np.pi * np.outer(y, m) / (b + 1))   # [y][m]
    eps_m = eps0 + 2.0 * t_y * np.cos(np.pi * m / (b + 1))
    Hb = eps0 * np.eye(b) + t_y * (np.eye(b, k=1) + np.eye(b, k=-1))
    H_d = np.broadcast_to(Hb.astype(np.complex128), (n_b, b, b)).copy()
    H_u = np.broadcast_to((t_x * np.eye(b)).astype(np.complex128), (max(n_b - 1, 0), b, b)).copy()
    H_l = H_u.copy()
    SR_d = np.zeros((n_e, n_b, b, b), dtype=np.complex128)
    gL = np.zeros((n_e, b, b), dtype=np.complex128)
    for e, E in enumerate(energies):
        lam = np.array([chain_lead_lambda(E, em, t_x) for em in eps_m])
        sig = phi @ np.diag(t_x * lam) @ phi.T
        SR_d[e, 0] += sig
        SR_d[e, n_b - 1] += sig
        gL[e] = 1j * (sig - sig.conj().T)
    SL_d = np.zeros_like(SR_d)
    prob = BTProblem(energies=energies, H_d=H_d, H_u=H_u, H_l=H_l, SR_d=SR_d, SL_d=SL_d)
    prob.gamma_L = gL          # per-energy contact broadening [n_e][b][b]
    prob.gamma_R = gL.copy()
    return prob


def bt_from_dense(M: np.ndarray, n_b: int):
    """Split a dense N x N matrix into BT blocks (diag, upper, lower); helper for tests."""
    N = M.shape[0]
    b = N // n_b
    d = np.stack([M[i * b:(i + 1) * b, i * b:(i + 1) * b] for i in range(n_b)])
    u = np.stack([M[i * b:(i + 1) * b, (i + 1) * b:(i + 2) * b] for i in range(n_b - 1)]) if n_b > 1 \
        else np.zeros((0, b, b), M.dtype)
    lo = np.stack([M[(i + 1) * b:(i + 2) * b, i * b:(i + 1) * b] for i in range(n_b - 1)]) if n_b > 1 \
        else np.zeros((0, b, b), M.dtype)
    return np.ascontiguousarray(d), np.ascontiguousarray(u), np.ascontiguousarray(lo)


# --------------------------------------------------------------------------
# Device-side construction of large synthetic workloads
# --------------------------------------------------------------------------

def random_bt_scalars(n_b: int, energies, eta: float = 1e-3, gamma: float = 0.5, mu_L: float = 0.1,
                      mu_R: float = -0.1, kT: float = 0.025):
    """Per-(energy, block) scalars of the synthetic device's self-energies:
    Sigma^R_ii = sr[e, i] * I and Sigma^<_ii = sl[e, i] * I (same recipe as
    random_bt_problem, so host and device inputs are bitwise identical)."""
    energies = np.atleast_1d(np.asarray(energies, dtype=np.float64))
    gam = np.zeros(n_b)
    gam[0] += gamma
    gam[-1] += gamma
    broad = eta + gam
    mu = np.linspace(mu_L, mu_R, n_b)
    f = fermi(energies[:, None], mu[None, :], kT)
    sr = np.broadcast_to(-1j * broad[None, :], (energies.size, n_b)).astype(np.complex128)
    sl = (2j * f * broad[None, :]).astype(np.complex128)
    return sr, sl


def diag_blocks_device(scal: np.ndarray, b: int, device="cuda"):
    """[n_e][n_b] complex scalars -> device tensor [n_e][n_b][b][b] of scal*I."""
    import torch
    n_e, n_b = scal.shape
    out = torch.zeros((n_e, n_b, b, b), dtype=torch.complex128, device=device)
    s = torch.from_numpy(np.ascontiguousarray(scal)).to(device)
    idx = torch.arange(b, device=device)
    out[:, :, idx, idx] = s[:, :, None].expand(n_e, n_b, b)
    return out


def device_random_problem(n_b: int, b: int, energies, seed: int = 0, device="cuda", **kw):
    """The synthetic device of random_bt_problem with its per-energy
    self-energies built directly in device memory (no host copy of the
    [n_e][n_b][b][b] arrays).  Returns a dict of device tensors plus the host
    energies; values are bitwise equal to random_bt_problem's."""
    import torch
    energies = np.atleast_1d(np.asarray(energies, dtype=np.float64))
    H_d, H_u, H_l = random_hamiltonian(n_b, b, seed)
    sr, sl = random_bt_scalars(n_b, energies, **kw)

    def dev(a):
        return torch.from_numpy(np.ascontiguousarray(a)).to(device)
    return dict(energies=energies, H_d=dev(H_d), H_u=dev(H_u), H_l=dev(H_l),
                SR_d=diag_blocks_device(sr, b, device), SL_d=diag_blocks_device(sl, b, device))


# --------------------------------------------------------------------------
# Screened Coulomb (W) system inputs (the W row of Table I)
# --------------------------------------------------------------------------

@dataclasses.dataclass
class WProblem:
    """Inputs of M = I - V P^R(E), B^<> = V P^<>(E) V^H (Table I, W row).
    V_d [n_b][b][b], V_u [n_b-1][b][b] (Hermitian BT Coulomb matrix, V_l = V_u^H);
    PR_d/u/l, PL_d/u/l, PG_d/u/l: [n_e][n_b or n_b-1][b][b] polarizations (BT)."""
    energies: np.ndarray
    V_d: np.ndarray
    V_u: np.ndarray
    PR_d: np.ndarray
    PR_u: np.ndarray
    PR_l: np.ndarray
    PL_d: np.ndarray
    PL_u: np.ndarray
    PL_l: np.ndarray
    PG_d: Optional[np.ndarray] = None
    PG_u: Optional[np.ndarray] = None
    PG_l: Optional[np.ndarray] = None

    @property
    def n_b(self) -> int:
        return int(self.V_d.shape[0])

    @property
    def b(self) -> int:
        return int(self.V_d.shape[1])

    @property
    def n_e(self) -> int:
        return int(self.energies.shape[0])


def w_base_matrices(n_b: int, b: int, seed: int, v_coupling: float = 0.3, c_k: float = 0.5):
    """Energy-independent parts of the synthetic W system, from PCG64([seed, 2]):
    V_ii = I + (X + X^H) / (4 sqrt(2b)) (Hermitian), V_{i,i+1} = v_coupling Y / sqrt(2b)
    (Y circular complex normal with E|y|^2 = 2, so E|v|^2 = v_coupling^2 / b);
    P0: a general complex BT matrix with entries of variance 1/b (blocks d, u, l);
    K: the Hermitian positive semidefinite BT matrix of diagonal blocks 2 c_k I and
    upper blocks c_k Z / |Z|_F.  Draw order: X_i, Y_i, P0 d, u, l, Z_i (R then J each)."""
    rng = np.random.default_rng([seed, 2])

    def cn(*shape):
        return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    nu = max(n_b - 1, 0)
    V_d = np.empty((n_b, b, b), np.complex128)
    for i in range(n_b):
        X = cn(b, b)
        V_d[i] = np.eye(b) + (X + X.conj().T) / (4.0 * math.sqrt(2.0 * b))
    V_u = np.empty((nu, b, b), np.complex128)
    for i in range(nu):
        V_u[i] = v_coupling * cn(b, b) / math.sqrt(2.0 * b)
    P0_d = cn(n_b, b, b) / math.sqrt(2.0 * b)
    P0_u = cn(nu, b, b) / math.sqrt(2.0 * b)
    P0_l = cn(nu, b, b) / math.sqrt(2.0 * b)
    K_d = np.broadcast_to(2.0 * c_k * np.eye(b), (n_b, b, b)).astype(np.complex128)
    K_u = np.empty((nu, b, b), np.complex128)
    for i in range(nu):
        Z = cn(b, b)
        K_u[i] = c_k * Z / np.linalg.norm(Z)
    return V_d, V_u, (P0_d, P0_u, P0_l), (K_d, K_u)


def w_scalars(energies, p_scale: float = 0.3, g_scale: float = 0.2, mu: float = 0.0, kT: float = 0.1):
    """Per-energy scalars of the polarization: P^R(E) = a(E) P0 - i g(E) K with
    a(E) = p_scale e^{iE} / (1 + E^2), g(E) = g_scale / (1 + E^2); occupation f(E)
    (Fermi function at mu, temperature kT) for P^< = -f (P^R - P^A)."""
    E = np.atleast_1d(np.asarray(energies, dtype=np.float64))
    a = p_scale * np.exp(1j * E) / (1.0 + E * E)
    g = g_scale / (1.0 + E * E)
    return a, g, fermi(E, mu, kT)


def random_w_problem(n_b: int, b: int, energies, seed: int = 0, with_greater: bool = False, **kw) -> WProblem:
    """Synthetic W system on the host (w_base_matrices, w_scalars):
    P^R = a P0 - i g K;  P^< = -f (P^R - P^A);  P^> = P^< + P^R - P^A.
    With ||V P^R|| well below 1, M = I - V P^R is well conditioned, as the W
    systems are (Section IV-A)."""
    E = np.atleast_1d(np.asarray(energies, dtype=np.float64))
    V_d, V_u, (P0_d, P0_u, P0_l), (K_d, K_u) = w_base_matrices(n_b, b, seed)
    a, g, f = w_scalars(E, **kw)
    K_l = np.conj(np.transpose(K_u, (0, 2, 1)))
    A = a[:, None, None, None]
    Gm = g[:, None, None, None]
    PR_d = A * P0_d[None] - 1j * Gm * K_d[None]
    PR_u = A * P0_u[None] - 1j * Gm * K_u[None]
    PR_l = A * P0_l[None] - 1j * Gm * K_l[None]
    H = lambda X: np.conj(np.swapaxes(X, -1, -2))
    D_d = PR_d - H(PR_d)                 # (P^R - P^A) blocks
    D_u = PR_u - H(PR_l)
    D_l = PR_l - H(PR_u)
    F = f[:, None, None, None]
    w = WProblem(energies=E, V_d=V_d, V_u=V_u, PR_d=PR_d, PR_u=PR_u, PR_l=PR_l,
                 PL_d=-F * D_d, PL_u=-F * D_u, PL_l=-F * D_l)
    if with_greater:
        w.PG_d, w.PG_u, w.PG_l = (1.0 - F) * D_d, (1.0 - F) * D_u, (1.0 - F) * D_l
    return w
