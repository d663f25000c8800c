"""Observables and error metrics computed from selected Green's-function blocks.

TEST INFRASTRUCTURE ONLY: used by the tests and the benchmark's CPU leg.

The paper's accuracy criterion is the electronic current and its conservation
along the device (Section II-B).  From the selected blocks:
  spectral function of block 1:  A_11 = i (G^R_11 - G^R_11^H)
  transmission seen from the left contact (broadening Gamma_L on block 1):
      T_L = Tr[Gamma_L A_11] - Tr[Gamma_L G^R_11 Gamma_L G^R_11^H]
    (since A = G^R Gamma_tot G^A, this is the Caroli transmission when the only
     other broadening is Gamma_R on the last block)
  particle current entering from the left contact:
      j_L = Re( i Tr[Gamma_L G^<_11] ) + f_L Tr[Gamma_L A_11]
  bond current between blocks i and i+1 (coupling of M is -(H - E S)_{i,i+1}):
      J_i = 2 Re Tr[ (H - E S)_{i,i+1} G^<_{i+1,i} ],  G^<_{i+1,i} = -(G^<_{i,i+1})^H
"""
from __future__ import annotations

import numpy as np


def _gam(gamma, k):
    g = np.asarray(gamma)
    return g[k] if g.ndim == 3 else g


def transmission_left(GR_11, gamma_L):
    """T_L per energy. GR_11: [n_e][b][b]; gamma_L: [b][b] or [n_e][b][b]."""
    n_e = GR_11.shape[0]
    T = np.empty(n_e)
    for k in range(n_e):
        G = GR_11[k]
        g = _gam(gamma_L, k)
        A = 1j * (G - G.conj().T)
        T[k] = (np.trace(g @ A) - np.trace(g @ G @ g @ G.conj().T)).real
    return T


def contact_current_left(GR_11, GL_11, gamma_L, f_L):
    """j_L per energy."""
    n_e = GR_11.shape[0]
    j = np.empty(n_e)
    for k in range(n_e):
        G = GR_11[k]
        g = _gam(gamma_L, k)
        A = 1j * (G - G.conj().T)
        j[k] = (1j * np.trace(g @ GL_11[k])).real + f_L[k] * np.trace(g @ A).real
    return j


def bond_currents(p, GL_u, energy_index=None):
    """J_i per energy and bond: [n_e][n_b-1]."""
    idx = list(range(p.n_e) if energy_index is None else energy_index)
    J = np.zeros((len(idx), p.n_b - 1))
    for k, e in enumerate(idx):
        E = float(p.energies[e])
        for i in range(p.n_b - 1):
            c = p.H_u[i] - (0.0 if p.S_u is None else E * p.S_u[i])
            Glo = -GL_u[k, i].conj().T
            J[k, i] = 2.0 * np.trace(c @ Glo).real
    return J


def rel_fro_err(X, Xref):
    """Relative Frobenius error per leading index (per energy and block):
    ||X - Xref||_F / ||Xref||_F, absolute where ||Xref||_F == 0."""
    X = np.asarray(X)
    Xref = np.asarray(Xref)
    ax = tuple(range(X.ndim - 2, X.ndim))
    num = np.sqrt(np.sum(np.abs(X - Xref) ** 2, axis=ax))
    den = np.sqrt(np.sum(np.abs(Xref) ** 2, axis=ax))
    return np.where(den > 0, num / np.where(den > 0, den, 1.0), num)
