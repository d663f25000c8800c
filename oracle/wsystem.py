"""FP64 oracle of the screened Coulomb system (the W row of Table I).

TEST INFRASTRUCTURE ONLY (see the package docstring): not used by the product.

Per energy the system is Eq. 2 with
    M(E) = I - V P^R(E),      B^<>(E) = V P^<>(E) V^H,     X^<> = W^<>,
V the (Hermitian, BT) Coulomb matrix and P the polarization.  Products of BT
matrices are wider than BT (V P^R has blocks two off the diagonal, V P^< V^H
three); the system solved is the BT one the paper states (Section II-A: every
quantity is tiled into BT form and only the BT entries are wanted), so M and B
are the BT blocks of those products.  This module writes that definition out:
dense products, then the BT blocks, then the G-system oracles with E = 1, S = I,
H = 0 and Sigma^R := BT(V P^R), Sigma^<> := BT(V P^<> V^H).
"""
from __future__ import annotations

import types

import numpy as np

from .rgf_oracle import _dense_from_blocks, dense_selected, rgf_selected


def _H(X):
    return np.conj(np.swapaxes(X, -1, -2))


def _bt_blocks(M, n_b, b):
    d = np.stack([M[i * b:(i + 1) * b, i * b:(i + 1) * b] for i in range(n_b)])
    u = np.stack([M[i * b:(i + 1) * b, (i + 1) * b:(i + 2) * b] for i in range(n_b - 1)]) if n_b > 1 \
        else np.zeros((0, b, b), M.dtype)
    lo = np.stack([M[(i + 1) * b:(i + 2) * b, i * b:(i + 1) * b] for i in range(n_b - 1)]) if n_b > 1 \
        else np.zeros((0, b, b), M.dtype)
    return d, u, lo


def w_assemble(w):
    """BT blocks of V P^R(E) and of V P^<>(E) V^H for every energy of a WProblem
    (dense products of the assembled matrices).  Returns a dict of
    [n_e][...][b][b] arrays: VPR_d/u/l, BL_d/u/l, and BG_d/u/l when P^> is given."""
    n_b, b, n_e = w.n_b, w.b, w.n_e
    V = _dense_from_blocks(list(w.V_d), list(w.V_u), list(_H(w.V_u)))
    out = {k: [] for k in ("VPR_d", "VPR_u", "VPR_l", "BL_d", "BL_u", "BL_l", "BG_d", "BG_u", "BG_l")}
    VH = V.conj().T
    for e in range(n_e):
        PR = _dense_from_blocks(list(w.PR_d[e]), list(w.PR_u[e]), list(w.PR_l[e]))
        for k, X in zip(("VPR_d", "VPR_u", "VPR_l"), _bt_blocks(V @ PR, n_b, b)):
            out[k].append(X)
        PL = _dense_from_blocks(list(w.PL_d[e]), list(w.PL_u[e]), list(w.PL_l[e]))
        for k, X in zip(("BL_d", "BL_u", "BL_l"), _bt_blocks(V @ PL @ VH, n_b, b)):
            out[k].append(X)
        if w.PG_d is not None:
            PG = _dense_from_blocks(list(w.PG_d[e]), list(w.PG_u[e]), list(w.PG_l[e]))
            for k, X in zip(("BG_d", "BG_u", "BG_l"), _bt_blocks(V @ PG @ VH, n_b, b)):
                out[k].append(X)
    return {k: np.stack(v) for k, v in out.items() if v}


def w_as_g_problem(w, asm=None):
    """The W system as a G-type problem for the oracles: energies 1, S = I, H = 0,
    Sigma^R = BT(V P^R), Sigma^< = BT(V P^< V^H) (and Sigma^>)."""
    asm = w_assemble(w) if asm is None else asm
    n_b, b = w.n_b, w.b
    z = np.zeros((n_b, b, b), np.complex128)
    zu = np.zeros((max(n_b - 1, 0), b, b), np.complex128)
    p = types.SimpleNamespace(
        energies=np.ones(w.n_e), H_d=z, H_u=zu, H_l=zu, S_d=None, S_u=None, S_l=None,
        SR_d=asm["VPR_d"], SR_u=asm["VPR_u"], SR_l=asm["VPR_l"],
        SL_d=asm["BL_d"], SL_u=asm["BL_u"], SL_l=asm["BL_l"],
        SG_d=asm.get("BG_d"), SG_u=asm.get("BG_u"), SG_l=asm.get("BG_l"),
        n_b=n_b, b=b, n_e=w.n_e)
    return p


def w_selected(w, method="dense", asm=None):
    """Selected blocks of M^-1 and W^<> = M^-1 B^<> M^-H (W row of Table I)."""
    p = w_as_g_problem(w, asm)
    return dense_selected(p) if method == "dense" else rgf_selected(p)
