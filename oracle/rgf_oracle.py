"""Plain FP64 oracle of the selected quadratic solve  M X^<> M^H = B^<>.

TEST INFRASTRUCTURE ONLY (see the package docstring): not used by the product.

Problem statement (paper, Section II-A, Eq. 2 and the G row of Table I):
  M(E) = E*S - H - Sigma^R(E)          (block tridiagonal, n_b blocks of size b)
  G^R  = M^-1,   G^< = G^R Sigma^< G^R^H,   G^> = G^R Sigma^> G^R^H
and only the entries on the BT pattern are wanted, independently per energy.

Block notation (0-based i):  A_i = M_ii,  U_i = M_{i,i+1},  L_i = M_{i+1,i};
B_i = B_ii,  BU_i = B_{i,i+1},  BL_i = B_{i+1,i}.

Outputs, per energy: GR_d[i] = G^R_ii, GR_u[i] = G^R_{i,i+1}, GR_l[i] = G^R_{i+1,i},
GL_d[i] = G^<_ii, GL_u[i] = G^<_{i,i+1} (the lower block is -GL_u^H, Section II-A),
and GG_d / GG_u for G^> when Sigma^> is given.
"""
from __future__ import annotations

import numpy as np

OUTPUT_KEYS = ("GR_d", "GR_u", "GR_l", "GL_d", "GL_u", "GG_d", "GG_u")


def _blk(arr, e, i):
    """Block i of a per-energy block array ([n_e][k][b][b]) or None."""
    if arr is None:
        return None
    return arr[e, i]


def _system_blocks(p, e):
    """The BT blocks of M(E_e) = E S - H - Sigma^R(E_e): (A[n_b], U[n_b-1], L[n_b-1]).
    Eq. 2 / Table I (G row)."""
    E = float(p.energies[e])
    n_b, b = p.n_b, p.b
    eye = np.eye(b, dtype=np.complex128)
    A, U, L = [], [], []
    for i in range(n_b):
        S = eye if p.S_d is None else p.S_d[i]
        A.append(E * S - p.H_d[i] - p.SR_d[e, i])
    for i in range(n_b - 1):
        Su = np.zeros((b, b), np.complex128) if p.S_d is None else p.S_u[i]
        Sl = np.zeros((b, b), np.complex128) if p.S_d is None else p.S_l[i]
        u = E * Su - p.H_u[i]
        lo = E * Sl - p.H_l[i]
        if p.SR_u is not None:
            u = u - p.SR_u[e, i]
        if p.SR_l is not None:
            lo = lo - p.SR_l[e, i]
        U.append(u)
        L.append(lo)
    return A, U, L


def _rhs_blocks(p, e, which):
    """BT blocks of B = Sigma^< (which='L') or Sigma^> (which='G'): (B[n_b], BU, BL);
    BU/BL are None when the self-energy is block diagonal."""
    d = getattr(p, "S%s_d" % which)
    u = getattr(p, "S%s_u" % which)
    lo = getattr(p, "S%s_l" % which)
    B = [d[e, i] for i in range(p.n_b)]
    BU = None if u is None else [u[e, i] for i in range(p.n_b - 1)]
    BL = None if lo is None else [lo[e, i] for i in range(p.n_b - 1)]
    return B, BU, BL


def _dense_from_blocks(D, U, L):
    n_b = len(D)
    b = D[0].shape[0]
    N = n_b * b
    M = np.zeros((N, N), dtype=np.complex128)
    for i in range(n_b):
        M[i * b:(i + 1) * b, i * b:(i + 1) * b] = D[i]
    for i in range(n_b - 1):
        if U is not None:
            M[i * b:(i + 1) * b, (i + 1) * b:(i + 2) * b] = U[i]
        if L is not None:
            M[(i + 1) * b:(i + 2) * b, i * b:(i + 1) * b] = L[i]
    return M


def assemble_dense(p, e):
    """Dense N x N matrices (M, Sigma^<, Sigma^> or None) at energy index e."""
    A, U, L = _system_blocks(p, e)
    M = _dense_from_blocks(A, U, L)
    B, BU, BL = _rhs_blocks(p, e, "L")
    Bl = _dense_from_blocks(B, BU, BL)
    Bg = None
    if p.SG_d is not None:
        B, BU, BL = _rhs_blocks(p, e, "G")
        Bg = _dense_from_blocks(B, BU, BL)
    return M, Bl, Bg


def _alloc_outputs(p, n_e, greater):
    n_b, b = p.n_b, p.b
    out = {
        "GR_d": np.zeros((n_e, n_b, b, b), np.complex128),
        "GR_u": np.zeros((n_e, n_b - 1, b, b), np.complex128),
        "GR_l": np.zeros((n_e, n_b - 1, b, b), np.complex128),
        "GL_d": np.zeros((n_e, n_b, b, b), np.complex128),
        "GL_u": np.zeros((n_e, n_b - 1, b, b), np.complex128),
    }
    if greater:
        out["GG_d"] = np.zeros((n_e, n_b, b, b), np.complex128)
        out["GG_u"] = np.zeros((n_e, n_b - 1, b, b), np.complex128)
    return out


def dense_selected(p, energy_index=None):
    """The plain definition: G^R = inv(M) (LAPACK, partial pivoting),
    G^<> = G^R B^<> G^R^H, then the BT blocks are sliced out.
    Feasible for N = n_b*b up to a few thousand."""
    idx = range(p.n_e) if energy_index is None else list(energy_index)
    idx = list(idx)
    greater = p.SG_d is not None
    out = _alloc_outputs(p, len(idx), greater)
    b, n_b = p.b, p.n_b
    for k, e in enumerate(idx):
        M, Bl, Bg = assemble_dense(p, e)
        G = np.linalg.inv(M)
        Gl = G @ Bl @ G.conj().T
        Gg = G @ Bg @ G.conj().T if greater else None
        for i in range(n_b):
            s = slice(i * b, (i + 1) * b)
            out["GR_d"][k, i] = G[s, s]
            out["GL_d"][k, i] = Gl[s, s]
            if greater:
                out["GG_d"][k, i] = Gg[s, s]
        for i in range(n_b - 1):
            s = slice(i * b, (i + 1) * b)
            t = slice((i + 1) * b, (i + 2) * b)
            out["GR_u"][k, i] = G[s, t]
            out["GR_l"][k, i] = G[t, s]
            out["GL_u"][k, i] = Gl[s, t]
            if greater:
                out["GG_u"][k, i] = Gg[s, t]
    return out


def _H(X):
    return X.conj().T


def _rgf_one(A, U, L, rhs_list):
    """Block recurrences for one energy.

    Forward (left-connected functions of the leading block submatrix, i.e.
    block Gaussian elimination of Section IV-A):
      x_0 = A_0^-1 ;   x_i = (A_i - L_{i-1} x_{i-1} U_{i-1})^-1
      xl_0 = x_0 B_0 x_0^H
      xl_i = x_i Q_i x_i^H,  Q_i = B_i + L_{i-1} xl_{i-1} L_{i-1}^H
                                     - BL_{i-1} x_{i-1}^H L_{i-1}^H - L_{i-1} x_{i-1} BU_{i-1}
    Backward (i = n-2 ... 0), starting from G_{n-1,n-1} = x_{n-1}, G^<_{n-1,n-1} = xl_{n-1}:
      G_{i,i+1} = -x_i U_i G_{i+1,i+1}
      G_{i+1,i} = -G_{i+1,i+1} L_i x_i
      G_ii      =  x_i - G_{i,i+1} L_i x_i
      G^<_ii    =  xl_i + x_i U_i G^<_{i+1,i+1} U_i^H x_i^H
                   - G_{i,i+1} L_i xl_i - xl_i L_i^H G_{i,i+1}^H
                   + G_{i,i+1} BL_i x_i^H + x_i BU_i G_{i,i+1}^H
      G^<_{i,i+1} = -x_i U_i G^<_{i+1,i+1} - xl_i L_i^H G_{i+1,i+1}^H + x_i BU_i G_{i+1,i+1}^H
    Every term is evaluated as written (no symmetry shortcut).  Each explicit
    inverse is LAPACK's (LU with partial pivoting).
    rhs_list: list of (B, BU, BL) right-hand sides (Sigma^<, optionally Sigma^>).
    Returns (GRd, GRu, GRl, [(GXd, GXu) per rhs]).
    """
    n = len(A)
    inv = np.linalg.inv
    x = [None] * n
    x[0] = inv(A[0])
    for i in range(1, n):
        x[i] = inv(A[i] - L[i - 1] @ x[i - 1] @ U[i - 1])
    xls = []
    for (B, BU, BL) in rhs_list:
        xl = [None] * n
        xl[0] = x[0] @ B[0] @ _H(x[0])
        for i in range(1, n):
            Q = B[i] + L[i - 1] @ xl[i - 1] @ _H(L[i - 1])
            if BL is not None:
                Q = Q - BL[i - 1] @ _H(x[i - 1]) @ _H(L[i - 1])
            if BU is not None:
                Q = Q - L[i - 1] @ x[i - 1] @ BU[i - 1]
            xl[i] = x[i] @ Q @ _H(x[i])
        xls.append(xl)

    GRd = [None] * n
    GRu = [None] * (n - 1)
    GRl = [None] * (n - 1)
    GRd[n - 1] = x[n - 1]
    for i in range(n - 2, -1, -1):
        GRu[i] = -x[i] @ U[i] @ GRd[i + 1]
        GRl[i] = -GRd[i + 1] @ L[i] @ x[i]
        GRd[i] = x[i] - GRu[i] @ L[i] @ x[i]
    outs = []
    for (B, BU, BL), xl in zip(rhs_list, xls):
        Gd = [None] * n
        Gu = [None] * (n - 1)
        Gd[n - 1] = xl[n - 1]
        for i in range(n - 2, -1, -1):
            Gd[i] = (xl[i]
                     + x[i] @ U[i] @ Gd[i + 1] @ _H(U[i]) @ _H(x[i])
                     - GRu[i] @ L[i] @ xl[i]
                     - xl[i] @ _H(L[i]) @ _H(GRu[i]))
            Gu[i] = -x[i] @ U[i] @ Gd[i + 1] - xl[i] @ _H(L[i]) @ _H(GRd[i + 1])
            if BL is not None:
                Gd[i] = Gd[i] + GRu[i] @ BL[i] @ _H(x[i])
            if BU is not None:
                Gd[i] = Gd[i] + x[i] @ BU[i] @ _H(GRu[i])
                Gu[i] = Gu[i] + x[i] @ BU[i] @ _H(GRd[i + 1])
        outs.append((Gd, Gu))
    return GRd, GRu, GRl, outs


def schur_complements(p, e):
    """The forward Schur complements of M(E_e) in block order (block Gaussian
    elimination, Section IV-A): S_0 = A_0, S_i = A_i - L_{i-1} S_{i-1}^-1 U_{i-1}.
    S_i is the Schur complement of the leading i-block submatrix in the leading
    (i+1)-block submatrix, so S_i^-1 is the last diagonal block of that
    submatrix's inverse; these are the matrices the recurrences invert, and their
    condition numbers (not only that of M) set the rounding error of the method."""
    A, U, L = _system_blocks(p, e)
    S = [A[0]]
    for i in range(1, len(A)):
        S.append(A[i] - L[i - 1] @ np.linalg.inv(S[i - 1]) @ U[i - 1])
    return S


def rgf_selected(p, energy_index=None):
    """Selected blocks by the block recurrences (see _rgf_one), per energy."""
    idx = list(range(p.n_e) if energy_index is None else energy_index)
    greater = p.SG_d is not None
    out = _alloc_outputs(p, len(idx), greater)
    n_b = p.n_b
    for k, e in enumerate(idx):
        A, U, L = _system_blocks(p, e)
        rhs = [_rhs_blocks(p, e, "L")]
        if greater:
            rhs.append(_rhs_blocks(p, e, "G"))
        GRd, GRu, GRl, outs = _rgf_one(A, U, L, rhs)
        for i in range(n_b):
            out["GR_d"][k, i] = GRd[i]
            out["GL_d"][k, i] = outs[0][0][i]
            if greater:
                out["GG_d"][k, i] = outs[1][0][i]
        for i in range(n_b - 1):
            out["GR_u"][k, i] = GRu[i]
            out["GR_l"][k, i] = GRl[i]
            out["GL_u"][k, i] = outs[0][1][i]
            if greater:
                out["GG_u"][k, i] = outs[1][1][i]
    return out
