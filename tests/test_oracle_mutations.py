"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake (a dropped term, a flipped sign, a wrong index,
a missing conjugate, a transposed operand) into a private copy of the oracle's
source, on the CPU, and checks that the exact brute-force / closed-form pins
reject the mutated oracle while accepting the real one.
"""
import inspect
import types

import numpy as np
import pytest

from oracle import rgf_oracle
from paper_2606_25595_amd import inputs
from tests.exact_rational import qinv, qmat, qmul, qH, to_complex
from tests.test_oracle_pins import gaussian_int_problem, chain_closed_form

SRC = inspect.getsource(rgf_oracle)

MUTATIONS = [
    ("drop_BL_forward", "Q = Q - BL[i - 1] @ _H(x[i - 1]) @ _H(L[i - 1])", "Q = Q"),
    ("drop_BU_forward", "Q = Q - L[i - 1] @ x[i - 1] @ BU[i - 1]", "Q = Q"),
    ("sign_GRu", "GRu[i] = -x[i] @ U[i] @ GRd[i + 1]", "GRu[i] = x[i] @ U[i] @ GRd[i + 1]"),
    ("swap_UL_GRl", "GRl[i] = -GRd[i + 1] @ L[i] @ x[i]", "GRl[i] = -GRd[i + 1] @ U[i] @ x[i]"),
    ("drop_term4_GLd", "- xl[i] @ _H(L[i]) @ _H(GRu[i]))", ")"),
    ("no_conj_H", "return X.conj().T", "return X.T"),
    ("index_forward_U", "x[i] = inv(A[i] - L[i - 1] @ x[i - 1] @ U[i - 1])",
     "x[i] = inv(A[i] - L[i - 1] @ x[i - 1] @ U[i - 1].T)"),
    ("drop_energy", "A.append(E * S - p.H_d[i] - p.SR_d[e, i])", "A.append(S - p.H_d[i] - p.SR_d[e, i])"),
    ("sign_BU_backward_upper", "Gu[i] = Gu[i] + x[i] @ BU[i] @ _H(GRd[i + 1])",
     "Gu[i] = Gu[i] - x[i] @ BU[i] @ _H(GRd[i + 1])"),
    ("no_conj_GLu", "- xl[i] @ _H(L[i]) @ _H(GRd[i + 1])", "- xl[i] @ _H(L[i]) @ GRd[i + 1]"),
    ("transpose_dense_lesser", "Gl = G @ Bl @ G.conj().T", "Gl = G @ Bl @ G.T"),
    ("dense_upper_lower_swap", 'out["GR_u"][k, i] = G[s, t]', 'out["GR_u"][k, i] = G[t, s]'),
    ("lesser_backward_PGP", "+ x[i] @ U[i] @ Gd[i + 1] @ _H(U[i]) @ _H(x[i])",
     "+ x[i] @ U[i] @ Gd[i + 1] @ _H(x[i])"),
]


def load(src):
    mod = types.ModuleType("mutated_oracle")
    exec(compile(src, "mutated_oracle", "exec"), mod.__dict__)
    return mod


def pins_pass(mod):
    """Exact brute force (BT Sigma, general S, greater) and the chain closed form."""
    for (n_b, b, seed) in [(3, 2, 2), (2, 2, 1)]:
        p = gaussian_int_problem(n_b, b, seed)
        M, Bl, Bg = rgf_oracle.assemble_dense(p, 0)
        G = qinv(qmat(M))
        GH = qH(G)
        refs = {"GR": to_complex(G), "GL": to_complex(qmul(qmul(G, qmat(Bl)), GH)),
                "GG": to_complex(qmul(qmul(G, qmat(Bg)), GH))}
        for solver in (mod.dense_selected, mod.rgf_selected):
            out = solver(p)
            for pre in ("GR", "GL", "GG"):
                d, u, lo = inputs.bt_from_dense(refs[pre], n_b)
                pairs = [(out[pre + "_d"][0], d), (out[pre + "_u"][0], u)]
                if pre == "GR":
                    pairs.append((out["GR_l"][0], lo))
                for got, ref in pairs:
                    if np.linalg.norm(got - ref) > 1e-11 * np.linalg.norm(ref):
                        return False
    E = np.array([-1.1, 0.3, 1.6])
    p = inputs.uniform_chain(3, 2, E)
    for solver in (mod.dense_selected, mod.rgf_selected):
        out = solver(p)
        for k, En in enumerate(E):
            G, Gl, _ = chain_closed_form(6, En, -1.0, p.f_L[k], p.f_R[k])
            d, u, lo = inputs.bt_from_dense(G, 3)
            if np.linalg.norm(out["GR_d"][k] - d) > 1e-11 * np.linalg.norm(d):
                return False
            d, u, lo = inputs.bt_from_dense(Gl, 3)
            if np.linalg.norm(out["GL_u"][k] - u) > 1e-10 * np.linalg.norm(u):
                return False
    return True


def test_unmutated_oracle_passes():
    assert pins_pass(load(SRC))


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_mutation_is_caught(name, old, new):
    assert old in SRC, "mutation target vanished from the oracle: %s" % name
    mutated = SRC.replace(old, new)
    assert mutated != SRC
    try:
        ok = pins_pass(load(mutated))
    except Exception:
        ok = False          # a crash also counts as caught
    assert not ok, "pins did not catch mutation %s" % name
