"""The seeded input generator: structure and reproducibility of the synthetic device."""
import numpy as np

from paper_2606_25595_amd import inputs


def test_hamiltonian_hermitian_and_variances():
    H_d, H_u, H_l = inputs.random_hamiltonian(6, 64, seed=0)
    for i in range(6):
        assert np.array_equal(H_d[i], H_d[i].conj().T)
    assert np.array_equal(H_l, np.conj(np.transpose(H_u, (0, 2, 1))))
    b = 64
    off = H_d[:, ~np.eye(b, dtype=bool)]
    assert abs(np.mean(np.abs(off) ** 2) * b - 1.0) < 0.05
    assert abs(np.var(np.real(np.diagonal(H_d, axis1=1, axis2=2))) * b - 1.0) < 0.2
    assert abs(np.mean(np.abs(H_u) ** 2) * b - 0.5) < 0.03


def test_reproducible_and_energy_subset_consistent():
    a = inputs.config_problem("tiny")
    b = inputs.config_problem("tiny", energy_index=[3, 17])
    assert np.array_equal(a.H_d, b.H_d) and np.array_equal(a.H_u, b.H_u)
    assert np.array_equal(a.SR_d[[3, 17]], b.SR_d)
    assert np.array_equal(a.SL_d[[3, 17]], b.SL_d)
    c = inputs.config_problem("tiny", seed=1)
    assert not np.array_equal(a.H_d, c.H_d)


def test_self_energies_structure():
    p = inputs.random_bt_problem(5, 8, np.linspace(-2, 2, 6), seed=2, with_greater=True)
    for e in range(p.n_e):
        for i in range(p.n_b):
            SR, SL, SG = p.SR_d[e, i], p.SL_d[e, i], p.SG_d[e, i]
            assert np.array_equal(SL, -SL.conj().T)          # lesser is skew-Hermitian
            assert np.array_equal(SG, -SG.conj().T)
            assert np.allclose(SG - SL, SR - SR.conj().T)     # Sigma^> - Sigma^< = Sigma^R - Sigma^A
            assert np.all(np.imag(np.diagonal(SR)) < 0)      # retarded: negative imaginary part
    assert np.all((p.f_L >= 0) & (p.f_L <= 1))


def test_fermi_limits():
    assert inputs.fermi(-100.0, 0.0, 0.025) == 1.0
    assert inputs.fermi(100.0, 0.0, 0.025) < 1e-300 or inputs.fermi(100.0, 0.0, 0.025) == 0.0
    assert abs(inputs.fermi(0.1, 0.1, 0.025) - 0.5) < 1e-15


def test_bt_self_energies_skew_hermitian_and_dissipative():
    """bt_sigma: Sigma^< is skew-Hermitian with -i Sigma^< >= 0, Sigma^> = Sigma^< +
    Sigma^R - Sigma^A, and the anti-Hermitian part of Sigma^R is <= -eta (so that
    M keeps sigma_min >= eta), all checked on the assembled dense matrices."""
    import numpy as np
    from paper_2606_25595_amd import inputs

    def dense(D, U, L):
        n, b = D.shape[0], D.shape[1]
        M = np.zeros((n * b, n * b), complex)
        for i in range(n):
            M[i * b:(i + 1) * b, i * b:(i + 1) * b] = D[i]
        for i in range(n - 1):
            M[i * b:(i + 1) * b, (i + 1) * b:(i + 2) * b] = U[i]
            M[(i + 1) * b:(i + 2) * b, i * b:(i + 1) * b] = L[i]
        return M

    eta = 1e-3
    p = inputs.random_bt_problem(4, 5, np.array([-0.3, 0.05, 0.6]), seed=2, eta=eta, with_greater=True,
                                 bt_sigma=0.2)
    for e in range(p.n_e):
        SL = dense(p.SL_d[e], p.SL_u[e], p.SL_l[e])
        SR = dense(p.SR_d[e], p.SR_u[e], p.SR_l[e])
        SG = dense(p.SG_d[e], p.SG_u[e], p.SG_l[e])
        assert np.allclose(SL, -SL.conj().T, atol=1e-15)
        assert np.linalg.eigvalsh(-1j * SL).min() >= -1e-14
        assert np.allclose(SG, SL + SR - SR.conj().T, atol=1e-15)
        assert np.linalg.eigvalsh(-(SR - SR.conj().T) / 2j).min() >= eta - 1e-13
