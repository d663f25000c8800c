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
