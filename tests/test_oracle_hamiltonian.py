"""Pins for the oracle's Hamiltonian (Sec. 5 eq. 5.1 in Pauli form; eq. 3.5)."""
import os

import numpy as np
import pytest

from oracle import hamiltonian as OH
from oracle.hamiltonian import Hamiltonian, apply_H, dense_H, spin_operator
from workloads import (chain_bonds, square_lattice_bonds, haar_factor, af1_index, af2_index,
                       heisenberg_tensors, xxz_tensors, uniform_field)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _random_model(n, rng, periodic=True):
    bonds = chain_bonds(n, periodic=periodic)
    J = rng.normal(size=(bonds.shape[0], 3, 3))
    h = rng.normal(size=(n, 3))
    return bonds, J, h


@pytest.mark.parametrize("n", [2, 3, 5, 7])
def test_gather_matches_kronecker(n):
    """Matrix-free Pauli gather == dense Kronecker H (general 3x3 tensors + fields)."""
    rng = np.random.default_rng(10 + n)
    bonds, J, h = _random_model(n, rng)
    V = haar_factor(2 ** n, 3, rng)
    Hd = dense_H(n, bonds, J, h)
    np.testing.assert_allclose(apply_H(n, bonds, J, h, V), Hd @ V, atol=1e-13)


def test_hermitian():
    n = 9
    rng = np.random.default_rng(4)
    bonds, J, h = _random_model(n, rng)
    u = haar_factor(2 ** n, 2, rng)
    v = haar_factor(2 ** n, 2, rng)
    lhs = u.conj().T @ apply_H(n, bonds, J, h, v)
    rhs = apply_H(n, bonds, J, h, u).conj().T @ v
    np.testing.assert_allclose(lhs, rhs, atol=1e-12)


def test_dimer_singlet_triplet():
    """H = (J/2) s_1.s_2 has the triplet at J/2 (x3) and the singlet at -3J/2."""
    J = 1.7
    H = dense_H(2, np.array([[0, 1]]), heisenberg_tensors(1, J), None)
    w = np.sort(np.linalg.eigvalsh(H))
    np.testing.assert_allclose(w, [-1.5 * J, 0.5 * J, 0.5 * J, 0.5 * J], atol=1e-14)
    # singlet (|01> - |10>)/sqrt 2 in bit labels: indices 2 (site0 up, site1 down) and 1
    s = np.zeros(4, complex)
    s[2], s[1] = 1 / np.sqrt(2), -1 / np.sqrt(2)
    np.testing.assert_allclose(H @ s, -1.5 * J * s, atol=1e-14)


def test_eq51_spin_form():
    """Pauli form == eq. (5.1) written with S = (hbar/2) s, J, DMI d and field b."""
    n, hbar = 3, 0.7
    Jx, d, b, gmuB = 1.3, np.array([0.2, -0.1, 0.4]), np.array([0.3, 0.5, -0.2]), 0.116
    bonds = np.array([[0, 1], [1, 2]])
    S = [[spin_operator(n, i, a, hbar) for a in range(3)] for i in range(n)]
    H51 = np.zeros((8, 8), complex)
    for i, j in bonds:
        H51 += (2 * Jx / hbar ** 2) * sum(S[i][a] @ S[j][a] for a in range(3))
        cross = [S[i][1] @ S[j][2] - S[i][2] @ S[j][1], S[i][2] @ S[j][0] - S[i][0] @ S[j][2],
                 S[i][0] @ S[j][1] - S[i][1] @ S[j][0]]
        H51 += (2 / hbar ** 2) * sum(d[c] * cross[c] for c in range(3))
    mu = -gmuB / hbar
    for i in range(n):
        H51 += -mu * sum(b[a] * S[i][a] for a in range(3))
    # Pauli-form tensor: J delta_ab + eps_abc d_c ; field h = g mu_B b
    T = np.diag([Jx] * 3).astype(float)
    T[0, 1], T[1, 0] = d[2], -d[2]
    T[1, 2], T[2, 1] = d[0], -d[0]
    T[2, 0], T[0, 2] = d[1], -d[1]
    Hp = dense_H(n, bonds, np.stack([T, T]), np.tile(gmuB * b, (n, 1)))
    np.testing.assert_allclose(Hp, H51, atol=1e-13)


def test_single_site_field_eigenvalues():
    h = np.array([[0.3, -0.4, 1.2]])
    H = dense_H(1, np.zeros((0, 2), int), np.zeros((0, 3, 3)), h)
    np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(H)),
                               [-0.5 * np.linalg.norm(h), 0.5 * np.linalg.norm(h)], atol=1e-14)


def test_xxz_conserves_total_sz():
    """XXZ bonds + z fields never leave a magnetisation sector (popcount)."""
    n = 8
    rng = np.random.default_rng(2)
    bonds = square_lattice_bonds(2, 4, periodic=True)
    J = xxz_tensors(rng.uniform(0.5, 1.5, bonds.shape[0]), rng.uniform(0.5, 1.5, bonds.shape[0]))
    h = uniform_field(n, (0, 0, 0.7))
    N = 2 ** n
    pop = np.array([bin(x).count("1") for x in range(N)])
    for k in (0, 3, 4):
        V = np.zeros((N, 1), complex)
        V[pop == k, 0] = rng.normal(size=(pop == k).sum())
        Y = apply_H(n, bonds, J, h, V)
        assert np.abs(Y[pop != k]).max() == 0.0


def test_af_index_golden():
    rows = np.loadtxt(os.path.join(GOLDEN, "af_states.txt"), dtype=int)
    for n, p1, o1, p2, o2 in rows:
        assert af1_index(n) == o1 and af2_index(n) == o2
        # paper index: binary string with site 1 leftmost, 1-based
        s1 = format(o1, f"0{n}b")[::-1]
        s2 = format(o2, f"0{n}b")[::-1]
        assert int(s1, 2) + 1 == p1 and int(s2, 2) + 1 == p2


def test_planted_sy_sign_error_is_caught(monkeypatch):
    """A flipped s^y sign in the gather breaks the Kronecker pin."""
    rng = np.random.default_rng(7)
    bonds, J, h = _random_model(3, rng)
    V = haar_factor(8, 2, rng)
    good = apply_H(3, bonds, J, h, V)
    orig = OH.apply_pauli

    def bad(V, site, a):
        out = orig(V, site, a)
        return -out if a == 1 else out

    monkeypatch.setattr(OH, "apply_pauli", bad)
    assert np.abs(OH.apply_H(3, bonds, J, h, V) - good).max() > 1e-3


def test_hamiltonian_class():
    rng = np.random.default_rng(1)
    bonds, J, h = _random_model(4, rng)
    H = Hamiltonian(4, bonds, J, h)
    V = haar_factor(16, 2, rng)
    np.testing.assert_allclose(H.apply(V), H.dense() @ V, atol=1e-13)


def test_row_sampled_apply_matches_full():
    from oracle.hamiltonian import apply_H_rows
    rng = np.random.default_rng(9)
    n = 8
    bonds, J, h = _random_model(n, rng)
    V = haar_factor(2 ** n, 4, rng)
    rows = rng.choice(2 ** n, size=37, replace=False)
    np.testing.assert_allclose(apply_H_rows(n, bonds, J, h, V, rows),
                               apply_H(n, bonds, J, h, V)[rows], atol=1e-13)
