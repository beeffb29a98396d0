"""Pins for stage matrices in low-rank form and the partial eigensolve (Sec. 3.7)."""
import numpy as np
import pytest

from oracle import rhs as OR, lowrank as OL
from oracle.hamiltonian import Hamiltonian
from oracle.metrics import rel_fro_error, dense_rho
from oracle.schemes import RK_TABLEAUX
from workloads import chain_bonds, haar_factor, dirichlet_spectrum


def _stages(n=6, r=3, seed=0, model="qLL", h=0.05):
    rng = np.random.default_rng(seed)
    bonds = chain_bonds(n, periodic=True)
    H = Hamiltonian(n, bonds, rng.normal(size=(bonds.shape[0], 3, 3)), rng.normal(size=(n, 3)))
    V = haar_factor(2 ** n, r, rng)
    lam = dirichlet_spectrum(r, rng)
    a, b = RK_TABLEAUX["RK4"]
    terms, Vj = [], V
    for j in range(4):
        out = OR.rhs(H, Vj, lam, model, 0.4)
        terms.append((Vj, out["Z"], out["W"]))
        if j < 3:
            K = OL.stage_matrix(V, lam, terms, h, a[j + 1, : j + 1])
            _, Vj = OL.partial_eig(K, r)
    return H, V, lam, terms, b


def test_lowrank_equals_dense_sum():
    """eq. (3.9): sum A_l V_l* + V_l B_l* == rho_k + h sum b_l f(K_l) (dense)."""
    H, V, lam, terms, b = _stages()
    h = 0.05
    K = OL.stage_matrix(V, lam, terms, h, b)
    Kd = dense_rho(V, lam) + h * sum(bl * OR.rhs_dense_from_factors(Vl, Zl, Wl)
                                      for bl, (Vl, Zl, Wl) in zip(b, terms))
    np.testing.assert_allclose(K.dense(), Kd, atol=1e-14)
    x = np.random.default_rng(1).normal(size=(K.N, 2)) + 0j
    np.testing.assert_allclose(K.matvec(x), Kd @ x, atol=1e-14)  # eq. (3.10)


@pytest.mark.parametrize("model", ["qLL", "qLLG"])
def test_partial_eig_matches_dense_eigh(model):
    H, V, lam, terms, b = _stages(model=model, seed=2)
    K = OL.stage_matrix(V, lam, terms, 0.05, b)
    w, U = OL.partial_eig(K, 3)
    wd, Ud = np.linalg.eigh(K.dense())
    od = np.argsort(wd)[::-1][:3]
    np.testing.assert_allclose(w, wd[od], atol=1e-14)
    assert rel_fro_error(U, lam, Ud[:, od], lam) < 1e-13
    np.testing.assert_allclose(U.conj().T @ U, np.eye(3), atol=1e-14)


def test_partial_eig_matches_irlm():
    """The exact range solve agrees with ARPACK's IRLM on the matvec g (Sec. 5 setup)."""
    H, V, lam, terms, b = _stages(n=10, r=4, seed=3)
    K = OL.stage_matrix(V, lam, terms, 0.05, b)
    w, U = OL.partial_eig(K, 4)
    w2, U2 = OL.partial_eig_irlm(K, 4)
    np.testing.assert_allclose(w, w2, atol=1e-12)
    assert rel_fro_error(U, lam, U2, lam) < 1e-10


def test_top_eigenvalues_close_to_lambda0():
    """After one step the top-r eigenvalues of K stay near Lambda_0 (O(h^2) drift)."""
    H, V, lam, terms, b = _stages(seed=4, h=0.01)
    K = OL.stage_matrix(V, lam, terms, 0.01, b)
    w, _ = OL.partial_eig(K, 3)
    assert np.abs(w - lam).max() < 1e-3
