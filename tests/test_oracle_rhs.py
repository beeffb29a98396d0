"""Pins for the oracle's low-rank right-hand side (eqs. 3.2, 3.3, 3.4, 4.1)."""
import numpy as np
import pytest

from oracle import rhs as OR
from oracle.hamiltonian import Hamiltonian
from oracle import dense as OD
from oracle.metrics import dense_rho
from workloads import chain_bonds, haar_factor, dirichlet_spectrum


def _setup(n=5, r=3, seed=0):
    rng = np.random.default_rng(seed)
    bonds = chain_bonds(n, periodic=True)
    J = rng.normal(size=(bonds.shape[0], 3, 3))
    h = rng.normal(size=(n, 3))
    H = Hamiltonian(n, bonds, J, h)
    V = haar_factor(2 ** n, r, rng)
    lam = dirichlet_spectrum(r, rng)
    return H, V, lam


@pytest.mark.parametrize("hbar", [1.0, 0.6])
def test_qll_matches_commutators(hbar):
    """f = Z V* + V W* equals (i/hbar)[rho,H] - (kappa/hbar)[rho,[rho,H]] (eq. 1.1)."""
    H, V, lam = _setup()
    out = OR.rhs(H, V, lam, "qLL", 0.37, hbar)
    f = OR.rhs_dense_from_factors(V, out["Z"], out["W"])
    fd = OD.rhs_qll(dense_rho(V, lam), H.dense(), 0.37, hbar)
    np.testing.assert_allclose(f, fd, atol=1e-14)


@pytest.mark.parametrize("hbar", [1.0, 0.6])
def test_qllg_implicit_residual(hbar):
    """The low-rank q-LLG f solves the implicit equation (1.2)."""
    H, V, lam = _setup(seed=1)
    out = OR.rhs(H, V, lam, "qLLG", 0.8, hbar)
    f = OR.rhs_dense_from_factors(V, out["Z"], out["W"])
    res = OD.rhs_qllg_residual(dense_rho(V, lam), f, H.dense(), 0.8, hbar)
    assert np.abs(res).max() < 1e-14


def test_qllg_matches_ei_sylvester():
    """Low-rank q-LLG f == V X V* from the dense Sylvester solve (eqs. 2.3-2.6)."""
    H, V, lam = _setup(seed=2)
    N, r = V.shape
    out = OR.rhs(H, V, lam, "qLLG", 0.5)
    f = OR.rhs_dense_from_factors(V, out["Z"], out["W"])
    Vfull = np.linalg.qr(np.concatenate([V, np.random.default_rng(0).normal(size=(N, N - r))], 1))[0]
    Vfull[:, :r] = V
    lam_full = np.concatenate([lam, np.zeros(N - r)])
    fd = OD.rhs_qllg_eig(Vfull, lam_full, H.dense(), 0.5)
    np.testing.assert_allclose(f, fd, atol=1e-14)


@pytest.mark.parametrize("model", ["qLL", "qLLG"])
def test_householder_equals_projector(model):
    """Vhat X12* through Householder reflectors == (I - V V*) Y diag(conj c)."""
    H, V, lam = _setup(n=7, r=4, seed=3)
    out = OR.rhs(H, V, lam, model, 0.3)
    c = OR.phi_coeffs(lam, model, 0.3)
    Y = out["Y"]
    Wp = (Y - V @ (V.conj().T @ Y)) * c.conj()[None, :]
    np.testing.assert_allclose(out["W"], Wp, atol=1e-14)
    assert np.abs(V.conj().T @ out["W"]).max() < 1e-14


def test_householder_reduces_to_unit_diagonal():
    """P_r ... P_1 V = [R~; 0] with R~ diagonal of unit modulus (V orthonormal)."""
    _, V, _ = _setup(n=6, r=5, seed=4)
    us, betas = OR.householder_vectors(V)
    QhV = V.copy()
    for u, b in zip(us, betas):
        QhV = QhV - b * np.outer(u, u.conj() @ QhV)
    Rt = QhV[:5]
    assert np.abs(QhV[5:]).max() < 1e-14
    np.testing.assert_allclose(np.abs(np.diag(Rt)), 1.0, atol=1e-14)
    assert np.abs(Rt - np.diag(np.diag(Rt))).max() < 1e-14
    # the product of reflectors is unitary and apply_left/apply_right are adjoint-consistent
    A = np.random.default_rng(1).normal(size=(V.shape[0], 3)) + 0j
    Q_A = OR.apply_left(A, us, betas)
    np.testing.assert_allclose(np.linalg.norm(Q_A, axis=0), np.linalg.norm(A, axis=0), rtol=1e-13)


def test_planted_missing_reflector_is_caught(monkeypatch):
    """Skipping the last reflector in the left action breaks the projector pin."""
    H, V, lam = _setup(n=6, r=3, seed=5)
    c = OR.phi_coeffs(lam, "qLL", 0.3)
    Y = H.apply(V)
    Wp = (Y - V @ (V.conj().T @ Y)) * c.conj()[None, :]
    orig = OR.apply_left
    monkeypatch.setattr(OR, "apply_left", lambda A, us, b: orig(A, us[:-1], b[:-1]))
    out = OR.rhs(H, V, lam, "qLL", 0.3)
    assert np.abs(out["W"] - Wp).max() > 1e-6


@pytest.mark.parametrize("model", ["qLL", "qLLG"])
def test_x11_structure_and_trace(model):
    H, V, lam = _setup(seed=6)
    out = OR.rhs(H, V, lam, model, 0.4)
    X11 = out["X11"]
    np.testing.assert_allclose(X11, X11.conj().T, atol=1e-15)
    assert np.abs(np.diag(X11)).max() < 1e-15
    f = OR.rhs_dense_from_factors(V, out["Z"], out["W"])
    assert abs(np.trace(f)) < 1e-14  # trace conservation


@pytest.mark.parametrize("model", ["qLL", "qLLG"])
def test_energy_dissipation_sign(model):
    """d<H>/dt = Tr(H f) <= 0 for kappa > 0 and == 0 for kappa = 0."""
    H, V, lam = _setup(n=6, r=3, seed=7)
    Hd = H.dense()
    for kappa in (0.0, 0.2, 1.0):
        out = OR.rhs(H, V, lam, model, kappa)
        f = OR.rhs_dense_from_factors(V, out["Z"], out["W"])
        dE = np.trace(Hd @ f).real
        if kappa == 0.0:
            assert abs(dE) < 1e-13
        else:
            assert dE < 0.0


def test_qll_qllg_equal_weight_rescale():
    """For equal nonzero eigenvalues lam, f_LLG = f_LL / (1 + kappa^2 lam^2)."""
    H, V, _ = _setup(n=6, r=3, seed=8)
    lam = np.full(3, 1.0 / 3.0)
    k = 0.7
    a = OR.rhs(H, V, lam, "qLL", k)
    b = OR.rhs(H, V, lam, "qLLG", k)
    fa = OR.rhs_dense_from_factors(V, a["Z"], a["W"])
    fb = OR.rhs_dense_from_factors(V, b["Z"], b["W"])
    np.testing.assert_allclose(fb, fa / (1 + k ** 2 * lam[0] ** 2), atol=1e-15)
