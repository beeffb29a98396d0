"""Pins for the LREI time steps (Secs. 3.6, 3.7) against dense EI, closed forms and
convergence orders."""
import numpy as np
import pytest

from oracle import schemes as OS, dense as OD, rhs as OR
from oracle.hamiltonian import Hamiltonian
from oracle.metrics import rel_fro_error, dense_rho
from oracle.observables import energy, magnetization
from workloads import (chain_bonds, haar_factor, dirichlet_spectrum, heisenberg_tensors,
                       uniform_field, af1_index, pure_factor)


def _random_H(n, rng):
    bonds = chain_bonds(n, periodic=True)
    return Hamiltonian(n, bonds, rng.normal(size=(bonds.shape[0], 3, 3)) * 0.5,
                       rng.normal(size=(n, 3)) * 0.5)


def _full_basis(V, rng):
    N, r = V.shape
    Q = np.linalg.qr(np.concatenate([V, rng.normal(size=(N, N - r))], axis=1))[0]
    Q[:, :r] = V
    return Q


@pytest.mark.parametrize("scheme", ["RK1", "RK2", "RK3", "RK4"])
@pytest.mark.parametrize("model", ["qLL", "qLLG"])
def test_lrei_rk_equals_dense_ei(scheme, model):
    """LREI-RK reproduces the dense EI-RK iteration (Sec. 3.7: not an approximation)."""
    rng = np.random.default_rng(11)
    n, r = 6, 3
    H = _random_H(n, rng)
    V = haar_factor(2 ** n, r, rng)
    lam = dirichlet_spectrum(r, rng)
    Hd = H.dense()
    U = _full_basis(V, rng)
    for _ in range(5):
        V = OS.lrei_rk_step(H, V, lam, model, 0.5, 0.02, scheme)
        U = OD.ei_rk_step(U, lam, Hd, model, 0.5, 0.02, scheme)
    assert rel_fro_error(V, lam, U[:, :r], lam) < 1e-12


def _dense_ei_ab(U, lam, Hd, model, kappa, h, steps, scheme):
    """Dense EI with Adams-Bashforth and an EI-RK4 start-up (same readings)."""
    N = Hd.shape[0]
    lf = np.zeros(N)
    lf[: lam.size] = lam
    bc = OS.AB_COEFFS[scheme]
    m = bc.size
    hist = []
    for k in range(steps):
        f = OD.dense_rhs(U, lf, Hd, model, kappa)
        hist.insert(0, f)
        hist = hist[:m]
        if k < m - 1:
            U = OD.ei_rk_step(U, lam, Hd, model, kappa, h, "RK4")
        else:
            K = dense_rho(U, lf) + h * sum(b * f for b, f in zip(bc, hist))
            U = OD.ei_project(K, lf)
    return U


@pytest.mark.parametrize("scheme", ["AB2", "AB3", "AB4"])
@pytest.mark.parametrize("model", ["qLL", "qLLG"])
def test_lrei_ab_equals_dense_ei(scheme, model):
    rng = np.random.default_rng(12)
    n, r = 5, 2
    H = _random_H(n, rng)
    V = haar_factor(2 ** n, r, rng)
    lam = dirichlet_spectrum(r, rng)
    Vl = OS.lrei_ab_run(H, V, lam, model, 0.5, 0.01, 7, scheme)
    U = _dense_ei_ab(_full_basis(V, rng), lam, H.dense(), model, 0.5, 0.01, 7, scheme)
    assert rel_fro_error(Vl, lam, U[:, :r], lam) < 1e-12


def _pure_setup(n=4):
    bonds = chain_bonds(n, periodic=False)
    H = Hamiltonian(n, bonds, heisenberg_tensors(bonds.shape[0], 1.0),
                    uniform_field(n, (0.4, 0.0, 0.3)))
    V0 = pure_factor(n, index=af1_index(n))
    return H, V0


def _order(model, scheme, hs, T=0.4, kappa=0.5):
    H, V0 = _pure_setup()
    lam = np.array([1.0])
    rho_ex = OD.exact_pure(H.dense(), V0[:, 0], kappa, T, model)
    errs = []
    for h in hs:
        V = OS.run(H, V0, lam, model, kappa, h, int(round(T / h)), scheme)
        errs.append(np.linalg.norm(dense_rho(V, lam) - rho_ex) / np.linalg.norm(rho_ex))
    return np.polyfit(np.log(hs), np.log(errs), 1)[0]


@pytest.mark.parametrize("scheme,order", [("RK1", 1), ("RK2", 2), ("RK3", 3), ("RK4", 4)])
@pytest.mark.parametrize("model", ["qLL", "qLLG"])
def test_rk_convergence_order_vs_exact(scheme, order, model):
    """RKm reaches O(h^m) against the pure-state solution (eq. 1.4; Sec. 5.1)."""
    p = _order(model, scheme, [0.04, 0.02, 0.01])
    assert abs(p - order) < 0.25, p


@pytest.mark.parametrize("scheme,order", [("AB2", 2), ("AB3", 3), ("AB4", 4)])
def test_ab_convergence_order_vs_exact(scheme, order):
    p = _order("qLL", scheme, [0.01, 0.005, 0.0025], T=0.2)
    assert abs(p - order) < 0.35, p


@pytest.mark.parametrize("model", ["qLL", "qLLG"])
def test_dimer_closed_form(model):
    """Heisenberg dimer from |site0 up, site1 down>: <s^z_0>(t) = cos(2Jt)/cosh(2 kappa J t).

    Derived from eq. (1.4): the state is (|T0> + |S>)/sqrt 2 with energies J/2 and
    -3J/2 of H = (J/2) s.s; q-LLG uses t / (1 + kappa^2).
    """
    J, kappa, T, h = 1.0, 0.5, 0.6, 0.005
    H = Hamiltonian(2, np.array([[0, 1]]), heisenberg_tensors(1, J), None)
    V = pure_factor(2, index=2)
    V = OS.run(H, V, np.array([1.0]), model, kappa, h, int(round(T / h)), "RK4")
    tt = T if model == "qLL" else T / (1 + kappa ** 2)
    rho = dense_rho(V, [1.0])
    # s^z on site 0 (bit 0): +1 on indices 0, 2 and -1 on 1, 3
    sz_site0 = np.real(rho[2, 2] + rho[0, 0] - rho[1, 1] - rho[3, 3])
    assert abs(sz_site0 - np.cos(2 * J * tt) / np.cosh(2 * kappa * J * tt)) < 1e-9


def test_pure_state_qll_qllg_discrete_rescale():
    """Pure states: LREI-qLLG with step h == LREI-qLL with step h/(1+kappa^2), to rounding."""
    rng = np.random.default_rng(5)
    n = 7
    H = _random_H(n, rng)
    V0 = haar_factor(2 ** n, 1, rng)
    lam = np.array([1.0])
    k, h = 0.6, 0.02
    a = OS.run(H, V0, lam, "qLLG", k, h, 5, "RK4")
    b = OS.run(H, V0, lam, "qLL", k, h / (1 + k ** 2), 5, "RK4")
    assert rel_fro_error(a, lam, b, lam) < 1e-13


def test_kappa_zero_is_von_neumann():
    rng = np.random.default_rng(6)
    n, r = 5, 2
    H = _random_H(n, rng)
    V = haar_factor(2 ** n, r, rng)
    lam = dirichlet_spectrum(r, rng)
    T, h = 0.2, 0.005
    Vt = OS.run(H, V, lam, "qLL", 0.0, h, int(round(T / h)), "RK4")
    import scipy.linalg as sla
    Ut = sla.expm(-1j * H.dense() * T)
    rho_ex = Ut @ dense_rho(V, lam) @ Ut.conj().T
    assert np.linalg.norm(dense_rho(Vt, lam) - rho_ex) / np.linalg.norm(rho_ex) < 1e-8
    assert abs(energy(H, Vt, lam) - energy(H, V, lam)) < 1e-9


def test_fixed_point_polarised():
    """|up...up> commutes with a Heisenberg + z-field H and stays fixed."""
    n = 6
    bonds = chain_bonds(n)
    H = Hamiltonian(n, bonds, heisenberg_tensors(bonds.shape[0], 1.0), uniform_field(n, (0, 0, 0.8)))
    V = pure_factor(n, index=0)
    Vt = OS.run(H, V, np.array([1.0]), "qLLG", 0.5, 0.05, 10, "RK4")
    assert rel_fro_error(Vt, [1.0], V, [1.0]) < 1e-14


@pytest.mark.parametrize("model", ["qLL", "qLLG"])
def test_invariants_and_energy_decrease(model):
    rng = np.random.default_rng(8)
    n, r = 7, 4
    H = _random_H(n, rng)
    V = haar_factor(2 ** n, r, rng)
    lam = dirichlet_spectrum(r, rng)
    E = [energy(H, V, lam)]
    for _ in range(10):
        V = OS.lrei_rk_step(H, V, lam, model, 0.5, 0.02, "RK4")
        E.append(energy(H, V, lam))
        np.testing.assert_allclose(V.conj().T @ V, np.eye(r), atol=1e-13)
    assert np.all(np.diff(E) < 0)
    rho = dense_rho(V, lam)
    w = np.sort(np.linalg.eigvalsh(rho))[::-1]
    np.testing.assert_allclose(w[:r], lam, atol=1e-13)   # spectrum = Lambda_0
    assert np.abs(w[r:]).max() < 1e-13                    # rank r, PSD
    assert abs(np.trace(rho).real - 1.0) < 1e-13


def test_planted_wrong_tableau_is_caught(monkeypatch):
    """A wrong RK4 weight breaks the fourth-order convergence pin."""
    monkeypatch.setitem(OS.RK_TABLEAUX, "RK4", (OS.RK_TABLEAUX["RK4"][0],
                                                np.array([1.0, 2.0, 2.0, 1.0]) / 6.0 * 1.001))
    p = _order("qLL", "RK4", [0.04, 0.02, 0.01])
    assert abs(p - 4) > 0.5
