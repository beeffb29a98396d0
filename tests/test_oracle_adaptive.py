"""Pins for the adaptive LREI-RK oracle (oracle/adaptive.py): the embedded
pairs against the Butcher order conditions, the error estimate against its
asymptotic order, against the distance of the two projected candidates and
against the true local error of the embedded solution (pure-state solution,
eq. 1.4), the third-order solution against the dense EI method of Sec. 2, and
the step-size controller against its defining rules."""
import math

import numpy as np
import pytest

from oracle import adaptive as OA, dense as OD, schemes as OS
from oracle.hamiltonian import Hamiltonian
from oracle.metrics import dense_rho, rel_fro_error
from workloads import (af1_index, chain_bonds, dirichlet_spectrum, haar_factor, heisenberg_tensors,
                       pure_factor, uniform_field)


def _conditions(a, b):
    """Left-hand sides of the order conditions up to order 4:
    sum b, sum b c, sum b c^2, sum b a c, sum b c^3, sum b c (a c),
    sum b a c^2, sum b a a c (c_i = sum_j a_ij)."""
    c = a.sum(axis=1)
    return np.array([b.sum(), b @ c, b @ c ** 2, b @ (a @ c), b @ c ** 3, b @ (c * (a @ c)),
                     b @ (a @ c ** 2), b @ (a @ (a @ c))])


def _extended(pair):
    """(a, b, b_hat) over every right-hand side: with FSAL the last stage is
    the new state, a_{s+1, :} = b."""
    a, b, bh, _, _, fsal = OA.PAIRS[pair]
    if not fsal:
        return a, b, bh
    s = b.size
    ae = np.zeros((s + 1, s + 1))
    ae[:s, :s] = a
    ae[s, :s] = b
    return ae, np.concatenate([b, [0.0]]), bh


EXACT = np.array([1.0, 0.5, 1.0 / 3.0, 1.0 / 6.0, 0.25, 0.125, 1.0 / 12.0, 1.0 / 24.0])


@pytest.mark.parametrize("pair", ["HE21", "BS32", "RK43"])
def test_pair_order_conditions(pair):
    """b meets the conditions of its order p; b_hat those of order q = p - 1
    and not all of order p (a genuine lower-order estimate)."""
    a, b, bh = _extended(pair)
    _, _, _, p, q, _ = OA.PAIRS[pair]
    nc = {1: 1, 2: 2, 3: 4, 4: 8}
    cb, ch = _conditions(a, b), _conditions(a, bh)
    assert np.allclose(cb[: nc[p]], EXACT[: nc[p]], atol=1e-15)
    assert np.allclose(ch[: nc[q]], EXACT[: nc[q]], atol=1e-15)
    assert not np.allclose(ch[: nc[p]], EXACT[: nc[p]], atol=1e-3)
    # the error weights sum to zero: E is O(h^{q+1}), not O(h)
    assert abs(OA.error_weights(pair).sum()) < 1e-15


def test_bs3_tableau_is_the_fixed_step_member():
    a, b, _, _, _, _ = OA.PAIRS["BS32"]
    at, bt = OS.RK_TABLEAUX["BS3"]
    assert np.array_equal(a, at) and np.array_equal(b, bt)
    # the order-4 pair advances with the classical RK4 step itself
    a, b, _, _, _, _ = OA.PAIRS["RK43"]
    at, bt = OS.RK_TABLEAUX["RK4"]
    assert np.array_equal(a, at) and np.array_equal(b, bt)


def _random_H(n, rng):
    bonds = chain_bonds(n, periodic=True)
    return Hamiltonian(n, bonds, rng.normal(size=(bonds.shape[0], 3, 3)) * 0.5,
                       rng.normal(size=(n, 3)) * 0.5)


def _full_basis(V, rng):
    N, r = V.shape
    Q = np.linalg.qr(np.concatenate([V, rng.normal(size=(N, N - r))], axis=1))[0]
    Q[:, :r] = V
    return Q


@pytest.mark.parametrize("model", ["qLL", "qLLG"])
def test_bs3_solution_equals_dense_ei(model):
    """The accepted state of an attempt is the EI-RK step of Sec. 2 (dense) with
    the Bogacki-Shampine tableau."""
    rng = np.random.default_rng(21)
    n, r = 6, 3
    H = _random_H(n, rng)
    V = haar_factor(2 ** n, r, rng)
    lam = dirichlet_spectrum(r, rng)
    U = _full_basis(V, rng)
    for _ in range(3):
        V, _ = OA.attempt(H, V, lam, model, 0.5, 0.02, "BS32")
        U = OD.ei_rk_step(U, lam, H.dense(), model, 0.5, 0.02, "BS3")
    assert rel_fro_error(V, lam, U[:, :r], lam) < 1e-12


def test_bs3_convergence_order_vs_exact():
    """Fixed-step BS3 reaches O(h^3) against the pure-state solution (eq. 1.4)."""
    H, V0 = _pure_setup()
    lam = np.array([1.0])
    T, kappa = 0.4, 0.5
    rho_ex = OD.exact_pure(H.dense(), V0[:, 0], kappa, T, "qLL")
    hs = [0.04, 0.02, 0.01]
    errs = [np.linalg.norm(dense_rho(OS.run(H, V0, lam, "qLL", kappa, h, int(round(T / h)), "BS3"), lam) - rho_ex)
            for h in hs]
    assert abs(np.polyfit(np.log(hs), np.log(errs), 1)[0] - 3.0) < 0.25


def _pure_setup(n=4):
    bonds = chain_bonds(n, periodic=False)
    H = Hamiltonian(n, bonds, heisenberg_tensors(bonds.shape[0], 1.0), uniform_field(n, (0.4, 0.0, 0.3)))
    return H, pure_factor(n, index=af1_index(n))


def test_tangent_error_equals_dense_projection():
    """||T(E)||_F against the tangent projection written out on dense matrices:
    T(E) = P E Q + Q E P + Q (E - diag) Q restricted to distinct eigenvalues,
    Q = V V*, P = I - Q."""
    rng = np.random.default_rng(3)
    N, r = 32, 3
    terms = [tuple(rng.normal(size=(N, r)) + 1j * rng.normal(size=(N, r)) for _ in range(3)) for _ in range(4)]
    e = np.array([0.3, -0.1, 0.0, -0.2])
    h = 0.7
    V = np.linalg.qr(rng.normal(size=(N, r)) + 1j * rng.normal(size=(N, r)))[0]
    for lam in (np.array([0.5, 0.3, 0.2]), np.array([0.4, 0.4, 0.2])):
        E = sum(h * el * (Z @ Vl.conj().T + Vl @ W.conj().T) for (Vl, Z, W), el in zip(terms, e))
        E = 0.5 * (E + E.conj().T)
        Q = V @ V.conj().T
        P = np.eye(N) - Q
        M = V.conj().T @ E @ V
        M[lam[:, None] == lam[None, :]] = 0.0  # rotations within an eigenspace leave rho unchanged
        T = P @ E @ Q + Q @ E @ P + V @ M @ V.conj().T
        got = OA.tangent_error(OA.error_matrix(terms, h, e), V, lam)
        assert abs(got - np.linalg.norm(T)) < 1e-12 * np.linalg.norm(T)


@pytest.mark.parametrize("pair", ["HE21", "BS32", "RK43"])
@pytest.mark.parametrize("model", ["qLL", "qLLG"])
def test_error_estimate_order(pair, model):
    """The estimate is O(h^{q+1}) for the embedded order q."""
    rng = np.random.default_rng(4)
    H = _random_H(5, rng)
    V = haar_factor(32, 2, rng)
    lam = dirichlet_spectrum(2, rng)
    hs = np.array([0.02, 0.01, 0.005])
    errs = [OA.attempt(H, V, lam, model, 0.5, h, pair)[1] for h in hs]
    q = OA.PAIRS[pair][4]
    assert abs(np.polyfit(np.log(hs), np.log(errs), 1)[0] - (q + 1)) < 0.1


@pytest.mark.parametrize("pair", ["HE21", "BS32", "RK43"])
def test_error_estimate_matches_projected_candidates(pair):
    """The estimate against the distance of the two projected candidates
    (eq. 3.9 with b and with b_hat): equal to leading order, while ||E||_F
    itself is not."""
    rng = np.random.default_rng(8)
    H = _random_H(5, rng)
    V = haar_factor(32, 3, rng)
    lam = dirichlet_spectrum(3, rng)
    ratios, full = [], []
    for h in (0.01, 0.0025):
        Vb, err, terms = OA.attempt(H, V, lam, "qLLG", 0.5, h, pair, return_terms=True)
        Vh = OA.embedded_solution(V, lam, terms, h, pair, 3)
        dist = np.linalg.norm(dense_rho(Vb, lam) - dense_rho(Vh, lam))
        ratios.append(dist / err)
        Ed = OA.error_matrix(terms, h, OA.error_weights(pair)).dense()
        full.append(dist / np.linalg.norm(0.5 * (Ed + Ed.conj().T)))
    # closer to 1 at the smaller step, down to the rounding of distances ~1e-10
    assert abs(ratios[1] - 1.0) < 1e-3 and abs(ratios[1] - 1.0) <= max(abs(ratios[0] - 1.0), 1e-5), ratios
    assert full[1] < 0.95, full


@pytest.mark.parametrize("pair", ["HE21", "BS32", "RK43"])
def test_error_estimate_matches_true_local_error(pair):
    """Against the pure-state solution (eq. 1.4): the true local error of the
    embedded candidate approaches the estimate as h -> 0 (the order-p
    solution's own error is an order smaller)."""
    H, V0 = _pure_setup()
    lam = np.array([1.0])
    Hd = H.dense()
    ratios = []
    for h in (0.02, 0.005):
        Vb, err, terms = OA.attempt(H, V0, lam, "qLL", 0.5, h, pair, return_terms=True)
        Vh = OA.embedded_solution(V0, lam, terms, h, pair, 1)
        ex = OD.exact_pure(Hd, V0[:, 0], 0.5, h, "qLL")
        true_hat = np.linalg.norm(dense_rho(Vh, lam) - ex)
        true_b = np.linalg.norm(dense_rho(Vb, lam) - ex)
        assert true_b < 0.2 * true_hat
        ratios.append(true_hat / err)
    assert abs(ratios[1] - 1.0) < 0.1, ratios


def test_planted_wrong_error_weight_is_caught(monkeypatch):
    """A mistyped embedded weight breaks the estimate's order."""
    a, b, bh, p, q, fsal = OA.PAIRS["BS32"]
    bad = bh.copy()
    bad[1] = 0.3
    monkeypatch.setitem(OA.PAIRS, "BS32", (a, b, bad, p, q, fsal))
    rng = np.random.default_rng(4)
    H = _random_H(5, rng)
    V = haar_factor(32, 2, rng)
    lam = dirichlet_spectrum(2, rng)
    hs = np.array([0.02, 0.01, 0.005])
    errs = [OA.attempt(H, V, lam, "qLL", 0.5, h, "BS32")[1] for h in hs]
    assert abs(np.polyfit(np.log(hs), np.log(errs), 1)[0] - 3.0) > 0.5


# ---- the controller ------------------------------------------------------------

def test_control_accept_and_growth_limits():
    # err = tol / 2^3: factor 0.9 * 2 = 1.8 for q = 2
    acc, t, h, done, failed = OA.control(1e-6 / 8, 0.1, 0.0, 10.0, 1e-6, 1e-9, 1.0, 2, False)
    assert acc and not done and not failed and t == 0.1 and abs(h - 0.18) < 1e-15
    # tiny error: growth capped at facmax, then at h_max
    assert OA.control(1e-30, 0.1, 0.0, 10.0, 1e-6, 1e-9, 1.0, 2, False)[2] == 0.5
    assert OA.control(1e-30, 0.1, 0.0, 10.0, 1e-6, 1e-9, 0.3, 2, False)[2] == 0.3
    assert OA.control(0.0, 0.1, 0.0, 10.0, 1e-6, 1e-9, 1.0, 2, False)[2] == 0.5
    # right after a rejection the step does not grow
    assert OA.control(1e-30, 0.1, 0.0, 10.0, 1e-6, 1e-9, 1.0, 2, True)[2] == 0.1


def test_control_reject_shrinks_and_fails_at_h_min():
    acc, t, h, done, failed = OA.control(8e-6, 0.1, 0.5, 10.0, 1e-6, 1e-9, 1.0, 2, False)
    assert not acc and t == 0.5 and abs(h - 0.1 * 0.9 * 0.5) < 1e-15 and not failed
    # huge error: shrink capped at facmin
    assert OA.control(1.0, 0.1, 0.5, 10.0, 1e-6, 1e-9, 1.0, 2, False)[2] == pytest.approx(0.02, rel=1e-15)
    # non-finite estimate: rejection with facmin
    acc, _, h, _, _ = OA.control(math.nan, 0.1, 0.5, 10.0, 1e-6, 1e-9, 1.0, 2, False)
    assert not acc and h == pytest.approx(0.02, rel=1e-15)
    # a rejection at h_min stops the integration
    assert OA.control(8e-6, 1e-3, 0.5, 10.0, 1e-6, 1e-3, 1.0, 2, False)[4]


def test_control_lands_on_t_end():
    # the proposal is clamped to the time left ...
    acc, t, h, done, _ = OA.control(1e-9, 0.1, 0.0, 0.15, 1e-6, 1e-9, 1.0, 2, False)
    assert acc and t == 0.1 and h == 0.15 - 0.1 and not done
    # ... and the clamped step ends exactly at t_end
    acc, t, h, done, _ = OA.control(1e-9, 0.15 - 0.1, 0.1, 0.15, 1e-6, 1e-9, 1.0, 2, False)
    assert acc and done and t == 0.15


def test_evolve_reaches_t_end_and_error_follows_tol():
    """Adaptive BS3(2) on the pure-state problem: reaches t_end exactly, and the
    global error against eq. 1.4 falls with the tolerance while the step
    count grows about like tol^(-1/3)."""
    H, V0 = _pure_setup()
    lam = np.array([1.0])
    T, kappa = 0.5, 0.5
    rho_ex = OD.exact_pure(H.dense(), V0[:, 0], kappa, T, "qLL")
    res = {}
    for tol in (1e-5, 1e-7):
        V, log = OA.evolve(H, V0, lam, "qLL", kappa, T, tol, 0.05, 1e-8, 1.0)
        assert log[-1] == "done"
        acc = [x for x in log[:-1] if x[3]]
        assert abs(sum(x[1] for x in acc) - T) < 1e-13
        assert all(x[2] <= tol for x in acc)
        res[tol] = (np.linalg.norm(dense_rho(V, lam) - rho_ex), len(acc))
    (e1, n1), (e2, n2) = res[1e-5], res[1e-7]
    assert e2 < e1 / 10
    assert 2.5 < n2 / n1 < 8.0, (n1, n2)


def test_evolve_stops_at_h_min():
    H, V0 = _pure_setup()
    V, log = OA.evolve(H, V0, np.array([1.0]), "qLL", 0.5, 0.5, 1e-14, 0.05, 0.01, 1.0)
    assert log[-1] == "h_min"
    assert not log[-2][3]
