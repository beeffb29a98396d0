"""Adaptive LREI-RK stepping with an embedded Runge-Kutta pair: plain reference.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper names time stepping that adapts the step size to local error
estimates as future work (Sec. 6).  The reading implemented here, and by the
GPU path:

* An embedded pair (a, b, b_hat) advances the state with the LREI-RK step of
  Sec. 3.7 for the tableau (a, b): stages by eq. 3.8, the new state by
  eq. 3.9, each followed by the partial eigendecomposition with Lambda_0.
  The embedded weights b_hat share those stages; a pair marked FSAL ("first
  same as last") also weights the right-hand side at the new state.
* Local error estimate.  The two candidate matrices of eq. 3.9,
  rho + h sum_l b_l f(rho_l) and rho + h sum_l b_hat_l f(rho_l), differ by
      E = h sum_l (b_l - b_hat_l) f(rho_l),   f(rho_l) = Z_l V_l* + V_l W_l*.
  The partial eigendecomposition with Lambda_0 keeps, to first order, only
  the part of E tangent to the fixed-spectrum manifold at the new state
  rho_new = V Lambda_0 V*: with P = I - V V* and M = V* E V,
      ||T(E)||_F^2 = 2 ||P E V||_F^2 + sum_{i != j, lam_i != lam_j} |M_ij|^2
  (the V-complement blocks and the rotations between distinct eigenvalues;
  the complement-complement block and the diagonal of M do not move the
  projected state).  ||T(E)||_F is the estimate: it equals the distance of
  the two projected candidates to leading order without a second
  eigendecomposition.  ||E||_F itself is not (E, a difference of tangent
  vectors at the stages, has a normal part of its own order).
* Step-size control (Hairer, Norsett & Wanner, Solving Ordinary Differential
  Equations I, Sec. II.4): accept when the estimate is <= tol; the next step is
  h min(facmax, max(facmin, 0.9 (tol / err)^(1 / (q + 1)))), q the order of
  the embedded solution, facmin = 0.2, facmax = 5 (1 right after a
  rejection); clamped to [h_min, h_max] and to the time left, so that the
  last accepted step lands on t_end exactly.  A rejection at h <= h_min
  stops the integration; a non-finite estimate counts as a rejection.

Pairs: Heun-Euler 2(1) (Heun's method with Euler embedded), Bogacki-Shampine
3(2) (Bogacki & Shampine, Appl. Math. Lett. 2, 1989), FSAL, and the classical
RK4 with an order-3 solution that replaces the last stage's weight by the
right-hand side at the new state, b_hat = (1, 2, 2, 0, 1) / 6 (FSAL; the
difference of the two is h (f(rho_new) - f(rho_4)) / 6).
"""
import math

import numpy as np

from .lowrank import LowRank, partial_eig, stage_matrix
from .rhs import rhs

FAC = 0.9
FACMIN = 0.2
FACMAX = 5.0

# name: (a [s x s], b [s], b_hat [s, or s + 1 with FSAL], order of b, order of b_hat, fsal)
PAIRS = {
    "HE21": (np.array([[0.0, 0.0], [1.0, 0.0]]), np.array([0.5, 0.5]), np.array([1.0, 0.0]), 2, 1, False),
    "BS32": (np.array([[0.0, 0.0, 0.0], [0.5, 0.0, 0.0], [0.0, 0.75, 0.0]]),
             np.array([2.0, 3.0, 4.0]) / 9.0,
             np.array([7.0 / 24.0, 0.25, 1.0 / 3.0, 0.125]), 3, 2, True),
    "RK43": (np.array([[0.0, 0.0, 0.0, 0.0], [0.5, 0.0, 0.0, 0.0], [0.0, 0.5, 0.0, 0.0], [0.0, 0.0, 1.0, 0.0]]),
             np.array([1.0, 2.0, 2.0, 1.0]) / 6.0,
             np.array([1.0, 2.0, 2.0, 0.0, 1.0]) / 6.0, 4, 3, True),
}


def error_weights(pair):
    """e = b - b_hat over every right-hand side the estimate uses."""
    a, b, bh, _, _, fsal = PAIRS[pair]
    bb = np.concatenate([b, [0.0]]) if fsal else b
    return bb - bh


def error_matrix(terms, h, e):
    """E = h sum_l e_l (Z_l V_l* + V_l W_l*) as a low-rank matrix."""
    K = LowRank()
    for (Vl, Zl, Wl), el in zip(terms, e):
        if el != 0.0:
            K.add(h * el * Zl, Vl, h * el * Wl)
    return K


def tangent_error(E, V, lam):
    """||T(E)||_F at rho = V diag(lam) V* (E low-rank, V orthonormal N x r)."""
    EV = 0.5 * (E.matvec(V) + _adjoint_matvec(E, V))  # Herm(E) V
    M = V.conj().T @ EV
    PEV = EV - V @ M
    lam = np.asarray(lam)
    off = (lam[:, None] != lam[None, :])
    return float(np.sqrt(2.0 * np.linalg.norm(PEV) ** 2 + np.sum(np.abs(M[off]) ** 2)))


def _adjoint_matvec(E, x):
    """E* x for E = sum_l A_l V_l* + V_l B_l*."""
    y = np.zeros_like(x, dtype=np.complex128)
    for A, V, B in E.terms:
        y += V @ (A.conj().T @ x) + B @ (V.conj().T @ x)
    return y


def attempt(H, V, lam0, model, kappa, h, pair="BS32", hbar=1.0, eig=partial_eig, return_terms=False):
    """One attempted step: the new support (order-p solution) and the error
    estimate ||T(E)||_F."""
    a, b, bh, _, _, fsal = PAIRS[pair]
    s = b.size
    r = V.shape[1]
    terms = []
    Vj = V
    for j in range(s):
        out = rhs(H, Vj, lam0, model, kappa, hbar)
        terms.append((Vj, out["Z"], out["W"]))
        if j + 1 < s:
            _, Vj = eig(stage_matrix(V, lam0, terms, h, a[j + 1, : j + 1]), r)
    _, Vnew = eig(stage_matrix(V, lam0, terms, h, b), r)
    if fsal:
        out = rhs(H, Vnew, lam0, model, kappa, hbar)
        terms.append((Vnew, out["Z"], out["W"]))
    err = tangent_error(error_matrix(terms, h, error_weights(pair)), Vnew, lam0)
    if return_terms:
        return Vnew, err, terms
    return Vnew, err


def embedded_solution(V, lam0, terms, h, pair, r, eig=partial_eig):
    """The embedded (order q) candidate: eq. 3.9 with b_hat (test helper)."""
    bh = PAIRS[pair][2]
    _, Vh = eig(stage_matrix(V, lam0, terms[: bh.size], h, bh), r)
    return Vh


def control(err, h, t, t_end, tol, h_min, h_max, q, after_reject):
    """Accept/reject an attempt of step h taken at time t, and the next step.

    Returns (accept, t_new, h_next, done, failed)."""
    rem = t_end - t
    last = h >= rem
    finite = math.isfinite(err)
    accept = finite and err <= tol
    if not finite:
        fac = FACMIN
    elif err > 0.0:
        fac = FAC * (tol / err) ** (1.0 / (q + 1))
    else:
        fac = FACMAX
    fac = min(1.0 if after_reject else FACMAX, max(FACMIN, fac))
    h_new = min(h * fac, h_max)
    failed = False
    if accept:
        t_new = t_end if last else t + h
    else:
        t_new = t
        failed = h <= h_min
    h_new = max(h_new, h_min)
    done = accept and last
    h_next = h_new if done else min(h_new, t_end - t_new)
    return accept, t_new, h_next, done, failed


def evolve(H, V, lam0, model, kappa, t_span, tol, h_init, h_min, h_max, max_attempts=100000,
           pair="BS32", hbar=1.0, eig=partial_eig):
    """Advance by t_span with step-size control; returns (V, log) where log
    lists (t, h, err, accepted) per attempt and ends with a status string
    ('done', 'h_min' or 'max_attempts')."""
    q = PAIRS[pair][4]
    t = 0.0
    h = min(h_init, h_max, t_span)
    after_reject = False
    log = []
    for _ in range(max_attempts):
        Vnew, err = attempt(H, V, lam0, model, kappa, h, pair, hbar, eig)
        accept, t_new, h_next, done, failed = control(err, h, t, t_span, tol, h_min, h_max, q, after_reject)
        log.append((t, h, err, accept))
        if accept:
            V = Vnew
        t, h, after_reject = t_new, h_next, not accept
        if done:
            return V, log + ["done"]
        if failed:
            return V, log + ["h_min"]
    return V, log + ["max_attempts"]
