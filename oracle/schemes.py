"""LREI-RK (Sec. 3.7) and LREI-AB (Sec. 3.8) time steps.

The state is (V, lam0): rho = V diag(lam0) V*, lam0 fixed for all time
(the spectrum-preserving projection of Sec. 2 / Sec. 3.7).

Readings:
* RK tableaux beyond RK2 are deferred by the paper to Butcher's book; we take
  RK1 = Euler, RK2 = the paper's Heun tableau (a21 = 1, b = (1/2, 1/2)),
  RK3 = Kutta's third-order method, RK4 = the classical method; BS3 is the
  third-order member of the Bogacki-Shampine 3(2) pair used for adaptive
  stepping.
* The AB2 coefficients as printed (3/2, -3/2) are garbled; the standard
  Adams-Bashforth coefficients are used: AB2 (3/2, -1/2), AB3 (23, -16, 5)/12,
  AB4 (55, -59, 37, -9)/24.
* AB start-up ("an RK method of global order m-1"): by default the first m-1
  steps are LREI-RK4 steps; the right-hand side stored for the history at each
  of those step points is the stage-1 right-hand side of that RK step.
"""
import numpy as np

from .rhs import rhs
from .lowrank import stage_matrix, partial_eig

RK_TABLEAUX = {
    "RK1": (np.zeros((1, 1)), np.array([1.0])),
    "RK2": (np.array([[0.0, 0.0], [1.0, 0.0]]), np.array([0.5, 0.5])),
    "RK3": (np.array([[0.0, 0.0, 0.0], [0.5, 0.0, 0.0], [-1.0, 2.0, 0.0]]),
            np.array([1.0, 4.0, 1.0]) / 6.0),
    "RK4": (np.array([[0.0, 0.0, 0.0, 0.0], [0.5, 0.0, 0.0, 0.0], [0.0, 0.5, 0.0, 0.0],
                      [0.0, 0.0, 1.0, 0.0]]),
            np.array([1.0, 2.0, 2.0, 1.0]) / 6.0),
    # Bogacki-Shampine (1989): the third-order solution of the adaptive pair
    # in oracle/adaptive.py, as a fixed-step scheme
    "BS3": (np.array([[0.0, 0.0, 0.0], [0.5, 0.0, 0.0], [0.0, 0.75, 0.0]]),
            np.array([2.0, 3.0, 4.0]) / 9.0),
}

AB_COEFFS = {
    "AB2": np.array([3.0, -1.0]) / 2.0,
    "AB3": np.array([23.0, -16.0, 5.0]) / 12.0,
    "AB4": np.array([55.0, -59.0, 37.0, -9.0]) / 24.0,
}


def lrei_rk_step(H, V, lam0, model, kappa, h, scheme="RK4", hbar=1.0, eig=partial_eig,
                 return_f1=False):
    """One LREI-RK step (eq. 3.7 in low-rank form, eqs. 3.8-3.9)."""
    a, b = RK_TABLEAUX[scheme]
    s = b.size
    r = V.shape[1]
    stage_terms = []
    Vj = V
    f1 = None
    for j in range(s):
        out = rhs(H, Vj, lam0, model, kappa, hbar)
        stage_terms.append((Vj, out["Z"], out["W"]))
        if j == 0:
            f1 = (Vj, out["Z"], out["W"])
        if j + 1 < s:
            K = stage_matrix(V, lam0, stage_terms, h, a[j + 1, : j + 1])
            _, Vj = eig(K, r)
    K = stage_matrix(V, lam0, stage_terms, h, b)
    _, Vnew = eig(K, r)
    if return_f1:
        return Vnew, f1
    return Vnew


def lrei_ab_run(H, V, lam0, model, kappa, h, n_steps, scheme="AB3", hbar=1.0,
                bootstrap="RK4", eig=partial_eig, callback=None):
    """n_steps of LREI-AB (Sec. 3.8) with an RK start-up; returns the final V."""
    bcoef = AB_COEFFS[scheme]
    m = bcoef.size
    r = V.shape[1]
    history = []  # most recent first: (V_l, Z_l, W_l)
    for k in range(n_steps):
        if k < m - 1:
            Vnew, f1 = lrei_rk_step(H, V, lam0, model, kappa, h, bootstrap, hbar, eig,
                                    return_f1=True)
            history.insert(0, f1)
        else:
            out = rhs(H, V, lam0, model, kappa, hbar)
            history.insert(0, (V, out["Z"], out["W"]))
            history = history[:m]
            K = stage_matrix(V, lam0, history, h, bcoef)
            _, Vnew = eig(K, r)
        V = Vnew
        if callback is not None:
            callback(k, V)
    return V


def run(H, V, lam0, model, kappa, h, n_steps, scheme="RK4", hbar=1.0, eig=partial_eig,
        callback=None):
    """Advance n_steps with an RK or AB scheme; returns the final support V."""
    if scheme.startswith("AB"):
        return lrei_ab_run(H, V, lam0, model, kappa, h, n_steps, scheme, hbar, eig=eig,
                           callback=callback)
    for k in range(n_steps):
        V = lrei_rk_step(H, V, lam0, model, kappa, h, scheme, hbar, eig)
        if callback is not None:
            callback(k, V)
    return V
