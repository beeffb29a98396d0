"""Dense N x N reference forms (small n only).

* q-LL right-hand side from commutators, eq. (1.1).
* q-LLG right-hand side through the eigenbasis (Sec. 2, eqs. 2.1-2.6):
  rho = V Lambda V*, X = V* rho_dot V solves (I + S) X - X S = D with
  D = (i/hbar) V* [rho, H] V and S = -i kappa Lambda, column-wise
  x_l = cwd(d_l, e + s - s_l e); rho_dot = V X V*.
* The EI-RK method of Sec. 2: every stage matrix is eigendecomposed and its
  eigenvalues replaced by Lambda(0) (top r get lam0, the rest zero).
* A plain (non-conservative) RK4 on the ODE, for convergence-order checks.
* The pure-state solution, eq. (1.4).  Reading: the printed right factor
  exp(+i H~ t / hbar) with H~ = (1 - i kappa) H is not the adjoint of the left
  factor; the solution of eq. (1.1) uses the adjoint, i.e.
  psi(t) = exp(-i H~ t / hbar) psi_0 / ||.||, rho = psi psi*.  For q-LLG the
  same formula holds with t -> t / (1 + kappa^2) (Sec. 1).
"""
import numpy as np
import scipy.linalg as sla

from .schemes import RK_TABLEAUX


def comm(A, B):
    return A @ B - B @ A


def rhs_qll(rho, H, kappa, hbar=1.0):
    """eq. (1.1): (i/hbar)[rho, H] - (kappa/hbar)[rho, [rho, H]]."""
    c = comm(rho, H)
    return (1j / hbar) * c - (kappa / hbar) * comm(rho, c)


def rhs_qllg_eig(V, lam, H, kappa, hbar=1.0):
    """q-LLG right-hand side through the full eigenbasis (eqs. 2.3-2.6)."""
    lam = np.asarray(lam, dtype=np.float64)
    rho = (V * lam[None, :]) @ V.conj().T
    D = (1j / hbar) * (V.conj().T @ comm(rho, H) @ V)
    s = -1j * kappa * lam
    # column l: x_l = d_l ./ (e + s - s_l e)
    denom = 1.0 + s[:, None] - s[None, :]
    X = D / denom
    return V @ X @ V.conj().T


def rhs_qllg_residual(rho, rho_dot, H, kappa, hbar=1.0):
    """Residual of the implicit q-LLG equation (1.2)."""
    return rho_dot - (1j / hbar) * comm(rho, H) - 1j * kappa * comm(rho, rho_dot)


def full_eig_desc(K):
    K = 0.5 * (K + K.conj().T)
    w, U = np.linalg.eigh(K)
    order = np.argsort(w)[::-1]
    return w[order], U[:, order]


def dense_rhs(V_full, lam_full, H, model, kappa, hbar=1.0):
    rho = (V_full * lam_full[None, :]) @ V_full.conj().T
    if model == "qLL":
        return rhs_qll(rho, H, kappa, hbar)
    return rhs_qllg_eig(V_full, lam_full, H, kappa, hbar)


def ei_project(K, lam0_full):
    """Eigenvectors of K (descending) with the spectrum replaced by Lambda(0)."""
    _, U = full_eig_desc(K)
    return U


def ei_rk_step(rho_V, lam0, H, model, kappa, h, scheme="RK4", hbar=1.0):
    """One EI-RK step of Sec. 2 on dense matrices; returns the new full eigenbasis.

    rho_V: full N x N eigenbasis of the current (projected) rho, descending.
    """
    N = H.shape[0]
    lam_full = np.zeros(N)
    lam_full[: lam0.size] = lam0
    a, b = RK_TABLEAUX[scheme]
    s = b.size
    K1 = (rho_V * lam_full[None, :]) @ rho_V.conj().T
    fs = []
    Vj = rho_V
    for j in range(s):
        fs.append(dense_rhs(Vj, lam_full, H, model, kappa, hbar))
        if j + 1 < s:
            K = K1 + h * sum(a[j + 1, l] * fs[l] for l in range(j + 1))
            Vj = ei_project(K, lam_full)
    K = K1 + h * sum(b[l] * fs[l] for l in range(s))
    return ei_project(K, lam_full)


def rk4_plain(rho, H, model, kappa, h, hbar=1.0):
    """One classical RK4 step on the ODE itself (no spectrum projection)."""
    def f(R):
        R = 0.5 * (R + R.conj().T)
        if model == "qLL":
            return rhs_qll(R, H, kappa, hbar)
        w, U = np.linalg.eigh(R)
        return rhs_qllg_eig(U, w, H, kappa, hbar)
    k1 = f(rho)
    k2 = f(rho + 0.5 * h * k1)
    k3 = f(rho + 0.5 * h * k2)
    k4 = f(rho + h * k3)
    return rho + h / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)


def exact_pure(H, psi0, kappa, t, model="qLL", hbar=1.0):
    """rho(t) for a pure initial state (eq. 1.4 with the adjoint right factor)."""
    tt = t if model == "qLL" else t / (1.0 + kappa ** 2)
    Ht = (1.0 - 1j * kappa) * H
    psi = sla.expm(-1j * Ht * tt / hbar) @ np.asarray(psi0, dtype=np.complex128).reshape(-1)
    psi = psi / np.linalg.norm(psi)
    return np.outer(psi, psi.conj())
