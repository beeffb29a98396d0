"""Stage matrices in low-rank form and their partial eigendecomposition.

A stage matrix (eq. 3.8) or the new step value (eq. 3.9) is kept as
    K = sum_l (A_l V_l* + V_l B_l*),
never as an N x N array.  ``LowRank`` stores the triples (A_l, V_l, B_l).

The partial eigendecomposition (Sec. 3.7) wants the r eigenpairs of the
Hermitian K with the largest eigenvalues (a reading: the paper's IRLM call
leaves the ordering unstated; the r largest algebraic ones, sorted
descending, pair with Lambda_0 sorted descending, Sec. 3.1).  Its plain
definition is computed exactly, without forming K:

    S1 = [A_1, V_1, A_2, V_2, ...],  S2 = [V_1, B_1, V_2, B_2, ...],  K = S1 S2*
    S1 = Q R (Householder QR, LAPACK)   =>   Q* K Q = R (S2* Q),
    eigh of that small Hermitian matrix; V_new = Q U_top.

range(K) lies in range(S1), so this is exact up to rounding even when S1 is
numerically rank deficient.  ``partial_eig_irlm`` runs the paper's own method
(ARPACK's implicitly restarted Lanczos on the matvec g of eq. 3.10) for
cross-checking.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla


class LowRank:
    def __init__(self):
        self.terms = []  # list of (A, V, B)

    def add(self, A, V, B):
        self.terms.append((np.asarray(A, np.complex128), np.asarray(V, np.complex128),
                           np.asarray(B, np.complex128)))

    @property
    def N(self):
        return self.terms[0][1].shape[0]

    def matvec(self, x):
        """g(x) = sum_l A_l (V_l* x) + V_l (B_l* x)  (eq. 3.10)."""
        x = np.asarray(x, dtype=np.complex128)
        y = np.zeros((self.N,) + x.shape[1:], dtype=np.complex128)
        for A, V, B in self.terms:
            y += A @ (V.conj().T @ x) + V @ (B.conj().T @ x)
        return y

    def dense(self):
        """K as a dense matrix (small N only)."""
        K = np.zeros((self.N, self.N), dtype=np.complex128)
        for A, V, B in self.terms:
            K += A @ V.conj().T + V @ B.conj().T
        return K

    def factors(self):
        S1 = np.concatenate([np.concatenate([A, V], axis=1) for A, V, B in self.terms], axis=1)
        S2 = np.concatenate([np.concatenate([V, B], axis=1) for A, V, B in self.terms], axis=1)
        return S1, S2


def stage_matrix(V1, lam0, stage_terms, h, coeffs):
    """K_{j+1} of eq. (3.8) (or rho_{k+1} of eq. (3.9) with b in place of a).

    stage_terms: list of (V_l, Z_l, W_l) for l = 1..j; coeffs: a_{j+1,l} (or b_l).
    A_1 = V_1 Lambda_0 + h a_1 Z_1, B_1 = h a_1 W_1; A_l = h a_l Z_l, B_l = h a_l W_l.
    The Lambda_0 term uses the fixed initial spectrum (Sec. 3.7).
    """
    K = LowRank()
    lam0 = np.asarray(lam0, dtype=np.float64)
    for l, ((Vl, Zl, Wl), a) in enumerate(zip(stage_terms, coeffs)):
        if l == 0:
            A = V1 * lam0[None, :] + h * a * Zl
            K.add(A, Vl, h * a * Wl)
        elif a != 0.0:
            K.add(h * a * Zl, Vl, h * a * Wl)
    if len(stage_terms) == 0:
        K.add(V1 * lam0[None, :], V1, np.zeros_like(V1))
    return K


def partial_eig(K, r):
    """The r largest eigenpairs of the Hermitian low-rank K, descending."""
    S1, S2 = K.factors()
    Q, R = sla.qr(S1, mode="economic")
    M = R @ (S2.conj().T @ Q)
    M = 0.5 * (M + M.conj().T)
    w, U = np.linalg.eigh(M)
    order = np.argsort(w)[::-1][:r]
    return w[order], Q @ U[:, order]


def partial_eig_irlm(K, r, tol=1e-13):
    """The paper's route: ARPACK IRLM (eigsh) with the matvec g (eq. 3.10)."""
    N = K.N
    op = spla.LinearOperator((N, N), matvec=lambda x: K.matvec(x.reshape(N, 1)).ravel(),
                             dtype=np.complex128)
    w, U = spla.eigsh(op, k=r, which="LA", ncv=max(2 * r + 1, 20), tol=tol)
    order = np.argsort(w)[::-1]
    return w[order], U[:, order]


def state_from_factor(A, tol=1e-14):
    """Initial partial eigendecomposition of rho_0 = A A* / Tr(A A*) (Sec. 3.7:
    the run starts from rho_0 = V Lambda_0 V*, r = rank rho_0), by
    Rayleigh-Ritz on the range of A: A = Q R, rho_0 = Q (R R*) Q* / Tr, so the
    eigenpairs come from the small matrix R R*.  Eigenvalues at or below
    tol * the largest are dropped (the rank).  Returns (lam descending, V)."""
    A = np.asarray(A, dtype=np.complex128)
    Q, R = np.linalg.qr(A)
    w, U = np.linalg.eigh(R @ R.conj().T)
    order = np.argsort(w)[::-1]
    w, U = w[order], U[:, order]
    keep = w > tol * w[0]
    return w[keep] / np.sum(w[keep]), Q @ U[:, keep]
