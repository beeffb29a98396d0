"""Low-rank right-hand side of q-LLG (Sec. 3.1-3.4) and q-LL (Sec. 4).

Given the support V (N x r, orthonormal columns) and the fixed spectrum
Lambda = diag(lam) of rho = V Lambda V*, the right-hand side is returned as
the pair (Z, W) of eq. (3.4):  rho_dot = Z V* + V W*,  with
Z = V X11 + W and W = Vhat X12*, where Vhat spans the complement of V.

Steps, in the paper's order:

1. Y = H V (matrix-free) and G = V* H V (Sec. 3.3).  G is Hermitian in exact
   arithmetic; it is symmetrised, (G + G*)/2, before use (a reading: the paper
   uses H = H* implicitly).
2. X11 and X12 from eq. (3.2) (q-LLG: componentwise division by the
   denominators E + L + L*) or eq. (4.1) (q-LL).  X12 = diag(c) (V* H Vhat)
   with c_a = (i/hbar) lam_a / (1 - i kappa lam_a) (q-LLG) or
   c_a = (1/hbar)(i - kappa lam_a) lam_a (q-LL).
3. The r Householder vectors of V (eq. 3.3) and their action (Sec. 3.4):
   Y* Vhat = last N-r columns of Y* P_1 ... P_r, and
   W = Vhat X12* = P_1 ... P_r [0; X12*].
4. Z = V X11 + W.

Householder phase convention (a reading; the paper fixes only P = I -
2 u u*/(u* u)): u = x + e^{i arg x_1} ||x|| e_1, which never cancels.  Only
Vhat Vhat* = I - V V* enters W, so the convention does not change results.
"""
import numpy as np


def phi_coeffs(lam, model, kappa, hbar=1.0):
    """Denominator-divided X-block coefficients of eqs. (3.2) / (4.1).

    Returns (Phi, c): X11 = Phi o (D11-numerator form) is not used directly;
    instead x_blocks() follows the paper's formulas.  c gives X12 = diag(c) A.
    """
    lam = np.asarray(lam, dtype=np.float64)
    if model == "qLLG":
        c = (1j / hbar) * lam / (1.0 - 1j * kappa * lam)
    elif model == "qLL":
        c = (1.0 / hbar) * (1j - kappa * lam) * lam
    else:
        raise ValueError(model)
    return c


def x11_block(G, lam, model, kappa, hbar=1.0):
    """X11 from eq. (3.2) (q-LLG) or eq. (4.1) (q-LL), G = V* H V (r x r)."""
    lam = np.asarray(lam, dtype=np.float64)
    r = lam.size
    L = np.diag(lam).astype(np.complex128)
    D11 = (1j / hbar) * (L @ G - G @ L)
    if model == "qLLG":
        # L11 = -i kappa [lam lam ... lam]: column vector lam repeated r times.
        L11 = -1j * kappa * np.tile(lam.reshape(r, 1), (1, r))
        denom = np.ones((r, r)) + L11 + L11.conj().T
        return D11 / denom
    if model == "qLL":
        return (D11 - (kappa / hbar) * (L @ L @ G + G @ L @ L)
                + (2.0 * kappa / hbar) * (L @ G @ L))
    raise ValueError(model)


def householder_vectors(V):
    """Householder vectors u_k and beta_k = 2/(u_k* u_k) reducing V to upper form.

    P_k = I - beta_k u_k u_k* (eq. 3.3); Q = P_1 ... P_r has V's span in its
    first r columns.  Each u_k is stored as a full N-vector (zero above row k).
    """
    A = np.array(V, dtype=np.complex128, copy=True)
    N, r = A.shape
    us, betas = [], []
    for k in range(r):
        x = A[k:, k]
        alpha = np.linalg.norm(x)
        x0 = x[0]
        phase = x0 / abs(x0) if abs(x0) > 0 else 1.0
        u = np.zeros(N, dtype=np.complex128)
        u[k:] = x
        u[k] += phase * alpha
        beta = 2.0 / np.vdot(u, u).real
        # apply P_k to the working matrix from the left: A <- A - beta u (u* A)
        A -= beta * np.outer(u, u.conj() @ A)
        us.append(u)
        betas.append(beta)
    return us, betas


def apply_right(A, us, betas):
    """A P_1 P_2 ... P_r using AP = A - beta w u*, w = A u (Sec. 3.4)."""
    A = np.array(A, dtype=np.complex128, copy=True)
    for u, beta in zip(us, betas):
        w = A @ u
        A -= beta * np.outer(w, u.conj())
    return A


def apply_left(A, us, betas):
    """P_1 P_2 ... P_r A using PA = A - beta u w*, w = A* u (Sec. 3.4)."""
    A = np.array(A, dtype=np.complex128, copy=True)
    for u, beta in zip(reversed(us), reversed(betas)):
        w = A.conj().T @ u
        A -= beta * np.outer(u, w.conj())
    return A


def rhs(H, V, lam, model, kappa, hbar=1.0):
    """Low-rank right-hand side (Z, W) at rho = V diag(lam) V*.

    H is an object with .apply(V) -> H V.  Returns a dict with Z, W, X11, G, Y.
    """
    V = np.asarray(V, dtype=np.complex128)
    lam = np.asarray(lam, dtype=np.float64)
    N, r = V.shape
    Y = H.apply(V)
    G = V.conj().T @ Y
    G = 0.5 * (G + G.conj().T)
    X11 = x11_block(G, lam, model, kappa, hbar)
    c = phi_coeffs(lam, model, kappa, hbar)
    us, betas = householder_vectors(V)
    # V* H Vhat = (H V)* Vhat = Y* Vhat: last N - r columns of Y* P_1 ... P_r
    AV = apply_right(Y.conj().T, us, betas)
    VhHVhat = AV[:, r:]
    X12 = c[:, None] * VhHVhat                     # r x (N - r)
    A0 = np.zeros((N, r), dtype=np.complex128)
    A0[r:, :] = X12.conj().T
    W = apply_left(A0, us, betas)                  # Vhat X12* = V [0; X12*]
    Z = V @ X11 + W
    return dict(Z=Z, W=W, X11=X11, G=G, Y=Y)


def rhs_dense_from_factors(V, Z, W):
    """rho_dot = Z V* + V W* as a dense matrix (small N only; eq. 3.4)."""
    return Z @ V.conj().T + V @ W.conj().T
