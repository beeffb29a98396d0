"""Expectation values from the factor only (Sec. 3.5, eq. 3.6).

<A> = Tr(A rho) = Tr(Lambda_0 (V* (A V))): apply A to the tall-skinny V, then
a small Gram product, then the trace against Lambda_0.
"""
import numpy as np

from .hamiltonian import apply_pauli


def expectation(apply_A, V, lam0):
    AV = apply_A(V)
    return float(np.real(np.trace(np.diag(lam0) @ (V.conj().T @ AV))))


def energy(H, V, lam0):
    """<H> = Tr(Lambda_0 V* H V)."""
    return expectation(H.apply, V, lam0)


def magnetization(n, V, lam0, hbar=1.0):
    """(M_x, M_y, M_z) with M_v = (1/n) sum_i S_i^v and S = (hbar/2) s (eq. 3.5)."""
    out = []
    for a in range(3):
        tot = 0.0
        for i in range(n):
            tot += expectation(lambda X: 0.5 * hbar * apply_pauli(X, i, a), V, lam0)
        out.append(tot / n)
    return np.array(out)
