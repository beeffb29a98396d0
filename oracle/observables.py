"""Expectation values from the factor only (Sec. 3.6, eq. 3.6).

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


# ---- two-spin reduced density matrix and entanglement (Sec. 3.6) -----------
#
# R_kl = Tr_rest(rho) for the spins at sites k and l, indexed by
# q = 2 b_k + b_l (b the bit of the site in the basis index; 0 = spin up):
# R[q, q'] = sum_a lambda_a sum_{other bits} v_a(b_k, b_l, rest)
#            conj(v_a(b_k', b_l', rest)).  The paper then takes nonlinear
# measures of this 4 x 4 matrix: concurrence (Wootters 1998), negativity
# (Vidal & Werner 2002) and the CHSH nonlocality measure (Horodecki 1995).

def pair_density(V, lam0, n, k, l):
    """R_kl (4 x 4) by the partial trace, written out on the state tensor."""
    V = np.asarray(V, dtype=np.complex128)
    r = V.shape[1]
    # index x = sum_i b_i 2^i: as a C-ordered tensor the axes are bits n-1 .. 0
    T = V.reshape((2,) * n + (r,))
    ak, al = n - 1 - k, n - 1 - l
    rest = [ax for ax in range(n) if ax not in (ak, al)]
    Tm = np.moveaxis(T, [ak, al] + rest, list(range(n)))   # (b_k, b_l, rest..., a)
    M = Tm.reshape(4, -1, r)                               # q = 2 b_k + b_l
    return np.einsum('pxa,qxa,a->pq', M, M.conj(), np.asarray(lam0, dtype=np.float64))


def _sy2():
    sy = np.array([[0, -1j], [1j, 0]])
    return np.kron(sy, sy)


def concurrence(R):
    """max(0, l1 - l2 - l3 - l4), l_i the square roots of the eigenvalues of
    R (sy x sy) conj(R) (sy x sy), descending."""
    Rt = _sy2() @ np.conj(R) @ _sy2()
    mu = np.linalg.eigvals(R @ Rt)
    l = np.sort(np.sqrt(np.clip(mu.real, 0, None)))[::-1]
    return max(0.0, l[0] - l[1] - l[2] - l[3])


def partial_transpose(R):
    """Transpose on the second spin: R^{T_l}[(i j), (i' j')] = R[(i j'), (i' j)]."""
    X = np.asarray(R).reshape(2, 2, 2, 2)
    return X.transpose(0, 3, 2, 1).reshape(4, 4)


def negativity(R):
    """Sum of |negative eigenvalues| of the partial transpose, (|R^T_l|_1 - 1) / 2."""
    w = np.linalg.eigvalsh(partial_transpose(R))
    return float(-np.sum(w[w < 0]))


def chsh_max(R):
    """Largest CHSH expectation over measurement settings, 2 sqrt(m1 + m2) with
    m1, m2 the two largest eigenvalues of T^T T, T_ij = Tr(R s_i x s_j)."""
    s = [np.array([[0, 1], [1, 0]]), np.array([[0, -1j], [1j, 0]]), np.array([[1, 0], [0, -1]])]
    T = np.array([[np.real(np.trace(R @ np.kron(a, b))) for b in s] for a in s])
    m = np.sort(np.linalg.eigvalsh(T.T @ T))[::-1]
    return 2.0 * np.sqrt(m[0] + m[1])
