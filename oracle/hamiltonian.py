"""Spin Hamiltonian of Sec. 5, eq. (5.1), applied without forming a matrix.

Pauli form: H = sum_{(i,j)} 1/2 sum_{a,b} J_ij^{ab} s^a_i s^b_j + 1/2 sum_i h_i . s_i.
With S = (hbar/2) s (eq. 3.5) this is eq. (5.1) term by term:
(2J/hbar^2) S_i.S_j = (J/2) s_i.s_j, (2/hbar^2) d.(S_i x S_j) = (1/2) d.(s_i x s_j)
and -mu b.S_i = (g mu_B / 2) b.s_i, i.e. h = g mu_B b.  hbar does not enter H.

Basis: site i is bit i of the row index; bit 0 means s^z = +1.
"""
import numpy as np

# Pauli matrices in the basis (|0> = up, |1> = down).
SX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
SY = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
SZ = np.array([[1, 0], [0, -1]], dtype=np.complex128)
PAULI = (SX, SY, SZ)


def _bits(N, site):
    return (np.arange(N, dtype=np.int64) >> site) & 1


def apply_pauli(V, site, a):
    """Rows of s^a_site @ V for a factor V of shape (N, r) (a = 0, 1, 2 for x, y, z).

    (s^a V)[x] = sum_{b'} s^a[b(x), b'] V[x with bit site set to b'].
    """
    N = V.shape[0]
    b = _bits(N, site)
    if a == 2:
        return (1 - 2 * b)[:, None] * V
    partner = np.arange(N, dtype=np.int64) ^ (1 << site)
    if a == 0:
        return V[partner]
    # s^y[0,1] = -i, s^y[1,0] = +i
    phase = np.where(b == 0, -1j, 1j)
    return phase[:, None] * V[partner]


def apply_H(n, bonds, J, h, V):
    """Y = H V for the Pauli-form Hamiltonian; V has shape (N, r), N = 2^n."""
    V = np.asarray(V, dtype=np.complex128)
    assert V.shape[0] == 2 ** n
    Y = np.zeros_like(V)
    for k, (i, j) in enumerate(np.asarray(bonds).reshape(-1, 2)):
        Jk = np.asarray(J[k], dtype=np.float64)
        for b in range(3):
            Vb = None
            for a in range(3):
                c = Jk[a, b]
                if c == 0.0:
                    continue
                if Vb is None:
                    Vb = apply_pauli(V, int(j), b)
                Y += 0.5 * c * apply_pauli(Vb, int(i), a)
    if h is not None:
        h = np.asarray(h, dtype=np.float64).reshape(n, 3)
        for i in range(n):
            for a in range(3):
                if h[i, a] != 0.0:
                    Y += 0.5 * h[i, a] * apply_pauli(V, i, a)
    return Y


def site_operator(n, site, M):
    """The 2^n x 2^n matrix of a one-site operator M on `site` (eq. 3.5).

    np.kron puts its left factor on the most significant bits, so site i
    (bit i) sits at Kronecker position n-1-i counted from the left.
    """
    left = np.eye(2 ** (n - 1 - site))
    right = np.eye(2 ** site)
    return np.kron(np.kron(left, M), right)


def dense_H(n, bonds, J, h):
    """Dense Hamiltonian from Kronecker products (small n only)."""
    assert n <= 12
    N = 2 ** n
    H = np.zeros((N, N), dtype=np.complex128)
    for k, (i, j) in enumerate(np.asarray(bonds).reshape(-1, 2)):
        for a in range(3):
            for b in range(3):
                c = J[k][a][b]
                if c != 0.0:
                    H += 0.5 * c * site_operator(n, int(i), PAULI[a]) @ site_operator(n, int(j), PAULI[b])
    if h is not None:
        h = np.asarray(h, dtype=np.float64).reshape(n, 3)
        for i in range(n):
            for a in range(3):
                if h[i, a] != 0.0:
                    H += 0.5 * h[i, a] * site_operator(n, i, PAULI[a])
    return H


def spin_operator(n, site, a, hbar=1.0):
    """S^a_site = (hbar/2) s^a as a dense matrix (eq. 3.5)."""
    return 0.5 * hbar * site_operator(n, site, PAULI[a])


def apply_H_rows(n, bonds, J, h, V, rows):
    """Rows `rows` of H V only, from the same Pauli strings (for spot checks at large n).

    For each Pauli string the destination row x couples to the single source
    row x ^ flip, with the phase of s^a_i s^b_j evaluated at the bits of x.
    """
    rows = np.asarray(rows, dtype=np.int64)
    V = np.asarray(V)
    out = np.zeros((rows.size, V.shape[1]), dtype=np.complex128)

    def elem(a, b):  # <b| s^a |b'> for the source bit b' implied by the flip
        if a == 0:
            return np.ones_like(b, dtype=np.complex128)
        if a == 1:
            return np.where(b == 0, -1j, 1j)
        return (1 - 2 * b).astype(np.complex128)

    def bit(x, s):
        return (x >> s) & 1

    for k, (i, j) in enumerate(np.asarray(bonds).reshape(-1, 2)):
        i, j = int(i), int(j)
        for a in range(3):
            for b in range(3):
                c = J[k][a][b]
                if c == 0.0:
                    continue
                flip = (0 if a == 2 else 1 << i) | (0 if b == 2 else 1 << j)
                ph = elem(a, bit(rows, i)) * elem(b, bit(rows, j))
                out += 0.5 * c * ph[:, None] * V[rows ^ flip]
    if h is not None:
        h = np.asarray(h, dtype=np.float64).reshape(n, 3)
        for i in range(n):
            for a in range(3):
                if h[i, a] != 0.0:
                    flip = 0 if a == 2 else 1 << i
                    out += 0.5 * h[i, a] * elem(a, bit(rows, i))[:, None] * V[rows ^ flip]
    return out


class Hamiltonian:
    """Bundle of the Hamiltonian description with a matrix-free apply."""

    def __init__(self, n, bonds, J, h):
        self.n = int(n)
        self.N = 2 ** self.n
        self.bonds = np.asarray(bonds, dtype=np.int64).reshape(-1, 2)
        self.J = np.asarray(J, dtype=np.float64).reshape(-1, 3, 3)
        self.h = None if h is None else np.asarray(h, dtype=np.float64).reshape(self.n, 3)

    def apply(self, V):
        return apply_H(self.n, self.bonds, self.J, self.h, V)

    def dense(self):
        return dense_H(self.n, self.bonds, self.J, self.h)
