"""Initial-state inputs: spectra and orthonormal factors (inputs only)."""
import numpy as np


def dirichlet_spectrum(r, rng):
    """A trace-one spectrum drawn from Dirichlet(1,...,1), sorted descending.

    Drawn as E_i ~ Exp(1), lambda = E / sum(E).
    """
    e = rng.exponential(1.0, size=r)
    lam = np.sort(e / e.sum())[::-1].copy()
    return lam


def haar_factor(N, r, rng):
    """An N x r factor with orthonormal columns, Haar distributed.

    QR of a complex Gaussian matrix with the phase of R's diagonal moved into
    Q (Mezzadri 2007), so the distribution does not depend on the QR routine's
    sign convention.
    """
    z = (rng.standard_normal((N, r)) + 1j * rng.standard_normal((N, r))) / np.sqrt(2.0)
    q, rr = np.linalg.qr(z)
    d = np.diag(rr)
    ph = d / np.abs(d)
    return np.ascontiguousarray(q * ph[None, :])


def basis_state_index(bits):
    """Basis index of a product state given per-site bits (site i = bit i)."""
    idx = 0
    for i, b in enumerate(bits):
        idx |= (int(b) & 1) << i
    return idx


def af1_index(n):
    """|AF1>: site 0 up, alternating (Sec. 5.1 footnote, in site-i = bit-i labels)."""
    return basis_state_index([i % 2 for i in range(n)])


def af2_index(n):
    """|AF2>: site 0 down, alternating (the complement of AF1)."""
    return basis_state_index([(i + 1) % 2 for i in range(n)])


def ghz_vector(n):
    """Textbook GHZ state (|0...0> + |1...1>)/sqrt(2)."""
    v = np.zeros(2 ** n, dtype=np.complex128)
    v[0] = v[-1] = 1.0 / np.sqrt(2.0)
    return v


def w_vector(n):
    """Textbook W state: equal superposition of the n single-flip states."""
    v = np.zeros(2 ** n, dtype=np.complex128)
    for i in range(n):
        v[1 << i] = 1.0 / np.sqrt(n)
    return v


def pure_factor(n, index=None, vector=None):
    """An N x 1 factor for a pure state given by a basis index or a vector."""
    N = 2 ** n
    if vector is None:
        vector = np.zeros(N, dtype=np.complex128)
        vector[index] = 1.0
    v = np.asarray(vector, dtype=np.complex128).reshape(N, 1)
    return v / np.linalg.norm(v)


def mixture_factor(vectors, weights):
    """Spectrum and orthonormal factor of sum_k w_k |v_k><v_k| for orthogonal v_k.

    The vectors must be mutually orthogonal (e.g. AF1, AF2, GHZ for n >= 3);
    returns (lambda, V) with lambda sorted descending.
    """
    w = np.asarray(weights, dtype=np.float64)
    order = np.argsort(-w, kind="stable")
    V = np.stack([np.asarray(vectors[k], dtype=np.complex128) / np.linalg.norm(vectors[k])
                  for k in order], axis=1)
    return w[order].copy(), np.ascontiguousarray(V)
