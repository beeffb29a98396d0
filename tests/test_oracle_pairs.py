"""CPU pins of the two-spin reduced density matrix and its entanglement
measures (oracle/observables.py, Sec. 3.6): brute-force partial trace of the
dense density matrix, product states, the singlet, Werner states (closed
forms of concurrence and negativity) and Tsirelson's bound."""
import numpy as np
import pytest

from oracle.observables import pair_density, concurrence, negativity, partial_transpose, chsh_max


def _rand_state(n, r, rng):
    Q, _ = np.linalg.qr(rng.normal(size=(2 ** n, r)) + 1j * rng.normal(size=(2 ** n, r)))
    lam = np.sort(rng.dirichlet(np.ones(r)))[::-1]
    return Q, lam


@pytest.mark.parametrize("n,k,l", [(3, 0, 1), (3, 2, 0), (4, 1, 3), (5, 4, 2), (2, 1, 0)])
def test_partial_trace_matches_dense_brute_force(n, k, l):
    rng = np.random.default_rng(10 * n + k)
    V, lam = _rand_state(n, 3, rng)
    rho = (V * lam) @ V.conj().T
    N = 2 ** n
    R = np.zeros((4, 4), complex)
    for x in range(N):
        for y in range(N):
            same_rest = all(((x >> i) & 1) == ((y >> i) & 1) for i in range(n) if i not in (k, l))
            if not same_rest:
                continue
            p = 2 * ((x >> k) & 1) + ((x >> l) & 1)
            q = 2 * ((y >> k) & 1) + ((y >> l) & 1)
            R[p, q] += rho[x, y]
    assert np.abs(pair_density(V, lam, n, k, l) - R).max() < 1e-14
    assert abs(np.trace(R) - 1) < 1e-14 and np.abs(R - R.conj().T).max() < 1e-15
    assert np.linalg.eigvalsh(R).min() > -1e-14


def test_product_state_gives_product_matrix():
    rng = np.random.default_rng(1)
    n = 4
    singles = []
    psi = np.ones(1)
    for i in range(n):  # site i is bit i: kron builds bit n-1 .. 0, so prepend
        s = rng.normal(size=2) + 1j * rng.normal(size=2)
        s /= np.linalg.norm(s)
        singles.append(s)
    for i in reversed(range(n)):
        psi = np.kron(psi, singles[i])
    R = pair_density(psi[:, None], [1.0], n, 1, 3)
    rk = np.outer(singles[1], singles[1].conj())
    rl = np.outer(singles[3], singles[3].conj())
    assert np.abs(R - np.kron(rk, rl)).max() < 1e-14
    assert concurrence(R) < 1e-7 and negativity(R) < 1e-14


def _singlet_on(n, k, l):
    psi = np.zeros(2 ** n, complex)
    psi[1 << l] = 1 / np.sqrt(2)       # b_k = 0, b_l = 1
    psi[1 << k] = -1 / np.sqrt(2)      # b_k = 1, b_l = 0
    return psi


def test_singlet_is_maximally_entangled():
    n, k, l = 3, 0, 2
    R = pair_density(_singlet_on(n, k, l)[:, None], [1.0], n, k, l)
    s = np.array([0, 1, -1, 0]) / np.sqrt(2)
    assert np.abs(R - np.outer(s, s)).max() < 1e-15
    assert abs(concurrence(R) - 1.0) < 1e-12
    assert abs(negativity(R) - 0.5) < 1e-12
    assert abs(chsh_max(R) - 2 * np.sqrt(2)) < 1e-12   # Tsirelson's bound


@pytest.mark.parametrize("p", [0.0, 0.2, 1 / 3, 0.5, 0.8, 1.0])
def test_werner_states(p):
    """p |singlet><singlet| + (1 - p) I/4: C = max(0, (3p - 1)/2),
    N = max(0, (3p - 1)/4), CHSH = 2 sqrt(2) p."""
    s = np.array([0, 1, -1, 0]) / np.sqrt(2)
    R = p * np.outer(s, s) + (1 - p) * np.eye(4) / 4
    assert abs(concurrence(R) - max(0.0, (3 * p - 1) / 2)) < 1e-7
    assert abs(negativity(R) - max(0.0, (3 * p - 1) / 4)) < 1e-12
    assert abs(chsh_max(R) - 2 * np.sqrt(2) * p) < 1e-12


def test_partial_transpose_definition():
    rng = np.random.default_rng(2)
    A = rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2))
    B = rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2))
    assert np.abs(partial_transpose(np.kron(A, B)) - np.kron(A, B.T)).max() < 1e-15
