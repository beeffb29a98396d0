"""The C ABI's host-side entanglement measures (lrei_pair_entanglement)
against the oracle's definitions on random two-spin density matrices, the
singlet, Werner states and product states.  Host code only: runs without a
GPU."""
import numpy as np
import pytest

from oracle.observables import concurrence, negativity, chsh_max


def _lib():
    from paper_2508_21200_amd import pair_entanglement
    return pair_entanglement


@pytest.mark.parametrize("seed", range(8))
def test_random_density_matrices(seed):
    ent = _lib()
    rng = np.random.default_rng(seed)
    rank = 1 + seed % 4
    A = rng.normal(size=(4, rank)) + 1j * rng.normal(size=(4, rank))
    R = A @ A.conj().T
    R /= np.trace(R).real
    c, n, b = ent(R)
    assert abs(c - concurrence(R)) < 1e-7
    assert abs(n - negativity(R)) < 1e-12
    assert abs(b - chsh_max(R)) < 1e-12


@pytest.mark.parametrize("p", [0.0, 0.3, 1 / 3, 0.6, 1.0])
def test_werner_closed_forms(p):
    ent = _lib()
    s = np.array([0, 1, -1, 0]) / np.sqrt(2)
    R = p * np.outer(s, s) + (1 - p) * np.eye(4) / 4
    c, n, b = ent(R)
    assert abs(c - max(0.0, (3 * p - 1) / 2)) < 1e-7
    assert abs(n - max(0.0, (3 * p - 1) / 4)) < 1e-12
    assert abs(b - 2 * np.sqrt(2) * p) < 1e-12


def test_product_state_and_errors():
    from paper_2508_21200_amd import LreiError
    ent = _lib()
    a = np.array([0.6, 0.8j])
    b = np.array([1.0, 1.0]) / np.sqrt(2)
    R = np.kron(np.outer(a, a.conj()), np.outer(b, b.conj()))
    c, n, bell = ent(R)
    assert c < 1e-7 and n < 1e-14 and bell <= 2.0 + 1e-12
    bad = R.copy()
    bad[0, 0] = np.nan
    with pytest.raises(LreiError):
        ent(bad)
