"""CPU pins of the initial eigendecomposition from a non-orthogonal factor
(oracle/lowrank.py state_from_factor) against numpy's dense eigh of A A*."""
import numpy as np
import pytest

from oracle.lowrank import state_from_factor


@pytest.mark.parametrize("N,m", [(16, 1), (64, 3), (128, 7)])
def test_matches_dense_eigh(N, m):
    rng = np.random.default_rng(N + m)
    A = rng.normal(size=(N, m)) + 1j * rng.normal(size=(N, m))
    lam, V = state_from_factor(A)
    rho = A @ A.conj().T
    rho /= np.trace(rho).real
    w = np.sort(np.linalg.eigvalsh(rho))[::-1][:m]
    assert np.abs(lam - w).max() < 1e-14
    assert np.abs((V * lam) @ V.conj().T - rho).max() < 1e-14
    assert np.abs(V.conj().T @ V - np.eye(m)).max() < 1e-13
    assert np.all(np.diff(lam) <= 0)


def test_rank_deficient_factor():
    rng = np.random.default_rng(3)
    B = rng.normal(size=(32, 3)) + 1j * rng.normal(size=(32, 3))
    A = np.concatenate([B, B[:, :1] * (2 - 1j)], axis=1)  # 4 columns, rank 3
    lam, V = state_from_factor(A)
    assert lam.size == 3 and abs(lam.sum() - 1) < 1e-14
    rho = A @ A.conj().T
    assert np.abs((V * lam) @ V.conj().T - rho / np.trace(rho).real).max() < 1e-14
