"""CPU pin of the full-rank (Werner) reduction of Sec. 5 (a full-rank
state): for rho_W = p I / N + (1 - p) rho_hat, the solution of q-LL or q-LLG
from rho_W is p I / N + (1 - p) rho_hat(t), with rho_hat solving the same
equation with damping (1 - p) kappa.  Checked on dense matrices with a plain
RK4 step of the ODE, which maps that affine family into itself exactly, and
on the right-hand sides."""
import numpy as np
import pytest

from oracle.dense import rk4_plain, rhs_qll, rhs_qllg_eig
from oracle.hamiltonian import Hamiltonian
from workloads import chain_bonds


def _setup(n, seed):
    rng = np.random.default_rng(seed)
    bonds = chain_bonds(n, periodic=False)
    J = rng.normal(size=(bonds.shape[0], 3, 3)) * 0.5
    h = rng.normal(size=(n, 3)) * 0.5
    H = Hamiltonian(n, bonds, J, h).dense()
    N = 2 ** n
    A = rng.normal(size=(N, 2)) + 1j * rng.normal(size=(N, 2))
    rho_hat = A @ A.conj().T
    rho_hat /= np.trace(rho_hat).real
    return H, rho_hat, N


@pytest.mark.parametrize("model", ["qLL", "qLLG"])
@pytest.mark.parametrize("p", [0.1, 0.5, 0.9])
def test_werner_step_equals_shifted_low_rank_step(model, p):
    n, kappa, h = 4, 0.4, 0.02
    H, rho_hat, N = _setup(n, 3)
    rho_w = p * np.eye(N) / N + (1 - p) * rho_hat
    full = rho_w
    low = rho_hat
    for _ in range(3):
        full = rk4_plain(full, H, model, kappa, h)
        low = rk4_plain(low, H, model, (1 - p) * kappa, h)
    assert np.abs(full - (p * np.eye(N) / N + (1 - p) * low)).max() < 1e-13


@pytest.mark.parametrize("model", ["qLL", "qLLG"])
def test_werner_rhs_scales(model):
    n, kappa, p = 3, 0.7, 0.35
    H, rho_hat, N = _setup(n, 4)
    rho_w = p * np.eye(N) / N + (1 - p) * rho_hat

    def f(R, k):
        if model == "qLL":
            return rhs_qll(R, H, k)
        w, U = np.linalg.eigh(0.5 * (R + R.conj().T))
        return rhs_qllg_eig(U, w, H, k)

    assert np.abs(f(rho_w, kappa) - (1 - p) * f(rho_hat, (1 - p) * kappa)).max() < 1e-13
    # the identity part is traceless against every Pauli-string observable
    assert abs(np.trace(H)) < 1e-12
