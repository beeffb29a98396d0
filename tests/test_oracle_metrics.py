"""Pins for the stable low-rank distance and the observables (eq. 3.6)."""
import numpy as np

from oracle.metrics import rel_fro_error, dense_rho
from oracle.observables import energy, magnetization
from oracle.hamiltonian import Hamiltonian, spin_operator
from workloads import haar_factor, dirichlet_spectrum, chain_bonds


def test_rel_fro_matches_dense():
    rng = np.random.default_rng(0)
    Va = haar_factor(64, 3, rng)
    Vb = haar_factor(64, 3, rng)
    la, lb = dirichlet_spectrum(3, rng), dirichlet_spectrum(3, rng)
    d = np.linalg.norm(dense_rho(Va, la) - dense_rho(Vb, lb)) / np.linalg.norm(dense_rho(Vb, lb))
    assert abs(rel_fro_error(Va, la, Vb, lb) - d) < 1e-14


def test_rel_fro_resolves_tiny_differences():
    """A 1e-12 rotation is measured to within a few percent (trace formula cannot)."""
    rng = np.random.default_rng(1)
    V = haar_factor(128, 2, rng)
    lam = np.array([0.7, 0.3])
    E = rng.normal(size=V.shape) * 1e-12
    V2 = np.linalg.qr(V + E)[0] * (np.diag(np.linalg.qr(V + E)[1]) / abs(np.diag(np.linalg.qr(V + E)[1])))
    ref = np.linalg.norm(dense_rho(V2, lam) - dense_rho(V, lam)) / np.linalg.norm(lam)
    got = rel_fro_error(V2, lam, V, lam)
    assert ref > 1e-13 and abs(got - ref) / ref < 0.05


def test_observables_match_dense_traces():
    rng = np.random.default_rng(2)
    n = 5
    bonds = chain_bonds(n)
    H = Hamiltonian(n, bonds, rng.normal(size=(bonds.shape[0], 3, 3)), rng.normal(size=(n, 3)))
    V = haar_factor(2 ** n, 3, rng)
    lam = dirichlet_spectrum(3, rng)
    rho = dense_rho(V, lam)
    assert abs(energy(H, V, lam) - np.trace(H.dense() @ rho).real) < 1e-13
    hbar = 0.8
    m = magnetization(n, V, lam, hbar)
    for a in range(3):
        ref = sum(np.trace(spin_operator(n, i, a, hbar) @ rho).real for i in range(n)) / n
        assert abs(m[a] - ref) < 1e-14
