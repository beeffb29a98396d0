"""The benchmark workloads as seeded synthetic problem instances.

Each config is a dict with the Hamiltonian (n, bonds, J tensors, fields), the
initial state (lambda, V), the model, damping, scheme, step size and step
count.  ``make_config(k, n=..., r=...)`` lets tests draw the same family at a
smaller size.

Seeds: config k, trajectory t uses ``PCG64(2508_21200 + 1000*k + t)``.
"""
import numpy as np

from .lattices import (chain_bonds, square_lattice_bonds, heisenberg_tensors, xxz_tensors,
                       uniform_field, random_fields)
from .states import dirichlet_spectrum, haar_factor

BASE_SEED = 2508_21200

CONFIGS = {
    1: dict(name="qLL_heisenberg_chain_n8_r4_rk4", model="qLL", n=8, r=4, kappa=0.1,
            scheme="RK4", dt=0.01, steps=100, precision="fp64"),
    2: dict(name="qLLG_xxz_chain_n16_r8_ab3", model="qLLG", n=16, r=8, kappa=0.05,
            scheme="AB3", dt=0.005, steps=50, precision="fp64+mixed"),
    3: dict(name="qLL_heisenberg_square4x5_n20_r16_rk4", model="qLL", n=20, r=16, kappa=0.5,
            scheme="RK4", dt=0.01, steps=20, precision="mixed"),
    4: dict(name="batched64_xxz_chains_n12-16_rk4", model="mixed", n=None, r=None, kappa=None,
            scheme="RK4", dt=0.01, steps=50, precision="mixed", n_traj=64),
    5: dict(name="qLLG_xxz_chain_n22_r16_rk4", model="qLLG", n=22, r=16, kappa=0.05,
            scheme="RK4", dt=0.01, steps=10, precision="mixed"),
}


def config_rng(k, traj=0):
    return np.random.Generator(np.random.PCG64(BASE_SEED + 1000 * k + traj))


def _xxz_chain(n, rng):
    bonds = chain_bonds(n, periodic=False)
    nb = bonds.shape[0]
    jxy = rng.uniform(0.5, 1.5, size=nb)
    jz = rng.uniform(0.5, 1.5, size=nb)
    J = xxz_tensors(jxy, jz)
    h = random_fields(n, 0.3, rng)
    return bonds, J, h


def make_config(k, traj=0, n=None, r=None, with_state=True):
    """Instantiate config k (optionally at another n / r) with its seeded inputs."""
    rng = config_rng(k, traj)
    base = dict(CONFIGS[k])
    out = dict(base)
    if k == 1:
        n = n or 8
        bonds = chain_bonds(n, periodic=False)
        J = heisenberg_tensors(bonds.shape[0], 1.0)
        h = uniform_field(n, (0.0, 0.0, 0.5))
        r = r or 4
    elif k == 2:
        n = n or 16
        bonds, J, h = _xxz_chain(n, rng)
        r = r or 8
    elif k == 3:
        if n is None or n == 20:
            n = 20
            bonds = square_lattice_bonds(4, 5, periodic=True)
        else:
            # a smaller periodic lattice of the same family (rows x cols = n)
            rows = 2 if n < 9 else 3 if n < 16 else 4
            cols = max(3, n // rows)
            n = rows * cols
            bonds = square_lattice_bonds(rows, cols, periodic=True)
        J = heisenberg_tensors(bonds.shape[0], rng.uniform(0.8, 1.2, size=bonds.shape[0]))
        h = uniform_field(n, (0.0, 0.0, 1.0))
        r = r or 16
    elif k == 4:
        n = n or int(rng.integers(12, 17))
        r = r or int(rng.choice([4, 8, 16]))
        bonds, J, h = _xxz_chain(n, rng)
        out["kappa"] = float(np.exp(rng.uniform(np.log(0.01), np.log(1.0))))
        out["model"] = "qLL" if traj % 2 == 0 else "qLLG"
    elif k == 5:
        n = n or 22
        bonds, J, h = _xxz_chain(n, rng)
        r = r or 16
    else:
        raise ValueError(f"unknown config {k}")
    out.update(n=n, r=r, bonds=bonds, J=J, h=h)
    if with_state:
        out["lam"] = dirichlet_spectrum(r, rng)
        out["V"] = haar_factor(2 ** n, r, rng)
    return out
