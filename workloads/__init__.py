"""Seeded synthetic inputs for LREI runs.

This module generates *inputs only*: lattices (bond lists), exchange tensors,
site fields, spectra and orthonormal factors.  It contains none of the LREI
method's arithmetic (no right-hand side, no stage combination, no
eigensolve), so both the CPU oracle and the GPU path may use it.

Conventions (shared by every consumer):

* Hamiltonian in Pauli form,
  ``H = sum_bonds 1/2 sum_ab J[a][b] s^a_i s^b_j + 1/2 sum_i h_i . s_i``,
  which equals the spin Hamiltonian of Sec. 5, eq. (5.1), with S = hbar*s/2,
  J^{ab} = J delta_ab + eps_abc d_c and h = g mu_B b.
* Site i is bit i of the basis index (least significant bit = site 0).
  Bit value 0 is spin up (s^z = +1).  The paper's Kronecker convention
  (Sec. 3.6, eq. (3.5), site 1 leftmost) is the same basis up to this
  relabelling.
* A factor V is an (N, r) complex array, row-major: the r columns of one
  basis state are contiguous.
"""
from .lattices import (chain_bonds, square_lattice_bonds, triangular_lattice_bonds,
                       heisenberg_tensors, xxz_tensors, dmi_tensor_z, uniform_field,
                       random_fields)
from .states import (dirichlet_spectrum, haar_factor, basis_state_index, af1_index,
                     af2_index, ghz_vector, w_vector, pure_factor, mixture_factor)
from .configs import CONFIGS, config_rng, make_config

__all__ = [
    "chain_bonds", "square_lattice_bonds", "triangular_lattice_bonds",
    "heisenberg_tensors", "xxz_tensors", "dmi_tensor_z", "uniform_field", "random_fields",
    "dirichlet_spectrum", "haar_factor", "basis_state_index", "af1_index", "af2_index",
    "ghz_vector", "w_vector", "pure_factor", "mixture_factor",
    "CONFIGS", "config_rng", "make_config",
]
