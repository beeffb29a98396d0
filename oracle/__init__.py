"""Plain CPU oracle for LREI (complex128, numpy/scipy).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The product path (the
HIP library and its Python binding) never calls into it, and it shares no code
with that path: the only common module is ``workloads`` (seeded inputs).

What it computes, step by step in the paper's order (arXiv 2508.21200):

* ``hamiltonian``  the spin Hamiltonian of Sec. 5 (eq. 5.1) applied matrix-free
  through Pauli strings (Sec. 3.6, eq. 3.5), plus a dense Kronecker builder for
  small n;
* ``rhs``          the low-rank q-LLG / q-LL right-hand side: X-blocks
  (eq. 3.2 / eq. 4.1), Householder reflectors of the support (eq. 3.3) and
  their action (Sec. 3.4), W, Z and f = Z V* + V W* (eq. 3.4);
* ``lowrank``      the stage matrices in low-rank form (eqs. 3.8, 3.9), the
  matvec g (eq. 3.10) and the partial eigendecomposition (its plain
  definition: the r largest eigenpairs, computed exactly);
* ``schemes``      LREI-RK (Sec. 3.7) and LREI-AB (Sec. 3.8) time steps with
  the spectrum held at Lambda_0;
* ``adaptive``     step-size control from local error estimates (the
  paper's future work, Sec. 6): embedded Heun-Euler 2(1) and
  Bogacki-Shampine 3(2) pairs in LREI form, the tangent-projected error
  estimate and the controller;
* ``observables``  energy and magnetisation (eq. 3.6);
* ``dense``        the dense EI method of Sec. 2 (eqs. 2.1-2.6), the dense
  commutator forms (eqs. 1.1, 1.2) and the pure-state solution (eq. 1.4);
* ``metrics``      a cancellation-free relative Frobenius distance of two
  low-rank density matrices.

Readings of the paper where it is silent or garbled are listed in the
module that takes them.  Every function here is pinned by the CPU tests in
``tests/test_oracle_*.py`` against closed forms, invariants, dense brute force
or library routines; none is marked "parity unpinned".
"""
from . import hamiltonian, rhs, lowrank, schemes, observables, dense, metrics  # noqa: F401
