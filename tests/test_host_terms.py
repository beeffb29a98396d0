"""CPU checks of host-side logic: the Hamiltonian term table (Pauli form of
eq. 5.1) against the oracle, and the exported C ABI of liblrei.so."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from oracle.hamiltonian import apply_H, dense_H
from workloads import chain_bonds, square_lattice_bonds, haar_factor, make_config

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2508_21200_amd", "liblrei.so")


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    out = tmp_path_factory.mktemp("h") / "libterms.so"
    src = [os.path.join(ROOT, "tests", "host", "terms_apply.cpp"),
           os.path.join(ROOT, "paper_2508_21200_amd", "csrc", "terms.cpp"),
           os.path.join(ROOT, "paper_2508_21200_amd", "csrc", "site_order.cpp")]
    cmd = ["/opt/rocm/bin/hipcc", "-x", "c++", "-O1", "-std=c++17", "-fPIC", "-shared",
           "-I" + os.path.join(ROOT, "include"), "-I/opt/rocm/include",
           "-D__HIP_PLATFORM_AMD__"] + src + ["-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True)
    lib = ctypes.CDLL(str(out))
    lib.terms_apply.restype = ctypes.c_int
    return lib


def _apply(lib, n, bonds, J, h, V):
    bonds = np.ascontiguousarray(bonds, dtype=np.int32)
    J = np.ascontiguousarray(J, dtype=np.float64)
    hh = None if h is None else np.ascontiguousarray(h, dtype=np.float64)
    V = np.ascontiguousarray(V, dtype=np.complex128)
    Y = np.zeros_like(V)
    bound = ctypes.c_double()
    st = lib.terms_apply(n, bonds.shape[0], bonds.ctypes.data_as(ctypes.c_void_p),
                         J.ctypes.data_as(ctypes.c_void_p),
                         None if hh is None else hh.ctypes.data_as(ctypes.c_void_p),
                         V.shape[1], V.ctypes.data_as(ctypes.c_void_p), Y.ctypes.data_as(ctypes.c_void_p),
                         ctypes.byref(bound))
    assert st == 0
    return Y, bound.value


@pytest.mark.parametrize("n", [2, 4, 7])
def test_term_table_general_tensors(harness, n):
    rng = np.random.default_rng(n)
    bonds = chain_bonds(n, periodic=n > 2)
    J = rng.normal(size=(bonds.shape[0], 3, 3))
    h = rng.normal(size=(n, 3))
    V = haar_factor(2 ** n, 3, rng)
    Y, bound = _apply(harness, n, bonds, J, h, V)
    np.testing.assert_allclose(Y, apply_H(n, bonds, J, h, V), atol=1e-13)
    # Gershgorin bound really bounds the spectrum
    w = np.linalg.eigvalsh(dense_H(n, bonds, J, h))
    assert np.abs(w).max() <= bound + 1e-12


@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_term_table_benchmark_families(harness, k):
    cfg = make_config(k, n=8 if k != 3 else 9, r=2)
    V = cfg["V"]
    Y, _ = _apply(harness, cfg["n"], cfg["bonds"], cfg["J"], cfg["h"], V)
    np.testing.assert_allclose(Y, apply_H(cfg["n"], cfg["bonds"], cfg["J"], cfg["h"], V), atol=1e-13)


@pytest.mark.parametrize("case", ["general", "heisenberg_lattice", "xxz_fields", "repeated_bond"])
def test_term_table_spread_is_frobenius(harness, case):
    """The scale of the Krylov recurrence, sqrt(Tr(H^2) / N), against the
    Frobenius norm of the dense Kronecker Hamiltonian (a repeated bond and
    one-site x, y, z fields included)."""
    rng = np.random.default_rng(7)
    if case == "general":
        n = 6
        bonds = chain_bonds(n, periodic=True)
        J = rng.normal(size=(bonds.shape[0], 3, 3))
        h = rng.normal(size=(n, 3))
    elif case == "repeated_bond":
        n = 5
        bonds = np.concatenate([chain_bonds(n, periodic=False), [[0, 1], [1, 3]]]).astype(np.int32)
        J = rng.normal(size=(bonds.shape[0], 3, 3))
        h = rng.normal(size=(n, 3))
    else:
        cfg = make_config(3 if case == "heisenberg_lattice" else 2, n=9, r=1, with_state=False)
        n, bonds, J, h = cfg["n"], cfg["bonds"], cfg["J"], cfg["h"]
    bonds = np.ascontiguousarray(bonds, dtype=np.int32)
    Jc = np.ascontiguousarray(J, dtype=np.float64)
    hc = None if h is None else np.ascontiguousarray(h, dtype=np.float64)
    sp = ctypes.c_double()
    assert harness.terms_spread(n, bonds.shape[0], bonds.ctypes.data_as(ctypes.c_void_p),
                                Jc.ctypes.data_as(ctypes.c_void_p),
                                None if hc is None else hc.ctypes.data_as(ctypes.c_void_p), ctypes.byref(sp)) == 0
    Hd = dense_H(n, bonds, J, h)
    assert abs(sp.value - np.linalg.norm(Hd) / np.sqrt(2 ** n)) < 1e-12 * sp.value


@pytest.mark.parametrize("case", ["square4x5", "square4x4", "chain16", "triangular3x4"])
def test_cluster_site_order(harness, case):
    """The tiled pass's site order is a permutation whose first k = 10 sites
    hold as many bonds as the best k-subset (brute force over all of them for
    these sizes), and every prefix is a connected-first growth (each prefix
    site after the first has a bond into the earlier ones, where possible)."""
    import itertools
    from workloads import triangular_lattice_bonds
    if case == "square4x5":
        bonds = square_lattice_bonds(4, 5, periodic=True)
    elif case == "square4x4":
        bonds = square_lattice_bonds(4, 4, periodic=True)
    elif case == "chain16":
        bonds = chain_bonds(16, periodic=False)
    else:
        bonds = triangular_lattice_bonds(3, 4, periodic=True)
    bonds = np.ascontiguousarray(bonds, dtype=np.int32)
    n = int(bonds.max()) + 1
    k = 10
    pos = np.zeros(n, dtype=np.int32)
    harness.site_order_cluster(n, bonds.shape[0], bonds.ctypes.data_as(ctypes.c_void_p), k,
                               pos.ctypes.data_as(ctypes.c_void_p))
    assert sorted(pos.tolist()) == list(range(n))
    low = {q for q in range(n) if pos[q] < k}
    inside = sum(1 for i, j in bonds if i in low and j in low)
    best = max(sum(1 for i, j in bonds if i in S and j in S) for S in map(set, itertools.combinations(range(n), k)))
    assert inside == best
    if case == "square4x5":
        assert best == 15  # two neighbouring rows of the torus


def test_library_exports_every_declared_symbol():
    header = open(os.path.join(ROOT, "include", "lrei.h")).read()
    declared = set(re.findall(r"LREI_API\s+[\w\s\*]+?\b(lrei_\w+)\s*\(", header))
    assert len(declared) >= 14
    lib = ctypes.CDLL(LIB)
    for name in declared:
        assert hasattr(lib, name), name
    from paper_2508_21200_amd import lrei
    assert declared == set(lrei.exported_symbols())


def test_create_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    from paper_2508_21200_amd import lrei
    lib = lrei.load()
    h = ctypes.c_void_p()
    st = lib.lrei_create(ctypes.byref(h), 0, None, None)
    assert st == 4 and not h.value  # LREI_E_DEVICE


@pytest.mark.parametrize("name", ["lrei_options", "lrei_stats", "lrei_tune_result", "lrei_batch_tune_result",
                                  "lrei_traj_desc", "lrei_adapt_result"])
def test_binding_structs_match_the_header(name, tmp_path):
    """Every ctypes structure of the binding has the C struct's size and each
    field its offset (a C program built from include/lrei.h prints them)."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    from paper_2508_21200_amd import lrei
    cls = getattr(lrei, name)
    fields = [f[0] for f in cls._fields_]
    cname = {"lambda_": "lambda"}
    src = ['#include <stdio.h>', '#include <stddef.h>', '#include "lrei.h"', "int main(void) {",
           f'  printf("%zu\\n", sizeof({name}));']
    src += [f'  printf("%zu\\n", offsetof({name}, {cname.get(f, f)}));' for f in fields]
    src += ["  return 0;", "}"]
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert vals[0] == ctypes.sizeof(cls), (name, vals[0], ctypes.sizeof(cls))
    for f, off in zip(fields, vals[1:]):
        assert getattr(cls, f).offset == off, (name, f)
