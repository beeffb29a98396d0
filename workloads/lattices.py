"""Bond lists, exchange tensors and site fields (inputs only)."""
import numpy as np


def chain_bonds(n, periodic=False):
    """Nearest-neighbour bonds (i, i+1) of an n-site chain; site i is bit i."""
    bonds = [(i, i + 1) for i in range(n - 1)]
    if periodic and n > 2:
        bonds.append((0, n - 1))
    return np.asarray(bonds, dtype=np.int32).reshape(-1, 2)


def square_lattice_bonds(rows, cols, periodic=True):
    """Nearest-neighbour bonds of a rows x cols square lattice.

    Site (x, y) (column x, row y) is bit cols*y + x (row-major).  With periodic
    boundaries every site has four bonds (rows, cols >= 3), e.g. 40 bonds for
    the 4 x 5 torus.
    """
    def site(x, y):
        return cols * y + x

    bonds = set()
    for y in range(rows):
        for x in range(cols):
            for dx, dy in ((1, 0), (0, 1)):
                xx, yy = x + dx, y + dy
                if xx >= cols or yy >= rows:
                    if not periodic:
                        continue
                    xx %= cols
                    yy %= rows
                a, b = site(x, y), site(xx, yy)
                if a == b:
                    continue
                bonds.add((min(a, b), max(a, b)))
    return np.asarray(sorted(bonds), dtype=np.int32).reshape(-1, 2)


def triangular_lattice_bonds(rows, cols, periodic=False):
    """Bonds of a triangular lattice built from a square grid plus one diagonal.

    Site (x, y) is bit cols*y + x.  Each site couples to (x+1, y), (x, y+1) and
    (x+1, y+1).  The paper's own cluster adjacency is not published; this is a
    synthetic stand-in of the same family.
    """
    def site(x, y):
        return cols * y + x

    bonds = set()
    for y in range(rows):
        for x in range(cols):
            for dx, dy in ((1, 0), (0, 1), (1, 1)):
                xx, yy = x + dx, y + dy
                if xx >= cols or yy >= rows:
                    if not periodic:
                        continue
                    xx %= cols
                    yy %= rows
                a, b = site(x, y), site(xx, yy)
                if a == b:
                    continue
                bonds.add((min(a, b), max(a, b)))
    return np.asarray(sorted(bonds), dtype=np.int32).reshape(-1, 2)


def heisenberg_tensors(n_bonds, J):
    """Isotropic exchange J * identity per bond; J may be a scalar or an array."""
    J = np.broadcast_to(np.asarray(J, dtype=np.float64), (n_bonds,))
    T = np.zeros((n_bonds, 3, 3))
    for a in range(3):
        T[:, a, a] = J
    return T


def xxz_tensors(jxy, jz):
    """XXZ exchange diag(Jxy, Jxy, Jz) per bond."""
    jxy = np.asarray(jxy, dtype=np.float64).reshape(-1)
    jz = np.asarray(jz, dtype=np.float64).reshape(-1)
    T = np.zeros((jxy.size, 3, 3))
    T[:, 0, 0] = jxy
    T[:, 1, 1] = jxy
    T[:, 2, 2] = jz
    return T


def dmi_tensor_z(J, d):
    """Exchange tensor of isotropic J plus a DMI vector d along z.

    In Pauli form the bond term is 1/2 [J s_i.s_j + d (s_i x s_j)_z], so the
    tensor has J on the diagonal and +d at (x, y), -d at (y, x).
    """
    T = np.diag([J, J, J]).astype(np.float64)
    T[0, 1] = d
    T[1, 0] = -d
    return T


def uniform_field(n, h):
    """The same field vector h (length 3) on every site."""
    return np.tile(np.asarray(h, dtype=np.float64).reshape(1, 3), (n, 1))


def random_fields(n, sigma, rng):
    """Independent N(0, sigma^2) field components on every site and axis."""
    return rng.normal(0.0, sigma, size=(n, 3))
