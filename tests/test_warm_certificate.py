"""CPU checks of the mathematics the projected eigensolve relies on.

* The warm-started eigensolve accepts a subspace X (orthonormal, m x r) of the
  Hermitian stage matrix K only if the Gershgorin lower bound of G = X* K X,
  minus |Res| (Res = K X - X G), exceeds T + |Res|, where
  T^2 = |K|_F^2 - |G|_F^2 - 2 |Res|_F^2.  The claim behind it: every
  eigenvalue of K other than the r nearest G's spectrum lies within T + |Res|
  of zero, so a passing certificate means X carries the r largest eigenvalues.
  Checked here on random Hermitian matrices with a planted top-r block, for
  subspaces at several distances from the true one, against numpy's eigh.
* The Lowdin step uses S^{-1/2} = I - E/2 + 3/8 E^2 - 5/16 E^3 for S = I + E,
  |E| <= 1e-6 entrywise; checked against the eigendecomposition.
"""
import numpy as np
import pytest


def _planted(m, r, rng, tail):
    """Hermitian K with r eigenvalues in [0.05, 1] and m - r of size <= tail."""
    Q, _ = np.linalg.qr(rng.normal(size=(m, m)) + 1j * rng.normal(size=(m, m)))
    top = np.sort(rng.uniform(0.05, 1.0, size=r))[::-1]
    rest = rng.uniform(-tail, tail, size=m - r)
    w = np.concatenate([top, rest])
    return (Q * w) @ Q.conj().T, Q[:, :r], w


def _certificate(K, X):
    G = X.conj().T @ K @ X
    G = 0.5 * (G + G.conj().T)
    Res = K @ X - X @ G
    res = np.linalg.norm(Res)
    T = np.sqrt(max(np.linalg.norm(K) ** 2 - np.linalg.norm(G) ** 2 - 2 * res ** 2, 0.0))
    off = np.abs(G) - np.diag(np.abs(np.diag(G)))
    lb = np.min(np.real(np.diag(G)) - off.sum(axis=1))
    return G, res, T, lb


@pytest.mark.parametrize("seed", range(12))
@pytest.mark.parametrize("eps", [1e-12, 1e-8, 1e-4, 1e-2])
def test_rest_of_spectrum_is_bounded(seed, eps):
    rng = np.random.default_rng(seed)
    m, r = 48, 8
    K, U, w = _planted(m, r, rng, tail=1e-3)
    # a subspace near the top-r one: rotate within it, then perturb out of it
    Rr, _ = np.linalg.qr(rng.normal(size=(r, r)) + 1j * rng.normal(size=(r, r)))
    X = U @ Rr + eps * (rng.normal(size=(m, r)) + 1j * rng.normal(size=(m, r)))
    X, _ = np.linalg.qr(X)
    G, res, T, lb = _certificate(K, X)
    ev = np.linalg.eigvalsh(K)
    theta = np.linalg.eigvalsh(G)
    # the r eigenvalues of K nearest the Ritz values; the rest must obey the bound
    idx = set()
    for t in theta:
        d = np.abs(ev - t)
        d[list(idx)] = np.inf
        idx.add(int(np.argmin(d)))
    rest = np.delete(ev, sorted(idx))
    assert np.max(np.abs(rest)) <= T + res + 1e-12
    # and a passing certificate really selects the r largest eigenvalues
    if lb - res > T + res:
        assert np.allclose(np.sort(ev)[-r:], np.sort(ev[sorted(idx)]), atol=2 * res + 1e-12)


def test_certificate_rejects_a_wrong_subspace():
    """A subspace that misses one of the top eigenvectors cannot pass."""
    rng = np.random.default_rng(5)
    m, r = 40, 6
    K, U, w = _planted(m, r, rng, tail=1e-3)
    Q, _ = np.linalg.qr(rng.normal(size=(m, m)) + 1j * rng.normal(size=(m, m)))
    evals, evecs = np.linalg.eigh(K)
    order = np.argsort(evals)[::-1]
    X = evecs[:, np.r_[order[: r - 1], order[r + 3]]]  # r-1 top vectors and one from the rest
    G, res, T, lb = _certificate(K, X)
    assert not (lb - res > T + res)


@pytest.mark.parametrize("dev", [1e-14, 1e-10, 1e-7, 1e-6])
def test_lowdin_series(dev):
    rng = np.random.default_rng(3)
    r = 16
    E = rng.normal(size=(r, r)) + 1j * rng.normal(size=(r, r))
    E = 0.5 * (E + E.conj().T)
    E *= dev / np.abs(E).max()
    S = np.eye(r) + E
    w, V = np.linalg.eigh(S)
    exact = (V / np.sqrt(w)) @ V.conj().T
    series = np.eye(r) - E / 2 + 3 / 8 * (E @ E) - 5 / 16 * (E @ E @ E)
    # the truncation (< 1e-19) is far below the rounding of the eigh reference itself
    assert np.abs(series - exact).max() <= 4e-15
    # and the result orthonormalises: (S^-1/2)* S S^-1/2 = I
    assert np.abs(series.conj().T @ S @ series - np.eye(r)).max() <= 1e-15
