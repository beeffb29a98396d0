"""CPU pins of the learned start rotation's reference (oracle/learned.py).

The reference is checked against things other than itself: the Cayley map
against scipy's matrix exponential and unitarity, the backpropagated gradient
against central finite differences of the loss, Adam's first step against its
closed form, the predictor against the exact eigenvectors of a perturbed
matrix, and the analytic rotation against an exactly invariant subspace.
"""
import numpy as np
import pytest
from scipy.linalg import expm

from oracle import learned as L


def _rand_skew(r, rng, scale):
    o = rng.normal(size=r * r) * scale
    return L.unpack_skew(o, r), o


def test_unpack_is_skew_hermitian_and_pack_is_its_adjoint():
    """unpack_skew is real-linear; pack_skew_grad must be its adjoint:
    Re sum conj(gA) unpack(o) = pack(gA) . o for every o and gA."""
    rng = np.random.default_rng(0)
    for r in (1, 2, 5, 16):
        A, o = _rand_skew(r, rng, 1.0)
        assert np.abs(A + A.conj().T).max() == 0.0
        gA = rng.normal(size=(r, r)) + 1j * rng.normal(size=(r, r))
        lhs = np.sum(np.conj(gA) * A).real
        assert abs(lhs - L.pack_skew_grad(gA, r) @ o) < 1e-12 * max(1.0, abs(lhs))


def test_cayley_unitary_and_second_order():
    rng = np.random.default_rng(1)
    r = 6
    assert np.array_equal(L.cayley(np.zeros((r, r), complex)), np.eye(r))
    for scale in (1.0, 1e-1, 1e-2):
        A, _ = _rand_skew(r, rng, scale)
        R = L.cayley(A)
        assert np.abs(R.conj().T @ R - np.eye(r)).max() < 1e-13
        # Cayley(A) = exp(A) + O(|A|^3)
        err = np.abs(R - expm(A)).max()
        assert err <= 0.2 * np.abs(A).max() ** 3 * r ** 2 + 1e-14


def test_loss_closed_forms():
    rng = np.random.default_rng(2)
    r = 4
    Q, _ = np.linalg.qr(rng.normal(size=(r, r)) + 1j * rng.normal(size=(r, r)))
    ph = np.exp(1j * rng.uniform(0, 2 * np.pi, r))
    # R = T up to column phases: zero loss
    assert L.loss_per_sample(Q, Q * ph[None, :]) < 1e-13
    # R = I: sum_a (1 - |T_aa|^2)
    assert abs(L.loss_per_sample(np.eye(r), Q) - np.sum(1 - np.abs(np.diag(Q)) ** 2)) < 1e-13


def _net(r, rng, scale=0.05):
    p = rng.normal(size=L.n_params(r)) * scale
    return p


def test_output_gradient_through_cayley_matches_finite_differences():
    rng = np.random.default_rng(3)
    r = 3
    T = rng.normal(size=(r, r)) + 1j * rng.normal(size=(r, r))
    o = rng.normal(size=r * r) * 0.7

    def f(ov):
        return L.loss_per_sample(L.cayley(L.unpack_skew(ov, r)), T)

    A = L.unpack_skew(o, r)
    I = np.eye(r)
    M = I - A / 2
    R = np.linalg.solve(M, I + A / 2)
    s = np.einsum('ca,ca->a', np.conj(R), T)
    gR = -2.0 * T * np.conj(s)[None, :]
    gA = np.linalg.solve(M.conj().T, gR @ (I + R).conj().T) / 2
    g = L.pack_skew_grad(gA, r)
    h = 1e-6
    fd = np.array([(f(o + h * e) - f(o - h * e)) / (2 * h) for e in np.eye(r * r)])
    assert np.abs(g - fd).max() < 1e-7 * max(1.0, np.abs(fd).max())


@pytest.mark.parametrize("r", [2, 3])
def test_parameter_gradient_matches_finite_differences(r):
    rng = np.random.default_rng(10 + r)
    p = _net(r, rng)
    B = 5
    X = rng.normal(size=(B, L.n_in(r)))
    T = rng.normal(size=(B, r, r)) + 1j * rng.normal(size=(B, r, r))
    l0, g = L.grad(p, X, T, r)
    assert abs(l0 - L.loss(p, X, T, r)) < 1e-12
    # a sample of parameters from every layer (weights and biases)
    idx = []
    off = 0
    for a, b in L.layer_shapes(r):
        idx += list(off + rng.choice(a * b, 8, replace=False))
        off += a * b
        idx += list(off + rng.choice(b, 3, replace=False))
        off += b
    h = 1e-5
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (L.loss(p + e, X, T, r) - L.loss(p - e, X, T, r)) / (2 * h)
        assert abs(g[i] - fd) < 1e-7 + 1e-5 * abs(fd), (i, g[i], fd)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(4)
    p = rng.normal(size=20)
    g = rng.normal(size=20)
    lr = 1e-3
    p1, m, v = L.adam_step(p, g, np.zeros(20), np.zeros(20), 1, lr)
    # bias-corrected first moments are g and g^2: a step of lr * sign(g)
    assert np.allclose(p1, p - lr * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_predictor_is_first_order_accurate():
    """For K = U diag(lam) U* + eps E, the span of Y0 is O(eps^2) from the
    top-r eigenvectors while u = U[:, :r] is O(eps) away."""
    rng = np.random.default_rng(5)
    m, r = 24, 4
    Q, _ = np.linalg.qr(rng.normal(size=(m, m)) + 1j * rng.normal(size=(m, m)))
    lam = np.array([1.0, 0.8, 0.6, 0.5])
    E = rng.normal(size=(m, m)) + 1j * rng.normal(size=(m, m))
    E = (E + E.conj().T) / 2
    u = Q[:, :r]
    errs_u, errs_y = [], []
    for eps in (1e-2, 1e-3):
        K = (Q[:, :r] * lam) @ Q[:, :r].conj().T + eps * E
        w, V = np.linalg.eigh(K)
        top = V[:, np.argsort(w)[::-1][:r]]

        def dist(Y):
            Yq, _ = np.linalg.qr(Y)
            return np.linalg.norm(Yq - top @ (top.conj().T @ Yq))

        errs_u.append(dist(u))
        errs_y.append(dist(L.predictor(K, u, np.eye(r), lam)))
    assert errs_u[0] / errs_u[1] > 8      # first order
    assert errs_y[0] / errs_y[1] > 80     # second order
    # with K = U diag(lam) U* exactly the predictor returns u R
    K0 = (Q[:, :r] * lam) @ Q[:, :r].conj().T
    R = L.cayley(_rand_skew(r, rng, 0.3)[0])
    assert np.abs(L.predictor(K0, u, R, lam) - u @ R).max() < 1e-13


def test_analytic_rotation_on_an_invariant_subspace():
    """If H maps span(V) into itself, V(t) = exp(-i t H) V = V exp(-i t G),
    G = V* H V, so T = V* V(t) = exp(-i t G); Cayley(-i t G) matches it to
    third order in t."""
    rng = np.random.default_rng(6)
    m, r = 12, 3
    Q, _ = np.linalg.qr(rng.normal(size=(m, m)) + 1j * rng.normal(size=(m, m)))
    Gs = rng.normal(size=(r, r)) + 1j * rng.normal(size=(r, r))
    Gs = (Gs + Gs.conj().T) / 2
    Hs = np.zeros((m, m), complex)
    Hs[:r, :r] = Gs
    Hs[r:, r:] = np.diag(rng.normal(size=m - r))
    H = Q @ Hs @ Q.conj().T
    V = Q[:, :r]
    G = V.conj().T @ H @ V
    for t in (1e-1, 1e-2):
        T = V.conj().T @ (expm(-1j * t * H) @ V)
        assert np.abs(T - expm(-1j * t * G)).max() < 1e-12
        assert np.abs(L.analytic_rotation(G, t) - T).max() < 0.1 * (t * np.abs(G).max()) ** 3 * r ** 2


def test_zero_network_gives_the_analytic_rotation():
    rng = np.random.default_rng(8)
    r = 3
    G = rng.normal(size=(r, r)) + 1j * rng.normal(size=(r, r))
    G = (G + G.conj().T) / 2
    x = L.features(G, 0.02, 0.1)
    p = np.zeros(L.n_params(r))
    R = L.rotations(p, x[None, :], r)[0]
    assert np.abs(R - L.analytic_rotation(G, 0.02)).max() < 1e-14
    # and the analytic parametrisation is -i s G itself
    assert np.abs(L.unpack_skew(L.analytic_params(x, r), r) + 1j * 0.02 * G).max() < 1e-14


def test_features_layout():
    rng = np.random.default_rng(7)
    r = 3
    G = rng.normal(size=(r, r)) + 1j * rng.normal(size=(r, r))
    G = (G + G.conj().T) / 2
    f = L.features(G, 0.01, 0.3)
    n = np.linalg.norm(G)
    assert f.shape == (L.n_in(r),)
    assert np.allclose(f[:r * r].reshape(r, r) + 1j * f[r * r:2 * r * r].reshape(r, r), G / n)
    assert abs(f[-2] - 0.01 * n) < 1e-15 and f[-1] == 0.3
