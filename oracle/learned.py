"""Learned start rotation for the stage eigensolve: plain float64 reference.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper does not have this component; it is a production form built on top
of the stage eigensolve of Sec. 3.7 (the r largest eigenvectors of each stage
matrix).  What it computes, in the order the GPU path does:

* features of a stage: the projected generator G = u* H u of the stage's
  input basis u (r x r Hermitian), normalised by its Frobenius norm, the
  dimensionless step s |G|_F (s = c h / hbar, c the stage's step fraction) and
  the damping kappa: 2 r^2 + 2 reals;
* a multilayer perceptron, three hidden layers of width 256 with SiLU
  activations, whose r^2 outputs o parametrise a skew-Hermitian correction
  (r imaginary diagonal entries, then the r (r - 1) / 2 upper off-diagonal
  entries as (re, im) pairs, row by row) to the analytic generator
  -i s G: A = unpack(o + o_an(x)), o_an the same parametrisation of
  -i s G read off the features (a network with zero output gives the
  analytic rotation);
* the Cayley map R = (I - A/2)^{-1} (I + A/2), a unitary r x r rotation;
* the training target of a stage: T = u* u_next, the overlap of the input
  basis with the stage's output eigenvectors (u_next), and the loss
  sum_a (1 - |(R* T)_aa|^2), invariant under the phases of u_next's columns;
* the start block for the stage eigensolve built from R:
  Y0 = u R + (I - u u*) K u R Lambda^{-1} (first-order eigenvector correction
  in the rotated basis; span(Y0) depends on R through Lambda^{-1});
* plain backpropagation of the loss, through the Cayley map
  (dR = (I - A/2)^{-1} (dA / 2) (I + R)), and Adam.

Parameter layout (one flat vector): W1 [in x 256] row-major, b1 [256],
W2 [256 x 256], b2, W3 [256 x 256], b3, W4 [256 x r^2], b4 [r^2]; a layer
computes h_out = h_in W + b.  Gradients use the convention g = dL/dRe + i dL/dIm
for complex intermediates.
"""
import numpy as np

WIDTH = 256


def n_in(r):
    return 2 * r * r + 2


def layer_shapes(r):
    """(fan_in, fan_out) of the four layers."""
    return [(n_in(r), WIDTH), (WIDTH, WIDTH), (WIDTH, WIDTH), (WIDTH, r * r)]


def n_params(r):
    return sum(a * b + b for a, b in layer_shapes(r))


def split(params, r):
    """Views (W, b) per layer into the flat parameter vector."""
    out, off = [], 0
    for a, b in layer_shapes(r):
        W = params[off:off + a * b].reshape(a, b)
        off += a * b
        bb = params[off:off + b]
        off += b
        out.append((W, bb))
    return out


def features(G, step, kappa):
    """2 r^2 + 2 inputs of one stage: Re, Im of G / |G|_F, step |G|_F, kappa."""
    G = np.asarray(G, dtype=np.complex128)
    nrm = np.linalg.norm(G)
    Gn = G / nrm if nrm > 0 else G
    return np.concatenate([Gn.real.ravel(), Gn.imag.ravel(), [step * nrm, kappa]])


def analytic_params(x, r):
    """r^2 reals of -i s G from the features x (G / |G| and s |G|)."""
    x = np.asarray(x, dtype=np.float64)
    sg = x[..., 2 * r * r]
    gre = x[..., :r * r].reshape(x.shape[:-1] + (r, r))
    gim = x[..., r * r:2 * r * r].reshape(x.shape[:-1] + (r, r))
    o = np.zeros(x.shape[:-1] + (r * r,))
    o[..., :r] = -sg[..., None] * np.diagonal(gre, axis1=-2, axis2=-1)
    k = r
    for a in range(r):
        for b in range(a + 1, r):
            o[..., k] = sg * gim[..., a, b]
            o[..., k + 1] = -sg * gre[..., a, b]
            k += 2
    return o


def unpack_skew(o, r):
    """Skew-Hermitian A from r^2 reals: A_aa = i o_a, then A_ab = o + i o'
    for a < b row by row, A_ba = -conj(A_ab)."""
    A = np.zeros((r, r), dtype=np.complex128)
    A[np.arange(r), np.arange(r)] = 1j * o[:r]
    k = r
    for a in range(r):
        for b in range(a + 1, r):
            z = o[k] + 1j * o[k + 1]
            A[a, b] = z
            A[b, a] = -np.conj(z)
            k += 2
    return A


def pack_skew_grad(gA, r):
    """Gradient with respect to the r^2 reals of unpack_skew, given
    gA = dL/dRe A + i dL/dIm A over all r^2 entries."""
    g = np.zeros(r * r)
    g[:r] = np.imag(np.diag(gA))
    k = r
    for a in range(r):
        for b in range(a + 1, r):
            q = np.conj(gA[a, b]) - gA[b, a]
            g[k] = q.real
            g[k + 1] = -q.imag
            k += 2
    return g


def cayley(A):
    n = A.shape[0]
    I = np.eye(n)
    return np.linalg.solve(I - A / 2, I + A / 2)


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(params, X, r):
    """Network outputs O [B x r^2] and the pre-activations of the hidden layers."""
    layers = split(params, r)
    h = np.asarray(X, dtype=np.float64)
    zs, hs = [], [h]
    for li, (W, b) in enumerate(layers):
        z = h @ W + b
        if li < 3:
            zs.append(z)
            h = silu(z)
            hs.append(h)
        else:
            h = z
    return h, zs, hs


def rotations(params, X, r):
    O, _, _ = forward(params, X, r)
    O = O + analytic_params(X, r)
    return np.stack([cayley(unpack_skew(o, r)) for o in O])


def loss_per_sample(R, T):
    d = np.einsum('ca,ca->a', np.conj(R), T)  # (R* T)_aa
    return np.sum(1.0 - np.abs(d) ** 2)


def loss(params, X, T, r):
    """Mean over the batch of sum_a (1 - |(R* T)_aa|^2)."""
    R = rotations(params, X, r)
    return np.mean([loss_per_sample(Rk, Tk) for Rk, Tk in zip(R, T)])


def grad(params, X, T, r):
    """Loss and its gradient with respect to the flat parameters (backprop)."""
    O, zs, hs = forward(params, X, r)
    B = O.shape[0]
    gO = np.zeros_like(O)
    L = 0.0
    I = np.eye(r)
    Oa = O + analytic_params(X, r)  # the analytic part does not depend on the parameters
    for k in range(B):
        A = unpack_skew(Oa[k], r)
        M = I - A / 2
        R = np.linalg.solve(M, I + A / 2)
        s = np.einsum('ca,ca->a', np.conj(R), T[k])
        L += np.sum(1.0 - np.abs(s) ** 2)
        gR = -2.0 * T[k] * np.conj(s)[None, :]           # dL/dR (g convention)
        gA = np.linalg.solve(M.conj().T, gR @ (I + R).conj().T) / 2
        gO[k] = pack_skew_grad(gA, r)
    gO /= B
    layers = split(params, r)
    grads = []
    g = gO
    for li in range(3, -1, -1):
        W, b = layers[li]
        h_in = hs[li]
        gW = h_in.T @ g
        gb = g.sum(axis=0)
        grads.append((gW, gb))
        if li > 0:
            g = (g @ W.T) * dsilu(zs[li - 1])
    flat = []
    for gW, gb in reversed(grads):
        flat.append(gW.ravel())
        flat.append(gb)
    return L / B, np.concatenate(flat)


def adam_step(params, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015, with bias correction); t counts from 1."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def analytic_rotation(G, step):
    """R = Cayley(-i step G): the in-span rotation of a step of the
    undamped flow V' = -(i/hbar) H V to second order in the step."""
    return cayley(-1j * step * np.asarray(G, dtype=np.complex128))


def predictor(K, u, R, lam):
    """Start block Y0 = u R + (I - u u*) K u R diag(1 / lam)."""
    X = u @ R
    KX = K @ X
    P = KX - u @ (u.conj().T @ KX)
    return X + P / np.asarray(lam)[None, :]
