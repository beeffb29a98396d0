"""GPU checks of the learned start rotation (lrei_net_*, lrei_record, the
predictor warm modes), through the C ABI.

* network loss, gradient, rotations and an Adam step against the float64
  reference in oracle/learned.py on seeded random samples (FP32 kernels: the
  tolerances are those of FP32 accumulation over a width of 256);
* recorded samples against the oracle: the features of a step's first stage
  against V* H V of the state (computed by the oracle's Hamiltonian), the
  targets against the invariants they must satisfy;
* every predictor mode (R = I, analytic, learned) keeps FP64 parity with the
  oracle: the residual certificate and the direct fallback decide the result;
* training on recorded samples lowers the loss.
"""
import numpy as np
import pytest

from oracle import learned as L
from oracle.hamiltonian import Hamiltonian
from oracle.metrics import rel_fro_error
from oracle.schemes import run as oracle_run
from workloads import make_config

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _samples(r, n, seed):
    """Random features and targets (T a random unitary times a contraction)."""
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, L.n_in(r)))
    T = []
    for _ in range(n):
        Q, _ = np.linalg.qr(rng.normal(size=(r, r)) + 1j * rng.normal(size=(r, r)))
        T.append(Q * rng.uniform(0.8, 1.0, size=r)[None, :])
    T = np.array(T)
    flat = np.concatenate([X, np.stack([T.real, T.imag], axis=-1).reshape(n, -1)], axis=1).astype(np.float32)
    return flat, X.astype(np.float32).astype(np.float64), T.astype(np.complex64).astype(np.complex128)


def _dev(a):
    return _torch().from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("r", [4, 16])
def test_loss_gradient_rotations_match_reference(r):
    from paper_2508_21200_amd import Net
    assert Net.param_count(r) == L.n_params(r)
    net = Net(r, seed=7)
    p = net.params().astype(np.float64)
    flat, X, T = _samples(r, 24, 100 + r)
    S = _dev(flat)
    loss, g = net.loss_grad(S)
    lref, gref = L.grad(p, X, T, r)
    print(f"r={r}: loss {loss:.8f} ref {lref:.8f}; |g-gref|/|gref| "
          f"{np.linalg.norm(g - gref) / np.linalg.norm(gref):.2e}")
    assert abs(loss - lref) <= 1e-5 * max(1.0, abs(lref))
    assert np.linalg.norm(g - gref) <= 2e-4 * np.linalg.norm(gref)
    R = net.rotations(S)
    Rref = L.rotations(p, X, r)
    assert np.abs(R - Rref).max() < 1e-5
    assert np.abs(np.einsum('bca,bcd->bad', R.conj(), R) - np.eye(r)).max() < 1e-12  # unitary in FP64
    net.close()


def test_adam_step_matches_reference():
    from paper_2508_21200_amd import Net
    r = 4
    net = Net(r, seed=3)
    p0 = net.params().astype(np.float64)
    flat, X, T = _samples(r, 32, 5)
    S = _dev(flat)
    _, gref = L.grad(p0, X, T, r)
    lr = 1e-3
    net.train(S, batch=32, epochs=1, lr=lr, seed=1)  # one batch: one Adam step from zero moments
    p1 = net.params().astype(np.float64)
    pref, _, _ = L.adam_step(p0, gref, np.zeros_like(p0), np.zeros_like(p0), 1, lr)
    big = np.abs(gref) > 1e-5  # sign(g) decides the first step where |g| is above FP32 noise
    assert np.abs(p1 - pref)[big].max() < 2e-6
    assert np.abs(p1 - p0).max() <= lr * 1.001


def _chain_ctx(precision="fp64", warm="analytic", n=8, r=4, seed_traj=0):
    from paper_2508_21200_amd import Context
    cfg = make_config(2, n=n, r=r, traj=seed_traj)
    c = Context(precision=precision, warm=warm)
    c.set_hamiltonian(cfg["n"], cfg["bonds"], cfg["J"], cfg["h"])
    c.set_rho(cfg["lam"], cfg["V"])
    return c, cfg


def test_recorded_features_and_targets():
    from paper_2508_21200_amd import net_sample_floats
    torch = _torch()
    r = 4
    c, cfg = _chain_ctx(r=r)
    steps = 3
    buf = torch.zeros((4 * steps + 5, net_sample_floats(r)), dtype=torch.float32, device="cuda")
    c.record(buf)
    kappa, dt = 0.2, 0.01
    c.step("qLLG", "RK4", dt, kappa, steps)
    n = c.record_count()
    assert n == 4 * steps
    S = buf.cpu().numpy()[:n]
    nin = L.n_in(r)
    for k in range(n):
        f, t = S[k, :nin], S[k, nin:]
        G = f[:r * r].reshape(r, r) + 1j * f[r * r:2 * r * r].reshape(r, r)
        assert abs(np.linalg.norm(G) - 1.0) < 1e-5
        assert np.abs(G - G.conj().T).max() < 1e-6
        assert f[-1] == np.float32(kappa)
        # RK4 stages 1 and 3 map a state to one at the same time: zero step
        if k % 4 in (1, 3):
            assert abs(f[-2]) < 1e-9
        T = (t[0::2] + 1j * t[1::2]).reshape(r, r)
        sv = np.linalg.svd(T, compute_uv=False)
        assert sv.max() < 1 + 1e-5 and sv.min() > 0.9
    # stage 0 of the first step: u = V_0, so G = V* H V / |V* H V| and s |G| = (dt / 2) |V* H V|
    H = Hamiltonian(cfg["n"], cfg["bonds"], cfg["J"], cfg["h"])
    V = cfg["V"]
    G0 = V.conj().T @ H.apply(V)
    f = S[0, :nin]
    Gf = f[:r * r].reshape(r, r) + 1j * f[r * r:2 * r * r].reshape(r, r)
    # stage 0's input basis holds V's coordinates in the orthonormal Krylov
    # basis, so its projected generator is V* H V itself
    Gn = G0 / np.linalg.norm(G0)
    assert np.abs(Gf - Gn).max() < 1e-6
    assert abs(f[-2] - 0.5 * dt * np.linalg.norm(G0)) < 1e-5 * max(1.0, 0.5 * dt * np.linalg.norm(G0))
    c.record(None)
    c.step("qLLG", "RK4", dt, kappa, 1)
    assert c.record_count() == 0
    c.close()


@pytest.mark.parametrize("warm", ["predict_identity", "predict_cayley", "learned"])
def test_predictor_modes_keep_parity(warm):
    from paper_2508_21200_amd import Net
    r = 4
    c, cfg = _chain_ctx(warm=warm, r=r)
    net = None
    if warm == "learned":
        net = Net(r, seed=11)
        c.attach_net(net)
    steps, dt, kappa = 4, 0.01, 0.2
    c.step("qLLG", "RK4", dt, kappa, steps)
    H = Hamiltonian(cfg["n"], cfg["bonds"], cfg["J"], cfg["h"])
    Vo = oracle_run(H, cfg["V"], cfg["lam"], "qLLG", kappa, dt, steps, "RK4")
    err = rel_fro_error(c.get_rho()[1], cfg["lam"], Vo, cfg["lam"])
    st = c.stats()
    print(f"{warm}: err {err:.2e}, accepted {st['warm_accepted']} rejected {st['warm_rejected']} "
          f"products {st['warm_iterations']} of {st['eigensolves']} eigensolves")
    assert err < 1e-10
    assert st["warm_accepted"] + st["warm_rejected"] <= st["eigensolves"]
    c.close()
    if net:
        net.close()


def test_untrained_network_steps_like_the_analytic_predictor():
    """A new network has a zero output layer, so its rotation is the analytic
    one: in-kernel inference must reproduce that predictor's solves (same
    products, same acceptances) and its result up to FP32 feature rounding."""
    from paper_2508_21200_amd import Net
    r = 4
    out = {}
    for warm in ("predict_cayley", "learned"):
        c, cfg = _chain_ctx(warm=warm, r=r)
        net = Net(r, seed=3) if warm == "learned" else None
        if net:
            c.attach_net(net)
        c.step("qLLG", "RK4", 0.01, 0.2, 4)
        st = c.stats()
        out[warm] = (c.get_rho()[1], st["warm_accepted"], st["warm_rejected"], st["warm_iterations"])
        c.close()
        if net:
            net.close()
    a, b = out["predict_cayley"], out["learned"]
    assert a[1:] == b[1:]
    assert rel_fro_error(a[0], cfg["lam"], b[0], cfg["lam"]) < 1e-12


def test_learned_needs_an_attached_network():
    from paper_2508_21200_amd import LreiError, Net
    c, _ = _chain_ctx(warm="learned", r=4)
    with pytest.raises(LreiError, match="attached network"):
        c.step("qLLG", "RK4", 0.01, 0.2, 1)
    net = Net(8)
    with pytest.raises(LreiError, match="rank"):
        c.attach_net(net)
    c.close()
    net.close()


def _excess(S, r, R):
    """Mean over samples of loss(R) - loss(polar(T)): the part of the loss a
    rotation can remove (T = u* u_next is not unitary; its polar factor is
    the best rotation)."""
    nin = L.n_in(r)
    out = []
    for k in range(S.shape[0]):
        t = S[k, nin:].astype(np.float64)
        T = (t[0::2] + 1j * t[1::2]).reshape(r, r)
        U, _, Wh = np.linalg.svd(T)
        out.append(L.loss_per_sample(R[k], T) - L.loss_per_sample(U @ Wh, T))
    return float(np.mean(out))


def _net_excess(net, B, r):
    return _excess(B.cpu().numpy(), r, net.rotations(B, B.shape[0]))


def _analytic_excess(B, r):
    S = B.cpu().numpy()
    nin = L.n_in(r)
    G = S[:, :r * r].reshape(-1, r, r) + 1j * S[:, r * r:2 * r * r].reshape(-1, r, r)
    R = np.array([L.analytic_rotation(g, float(f)) for g, f in zip(G, S[:, nin - 2])])
    return _excess(S, r, R)


def _train_pick(net, p0, train, val, r, lrs=(1e-4, 3e-5, 1e-5)):
    """Adam at each step size from the same start; keeps the parameters that
    score best on the validation samples."""
    best = None
    for lr in lrs:
        net.set_params(p0)
        losses = net.train(train, train.shape[0], batch=64, epochs=60, lr=lr, seed=4)
        ev = _net_excess(net, val, r)
        print(f"  lr {lr:.0e}: validation excess {ev:.3e}; epoch means {losses[0]:.6e} .. {losses[-1]:.6e}")
        if best is None or ev < best[0]:
            best = (ev, lr, net.params())
    net.set_params(best[2])
    return best[1]


def test_training_gain_on_held_out_steps():
    """Recorded stages of three chain trajectories (r = 4), each split in
    time: the first 30 steps train the network, steps 30-34 pick the Adam step
    size, steps 35-39 are held out.  On the held-out steps the trained network
    must remove at least half of the excess loss the analytic rotation leaves.
    The same network scored on two other trajectories (own couplings, fields,
    spectrum and damping) is reported too: the inputs (G, the step, the
    damping) do not carry the spectrum Lambda_0 or the coupling of the support
    to its complement, which set the rotation beyond first order, so what is
    learned is specific to the trajectories trained on."""
    from paper_2508_21200_amd import Net, net_sample_floats
    torch = _torch()
    r = 4
    per = 40
    ns = 4 * per  # RK4 stages recorded per trajectory
    buf = torch.zeros((5 * ns, net_sample_floats(r)), dtype=torch.float32, device="cuda")
    total = 0
    for t in range(5):
        c, _ = _chain_ctx(r=r, n=8, seed_traj=t)
        c.record(buf[total:])
        c.step("qLLG", "RK4", 0.01, 0.05 + 0.1 * t, per)
        total += c.record_count()
        c.close()
    assert total == 5 * ns
    # samples are recorded stage by stage, four per step
    tr_idx, va_idx, te_idx = [], [], []
    for t in range(3):
        tr_idx += range(t * ns, t * ns + 4 * 30)
        va_idx += range(t * ns + 4 * 30, t * ns + 4 * 35)
        te_idx += range(t * ns + 4 * 35, (t + 1) * ns)
    pick = lambda idx: buf[torch.tensor(idx, device="cuda")].contiguous()
    train, val, test, other = pick(tr_idx), pick(va_idx), pick(te_idx), buf[3 * ns:].contiguous()
    net = Net(r, seed=2)
    p0 = net.params()
    ex_an_test = _analytic_excess(test, r)
    assert abs(_net_excess(net, test, r) - ex_an_test) <= 1e-3 * ex_an_test + 1e-12  # zero output layer
    lr = _train_pick(net, p0, train, val, r)
    ex_test = _net_excess(net, test, r)
    ex_an_other, ex_other = _analytic_excess(other, r), _net_excess(net, other, r)
    print(f"held-out steps (lr {lr:.0e}): excess loss analytic {ex_an_test:.3e}, trained {ex_test:.3e} "
          f"({ex_an_test / ex_test:.1f}x lower); other trajectories: analytic {ex_an_other:.3e}, "
          f"trained {ex_other:.3e}")
    assert ex_test <= 0.5 * ex_an_test
    net.close()
