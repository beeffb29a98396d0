"""GPU parity of batched trajectories (lrei_batch_* through the C ABI).

Every trajectory of a batch must match the oracle's run of that trajectory
alone (FP64 path: 1e-11 relative Frobenius on rho after a few steps, as the
single-trajectory tests; mixed path: 1e-5), and the batch must match the
single-trajectory context on the same inputs.  Inputs come from the seeded
generators; expected values from ``oracle`` only.
"""
import numpy as np
import pytest

from oracle.hamiltonian import Hamiltonian
from oracle.metrics import rel_fro_error
from oracle.observables import energy as oracle_energy
from oracle.schemes import run as oracle_run
from workloads import make_config, CONFIGS

pytestmark = pytest.mark.gpu


def _traj(cfg):
    return dict(n=cfg["n"], bonds=cfg["bonds"], J=cfg["J"], h=cfg["h"], lam=cfg["lam"], V=cfg["V"],
                model=cfg["model"], kappa=cfg["kappa"])


def _mixed_batch():
    """Heterogeneous small batch: several n and r (r > 16 included), both
    models, complex and real coefficient tables, a tiny N below one tile."""
    shapes = [(6, 3), (7, 1), (8, 4), (9, 8), (10, 16), (5, 2), (9, 20), (4, 4)]
    trajs = []
    for t, (n, r) in enumerate(shapes):
        cfg = make_config(4, traj=t, n=n, r=r)
        trajs.append(_traj(cfg))
    # a real-coefficient Hamiltonian (Heisenberg chain with a z field)
    c1 = make_config(1, n=7, r=3)
    c1["model"], c1["kappa"] = "qLLG", 0.3
    trajs.append(_traj(c1))
    return trajs


def _oracle(t, scheme, dt, steps):
    H = Hamiltonian(t["n"], t["bonds"], t["J"], t["h"])
    return oracle_run(H, t["V"], t["lam"], t["model"], t["kappa"], dt, steps, scheme)


@pytest.mark.parametrize("scheme", ["RK1", "RK2", "RK3", "RK4"])
def test_batch_matches_oracle_fp64(scheme):
    from paper_2508_21200_amd import Batch
    trajs = _mixed_batch()
    b = Batch(trajs, precision="fp64")
    b.step(scheme, 0.01, 3)
    for q, t in enumerate(trajs):
        lam, Vg = b.get_rho(q)
        assert np.array_equal(lam, t["lam"])
        Vo = _oracle(t, scheme, 0.01, 3)
        err = rel_fro_error(Vg, t["lam"], Vo, t["lam"])
        print(f"{scheme} traj {q} n={t['n']} r={t['lam'].size} {t['model']}: {err:.3e}")
        assert err < 1e-11
    b.close()


def test_batch_matches_single_context():
    from paper_2508_21200_amd import Batch, Context
    trajs = _mixed_batch()
    b = Batch(trajs, precision="fp64")
    b.step("RK4", 0.01, 4)
    for q, t in enumerate(trajs):
        c = Context(precision="fp64")
        c.set_hamiltonian(t["n"], t["bonds"], t["J"], t["h"])
        c.set_rho(t["lam"], t["V"])
        c.step(t["model"], "RK4", 0.01, t["kappa"], 4)
        err = rel_fro_error(b.get_rho(q)[1], t["lam"], c.get_rho()[1], t["lam"])
        assert err < 1e-13, (q, err)
        c.close()


def test_batch_graph_replay_equals_eager():
    from paper_2508_21200_amd import Batch
    trajs = _mixed_batch()
    out = []
    for use_graph in (True, False):
        b = Batch(trajs, precision="fp64", use_graph=use_graph)
        for _ in range(3):
            b.step("RK4", 0.01, 2)
        out.append([b.get_rho(q)[1] for q in range(len(trajs))])
        b.close()
    for a, c in zip(*out):
        assert np.array_equal(a, c)


def test_batch_scheme_and_dt_changes():
    from paper_2508_21200_amd import Batch
    trajs = _mixed_batch()[:4]
    b = Batch(trajs, precision="fp64")
    b.step("RK4", 0.01, 2)
    b.step("RK2", 0.02, 1)
    b.step("RK4", 0.005, 2)
    for q, t in enumerate(trajs):
        H = Hamiltonian(t["n"], t["bonds"], t["J"], t["h"])
        Vo = oracle_run(H, t["V"], t["lam"], t["model"], t["kappa"], 0.01, 2, "RK4")
        Vo = oracle_run(H, Vo, t["lam"], t["model"], t["kappa"], 0.02, 1, "RK2")
        Vo = oracle_run(H, Vo, t["lam"], t["model"], t["kappa"], 0.005, 2, "RK4")
        assert rel_fro_error(b.get_rho(q)[1], t["lam"], Vo, t["lam"]) < 1e-11


def test_batch_mixed_within_1e5():
    from paper_2508_21200_amd import Batch
    trajs = _mixed_batch()
    b = Batch(trajs, precision="mixed")
    b.step("RK4", 0.01, 10)
    for q, t in enumerate(trajs):
        Vo = _oracle(t, "RK4", 0.01, 10)
        err = rel_fro_error(b.get_rho(q)[1], t["lam"], Vo, t["lam"])
        print(f"mixed traj {q}: {err:.3e}")
        assert err < 1e-5


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_autotune_keeps_parity(precision):
    """lrei_batch_autotune between steps: every candidate shape it times runs on
    the device, the chosen shapes cover every rank of the batch, and after it
    (the step graph captured again) every trajectory still matches the oracle
    (FP64 1e-11, mixed 1e-5) and, in FP64, the untuned batch to 1e-12 (the Gram
    partial sums split differently)."""
    from paper_2508_21200_amd import Batch
    trajs = _mixed_batch()
    ref = Batch(trajs, precision=precision)
    ref.step("RK4", 0.01, 3)
    b = Batch(trajs, precision=precision)
    b.step("RK4", 0.01, 2)
    res = b.autotune(iters=3)
    print(f"{precision}: default {res['ms_default']:.4f} ms, tuned {res['ms']:.4f} ms, "
          f"{len(res['tried'])} tried, choice {res['choice']}")
    ranks = sorted({int(t["lam"].size) for t in trajs})
    assert sorted(res["choice"]) == ranks
    assert len(res["tried"]) >= len(ranks)
    assert res["ms_default"] > 0 and res["ms"] > 0
    assert all(ms > 0 for _, _, _, ms in res["tried"])
    b.step("RK4", 0.01, 1)
    tol = 1e-11 if precision == "fp64" else 1e-5
    for q, t in enumerate(trajs):
        Vg = b.get_rho(q)[1]
        Vo = _oracle(t, "RK4", 0.01, 3)
        err = rel_fro_error(Vg, t["lam"], Vo, t["lam"])
        print(f"tuned {precision} traj {q} n={t['n']} r={t['lam'].size}: {err:.3e}")
        assert err < tol
        if precision == "fp64":
            assert rel_fro_error(Vg, t["lam"], ref.get_rho(q)[1], t["lam"]) < 1e-12
    b.close()
    ref.close()


def test_batch_energies():
    from paper_2508_21200_amd import Batch
    trajs = _mixed_batch()
    b = Batch(trajs, precision="fp64")
    e = b.energies()
    for q, t in enumerate(trajs):
        H = Hamiltonian(t["n"], t["bonds"], t["J"], t["h"])
        assert abs(e[q] - oracle_energy(H, t["V"], t["lam"])) < 1e-11 * max(1.0, abs(e[q]))


def test_batch_invalid_inputs():
    from paper_2508_21200_amd import Batch, LreiError
    trajs = _mixed_batch()[:3]
    bad = [dict(t) for t in trajs]
    bad[2]["lam"] = -bad[2]["lam"]
    with pytest.raises(LreiError, match="trajectory 2"):
        Batch(bad)
    bad = [dict(t) for t in trajs]
    V = bad[1]["V"].copy()
    V[:, 0] *= 1.1
    bad[1]["V"] = V
    with pytest.raises(LreiError, match="trajectory 1"):
        Batch(bad)
    bad = [dict(t) for t in trajs]
    bad[0]["bonds"] = np.array([[1, 0]])
    bad[0]["J"] = np.eye(3)[None]
    with pytest.raises(LreiError, match="trajectory 0"):
        Batch(bad)
    b = Batch(trajs)
    before = b.get_rho(0)[1].copy()
    with pytest.raises(LreiError):
        b.step("AB3", 0.01, 1)
    with pytest.raises(LreiError):
        b.step("RK4", -0.01, 1)
    with pytest.raises(LreiError):
        b.get_rho(3)
    assert np.array_equal(b.get_rho(0)[1], before)


@pytest.fixture(scope="module")
def cfg4_trajs():
    k = 4
    return [_traj(make_config(k, traj=t)) for t in range(CONFIGS[k]["n_traj"])]


def test_cfg4_batch_mixed_vs_fp64_and_oracle(cfg4_trajs):
    """The 64-trajectory XXZ workload (n 12..16, r in {4, 8, 16}): mixed batch
    against the FP64 batch on every trajectory, and both against the oracle on
    the two smallest trajectories."""
    from paper_2508_21200_amd import Batch
    steps = 5
    runs = {}
    for prec in ("fp64", "mixed"):
        b = Batch(cfg4_trajs, precision=prec)
        b.step("RK4", 0.01, steps)
        runs[prec] = [b.get_rho(q)[1] for q in range(len(cfg4_trajs))]
        b.close()
    worst = 0.0
    for q, t in enumerate(cfg4_trajs):
        worst = max(worst, rel_fro_error(runs["mixed"][q], t["lam"], runs["fp64"][q], t["lam"]))
    print(f"cfg4 mixed vs fp64 worst rel_fro_error over 64 trajectories: {worst:.3e}")
    assert worst < 1e-5
    order = sorted(range(len(cfg4_trajs)), key=lambda q: (cfg4_trajs[q]["n"], cfg4_trajs[q]["lam"].size))
    for q in order[:2]:
        t = cfg4_trajs[q]
        Vo = _oracle(t, "RK4", 0.01, steps)
        assert rel_fro_error(runs["fp64"][q], t["lam"], Vo, t["lam"]) < 1e-10
        assert rel_fro_error(runs["mixed"][q], t["lam"], Vo, t["lam"]) < 1e-5
