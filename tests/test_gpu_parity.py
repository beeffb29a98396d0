"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerances: FP64 path 1e-10 relative Frobenius on rho (per-step checks use
1e-11); mixed path 1e-5.  Every test builds its inputs from the seeded
workload generators and computes the expected values with ``oracle`` only.
"""
import numpy as np
import pytest

from oracle.hamiltonian import Hamiltonian, apply_H, apply_H_rows
from oracle.schemes import lrei_rk_step, run as oracle_run
from oracle.metrics import rel_fro_error
from oracle.observables import energy as oracle_energy, magnetization as oracle_mag
from workloads import (make_config, chain_bonds, square_lattice_bonds, haar_factor, dirichlet_spectrum,
                       heisenberg_tensors, uniform_field, pure_factor, af1_index, xxz_tensors)

pytestmark = pytest.mark.gpu


def _ctx(precision="fp64", **kw):
    from paper_2508_21200_amd import Context
    return Context(device=0, precision=precision, **kw)


def _random_model(n, rng, periodic=True):
    bonds = chain_bonds(n, periodic=periodic and n > 2)
    J = rng.normal(size=(bonds.shape[0], 3, 3)) * 0.5
    h = rng.normal(size=(n, 3)) * 0.5
    return bonds, J, h


@pytest.mark.parametrize("n,r", [(6, 1), (7, 3), (8, 4), (9, 16), (10, 20), (8, 32), (12, 8)])
def test_apply_hamiltonian(n, r):
    rng = np.random.default_rng(100 + n + r)
    bonds, J, h = _random_model(n, rng)
    X = haar_factor(2 ** n, r, rng)
    ctx = _ctx()
    ctx.set_hamiltonian(n, bonds, J, h)
    Y = ctx.apply_hamiltonian(X)
    Yo = apply_H(n, bonds, J, h, X)
    assert np.abs(Y - Yo).max() <= 1e-13 * max(1.0, np.abs(Yo).max())


@pytest.mark.parametrize("scheme", ["RK1", "RK2", "RK3", "RK4"])
@pytest.mark.parametrize("model", ["qLL", "qLLG"])
@pytest.mark.parametrize("n,r", [(6, 3), (9, 4)])
def test_rk_steps_fp64(scheme, model, n, r):
    rng = np.random.default_rng(7 * n + r)
    bonds, J, h = _random_model(n, rng)
    V = haar_factor(2 ** n, r, rng)
    lam = dirichlet_spectrum(r, rng)
    ctx = _ctx()
    ctx.set_hamiltonian(n, bonds, J, h)
    ctx.set_rho(lam, V)
    ctx.step(model, scheme, 0.02, 0.5, 3)
    _, Vg = ctx.get_rho()
    H = Hamiltonian(n, bonds, J, h)
    Vo = V
    for _ in range(3):
        Vo = lrei_rk_step(H, Vo, lam, model, 0.5, 0.02, scheme)
    err = rel_fro_error(Vg, lam, Vo, lam)
    print(f"{model} {scheme} n={n} r={r}: rel_fro_error={err:.3e}")
    assert err < 1e-11


@pytest.mark.parametrize("hmode", [0, 1])
def test_householder_and_projector_agree(hmode):
    cfg = make_config(2, n=10, r=6)
    ctx = _ctx(householder_mode=hmode)
    ctx.set_hamiltonian(cfg["n"], cfg["bonds"], cfg["J"], cfg["h"])
    ctx.set_rho(cfg["lam"], cfg["V"])
    ctx.step("qLLG", "RK4", 0.01, 0.05, 5)
    _, Vg = ctx.get_rho()
    H = Hamiltonian(cfg["n"], cfg["bonds"], cfg["J"], cfg["h"])
    Vo = oracle_run(H, cfg["V"], cfg["lam"], "qLLG", 0.05, 0.01, 5, "RK4")
    assert rel_fro_error(Vg, cfg["lam"], Vo, cfg["lam"]) < 1e-11


def test_cfg1_full_run_fp64():
    """Heisenberg chain n=8, r=4, q-LL, RK4 dt=0.01 x 100 (the small parity workload)."""
    cfg = make_config(1)
    ctx = _ctx()
    ctx.set_hamiltonian(cfg["n"], cfg["bonds"], cfg["J"], cfg["h"])
    ctx.set_rho(cfg["lam"], cfg["V"])
    ctx.step(cfg["model"], "RK4", cfg["dt"], cfg["kappa"], cfg["steps"])
    _, Vg = ctx.get_rho()
    H = Hamiltonian(cfg["n"], cfg["bonds"], cfg["J"], cfg["h"])
    Vo = oracle_run(H, cfg["V"], cfg["lam"], cfg["model"], cfg["kappa"], cfg["dt"], cfg["steps"], "RK4")
    err = rel_fro_error(Vg, cfg["lam"], Vo, cfg["lam"])
    print(f"cfg1 100 steps rel_fro_error={err:.3e} stats={ctx.stats()}")
    assert err < 1e-10


def test_mixed_precision_within_1e5():
    cfg = make_config(2, n=12, r=8)
    ctx = _ctx("mixed")
    ctx.set_hamiltonian(cfg["n"], cfg["bonds"], cfg["J"], cfg["h"])
    ctx.set_rho(cfg["lam"], cfg["V"])
    ctx.step("qLLG", "RK4", 0.005, 0.05, 20)
    _, Vg = ctx.get_rho()
    H = Hamiltonian(cfg["n"], cfg["bonds"], cfg["J"], cfg["h"])
    Vo = oracle_run(H, cfg["V"], cfg["lam"], "qLLG", 0.05, 0.005, 20, "RK4")
    err = rel_fro_error(Vg, cfg["lam"], Vo, cfg["lam"])
    print(f"mixed n=12 r=8 20 steps rel_fro_error={err:.3e}")
    assert err < 1e-5


def test_observables():
    rng = np.random.default_rng(3)
    n, r = 9, 5
    bonds, J, h = _random_model(n, rng)
    V = haar_factor(2 ** n, r, rng)
    lam = dirichlet_spectrum(r, rng)
    ctx = _ctx()
    ctx.set_hamiltonian(n, bonds, J, h, hbar=0.8)
    ctx.set_rho(lam, V)
    e, m = ctx.observables()
    H = Hamiltonian(n, bonds, J, h)
    assert abs(e - oracle_energy(H, V, lam)) < 1e-12
    np.testing.assert_allclose(m, oracle_mag(n, V, lam, hbar=0.8), atol=1e-13)


def test_fixed_point_and_tiny_systems():
    """Degenerate Krylov spaces: a commuting pure state, and N smaller than the basis."""
    n = 6
    bonds = chain_bonds(n)
    J = heisenberg_tensors(bonds.shape[0], 1.0)
    h = uniform_field(n, (0, 0, 0.8))
    V = pure_factor(n, index=0)
    ctx = _ctx()
    ctx.set_hamiltonian(n, bonds, J, h)
    ctx.set_rho([1.0], V)
    ctx.step("qLLG", "RK4", 0.05, 0.5, 10)
    _, Vg = ctx.get_rho()
    assert rel_fro_error(Vg, [1.0], V, [1.0]) < 1e-13
    # n = 2 and n = 3: 5 r exceeds N, the Krylov space saturates
    for n, r in ((2, 1), (2, 2), (3, 2), (3, 4)):
        rng = np.random.default_rng(n * 10 + r)
        bonds, Jr, hr = _random_model(n, rng)
        V = haar_factor(2 ** n, r, rng)
        lam = dirichlet_spectrum(r, rng)
        ctx = _ctx()
        ctx.set_hamiltonian(n, bonds, Jr, hr)
        ctx.set_rho(lam, V)
        ctx.step("qLL", "RK4", 0.02, 0.3, 4)
        _, Vg = ctx.get_rho()
        H = Hamiltonian(n, bonds, Jr, hr)
        Vo = oracle_run(H, V, lam, "qLL", 0.3, 0.02, 4, "RK4")
        err = rel_fro_error(Vg, lam, Vo, lam)
        print(f"tiny n={n} r={r}: {err:.3e} stats={ctx.stats()}")
        assert err < 1e-11


def test_pure_af_state_convergence_to_exact():
    """Pure |AF1> on a chain: GPU LREI-RK4 agrees with the oracle step for step."""
    n = 8
    bonds = chain_bonds(n)
    H = Hamiltonian(n, bonds, heisenberg_tensors(bonds.shape[0], 1.0), uniform_field(n, (0.4, 0, 0.3)))
    V = pure_factor(n, index=af1_index(n))
    ctx = _ctx()
    ctx.set_hamiltonian(n, H.bonds, H.J, H.h)
    ctx.set_rho([1.0], V)
    ctx.step("qLLG", "RK4", 0.01, 0.5, 20)
    _, Vg = ctx.get_rho()
    Vo = oracle_run(H, V, np.array([1.0]), "qLLG", 0.5, 0.01, 20, "RK4")
    assert rel_fro_error(Vg, [1.0], Vo, [1.0]) < 1e-11


def test_graph_replay_equals_eager():
    cfg = make_config(2, n=10, r=8)
    out = []
    for use_graph in (True, False):
        ctx = _ctx(use_graph=use_graph)
        ctx.set_hamiltonian(cfg["n"], cfg["bonds"], cfg["J"], cfg["h"])
        ctx.set_rho(cfg["lam"], cfg["V"])
        for _ in range(3):
            ctx.step("qLLG", "RK4", 0.01, 0.05, 2)
        out.append(ctx.get_rho()[1])
    assert np.array_equal(out[0], out[1])  # deterministic, bitwise


def test_checkpoint_resume_bitwise():
    cfg = make_config(2, n=9, r=4)
    a = _ctx()
    a.set_hamiltonian(cfg["n"], cfg["bonds"], cfg["J"], cfg["h"])
    a.set_rho(cfg["lam"], cfg["V"])
    a.step("qLL", "RK4", 0.01, 0.2, 6)
    blob = a.get_state()
    a.step("qLL", "RK4", 0.01, 0.2, 4)
    b = _ctx()
    b.set_hamiltonian(cfg["n"], cfg["bonds"], cfg["J"], cfg["h"])
    b.set_state(blob)
    b.step("qLL", "RK4", 0.01, 0.2, 4)
    assert np.array_equal(a.get_rho()[1], b.get_rho()[1])


def test_invalid_inputs_leave_state():
    from paper_2508_21200_amd import LreiError
    cfg = make_config(2, n=8, r=4)
    ctx = _ctx()
    ctx.set_hamiltonian(cfg["n"], cfg["bonds"], cfg["J"], cfg["h"])
    ctx.set_rho(cfg["lam"], cfg["V"])
    before = ctx.get_rho()[1].copy()
    bad = cfg["V"].copy()
    bad[:, 0] *= 1.1
    for lam, V in ((cfg["lam"], bad), (cfg["lam"][::-1].copy(), cfg["V"]), (-cfg["lam"], cfg["V"])):
        with pytest.raises(LreiError):
            ctx.set_rho(lam, V)
    assert np.array_equal(ctx.get_rho()[1], before)
    with pytest.raises(LreiError):
        ctx.step("qLL", "RK4", -0.1, 0.1, 1)
    with pytest.raises(LreiError):
        ctx.step("qLL", "RK4", 0.1, -0.1, 1)


def test_full_size_hv_sampled_rows():
    """4x5 periodic Heisenberg lattice, n=20, r=16: sampled rows of H V vs the oracle."""
    cfg = make_config(3)
    ctx = _ctx()
    ctx.set_hamiltonian(cfg["n"], cfg["bonds"], cfg["J"], cfg["h"])
    Y = ctx.apply_hamiltonian(cfg["V"])
    rows = np.random.default_rng(0).choice(2 ** 20, size=256, replace=False)
    rows = np.concatenate([rows, [0, 1, 2 ** 20 - 1]])
    Yo = apply_H_rows(cfg["n"], cfg["bonds"], cfg["J"], cfg["h"], cfg["V"], rows)
    assert np.abs(Y[rows] - Yo).max() < 1e-13 * np.abs(Yo).max()


# ---- Adams-Bashforth schemes (Sec. 3.8) -------------------------------------

@pytest.mark.parametrize("scheme", ["AB2", "AB3", "AB4"])
@pytest.mark.parametrize("model", ["qLL", "qLLG"])
def test_ab_steps_fp64(scheme, model):
    """RK4 start-up, then AB steps with the orthonormal history basis, against the oracle."""
    n, r, steps = 8, 4, 8
    rng = np.random.default_rng(11 * n + r + len(scheme))
    bonds, J, h = _random_model(n, rng)
    V = haar_factor(2 ** n, r, rng)
    lam = dirichlet_spectrum(r, rng)
    ctx = _ctx()
    ctx.set_hamiltonian(n, bonds, J, h)
    ctx.set_rho(lam, V)
    ctx.step(model, scheme, 0.01, 0.3, steps)
    _, Vg = ctx.get_rho()
    H = Hamiltonian(n, bonds, J, h)
    Vo = oracle_run(H, V, lam, model, 0.3, 0.01, steps, scheme)
    err = rel_fro_error(Vg, lam, Vo, lam)
    print(f"{model} {scheme} n={n} r={r} {steps} steps: rel_fro_error={err:.3e} stats={ctx.stats()}")
    assert err < 1e-11


@pytest.mark.parametrize("householder_mode", [0, 1])
def test_ab_split_calls_and_modes(householder_mode):
    """An AB run split over calls equals one call (bitwise); both complement forms agree with the oracle."""
    cfg = make_config(2, n=9, r=6)
    out = []
    for split in ((9,), (2, 3, 4)):
        ctx = _ctx(householder_mode=householder_mode)
        ctx.set_hamiltonian(cfg["n"], cfg["bonds"], cfg["J"], cfg["h"])
        ctx.set_rho(cfg["lam"], cfg["V"])
        for k in split:
            ctx.step("qLLG", "AB3", 0.005, 0.05, k)
        out.append(ctx.get_rho()[1])
    assert np.array_equal(out[0], out[1])
    H = Hamiltonian(cfg["n"], cfg["bonds"], cfg["J"], cfg["h"])
    Vo = oracle_run(H, cfg["V"], cfg["lam"], "qLLG", 0.05, 0.005, 9, "AB3")
    assert rel_fro_error(out[0], cfg["lam"], Vo, cfg["lam"]) < 1e-11


def test_ab_restarts_when_dt_changes():
    """Changing dt starts a new AB run (new RK start-up) from the current state, as the oracle does."""
    cfg = make_config(2, n=8, r=4)
    ctx = _ctx()
    ctx.set_hamiltonian(cfg["n"], cfg["bonds"], cfg["J"], cfg["h"])
    ctx.set_rho(cfg["lam"], cfg["V"])
    ctx.step("qLL", "AB2", 0.01, 0.2, 4)
    ctx.step("qLL", "AB2", 0.005, 0.2, 3)
    _, Vg = ctx.get_rho()
    H = Hamiltonian(cfg["n"], cfg["bonds"], cfg["J"], cfg["h"])
    Vo = oracle_run(H, cfg["V"], cfg["lam"], "qLL", 0.2, 0.01, 4, "AB2")
    Vo = oracle_run(H, Vo, cfg["lam"], "qLL", 0.2, 0.005, 3, "AB2")
    assert rel_fro_error(Vg, cfg["lam"], Vo, cfg["lam"]) < 1e-11


def test_ab_rejects_unsupported_sizes():
    from paper_2508_21200_amd import LreiError
    rng = np.random.default_rng(5)
    n = 3
    bonds, J, h = _random_model(n, rng)
    ctx = _ctx()
    ctx.set_hamiltonian(n, bonds, J, h)
    ctx.set_rho(dirichlet_spectrum(2, rng), haar_factor(8, 2, rng))
    with pytest.raises(LreiError):
        ctx.step("qLL", "AB2", 0.01, 0.1, 1)  # N = 8 < (2m + 2) r = 12
    n = 7
    bonds, J, h = _random_model(n, rng)
    ctx = _ctx()
    ctx.set_hamiltonian(n, bonds, J, h)
    ctx.set_rho(dirichlet_spectrum(20, rng), haar_factor(128, 20, rng))
    with pytest.raises(LreiError):
        ctx.step("qLL", "AB3", 0.01, 0.1, 1)  # r > 16


@pytest.fixture(scope="module")
def cfg2_oracle10():
    """Oracle reference for the n = 16 XXZ chain, r = 8, q-LLG, AB3 dt 0.005: first 10 steps."""
    cfg = make_config(2)
    H = Hamiltonian(cfg["n"], cfg["bonds"], cfg["J"], cfg["h"])
    return cfg, oracle_run(H, cfg["V"], cfg["lam"], cfg["model"], cfg["kappa"], cfg["dt"], 10, cfg["scheme"])


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 1e-5)])
def test_cfg2_ab3_parity(cfg2_oracle10, precision, tol):
    cfg, Vo = cfg2_oracle10
    ctx = _ctx(precision)
    ctx.set_hamiltonian(cfg["n"], cfg["bonds"], cfg["J"], cfg["h"])
    ctx.set_rho(cfg["lam"], cfg["V"])
    ctx.step(cfg["model"], cfg["scheme"], cfg["dt"], cfg["kappa"], 10)
    _, Vg = ctx.get_rho()
    err = rel_fro_error(Vg, cfg["lam"], Vo, cfg["lam"])
    print(f"n=16 r=8 AB3 {precision}: 10 steps rel_fro_error={err:.3e}")
    assert err < tol


def test_cfg2_ab3_full_run_properties():
    """All 50 steps: mixed agrees with FP64 within 1e-5, the factor stays orthonormal, and the
    q-LLG energy does not increase (kappa > 0 dissipates)."""
    cfg = make_config(2)
    res = {}
    for precision in ("fp64", "mixed"):
        ctx = _ctx(precision)
        ctx.set_hamiltonian(cfg["n"], cfg["bonds"], cfg["J"], cfg["h"])
        ctx.set_rho(cfg["lam"], cfg["V"])
        e0, _ = ctx.observables()
        ctx.step(cfg["model"], cfg["scheme"], cfg["dt"], cfg["kappa"], cfg["steps"])
        e1, _ = ctx.observables()
        res[precision] = (ctx.get_rho()[1], e0, e1)
    V64, e0, e1 = res["fp64"]
    assert np.abs(V64.conj().T @ V64 - np.eye(cfg["r"])).max() < 1e-12
    assert e1 <= e0 + 1e-12
    assert rel_fro_error(res["mixed"][0], cfg["lam"], V64, cfg["lam"]) < 1e-5


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_ab_checkpoint_resume_bitwise(precision):
    """A checkpoint taken inside an AB3 run carries the history: resuming continues bitwise."""
    cfg = make_config(2, n=9, r=4)
    a = _ctx(precision)
    a.set_hamiltonian(cfg["n"], cfg["bonds"], cfg["J"], cfg["h"])
    a.set_rho(cfg["lam"], cfg["V"])
    a.step("qLLG", "AB3", 0.005, 0.05, 5)
    blob = a.get_state()
    a.step("qLLG", "AB3", 0.005, 0.05, 4)
    b = _ctx(precision)
    b.set_hamiltonian(cfg["n"], cfg["bonds"], cfg["J"], cfg["h"])
    b.set_state(blob)
    b.step("qLLG", "AB3", 0.005, 0.05, 4)
    assert np.array_equal(a.get_rho()[1], b.get_rho()[1])
    if precision == "fp64":
        H = Hamiltonian(cfg["n"], cfg["bonds"], cfg["J"], cfg["h"])
        Vo = oracle_run(H, cfg["V"], cfg["lam"], "qLLG", 0.05, 0.005, 9, "AB3")
        assert rel_fro_error(b.get_rho()[1], cfg["lam"], Vo, cfg["lam"]) < 1e-11


def test_autotune_keeps_results_and_caches(tmp_path):
    """Tuning the H.V launch shape changes speed only; a cache file replays the choice."""
    cfg = make_config(2, n=12, r=8)
    cache = tmp_path / "tune.txt"
    out = []
    for tune in (False, True, True):
        ctx = _ctx(autotune_cache=cache)
        ctx.set_hamiltonian(cfg["n"], cfg["bonds"], cfg["J"], cfg["h"])
        ctx.set_rho(cfg["lam"], cfg["V"])
        if tune:
            res = ctx.autotune()
            out.append(res)
        ctx.step("qLLG", "RK4", 0.005, 0.05, 4)
        out.append(ctx.get_rho()[1])
    V0, t1, V1, t2, V2 = out
    assert t1["from_cache"] is False and len(t1["tried"]) >= 2
    assert t2["from_cache"] is True and (t2["epl"], t2["grid"]) == (t1["epl"], t1["grid"])
    assert rel_fro_error(V1, cfg["lam"], V0, cfg["lam"]) < 1e-12
    assert np.array_equal(V1, V2)


@pytest.mark.parametrize("r,hmode", [(20, 1), (20, 0), (32, 1)])
def test_rk4_large_rank(r, hmode):
    """r > 16: the column-parallel Householder path and projected problems up to order 5 r = 160."""
    n = 9
    rng = np.random.default_rng(900 + r + hmode)
    bonds, J, h = _random_model(n, rng)
    V = haar_factor(2 ** n, r, rng)
    lam = dirichlet_spectrum(r, rng)
    ctx = _ctx(householder_mode=hmode)
    ctx.set_hamiltonian(n, bonds, J, h)
    ctx.set_rho(lam, V)
    ctx.step("qLLG", "RK4", 0.01, 0.3, 2)
    _, Vg = ctx.get_rho()
    H = Hamiltonian(n, bonds, J, h)
    Vo = oracle_run(H, V, lam, "qLLG", 0.3, 0.01, 2, "RK4")
    err = rel_fro_error(Vg, lam, Vo, lam)
    print(f"r={r} hmode={hmode}: {err:.3e}")
    assert err < 1e-11


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_rk4_degenerate_spectrum(precision):
    """Lambda_0 with an exactly repeated and a nearly repeated pair: the warm
    solver's Ritz step meets eigenvalue gaps of order h (the Newton refinement
    of the Ritz vectors may not contract there and the Jacobi solve takes
    over).  rho = V Lambda_0 V* is unique however a repeated pair's vectors
    are rotated; 4 RK4 steps against the oracle."""
    n, r = 9, 8
    rng = np.random.default_rng(1300)
    bonds, J, h = _random_model(n, rng)
    V = haar_factor(2 ** n, r, rng)
    lam = np.array([0.3, 0.2, 0.2, 0.12, 0.1 + 1e-9, 0.1, 0.05, 0.03])
    lam = lam / lam.sum()
    ctx = _ctx(precision)
    ctx.set_hamiltonian(n, bonds, J, h)
    ctx.set_rho(lam, V)
    ctx.step("qLL", "RK4", 0.01, 0.5, 4)
    st = ctx.stats()
    H = Hamiltonian(n, bonds, J, h)
    Vo = oracle_run(H, V, lam, "qLL", 0.5, 0.01, 4, "RK4")
    err = rel_fro_error(ctx.get_rho()[1], lam, Vo, lam)
    print(f"{precision}: {err:.3e}, warm accepted {st['warm_accepted']} of {st['eigensolves']}")
    assert err < (1e-11 if precision == "fp64" else 1e-5)


@pytest.mark.parametrize("r", [20, 27, 32])
def test_rk4_large_rank_mixed(r):
    """Mixed precision above r = 16 (two columns per lane, three Gram items
    per wave, the Gram partial sums of up to 3 r^2 entries staged in LDS):
    3 RK4 steps against the oracle."""
    cfg = make_config(2, n=10, r=16)
    rng = np.random.default_rng(1200 + r)
    lam = dirichlet_spectrum(r, rng)
    V = haar_factor(2 ** cfg["n"], r, rng)
    ctx = _ctx("mixed")
    ctx.set_hamiltonian(cfg["n"], cfg["bonds"], cfg["J"], cfg["h"])
    ctx.set_rho(lam, V)
    ctx.step("qLLG", "RK4", 0.01, 0.05, 3)
    st = ctx.stats()
    H = Hamiltonian(cfg["n"], cfg["bonds"], cfg["J"], cfg["h"])
    Vo = oracle_run(H, V, lam, "qLLG", 0.05, 0.01, 3, "RK4")
    err = rel_fro_error(ctx.get_rho()[1], lam, Vo, lam)
    print(f"mixed r={r}: {err:.3e}, dropped {st['dropped_directions']}")
    assert st["dropped_directions"] == 0
    assert err < 1e-5


@pytest.mark.parametrize("case", ["chain_n10_r6", "lattice_n12_r16", "chain_n9_r20", "tiny_n4_r4"])
def test_warm_start_matches_direct_solve(case):
    """Stage eigensolves by subspace iteration from the predicted basis (the
    default) against the direct tridiagonal solver: same rho to rounding, and
    every eigensolve accounted for as accepted or fallen back."""
    if case == "chain_n10_r6":
        cfg = make_config(2, n=10, r=6)
    elif case == "lattice_n12_r16":
        cfg = make_config(3, n=12, r=16)
    elif case == "chain_n9_r20":
        cfg = make_config(2, n=9, r=20)
    else:
        cfg = make_config(2, n=4, r=4)
    out, st = {}, {}
    for warm in ("plain", "analytic"):
        ctx = _ctx(warm=warm)
        ctx.set_hamiltonian(cfg["n"], cfg["bonds"], cfg["J"], cfg["h"])
        ctx.set_rho(cfg["lam"], cfg["V"])
        ctx.step(cfg["model"], "RK4", 0.01, cfg["kappa"], 5)
        out[warm] = ctx.get_rho()[1]
        st[warm] = ctx.stats()
        ctx.close()
    err = rel_fro_error(out["analytic"], cfg["lam"], out["plain"], cfg["lam"])
    s = st["analytic"]
    print(f"{case}: warm vs direct {err:.3e}; accepted {s['warm_accepted']} rejected {s['warm_rejected']} "
          f"iterations {s['warm_iterations']} of {s['eigensolves']} eigensolves")
    assert err < 1e-12
    # stages whose workspace does not fit the on-chip arena go straight to the direct solver
    assert s["warm_accepted"] + s["warm_rejected"] <= s["eigensolves"] == 20
    assert st["plain"]["warm_accepted"] == st["plain"]["warm_rejected"] == 0
    if case != "tiny_n4_r4":
        assert s["warm_accepted"] > 0


def test_warm_start_falls_back_on_large_steps():
    """A step far beyond the usual size: the rest of each stage spectrum is no
    longer small, so subspace iteration may not converge or certify; whatever
    path each eigensolve takes, the result must match the oracle."""
    rng = np.random.default_rng(41)
    n, r = 7, 4
    bonds, J, h = _random_model(n, rng)
    V = haar_factor(2 ** n, r, rng)
    lam = dirichlet_spectrum(r, rng)
    ctx = _ctx()
    ctx.set_hamiltonian(n, bonds, J, h)
    ctx.set_rho(lam, V)
    ctx.step("qLLG", "RK4", 0.4, 0.3, 2)
    s = ctx.stats()
    H = Hamiltonian(n, bonds, J, h)
    Vo = oracle_run(H, V, lam, "qLLG", 0.3, 0.4, 2, "RK4")
    err = rel_fro_error(ctx.get_rho()[1], lam, Vo, lam)
    print(f"large step: {err:.3e}; accepted {s['warm_accepted']} rejected {s['warm_rejected']}")
    assert err < 1e-10
    assert s["warm_accepted"] + s["warm_rejected"] <= s["eigensolves"]


def test_warm_mode_out_of_range_is_rejected():
    """Unknown start modes fail at creation; the learned mode is accepted
    there and needs an attached network to step (tests/test_gpu_learned.py)."""
    from paper_2508_21200_amd import Context, LreiError
    from paper_2508_21200_amd import lrei as _l
    _l.WARM["bogus"] = 7
    try:
        with pytest.raises(LreiError):
            Context(precision="fp64", warm="bogus")
    finally:
        del _l.WARM["bogus"]


# ---- two-spin reduced density matrices (Sec. 3.6) ----------------------------

def _random_state(n, r, rng):
    return haar_factor(2 ** n, r, rng), dirichlet_spectrum(r, rng)


@pytest.mark.parametrize("n,r,prec", [(6, 1, "fp64"), (8, 4, "fp64"), (11, 20, "fp64"), (12, 8, "mixed"),
                                      (9, 3, "mixed")])
def test_pair_density_matches_oracle(n, r, prec):
    from oracle.observables import pair_density
    rng = np.random.default_rng(100 + n + r)
    bonds, J, h = _random_model(n, rng)
    V, lam = _random_state(n, r, rng)
    c = _ctx(prec)
    c.set_hamiltonian(n, bonds, J, h)
    c.set_rho(lam, V)
    pairs = [(0, 1), (n - 1, 0), (2, n - 2), (n // 2, 1), (3, 2)]
    R = c.pair_density(pairs)
    tol = 1e-13 if prec == "fp64" else 1e-6
    for (k, l), Rg in zip(pairs, R):
        Ro = pair_density(V, lam, n, k, l)
        assert np.abs(Rg - Ro).max() < tol, (k, l, np.abs(Rg - Ro).max())
    c.close()


def test_pair_density_after_steps_and_invalid_pairs():
    from paper_2508_21200_amd import LreiError, pair_entanglement
    from oracle.observables import pair_density, concurrence
    rng = np.random.default_rng(7)
    n, r = 8, 3
    bonds, J, h = _random_model(n, rng)
    V, lam = _random_state(n, r, rng)
    c = _ctx("fp64")
    c.set_hamiltonian(n, bonds, J, h)
    c.set_rho(lam, V)
    c.step("qLLG", "RK4", 0.01, 0.3, 5)
    H = Hamiltonian(n, bonds, J, h)
    Vo = oracle_run(H, V, lam, "qLLG", 0.3, 0.01, 5, "RK4")
    R = c.pair_density([(1, 4), (6, 5)])
    for (k, l), Rg in zip([(1, 4), (6, 5)], R):
        Ro = pair_density(Vo, lam, n, k, l)
        assert np.abs(Rg - Ro).max() < 1e-11
        assert abs(pair_entanglement(Rg)[0] - concurrence(Ro)) < 1e-6
    before = c.get_rho()[1].copy()
    for bad in ([(2, 2)], [(0, n)], [(-1, 3)]):
        with pytest.raises(LreiError):
            c.pair_density(bad)
    assert np.array_equal(c.get_rho()[1], before)
    c.close()


def test_pair_density_full_size():
    """n = 20, r = 16 (the lattice workload's state, mixed storage) on a few
    pairs against the oracle's partial trace of the same input."""
    from oracle.observables import pair_density
    cfg = make_config(3)
    c = _ctx("mixed")
    c.set_hamiltonian(cfg["n"], cfg["bonds"], cfg["J"], cfg["h"])
    c.set_rho(cfg["lam"], cfg["V"])
    pairs = [(0, 1), (0, 5), (19, 3), (12, 13)]
    R = c.pair_density(pairs)
    for (k, l), Rg in zip(pairs, R):
        Ro = pair_density(cfg["V"], cfg["lam"], cfg["n"], k, l)
        assert np.abs(Rg - Ro).max() < 1e-6
        assert abs(np.trace(Rg).real - 1.0) < 1e-6
    c.close()


@pytest.mark.parametrize("model", ["qLL", "qLLG"])
def test_maximally_mixed_admixture(model):
    """rho = p I / N + (1 - p) V Lambda V*: the low-rank part follows the
    oracle's run with damping (1 - p) kappa, and the observables and pair
    matrices are those of the full state."""
    from paper_2508_21200_amd import LreiError
    from oracle.observables import pair_density
    rng = np.random.default_rng(11)
    n, r, p, kappa = 7, 3, 0.3, 0.4
    bonds, J, h = _random_model(n, rng)
    V, lam = _random_state(n, r, rng)
    c = _ctx("fp64")
    c.set_hamiltonian(n, bonds, J, h)
    c.set_rho(lam, V)
    c.set_mixing(p)
    c.step(model, "RK4", 0.01, kappa, 4)
    H = Hamiltonian(n, bonds, J, h)
    Vo = oracle_run(H, V, lam, model, (1 - p) * kappa, 0.01, 4, "RK4")
    assert rel_fro_error(c.get_rho()[1], lam, Vo, lam) < 1e-11
    e, m = c.observables()
    assert abs(e - (1 - p) * oracle_energy(H, Vo, lam)) < 1e-11
    assert np.abs(m - (1 - p) * oracle_mag(n, Vo, lam)).max() < 1e-11
    R = c.pair_density([(0, 3)])[0]
    assert np.abs(R - (p * np.eye(4) / 4 + (1 - p) * pair_density(Vo, lam, n, 0, 3))).max() < 1e-12
    for bad in (1.0, -0.1, float("nan")):
        with pytest.raises(LreiError):
            c.set_mixing(bad)
    c.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_state_from_factor(prec):
    """rho_0 = A A* / Tr from a non-orthogonal (and a rank-deficient) factor,
    against the oracle's range Rayleigh-Ritz, then a step vs the oracle."""
    from oracle.lowrank import state_from_factor
    rng = np.random.default_rng(21)
    n = 9
    bonds, J, h = _random_model(n, rng)
    B = rng.normal(size=(2 ** n, 4)) + 1j * rng.normal(size=(2 ** n, 4))
    for A in (B, np.concatenate([B, B[:, 1:2] * (0.5 + 2j)], axis=1)):
        c = _ctx(prec)
        c.set_hamiltonian(n, bonds, J, h)
        c.set_rho_factor(A)
        lam_o, V_o = state_from_factor(A)
        lam, V = c.get_rho()
        assert lam.size == lam_o.size == 4
        assert np.abs(lam - lam_o).max() < 1e-14
        tol = 1e-12 if prec == "fp64" else 1e-6
        assert rel_fro_error(V, lam, V_o, lam_o) < tol
        c.step("qLL", "RK4", 0.01, 0.2, 2)
        H = Hamiltonian(n, bonds, J, h)
        Vs = oracle_run(H, V_o, lam_o, "qLL", 0.2, 0.01, 2, "RK4")
        assert rel_fro_error(c.get_rho()[1], lam_o, Vs, lam_o) < (1e-11 if prec == "fp64" else 1e-5)
        c.close()


def test_full_size_step_properties():
    """The 4x5 lattice workload at full size (n = 20, r = 16) in the launch
    configuration the benchmark times (mixed storage, autotuned H.V shape,
    captured step graph): properties that hold at any size, since the
    oracle's own full-size step takes minutes.
    * mixed against FP64 after 10 RK4 steps: <= 1e-5 relative Frobenius;
    * kappa = 0 conserves Tr(rho H) along the exact flow and LREI-RK4 keeps
      it to O(h^4); kappa = 0.5 drives it down (the oracle on the 3 x 4
      lattice over 10 steps of h = 0.01: 7e-8 against 0.24): the drift at
      kappa = 0 stays below 1e-4 of the change at kappa = 0.5 (FP64);
    * the support stays orthonormal (FP64 to 1e-12, mixed to its FP32
      storage rounding)."""
    import torch
    from tests_support_rel import rel_fro_gpu
    cfg = make_config(3)
    V0 = torch.from_numpy(cfg["V"]).cuda()
    out = {}
    for prec in ("fp64", "mixed"):
        c = _ctx(prec)
        c.set_hamiltonian(cfg["n"], cfg["bonds"], cfg["J"], cfg["h"])
        c.set_rho(cfg["lam"], V0)
        if prec == "mixed":
            c.autotune()
        c.step("qLL", "RK4", 0.01, 0.5, 10)
        _, V = c.get_rho(torch.empty_like(V0))
        G = (V.conj().T @ V).cpu().numpy()
        dev = np.abs(G - np.eye(G.shape[0])).max()
        assert dev < (1e-12 if prec == "fp64" else 1e-6), (prec, dev)
        out[prec] = V
        c.close()
    err = rel_fro_gpu(out["mixed"], out["fp64"], cfg["lam"])
    print(f"n=20 r=16, 10 RK4 steps: mixed vs FP64 {err:.2e}")
    assert err < 1e-5
    e = {}
    for kappa in (0.0, 0.5):
        c = _ctx("fp64")
        c.set_hamiltonian(cfg["n"], cfg["bonds"], cfg["J"], cfg["h"])
        c.set_rho(cfg["lam"], V0)
        e0, _ = c.observables()
        c.step("qLL", "RK4", 0.01, kappa, 10)
        e[kappa] = c.observables()[0] - e0
        c.close()
    print(f"energy change over 10 steps: kappa = 0 {e[0.0]:.3e}, kappa = 0.5 {e[0.5]:.3e}")
    assert abs(e[0.0]) <= 1e-4 * abs(e[0.5])


def test_mixed_promotion_mechanics():
    """A floor above every pivot ratio promotes a mixed context at the first
    check (after 16 steps): the run continues in FP64 and matches the oracle
    to the mixed bound; observables, pair matrices, AB steps and adaptive
    stepping work afterwards, and an adaptive run promotes the same way."""
    rng = np.random.default_rng(21)
    n, r = 8, 4
    bonds, J, h = _random_model(n, rng)
    V, lam = _random_state(n, r, rng)
    H = Hamiltonian(n, bonds, J, h)
    c = _ctx("mixed", mixed_pivot_floor=1.0)
    c.set_hamiltonian(n, bonds, J, h)
    c.set_rho(lam, V)
    c.step("qLLG", "RK4", 0.01, 0.3, 24)
    assert c.stats()["precision_promoted"] == 1
    Vo = oracle_run(H, V, lam, "qLLG", 0.3, 0.01, 24, "RK4")
    assert rel_fro_error(c.get_rho()[1], lam, Vo, lam) < 1e-5
    c.observables()
    c.pair_density([[0, 1]])
    c.step("qLLG", "AB3", 0.01, 0.3, 4)
    c.step("qLLG", "RK4", 0.01, 0.3, 2)
    c.close()
    c = _ctx("mixed", mixed_pivot_floor=1.0)
    c.set_hamiltonian(n, bonds, J, h)
    c.set_rho(lam, V)
    res = c.evolve_adaptive("qLLG", 0.3, 0.2, 1e-6, 0.01, h_min=1e-8, h_max=1.0, pair="RK43")
    assert res["status"] == "done" and c.stats()["precision_promoted"] == 1
    Vo, log = OA_evolve(H, V, lam, "qLLG", 0.3, 0.2, 1e-6, 0.01, 1e-8, 1.0, "RK43")
    assert rel_fro_error(c.get_rho()[1], lam, Vo, lam) < 1e-5
    c.close()


def OA_evolve(H, V, lam, model, kappa, T, tol, h0, h_min, h_max, pair):
    from oracle import adaptive
    return adaptive.evolve(H, V, lam, model, kappa, T, tol, h0, h_min, h_max, pair=pair)
