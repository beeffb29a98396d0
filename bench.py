#!/usr/bin/env python3
"""LREI throughput benchmark on one MI355X.

Workload (default): the 4x5 periodic square-lattice Heisenberg model, n = 20
(N = 1,048,576), J ~ U[0.8, 1.2] per bond, field (0, 0, 1), q-LL with
kappa = 0.5, rank r = 16 (Dirichlet spectrum, Haar factor), LREI-RK4 with
dt = 0.01, mixed precision (complex FP32 N-space passes, FP64 projected step).

One "step" is one LREI-RK4 time step: four matrix-free H.V passes with fused
Gram products, the FP64 projected step (Householder complement action, stage
combination, four partial eigensolves) and the basis combination.

Prints one JSON line.  Extra fields: `roofline` for the dominant kernel (the
H.V pass), `cpu_baseline` (one complete step of the CPU oracle on the same
inputs, measured in a child process that runs beside the GPU work), `parity`
(relative Frobenius error of one GPU step, mixed and FP64, against that oracle
step), `fp64_path` (the FP64 GPU path's rate on the same workload),
`kernels_ms` (per-kernel averages), `batch` (the 64-trajectory batched
workload: its rate, its smallest trajectories against the oracle, and its rate
against the FP64 batch and against the plain FP64 path).
"""
import argparse
import json
import os
import subprocess
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=3,
                    help="3: the n=20 lattice (default); 4: 64 batched trajectories; 2, 5: other single "
                         "workloads")
    ap.add_argument("--precision", default=None, choices=[None, "fp64", "mixed"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default H.V launch shape")
    ap.add_argument("--tune-cache", default=None,
                    help="autotuner cache file: a stored choice is reused without timing trials")
    ap.add_argument("--profile-only", action="store_true",
                    help="run warmup + timed steps only (for rocprofv3 runs)")
    ap.add_argument("--kernels-only", action="store_true",
                    help="set up the workload and launch each kernel of a step eagerly, 20 times "
                         "(for rocprofv3 --pmc runs)")
    ap.add_argument("--learned-report", action="store_true",
                    help="train the learned start rotation on recorded n=14 chain stages and compare the "
                         "eigensolve start modes on the n=22 chain (config 5); prints one JSON line")
    ap.add_argument("--rk-vs-ab", action="store_true",
                    help="time LREI-RK4 and LREI-AB4 steps on triangular lattices n = 10..20 (r = 3 mixture of "
                         "AF1, AF2, GHZ; DMI and transverse field of Sec. 5); prints one JSON line")
    ap.add_argument("--adaptive-report", action="store_true",
                    help="work-precision table: adaptive RK4(3) / BS3(2) / HE2(1) against fixed-step RK4")
    ap.add_argument("--scaling-report", action="store_true",
                    help="q-LLG RK4 step time with observables against n (triangular lattices) and r = 1..4")
    ap.add_argument("--train-only", action="store_true",
                    help="with --learned-report: record and train only (no evaluation runs); for counter "
                         "collection on the training kernels")
    ap.add_argument("--train-traj", type=int, default=100)
    ap.add_argument("--train-steps", type=int, default=200)
    ap.add_argument("--train-epochs", type=int, default=20)
    ap.add_argument("--train-lr", type=float, nargs="+", default=[1e-6, 3e-7, 1e-7],
                    help="Adam step sizes tried; the best on the validation trajectories is kept")
    ap.add_argument("--oracle-deadline", type=float, default=420.0,
                    help="seconds after start by which the oracle step (cpu_baseline, parity) must finish; "
                         "past it the child is stopped and both are reported as not measured")
    ap.add_argument("--oracle-child", default=None, metavar="DIR",
                    help=argparse.SUPPRESS)  # internal: run one oracle step of --config and write it to DIR
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="run a plain device-to-device copy of MIB MiB five times and exit "
                         "(reference kernel for scaling FETCH_SIZE / WRITE_SIZE counters)")
    return ap.parse_args()


def rel_fro(torch, V1, V2, lam):
    """Relative Frobenius distance of V1 diag(lam) V1* and V2 diag(lam) V2*
    (measurement helper).  With [V1, V2] = Q R the difference is
    Q (R D R*) Q*, D = diag(lam, -lam), so its norm is |R D R*|_F, formed
    without the cancellation of subtracting two nearly equal matrices."""
    dev = "cuda"
    W = torch.cat([torch.as_tensor(V1, device=dev), torch.as_tensor(V2, device=dev)], dim=1).to(torch.complex128)
    la = torch.as_tensor(np.asarray(lam, dtype=np.float64), device=dev)
    _, R = torch.linalg.qr(W, mode="r")
    D = torch.cat([la, -la]).to(torch.complex128)
    diff = torch.linalg.norm((R * D[None, :]) @ R.conj().T)
    _, R2 = torch.linalg.qr(W[:, V1.shape[1]:], mode="r")
    ref = torch.linalg.norm((R2 * la.to(torch.complex128)[None, :]) @ R2.conj().T)
    return float(diff / ref)


def measured_copy_gbs(torch, mib=1024, reps=10):
    """Streaming-copy bandwidth of this GPU: a device-to-device copy of `mib`
    MiB timed with events (bytes read + bytes written per copy)."""
    n = (mib << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    gbs = 2 * (mib << 20) / (ms * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return {"GBs": round(gbs, 1), "bytes_per_copy": 2 * (mib << 20),
            "method": f"torch device-to-device copy of {mib} MiB, {reps} copies timed with events"}


def source_digest():
    """Digest of the sources that decide the H.V pass's memory traffic (the
    N-space kernels and the site -> row-bit order); a stored traffic figure is
    only used while it matches."""
    import hashlib
    h = hashlib.sha256()
    for name in ("nspace.hip", "site_order.cpp"):
        with open(os.path.join(ROOT, "paper_2508_21200_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_child(args):
    """Child process: one complete oracle LREI step of the workload from its
    initial state (all rows, no sampling); writes V and the wall time."""
    from workloads import make_config
    from oracle.hamiltonian import Hamiltonian
    from oracle.schemes import lrei_rk_step
    cfg = make_config(args.config)
    H = Hamiltonian(cfg["n"], cfg["bonds"], cfg["J"], cfg["h"])
    t0 = time.perf_counter()
    V1 = lrei_rk_step(H, cfg["V"], cfg["lam"], cfg["model"], cfg["kappa"], cfg["dt"], cfg["scheme"])
    t = time.perf_counter() - t0
    np.save(os.path.join(args.oracle_child, "V1.npy"), V1)
    with open(os.path.join(args.oracle_child, "t.json"), "w") as f:
        json.dump({"seconds": t}, f)


class OracleStep:
    """One oracle step of the benchmark workload in a child process, started
    before the GPU work.  The child keeps off the CPU this process runs on and
    leaves one more core free, so the timed GPU region is not disturbed; its
    BLAS uses the remaining cores (numpy's gathers are single-threaded)."""

    def __init__(self, args):
        self.dir = tempfile.mkdtemp(prefix="lrei_oracle_")
        self.all_cpus = os.sched_getaffinity(0)
        cpus = sorted(self.all_cpus)
        keep = cpus[2:] if len(cpus) > 2 else cpus
        self.threads = len(keep)
        env = dict(os.environ)
        for k in ("OPENBLAS_NUM_THREADS", "OMP_NUM_THREADS", "MKL_NUM_THREADS"):
            env[k] = str(self.threads)
        cmd = [sys.executable, os.path.abspath(__file__), "--oracle-child", self.dir, "--config", str(args.config)]
        self.t_start = time.perf_counter()
        self.proc = subprocess.Popen(cmd, env=env, stdout=subprocess.DEVNULL, stderr=subprocess.PIPE,
                                     preexec_fn=lambda: os.sched_setaffinity(0, keep))
        if len(cpus) > 2:  # this process (and the GPU runtime's threads) on the other two
            os.sched_setaffinity(0, cpus[:2])

    def wait(self, deadline_s, t0):
        """Waits for the child until `deadline_s` after `t0`, printing a
        progress line every 30 s."""
        while self.proc.poll() is None:
            left = deadline_s - (time.perf_counter() - t0)
            if left <= 0:
                break
            try:
                self.proc.wait(timeout=min(30.0, left))
            except subprocess.TimeoutExpired:
                print(f"[bench] oracle step still running ({time.perf_counter() - self.t_start:.0f} s)",
                      file=sys.stderr, flush=True)
        if self.proc.poll() is None:
            self.proc.kill()
            self.proc.wait()
            return None, {"value": None, "unit": "steps/s", "cores": self.threads, "kind": "oracle",
                          "sample": (f"one complete oracle step did not finish within the benchmark's time "
                                     f"budget ({time.perf_counter() - self.t_start:.0f} s, {cpu_model()}); "
                                     f"not measured")}
        if self.proc.returncode != 0:
            err = self.proc.stderr.read().decode(errors="replace")[-400:]
            return None, {"value": None, "unit": "steps/s", "cores": self.threads, "kind": "oracle",
                          "sample": f"the oracle child failed: {err}"}
        V1 = np.load(os.path.join(self.dir, "V1.npy"))
        with open(os.path.join(self.dir, "t.json")) as f:
            t = json.load(f)["seconds"]
        return V1, {"value": 1.0 / t, "unit": "steps/s", "cores": self.threads, "kind": "oracle",
                    "sample": (f"one complete oracle LREI step of this workload from its initial state: all "
                               f"2^n rows, no sampling, no scaling; {t:.1f} s wall on {cpu_model()}, BLAS threads "
                               f"{self.threads} (numpy's row gathers in the oracle's H.V are single-threaded)")}

    def cleanup(self):
        import shutil
        shutil.rmtree(self.dir, ignore_errors=True)
        os.sched_setaffinity(0, self.all_cpus)


def cpu_baseline_batch(trajs, budget_s=20.0):
    """The CPU oracle's full LREI-RK4 step on the batched workload, bounded.

    Sample: one oracle RK4 step per trajectory, trajectories taken in order
    until `budget_s` seconds have been spent; the rate is scaled to the whole
    batch by the ratio of summed N*r (the oracle's work is linear in N*r at
    these sizes)."""
    from oracle.hamiltonian import Hamiltonian
    from oracle.schemes import lrei_rk_step
    done, nr_done, t_all = 0, 0, 0.0
    for t in trajs:
        H = Hamiltonian(t["n"], t["bonds"], t["J"], t["h"])
        t0 = time.perf_counter()
        lrei_rk_step(H, t["V"], t["lam"], t["model"], t["kappa"], 0.01, "RK4")
        t_all += time.perf_counter() - t0
        done += 1
        nr_done += (2 ** t["n"]) * t["lam"].size
        if t_all > budget_s:
            break
    nr_total = sum((2 ** t["n"]) * t["lam"].size for t in trajs)
    t_batch_step = t_all * nr_total / nr_done
    return {
        "value": len(trajs) / t_batch_step, "unit": "trajectory-steps/s", "cores": 1, "kind": "oracle",
        "sample": (f"oracle LREI-RK4 step (N-space Householder action, exact partial eigensolve) on "
                   f"{done} of {len(trajs)} trajectories, {t_all:.2f} s, scaled by summed N*r to the "
                   f"whole batch"),
    }


def run_rk_vs_ab(args, torch):
    """RK4 against AB4 step time (the paper's complexity comparison, Sec. 5).

    Triangular lattices (rows x cols = n, periodic), J = 1, DMI d = 0.4 along
    z, field 0.116 along x, q-LLG with kappa = 0.5, dt = 0.01, rank-3 start
    0.5 |AF1> + 0.3 |AF2> + 0.2 |GHZ>, mixed precision.  AB4 is timed after
    its three RK4 start-up steps."""
    from paper_2508_21200_amd import Context
    from workloads import triangular_lattice_bonds, af1_index, af2_index, ghz_vector, mixture_factor

    shapes = [(2, 5), (3, 4), (2, 7), (4, 4), (3, 6), (4, 5)]
    rows_out = []
    for rows, cols in shapes:
        n = rows * cols
        N = 2 ** n
        bonds = triangular_lattice_bonds(rows, cols, periodic=True)
        Jt = np.eye(3) + np.array([[0.0, 0.4, 0.0], [-0.4, 0.0, 0.0], [0.0, 0.0, 0.0]])
        J = np.repeat(Jt[None], bonds.shape[0], axis=0)
        h = np.tile([0.116, 0.0, 0.0], (n, 1))
        e1, e2 = np.zeros(N, complex), np.zeros(N, complex)
        e1[af1_index(n)] = 1.0
        e2[af2_index(n)] = 1.0
        lam, V = mixture_factor([e1, e2, ghz_vector(n)], [0.5, 0.3, 0.2])
        res = {"n": n, "lattice": f"{rows}x{cols} periodic triangular", "bonds": int(bonds.shape[0])}
        for scheme, warm in (("RK4", 2), ("AB4", 5)):
            c = Context(precision="mixed", autotune_cache=args.tune_cache)
            c.set_hamiltonian(n, bonds, J, h)
            c.set_rho(lam, V)
            c.step("qLLG", scheme, 0.01, 0.5, warm)
            c.synchronize()
            steps = 20
            a = time.perf_counter()
            c.step("qLLG", scheme, 0.01, 0.5, steps)
            c.synchronize()
            res[f"{scheme}_ms_per_step"] = round(1e3 * (time.perf_counter() - a) / steps, 4)
            c.close()
        res["RK4_over_AB4"] = round(res["RK4_ms_per_step"] / res["AB4_ms_per_step"], 3)
        rows_out.append(res)
        print(f"[rk-vs-ab] {json.dumps(res)}", file=sys.stderr, flush=True)
    print(json.dumps({"report": "LREI-RK4 vs LREI-AB4 step time", "model": "qLLG", "kappa": 0.5, "dt": 0.01,
                      "r": 3, "precision": "mixed", "rows": rows_out}))


def run_adaptive_report(args, torch):
    """Adaptive stepping against fixed-step RK4 at equal accuracy.

    Two workloads: the 4 x 5 periodic Heisenberg lattice (n = 20, r = 16,
    q-LL, kappa = 0.5, T = 0.16) and the 3 x 3 periodic triangular DMI lattice
    (J = 1, d = 0.4 along z, field 0.116 along x, pure |AF1> start, q-LLG,
    kappa = 0.5, T = 2: the damped dynamics slow down as the state relaxes).
    Error: relative Frobenius distance of rho(T) from FP64 fixed-step RK4 at
    a step 8 times below the finest one in the table.  Wall time of the whole
    call (adaptive: including its reads of the controller state)."""
    from paper_2508_21200_amd import Context
    from workloads import make_config, triangular_lattice_bonds, af1_index, pure_factor

    cfg = make_config(3)
    n = 9
    tb = triangular_lattice_bonds(3, 3, periodic=True)
    Jt = np.eye(3) + np.array([[0.0, 0.4, 0.0], [-0.4, 0.0, 0.0], [0.0, 0.0, 0.0]])
    tri = {"n": n, "bonds": tb, "J": np.repeat(Jt[None], tb.shape[0], axis=0), "h": np.tile([0.116, 0.0, 0.0], (n, 1)),
           "lam": np.array([1.0]), "V": pure_factor(n, index=af1_index(n))}
    loads = [("heisenberg_square4x5_n20_r16", cfg, "qLL", 0.16, [0.04, 0.02, 0.01], [1e-6, 1e-7, 1e-8, 1e-9],
              ["fp64", "mixed"]),
             ("triangular3x3_dmi_pure_af1", tri, "qLLG", 2.0, [0.1, 0.05, 0.025, 0.0125],
              [1e-4, 1e-5, 1e-6, 1e-7, 1e-8], ["fp64"])]
    rows = []
    for name, w, model, T, hs, tols, precs in loads:
        V0 = torch.from_numpy(np.ascontiguousarray(w["V"])).cuda()

        def ctx(prec):
            c = Context(precision=prec, autotune_cache=args.tune_cache)
            c.set_hamiltonian(w["n"], w["bonds"], w["J"], w["h"])
            c.set_rho(w["lam"], V0)
            return c

        href = hs[-1] / 8
        c = ctx("fp64")
        c.step(model, "RK4", href, 0.5, int(round(T / href)))
        Vref = c.get_rho(torch.empty_like(V0))[1].clone()
        c.close()
        for prec in precs:
            def record(method, param, fn):
                c = ctx(prec)
                # launch attributes and graph capture outside the timing
                if method == "RK4":
                    c.step(model, "RK4", param, 0.5, 1)
                else:
                    c.evolve_adaptive(model, 0.5, 1e-3, 1.0, 1e-3, h_min=1e-9, h_max=1.0, pair=method)
                c.set_rho(w["lam"], V0)
                c.synchronize()
                a = time.perf_counter()
                info = fn(c)
                c.synchronize()
                ms = 1e3 * (time.perf_counter() - a)
                err = rel_fro(torch, c.get_rho(torch.empty_like(V0))[1], Vref, w["lam"])
                c.close()
                row = {"workload": name, "precision": prec, "method": method, "param": param, "ms": round(ms, 2),
                       "rel_err": float(err)}
                row.update(info)
                rows.append(row)
                print(f"[adaptive] {json.dumps(row)}", file=sys.stderr, flush=True)

            for dt in hs:
                steps = int(round(T / dt))
                record("RK4", dt, lambda c, dt=dt, steps=steps: (c.step(model, "RK4", dt, 0.5, steps),
                                                                 {"steps": steps, "passes": 4 * steps})[1])
            for pair in ("RK43", "BS32", "HE21"):
                for tol in tols:
                    def run(c, tol=tol, pair=pair):
                        r = c.evolve_adaptive(model, 0.5, T, tol, hs[0] / 4, h_min=1e-9, h_max=T, pair=pair)
                        passes = {"RK43": 5, "BS32": 4, "HE21": 2}[pair] * r["attempts"]
                        return {"steps": r["accepted"], "rejected": r["rejected"], "passes": passes,
                                "status": r["status"]}
                    record(pair, tol, run)
    print(json.dumps({"report": "adaptive stepping vs fixed-step RK4", "kappa": 0.5, "rows": rows}))


def run_scaling_report(args, torch):
    """Step time against the number of spins and the rank (the paper's
    complexity test, Sec. 5): periodic triangular lattices, J = 1, DMI
    d = 0.4 along z, field 0.116 along x, q-LLG with kappa = 0.5, LREI-RK4,
    dt = 0.01, mixed precision; the rank-r start is the mixture of |AF1>,
    |AF2>, |GHZ>, |W> with weights (1), (0.75, 0.25), (0.5, 0.3, 0.2) or
    (0.4, 0.3, 0.2, 0.1), built on the device.  Per step: the RK4 step, the
    energy and magnetisation, and the two-spin state and concurrence of
    sites (0, 1)."""
    from paper_2508_21200_amd import Context, pair_entanglement
    from workloads import triangular_lattice_bonds, af1_index, af2_index

    weights = {1: [1.0], 2: [0.75, 0.25], 3: [0.5, 0.3, 0.2], 4: [0.4, 0.3, 0.2, 0.1]}
    shapes = [(3, 4), (4, 4), (4, 5), (4, 6), (2, 13), (4, 7)]
    rows_out = []
    for rows, cols in shapes:
        n = rows * cols
        N = 1 << n
        bonds = triangular_lattice_bonds(rows, cols, periodic=True)
        Jt = np.eye(3) + np.array([[0.0, 0.4, 0.0], [-0.4, 0.0, 0.0], [0.0, 0.0, 0.0]])
        J = np.repeat(Jt[None], bonds.shape[0], axis=0)
        h = np.tile([0.116, 0.0, 0.0], (n, 1))
        for r in (1, 2, 3, 4):
            lam = np.array(weights[r])
            V = torch.zeros((N, r), dtype=torch.complex128, device="cuda")
            V[af1_index(n), 0] = 1.0
            if r > 1:
                V[af2_index(n), 1] = 1.0
            if r > 2:
                V[0, 2] = V[N - 1, 2] = 2 ** -0.5
            if r > 3:
                V[torch.tensor([1 << i for i in range(n)], device="cuda"), 3] = n ** -0.5
            c = Context(precision="mixed", autotune_cache=args.tune_cache)
            c.set_hamiltonian(n, bonds, J, h)
            c.set_rho(lam, V)
            del V
            torch.cuda.empty_cache()
            c.step("qLLG", "RK4", 0.01, 0.5, 1)
            c.observables()
            c.pair_density([[0, 1]])
            c.synchronize()
            steps = 5 if n >= 24 else 20
            a = time.perf_counter()
            c.step("qLLG", "RK4", 0.01, 0.5, steps)
            c.synchronize()
            bare = 1e3 * (time.perf_counter() - a) / steps
            a = time.perf_counter()
            for _ in range(steps):
                c.step("qLLG", "RK4", 0.01, 0.5, 1)
                e, m = c.observables()
                conc = pair_entanglement(c.pair_density([[0, 1]])[0])[0]
            full = 1e3 * (time.perf_counter() - a) / steps
            c.close()
            res = {"n": n, "lattice": f"{rows}x{cols} periodic triangular", "bonds": int(bonds.shape[0]), "r": r,
                   "ms_per_step": round(bare, 3), "ms_per_step_with_observables": round(full, 3),
                   "energy": round(e, 6), "concurrence_01": round(conc, 6)}
            rows_out.append(res)
            print(f"[scaling] {json.dumps(res)}", file=sys.stderr, flush=True)
    print(json.dumps({"report": "LREI-RK4 q-LLG step time against n and r", "kappa": 0.5, "dt": 0.01,
                      "precision": "mixed", "rows": rows_out}))


def run_learned_report(args, torch):
    """Learned start rotation against the other eigensolve starts.

    Training data: RK4 stages of random XXZ chains (n = 14, r = 16, q-LLG,
    couplings as the n = 22 workload, damping log-uniform in [0.01, 0.5]),
    recorded by the library while stepping in FP64; the last tenth of the
    trajectories is held out.  Evaluation: the n = 22 chain (config 5), RK4,
    dt = 0.01, mixed precision, every start mode timed over the same steps and
    compared with the FP64 direct-solve run."""
    from paper_2508_21200_amd import Context, Net, net_sample_floats
    from workloads import make_config

    r, steps_per, n_traj = 16, args.train_steps, args.train_traj
    sf = net_sample_floats(r)
    buf = torch.zeros((4 * steps_per * n_traj, sf), dtype=torch.float32, device="cuda")
    rng = np.random.default_rng(2024)
    t0 = time.perf_counter()
    total, bounds = 0, []
    for t in range(n_traj):
        cfg = make_config(5, traj=1000 + t, n=14)
        kap = float(np.exp(rng.uniform(np.log(0.01), np.log(0.5))))
        c = Context(precision="fp64")
        c.set_hamiltonian(cfg["n"], cfg["bonds"], cfg["J"], cfg["h"])
        c.set_rho(cfg["lam"], cfg["V"])
        c.record(buf[total:])
        c.step("qLLG", "RK4", 0.01, kap, steps_per)
        total += c.record_count()
        bounds.append(total)
        c.close()
        if t % 20 == 0:
            print(f"[learned] recorded trajectory {t}: {total} samples", file=sys.stderr, flush=True)
    t_rec = time.perf_counter() - t0
    # trajectories split 80 / 10 / 10: training, validation (picks the step
    # size), held-out test
    n_tr, n_va = bounds[int(0.8 * n_traj) - 1], bounds[int(0.9 * n_traj) - 1]
    train, val, held = buf[:n_tr], buf[n_tr:n_va], buf[n_va:total]

    def excess(R, S):
        """mean of loss(R) - loss(polar(T)) over samples S (host)."""
        nin = 2 * r * r + 2
        t = S[:, nin:].astype(np.float64)
        T = (t[:, 0::2] + 1j * t[:, 1::2]).reshape(-1, r, r)
        U, _, Wh = np.linalg.svd(T)
        best = U @ Wh
        d = lambda A: np.einsum("kca,kca->ka", np.conj(A), T)  # (A* T)_aa
        return float(np.mean(np.sum(np.abs(d(best)) ** 2 - np.abs(d(R)) ** 2, axis=1)))

    Sh, Sv = held.cpu().numpy(), val.cpu().numpy()
    nin = 2 * r * r + 2
    I = np.eye(r)
    net = Net(r, seed=5)
    p0 = net.params()
    ex0 = excess(net.rotations(held), Sh)  # untrained: the analytic rotation
    t1 = time.perf_counter()
    sweep, best = [], None
    for lr in args.train_lr:
        net.set_params(p0)
        losses = net.train(train, batch=256, epochs=args.train_epochs, lr=lr, seed=9)
        ev = excess(net.rotations(val), Sv)
        sweep.append({"lr": lr, "validation_excess": ev, "epoch_loss_first_last": [float(losses[0]),
                                                                                   float(losses[-1])]})
        if best is None or ev < best[1]:
            best = (lr, ev, net.params())
    net.set_params(best[2])
    t_train = time.perf_counter() - t1
    training = {"samples": int(n_tr), "validation": int(n_va - n_tr), "held_out": int(total - n_va),
                "record_s": round(t_rec, 2), "train_s": round(t_train, 2), "epochs": args.train_epochs,
                "lr_sweep": sweep, "lr": best[0],
                "held_out_excess_loss": {"identity": excess(np.broadcast_to(I, (len(Sh), r, r)), Sh),
                                         "analytic": ex0,
                                         "network_trained": excess(net.rotations(held), Sh)}}
    print(f"[learned] trained: {json.dumps(training)}", file=sys.stderr, flush=True)
    if args.train_only:
        net.close()
        print(json.dumps({"report": "learned start rotation: training only", "training": training}))
        return

    cfg = make_config(5)
    model, dt, kappa, steps, warm_steps = cfg["model"], cfg["dt"], cfg["kappa"], cfg["steps"], 2

    def run(prec, warm):
        c = Context(precision=prec, warm=warm, autotune_cache=args.tune_cache)
        c.set_hamiltonian(cfg["n"], cfg["bonds"], cfg["J"], cfg["h"])
        c.set_rho(cfg["lam"], cfg["V"])
        if warm == "learned":
            c.attach_net(net)
        if not args.no_autotune:
            c.autotune()
        c.step(model, "RK4", dt, kappa, warm_steps)
        c.synchronize()
        s0 = c.stats()
        a = time.perf_counter()
        c.step(model, "RK4", dt, kappa, steps)
        c.synchronize()
        el = time.perf_counter() - a
        s1 = c.stats()
        V = c.get_rho()[1]
        c.close()
        de = {k: s1[k] - s0[k] for k in ("eigensolves", "warm_accepted", "warm_rejected", "warm_iterations")}
        return V, el, de

    Vref, el_ref, de_ref = run("fp64", "plain")
    modes = {"fp64_plain": {"ms_per_step": round(1e3 * el_ref / steps, 4), "steps_per_s": round(steps / el_ref, 2),
                            "eigensolves": de_ref["eigensolves"], "precision": "fp64",
                            "note": "the plain FP64 GPU path: direct solve, FP64 storage (the reference)"}}
    print(f"[learned] fp64_plain: {json.dumps(modes['fp64_plain'])}", file=sys.stderr, flush=True)
    for warm in ("plain", "analytic", "predict_identity", "predict_cayley", "learned"):
        V, el, de = run("mixed", warm)
        modes[warm] = {"ms_per_step": round(1e3 * el / steps, 4), "steps_per_s": round(steps / el, 2),
                       "eigensolves": de["eigensolves"], "warm_accepted": de["warm_accepted"],
                       "warm_rejected": de["warm_rejected"],
                       "block_products_per_warm_solve": round(
                           de["warm_iterations"] / max(1, de["warm_accepted"] + de["warm_rejected"]), 3),
                       "rel_fro_vs_fp64_plain": rel_fro(torch, V, Vref, cfg["lam"])}
        print(f"[learned] {warm}: {json.dumps(modes[warm])}", file=sys.stderr, flush=True)
    net.close()
    print(json.dumps({"report": "learned start rotation vs plain start",
                      "workload": {"name": cfg["name"], "n": cfg["n"], "N": 2 ** cfg["n"], "r": cfg["r"],
                                   "model": model, "kappa": kappa, "scheme": "RK4", "dt": dt,
                                   "timed_steps": steps, "warmup_steps": warm_steps, "precision": "mixed"},
                      "training": training, "modes": modes}))


def batch_trajectories():
    """The batched workload's 64 trajectories (inputs only)."""
    from workloads import make_config, CONFIGS
    base = CONFIGS[4]
    trajs = []
    for t in range(base["n_traj"]):
        c = make_config(4, traj=t)
        trajs.append(dict(n=c["n"], bonds=c["bonds"], J=c["J"], h=c["h"], lam=c["lam"], V=c["V"],
                          model=c["model"], kappa=c["kappa"]))
    return base, trajs


def measure_batch(args, torch, precision, steps, warmup, n_oracle=2):
    """The batched workload: 64 independent XXZ-chain trajectories (n 12..16,
    r in {4, 8, 16}, half q-LL / half q-LLG, kappa log-uniform in [0.01, 1]),
    LREI-RK4 dt = 0.01, advanced together.  Returns the measured rate, the
    worst error of the `n_oracle` smallest trajectories against the CPU oracle
    (the same warmup + timed steps), the worst distance of every trajectory
    from the FP64 batch, and the rates of the FP64 batch and of the plain FP64
    path (each trajectory in its own single FP64 context, one after another)."""
    from paper_2508_21200_amd import Batch, Context
    base, trajs = batch_trajectories()
    dt, scheme = base["dt"], base["scheme"]
    b = Batch(trajs, precision=precision)
    print(f"[bench] workload {base['name']} precision={precision} warmup={warmup} steps={steps}",
          file=sys.stderr, flush=True)
    tune = None
    if not args.no_autotune:
        tune = b.autotune(iters=10)
        print(f"[bench] batch H.V shapes: {tune['ms_default']:.4f} -> {tune['ms']:.4f} ms per pass, "
              f"{tune['choice']}", file=sys.stderr, flush=True)
    if warmup > 0:
        b.step(scheme, dt, warmup)
    b.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(scheme, dt, steps)
    b.synchronize()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    print(f"[bench] batch: timed {steps} steps in {elapsed:.4f} s", file=sys.stderr, flush=True)
    out = {"elapsed": elapsed, "trajs": trajs, "base": base}
    if tune is not None:
        out["hv_tuning"] = {"ms_default": round(tune["ms_default"], 5), "ms": round(tune["ms"], 5),
                            "choice": {str(r): c for r, c in tune["choice"].items()},
                            "tried": len(tune["tried"]),
                            "note": "one batched pass + its reduction, every rank class (lrei_batch_autotune)"}
    if args.profile_only:
        return out
    out["kernels_ms"] = b.profile_kernels(scheme, dt, iters=20)
    elem = 8 if precision == "mixed" else 16
    nr_total = sum((2 ** t["n"]) * t["lam"].size for t in trajs)
    out["hv_bytes"] = 2 * nr_total * elem  # read P_j, write P_{j+1}, every trajectory
    out["nr_total"] = nr_total
    if args.no_parity:
        b.close()
        return out
    # the smallest trajectories' results, for the comparison with the CPU
    # oracle (batch_oracle_parity, run once the CPU is free)
    order = sorted(range(len(trajs)), key=lambda q: (2 ** trajs[q]["n"]) * trajs[q]["lam"].size)[:n_oracle]
    out["for_oracle"] = {"order": order, "V": {q: b.get_rho(q)[1] for q in order}, "steps": warmup + steps,
                         "dt": dt, "scheme": scheme}
    if precision == "mixed":
        ref = Batch(trajs, precision="fp64")
        if not args.no_autotune:
            ref.autotune(iters=10)
        if warmup > 0:
            ref.step(scheme, dt, warmup)
        ref.synchronize()
        t1 = time.perf_counter()
        ref.step(scheme, dt, steps)
        ref.synchronize()
        t_fp64_batch = time.perf_counter() - t1
        worst = 0.0
        for q, t in enumerate(trajs):
            worst = max(worst, rel_fro(torch, b.get_rho(q)[1], ref.get_rho(q)[1], t["lam"]))
        ref.close()
        # the plain FP64 GPU path: one single-trajectory context per
        # trajectory, stepped one after the other (same steps, graphs warm)
        plain = []
        for t in trajs:
            c = Context(precision="fp64", autotune_cache=args.tune_cache)
            c.set_hamiltonian(t["n"], t["bonds"], t["J"], t["h"])
            c.set_rho(t["lam"], t["V"])
            c.step(t["model"], scheme, dt, t["kappa"], max(warmup, 1))
            plain.append(c)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for q, t in enumerate(trajs):
            plain[q].step(t["model"], scheme, dt, t["kappa"], steps)
        for c in plain:
            c.synchronize()
        t_plain = time.perf_counter() - t1
        for c in plain:
            c.close()
        n = len(trajs) * steps
        out["vs_fp64"] = {"vs": "FP64 GPU batch, same inputs and step count", "rel_fro_worst_trajectory": worst}
        out["compare"] = {"plain_fp64_single_contexts_traj_steps_per_s": round(n / t_plain, 1),
                          "fp64_batch_traj_steps_per_s": round(n / t_fp64_batch, 1),
                          "mixed_batch_over_plain_fp64": round(t_plain / elapsed, 2),
                          "mixed_batch_over_fp64_batch": round(t_fp64_batch / elapsed, 2),
                          "note": "the plain path runs each trajectory in its own FP64 context, one after the "
                                  "other; the FP64 batch is this launch packing in FP64 storage"}
    b.close()
    return out


def batch_oracle_parity(m):
    """The smallest trajectories of a measured batch against the CPU oracle
    (same inputs, same total step count); numpy's BLAS is held to one thread
    for these small problems."""
    if "for_oracle" not in m:
        return
    from threadpoolctl import threadpool_limits
    from oracle.hamiltonian import Hamiltonian
    from oracle.schemes import run as oracle_run
    from oracle.metrics import rel_fro_error
    fo, trajs = m["for_oracle"], m["trajs"]
    worst, t0 = 0.0, time.perf_counter()
    with threadpool_limits(limits=1):
        for q in fo["order"]:
            t = trajs[q]
            H = Hamiltonian(t["n"], t["bonds"], t["J"], t["h"])
            Vo = oracle_run(H, t["V"], t["lam"], t["model"], t["kappa"], fo["dt"], fo["steps"], fo["scheme"])
            worst = max(worst, rel_fro_error(fo["V"][q], t["lam"], Vo, t["lam"]))
    m["oracle"] = {"vs": "oracle", "trajectories": [dict(index=q, n=trajs[q]["n"], r=int(trajs[q]["lam"].size),
                                                         model=trajs[q]["model"]) for q in fo["order"]],
                   "steps": fo["steps"], "rel_fro_worst": worst, "oracle_s": round(time.perf_counter() - t0, 2),
                   "note": "the smallest trajectories of the batch (by N r) against the CPU complex128 oracle; "
                           "bound 1e-5 (mixed), 1e-10 (FP64)"}


def batch_summary(m, precision, steps):
    """The batch measurement as a sub-object of a bench line."""
    n = len(m["trajs"]) * steps
    res = {"metric": "LREI trajectory-steps/s (64 batched trajectories)",
           "value": n / m["elapsed"], "unit": "trajectory-steps/s", "steps": steps,
           "ms_per_step": 1e3 * m["elapsed"] / steps, "precision": precision,
           "workload": m["base"]["name"]}
    if "kernels_ms" in m:
        kms = m["kernels_ms"]
        ach = m["hv_bytes"] / (kms["hv_pass"] * 1e-3) / 1e9
        res["hv_pass"] = {"ms": round(kms["hv_pass"], 5), "algorithmic_bytes": m["hv_bytes"],
                          "GBs": round(ach, 1), "frac_of_hbm_peak": round(ach / HBM_PEAK_GBS, 4),
                          "model": "2 sum_t N_t r_t c per pass (read P_j, write P_{j+1})"}
        res["kernels_ms"] = {k: round(v, 5) for k, v in kms.items()}
    if "hv_tuning" in m:
        res["hv_tuning"] = m["hv_tuning"]
    for k in ("oracle", "vs_fp64", "compare"):
        if k in m:
            res[{"oracle": "parity", "vs_fp64": "vs_fp64_batch", "compare": "vs_plain_fp64"}[k]] = m[k]
    return res


def run_batch(args, torch):
    """Prints the bench line of the batched workload (--config 4)."""
    precision = args.precision or "mixed"
    steps = args.steps
    m = measure_batch(args, torch, precision, steps, args.warmup)
    if args.profile_only:
        print(json.dumps({"steps": steps, "ms_per_step": 1e3 * m["elapsed"] / steps}))
        return
    batch_oracle_parity(m)
    trajs, base = m["trajs"], m["base"]
    summ = batch_summary(m, precision, steps)
    cpu = None if args.no_cpu_baseline else cpu_baseline_batch(trajs)
    rs = sorted({t["lam"].size for t in trajs})
    line = {
        "metric": summ["metric"],
        "value": summ["value"],
        "unit": "trajectory-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": summ["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64+f64" if precision == "mixed" else "c128",
        "data": "synthetic",
        "config": {"workload": base["name"], "n_traj": len(trajs), "n_range": [12, 16], "r_values": rs,
                   "sum_N_r": m["nr_total"], "scheme": base["scheme"], "dt": base["dt"], "precision": precision,
                   "models": "q-LL (even trajectories), q-LLG (odd)", "lattice": "open XXZ chains"},
        "roofline": {"bound": "hbm", "achieved": summ["hv_pass"]["GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": summ["hv_pass"]["frac_of_hbm_peak"], "traffic": None,
                     "kernel": "k_hv_batch (all trajectories' H.V passes, fused Grams)",
                     "algorithmic_bytes_per_launch": m["hv_bytes"]},
        "cpu_baseline": cpu,
        "parity": summ.get("parity"),
        "vs_fp64_batch": summ.get("vs_fp64_batch"),
        "vs_plain_fp64": summ.get("vs_plain_fp64"),
        "kernels_ms": summ.get("kernels_ms"),
        "hv_tuning": summ.get("hv_tuning"),
    }
    print(json.dumps(line))


def main():
    args = parse()
    if args.oracle_child:
        oracle_child(args)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "requested_gpus": args.gpus}))
        sys.exit(2)
    t_main = time.perf_counter()
    single = not (args.copy_calibration or args.config == 4 or args.learned_report or args.rk_vs_ab or
                  args.adaptive_report or args.scaling_report or args.kernels_only or args.profile_only)
    # the oracle's step runs beside the GPU work (it takes minutes at n = 20)
    from workloads.configs import CONFIGS
    rk = args.config in CONFIGS and CONFIGS[args.config]["scheme"].startswith("RK")
    oracle = OracleStep(args) if single and rk and not (args.no_cpu_baseline and args.no_parity) else None
    import torch
    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nbytes, "launches": 5}))
        return
    if args.config == 4:
        run_batch(args, torch)
        return
    if args.learned_report:
        run_learned_report(args, torch)
        return
    if args.rk_vs_ab:
        run_rk_vs_ab(args, torch)
        return
    if args.adaptive_report:
        run_adaptive_report(args, torch)
        return
    if args.scaling_report:
        run_scaling_report(args, torch)
        return
    from paper_2508_21200_amd import Context
    from workloads import make_config

    cfg = make_config(args.config)
    precision = args.precision or ("fp64" if cfg["precision"] == "fp64" else "mixed")
    scheme = cfg["scheme"]
    model = cfg["model"]
    dt, kappa = cfg["dt"], cfg["kappa"]
    one_step = scheme.startswith("RK")  # the oracle comparison takes one step from the initial state

    def make_ctx(prec):
        c = Context(device=0, precision=prec, autotune_cache=args.tune_cache)
        c.set_hamiltonian(cfg["n"], cfg["bonds"], cfg["J"], cfg["h"])
        c.set_rho(cfg["lam"], cfg["V"])
        return c

    ctx = make_ctx(precision)
    tuning = None if args.no_autotune else ctx.autotune()  # launch shape of the H.V pass, outside the timed region
    if args.kernels_only:
        ctx.step(model, scheme, dt, kappa, 1)  # the per-kernel launches reuse the step's buffers
        kms = ctx.profile_kernels(model, scheme, dt, kappa, iters=20)
        print(json.dumps({"kernels_ms": kms}))
        return
    V1_gpu = {}
    if not args.no_parity and one_step:
        ctx.step(model, scheme, dt, kappa, 1)
        V1_gpu[precision] = ctx.get_rho()[1]
        ctx.set_rho(cfg["lam"], cfg["V"])  # back to the initial state (same rank: the tuned shape stays)

    def timed_run(c, prec):
        print(f"[bench] workload {cfg['name']} precision={prec} warmup={args.warmup} steps={args.steps}",
              file=sys.stderr, flush=True)
        if args.warmup > 0:
            c.step(model, scheme, dt, kappa, args.warmup)
        torch.cuda.synchronize()
        c.synchronize()
        t0 = time.perf_counter()
        c.step(model, scheme, dt, kappa, args.steps)
        c.synchronize()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        print(f"[bench] {prec}: timed {args.steps} steps in {el:.4f} s", file=sys.stderr, flush=True)
        return el

    elapsed = timed_run(ctx, precision)
    stats = ctx.stats()
    if args.profile_only:
        print(json.dumps({"steps": args.steps, "ms_per_step": 1e3 * elapsed / args.steps}))
        return

    kms = ctx.profile_kernels(model, scheme, dt, kappa, iters=20)
    elem = 8 if precision == "mixed" else 16
    F = (2 ** cfg["n"]) * cfg["r"] * elem
    hv_bytes = 2 * F  # algorithmic: read P_j once, write P_{j+1} once (partner rows are re-reads of P_j)
    achieved = hv_bytes / (kms["hv_pass"] * 1e-3) / 1e9
    traffic = None
    tfile = os.path.join(ROOT, "profiles", "hv_pass_traffic.json")
    if os.path.exists(tfile):
        try:
            with open(tfile) as f:
                t = json.load(f)
            if (t.get("precision") == precision and t.get("workload") == cfg["name"]
                    and t.get("source_digest") == source_digest()):
                traffic = t.get("bytes_per_launch")
        except Exception:
            traffic = None
    copy = measured_copy_gbs(torch)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "traffic_over_algorithmic": None if traffic is None else round(traffic / hv_bytes, 3),
                "kernel": ("k_hv_tile" if (tuning or {}).get("tile_bits") else
                           "k_hv (compacted gathers)" if (tuning or {}).get("compact") else "k_hv"),
                "algorithmic_bytes_per_launch": hv_bytes,
                "algorithmic_model": "2F per pass, F = N r c (read P_j, write P_{j+1})",
                "measured_copy_peak": copy, "frac_of_copy_peak": round(achieved / copy["GBs"], 4)}

    # the FP64 path on the same workload: its rate, its one-step result, and
    # the mixed run's distance from it after the timed steps
    fp64 = None
    V_end = ctx.get_rho()[1]
    if precision == "mixed" and not args.no_parity:
        ref = make_ctx("fp64")
        if one_step:
            ref.step(model, scheme, dt, kappa, 1)
            V1_gpu["fp64"] = ref.get_rho()[1]
            ref.set_rho(cfg["lam"], cfg["V"])
        el64 = timed_run(ref, "fp64")
        _, Vr = ref.get_rho()
        fp64 = {"steps_per_s": args.steps / el64, "ms_per_step": 1e3 * el64 / args.steps,
                "mixed_over_fp64": round(el64 / elapsed, 3),
                "mixed_vs_fp64_after_timed_steps": rel_fro(torch, V_end, Vr, cfg["lam"]),
                "note": "FP64 GPU path (complex FP64 N-space passes), same inputs, warmup and steps; the "
                        "distance is after warmup + timed steps"}
        ref.close()

    # two-spin reduced density matrices of 64 site pairs in one call (one fused
    # pass over the state per pair; algorithmic bytes F per pair)
    pairs = [(k, l) for k in range(cfg["n"]) for l in range(cfg["n"]) if k != l][:64]
    ctx.pair_density(pairs)
    t2 = time.perf_counter()
    for _ in range(5):
        ctx.pair_density(pairs)
    t_pairs = (time.perf_counter() - t2) / 5
    pair_obs = {"pairs": len(pairs), "ms_per_call": round(1e3 * t_pairs, 4),
                "algorithmic_GBs": round(len(pairs) * F / t_pairs / 1e9, 1),
                "note": "host wall clock of the synchronous ABI call (upload of the pair list, passes, "
                        "reduction, copy-back)"}

    # the batched workload, measured while the oracle step finishes
    bm = None
    if args.config == 3:
        bm = measure_batch(args, torch, "mixed" if precision == "mixed" else "fp64", args.steps, args.warmup)

    cpu = None
    parity = None
    if oracle is not None:
        V1_o, cpu = oracle.wait(args.oracle_deadline, t_main)
        oracle.cleanup()
        if V1_o is not None:
            from oracle.metrics import rel_fro_error
            parity = {"vs": "oracle", "steps": 1,
                      "note": "one step from the workload's initial state, GPU against the CPU complex128 oracle; "
                              "bounds: mixed 1e-5, FP64 1e-10"}
            for prec, Vg in V1_gpu.items():
                parity[f"rel_fro_{prec}"] = rel_fro_error(Vg, cfg["lam"], V1_o, cfg["lam"])
        elif V1_gpu:
            parity = {"vs": "oracle", "steps": 1, "rel_fro_mixed": None, "rel_fro_fp64": None,
                      "note": "the oracle step did not complete: " + cpu["sample"]}
    batch = None
    if bm is not None:
        batch_oracle_parity(bm)  # after the oracle step: the CPU is free again
        batch = batch_summary(bm, "mixed" if precision == "mixed" else "fp64", args.steps)
    line = {
        "metric": "LREI steps/s (n=20, r=16)" if args.config == 3 else f"LREI steps/s ({cfg['name']})",
        "value": args.steps / elapsed,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64+f64" if precision == "mixed" else "c128",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "n": cfg["n"], "N": 2 ** cfg["n"], "r": cfg["r"],
                   "model": model, "kappa": kappa, "scheme": scheme, "dt": dt, "precision": precision,
                   "lattice": "4x5 periodic square, 40 bonds" if args.config == 3 else "chain"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity": parity,
        "fp64_path": fp64,
        "kernels_ms": {k: round(v, 5) for k, v in kms.items()},
        "pair_density": pair_obs,
        "batch": batch,
        "hv_tuning": None if tuning is None else {
            "epl": tuning["epl"], "grid": tuning["grid"], "tile_bits": tuning["tile_bits"],
            "tile_waves": tuning["tile_waves"], "ms": round(tuning["ms"], 5),
            "tried": [[e, g, tile, round(t, 5)] for (e, g, w, t), tile in zip(tuning["tried"], tuning["tried_tile"])],
            "compact": tuning.get("compact"), "overlap_grid": tuning.get("overlap_grid"),
            "tried_fields": "columns per lane, workgroups, variant (0: untiled, 1: untiled with compacted "
                            "gathers, 100 tile_bits + waves: tiled), ms"},
        "eig_stats": {k: stats[k] for k in ("eigensolves", "warm_accepted", "warm_rejected", "warm_iterations",
                                            "dropped_directions", "min_pivot_ratio", "ortho_error")},
        "projected_phase_ms_per_step": dict(zip(
            ["gram_setup", "cholesky", "r_inverse", "h_apply", "householder", "stage_matrix", "eigensolve", "tail"],
            [round(v / args.steps, 4) for v in stats["phase_ms"]])),
        "eigensolve_parts_ms_per_step": dict(zip(
            ["tridiagonalisation", "multisection", "inverse_iteration", "back_transform",
             "warm_solver", "warm_ritz_step"],
            [round(v / args.steps, 4) for v in stats["eig_phase_ms"]])),
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
