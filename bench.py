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
H.V pass), `cpu_baseline` (the CPU oracle on a bounded sample), `parity`
(relative Frobenius error of the timed run against the FP64 GPU path on the
same inputs), `kernels_ms` (per-kernel averages).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=3)
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
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="run a plain device-to-device copy of MIB MiB five times and exit "
                         "(reference kernel for scaling FETCH_SIZE / WRITE_SIZE counters)")
    return ap.parse_args()


def source_digest():
    """Digest of the N-space kernel source; a stored traffic figure is only used while it matches."""
    import hashlib
    with open(os.path.join(ROOT, "paper_2508_21200_amd", "csrc", "nspace.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def cpu_baseline(cfg, n_rows=1 << 17, repeats=4):
    """The CPU oracle timed on a bounded sample of the same workload.

    Sample: the oracle's matrix-free H.V (Pauli-string gather) evaluated on
    `n_rows` random rows of the n=20, r=16 state, `repeats` times (the four
    RK4 stages), scaled to all N rows.  The oracle's Householder action and
    partial eigensolves are not included, so its true step rate is lower.
    """
    from oracle.hamiltonian import apply_H_rows
    N = 2 ** cfg["n"]
    rows = np.random.default_rng(0).choice(N, size=n_rows, replace=False)
    t0 = time.perf_counter()
    for _ in range(repeats):
        apply_H_rows(cfg["n"], cfg["bonds"], cfg["J"], cfg["h"], cfg["V"], rows)
    t = time.perf_counter() - t0
    t_step = t * (N / n_rows)
    return {
        "value": 1.0 / t_step, "unit": "steps/s", "cores": 1, "kind": "oracle",
        "sample": (f"oracle H.V on {n_rows} random rows x {repeats} (one per RK4 stage) of the "
                   f"n={cfg['n']} r={cfg['r']} state, scaled x{N // n_rows} to all rows; "
                   f"excludes the oracle's Householder and eigensolve work, so the true oracle "
                   f"step rate is lower; measured {t:.2f} s, numpy single-threaded gathers"),
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "requested_gpus": args.gpus}))
        sys.exit(2)
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
    from paper_2508_21200_amd import Context
    from workloads import make_config

    cfg = make_config(args.config)
    precision = args.precision or ("fp64" if cfg["precision"] == "fp64" else "mixed")
    scheme = cfg["scheme"]
    model = cfg["model"]
    dt, kappa = cfg["dt"], cfg["kappa"]

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
    print(f"[bench] workload {cfg['name']} precision={precision} warmup={args.warmup} "
          f"steps={args.steps}", file=sys.stderr, flush=True)
    if args.warmup > 0:
        ctx.step(model, scheme, dt, kappa, args.warmup)
    torch.cuda.synchronize()
    ctx.synchronize()
    t0 = time.perf_counter()
    ctx.step(model, scheme, dt, kappa, args.steps)
    ctx.synchronize()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    print(f"[bench] timed {args.steps} steps in {elapsed:.4f} s", file=sys.stderr, flush=True)
    stats = ctx.stats()
    if args.profile_only:
        print(json.dumps({"steps": args.steps, "ms_per_step": 1e3 * elapsed / args.steps}))
        return

    kms = ctx.profile_kernels(model, scheme, dt, kappa, iters=20)
    elem = 8 if precision == "mixed" else 16
    F = (2 ** cfg["n"]) * cfg["r"] * elem
    hv_bytes = 3 * F  # read P_j, read P_{j-1}, write P_{j+1}
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
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "k_cheb (H.V Chebyshev pass, fused Grams)",
                "algorithmic_bytes_per_launch": hv_bytes}

    parity = None
    if not args.no_parity:
        _, Vt = ctx.get_rho()
        if precision == "fp64":
            parity = {"vs": "self (fp64)", "rel_fro": 0.0}
        else:
            from oracle.metrics import rel_fro_error
            ref = make_ctx("fp64")
            ref.step(model, scheme, dt, kappa, args.warmup + args.steps)
            _, Vr = ref.get_rho()
            parity = {"vs": "FP64 GPU path, same inputs and step count",
                      "rel_fro": rel_fro_error(Vt, cfg["lam"], Vr, cfg["lam"])}
            ref.close()

    cpu = None if args.no_cpu_baseline else cpu_baseline(cfg)
    line = {
        "metric": "LREI steps/s (n=20, r=16)",
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
        "kernels_ms": {k: round(v, 5) for k, v in kms.items()},
        "hv_tuning": None if tuning is None else {
            "epl": tuning["epl"], "grid": tuning["grid"], "win_bits": tuning["win_bits"],
            "n_sweeps": tuning["n_sweeps"], "ms": round(tuning["ms"], 5),
            "tried": [[e, g, w, round(t, 5)] for e, g, w, t in tuning["tried"]]},
        "eig_stats": {k: stats[k] for k in ("eigensolves", "jacobi_sweeps", "max_sweeps_one_solve",
                                            "dropped_directions", "min_pivot_ratio", "ortho_error")},
        "projected_phase_ms_per_step": dict(zip(
            ["gram_setup", "cholesky", "r_inverse", "h_apply", "householder", "stage_matrix", "eigensolve", "tail"],
            [round(v / args.steps, 4) for v in stats["phase_ms"]])),
        "eigensolve_parts_ms_per_step": dict(zip(
            ["tridiagonalisation", "multisection", "inverse_iteration", "back_transform",
             "tridiag_Av", "tridiag_update"],
            [round(v / args.steps, 4) for v in stats["eig_phase_ms"]])),
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
