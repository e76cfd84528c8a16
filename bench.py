"""Benchmark of the MI355X ADMM / associative-scan QP solver.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload quadruped]

A step is one complete QP solve (every factor epoch and every ADMM
iteration, cold start z = y = 0, rho_0 = 1, OSQP-style rho adaptation) to a
primal and dual residual of 1e-5, on a problem whose data is already resident
in device memory (set up before the timed region).  The default workload is
the quadruped-shaped time-varying QP: nx = 61, nu = 12, N = 128, 40 polytopic
rows per stage.  Prints one JSON line.

The line carries
  * value      solves/s over the K timed steps;
  * roofline   for the dominant kernel (the persistent ADMM iteration kernel):
               algorithmic bytes of one cached iteration (each stage's fixed
               operators read once per direction) times its iterations, over
               its device time measured with HIP events on its stream;
  * cpu_baseline  the FP64 CPU oracle (sequential Riccati ADMM, one thread) on
               a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "QP solves/s and ms/solve at 1e-5 residual; warm-start vs cold-start ADMM"
HBM_PEAK_GBS = 8000.0
TOL = 1e-5


def floor_bytes(p, word=4):
    """Algorithmic bytes of one cached ADMM iteration: every stage's fixed
    operators (Abar twice -- backward and forward -- B and K both ways, Gamma,
    C and D) read once, plus the terminal rows."""
    N, nx, nu, nc, nf = p.N, p.nx, p.nu, p.nc, p.nf
    return word * (N * (2 * nx * nx + 3 * nx * nu + nu * nu + nc * (nx + nu)) + nf * nx)


def make_workload(name):
    from paper_2604_07644_amd import workloads as W
    if name == "quadruped":
        p = W.quadruped_qp(0)
        desc = "quadruped-shaped time-varying LQ QP, nx=61 nu=12 N=128, 40 polytopic rows/stage"
    elif name == "box":
        p = W.box_lq()
        desc = "box-constrained LQ QP, nx=4 nu=2 N=32"
    elif name == "humanoid":
        p = W.humanoid_qp(0)
        desc = "humanoid-shaped LQ QP, nx=75 nu=19 N=2048, 40 polytopic rows/stage"
    else:
        raise SystemExit(f"unknown workload {name}")
    return p, desc


def cpu_baseline(p, budget_s=10.0):
    import oracle
    t0 = time.perf_counter()
    n = 0
    iters = []
    while True:
        r = oracle.qp_solve(p, rho=1.0, tol=TOL)
        iters.append(r["iters"])
        n += 1
        el = time.perf_counter() - t0
        if (el >= budget_s and n >= 2) or n >= 200:
            break
    return dict(value=n / el, unit="solves/s", cores=1, kind="oracle",
                sample=f"{n} cold-start solves of the same QP at tol {TOL:g} "
                       f"(FP64 sequential Riccati ADMM, {int(np.median(iters))} iterations each)",
                ms_per_solve=1e3 * el / n)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="quadruped")
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=10.0)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch
    from paper_2604_07644_amd import gsls

    p, desc = make_workload(args.workload)
    prec = gsls.MIXED if args.precision == "mixed" else gsls.FP64
    stream = torch.cuda.current_stream().cuda_stream
    q = gsls.QP(p, gsls.default_settings(precision=prec), stream=stream)
    for _ in range(args.warmup):
        q.solve(rho=1.0, tol=TOL)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = []
    for _ in range(args.steps):
        res.append(q.solve(rho=1.0, tol=TOL))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    _, lay = q.phase_cycles()
    q.close()

    ok = all(r["status"] == gsls.SOLVED for r in res)
    iters = [r["iterations"] for r in res]
    ms_iter = float(np.mean([r["ms_iterate"] for r in res]))
    ms_fact = float(np.mean([r["ms_factor"] for r in res]))
    launches = float(np.mean([r["rho_updates"] + 1 for r in res]))
    word = 4 if prec == gsls.MIXED else 8
    bytes_per_iter = floor_bytes(p, word)
    mean_iters = float(np.mean(iters))
    achieved = bytes_per_iter * mean_iters / (ms_iter * 1e-3) / 1e9
    line = {
        "metric": METRIC,
        "value": args.steps / wall,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if prec == gsls.MIXED else "f64",
        "data": "synthetic (seeded generator; no robot models or datasets)",
        "config": {"workload": desc, "tol": TOL, "start": "cold", "rho0": 1.0,
                   "precision": args.precision, "iterations": int(np.median(iters)),
                   "rho_updates": int(np.median([r["rho_updates"] for r in res])),
                   "all_solved": ok, "ms_factor_per_solve": ms_fact, "ms_iterate_per_solve": ms_iter,
                   "chunks": {"factor": lay[0], "iteration": lay[1], "lds_resident": lay[2], "max_chunk": lay[3]}},
        "roofline": {"kernel": "k_admm (persistent ADMM iteration)", "bound": "hbm",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_iteration": bytes_per_iter, "iterations_per_launch": mean_iters / launches,
                     "avg_launch_ms": ms_iter / launches},
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(p, args.cpu_budget)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
