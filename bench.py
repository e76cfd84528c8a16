"""Benchmark of the MI355X ADMM / associative-scan QP solver.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload batch]

Default workload (the headline metric, warm-start vs cold-start ADMM): the
uneven batch of 512 box-constrained LTV-QPs (nx in {12,36,61,75}, nu in
{4,12,19}, N ~ U{16..512}) solved to a primal and dual residual of 1e-5 in one
graph-replayed persistent launch.  A step is one whole batch: the K timed
steps are run from a cold start (z = y = 0, rho = 1) and then from the learned
warm start (prediction included); value is the warm-start solves/s and the
cold-start figures sit beside it.  Problem data are resident in device memory
before the timed region.

Other workloads (--workload): quadruped | box | humanoid | long (one QP per
step, cold start), sls, robust, sqp.

The line carries
  * value      solves/s over the K timed steps;
  * roofline   for the dominant kernel: algorithmic (floor) bytes of the
               iterations it ran -- each stage's fixed operators read once per
               direction -- over its device time measured with HIP events on
               its stream;
  * cpu_baseline  the FP64 CPU oracle on a bounded sample of the same workload
               (the batch: built for the host, OpenMP over the instances).
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

# HBM bytes per launch (averaged over the launches of a run), from rocprofv3
# FETCH_SIZE and WRITE_SIZE runs scaled by the same counters on a 256 MiB
# device copy in the same process (profiles/*_hbm_traffic.md).  Valid only for
# the kernel sources they were taken on: reported while the hash of those
# sources matches.
K_ADMM_TRAFFIC = {
    "quadruped": {"src_sha256_16": "68ef4925e7ba47bb", "sources": ("iterate.hip", "dev_common.hpp", "solver.hpp"),
                  "bytes_per_launch": 1.9077e8},
    "humanoid": {"src_sha256_16": "68ef4925e7ba47bb", "sources": ("iterate.hip", "dev_common.hpp", "solver.hpp"),
                 "bytes_per_launch": 1.4470e10},
}
# The same for k_batch on the 512-instance batch (learned warm start, predicted rho0).
K_BATCH_TRAFFIC = {"src_sha256_16": "66f29ffb6c8faca7", "sources": ("batch.hip", "batch.hpp", "dev_common.hpp"),
                   "bytes_per_launch": 1.1720e12}


def kernel_traffic(entry):
    if not entry.get("bytes_per_launch"):
        return None
    import hashlib
    h = hashlib.sha256()
    for s in entry["sources"]:
        with open(os.path.join(ROOT, "paper_2604_07644_amd", "csrc", s), "rb") as f:
            h.update(f.read())
    return entry["bytes_per_launch"] if h.hexdigest()[:16] == entry["src_sha256_16"] else None
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
    elif name == "long":
        p = W.pendulum_like(N=3000, links=15)
        desc = ("15-link-pendulum-shaped LTV-QP, nx=30 nu=15 N=3000 (135,000 variables), torque box, "
                "tol 1e-2 as in the paper's long-horizon study")
        return p, desc, 1e-2
    else:
        raise SystemExit(f"unknown workload {name}")
    return p, desc, TOL


def sls_flops(p):
    """Algorithmic FP32 flops of one SLS instance: per (column j, stage k > j)
    the Riccati step Z = [A|B]^T P [A|B] + G^T diag(tau) G, K = -Z_uu^{-1} Z_ux,
    P = Z_xx + Z_ux^T K, and the forward step Phi^u = K Phi^x, margins
    G [Phi^x; Phi^u], Phi^x' = [A|B] [Phi^x; Phi^u]; plus the terminal terms."""
    N, nx, nu, nc, nf = p.N, p.nx, p.nu, p.nc, p.nf
    nxu = nx + nu
    bwd = 2 * nx * nx * nxu + 2 * nxu * nxu * nx + 2 * nxu * nxu * nc + 2 * nu * nu * nx + 2 * nx * nx * nu
    fwd = 2 * nu * nx * nx + 2 * nc * nxu * nx + 2 * nx * nxu * nx
    steps = N * (N - 1) // 2
    return steps * (bwd + fwd) + N * (2 * nx * nx * nf + 2 * nf * nx * nx)


def bench_sls(args):
    """SLS batch: 64 quadruped-shaped instances (nx=61, nu=12, N=64, 40 rows),
    tau from each instance's nominal ADMM multipliers (App. B), |w|_inf <= 0.01."""
    import torch
    from paper_2604_07644_amd import gsls, workloads as W
    count = 64
    probs, E, wb = W.sls_batch(count)
    p0 = probs[0]
    Qb, Rb, QbN = np.eye(p0.nx), np.eye(p0.nu), np.eye(p0.nx)
    q = gsls.QP(p0, gsls.default_settings(precision=gsls.MIXED),
                stream=torch.cuda.current_stream().cuda_stream)
    base = q.sls_solve(E, None, Qb, Rb, QbN, rownorm=1, wbound=wb)       # tau = 0
    taus = []
    for p in probs:
        q.update_bounds(p.l, p.u)
        q.solve(x0=p.x0, rho=1.0, tol=TOL)
        lam = q.get()["lam"]
        taus.append(q.sls_tau(lam, base["Phi_x"], base["Phi_u"]))
    for _ in range(args.warmup):
        q.sls_solve_batch(E, taus, Qb, Rb, QbN, rownorm=1, wbound=wb)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dev_ms = []
    for _ in range(args.steps):
        dev_ms.append(q.sls_solve_batch(E, taus, Qb, Rb, QbN, rownorm=1, wbound=wb)["ms"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    q.close()
    flops = sls_flops(p0) * count
    ms = float(np.mean(dev_ms))
    achieved = flops / (ms * 1e-3) / 1e12
    line = {
        "metric": "SLS instances/s (Phi^x, Phi^u and reachable-set margins)",
        "value": count * args.steps / wall, "unit": "instances/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * wall / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic (seeded generator)",
        "config": {"workload": "SLS batch of 64 quadruped-shaped instances, nx=61 nu=12 N=64, 40 rows/stage, "
                               "|w|_inf <= 0.01, tau from nominal ADMM multipliers",
                   "device_ms_per_batch": ms},
        "roofline": {"kernel": "k_sls (persistent SLS columns)", "bound": "mfma", "achieved": achieved,
                     "peak": 157.3, "unit": "TFLOP/s", "frac": achieved / 157.3, "traffic": None,
                     "flops_per_batch": flops},
    }
    if not args.no_cpu:
        import oracle
        t0 = time.perf_counter()
        n = 0
        while True:
            oracle.sls_solve(probs[n % count], E, taus[n % count], Qb, Rb, QbN, rownorm=1, wbound=wb,
                             want_phi=False)
            n += 1
            el = time.perf_counter() - t0
            if el >= args.cpu_budget or n >= 50:
                break
        line["cpu_baseline"] = {"value": n / el, "unit": "instances/s", "cores": 1, "kind": "oracle",
                                "sample": f"{n} instances of the same batch (FP64 per-column Riccati)"}
    print(json.dumps(line), flush=True)


def bench_robust(args):
    """Robust MPC by the FastSLS alternation (Sec. III-D, App. B) on one
    quadruped-shaped instance of the SLS workload (nx=61, nu=12, N=64, 40 rows,
    |w|_inf <= 0.01): a fixed three passes of nominal ADMM solve with tightened
    rows and tau-weighted SLS controller update, then the final nominal solve.
    (At this scale the per-row margins keep moving between passes while their
    total settles, so the passes are counted rather than run to a threshold.)"""
    import torch
    from paper_2604_07644_amd import gsls, workloads as W
    probs, E, wb = W.sls_batch(1)
    p = probs[0]
    Qb, Rb, QbN = np.eye(p.nx), np.eye(p.nu), np.eye(p.nx)
    passes = 3
    kw = dict(rownorm=1, wbound=wb, eps=1e-8, rho=1.0, tol=TOL, max_passes=passes, htol=0.0)
    q = gsls.QP(p, gsls.default_settings(precision=gsls.MIXED), stream=torch.cuda.current_stream().cuda_stream)
    for _ in range(args.warmup):
        q.robust_solve(E, Qb, Rb, QbN, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = []
    for _ in range(args.steps):
        res.append(q.robust_solve(E, Qb, Rb, QbN, **kw))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    q.close()
    r = res[-1]
    ms_nom = float(np.mean([x["ms_nominal"] for x in res]))
    ms_ctl = float(np.mean([x["ms_controller"] for x in res]))
    sls_runs = r["passes"] + 1
    if ms_ctl >= ms_nom:
        flops = sls_flops(p) * sls_runs
        achieved = flops / (ms_ctl * 1e-3) / 1e12
        roof = {"kernel": "k_sls (persistent SLS columns)", "bound": "mfma", "achieved": achieved, "peak": 157.3,
                "unit": "TFLOP/s", "frac": achieved / 157.3, "traffic": None, "flops_per_solve": flops,
                "device_ms_per_solve": ms_ctl}
    else:
        byts = floor_bytes(p) * r["qp_iterations"]
        achieved = byts / (ms_nom * 1e-3) / 1e9
        roof = {"kernel": "k_admm and factor epochs (nominal solves)", "bound": "hbm", "achieved": achieved,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                "floor_bytes_per_solve": byts, "device_ms_per_solve": ms_nom}
    line = {
        "metric": "robust MPC solves/s (3 FastSLS alternation passes + final nominal solve)",
        "value": args.steps / wall, "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic (seeded generator)",
        "config": {"workload": "robust MPC on one quadruped-shaped QP, nx=61 nu=12 N=64, 40 rows/stage, "
                               "|w|_inf <= 0.01, E_t ~ N(0, 0.01)",
                   "status": r["status"], "passes": r["passes"], "qp_solves": r["qp_solves"],
                   "qp_iterations": r["qp_iterations"], "ms_nominal": ms_nom, "ms_controller": ms_ctl},
        "roofline": roof,
    }
    if not args.no_cpu:
        from oracle import robust as R
        t0 = time.perf_counter()
        R.robust_alternation(p, E, Qb, Rb, QbN, rownorm=1, wbound=wb, eps=1e-8, rho=1.0, tol=TOL,
                             max_passes=passes, htol=0.0)
        t = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": 1.0 / t, "unit": "solves/s", "cores": 1, "kind": "oracle",
                                "sample": "one full alternation of the same instance (FP64 Riccati ADMM and "
                                          "per-column SLS)"}
    print(json.dumps(line), flush=True)


def bench_sqp(args):
    """SQP on the Dubins car of App. C at the paper's scale (20 m, 30 obstacles:
    N=200, dt=0.1, v=1), QP and step tolerance 1e-2 as in the paper's
    real-time experiments, mixed precision; the config also reports one
    real-time-iteration update (linearisation, controller synthesis,
    tightened nominal solve) of the planar quadrotor of App. D (N=40, one
    obstacle)."""
    import torch
    from paper_2604_07644_amd import gsls, workloads as W
    stream = torch.cuda.current_stream().cuda_stream
    sc = W.dubins_scenario(N=200, n_obs=30, seed=0)
    q = gsls.SQP(sc, gsls.default_settings(precision=gsls.MIXED), stream=stream)
    kw = dict(max_iter=40, alpha=1.0, tol_qp=1e-2, tol_step=1e-2)
    for _ in range(args.warmup):
        q.solve(sc["x0"], sc["X"], sc["U"], **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = []
    for _ in range(args.steps):
        res.append(q.solve(sc["x0"], sc["X"], sc["U"], **kw)[2])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    q.close()
    r = res[-1]
    ms_qp = float(np.mean([x["ms_qp"] for x in res]))
    ms_lin = float(np.mean([x["ms_linearize"] for x in res]))
    # RTI update of the quadrotor
    sq = W.quadrotor_scenario(N=40, n_obs=1, seed=3)
    qq = gsls.SQP(sq, gsls.default_settings(precision=gsls.MIXED), stream=stream)
    I6, I2 = np.eye(6), np.eye(2)
    rti_kw = dict(rownorm=1, wbound=1.0, tol_qp=1e-2, max_passes=0)
    qq.rti_step(sq["x0"], sq["X"], sq["U"], sq["E"], I6, I2, I6, **rti_kw)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rts = [qq.rti_step(sq["x0"], sq["X"], sq["U"], sq["E"], I6, I2, I6, **rti_kw)[2] for _ in range(args.steps)]
    torch.cuda.synchronize()
    rti_wall = (time.perf_counter() - t1) / args.steps
    qq.close()
    nc, N = 30 + 1, 200
    # floor bytes of one ADMM iteration (as floor_bytes(): nx=3, nu=1, nc=31, nf=30)
    byts = 4 * (N * (2 * 3 * 3 + 3 * 3 * 1 + 1 + nc * 4) + 30 * 3) * r["qp_iterations"]
    achieved = byts / (ms_qp * 1e-3) / 1e9
    line = {
        "metric": "SQP solves/s (Dubins car, 30 obstacles, N=200, tol 1e-2)",
        "value": args.steps / wall, "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic (seeded scenario; the paper's obstacle layout is not given)",
        "config": {"workload": "Dubins car (App. C) SQP, N=200, dt=0.1, v=1, 30 obstacles, |omega| <= 1.5",
                   "status": r["status"], "sqp_iterations": r["iterations"], "qp_iterations": r["qp_iterations"],
                   "ms_qp": ms_qp, "ms_linearize": ms_lin,
                   "rti_quadrotor": {"ms_per_update": 1e3 * rti_wall, "status": rts[-1]["status"],
                                     "qp_iterations": rts[-1]["qp_iterations"],
                                     "ms_nominal": float(np.mean([x["ms_nominal"] for x in rts])),
                                     "ms_controller": float(np.mean([x["ms_controller"] for x in rts]))}},
        "roofline": {"kernel": "k_admm (the SQP's QP solves)", "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "floor_bytes_per_solve": byts, "device_ms_per_solve": ms_qp},
    }
    if not args.no_cpu:
        from oracle import sqp as S
        md = S.from_scenario(sc)
        t0 = time.perf_counter()
        S.sqp(md, sc["x0"], sc["X"], sc["U"], **kw)
        t = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": 1.0 / t, "unit": "solves/s", "cores": 1, "kind": "oracle",
                                "sample": "one SQP solve of the same scenario (numpy linearisation, FP64 Riccati ADMM)"}
    print(json.dumps(line), flush=True)


def batch_floor_bytes(p):
    """Floor bytes of one cached iteration of a batch instance: as floor_bytes,
    without the constraint matrices when the rows are the plain box [x; u]
    (the batched kernel then applies G = I structurally)."""
    N, nx, nu, nc, nf = p.N, p.nx, p.nu, p.nc, p.nf
    box = p.meta.get("kind") in ("uneven", "box_lq")
    rows = 0 if box else N * nc * (nx + nu) + nf * nx
    return 4 * (N * (2 * nx * nx + 3 * nx * nu + nu * nu) + rows)


def bench_batch(args):
    """The uneven batch: 512 box-constrained QPs (nx in {12,36,61,75}, nu in
    {4,12,19}, N ~ U{16..512}, per-instance bound scales) solved to a primal
    and dual residual of 1e-5 in one graph-replayed persistent launch, from a
    cold start and from the learned warm start (the trained model in
    paper_2604_07644_amd/data/ws_box.bin; its prediction is inside the timed
    region).  value: solves/s of the learned-warm-start solver; the cold-start
    figures sit beside it in config.  roofline: k_batch, the floor bytes of
    every iteration each instance ran (its stage operators read once per
    direction) over the launch's device time (HIP events around the replayed
    graph on the solver's stream, minus the prediction).  cpu_baseline: the
    FP64 oracle compiled for this host (-O3 -march=native, OpenMP over the
    instances, one sequential solve per thread) on every 16th instance of the
    batch, cold start."""
    import torch
    from paper_2604_07644_amd import gsls, workloads as W
    count = 512
    probs = W.uneven_batch(count=count)
    stream = torch.cuda.current_stream().cuda_stream
    b = gsls.Batch(probs, stream=stream)
    from paper_2604_07644_amd import autotune
    tuned = autotune.lookup(autotune.batch_key(probs))
    if args.gang is not None or args.park_share is not None:
        b.set_schedule(gang=args.gang or 0, park_share=args.park_share or 0.0)
        source = "command line"
    elif tuned is not None:
        b.set_schedule(gang=tuned["gang"], park_share=tuned["park_share"])
        source = "autotuned (paper_2604_07644_amd/data/tuned.json)"
    else:
        source = "library defaults"
    gang, share, park_at = b.schedule()
    model = os.path.join(ROOT, "paper_2604_07644_amd", "data", "ws_box.bin")
    ws = gsls.WarmStart(path=model, stream=stream) if os.path.exists(model) else None

    def run(warm, parts=gsls.WS_ALL):
        for _ in range(args.warmup):
            b.solve_ws(ws, tol=TOL, parts=parts) if warm else b.solve(tol=TOL)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dev_ms, pred_ms, last = [], [], None
        for _ in range(args.steps):
            if warm:
                last, ms, msp = b.solve_ws(ws, tol=TOL, parts=parts)
            else:
                last, ms = b.solve(tol=TOL)
                msp = 0.0
            dev_ms.append(ms)
            pred_ms.append(msp)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        it = np.array([r["iterations"] for r in last])
        work = float(sum(r["ms_factor"] + r["ms_iterate"] for r in last))
        return dict(solves_per_s=count * args.steps / wall, ms_per_step=1e3 * wall / args.steps,
                    device_ms_per_batch=float(np.mean(dev_ms)), predict_ms=float(np.mean(pred_ms)),
                    solve_ms=float(np.mean(dev_ms) - np.mean(pred_ms)),
                    all_solved=all(r["status"] == gsls.SOLVED for r in last),
                    iterations_mean=float(it.mean()), iterations_median=float(np.median(it)),
                    iterations_max=int(it.max()), instance_ms_sum=work,
                    max_r_dyn=float(max(r["r_dyn"] for r in last)), iters=it)

    cold = run(False)
    parts = {"rho": gsls.WS_RHO, "all": gsls.WS_ALL}[args.ws_parts]
    warm = run(True, parts) if ws is not None else None
    # the other composition of the learned start, reported beside it
    other = run(True, gsls.WS_ALL if parts != gsls.WS_ALL else gsls.WS_RHO) if ws is not None else None
    main = warm if warm is not None else cold
    byts = float(sum(batch_floor_bytes(p) * it for p, it in zip(probs, main["iters"])))
    ms = main["solve_ms"]
    achieved = byts / (ms * 1e-3) / 1e9
    for d in (cold, warm, other):
        if d is not None:
            d.pop("iters")
    b.close()
    if ws is not None:
        ws.close()
    line = {
        "metric": METRIC, "value": main["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": main["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64 (bf16 MLP)",
        "data": "synthetic (seeded generator; no robot models or datasets)",
        "config": {"workload": "uneven batch: 512 box-constrained LTV-QPs, nx in {12,36,61,75}, nu in {4,12,19}, "
                               "N ~ U{16..512}, one graph-replayed persistent launch, warm vs cold start",
                   "tol": TOL, "start": "learned warm" if warm is not None else "cold",
                   "warm_start_parts": {"rho": "predicted rho0, z0 = y0 = 0",
                                        "all": "predicted rho0, z0 and y0"}[args.ws_parts],
                   "schedule": {"gang": gang, "park_share": share, "source": source,
                                "instances_eligible_for_gangs": int(np.sum(park_at < 2 ** 31 - 1))},
                   "warm_vs_cold_speedup": (warm["solves_per_s"] / cold["solves_per_s"]) if warm else None,
                   "cold": cold, "warm": warm,
                   "warm_other_parts": other},
        "roofline": {"kernel": "k_batch (persistent batched ADMM)", "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": kernel_traffic(K_BATCH_TRAFFIC),
                     "floor_bytes_per_launch": byts, "avg_launch_ms": ms},
    }
    if not args.no_cpu:
        import tempfile
        from oracle import native
        sample = probs[::16]
        with tempfile.TemporaryDirectory() as td:
            lib = native.load_native(td)
            t0 = time.perf_counter()
            it, threads = native.qp_solve_many(sample, rho=1.0, tol=TOL, lib=lib)
            el = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": len(sample) / el, "unit": "solves/s", "cores": threads, "kind": "oracle",
                                "sample": f"every 16th instance of the batch ({len(sample)} QPs), cold start, "
                                          f"tol {TOL:g}; FP64 Riccati ADMM built -O3 -march=native, OpenMP over "
                                          f"instances on {threads} threads ({os.cpu_count()} logical CPUs)",
                                "iterations_median": float(np.median(it)), "seconds": el}
    print(json.dumps(line), flush=True)


def copy_calibration(mib=256, reps=3):
    """A plain device copy of known size, for scaling the FETCH_SIZE and
    WRITE_SIZE counters: each launch reads and writes mib MiB."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, device="cuda", dtype=torch.float32)
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_kib_per_launch": mib * 1024, "launches": reps}), flush=True)


def measured_peaks(reps=10):
    """Achievable peaks of this GPU, measured with library kernels: a 1 GiB
    device-to-device copy (read + write bytes per second) and square GEMMs
    (torch.mm, 8192^3 in BF16 and FP32, 4096^3 in FP64)."""
    import torch
    out = {}
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    n = (1 << 30) // 4
    a = torch.ones(n, device="cuda", dtype=torch.float32)
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = ev(), ev()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    out["copy_GBps"] = 2 * a.numel() * 4 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    for dt, n in ((torch.bfloat16, 8192), (torch.float32, 8192), (torch.float64, 4096)):
        x = torch.randn(n, n, device="cuda", dtype=dt)
        y = torch.randn(n, n, device="cuda", dtype=dt)
        z = torch.mm(x, y)
        e0, e1 = ev(), ev()
        e0.record()
        for _ in range(reps):
            z = torch.mm(x, y)
        e1.record()
        torch.cuda.synchronize()
        out[f"gemm_{str(dt).split('.')[-1]}_TFLOPs"] = 2 * n ** 3 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e12
        del x, y, z
    print(json.dumps({"measured_peaks": out, "published": {"hbm_GBps": 8000, "bf16_TFLOPs": 2500,
                                                           "fp32_TFLOPs": 157.3, "fp64_TFLOPs": 78.6}}),
          flush=True)


def cpu_baseline(p, budget_s=10.0, tol=TOL):
    import oracle
    t0 = time.perf_counter()
    n = 0
    iters = []
    while True:
        r = oracle.qp_solve(p, rho=1.0, tol=tol)
        iters.append(r["iters"])
        n += 1
        el = time.perf_counter() - t0
        if (el >= budget_s and n >= 2) or n >= 200:
            break
    return dict(value=n / el, unit="solves/s", cores=1, kind="oracle",
                sample=f"{n} cold-start solves of the same QP at tol {tol:g} "
                       f"(FP64 sequential Riccati ADMM, {int(np.median(iters))} iterations each)",
                ms_per_solve=1e3 * el / n)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="batch")
    ap.add_argument("--gang", type=int, default=None, help="batch: workgroups per gang (0 auto, 1 off)")
    ap.add_argument("--park-share", type=float, default=None, help="batch: solo work budget (0 auto)")
    ap.add_argument("--ws-parts", default="rho", choices=["rho", "all"],
                    help="batch: parts of the learned start used for value (rho: predicted rho0 only; all: rho0, z0, y0)")
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=10.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 256 MiB device copy (counter calibration)")
    ap.add_argument("--with-copy", action="store_true",
                    help="run the 256 MiB copy calibration before the benchmark, in the same process")
    ap.add_argument("--peaks", action="store_true",
                    help="measure the achievable copy bandwidth and GEMM rates, then exit")
    args = ap.parse_args()
    if args.peaks:
        measured_peaks()
        return
    # a batch step is one whole 512-instance batch (about a second): fewer steps
    if args.steps is None:
        args.steps = 5 if args.workload == "batch" else 20
    if args.warmup is None:
        args.warmup = 1 if args.workload == "batch" else 3
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    if args.copy_calibration or args.with_copy:
        copy_calibration()
        if args.copy_calibration:
            return
    if args.workload == "sls":
        bench_sls(args)
        return
    if args.workload == "batch":
        bench_batch(args)
        return
    if args.workload == "robust":
        bench_robust(args)
        return
    if args.workload == "sqp":
        bench_sqp(args)
        return

    import torch
    from paper_2604_07644_amd import gsls

    p, desc, tol = make_workload(args.workload)
    prec = gsls.MIXED if args.precision == "mixed" else gsls.FP64
    stream = torch.cuda.current_stream().cuda_stream
    from paper_2604_07644_amd import autotune
    tuned = autotune.lookup(autotune.qp_key(p, prec))
    chunks = dict(chunks_epoch=tuned["chunks_epoch"], chunks_iter=tuned["chunks_iter"]) if tuned else {}
    q = gsls.QP(p, gsls.default_settings(precision=prec, **chunks), stream=stream)
    for _ in range(args.warmup):
        q.solve(rho=1.0, tol=tol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = []
    for _ in range(args.steps):
        res.append(q.solve(rho=1.0, tol=tol))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    _, lay = q.phase_cycles()
    q.close()

    ok = all(r["status"] == gsls.SOLVED for r in res)
    one_wave = tuple(lay) == (1, 1, 1, p.N)
    iters = [r["iterations"] for r in res]
    ms_iter = float(np.mean([r["ms_iterate"] for r in res]))
    ms_fact = float(np.mean([r["ms_factor"] for r in res]))
    launches = float(np.mean([r["rho_updates"] + 1 for r in res]))
    word = 4 if prec == gsls.MIXED else 8
    bytes_per_iter = floor_bytes(p, word)
    mean_iters = float(np.mean(iters))
    achieved = bytes_per_iter * mean_iters / (ms_iter * 1e-3) / 1e9
    line = {
        "metric": METRIC if tol == TOL else f"QP solves/s and ms/solve at {tol:g} residual (long horizon)",
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
        "config": {"workload": desc, "tol": tol, "start": "cold", "rho0": 1.0,
                   "precision": args.precision, "iterations": int(np.median(iters)),
                   "rho_updates": int(np.median([r["rho_updates"] for r in res])),
                   "all_solved": ok, "ms_factor_per_solve": ms_fact, "ms_iterate_per_solve": ms_iter,
                   "chunks": {"factor": lay[0], "iteration": lay[1], "lds_resident": lay[2], "max_chunk": lay[3],
                              "source": "autotuned (paper_2604_07644_amd/data/tuned.json)" if tuned
                              else "library defaults"}},
        "roofline": {"kernel": "k_admm (persistent ADMM iteration)", "bound": "hbm",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": kernel_traffic(K_ADMM_TRAFFIC[args.workload]) if args.workload in K_ADMM_TRAFFIC else None,
                     "bytes_per_iteration": bytes_per_iter, "iterations_per_launch": mean_iters / launches,
                     "avg_launch_ms": ms_iter / launches},
    }
    if one_wave:
        # the one-wavefront path: the whole solve is one launch of one wave,
        # bound by its own FP64 issue rate, not by memory
        ms_kernel = float(np.mean([r["ms_total"] for r in res]))
        flops = tiny_flops_per_iteration(p) * mean_iters
        achieved = flops / (ms_kernel * 1e-3) / 1e9
        one_simd = FP64_VECTOR_PEAK_GFS / 1024.0
        line["dtype"] = "f64"
        line["roofline"] = {"kernel": "k_tiny (one-wavefront solve)", "bound": "alu", "achieved": achieved,
                            "peak": FP64_VECTOR_PEAK_GFS, "unit": "GFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_GFS,
                            "peak_one_simd": one_simd, "frac_one_simd": achieved / one_simd, "traffic": None,
                            "flops_per_iteration": tiny_flops_per_iteration(p), "avg_launch_ms": ms_kernel}
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(p, args.cpu_budget, tol)
    print(json.dumps(line), flush=True)


FP64_VECTOR_PEAK_GFS = 78.6e3   # published FP64 vector rate: 256 CUs x 4 SIMDs x 16 lanes x 2 x 2.4 GHz


def tiny_flops_per_iteration(p):
    """Algorithmic FP64 flops of one ADMM iteration of the Riccati-form x-update
    (per stage: linear terms, feed-forward solve, backward and forward
    recursions, constraint map, projection, dual residual)."""
    nx, nu, nc = p.nx, p.nu, p.nc
    per_stage = 6 * nx * nx + 8 * nx * nu + 2 * nu * nu + 6 * nc * (nx + nu) + 4 * nc
    return p.N * per_stage + 4 * p.nf * nx


if __name__ == "__main__":
    main()
