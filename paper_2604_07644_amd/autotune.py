"""Autotuner of the launch schedules, measured on the GPU.

    python -m paper_2604_07644_amd.autotune [--workloads batch,quadruped,humanoid]
                                            [--out paper_2604_07644_amd/data/tuned.json]

What is tuned (the "tiles" of this solver are horizon chunks and workgroup
gangs, not GEMM tiles):
  * the batched solver (gsls_batch_set_schedule): workgroups per gang and the
    solo work budget after which an instance is handed to a gang, timed on
    the batch itself, cold and with the learned start (predicted rho0), the
    score being the sum of the two device times per batch;
  * the single-instance solver (gsls_settings.chunks_epoch / chunks_iter): the
    number of horizon chunks of the factor scan and of the iteration kernel,
    timed as whole solves.
Every candidate's solution must still satisfy the stopping test (all
instances solved); a candidate that does not is discarded.  The winners are
stored per workload key (the shapes, hashed for a batch) in a JSON cache that
bench.py reads and reports.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

CACHE = os.path.join(ROOT, "paper_2604_07644_amd", "data", "tuned.json")
TOL = 1e-5


def batch_key(probs) -> str:
    h = hashlib.sha1()
    for p in probs:
        h.update(f"{p.N},{p.nx},{p.nu},{p.nc},{p.nf};".encode())
    return f"batch:{len(probs)}:{h.hexdigest()[:16]}"


def qp_key(p, precision) -> str:
    return f"qp:{p.N}x{p.nx}x{p.nu}x{p.nc}x{p.nf}:{'fp64' if precision else 'mixed'}"


def load(path=CACHE) -> dict:
    if not os.path.exists(path):
        return {"version": 1, "entries": {}}
    with open(path) as f:
        return json.load(f)


def lookup(key, path=CACHE):
    return load(path)["entries"].get(key)


def _device():
    import torch
    return torch.cuda.current_stream().cuda_stream


def tune_batch(probs, model_path, reps=2, log=print):
    from paper_2604_07644_amd import gsls
    stream = _device()
    b = gsls.Batch(probs, stream=stream)
    ws = gsls.WarmStart(path=model_path, stream=stream) if os.path.exists(model_path) else None
    cands = [(1, 1.0)] + [(g, s) for g in (16, 24, 32) for s in (0.5, 0.75, 0.9, 1.0, 1.1, 1.25, 1.5)]
    results = []
    for g, s in cands:
        b.set_schedule(gang=g, park_share=s)
        gg, ss, _ = b.schedule()
        b.solve(tol=TOL)
        cold, warm, ok = [], [], True
        for _ in range(reps):
            r, ms = b.solve(tol=TOL)
            ok = ok and all(x["status"] == gsls.SOLVED for x in r)
            cold.append(ms)
            if ws is not None:
                r, ms, _ = b.solve_ws(ws, tol=TOL, parts=gsls.WS_RHO)
                ok = ok and all(x["status"] == gsls.SOLVED for x in r)
                warm.append(ms)
        score = float(np.mean(cold) + (np.mean(warm) if warm else 0.0))
        d = dict(gang=gg, park_share=ss, cold_ms=float(np.mean(cold)),
                 warm_ms=float(np.mean(warm)) if warm else None, score=score, ok=ok)
        log(json.dumps(d))
        results.append(d)
    b.close()
    if ws is not None:
        ws.close()
    good = [d for d in results if d["ok"]]
    best = min(good, key=lambda d: d["score"])
    return dict(kind="batch", gang=best["gang"], park_share=best["park_share"], cold_ms=best["cold_ms"],
                warm_ms=best["warm_ms"], candidates=results)


def tune_qp(p, precision, reps=3, log=print):
    from paper_2604_07644_amd import gsls
    stream = _device()
    N = p.N
    iters = sorted({0} | {c for c in (N, N // 2, N // 4, N // 8, 128, 64, 32) if 1 <= c <= min(256, N)})
    epochs = sorted({0} | {c for c in (N // 2, N // 4, 64) if 1 <= c <= min(256, N)})
    results = []
    for ce in epochs:
        for ci in iters:
            try:
                q = gsls.QP(p, gsls.default_settings(precision=precision, chunks_epoch=ce, chunks_iter=ci),
                            stream=stream)
            except gsls.GslsError:
                continue
            q.solve(rho=1.0, tol=TOL)
            ms, ok = [], True
            for _ in range(reps):
                t0 = time.perf_counter()
                r = q.solve(rho=1.0, tol=TOL)
                ms.append(1e3 * (time.perf_counter() - t0))
                ok = ok and r["status"] == gsls.SOLVED
            _, lay = q.phase_cycles(-1)
            q.close()
            d = dict(chunks_epoch=ce, chunks_iter=ci, layout=[int(x) for x in lay], ms=float(np.median(ms)), ok=ok)
            log(json.dumps(d))
            results.append(d)
    good = [d for d in results if d["ok"]]
    best = min(good, key=lambda d: d["ms"])
    return dict(kind="qp", chunks_epoch=best["chunks_epoch"], chunks_iter=best["chunks_iter"],
                layout=best["layout"], ms=best["ms"], candidates=results)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workloads", default="batch,quadruped,humanoid")
    ap.add_argument("--out", default=CACHE)
    args = ap.parse_args()
    from paper_2604_07644_amd import gsls, workloads as W
    cache = load(args.out)
    log = lambda s: print(s, flush=True)  # noqa: E731
    for wl in args.workloads.split(","):
        t0 = time.perf_counter()
        if wl == "batch":
            probs = W.uneven_batch(count=512)
            key = batch_key(probs)
            entry = tune_batch(probs, os.path.join(ROOT, "paper_2604_07644_amd", "data", "ws_box.bin"), log=log)
        else:
            p = {"quadruped": lambda: W.quadruped_qp(0), "humanoid": lambda: W.humanoid_qp(0),
                 "box": W.box_lq}[wl]()
            key = qp_key(p, gsls.MIXED)
            entry = tune_qp(p, gsls.MIXED, log=log)
        entry["workload"] = wl
        entry["tuned_seconds"] = time.perf_counter() - t0
        cache["entries"][key] = entry
        log(json.dumps({"key": key, **{k: v for k, v in entry.items() if k != "candidates"}}))
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(cache, f, indent=1)


if __name__ == "__main__":
    main()
