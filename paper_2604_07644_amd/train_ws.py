"""Train the learned warm start of the batched solver on the GPU.

    python -m paper_2604_07644_amd.train_ws --instances 4096 --epochs 20 \
        --out paper_2604_07644_amd/data/ws_box.bin

Training data are solver-generated: box-constrained instances of uneven
shape (nx in {12,36,61,75}, nu in {4,12,19}, N ~ U{16..512}; instance ids
from 10^6 up, disjoint from the benchmark's ids 0..511) are solved cold by the
batched solver at tol 1e-5, and each solved instance contributes its feature
rows (gsls_ws_features) and target rows (gsls_ws_targets: z, lambda and
log10 of the final rho).  Training runs the library's BF16 forward/backward
and Adam kernels (gsls_ws_train_step) on shuffled row mini-batches; the row
permutation of each epoch is drawn by torch (random numbers passed in as
indices).  Problem generation is host work, spread over worker processes.
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

TRAIN_FIRST_ID = 10 ** 6


def _gen(args):
    from paper_2604_07644_amd import workloads as W
    first, count = args
    return W.uneven_batch(count=count, first_instance=first)


def generate_problems(n, first=TRAIN_FIRST_ID, chunk=64, workers=12):
    jobs = [(first + i, min(chunk, n - i)) for i in range(0, n, chunk)]
    if workers <= 1:
        return [p for j in jobs for p in _gen(j)]
    with mp.get_context("spawn").Pool(workers) as pool:
        out = pool.map(_gen, jobs)
    return [p for ps in out for p in ps]


def build_dataset(ws, probs, batch=512, tol=1e-5, log=print):
    """Cold-solves the problems in batches; returns device tensors (X, T, M)
    of the solved instances' rows."""
    import torch
    from paper_2604_07644_amd import gsls
    Xs, Ts, Ms = [], [], []
    solved = 0
    for i in range(0, len(probs), batch):
        chunk = probs[i:i + batch]
        b = gsls.Batch(chunk, stream=torch.cuda.current_stream().cuda_stream)
        res, ms = b.solve(tol=tol)
        X = ws.features(b)
        T, M = gsls.WarmStart.targets(b)
        keep = np.array([r["status"] == gsls.SOLVED for r in res])
        rows = np.repeat(keep, [p.N + 1 for p in chunk])
        sel = torch.tensor(np.nonzero(rows)[0], device="cuda", dtype=torch.long)
        Xs.append(X.index_select(0, sel)); Ts.append(T.index_select(0, sel)); Ms.append(M.index_select(0, sel))
        solved += int(keep.sum())
        log(f"dataset: batch {i // batch}: {len(chunk)} instances, {int(keep.sum())} solved, "
            f"{ms:.1f} ms, mean iterations {np.mean([r['iterations'] for r in res]):.1f}")
        b.close()
    return torch.cat(Xs), torch.cat(Ts), torch.cat(Ms), solved


def train(ws, X, T, M, epochs=20, rows_per_step=8192, lr=1e-3, seed=0, log=print):
    import torch
    n = X.shape[0]
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    hist = []
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g, device="cuda").to(torch.int32)
        t0 = time.perf_counter()
        steps = 0
        for i in range(0, n - rows_per_step + 1, rows_per_step):
            ws.train_step(X, T, M, idx=perm[i:i + rows_per_step], lr=lr)
            steps += 1
        torch.cuda.synchronize()
        # loss on a fixed slice of the training rows
        loss, _ = ws.loss_grad(X, T, M, idx=perm[:min(n, 65536)])
        hist.append(loss)
        log(f"epoch {ep}: {steps} steps in {time.perf_counter() - t0:.2f} s, loss {loss:.5f}")
    return hist


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--instances", type=int, default=4096)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--rows-per-step", type=int, default=8192)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--workers", type=int, default=12)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--stream", action="store_true",
                    help="generate and solve 512 instances at a time in this process (large training sets)")
    ap.add_argument("--out", default=os.path.join(ROOT, "paper_2604_07644_amd", "data", "ws_box.bin"))
    args = ap.parse_args()

    import torch
    from paper_2604_07644_amd import gsls, workloads as W
    ws = gsls.WarmStart(W.ws_init(args.seed).astype(np.float32), W.ws_sketch().astype(np.float32),
                        stream=torch.cuda.current_stream().cuda_stream)
    log = lambda s: print(s, flush=True)  # noqa: E731
    t1 = time.perf_counter()
    if args.stream:
        # generate (worker processes), solve and keep only the device rows,
        # 512 instances at a time: host memory holds one batch's problem data
        Xs, Ts, Ms, solved = [], [], [], 0
        for i in range(0, args.instances, 512):
            probs = generate_problems(min(512, args.instances - i), first=TRAIN_FIRST_ID + i,
                                      workers=args.workers)
            X, T, M, n = build_dataset(ws, probs, log=log)
            Xs.append(X); Ts.append(T); Ms.append(M)
            solved += n
            del probs
            log(f"streamed {i + 512} instances in {time.perf_counter() - t1:.1f} s")
        X, T, M = torch.cat(Xs), torch.cat(Ts), torch.cat(Ms)
        del Xs, Ts, Ms
    else:
        t0 = time.perf_counter()
        probs = generate_problems(args.instances, workers=args.workers)
        print(f"generated {len(probs)} problems in {time.perf_counter() - t0:.1f} s", flush=True)
        X, T, M, solved = build_dataset(ws, probs, log=log)
        del probs
    print(f"dataset: {solved} solved instances, {X.shape[0]} rows in {time.perf_counter() - t1:.1f} s",
          flush=True)
    t2 = time.perf_counter()
    hist = train(ws, X, T, M, epochs=args.epochs, rows_per_step=args.rows_per_step, lr=args.lr,
                 seed=args.seed, log=log)
    print(f"training: {time.perf_counter() - t2:.1f} s", flush=True)
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    ws.save(args.out)
    print(json.dumps({"instances": solved, "rows": int(X.shape[0]), "epochs": args.epochs,
                      "loss_first": hist[0], "loss_last": hist[-1], "out": args.out}), flush=True)


if __name__ == "__main__":
    main()
