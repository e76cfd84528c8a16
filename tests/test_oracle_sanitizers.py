"""The C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
runs its entry points (Riccati factor, ADMM solve with box and general rows,
the OpenMP batch driver, SLS responses and margin weights) on small problems
without a report: memory errors or undefined behaviour in the code that every
parity test trusts would otherwise go unnoticed."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys
sys.path.insert(0, {root!r})
import numpy as np
import oracle.native as nat
nat.lib_path = {lib!r}
from paper_2604_07644_amd import workloads as W
p = W.box_lq()
nat.qp_factor(p, 1.0)
r = nat.qp_solve(p, rho=1.0, tol=1e-6)
assert r["iters"] > 0
g = W.random_small(12, 5, 3, 4, 3, seed=7)
r = nat.qp_solve(g, rho=0.3, tol=1e-6)
it, thr = nat.qp_solve_many([W.box_lq(), g], rho=1.0, tol=1e-5, lib=nat._load())
probs, E, wb = W.sls_batch(1, N=8, nx=8, nu=3, nc=6)
q = probs[0]
Qb, Rb, QbN = np.eye(q.nx), np.eye(q.nu), np.eye(q.nx)
tau0 = np.zeros(q.N * q.N * q.nc + q.N * q.nf)
s = nat.sls_solve(q, E, tau0, Qb, Rb, QbN, rownorm=1, wbound=wb)
lam = nat.qp_solve(q, rho=1.0, tol=1e-5)["lam"]
tau = nat.sls_tau(q, lam, s["Phi_x"], s["Phi_u"])
nat.sls_solve(q, E, tau, Qb, Rb, QbN, rownorm=1, wbound=wb)
print("sanitized oracle ok")
"""


def _runtime(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return out if os.path.isabs(out) and os.path.exists(out) else None


@pytest.mark.timeout(600)
def test_oracle_under_asan_and_ubsan(tmp_path):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if asan is None or ubsan is None:
        pytest.skip("gcc sanitizer runtimes not installed")
    from oracle import build
    lib = build.build_sanitized(str(tmp_path))
    env = dict(os.environ)
    env["LD_PRELOAD"] = f"{asan}:{ubsan}"
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["OMP_NUM_THREADS"] = "2"
    r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT, lib=lib)], capture_output=True, text=True,
                       env=env, timeout=540)
    assert r.returncode == 0 and "sanitized oracle ok" in r.stdout, (r.returncode, r.stdout[-2000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
