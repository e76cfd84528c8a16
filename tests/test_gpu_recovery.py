"""GPU tests of a single-instance solve's outcome handling: the infeasibility
suspicion (GSLS_INFEASIBLE_SUSPECTED) and the FP64 continuation of a
mixed-precision solve that reaches its iteration limit
(gsls_settings.fp64_fallback).

The reading of the suspicion is pinned by the oracle's own run of the same
infeasible QP: the rho rule drives rho to its clamp while r_p settles at the
distance between the constraint sets.  The continuation must reach the
oracle's solution.
"""
import numpy as np
import pytest

import oracle
from paper_2604_07644_amd import workloads as W

pytestmark = pytest.mark.gpu

from paper_2604_07644_amd import gsls  # noqa: E402  (fails loudly without libgsls.so)


def _err(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _infeasible_box():
    p = W.box_lq()
    p.x0 = p.x0.copy()
    p.x0[0] = 7.0          # the stage-0 row |x_0| <= 5 cannot hold
    return p


@pytest.mark.parametrize("chunks", [0, 8])     # one-wavefront path, multi-workgroup scans
@pytest.mark.parametrize("prec", [gsls.FP64, gsls.MIXED])
def test_infeasible_start_is_suspected(chunks, prec):
    p = _infeasible_box()
    o = oracle.qp_solve(p, rho=1.0, tol=1e-5, settings=oracle.Settings(max_iter=600))
    assert o["status"] == 2 and o["rho"] >= 1e6 and o["r_p"] > 1.0
    s = gsls.default_settings(precision=prec, chunks_iter=chunks, chunks_epoch=chunks, fp64_fallback=1)
    s.max_iter = 600
    q = gsls.QP(p, s)
    _, lay = q.phase_cycles(-1)
    r = q.solve(rho=1.0, tol=1e-5)
    q.close()
    assert (lay == (1, 1, 1, p.N)) == (chunks == 0)
    assert r["status"] == gsls.INFEASIBLE_SUSPECTED, r
    assert r["iterations"] == 600 and r["fallback"] == 0
    assert r["rho"] >= 1e6 and abs(r["r_p"] - o["r_p"]) <= 1e-6 * o["r_p"]


def test_limit_on_a_feasible_problem_is_not_suspected():
    p = W.polytopic_lq(40, 12, 4, 10, cfg_id=1, instance_id=5)
    s = gsls.default_settings(precision=gsls.FP64)
    s.max_iter = 20
    q = gsls.QP(p, s)
    r = q.solve(rho=1.0, tol=1e-7)
    q.close()
    assert r["status"] == gsls.MAX_ITER and r["iterations"] == 20


def test_mixed_solve_at_its_limit_continues_in_fp64():
    p = W.polytopic_lq(40, 12, 4, 10, cfg_id=1, instance_id=5)
    ref = oracle.qp_solve(p, rho=1.0, tol=1e-10)
    out = {}
    # the oracle needs 179 iterations at tol 1e-7: the mixed solve stops at 120
    # and the FP64 continuation (a fresh budget of 120) finishes it
    for fb in (0, 1):
        s = gsls.default_settings(precision=gsls.MIXED, fp64_fallback=fb)
        s.max_iter = 120
        q = gsls.QP(p, s)
        r = q.solve(rho=1.0, tol=1e-7)
        out[fb] = (r, q.get())
        q.close()
    r0, _ = out[0]
    assert r0["status"] == gsls.MAX_ITER and r0["iterations"] == 120 and r0["fallback"] == 0
    r1, g1 = out[1]
    assert r1["status"] == gsls.SOLVED and r1["fallback"] == 1 and 120 < r1["iterations"] < 240, r1
    assert r1["r_p"] <= 1e-7 and r1["r_d"] <= 1e-7
    assert r1["factorizations"] >= 2 and r1["ms_total"] >= r1["ms_factor"]
    assert _err(g1["X"], ref["X"]) <= 1e-5 and _err(g1["U"], ref["U"]) <= 1e-5
    assert r1["r_dyn"] <= 1e-12 * max(1.0, float(np.abs(ref["X"]).max()))
