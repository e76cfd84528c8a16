"""GPU parity of the one-wavefront path (tiny problems: nx, nu <= 4, at most 8
rows per stage and 8 terminal rows, N <= 63, automatic chunking) against the
FP64 CPU oracle.

The path computes in FP64 in both precision modes, so it is held to the FP64
bars: fixed rho follows the oracle iterate by iterate; adaptive rho takes the
same iterations and rho updates.  It is also checked against the
multi-workgroup scan path on the same problem (explicit chunking).
"""
import ctypes as ct

import numpy as np
import pytest

import oracle
from paper_2604_07644_amd import workloads as W

pytestmark = pytest.mark.gpu

from paper_2604_07644_amd import gsls  # noqa: E402  (fails loudly without libgsls.so)

PROBLEMS = {
    "box": lambda: W.box_lq(),
    "box_3x1": lambda: W.box_lq(N=20, nx=3, nu=1, cfg_id=3),               # box rows, padded lanes
    "box_no_terminal": lambda: W.box_lq(N=24, terminal_box=False),         # general rows (nf = 0)
    "general_4x3": lambda: W.random_small(23, 4, 3, 5, 2, seed=1),
    "one_stage": lambda: W.random_small(1, 3, 1, 2, 1, seed=4),
    "n63_full_rows": lambda: W.random_small(63, 4, 4, 8, 8, seed=5),
    "no_rows": lambda: W.random_small(9, 2, 1, 0, 0, seed=6),
    "one_sided": lambda: W.random_small(17, 4, 2, 6, 3, seed=7, lower=False),
    "n32_nu1": lambda: W.random_small(32, 3, 1, 4, 0, seed=8),
}


def _err(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)) if np.size(b) else 0.0


def _close_all(g, o, tol):
    for k in ("X", "U", "z", "lam"):
        assert _err(g[k], o[k]) <= tol, (k, _err(g[k], o[k]))


def _solve(p, prec=gsls.FP64, iters=None, tol=1e-7, adaptive=True, ci=0, ce=0, rho=1.0, z0=None, y0=None):
    s = gsls.default_settings(precision=prec, adaptive_rho=int(adaptive), chunks_iter=ci, chunks_epoch=ce)
    if iters:
        s.max_iter = iters
    q = gsls.QP(p, s)
    _, lay = q.phase_cycles(-1)
    r = q.solve(rho=rho, tol=0.0 if iters else tol, z0=z0, y0=y0)
    g = q.get()
    q.close()
    return r, g, lay


def _orc(p, iters=None, tol=1e-7, adaptive=True, rho=1.0):
    return oracle.qp_solve(p, rho=rho, tol=0.0 if iters else tol,
                           settings=oracle.Settings(max_iter=iters or 10000, adaptive=adaptive))


def test_layout_reports_the_one_wave_path():
    p = W.box_lq()
    for prec in (gsls.FP64, gsls.MIXED):
        q = gsls.QP(p, gsls.default_settings(precision=prec))
        assert q.phase_cycles(-1)[1] == (1, 1, 1, p.N)
        q.close()
    q = gsls.QP(p, gsls.default_settings(chunks_iter=4))
    assert q.phase_cycles(-1)[1][1] == 4
    q.close()
    big = W.random_small(64, 4, 2, 4, 2, seed=9)       # N = 64: the scan path
    q = gsls.QP(big, gsls.default_settings())
    assert q.phase_cycles(-1)[1] != (1, 1, 1, 64)
    q.close()


@pytest.mark.parametrize("name", sorted(PROBLEMS))
@pytest.mark.parametrize("iters", [1, 7, 60])
def test_fixed_rho_iterates_equal_oracle(name, iters):
    p = PROBLEMS[name]()
    r, g, lay = _solve(p, iters=iters, adaptive=False)
    assert lay == (1, 1, 1, p.N)
    o = _orc(p, iters=iters, adaptive=False)
    assert r["iterations"] == o["iters"]
    assert r["status"] == (gsls.SOLVED if o["status"] == 1 else gsls.MAX_ITER)
    _close_all(g, o, 1e-10)
    assert r["r_dyn"] <= 1e-12 * max(1.0, float(np.abs(o["X"]).max()))


@pytest.mark.parametrize("name", sorted(PROBLEMS))
@pytest.mark.parametrize("prec", [gsls.FP64, gsls.MIXED])
def test_adaptive_follows_oracle(name, prec):
    p = PROBLEMS[name]()
    r, g, _ = _solve(p, prec=prec, tol=1e-7)
    o = _orc(p, tol=1e-7)
    assert o["status"] == 1 and r["status"] == gsls.SOLVED
    assert r["iterations"] == o["iters"] and r["rho_updates"] == o["rho_updates"]
    assert r["factorizations"] == o["rho_updates"] + 1
    # rho is a ratio of residuals (differences of close numbers): relative 1e-8
    assert abs(r["rho"] - o["rho"]) <= 1e-8 * o["rho"]
    _close_all(g, o, 1e-9)
    assert r["ms_total"] > 0 and 0 < r["ms_factor"] + r["ms_iterate"] <= 1.05 * r["ms_total"] + 0.01


@pytest.mark.parametrize("name", ["box", "general_4x3"])
def test_agrees_with_scan_path(name):
    p = PROBLEMS[name]()
    r1, g1, lay1 = _solve(p, tol=1e-8)
    r2, g2, lay2 = _solve(p, tol=1e-8, ci=p.N, ce=p.N)
    assert lay1 == (1, 1, 1, p.N) and lay2[1] == p.N
    assert r1["iterations"] == r2["iterations"] and r1["rho_updates"] == r2["rho_updates"]
    _close_all(g1, g2, 1e-9)


def test_warm_start_and_resolve_on_one_handle():
    p = PROBLEMS["general_4x3"]()
    o = _orc(p, tol=1e-10)
    q = gsls.QP(p, gsls.default_settings(precision=gsls.FP64))
    r = q.solve(rho=o["rho"], tol=1e-8, z0=o["z"], y0=o["y"])
    assert r["status"] == gsls.SOLVED and r["iterations"] <= 2
    np.testing.assert_allclose(q.get()["X"], o["X"], atol=1e-8)
    # a cold solve on the same handle afterwards starts from z = y = 0 again
    r = q.solve(rho=1.0, tol=1e-7)
    o = _orc(p, tol=1e-7)
    assert r["iterations"] == o["iters"]
    _close_all(q.get(), o, 1e-9)
    q.close()


def test_update_data_replaces_the_problem():
    p1, p2 = W.random_small(23, 4, 3, 5, 2, seed=11), W.random_small(23, 4, 3, 5, 2, seed=12)
    q = gsls.QP(p1, gsls.default_settings(precision=gsls.FP64))
    q.solve(rho=1.0, tol=1e-7)
    d, keep = gsls.make_desc(p2)
    assert gsls.lib.gsls_qp_update_data(q.h, ct.byref(d)) == gsls.OK
    r = q.solve(x0=p2.x0, rho=1.0, tol=1e-7)
    o = _orc(p2, tol=1e-7)
    assert r["iterations"] == o["iters"] and r["rho_updates"] == o["rho_updates"]
    _close_all(q.get(), o, 1e-9)
    q.close()


def test_indefinite_control_block_is_reported():
    p = PROBLEMS["general_4x3"]()
    p.R[7] = -1e3 * np.eye(p.nu)
    p.D[7] = 0.0
    q = gsls.QP(p, gsls.default_settings(precision=gsls.FP64))
    with pytest.raises(gsls.GslsError) as ei:
        q.solve(rho=1e-3, tol=1e-6)
    assert ei.value.code == gsls.ERR_NOT_PD
    q.close()


def test_device_descriptor_matches_host():
    """Problem data, x0 and the warm start in device memory (GSLS_DEVICE) on the
    one-wavefront path: the same FP64 solves, bit for bit, as from host memory."""
    import torch
    p = PROBLEMS["general_4x3"]()
    s = gsls.default_settings(precision=gsls.FP64)
    q = gsls.QP(p, s)
    rh = q.solve(rho=1.0, tol=1e-7)
    gh = q.get()
    rhw = q.solve(rho=rh["rho"], tol=1e-9, z0=gh["z"], y0=gh["lam"] / rh["rho"])
    ghw = q.get()
    q.close()

    def dev(a):
        return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")

    def dptr(t):
        return ct.cast(ct.c_void_p(t.data_ptr()), ct.POINTER(ct.c_double))

    keep = {k: dev(getattr(p, k)) for k in ("A", "B", "b", "Q", "R", "S", "q", "r", "C", "D", "l", "u")}
    keep["CN"] = dev(np.asarray(p.CN).reshape(p.nf, p.nx))
    d = gsls.QPDesc(N=p.N, nx=p.nx, nu=p.nu, nc=p.nc, nf=p.nf, mem=gsls.DEVICE)
    for k, t in keep.items():
        setattr(d, k, dptr(t))
    h = ct.c_void_p()
    assert gsls.lib.gsls_qp_setup(ct.byref(d), ct.byref(s), None, ct.byref(h)) == gsls.OK
    lay = (ct.c_int32 * 4)()
    assert gsls.lib.gsls_debug_phase_cycles(h, -1, None, lay) == gsls.OK and tuple(lay) == (1, 1, 1, p.N)
    x0 = dev(p.x0)
    r = gsls.Result()
    assert gsls.lib.gsls_qp_solve(h, dptr(x0), 1.0, 1e-7, ct.byref(r)) == gsls.OK
    X = np.zeros((p.N + 1, p.nx)); z = np.zeros(p.m); lam = np.zeros(p.m)
    P = ct.POINTER(ct.c_double)
    assert gsls.lib.gsls_qp_get(h, X.ctypes.data_as(P), None, z.ctypes.data_as(P), lam.ctypes.data_as(P)) == gsls.OK
    assert r.iterations == rh["iterations"] and r.rho_updates == rh["rho_updates"]
    np.testing.assert_array_equal(X, gh["X"])
    z0, y0 = dev(z), dev(lam / r.rho)
    assert gsls.lib.gsls_qp_solve_warm(h, dptr(x0), r.rho, 1e-9, dptr(z0), dptr(y0), ct.byref(r)) == gsls.OK
    assert gsls.lib.gsls_qp_get(h, X.ctypes.data_as(P), None, None, None) == gsls.OK
    assert r.iterations == rhw["iterations"]
    np.testing.assert_array_equal(X, ghw["X"])
    gsls.lib.gsls_qp_free(h)
