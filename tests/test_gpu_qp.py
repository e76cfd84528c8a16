"""GPU parity of the ADMM QP solver (C ABI via the ctypes binding) against the
FP64 CPU oracle.

Bars: FP64 mode follows the oracle iterate by iterate (same iteration count,
same rho updates, solution to ~1e-10); mixed mode (FP32 scans, FP64
factorisations and state) reaches r_p, r_d <= tol and its primal solution
satisfies |x - x*|_inf <= 1e-4 |x*|_inf against the oracle run to a tight
tolerance.
"""
import numpy as np
import pytest

import oracle
from paper_2604_07644_amd import workloads as W

pytestmark = pytest.mark.gpu

from paper_2604_07644_amd import gsls  # noqa: E402  (fails loudly without libgsls.so)


def _err(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _gpu(p, prec, iters=None, tol=1e-6, rho=1.0, adaptive=True, ce=0, ci=0, z0=None, y0=None):
    s = gsls.default_settings(precision=prec, adaptive_rho=int(adaptive), chunks_epoch=ce, chunks_iter=ci)
    if iters:
        s.max_iter = iters
    q = gsls.QP(p, s)
    r = q.solve(rho=rho, tol=0.0 if iters else tol, z0=z0, y0=y0)
    g = q.get()
    q.close()
    return r, g


def _orc(p, iters=None, tol=1e-6, rho=1.0, adaptive=True, z0=None, y0=None):
    return oracle.qp_solve(p, rho=rho, tol=0.0 if iters else tol,
                           settings=oracle.Settings(max_iter=iters or 10000, adaptive=adaptive), z0=z0, y0=y0)


def _close_all(g, o, tol):
    for k in ("X", "U", "z", "lam"):
        assert _err(g[k], o[k]) <= tol, (k, _err(g[k], o[k]))


CHUNKS = [(0, 0), (1, 1), (3, 5), (32, 32), (7, 2)]


@pytest.mark.parametrize("ce,ci", CHUNKS)
@pytest.mark.parametrize("iters", [1, 7, 60])
def test_fp64_box_iterates_equal_oracle(iters, ce, ci):
    p = W.box_lq()
    r, g = _gpu(p, gsls.FP64, iters=iters, adaptive=False, ce=ce, ci=ci)
    o = _orc(p, iters=iters, adaptive=False)
    assert r["iterations"] == o["iters"] == iters
    _close_all(g, o, 1e-11)


@pytest.mark.parametrize("ce,ci", [(1, 1), (4, 6), (7, 23), (23, 7), (2, 3)])
def test_fp64_general_problem_iterates(ce, ci):
    """Every term present: S, b, q, r, two-sided / one-sided / free rows, terminal rows;
    chunk counts that leave ragged chunks."""
    p = W.random_small(23, 5, 3, 4, 3, seed=1)
    r, g = _gpu(p, gsls.FP64, iters=30, adaptive=False, ce=ce, ci=ci)
    o = _orc(p, iters=30, adaptive=False)
    _close_all(g, o, 1e-10)


@pytest.mark.parametrize("maker", ["box", "small", "poly"])
def test_fp64_adaptive_matches_oracle(maker):
    p = {"box": W.box_lq(), "small": W.random_small(23, 5, 3, 4, 3, seed=2),
         "poly": W.polytopic_lq(40, 12, 4, 10, cfg_id=1, instance_id=5)}[maker]
    r, g = _gpu(p, gsls.FP64, tol=1e-7)
    o = _orc(p, tol=1e-7)
    assert r["status"] == gsls.SOLVED and o["status"] == 1
    assert r["iterations"] == o["iters"] and r["rho_updates"] == o["rho_updates"]
    _close_all(g, o, 1e-9)


@pytest.mark.parametrize("maker", ["box", "poly", "small"])
def test_mixed_solution_parity(maker):
    p = {"box": W.box_lq(), "small": W.random_small(23, 5, 3, 4, 3, seed=3),
         "poly": W.polytopic_lq(40, 12, 4, 10, cfg_id=1, instance_id=6)}[maker]
    r, g = _gpu(p, gsls.MIXED, tol=1e-5)
    ref = _orc(p, tol=1e-10)
    assert r["status"] == gsls.SOLVED, r
    assert r["r_p"] <= 1e-5 and r["r_d"] <= 1e-5
    assert _err(g["X"], ref["X"]) <= 1e-4
    assert _err(g["U"], ref["U"]) <= 1e-4


def test_quadruped_mixed_parity():
    """nx=61, nu=12, N=128, 40 polytopic rows per stage, tol 1e-5."""
    p = W.quadruped_qp(0)
    r, g = _gpu(p, gsls.MIXED, tol=1e-5)
    ref = _orc(p, tol=1e-10)
    assert r["status"] == gsls.SOLVED, r
    assert _err(g["X"], ref["X"]) <= 1e-4, _err(g["X"], ref["X"])
    assert _err(g["U"], ref["U"]) <= 1e-4


def test_quadruped_fp64_follows_oracle():
    p = W.quadruped_qp(1)
    r, g = _gpu(p, gsls.FP64, tol=1e-5)
    o = _orc(p, tol=1e-5)
    assert r["iterations"] == o["iters"] and r["rho_updates"] == o["rho_updates"]
    _close_all(g, o, 1e-9)


@pytest.mark.parametrize("ci", [0, 4])
def test_humanoid_shape_fp64_follows_oracle(ci):
    """nx=75, nu=19 (nx + nu = 94), 40 rows, N=48: the widest iteration
    variant; ci=4 gives 12-stage chunks whose operators are read from global
    memory instead of LDS."""
    p = W.humanoid_qp(1, N=48)
    r, g = _gpu(p, gsls.FP64, tol=1e-5, ci=ci)
    o = _orc(p, tol=1e-5)
    assert r["status"] == gsls.SOLVED and o["status"] == 1
    assert r["iterations"] == o["iters"] and r["rho_updates"] == o["rho_updates"]
    _close_all(g, o, 1e-9)


@pytest.mark.parametrize("ci", [0, 4])
def test_humanoid_shape_mixed_parity(ci):
    """ci=4: 12-stage chunks with the operators read from global memory
    (the FP32 variant the full-length humanoid QP runs)."""
    p = W.humanoid_qp(0, N=48)
    r, g = _gpu(p, gsls.MIXED, tol=1e-5, ci=ci)
    ref = _orc(p, tol=1e-10)
    assert r["status"] == gsls.SOLVED, r
    assert _err(g["X"], ref["X"]) <= 1e-4, _err(g["X"], ref["X"])
    assert _err(g["U"], ref["U"]) <= 1e-4


@pytest.mark.parametrize("N,want", [(1, (1, 1, 1, 1)), (23, (23, 23, 1, 1)), (128, (128, 128, 1, 1)),
                                     (300, (256, 256, 1, 2))])
def test_default_layout_is_one_stage_per_workgroup(N, want):
    """The default scans use one horizon stage per workgroup (factor chunks and
    iteration workgroups) up to 256, then ceil(N / 256) stages each."""
    p = W.random_small(N, 5, 3, 4, 3, seed=7)
    q = gsls.QP(p, gsls.default_settings(precision=gsls.MIXED))
    _, lay = q.phase_cycles(-1)
    q.close()
    assert lay == want, lay


def test_horizon_beyond_the_grid_is_rejected():
    """256 workgroups of at most 64 stages: N = 16385 is refused with
    GSLS_ERR_DIM at creation, N = 16384 is accepted."""
    ok = W.random_small(16384, 2, 1, 0, 0, seed=8)
    q = gsls.QP(ok, gsls.default_settings(precision=gsls.MIXED))
    _, lay = q.phase_cycles(-1)
    q.close()
    assert lay[1] == 256 and lay[3] == 64
    bad = W.random_small(16385, 2, 1, 0, 0, seed=8)
    with pytest.raises(gsls.GslsError) as e:
        gsls.QP(bad, gsls.default_settings(precision=gsls.MIXED))
    assert e.value.code == gsls.ERR_DIM


def test_chunking_beyond_the_local_data_share_is_rejected():
    """64-stage chunks of humanoid-width stages (nx=75, nu=19, 40 rows) need
    more local memory per workgroup than a compute unit has: refused at set-up
    with GSLS_ERR_DIM (not a failed launch); the default chunking is accepted."""
    p = W.humanoid_qp(0, N=2048)
    with pytest.raises(gsls.GslsError) as e:
        gsls.QP(p, gsls.default_settings(precision=gsls.MIXED, chunks_iter=32))
    assert e.value.code == gsls.ERR_DIM
    q = gsls.QP(p, gsls.default_settings(precision=gsls.MIXED))
    q.close()


def test_single_stage_and_unconstrained():
    p = W.random_small(1, 3, 2, 2, 1, seed=4)
    r, g = _gpu(p, gsls.FP64, iters=9, adaptive=False)
    o = _orc(p, iters=9, adaptive=False)
    _close_all(g, o, 1e-11)
    p = W.random_small(17, 4, 2, 0, 0, seed=5)
    r, g = _gpu(p, gsls.FP64, tol=1e-9)
    o = _orc(p, tol=1e-9)
    assert r["iterations"] == o["iters"] == 1
    np.testing.assert_allclose(g["X"], o["X"], atol=1e-11)


def test_warm_start_from_solution_converges_at_once():
    p = W.box_lq()
    o = _orc(p, tol=1e-10)
    rho = o["rho"]
    r, g = _gpu(p, gsls.FP64, tol=1e-8, rho=rho, z0=o["z"], y0=o["y"])
    assert r["status"] == gsls.SOLVED and r["iterations"] <= 2
    np.testing.assert_allclose(g["X"], o["X"], atol=1e-8)


def test_indefinite_cost_is_reported():
    p = W.box_lq()
    p.R[5] = -np.eye(p.nu)
    q = gsls.QP(p, gsls.default_settings(precision=gsls.FP64))
    with pytest.raises(gsls.GslsError) as ei:
        q.solve(rho=1e-3, tol=1e-6)
    assert ei.value.code == gsls.ERR_NOT_PD


def test_update_bounds_then_resolve():
    p = W.box_lq()
    q = gsls.QP(p, gsls.default_settings(precision=gsls.FP64))
    p2 = p.copy()
    p2.u = p.u * 0.8; p2.l = p.l * 0.8
    q.update_bounds(p2.l, p2.u)
    q.solve(rho=1.0, tol=1e-7)
    g = q.get()
    o = _orc(p2, tol=1e-7)
    _close_all(g, o, 1e-9)


def test_device_descriptor_matches_host():
    """Problem data, x0 and the warm start given in device memory (torch
    tensors, GSLS_DEVICE): the same FP64 solve, iterate for iterate, as from
    host memory (cold, then warm from the cold solution)."""
    import ctypes as ct
    import torch
    p = W.polytopic_lq(40, 12, 4, 10, cfg_id=1, instance_id=7)
    s = gsls.default_settings(precision=gsls.FP64)
    q = gsls.QP(p, s)
    rh = q.solve(rho=1.0, tol=1e-7)
    gh = q.get()
    rhw = q.solve(rho=rh["rho"], tol=1e-8, z0=gh["z"], y0=gh["lam"] / rh["rho"])
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
    x0 = dev(p.x0)
    r = gsls.Result()
    assert gsls.lib.gsls_qp_solve(h, dptr(x0), 1.0, 1e-7, ct.byref(r)) == gsls.OK
    X = np.zeros((p.N + 1, p.nx)); z = np.zeros(p.m); lam = np.zeros(p.m)
    assert gsls.lib.gsls_qp_get(h, X.ctypes.data_as(ct.POINTER(ct.c_double)), None,
                                z.ctypes.data_as(ct.POINTER(ct.c_double)),
                                lam.ctypes.data_as(ct.POINTER(ct.c_double))) == gsls.OK
    assert r.iterations == rh["iterations"] and r.rho_updates == rh["rho_updates"]
    np.testing.assert_array_equal(X, gh["X"])
    z0, y0 = dev(z), dev(lam / r.rho)
    assert gsls.lib.gsls_qp_solve_warm(h, dptr(x0), r.rho, 1e-8, dptr(z0), dptr(y0), ct.byref(r)) == gsls.OK
    assert gsls.lib.gsls_qp_get(h, X.ctypes.data_as(ct.POINTER(ct.c_double)), None, None, None) == gsls.OK
    assert r.iterations == rhw["iterations"]
    np.testing.assert_array_equal(X, ghw["X"])
    gsls.lib.gsls_qp_free(h)
