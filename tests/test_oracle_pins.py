"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

Nothing here compares the oracle with itself: each check uses an independent
route (closed-form DARE, a dense KKT solve, elimination of the states,
active-set enumeration, KKT conditions, finite differences, the worst-case
disturbance) so that a dropped term, a wrong sign, index or transpose in the
oracle fails at least one of them.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from oracle import dense, scan
from paper_2604_07644_amd import workloads as W


def _ti_problem(N=12, nx=3, nu=2, nc=0, nf=0, seed=0):
    """Time-invariant problem (same A, B, Q, R, C, D every stage)."""
    rng = np.random.default_rng([5, seed])
    A = np.eye(nx) + 0.3 * rng.standard_normal((nx, nx))
    B = rng.standard_normal((nx, nu))
    M = rng.standard_normal((nx, nx)); Q = M @ M.T + np.eye(nx)
    M = rng.standard_normal((nu, nu)); R = M @ M.T + 0.5 * np.eye(nu)
    C = rng.standard_normal((nc, nx)); D = rng.standard_normal((nc, nu))
    p = W.random_small(N, nx, nu, nc, nf, seed=seed)
    p.A[:] = A; p.B[:] = B; p.Q[:] = Q; p.R[:] = R; p.C[:] = C; p.D[:] = D
    p.S[:] = 0; p.b[:] = 0
    return p


@pytest.mark.parametrize("rho", [0.0, 0.7])
def test_riccati_factor_equals_dare(rho):
    """Time-invariant data with Q_N = P_DARE: every P_i is P_DARE, every K_i is
    K_DARE (closed form), including the rho-augmented cross term S + rho D^T C."""
    p = _ti_problem(nc=2)
    A, B = p.A[0], p.B[0]
    Qh = p.Q[0] + rho * p.C[0].T @ p.C[0]
    Rh = p.R[0] + rho * p.D[0].T @ p.D[0]
    Sh = rho * p.D[0].T @ p.C[0]              # nu x nx
    P = sla.solve_discrete_are(A, B, Qh, Rh, s=Sh.T)
    K = -np.linalg.solve(Rh + B.T @ P @ B, B.T @ P @ A + Sh)
    p.Q[-1] = P
    p.nf = 0
    Po, Ko = oracle.qp_factor(p, rho)
    for i in range(p.N + 1):
        np.testing.assert_allclose(Po[i], P, rtol=1e-9, atol=1e-9)
    for i in range(p.N):
        np.testing.assert_allclose(Ko[i], K, rtol=1e-9, atol=1e-9)


def test_unconstrained_one_iteration_equals_condensed_lq():
    """nc = nf = 0: ADMM stops after one x-update at the LQ optimum, which the
    state-eliminated normal equations give independently."""
    p = W.random_small(10, 4, 2, 0, 0, seed=3)
    r = oracle.qp_solve(p, rho=1.0, tol=1e-12)
    assert r["status"] == 1 and r["iters"] == 1
    X, U = dense.condensed_lq(p, p.Q, p.R, p.S, p.q, p.r)
    np.testing.assert_allclose(r["X"], X, atol=1e-10)
    np.testing.assert_allclose(r["U"], U, atol=1e-10)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_riccati_xupdate_equals_dense_kkt(seed):
    """One ADMM x-update from an arbitrary (z, y) equals the dense KKT solve of
    eq. (primal_update), with every term present (S, b, q, r, terminal rows)."""
    p = W.random_small(7, 4, 3, 3, 2, seed=seed)
    rng = np.random.default_rng(seed)
    z0 = rng.standard_normal(p.m); y0 = rng.standard_normal(p.m); rho = 0.37
    r = oracle.qp_solve(p, rho=rho, tol=0.0, settings=oracle.Settings(max_iter=1, adaptive=False),
                        z0=z0, y0=y0)
    H, h, Eq, e, Gm = dense.assemble(p)
    xi, _ = dense.lq_solve(H + rho * Gm.T @ Gm, h + rho * Gm.T @ (y0 - z0), Eq, e)
    X, U = dense.split(p, xi)
    np.testing.assert_allclose(r["X"], X, atol=1e-10)
    np.testing.assert_allclose(r["U"], U, atol=1e-10)
    # the same minimiser by state elimination with the augmented costs
    Qh, Rh, Sh, qh, rh = scan.augmented(p, rho, y0, z0)
    X2, U2 = dense.condensed_lq(p, Qh, Rh, Sh, qh, rh)
    np.testing.assert_allclose(r["X"], X2, atol=1e-9)


@pytest.mark.parametrize("iters", [1, 5, 40])
def test_riccati_admm_iterates_equal_dense_admm(iters):
    """Fixed rho: the Riccati ADMM and the dense-KKT ADMM agree iterate by iterate."""
    p = W.random_small(8, 3, 2, 4, 3, seed=11)
    a = oracle.qp_solve(p, rho=0.8, tol=0.0, settings=oracle.Settings(max_iter=iters, adaptive=False))
    b = dense.admm(p, rho=0.8, tol=0.0, max_iter=iters, adaptive=False)
    for k in ("X", "U", "z", "y"):
        np.testing.assert_allclose(a[k], b[k], atol=1e-10)


def test_adaptive_rho_trajectories_agree():
    p = W.box_lq()
    a = oracle.qp_solve(p, rho=1.0, tol=1e-6)
    b = dense.admm(p, rho=1.0, tol=1e-6)
    assert a["iters"] == b["iters"] and a["rho_updates"] == b["rho_updates"] > 0
    np.testing.assert_allclose(a["rho"], b["rho"], rtol=1e-9)
    np.testing.assert_allclose(a["X"], b["X"], atol=1e-9)


def _tiny_box(seed):
    p = W.box_lq(N=3, nx=2, nu=1, cfg_id=50, instance_id=seed, xmax=1.2, umax=0.4,
                 terminal_box=False)
    # bound only the controls and the first state coordinate: 3 stages x 2 rows
    p.C = p.C[:, [0, 2], :]; p.D = p.D[:, [0, 2], :]; p.nc = 2
    p.l = np.tile([-1.2, -0.4], 3); p.u = -p.l
    p.x0 = np.array([1.0, -0.8])
    return p


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_admm_equals_active_set_bruteforce(seed):
    """Tiny box QPs: ADMM run to 1e-11 reaches the optimum found by enumerating
    every active set."""
    p = _tiny_box(seed)
    ex = dense.active_set_qp(p)
    r = oracle.qp_solve(p, rho=1.0, tol=1e-11, settings=oracle.Settings(max_iter=100000))
    assert r["status"] == 1
    np.testing.assert_allclose(r["X"], ex["X"], atol=1e-8)
    np.testing.assert_allclose(r["U"], ex["U"], atol=1e-8)
    np.testing.assert_allclose(r["lam"], ex["lam"], atol=1e-7)


@pytest.mark.parametrize("maker", ["box", "small", "quad"])
def test_admm_solution_satisfies_kkt(maker):
    if maker == "box":
        p, tol = W.box_lq(), 1e-8
    elif maker == "small":
        p, tol = W.random_small(9, 4, 2, 5, 3, seed=4), 1e-8
    else:
        p, tol = W.polytopic_lq(16, 8, 3, 6, cfg_id=1, instance_id=3), 1e-8
    r = oracle.qp_solve(p, rho=1.0, tol=tol)
    assert r["status"] == 1
    k = dense.kkt_residuals(p, r["X"], r["U"], r["lam"])
    # r_d bounds the stationarity residual and r_p the bound violation
    assert k["stat"] <= 10 * tol and k["prim"] <= 10 * tol and k["dyn"] <= 1e-12
    assert k["comp"] <= 1e-5


# ------------------------------------------------------------------ scans

def _rand_elem(rng, n):
    M = rng.standard_normal((n, n)); P = M @ M.T / n
    M = rng.standard_normal((n, n)); C = M @ M.T / n
    return (P, rng.standard_normal(n), rng.standard_normal((n, n)) / np.sqrt(n), C,
            rng.standard_normal(n))


def test_combine_is_associative_with_identity():
    rng = np.random.default_rng(0)
    a, b, c = (_rand_elem(rng, 5) for _ in range(3))
    l = scan.combine(scan.combine(a, b), c)
    r = scan.combine(a, scan.combine(b, c))
    for x, y in zip(l, r):
        np.testing.assert_allclose(x, y, rtol=1e-12, atol=1e-12)
    e = scan.identity(5)
    for x, y in zip(scan.combine(e, a), a):
        assert np.array_equal(x, y) or np.allclose(x, y, rtol=0, atol=0)
    for x, y in zip(scan.combine(a, e), a):
        np.testing.assert_allclose(x, y, rtol=0, atol=1e-15)


@pytest.mark.parametrize("tree", [False, True])
def test_suffix_scan_gives_riccati_and_kkt_solution(tree):
    """The reverse scan's P_i equal the Riccati P_i; the scan's x-update equals
    the dense KKT solve."""
    p = W.random_small(13, 4, 2, 3, 2, seed=7)
    rng = np.random.default_rng(3)
    y = rng.standard_normal(p.m); z = rng.standard_normal(p.m); rho = 1.3
    s = scan.lqr_by_scan(p, rho, y, z, tree=tree)
    P, K = oracle.qp_factor(p, rho)
    np.testing.assert_allclose(s["P"], P, rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(s["K"], K, rtol=1e-10, atol=1e-10)
    H, h, Eq, e, Gm = dense.assemble(p)
    xi, _ = dense.lq_solve(H + rho * Gm.T @ Gm, h + rho * Gm.T @ (y - z), Eq, e)
    X, U = dense.split(p, xi)
    np.testing.assert_allclose(s["X"], X, atol=1e-10)
    np.testing.assert_allclose(s["U"], U, atol=1e-10)


def test_printed_p_sign_is_wrong():
    """The p-rule's printed minus sign does not give the Riccati p_i; the
    reading with plus does (previous test)."""
    p = W.random_small(9, 3, 2, 2, 0, seed=8)
    rng = np.random.default_rng(4)
    y = rng.standard_normal(p.m); z = rng.standard_normal(p.m)
    Qh, Rh, Sh, qh, rh = scan.augmented(p, 1.0, y, z)
    els = scan.elements(p, Qh, Rh, Sh, qh, rh)
    good = scan.suffix_scan(els)
    bad = scan.suffix_scan(els, op=lambda a, b: scan.combine(a, b, p_sign=-1.0))
    assert np.max(np.abs(good[0][1] - bad[0][1])) > 1e-3


def test_forward_scan_equals_rollout():
    p = W.random_small(11, 4, 2, 0, 0, seed=9)
    rng = np.random.default_rng(1)
    K = rng.standard_normal((p.N, p.nu, p.nx)) * 0.3; k = rng.standard_normal((p.N, p.nu))
    X, U = scan.forward_scan(p, K, k, p.x0)
    x = p.x0.copy()
    for i in range(p.N):
        np.testing.assert_allclose(X[i], x, atol=1e-12)
        u = K[i] @ x + k[i]
        np.testing.assert_allclose(U[i], u, atol=1e-12)
        x = p.A[i] @ x + p.B[i] @ u + p.b[i]
    np.testing.assert_allclose(X[-1], x, atol=1e-12)


# -------------------------------------------------------------------- SLS

def _sls_small(N=7, nx=3, nu=2, nc=4, nf=2, seed=0, ti=False):
    p = _ti_problem(N, nx, nu, nc, nf, seed) if ti else W.random_small(N, nx, nu, nc, nf, seed)
    rng = np.random.default_rng([6, seed])
    E = rng.standard_normal((N, nx, nx)) * 0.3
    return p, E


def test_sls_tau_zero_is_lqr_closed_form():
    """tau = 0, time-invariant, Qbar_N = P_DARE: every column's gain is K_DARE
    and Phi^x_{k,j} = (A + B K)^{k-j-1} E_j."""
    p, E = _sls_small(ti=True, nc=3, nf=2)
    A, B = p.A[0], p.B[0]
    Qb = np.eye(p.nx); Rb = np.eye(p.nu)
    P = sla.solve_discrete_are(A, B, Qb, Rb)
    K = -np.linalg.solve(Rb + B.T @ P @ B, B.T @ P @ A)
    tau = np.zeros(p.N * p.N * p.nc + p.N * p.nf)
    r = oracle.sls_solve(p, E, tau, Qb, Rb, P, want_K=True)
    offx, offu = oracle.native.sls_layout(p.N)
    Acl = A + B @ K
    for j in range(p.N):
        for k in range(j + 1, p.N + 1):
            F = np.linalg.matrix_power(Acl, k - j - 1) @ E[j]
            np.testing.assert_allclose(r["Phi_x"][offx[j] + k - j - 1], F, atol=1e-9)
            if k < p.N:
                np.testing.assert_allclose(r["K"][k, j], K, atol=1e-9)
                np.testing.assert_allclose(r["Phi_u"][offu[j] + k - j - 1], K @ F, atol=1e-9)


def _rand_tau(p, rng):
    return np.abs(rng.standard_normal(p.N * p.N * p.nc + p.N * p.nf)) * 2.0


def test_sls_dynamics_invariant_and_robust_scan():
    """Phi^x_{k+1,j} = A_k Phi^x_{k,j} + B_k Phi^u_{k,j}; the robust CVF suffix
    scan gives the same gains as the per-column Riccati recursion."""
    p, E = _sls_small(seed=2)
    rng = np.random.default_rng(2)
    tau = _rand_tau(p, rng)
    Qb, Rb, QbN = np.eye(p.nx), 0.5 * np.eye(p.nu), 2.0 * np.eye(p.nx)
    r = oracle.sls_solve(p, E, tau, Qb, Rb, QbN, want_K=True)
    offx, offu = oracle.native.sls_layout(p.N)
    N = p.N
    ts = tau[:N * N * p.nc].reshape(N, N, p.nc); tN = tau[N * N * p.nc:].reshape(N, p.nf)
    for j in range(N):
        np.testing.assert_allclose(r["Phi_x"][offx[j]], E[j], atol=0)
        for k in range(j + 1, N):
            Fx = r["Phi_x"][offx[j] + k - j - 1]; Fu = r["Phi_u"][offu[j] + k - j - 1]
            np.testing.assert_allclose(r["Phi_x"][offx[j] + k - j], p.A[k] @ Fx + p.B[k] @ Fu,
                                       atol=1e-12)
        col = {k: ts[k, j] for k in range(j + 1, N)}; col[N] = tN[j]
        els = scan.robust_elements(p, col, j, Qb, Rb, QbN)
        suf = scan.suffix_scan(els)
        for t, k in enumerate(range(j + 1, N)):
            Pn = suf[t + 1][0]
            T = np.diag(ts[k, j])
            Qu = p.D[k].T @ T @ p.D[k] + Rb; Qux = p.D[k].T @ T @ p.C[k]
            Kk = -np.linalg.solve(Qu + p.B[k].T @ Pn @ p.B[k], Qux + p.B[k].T @ Pn @ p.A[k])
            np.testing.assert_allclose(r["K"][k, j], Kk, atol=1e-10)


@pytest.mark.parametrize("rownorm", [2, 1])
def test_sls_margin_is_attained_by_worst_case_disturbance(rownorm):
    """Closed loop under disturbance feedback: the aligned worst-case w_j makes
    row i of C_k dx_k + D_k du_k equal h_k[i] exactly; random admissible w
    never exceed it."""
    p, E = _sls_small(seed=5, nc=3, nf=2)
    rng = np.random.default_rng(5)
    tau = _rand_tau(p, rng); wb = 0.3
    Qb, Rb, QbN = np.eye(p.nx), np.eye(p.nu), np.eye(p.nx)
    r = oracle.sls_solve(p, E, tau, Qb, Rb, QbN, rownorm=rownorm, wbound=wb)
    offx, offu = oracle.native.sls_layout(p.N)
    N = p.N

    def deviation(ws, k):
        """closed-loop deviation (C dx + D du) at stage k from Phi and w."""
        dx = np.zeros(p.nx); du = np.zeros(p.nu)
        for j in range(k):
            dx += r["Phi_x"][offx[j] + k - j - 1] @ ws[j]
            if k < N:
                du += r["Phi_u"][offu[j] + k - j - 1] @ ws[j]
        return (p.C[k] @ dx + p.D[k] @ du) if k < N else p.CN @ dx

    for k in (2, N - 1, N):
        rows = p.nc if k < N else p.nf
        for i in range(rows):
            ws = []
            for j in range(N):
                if j < k:
                    Fx = r["Phi_x"][offx[j] + k - j - 1]
                    M = (p.C[k] @ Fx + p.D[k] @ r["Phi_u"][offu[j] + k - j - 1]) if k < N else p.CN @ Fx
                    row = M[i]
                    w = row / np.linalg.norm(row) if rownorm == 2 else np.sign(row)
                    ws.append(wb * w)
                else:
                    ws.append(np.zeros(p.nx))
            hv = r["h"][k, i] if k < N else r["hf"][i]
            np.testing.assert_allclose(deviation(ws, k)[i], hv, rtol=1e-12)
            for _ in range(20):
                wr = rng.standard_normal((N, p.nx))
                wr = wb * (wr / np.linalg.norm(wr, axis=1, keepdims=True) if rownorm == 2
                           else np.sign(wr))
                assert abs(deviation(wr, k)[i]) <= hv * (1 + 1e-12)


def test_sls_tau_matches_gradient_of_tightening():
    """tau_{k,j} makes the quadratic surrogate 1/2 tau |M_r|^2 have the same
    gradient as the multiplier-weighted smoothed margin |lambda| sqrt(|M_r|^2+eps)
    (App. B), checked by finite differences on each row."""
    p, E = _sls_small(seed=6, nc=3, nf=2)
    rng = np.random.default_rng(6)
    tau0 = _rand_tau(p, rng)
    r = oracle.sls_solve(p, E, tau0, np.eye(p.nx), np.eye(p.nu), np.eye(p.nx))
    lam = rng.standard_normal(p.m)
    eps = 1e-8
    tau = oracle.sls_tau(p, lam, r["Phi_x"], r["Phi_u"], eps)
    offx, offu = oracle.native.sls_layout(p.N)
    N = p.N
    for (k, j) in [(1, 0), (4, 2), (N - 1, 0), (N, 3)]:
        Fx = r["Phi_x"][offx[j] + k - j - 1]
        M = (p.C[k] @ Fx + p.D[k] @ r["Phi_u"][offu[j] + k - j - 1]) if k < N else p.CN @ Fx
        for i in range(M.shape[0]):
            li = lam[k * p.nc + i]
            f = lambda row: abs(li) * np.sqrt(row @ row + eps)  # noqa: E731
            g = np.zeros(p.nx); hstep = 1e-6
            for c in range(p.nx):
                e = np.zeros(p.nx); e[c] = hstep
                g[c] = (f(M[i] + e) - f(M[i] - e)) / (2 * hstep)
            t = tau[(k * N + j) * p.nc + i] if k < N else tau[N * N * p.nc + j * p.nf + i]
            np.testing.assert_allclose(g, t * M[i], rtol=1e-5, atol=1e-9)


def _rho_case(primal_dominant):
    """Small QP with general rows, a penalty and a starting iterate chosen so
    that, after one x-update, the scaled primal residual dominates the scaled
    dual residual (tight rows, small rho, start at z = y = 0) or the reverse
    (a large rho that pins G xi to a start z which the projection then moves)."""
    p = W.random_small(6, 3, 2, 4, 2, seed=21, lower=True)
    m = p.m
    rng = np.random.default_rng([21, 1])
    if primal_dominant:
        # rows that the first step violates by a lot
        p.l = -0.02 * np.ones(m); p.u = 0.02 * np.ones(m)
        z0 = np.zeros(m); y0 = np.zeros(m); rho = 0.7
    else:
        p.l = -0.3 * np.ones(m); p.u = 0.3 * np.ones(m)
        z0 = rng.uniform(-0.15, 0.15, m); y0 = np.zeros(m); rho = 10.0
    return p, z0, y0, rho


def _scaled_residuals(p, rho, X, U, z_prev, z, y):
    """The two scaled residuals of the rule, from the dense assembly: primal
    |G xi - z| / max(|G xi|, |z|), dual rho |G^T (z - z_prev)| /
    max(|H xi|, |G^T rho y|, |h|) (infinity norms)."""
    H, h, Eq, e, Gm = dense.assemble(p)
    xi = dense.join(p, X, U)
    v = Gm @ xi
    rp = np.max(np.abs(v - z))
    rd = rho * np.max(np.abs(Gm.T @ (z - z_prev)))
    ps = max(np.max(np.abs(v)), np.max(np.abs(z)))
    ds = max(np.max(np.abs(H @ xi)), np.max(np.abs(Gm.T @ (rho * y))), np.max(np.abs(h)))
    return rp / ps, rd / ds


@pytest.mark.parametrize("primal_dominant", [True, False])
def test_rho_rule_direction_magnitude_and_dual_continuity(primal_dominant):
    """The adaptive penalty (Sec. IV-A, which defers to the residual-balancing
    rule of OSQP): when the scaled primal residual dominates, rho must grow,
    when the scaled dual residual dominates it must shrink, by the square root
    of their ratio (the geometric mean that balances them), and the change
    must leave the unscaled multiplier lambda = rho y untouched, so that the
    iteration continues exactly as a fresh run at the new rho started from
    (z, lambda / rho_new).  The residuals are measured here on the dense
    assembly of the QP, not read from the oracle."""
    p, z0, y0, rho = _rho_case(primal_dominant)
    fixed = oracle.Settings(max_iter=1, adaptive=False)
    one = oracle.qp_solve(p, rho=rho, tol=0.0, settings=fixed, z0=z0, y0=y0)
    sp, sd = _scaled_residuals(p, rho, one["X"], one["U"], z0, one["z"], one["y"])
    assert (sp > 10 * sd) if primal_dominant else (sd > 10 * sp)
    # rule applied after iteration 1 (sigma = 1, always applied), then one more
    # iteration at the new rho
    adapt = oracle.Settings(max_iter=2, adaptive=True, sigma=1, rho_tol=1.0 + 1e-12)
    two = oracle.qp_solve(p, rho=rho, tol=0.0, settings=adapt, z0=z0, y0=y0)
    assert two["rho_updates"] == 1
    rho_new = two["rho"]
    assert (rho_new > rho) if primal_dominant else (rho_new < rho)
    np.testing.assert_allclose(rho_new / rho, np.sqrt(sp / sd), rtol=1e-8)
    # dual continuity: lambda = rho y kept, so a fresh iteration at rho_new from
    # (z1, y1 rho / rho_new) reproduces the adaptive run's second iterate
    fresh = oracle.qp_solve(p, rho=rho_new, tol=0.0, settings=fixed, z0=one["z"], y0=one["y"] * rho / rho_new)
    for k in ("X", "U", "z", "y"):
        np.testing.assert_allclose(two[k], fresh[k], rtol=1e-10, atol=1e-12)


def test_rho_rule_band_and_clamp():
    """No change while the proposed factor stays inside [1/rho_tol, rho_tol];
    the proposal is clamped to [rho_min, rho_max]."""
    p, z0, y0, rho = _rho_case(True)
    one = oracle.qp_solve(p, rho=rho, tol=0.0, settings=oracle.Settings(max_iter=1, adaptive=False), z0=z0, y0=y0)
    sp, sd = _scaled_residuals(p, rho, one["X"], one["U"], z0, one["z"], one["y"])
    factor = np.sqrt(sp / sd)
    wide = oracle.Settings(max_iter=2, adaptive=True, sigma=1, rho_tol=2 * factor)
    r = oracle.qp_solve(p, rho=rho, tol=0.0, settings=wide, z0=z0, y0=y0)
    assert r["rho_updates"] == 0 and r["rho"] == rho
    cap = rho * factor / 3
    clamp = oracle.Settings(max_iter=2, adaptive=True, sigma=1, rho_tol=1.0 + 1e-12, rho_max=cap)
    r = oracle.qp_solve(p, rho=rho, tol=0.0, settings=clamp, z0=z0, y0=y0)
    assert r["rho_updates"] == 1 and r["rho"] == cap
