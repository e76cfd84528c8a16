"""Dense FP64 references for the stage-structured LTV-QP (numpy).

TEST INFRASTRUCTURE ONLY; small sizes (KKT dimension up to a few thousand).

The QP is eq. (sqp_qp) of Sec. III-B with two-sided rows l <= G(xi) <= u.
Decision vector xi = (x_0, ..., x_N, u_0, ..., u_{N-1}).

  * ``assemble``        H, h (cost), Eq, e (dynamics and initial state),
                        Gm (constraint map G of Sec. IV-A).
  * ``lq_solve``        exact minimiser of the equality-constrained QP by one
                        dense KKT solve (the ADMM x-update, eq. (primal_update)).
  * ``admm``            ADMM of Sec. III-C on eq. (admm_qp) with the dense KKT
                        x-update; same rho rule and residuals as the Riccati
                        oracle but written independently of it.
  * ``kkt_residuals``   stationarity / feasibility / sign / complementarity.
  * ``active_set_qp``   exact optimum by enumerating active sets (tiny QPs).
  * ``condensed_lq``    unconstrained LQ optimum by eliminating the states
                        (a second, independent exact solve).
"""
from __future__ import annotations

import itertools

import numpy as np


def _xi_index(prob):
    N, nx, nu = prob.N, prob.nx, prob.nu
    nX = (N + 1) * nx
    xs = [slice(k * nx, (k + 1) * nx) for k in range(N + 1)]
    us = [slice(nX + k * nu, nX + (k + 1) * nu) for k in range(N)]
    return nX + N * nu, xs, us


def assemble(prob):
    """Dense H, h, Eq, e, Gm for the QP."""
    N, nx, nu, nc, nf = prob.N, prob.nx, prob.nu, prob.nc, prob.nf
    n, xs, us = _xi_index(prob)
    H = np.zeros((n, n)); h = np.zeros(n)
    for k in range(N):
        H[xs[k], xs[k]] = prob.Q[k]
        H[us[k], us[k]] = prob.R[k]
        H[us[k], xs[k]] = prob.S[k]
        H[xs[k], us[k]] = prob.S[k].T
        h[xs[k]] = prob.q[k]; h[us[k]] = prob.r[k]
    H[xs[N], xs[N]] = prob.Q[N]; h[xs[N]] = prob.q[N]
    neq = (N + 1) * nx
    Eq = np.zeros((neq, n)); e = np.zeros(neq)
    Eq[0:nx, xs[0]] = np.eye(nx); e[0:nx] = prob.x0
    for k in range(N):
        r = slice((k + 1) * nx, (k + 2) * nx)
        Eq[r, xs[k + 1]] = np.eye(nx)
        Eq[r, xs[k]] = -prob.A[k]
        Eq[r, us[k]] = -prob.B[k]
        e[r] = prob.b[k]
    m = N * nc + nf
    Gm = np.zeros((m, n))
    for k in range(N):
        Gm[k * nc:(k + 1) * nc, xs[k]] = prob.C[k]
        Gm[k * nc:(k + 1) * nc, us[k]] = prob.D[k]
    if nf:
        Gm[N * nc:, xs[N]] = prob.CN
    return H, h, Eq, e, Gm


def split(prob, xi):
    n, xs, us = _xi_index(prob)
    X = np.stack([xi[s] for s in xs]); U = np.stack([xi[s] for s in us]) if prob.N else None
    return X, U


def join(prob, X, U):
    return np.concatenate([X.reshape(-1), U.reshape(-1)])


def lq_solve(H, h, Eq, e):
    """argmin 1/2 xi^T H xi + h^T xi  s.t.  Eq xi = e, by one dense KKT solve.
    Returns (xi, mu) with H xi + h + Eq^T mu = 0."""
    n = H.shape[0]; neq = Eq.shape[0]
    K = np.zeros((n + neq, n + neq))
    K[:n, :n] = H; K[:n, n:] = Eq.T; K[n:, :n] = Eq
    sol = np.linalg.solve(K, np.concatenate([-h, e]))
    return sol[:n], sol[n:]


def admm(prob, rho=1.0, tol=1e-6, max_iter=10000, adaptive=True, sigma=25, rho_min=1e-6,
         rho_max=1e6, rho_tol=5.0, z0=None, y0=None):
    """ADMM with the dense KKT x-update.  Returns dict like oracle.qp_solve."""
    H, h, Eq, e, Gm = assemble(prob)
    l, u = prob.l, prob.u
    m = Gm.shape[0]
    z = np.zeros(m) if z0 is None else np.array(z0, float)
    y = np.zeros(m) if y0 is None else np.array(y0, float)
    hn = np.max(np.abs(h)) if h.size else 0.0
    nupd = 0
    status = 2
    it = 0
    rp = rd = np.inf
    xi = None
    for it in range(1, max_iter + 1):
        # x-update: minimise J + rho/2 |G xi - z + y|^2 subject to the dynamics
        xi, _ = lq_solve(H + rho * Gm.T @ Gm, h + rho * Gm.T @ (y - z), Eq, e)
        v = Gm @ xi
        zn = np.clip(v + y, l, u)
        y = y + v - zn
        rp = np.max(np.abs(v - zn)) if m else 0.0
        rd = rho * np.max(np.abs(Gm.T @ (zn - z))) if m else 0.0
        z = zn
        if rp <= tol and rd <= tol:
            status = 1
            break
        if it == max_iter:
            break
        if adaptive and it % sigma == 0:
            ps = max(np.max(np.abs(v)), np.max(np.abs(z)))
            ds = max(np.max(np.abs(H @ xi)), np.max(np.abs(Gm.T @ (rho * y))), hn)
            rn = rho * np.sqrt((rp / (ps + 1e-10)) / (rd / (ds + 1e-10) + 1e-10))
            rn = min(max(rn, rho_min), rho_max)
            if rn > rho * rho_tol or rn < rho / rho_tol:
                y = y * (rho / rn)
                rho = rn
                nupd += 1
    X, U = split(prob, xi)
    return dict(X=X, U=U, z=z, y=y, lam=rho * y, iters=it, r_p=rp, r_d=rd, rho=rho,
                rho_updates=nupd, status=status)


def kkt_residuals(prob, X, U, lam):
    """KKT residuals of a primal-dual point of the QP with multipliers lam of
    the rows l <= G xi <= u (lam > 0 pushes against the upper bound).

    Returns dict: stat (|H xi + h + G^T lam + Eq^T mu|_inf with the least-squares
    dynamics multiplier mu), prim (bound violation), dyn (dynamics residual),
    comp (max of |lam_i| times the slack of the bound its sign selects)."""
    H, h, Eq, e, Gm = assemble(prob)
    xi = join(prob, X, U)
    g = H @ xi + h + Gm.T @ lam
    mu, *_ = np.linalg.lstsq(Eq.T, -g, rcond=None)
    stat = np.max(np.abs(g + Eq.T @ mu))
    v = Gm @ xi
    prim = max(np.max(np.maximum(v - prob.u, 0.0), initial=0.0),
               np.max(np.maximum(prob.l - v, 0.0), initial=0.0))
    dyn = np.max(np.abs(Eq @ xi - e))
    # complementarity: a positive multiplier needs the upper bound active, a
    # negative one the lower bound; an infinite bound admits no multiplier
    up_slack = np.where(np.isfinite(prob.u), prob.u - v, 1e30)
    lo_slack = np.where(np.isfinite(prob.l), v - prob.l, 1e30)
    pos = np.maximum(lam, 0.0); neg = np.maximum(-lam, 0.0)
    comp = max(np.max(pos * up_slack, initial=0.0), np.max(neg * lo_slack, initial=0.0))
    return dict(stat=stat, prim=prim, dyn=dyn, comp=comp)


def active_set_qp(prob, max_rows=12):
    """Exact optimum of a tiny QP by enumeration: every row is inactive, at its
    lower bound or at its upper bound; for each choice solve the equality
    QP and keep the point that is primal feasible with multipliers of the right
    sign.  The primal optimum of a strictly convex QP is unique."""
    H, h, Eq, e, Gm = assemble(prob)
    m = Gm.shape[0]
    if m > max_rows:
        raise ValueError("active_set_qp: too many rows for enumeration")
    choices = []
    for i in range(m):
        c = [0]
        if np.isfinite(prob.l[i]):
            c.append(-1)
        if np.isfinite(prob.u[i]):
            c.append(1)
        choices.append(c)
    best = None
    for pat in itertools.product(*choices):
        act = [i for i in range(m) if pat[i] != 0]
        bnd = np.array([prob.u[i] if pat[i] > 0 else prob.l[i] for i in act])
        Ea = np.vstack([Eq, Gm[act]]) if act else Eq
        ea = np.concatenate([e, bnd]) if act else e
        try:
            xi, mu = lq_solve(H, h, Ea, ea)
        except np.linalg.LinAlgError:
            continue
        # skip active sets whose equality system is inconsistent or degenerate
        if (np.max(np.abs(Ea @ xi - ea)) > 1e-9
                or np.max(np.abs(H @ xi + h + Ea.T @ mu)) > 1e-9):
            continue
        v = Gm @ xi
        if np.any(v > prob.u + 1e-9) or np.any(v < prob.l - 1e-9):
            continue
        lam_a = mu[Eq.shape[0]:]
        ok = all((pat[i] > 0 and lam_a[t] >= -1e-9) or (pat[i] < 0 and lam_a[t] <= 1e-9)
                 for t, i in enumerate(act))
        if not ok:
            continue
        lam = np.zeros(m)
        lam[act] = lam_a
        cost = 0.5 * xi @ H @ xi + h @ xi
        if best is None or cost < best[0] - 1e-12:
            best = (cost, xi, lam)
    if best is None:
        raise ValueError("active_set_qp: infeasible")
    X, U = split(prob, best[1])
    return dict(X=X, U=U, lam=best[2], cost=best[0])


def condensed_lq(prob, Qh, Rh, Sh, qh, rh):
    """Unconstrained LQ optimum by eliminating the states: x = F x0 + Gu u + g,
    then the normal equations in u alone.  Independent of the KKT solve."""
    N, nx, nu = prob.N, prob.nx, prob.nu
    nX = (N + 1) * nx
    F = np.zeros((nX, nx)); Gu = np.zeros((nX, N * nu)); g = np.zeros(nX)
    F[:nx] = np.eye(nx)
    for k in range(N):
        r0, r1 = slice(k * nx, (k + 1) * nx), slice((k + 1) * nx, (k + 2) * nx)
        F[r1] = prob.A[k] @ F[r0]
        Gu[r1] = prob.A[k] @ Gu[r0]
        Gu[r1, k * nu:(k + 1) * nu] += prob.B[k]
        g[r1] = prob.A[k] @ g[r0] + prob.b[k]
    Hx = np.zeros((nX, nX)); Hu = np.zeros((N * nu, N * nu)); Hux = np.zeros((N * nu, nX))
    hx = np.zeros(nX); hu = np.zeros(N * nu)
    for k in range(N):
        Hx[k * nx:(k + 1) * nx, k * nx:(k + 1) * nx] = Qh[k]
        Hu[k * nu:(k + 1) * nu, k * nu:(k + 1) * nu] = Rh[k]
        Hux[k * nu:(k + 1) * nu, k * nx:(k + 1) * nx] = Sh[k]
        hx[k * nx:(k + 1) * nx] = qh[k]; hu[k * nu:(k + 1) * nu] = rh[k]
    Hx[N * nx:, N * nx:] = Qh[N]; hx[N * nx:] = qh[N]
    xa = F @ prob.x0 + g
    # cost(u) = 1/2 x^T Hx x + u^T Hux x + 1/2 u^T Hu u + hx^T x + hu^T u, x = xa + Gu u
    M = Gu.T @ Hx @ Gu + Hux @ Gu + Gu.T @ Hux.T + Hu
    rhs = Gu.T @ (Hx @ xa + hx) + Hux @ xa + hu
    uu = np.linalg.solve(M, -rhs)
    X = (xa + Gu @ uu).reshape(N + 1, nx)
    return X, uu.reshape(N, nu)
