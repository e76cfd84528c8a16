"""FastSLS alternation (robust MPC composition) on one LTV-QP, in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. III-D alternates two problems until they agree:
  (A) the nominal trajectory, eq. (nmpc_problem_tightened): the QP with its
      constraints tightened by the reachable-set margins h of the current
      controller, g + h <= 0 (the QP of Sec. III-B with rows l <= G xi <= u);
  (B) the controller, eq. (fastsls_qp): the SLS problem whose weights tau are
      the multipliers of (A) divided by the responses' row norms (App. B).
Readings taken here (the paper fixes none of them):
  * a row l <= g <= u is tightened on its finite sides, l + h <= g <= u - h:
    h bounds |row . (x - xbar; u - ubar)| over the disturbance set;
  * the first controller has tau = 0 (objective H~_0);
  * one pass = nominal solve with the current margins, tau from its
    multipliers and the current responses, SLS with that tau (new responses
    and margins).  The alternation stops when the margins move by at most
    htol * max(1, |h|_inf), or after max_passes passes, and ends with one more
    nominal solve with the final margins, so the returned trajectory and
    margins belong together;
  * every nominal solve starts cold (z = y = 0) from the given rho.
Outcome codes follow the C ABI: 1 converged, 2 pass limit reached,
4 tightened bounds cross (l + h > u - h on some row), 5 a nominal solve did
not converge.
"""
from __future__ import annotations

import numpy as np

from .native import qp_solve, sls_solve, sls_tau

CONVERGED, PASS_LIMIT, TIGHTENING_INFEASIBLE, NOMINAL_FAILED = 1, 2, 4, 5


def margin_rows(h, hf):
    """Margins in the row layout of l and u: stage rows k*nc.., then terminal rows."""
    return np.concatenate([np.asarray(h, dtype=np.float64).ravel(), np.asarray(hf, dtype=np.float64).ravel()])


def tighten(l, u, hrow):
    """l + h on finite lower sides, u - h on finite upper sides."""
    l = np.asarray(l, dtype=np.float64); u = np.asarray(u, dtype=np.float64)
    return np.where(np.isfinite(l), l + hrow, l), np.where(np.isfinite(u), u - hrow, u)


def robust_alternation(p, E, Qbar, Rbar, QbarN, rownorm=1, wbound=1.0, eps=1e-8, rho=1.0, tol=1e-6,
                       max_passes=10, htol=1e-3):
    N, nc, nf = p.N, p.nc, p.nf
    ctl = sls_solve(p, E, np.zeros(N * N * nc + N * nf), Qbar, Rbar, QbarN, rownorm=rownorm, wbound=wbound)
    hrow = margin_rows(ctl["h"], ctl["hf"])
    passes = qp_solves = qp_iters = 0
    change = np.inf
    status = PASS_LIMIT
    nom = None
    while True:
        lt, ut = tighten(p.l, p.u, hrow)
        if np.any(lt > ut):
            status = TIGHTENING_INFEASIBLE
            break
        q = p.copy()
        q.l, q.u = lt, ut
        nom = qp_solve(q, rho=rho, tol=tol)
        qp_solves += 1
        qp_iters += nom["iters"]
        if nom["status"] != 1:
            status = NOMINAL_FAILED
            break
        if status == CONVERGED or passes >= max_passes:
            break
        tau = sls_tau(p, nom["lam"], ctl["Phi_x"], ctl["Phi_u"], eps=eps)
        ctl = sls_solve(p, E, tau, Qbar, Rbar, QbarN, rownorm=rownorm, wbound=wbound)
        hnew = margin_rows(ctl["h"], ctl["hf"])
        change = float(np.max(np.abs(hnew - hrow))) if hrow.size else 0.0
        hrow = hnew
        passes += 1
        if change <= htol * max(1.0, float(np.max(np.abs(hrow))) if hrow.size else 0.0):
            status = CONVERGED
    out = dict(status=status, passes=passes, qp_solves=qp_solves, qp_iterations=qp_iters, h_change=change,
               h=ctl["h"], hf=ctl["hf"], Phi_x=ctl["Phi_x"], Phi_u=ctl["Phi_u"], l=lt, u=ut)
    if nom is not None:
        out.update(X=nom["X"], U=nom["U"], lam=nom["lam"], qp_status=nom["status"])
    return out
