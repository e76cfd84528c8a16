"""Pins of the oracle's FastSLS alternation (Sec. III-D, App. B).

The alternation composes pinned pieces (ADMM, per-column SLS Riccati, App. B
tau); what is new is the tightening and the loop.  They are checked against
facts that hold independently of the oracle's code:
  * with no disturbance the margins vanish and the result is the plain QP's;
  * the margin of a row is the support function of the reachable set: the
    vertex disturbance w_j = wbound sign(row Phi_{k,j}) moves the row by
    exactly +h (and -w by -h), computed here from the responses directly;
  * the returned nominal trajectory is robustly feasible: nominal row value
    plus / minus its margin stays inside the untightened bounds (up to the ADMM
    tolerance), for one-sided, two-sided and terminal rows;
  * margins larger than a two-sided row's half-width are reported as an
    infeasible tightening.
"""
import numpy as np

import oracle
from oracle import robust as R
from oracle.native import sls_layout
from paper_2604_07644_amd import workloads as W

TOL = 1e-8


def _weights(p):
    return np.eye(p.nx), np.eye(p.nu), np.eye(p.nx)


def _two_sided_case():
    p = W.random_small(10, 4, 2, 3, 2, seed=11)
    E = 0.05 * np.stack([np.eye(p.nx)] * p.N)
    return p, E


def test_no_disturbance_reduces_to_the_nominal_qp():
    p, E, wb = W.robust_case(instance_id=1)
    out = R.robust_alternation(p, np.zeros_like(E), *_weights(p), rownorm=1, wbound=wb, tol=TOL)
    assert out["status"] == R.CONVERGED and out["passes"] == 1 and out["qp_solves"] == 2
    assert np.all(out["h"] == 0.0)
    ref = oracle.qp_solve(p, rho=1.0, tol=TOL)
    np.testing.assert_array_equal(out["X"], ref["X"])
    np.testing.assert_array_equal(out["U"], ref["U"])


def _check_support_and_feasibility(p, out, wb):
    N, nc, nf = p.N, p.nc, p.nf
    offx, offu = sls_layout(N)
    Px, Pu, X, U = out["Phi_x"], out["Phi_u"], out["X"], out["U"]
    assert np.all(out["h"][0] == 0.0)
    for k in range(1, N + 1):
        rows = range(nf) if k == N else range(nc)
        for r in rows:
            dev = 0.0
            for j in range(k):
                if k == N:
                    a = p.CN[r] @ Px[offx[j] + (k - j - 1)]
                else:
                    a = p.C[k][r] @ Px[offx[j] + (k - j - 1)] + p.D[k][r] @ Pu[offu[j] + (k - j - 1)]
                dev += a @ (wb * np.sign(a))
            h = out["hf"][r] if k == N else out["h"][k, r]
            assert abs(dev - h) <= 1e-9 * max(1.0, abs(dev)), (k, r, dev, h)
            i = N * nc + r if k == N else k * nc + r
            g = p.CN[r] @ X[N] if k == N else p.C[k][r] @ X[k] + p.D[k][r] @ U[k]
            if np.isfinite(p.u[i]):
                assert g + dev <= p.u[i] + 10 * TOL, (k, r, g + dev, p.u[i])
            if np.isfinite(p.l[i]):
                assert g - dev >= p.l[i] - 10 * TOL, (k, r, g - dev, p.l[i])


def test_margins_are_attained_and_the_nominal_is_robustly_feasible():
    p, E, wb = W.robust_case(instance_id=2)
    out = R.robust_alternation(p, E, *_weights(p), rownorm=1, wbound=wb, tol=TOL, max_passes=20)
    assert out["status"] == R.CONVERGED, out["status"]
    assert np.max(out["h"]) > 1e-3            # the disturbance matters
    _check_support_and_feasibility(p, out, wb)
    # the final nominal solve used exactly the returned margins
    lt, ut = R.tighten(p.l, p.u, R.margin_rows(out["h"], out["hf"]))
    np.testing.assert_array_equal(out["u"], ut)


def test_two_sided_and_terminal_rows():
    p, E = _two_sided_case()
    out = R.robust_alternation(p, E, *_weights(p), rownorm=1, wbound=0.1, tol=TOL, max_passes=20)
    assert out["status"] == R.CONVERGED, out["status"]
    assert np.max(out["hf"]) > 0.0
    _check_support_and_feasibility(p, out, 0.1)


def test_tightening_beyond_the_row_width_is_reported():
    p, E = _two_sided_case()
    out = R.robust_alternation(p, E, *_weights(p), rownorm=1, wbound=50.0, tol=TOL)
    assert out["status"] == R.TIGHTENING_INFEASIBLE
    assert out["qp_solves"] == 0
