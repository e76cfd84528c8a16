"""Pins of the oracle's SQP on the analytic models (App. C, App. D; Sec. III-B).

* The hand-written Jacobians of the Dubins car and the Euler-discretised
  planar quadrotor match central finite differences of the dynamics, and the
  obstacle-row gradients those of the obstacle function.
* The SQP's fixed point is the nonlinear problem's KKT point: on small
  horizons with an active obstacle it matches the solution of the same
  nonlinear program by scipy's SLSQP (an independent sequential QP solver with
  its own line search and active set), and it satisfies the dynamics and the
  obstacle rows.
"""
import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import sqp as S
from paper_2604_07644_amd import workloads as W


def _models():
    return [S.from_scenario(W.dubins_scenario(N=20, n_obs=1, seed=3)),
            S.from_scenario(W.quadrotor_scenario(N=40, n_obs=1, seed=3))]


@pytest.mark.parametrize("idx", [0, 1])
def test_jacobians_match_finite_differences(idx):
    md = _models()[idx]
    rng = np.random.default_rng(5)
    for _ in range(5):
        x = rng.standard_normal(md.nx)
        u = rng.standard_normal(md.nu) + (0.0 if md.kind == S.DUBINS else 10.0)
        A, B = S.jacobians(md, x, u)
        h = 1e-6
        Af = np.stack([(S.step(md, x + h * e, u) - S.step(md, x - h * e, u)) / (2 * h) for e in np.eye(md.nx)], 1)
        Bf = np.stack([(S.step(md, x, u + h * e) - S.step(md, x, u - h * e)) / (2 * h) for e in np.eye(md.nu)], 1)
        np.testing.assert_allclose(A, Af, atol=1e-8)
        np.testing.assert_allclose(B, Bf, atol=1e-8)
        g, G = S.obstacle_rows(md, x)
        Gf = np.stack([(S.obstacle_rows(md, x + h * e)[0] - S.obstacle_rows(md, x - h * e)[0]) / (2 * h)
                       for e in np.eye(md.nx)], 1)
        np.testing.assert_allclose(G, Gf, atol=1e-7)


def _nlp(md, x0, X0, U0):
    """The nonlinear program of the SQP, solved by SLSQP over (X, U)."""
    N, nx, nu = md.N, md.nx, md.nu
    nX = (N + 1) * nx

    def unpack(z):
        return z[:nX].reshape(N + 1, nx), z[nX:].reshape(N, nu)

    def cost(z):
        X, U = unpack(z)
        ex = X[:N] - md.x_ref[:N]; eu = U - md.u_ref; eN = X[N] - md.x_ref[N]
        return 0.5 * (np.einsum("ki,ij,kj->", ex, md.Q, ex) + np.einsum("ki,ij,kj->", eu, md.R, eu)
                      + eN @ md.QN @ eN)

    def dyn(z):
        X, U = unpack(z)
        return np.concatenate([X[0] - x0] + [S.step(md, X[k], U[k]) - X[k + 1] for k in range(N)])

    def obs(z):
        X, _ = unpack(z)
        return -np.concatenate([S.obstacle_rows(md, X[k])[0] for k in range(N + 1)])

    bounds = [(None, None)] * nX + [(lo, hi) for _ in range(N) for lo, hi in zip(md.u_min, md.u_max)]
    res = minimize(cost, np.concatenate([X0.ravel(), U0.ravel()]), method="SLSQP", bounds=bounds,
                   constraints=[{"type": "eq", "fun": dyn}, {"type": "ineq", "fun": obs}],
                   options={"maxiter": 500, "ftol": 1e-12})
    assert res.success, res.message
    return unpack(res.x)


# (model, QP tolerance, step tolerance, bar against the NLP solution): the
# quadrotor's QPs are badly scaled for ADMM (rotor-arm gain L/J = 25) and are
# solved to 1e-4, which bounds how closely the fixed point is reached
CASES = [(0, 1e-6, 1e-5, 5e-4), (1, 1e-4, 1e-3, 3e-3)]


@pytest.mark.parametrize("idx,tol_qp,tol_step,bar", CASES)
def test_sqp_fixed_point_is_the_nlp_solution(idx, tol_qp, tol_step, bar):
    md = _models()[idx]
    sc = (W.dubins_scenario(N=20, n_obs=1, seed=3), W.quadrotor_scenario(N=40, n_obs=1, seed=3))[idx]
    out = S.sqp(md, sc["x0"], sc["X"], sc["U"], max_iter=40, alpha=1.0, tol_qp=tol_qp, tol_step=tol_step)
    assert out["status"] == 1, out["steps"]
    X, U = out["X"], out["U"]
    # feasibility of the nonlinear problem
    defect = max(np.max(np.abs(S.step(md, X[k], U[k]) - X[k + 1])) for k in range(md.N))
    assert defect <= tol_step and np.max(np.abs(X[0] - sc["x0"])) <= 1e-12
    g = np.concatenate([S.obstacle_rows(md, x)[0] for x in X])
    assert np.max(g) <= tol_step
    assert np.max(g) >= -1e-3          # an obstacle is active
    Xs, Us = _nlp(md, sc["x0"], sc["X"], sc["U"])
    np.testing.assert_allclose(X, Xs, atol=bar)
    np.testing.assert_allclose(U, Us, atol=bar * max(1.0, np.max(np.abs(Us)) / 10.0))
