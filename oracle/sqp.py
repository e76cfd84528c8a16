"""SQP on the paper's analytic models, in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Models (App. C, App. D), state x, input u, time step dt:
  Dubins car   x = (px, py, theta), u = omega, constant speed v:
               f(x, u) = (px + v cos(theta) dt, py + v sin(theta) dt, theta + omega dt)
  quadrotor    x = (px, py, phi, vx, vy, phidot), u = (u1, u2), mass m, gravity g,
               arm L, inertia J; continuous dynamics
               xdot = (vx, vy, phidot, -(u1+u2) sin(phi)/m, (u1+u2) cos(phi)/m - g, L (u2-u1)/J)
               discretised by one explicit Euler step, f(x, u) = x + dt xdot (a
               reading: the paper gives the continuous model; the Dubins car it
               prints is the same Euler step)
Constraints: per obstacle (cx, cy, r) the row g = r^2 - (px-cx)^2 - (py-cy)^2 <= 0
(eq. (obstacle_constraints)) at every stage and at the terminal state, and the
input box u_min <= u <= u_max.

SQP (Sec. III-B, eq. (sqp_qp)) around a nominal (X, U): the QP in (dx, du) with
  A_k = df/dx, B_k = df/du, b_k = f(x_k, u_k) - x_{k+1}   (defect of the nominal),
  dx_0 = xbar_0 - x_0,
  stage rows: obstacle gradients C_k dx_k <= -g(x_k); input box
              u_min - u_k <= du_k <= u_max - u_k;  terminal obstacle rows,
  cost: the tracking cost 1/2 (x - x_ref_k)' Q (x - x_ref_k) + 1/2 (u - u_ref_k)' R (u - u_ref_k)
        (terminal Q_N) with its gradient at the nominal as q, r and its Hessian
        as Q, R, S = 0.
Readings: the cost is not given for these models (quadratic tracking taken);
the Hessian is the cost's (Gauss-Newton): the exact Lagrangian Hessian adds
multiplier-weighted constraint and dynamics curvature, which for these concave
obstacle rows (Hessian -2I in position) makes the QP non-convex, whereas the
fixed point of the iteration (a zero step) is the nonlinear problem's KKT point
with either Hessian.  Step: x <- x + alpha dx, u <- u + alpha du; stop when
max |(dx, du)| <= tol_step or after max_iter iterations.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from paper_2604_07644_amd.workloads import QPProblem
from .native import qp_solve

DUBINS, QUADROTOR = 1, 2
INF = float("inf")


@dataclass
class Model:
    kind: int
    N: int
    dt: float
    Q: np.ndarray
    R: np.ndarray
    QN: np.ndarray
    x_ref: np.ndarray      # [N+1, nx] per-stage reference
    u_ref: np.ndarray      # [N, nu]
    u_min: np.ndarray
    u_max: np.ndarray
    obstacles: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    v: float = 1.0
    mass: float = 2.0576
    grav: float = 9.81
    arm: float = 0.25
    inertia: float = 0.01

    @property
    def nx(self):
        return 3 if self.kind == DUBINS else 6

    @property
    def nu(self):
        return 1 if self.kind == DUBINS else 2


def from_scenario(sc) -> Model:
    """Model from a scenario dict of paper_2604_07644_amd.workloads."""
    keys = ("kind", "N", "dt", "Q", "R", "QN", "x_ref", "u_ref", "u_min", "u_max", "obstacles", "v", "mass",
            "grav", "arm", "inertia")
    return Model(**{k: sc[k] for k in keys if k in sc})


def step(md: Model, x, u):
    x = np.asarray(x, dtype=np.float64); u = np.asarray(u, dtype=np.float64)
    if md.kind == DUBINS:
        return np.array([x[0] + md.v * np.cos(x[2]) * md.dt, x[1] + md.v * np.sin(x[2]) * md.dt,
                         x[2] + u[0] * md.dt])
    T = u[0] + u[1]
    xdot = np.array([x[3], x[4], x[5], -T * np.sin(x[2]) / md.mass, T * np.cos(x[2]) / md.mass - md.grav,
                     md.arm * (u[1] - u[0]) / md.inertia])
    return x + md.dt * xdot


def jacobians(md: Model, x, u):
    """(A, B) = (df/dx, df/du), differentiated by hand from step()."""
    dt = md.dt
    if md.kind == DUBINS:
        A = np.eye(3)
        A[0, 2] = -md.v * np.sin(x[2]) * dt
        A[1, 2] = md.v * np.cos(x[2]) * dt
        B = np.array([[0.0], [0.0], [dt]])
        return A, B
    T = u[0] + u[1]
    s, c = np.sin(x[2]), np.cos(x[2])
    A = np.eye(6)
    A[0, 3] = A[1, 4] = A[2, 5] = dt
    A[3, 2] = -dt * T * c / md.mass
    A[4, 2] = -dt * T * s / md.mass
    B = np.zeros((6, 2))
    B[3, :] = -dt * s / md.mass
    B[4, :] = dt * c / md.mass
    B[5, 0] = -dt * md.arm / md.inertia
    B[5, 1] = dt * md.arm / md.inertia
    return A, B


def obstacle_rows(md: Model, x):
    """(g, dg/dx) of the obstacle rows at state x."""
    ob = md.obstacles
    dx, dy = x[0] - ob[:, 0], x[1] - ob[:, 1]
    g = ob[:, 2] ** 2 - dx ** 2 - dy ** 2
    G = np.zeros((ob.shape[0], md.nx))
    G[:, 0] = -2.0 * dx
    G[:, 1] = -2.0 * dy
    return g, G


def linearize(md: Model, X, U, x0):
    """The QP of one SQP iteration around the nominal (X, U), as a QPProblem in (dx, du)."""
    N, nx, nu, no = md.N, md.nx, md.nu, md.obstacles.shape[0]
    nc, nf = no + nu, no
    A = np.empty((N, nx, nx)); B = np.empty((N, nx, nu)); b = np.empty((N, nx))
    C = np.zeros((N, nc, nx)); D = np.zeros((N, nc, nu))
    l = np.empty(N * nc + nf); u = np.empty(N * nc + nf)
    for k in range(N):
        A[k], B[k] = jacobians(md, X[k], U[k])
        b[k] = step(md, X[k], U[k]) - X[k + 1]
        g, Gx = obstacle_rows(md, X[k])
        C[k, :no] = Gx
        D[k, no:] = np.eye(nu)
        l[k * nc:k * nc + no] = -INF
        u[k * nc:k * nc + no] = -g
        l[k * nc + no:(k + 1) * nc] = md.u_min - U[k]
        u[k * nc + no:(k + 1) * nc] = md.u_max - U[k]
    g, CN = obstacle_rows(md, X[N])
    l[N * nc:] = -INF
    u[N * nc:] = -g
    Q = np.empty((N + 1, nx, nx)); Q[:N] = md.Q; Q[N] = md.QN
    R = np.broadcast_to(md.R, (N, nu, nu)).copy()
    q = np.empty((N + 1, nx))
    q[:N] = (X[:N] - md.x_ref[:N]) @ md.Q.T
    q[N] = md.QN @ (X[N] - md.x_ref[N])
    r = (U - md.u_ref) @ md.R.T
    return QPProblem(N, nx, nu, nc, nf, A, B, b, Q, R, np.zeros((N, nu, nx)), q, r, C, D, CN, l, u,
                     np.asarray(x0, dtype=np.float64) - X[0])


def sqp(md: Model, x0, X, U, max_iter=20, alpha=1.0, tol_qp=1e-8, tol_step=1e-6, rho=1.0):
    """SQP iterations from the nominal (X, U).  Returns the final nominal and
    the iteration record.  status: 1 step below tol_step, 2 iteration limit,
    5 a QP did not converge."""
    X = np.array(X, dtype=np.float64); U = np.array(U, dtype=np.float64)
    steps, qp_iters = [], 0
    status = 2
    for it in range(max_iter):
        qp = linearize(md, X, U, x0)
        sol = qp_solve(qp, rho=rho, tol=tol_qp)
        qp_iters += sol["iters"]
        if sol["status"] != 1:
            status = 5
            break
        dX, dU = sol["X"], sol["U"]
        X += alpha * dX
        U += alpha * dU
        st = float(max(np.max(np.abs(dX)), np.max(np.abs(dU))))
        steps.append(st)
        if st <= tol_step:
            status = 1
            break
    return dict(X=X, U=U, status=status, iterations=len(steps), steps=steps, qp_iterations=qp_iters)


def rollout(md: Model, x0, U):
    X = np.empty((md.N + 1, md.nx)); X[0] = x0
    for k in range(md.N):
        X[k + 1] = step(md, X[k], U[k])
    return X
