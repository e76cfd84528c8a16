"""Seeded synthetic stage-structured LTV-QP and SLS workloads.

These generators stand in for the paper's robot workloads (the MuJoCo quadruped
and humanoid models of Sec. V-C / App. E are not available): they produce
problems of the same shapes (state dimension, control dimension, horizon,
constraint rows per stage) and the scale stated in the abstract (about 2e5
decision variables and 8e4 constraints).  The problem data follow the LTV-QP
of Sec. III-B, eq. (sqp_qp): dynamics x_{k+1} = A_k x_k + B_k u_k + b_k, stage
costs (Q_k, S_k, R_k, q_k, r_k), terminal cost (Q_N, q_N), and two-sided
constraint rows  l <= C_k x_k + D_k u_k <= u  (one-sided rows use l = -inf,
which is the paper's  z <= f  form), terminal rows  l <= C_N x_N <= u.

This module holds input generation only: random draws, the zero-input
roll-out used to make the drawn polytopes feasible, and packing.  It contains
none of the solver's arithmetic and is shared by the tests, the benchmark and
the smoke check.

Random draws use ``numpy.random.default_rng([cfg_id, instance_id])``.  In
``N(0, v)`` the second argument is a variance.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

INF = float("inf")


@dataclass
class QPProblem:
    """One stage-structured LTV-QP, all arrays float64, row-major."""
    N: int
    nx: int
    nu: int
    nc: int
    nf: int
    A: np.ndarray   # [N, nx, nx]
    B: np.ndarray   # [N, nx, nu]
    b: np.ndarray   # [N, nx]
    Q: np.ndarray   # [N+1, nx, nx]
    R: np.ndarray   # [N, nu, nu]
    S: np.ndarray   # [N, nu, nx]
    q: np.ndarray   # [N+1, nx]
    r: np.ndarray   # [N, nu]
    C: np.ndarray   # [N, nc, nx]
    D: np.ndarray   # [N, nc, nu]
    CN: np.ndarray  # [nf, nx]
    l: np.ndarray   # [N*nc + nf]
    u: np.ndarray   # [N*nc + nf]
    x0: np.ndarray  # [nx]
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return self.N * self.nc + self.nf

    def copy(self) -> "QPProblem":
        kw = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in self.__dict__.items()}
        kw["meta"] = dict(self.meta)
        return QPProblem(**kw)


def _rng(cfg_id: int, instance_id: int) -> np.random.Generator:
    return np.random.default_rng([int(cfg_id), int(instance_id)])


def _normal(rng, var, shape):
    return rng.standard_normal(shape) * np.sqrt(var)


def _spectral_clip(A: np.ndarray, rmax: float) -> np.ndarray:
    rad = np.max(np.abs(np.linalg.eigvals(A)))
    return A * (rmax / rad) if rad > rmax else A


def _box_rows(nx: int, nu: int):
    C = np.zeros((nx + nu, nx))
    D = np.zeros((nx + nu, nu))
    C[:nx, :nx] = np.eye(nx)
    D[nx:, :] = np.eye(nu)
    return C, D


def _draw_x0(rng, nx, var, xmax=None):
    while True:
        x0 = _normal(rng, var, nx)
        if xmax is None or np.max(np.abs(x0)) <= xmax:
            return x0


def box_lq(N=32, nx=4, nu=2, cfg_id=0, instance_id=0, xmax=5.0, umax=1.0,
           a_scale=0.05, b_var=0.1, terminal_box=True) -> QPProblem:
    """Box-constrained LQ QP (the plain-ADMM workload: nx=4, nu=2, N=32).

    A_t = I + a_scale*G_t, G_t ~ N(0, 1/nx); B_t ~ N(0, b_var); Q_t = diag U[1,10];
    R_t = diag U[0.1,1]; q = r = 0; S = 0; b = 0; |x| <= xmax, |u| <= umax per
    stage and |x_N| <= xmax at the terminal stage; x0 ~ N(0,1), redrawn until
    |x0|_inf <= xmax.  Per stage the draw order is A, B, Q, R; then Q_N, x0.
    """
    rng = _rng(cfg_id, instance_id)
    A = np.empty((N, nx, nx)); B = np.empty((N, nx, nu))
    Q = np.zeros((N + 1, nx, nx)); R = np.zeros((N, nu, nu))
    for t in range(N):
        A[t] = np.eye(nx) + a_scale * _normal(rng, 1.0 / nx, (nx, nx))
        B[t] = _normal(rng, b_var, (nx, nu))
        Q[t] = np.diag(rng.uniform(1.0, 10.0, nx))
        R[t] = np.diag(rng.uniform(0.1, 1.0, nu))
    Q[N] = np.diag(rng.uniform(1.0, 10.0, nx))
    x0 = _draw_x0(rng, nx, 1.0, xmax)
    Cb, Db = _box_rows(nx, nu)
    nc = nx + nu
    C = np.broadcast_to(Cb, (N, nc, nx)).copy()
    D = np.broadcast_to(Db, (N, nc, nu)).copy()
    lo = np.concatenate([-xmax * np.ones(nx), -umax * np.ones(nu)])
    hi = -lo
    nf = nx if terminal_box else 0
    CN = np.eye(nx) if terminal_box else np.zeros((0, nx))
    l = np.concatenate([np.tile(lo, N), -xmax * np.ones(nf)])
    u = np.concatenate([np.tile(hi, N), xmax * np.ones(nf)])
    return QPProblem(N, nx, nu, nc, nf, A, B, np.zeros((N, nx)), Q, R,
                     np.zeros((N, nu, nx)), np.zeros((N + 1, nx)), np.zeros((N, nu)),
                     C, D, CN, l, u, x0,
                     meta=dict(kind="box_lq", cfg_id=cfg_id, instance_id=instance_id,
                               xmax=xmax, umax=umax))


def polytopic_lq(N, nx, nu, nc=40, cfg_id=1, instance_id=0, a_scale=0.02,
                 a_var=None, b_var=0.05, x0_var=0.25, rho_max=1.05, ref_var=1.0,
                 shared_dynamics_seed=None) -> QPProblem:
    """Time-varying LQ QP with random polytopic stage constraints.

    A_t = I + a_scale*M_t, M_t ~ N(0, 1/nx), rescaled so its spectral radius is
    at most rho_max; B_t ~ N(0, b_var); Q_t = diag U[1,10]; R_t = diag U[0.1,1].
    Per stage, nc rows [C_t D_t] drawn N(0,1) and normalised to unit 2-norm;
    upper bounds d_t = s_t + (C_t xbar_t)^+ with s_t ~ U[0.5, 2] and xbar the
    zero-input roll-out from x0 (so u = 0 is strictly feasible); l = -inf.
    No terminal rows.  x0 ~ N(0, x0_var).

    Linear costs come from a constant tracking reference x_ref ~ N(0, ref_var):
    q_t = -Q_t x_ref (t = 0..N), r_t = 0, i.e. the stage cost is
    1/2 (x - x_ref)^T Q (x - x_ref) up to a constant.  An SQP linearisation
    produces such non-zero gradients; without them the optimum stays near the
    origin and no drawn row is ever active.  x_ref is drawn after x0 (from the
    shared seed when ``shared_dynamics_seed`` is given).

    With ``shared_dynamics_seed`` the stage data are drawn from that seed and
    only x0 from (cfg_id, instance_id): a batch of instances that differ only
    in their initial state.
    """
    a_var = 1.0 / nx if a_var is None else a_var
    rng = _rng(cfg_id, instance_id if shared_dynamics_seed is None else shared_dynamics_seed)
    A = np.empty((N, nx, nx)); B = np.empty((N, nx, nu))
    Q = np.zeros((N + 1, nx, nx)); R = np.zeros((N, nu, nu))
    C = np.empty((N, nc, nx)); D = np.empty((N, nc, nu)); s = np.empty((N, nc))
    for t in range(N):
        A[t] = _spectral_clip(np.eye(nx) + a_scale * _normal(rng, a_var, (nx, nx)), rho_max)
        B[t] = _normal(rng, b_var, (nx, nu))
        Q[t] = np.diag(rng.uniform(1.0, 10.0, nx))
        R[t] = np.diag(rng.uniform(0.1, 1.0, nu))
        G = rng.standard_normal((nc, nx + nu))
        G /= np.linalg.norm(G, axis=1, keepdims=True)
        C[t] = G[:, :nx]; D[t] = G[:, nx:]
        s[t] = rng.uniform(0.5, 2.0, nc)
    Q[N] = np.diag(rng.uniform(1.0, 10.0, nx))
    xref = _normal(rng, ref_var, nx) if shared_dynamics_seed is not None else None
    if shared_dynamics_seed is not None:
        rng = _rng(cfg_id, instance_id)
    x0 = _normal(rng, x0_var, nx)
    if xref is None:
        xref = _normal(rng, ref_var, nx)
    q = -np.einsum("tij,j->ti", Q, xref)
    xbar = x0.copy(); d = np.empty((N, nc))
    with np.errstate(over="ignore", invalid="ignore"):
        for t in range(N):
            d[t] = s[t] + np.maximum(C[t] @ xbar, 0.0)
            xbar = A[t] @ xbar
    d[~np.isfinite(d)] = INF
    l = -INF * np.ones(N * nc); u = d.reshape(-1).copy()
    return QPProblem(N, nx, nu, nc, 0, A, B, np.zeros((N, nx)), Q, R,
                     np.zeros((N, nu, nx)), q, np.zeros((N, nu)),
                     C, D, np.zeros((0, nx)), l, u, x0,
                     meta=dict(kind="polytopic_lq", cfg_id=cfg_id, instance_id=instance_id,
                               xref=xref))


def quadruped_qp(instance_id=0) -> QPProblem:
    """Quadruped-shaped QP: nx=61, nu=12, N=128, 40 polytopic rows per stage."""
    return polytopic_lq(128, 61, 12, 40, cfg_id=1, instance_id=instance_id,
                        a_scale=0.02, b_var=0.05, x0_var=0.25, rho_max=1.05)


def humanoid_qp(instance_id=0, N=2048) -> QPProblem:
    """Humanoid-shaped QP at the paper's scale: nx=75, nu=19, N=2048, 40 rows
    per stage (192,587 variables, 81,920 rows).  Dynamics, costs and x0 as in
    the box workload (A = I + 0.05 G, B ~ N(0, 0.1), x0 ~ N(0, 1))."""
    return polytopic_lq(N, 75, 19, 40, cfg_id=2, instance_id=instance_id,
                        a_scale=0.05, b_var=0.1, x0_var=1.0, rho_max=1.05)


def sls_batch(count=64, N=64, nx=61, nu=12, nc=40, e_var=0.01, cfg_id=3):
    """SLS workload: one quadruped-shaped polytopic QP (shared stage data) and
    ``count`` initial states, plus disturbance maps E_t ~ N(0, e_var) and the
    disturbance bound |w|_inf <= 0.01."""
    probs = [polytopic_lq(N, nx, nu, nc, cfg_id=cfg_id, instance_id=i, a_scale=0.02,
                          b_var=0.05, x0_var=0.25, rho_max=1.05,
                          shared_dynamics_seed=10 ** 9) for i in range(count)]
    rng = _rng(cfg_id, 10 ** 9 + 1)
    E = _normal(rng, e_var, (N, nx, nx))
    return probs, E, 0.01


def robust_case(N=16, nx=6, nu=2, nc=8, cfg_id=6, instance_id=0, e_var=0.01, wbound=0.05):
    """Robust MPC case: a polytopic QP as in polytopic_lq (one-sided rows,
    no terminal rows) with disturbance maps E_t ~ N(0, e_var) and the bound
    |w|_inf <= wbound."""
    p = polytopic_lq(N, nx, nu, nc, cfg_id=cfg_id, instance_id=instance_id)
    rng = _rng(cfg_id, 10 ** 9 + 2 + instance_id)
    E = _normal(rng, e_var, (N, nx, nx))
    return p, E, wbound


def pendulum_like(N=3000, links=15, kappa=1.0, cfg_id=7, instance_id=0, dt=0.02, umax=2.0):
    """Torque-limited n-link-pendulum-shaped LTV-QP at the paper's long-horizon
    scale (its pendulum model is not given): nx = 2n (angles and rates),
    nu = n (joint torques).  A_t = [[I, dt I], [dt K_t, I]] with K_t = (G_t +
    G_t^T)/2, G_t ~ N(0, 1/n) (the linearisation about the upright position:
    an indefinite stiffness), B_t = [[0], [dt M^-1]] with the shared mass
    matrix M = L L^T + I, L ~ N(0, 1/n); torque rows -umax <= u <= umax
    (C = 0, D = I, nc = n), no terminal rows; Q_t = diag of nx values
    log-spaced from 1 to kappa (kappa: the cost's condition number), Q_N = Q,
    R_t = 0.1 I, q = r = 0; x0 ~ N(0, 0.25).  N = 3000, n = 15 gives 135,000
    decision variables."""
    nx, nu = 2 * links, links
    rng = _rng(cfg_id, instance_id)
    L = _normal(rng, 1.0 / links, (links, links))
    Minv = np.linalg.inv(L @ L.T + np.eye(links))
    A = np.empty((N, nx, nx)); B = np.zeros((N, nx, nu))
    for t in range(N):
        G = _normal(rng, 1.0 / links, (links, links))
        K = 0.5 * (G + G.T)
        A[t] = np.block([[np.eye(links), dt * np.eye(links)], [dt * K, np.eye(links)]])
        B[t, links:, :] = dt * Minv
    qd = np.logspace(0.0, np.log10(kappa), nx) if kappa > 1.0 else np.ones(nx)
    Q = np.broadcast_to(np.diag(qd), (N + 1, nx, nx)).copy()
    R = np.broadcast_to(0.1 * np.eye(nu), (N, nu, nu)).copy()
    x0 = _normal(rng, 0.25, nx)
    C = np.zeros((N, nu, nx)); D = np.broadcast_to(np.eye(nu), (N, nu, nu)).copy()
    l = -umax * np.ones(N * nu); u = umax * np.ones(N * nu)
    return QPProblem(N, nx, nu, nu, 0, A, B, np.zeros((N, nx)), Q, R, np.zeros((N, nu, nx)),
                     np.zeros((N + 1, nx)), np.zeros((N, nu)), C, D, np.zeros((0, nx)), l, u, x0,
                     meta=dict(kind="pendulum_like", cfg_id=cfg_id, instance_id=instance_id, kappa=kappa))


def dubins_scenario(N=60, n_obs=3, seed=0, dt=0.1, v=1.0):
    """Dubins car (App. C): speed v, time step dt, a straight reference along
    +x at the car's speed, x_ref_k = (k dt v, 0, 0), u_ref = 0; n_obs circular
    obstacles with centres x ~ U[0.25, 0.75] of the path length, radii
    r ~ U[0.25, 0.4] and y = r - U[0.05, 0.15] (all on the left), so the
    reference (and the straight initial guess) cuts 5-15 cm into each;
    |omega| <= 1.5; Q = diag(1, 1, 0.1), Q_N = 10 Q,
    R = 0.1; disturbance scaling E = 0.025 I (App. C).  Returns a dict of model
    parameters, the initial state and an initial nominal (X, U)."""
    rng = _rng(8, seed)
    Lp = N * dt * v
    cx = np.sort(rng.uniform(0.25 * Lp, 0.75 * Lp, n_obs))
    r = rng.uniform(0.25, 0.4, n_obs)
    cy = r - rng.uniform(0.05, 0.15, n_obs)
    x_ref = np.zeros((N + 1, 3)); x_ref[:, 0] = dt * v * np.arange(N + 1)
    Q = np.diag([1.0, 1.0, 0.1])
    return dict(kind=1, N=N, dt=dt, v=v, Q=Q, R=0.1 * np.eye(1), QN=10.0 * Q, x_ref=x_ref,
                u_ref=np.zeros((N, 1)), u_min=np.array([-1.5]), u_max=np.array([1.5]),
                obstacles=np.stack([cx, cy, r], axis=1), x0=np.zeros(3), X=x_ref.copy(),
                U=np.zeros((N, 1)), E=0.025 * np.eye(3))


def quadrotor_scenario(N=50, n_obs=2, seed=0, dt=0.05):
    """Planar quadrotor (App. D: m = 2.0576, g = 9.81, L = 0.25, J = 0.01):
    a flight from rest at the origin to (2, 0) along a straight reference at
    constant speed, hover thrust as the input reference, rotor thrusts in
    [0, 3 m g / 2]; n_obs obstacles with centres x ~ U[0.6, 1.4], radii
    r ~ U[0.15, 0.25] and |y| = r - U[0.03, 0.08] on alternating sides (the
    reference cuts into each); Q = diag(5, 5, 1, 0.5, 0.5, 0.1), Q_N = 10 Q,
    R = 0.1 I; disturbance
    scaling E = 0.05 diag(0, 0, 0, 1, 1, 0) (App. D).  Returns a dict as
    dubins_scenario does; the initial nominal is the reference path with
    hover thrust."""
    rng = _rng(9, seed)
    m, g = 2.0576, 9.81
    hover = m * g / 2.0
    cx = np.sort(rng.uniform(0.6, 1.4, n_obs))
    r = rng.uniform(0.15, 0.25, n_obs)
    cy = (r - rng.uniform(0.03, 0.08, n_obs)) * np.where(np.arange(n_obs) % 2 == 0, 1.0, -1.0)
    x_ref = np.zeros((N + 1, 6)); x_ref[:, 0] = np.linspace(0.0, 2.0, N + 1)
    x_ref[:, 3] = 2.0 / (N * dt)
    Q = np.diag([5.0, 5.0, 1.0, 0.5, 0.5, 0.1])
    return dict(kind=2, N=N, dt=dt, Q=Q, R=0.1 * np.eye(2), QN=10.0 * Q, x_ref=x_ref,
                u_ref=np.full((N, 2), hover), u_min=np.zeros(2), u_max=np.full(2, 3.0 * hover),
                obstacles=np.stack([cx, cy, r], axis=1), x0=np.zeros(6), X=x_ref.copy(),
                U=np.full((N, 2), hover), E=0.05 * np.diag([0.0, 0.0, 0.0, 1.0, 1.0, 0.0]),
                mass=m, grav=g, arm=0.25, inertia=0.01)


NX_CLASSES = (12, 36, 61, 75)
NU_CLASSES = (4, 12, 19)


def uneven_batch(count=512, cfg_id=4, first_instance=0, nmin=16, nmax=512):
    """Batch of box-constrained QPs of uneven shape: nx in {12,36,61,75},
    nu in {4,12,19} drawn independently and uniformly, N ~ U{nmin..nmax};
    per-instance bound scales xmax ~ U[3,7], umax ~ U[0.5,1.5]; stage data as
    in the box workload."""
    out = []
    for i in range(first_instance, first_instance + count):
        rng = _rng(cfg_id, i)
        nx = int(rng.choice(NX_CLASSES)); nu = int(rng.choice(NU_CLASSES))
        N = int(rng.integers(nmin, nmax + 1))
        xmax = float(rng.uniform(3.0, 7.0)); umax = float(rng.uniform(0.5, 1.5))
        p = box_lq(N=N, nx=nx, nu=nu, cfg_id=cfg_id, instance_id=10 ** 7 + i,
                   xmax=xmax, umax=umax, terminal_box=True)
        p.meta.update(dict(kind="uneven", batch_index=i))
        out.append(p)
    return out


def random_small(N, nx, nu, nc, nf, seed, general=True, b_nonzero=True, s_nonzero=True,
                 q_nonzero=True, lower=True):
    """Small random strictly convex LTV-QP with every term present (S, b, q, r,
    two-sided rows, terminal rows) for parity tests of the general path."""
    rng = np.random.default_rng([99, seed])
    A = np.eye(nx) + 0.3 * rng.standard_normal((N, nx, nx)) / np.sqrt(nx)
    B = rng.standard_normal((N, nx, nu)) * 0.5
    b = rng.standard_normal((N, nx)) * 0.1 if b_nonzero else np.zeros((N, nx))
    Q = np.empty((N + 1, nx, nx)); R = np.empty((N, nu, nu)); S = np.zeros((N, nu, nx))
    for t in range(N + 1):
        M = rng.standard_normal((nx, nx)); Q[t] = M @ M.T / nx + 0.5 * np.eye(nx)
    for t in range(N):
        M = rng.standard_normal((nu, nu)); R[t] = M @ M.T / nu + 0.5 * np.eye(nu)
        if s_nonzero:
            # keep [[Q S^T],[S R]] positive definite: S small relative to Q, R
            S[t] = 0.1 * rng.standard_normal((nu, nx))
    q = rng.standard_normal((N + 1, nx)) * (0.5 if q_nonzero else 0.0)
    r = rng.standard_normal((N, nu)) * (0.5 if q_nonzero else 0.0)
    C = rng.standard_normal((N, nc, nx)); D = rng.standard_normal((N, nc, nu))
    CN = rng.standard_normal((nf, nx))
    m = N * nc + nf
    x0 = rng.standard_normal(nx) * 0.3
    # bounds around the row values of a random roll-out, so the QP is feasible
    ub = rng.standard_normal((N, nu)) * 0.3
    xb = x0.copy(); vb = np.empty(m)
    for t in range(N):
        vb[t * nc:(t + 1) * nc] = C[t] @ xb + D[t] @ ub[t]
        xb = A[t] @ xb + B[t] @ ub[t] + b[t]
    vb[N * nc:] = CN @ xb
    hi = vb + rng.uniform(0.05, 0.6, m)
    lo = vb - rng.uniform(0.05, 0.6, m) if lower else -INF * np.ones(m)
    if lower:
        # a few one-sided and a few unbounded rows
        k = rng.random(m)
        lo[k < 0.2] = -INF
        hi[(k > 0.9)] = INF
    return QPProblem(N, nx, nu, nc, nf, A, B, b, Q, R, S, q, r, C, D, CN, lo, hi, x0,
                     meta=dict(kind="random_small", seed=seed))


# ------------------------------------------------------ learned warm start
WS_SIZES = (160, 512, 512, 512, 192)


def ws_sketch(seed=7):
    """Fixed random projection (64 x 94, entries N(0, 1/94)) of the 94-slot
    linearisation vector of a stage onto the 64-d sketch."""
    rng = np.random.default_rng([5, seed])
    return rng.standard_normal((64, 94)) / np.sqrt(94.0)


def ws_init(seed=0, sizes=WS_SIZES):
    """Initial MLP parameters as one flat float64 vector (W1, b1, W2, b2, ...;
    W row-major d_in x d_out): weights U[-sqrt(6/d_in), sqrt(6/d_in)] (He
    uniform, for ReLU layers), biases 0."""
    rng = np.random.default_rng([6, seed])
    parts = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        lim = np.sqrt(6.0 / a)
        parts.append(rng.uniform(-lim, lim, a * b))
        parts.append(np.zeros(b))
    return np.concatenate(parts)
