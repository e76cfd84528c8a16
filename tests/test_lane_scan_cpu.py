"""CPU check of the algebra the one-wavefront path relies on (numpy, FP64, no
GPU): one ADMM iteration of the Riccati-form x-update written as two affine
recurrences over the horizon,

    p_k = c_k + Abar_k^T p_{k+1},  c_k = qhat_k + K_k^T rhat_k + Abar_k^T P_{k+1} b_k,
    x_{k+1} = Abar_k x_k + B_k kff_k + b_k,  kff_k = -H_k^{-1}(rhat_k + B_k^T (p_{k+1} + P_{k+1} b_k)),

each solved by a Kogge-Stone scan over stages whose level-d maps are products
of 2^d consecutive Abar^T (the forward scan reads the same maps transposed,
from the lane 2^d below).  Sec. IV-A (associative scans with cached factors),
eq. (controller_cache).  The iterates must equal the oracle's sequential
Riccati ADMM (fixed rho and with the rho rule) to rounding.
"""
import numpy as np
import pytest

import oracle
from paper_2604_07644_amd import workloads as W


def _factor(p, rho):
    N, nx, nu = p.N, p.nx, p.nu
    C, D, CN = p.C, p.D, np.asarray(p.CN).reshape(p.nf, nx)
    P = np.zeros((N + 1, nx, nx)); K = np.zeros((N, nu, nx)); Hinv = np.zeros((N, nu, nu))
    P[N] = p.Q[N] + rho * CN.T @ CN
    for k in range(N - 1, -1, -1):
        Qh = p.Q[k] + rho * C[k].T @ C[k]
        Rh = p.R[k] + rho * D[k].T @ D[k]
        Sh = p.S[k] + rho * D[k].T @ C[k]
        H = Rh + p.B[k].T @ P[k + 1] @ p.B[k]
        G = Sh + p.B[k].T @ P[k + 1] @ p.A[k]
        Hinv[k] = np.linalg.inv(H)
        K[k] = -Hinv[k] @ G
        Pk = Qh + p.A[k].T @ P[k + 1] @ p.A[k] + G.T @ K[k]
        P[k] = 0.5 * (Pk + Pk.T)
    Ab = p.A + np.einsum("kij,kjl->kil", p.B, K)
    pb = np.einsum("kij,kj->ki", P[1:], p.b)
    c0 = p.q[:N] + np.einsum("ktc,kt->kc", K, p.r) + np.einsum("kij,ki->kj", Ab, pb)
    # level-d maps: M[d][k] = Abar_k^T ... Abar_{k+2^d-1}^T where k + 2^d <= N, else 0
    nlev = 1
    while (1 << nlev) <= N:
        nlev += 1
    M = np.zeros((nlev, N + 1, nx, nx))
    M[0, :N] = np.transpose(Ab, (0, 2, 1))
    for d in range(1, nlev):
        o = 1 << d
        for k in range(N + 1):
            if k + o <= N:
                M[d, k] = M[d - 1, k] @ M[d - 1, k + o // 2]
    return dict(K=K, Hinv=Hinv, pb=pb, c0=c0, M=M, nlev=nlev)


def _iterate(p, f, rho, z, y, fwd_spec="kji,kj->ki"):
    N, nx, nc = p.N, p.nx, p.nc
    CN = np.asarray(p.CN).reshape(p.nf, nx)
    w = y - z
    ws, wN = w[:N * nc].reshape(N, nc), w[N * nc:]
    tx = np.einsum("kri,kr->ki", p.C, ws); tu = np.einsum("kri,kr->ki", p.D, ws)
    c = np.zeros((N + 1, nx))
    c[:N] = f["c0"] + rho * (tx + np.einsum("ktj,kt->kj", f["K"], tu))
    c[N] = p.q[N] + rho * CN.T @ wN
    rh = p.r + rho * tu
    for d in range(f["nlev"]):                      # suffix scan, partner k + 2^d
        o = 1 << d
        c = c + np.concatenate([np.einsum("kij,kj->ki", f["M"][d, :N + 1 - o], c[o:]), np.zeros((o, nx))])
    s = c[1:] + f["pb"]
    kff = -np.einsum("kij,kj->ki", f["Hinv"], rh + np.einsum("kji,kj->ki", p.B, s))
    x = np.zeros((N + 1, nx)); x[0] = p.x0
    x[1:] = np.einsum("kij,kj->ki", p.B, kff) + p.b
    for d in range(f["nlev"]):                      # prefix scan, partner k - 2^d, maps transposed
        o = 1 << d
        add = np.zeros_like(x)
        add[o:] = np.einsum(fwd_spec, f["M"][d, :N + 1 - o], x[:N + 1 - o])
        x = x + add
    u = np.einsum("kij,kj->ki", f["K"], x[:N]) + kff
    v = np.concatenate([(np.einsum("kij,kj->ki", p.C, x[:N]) + np.einsum("kij,kj->ki", p.D, u)).ravel(), CN @ x[N]])
    zn = np.clip(v + y, p.l, p.u)
    yn = y + v - zn
    return x, u, zn, yn


@pytest.mark.parametrize("maker", [lambda: W.box_lq(), lambda: W.random_small(23, 4, 3, 5, 2, seed=1),
                                   lambda: W.random_small(1, 3, 1, 2, 1, seed=4),
                                   lambda: W.random_small(40, 5, 2, 4, 3, seed=3)])
def test_lane_scans_equal_sequential_riccati(maker):
    p = maker()
    iters, rho = 40, 1.0
    f = _factor(p, rho)
    z = np.zeros(p.m); y = np.zeros(p.m)
    for _ in range(iters):
        x, u, z, y = _iterate(p, f, rho, z, y)
    o = oracle.qp_solve(p, rho=rho, tol=0.0, settings=oracle.Settings(max_iter=iters, adaptive=False))
    scale = max(1.0, float(np.abs(o["X"]).max()))
    assert np.abs(x - o["X"]).max() <= 1e-11 * scale
    assert np.abs(u - o["U"]).max() <= 1e-11 * max(1.0, float(np.abs(o["U"]).max()))
    assert np.abs(z - o["z"]).max() <= 1e-11 * max(1.0, float(np.abs(o["z"]).max()))


def test_planted_untransposed_forward_maps_are_caught():
    """The forward scan must read the backward maps transposed: reading them
    as stored (a plausible slip) gives a different trajectory from the oracle's."""
    p = W.random_small(23, 4, 3, 5, 2, seed=1)
    f = _factor(p, 1.0)
    z = np.zeros(p.m); y = np.zeros(p.m)
    x_bad, *_ = _iterate(p, f, 1.0, z, y, fwd_spec="kij,kj->ki")
    o = oracle.qp_solve(p, rho=1.0, tol=0.0, settings=oracle.Settings(max_iter=1, adaptive=False))
    assert np.abs(x_bad - o["X"]).max() > 1e-3
