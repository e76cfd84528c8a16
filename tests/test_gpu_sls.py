"""GPU parity of the SLS controller synthesis (gsls_sls_solve / _batch /
gsls_sls_tau) against the FP64 per-column Riccati oracle.

The GPU path runs FP32 matrix-core products with the nu x nu inverse in FP64;
responses and margins are compared relative to their largest magnitude.
"""
import numpy as np
import pytest

import oracle
from paper_2604_07644_amd import workloads as W

pytestmark = pytest.mark.gpu

from paper_2604_07644_amd import gsls  # noqa: E402  (fails loudly without libgsls.so)


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-30))


def _small(N=7, nx=3, nu=2, nc=4, nf=2, seed=0):
    p = W.random_small(N, nx, nu, nc, nf, seed=seed)
    rng = np.random.default_rng([17, seed])
    E = rng.standard_normal((N, nx, nx)) * 0.3
    tau = np.abs(rng.standard_normal(N * N * nc + N * nf)) * 2.0
    return p, E, tau


@pytest.mark.parametrize("rownorm", [2, 1])
@pytest.mark.parametrize("shape", [(7, 3, 2, 4, 2), (12, 9, 4, 6, 0), (5, 17, 3, 20, 5)])
def test_sls_small_matches_oracle(shape, rownorm):
    p, E, tau = _small(*shape, seed=sum(shape))
    Qb, Rb, QbN = np.eye(p.nx), 0.5 * np.eye(p.nu), 2.0 * np.eye(p.nx)
    q = gsls.QP(p)
    g = q.sls_solve(E, tau, Qb, Rb, QbN, rownorm=rownorm, wbound=0.3)
    q.close()
    o = oracle.sls_solve(p, E, tau, Qb, Rb, QbN, rownorm=rownorm, wbound=0.3)
    assert _rel(g["Phi_x"], o["Phi_x"]) < 1e-4
    assert _rel(g["Phi_u"], o["Phi_u"]) < 1e-4
    assert _rel(g["h"], o["h"]) < 1e-4
    if p.nf:
        assert _rel(g["hf"], o["hf"]) < 1e-4


def test_sls_quadruped_shape_single():
    """nx=61, nu=12, N=64, 40 rows per stage: the SLS workload shape."""
    probs, E, wb = W.sls_batch(1)
    p = probs[0]
    rng = np.random.default_rng(3)
    tau = np.abs(rng.standard_normal(p.N * p.N * p.nc)) * 0.5
    Qb, Rb, QbN = np.eye(p.nx), np.eye(p.nu), np.eye(p.nx)
    q = gsls.QP(p)
    g = q.sls_solve(E, tau, Qb, Rb, QbN, rownorm=1, wbound=wb)
    q.close()
    o = oracle.sls_solve(p, E, tau, Qb, Rb, QbN, rownorm=1, wbound=wb)
    assert _rel(g["h"], o["h"]) < 1e-3, _rel(g["h"], o["h"])
    assert _rel(g["Phi_x"], o["Phi_x"]) < 1e-3


def test_sls_batch_each_instance_matches():
    p, E, _ = _small(9, 5, 2, 6, 3, seed=11)
    rng = np.random.default_rng(12)
    taus = [np.abs(rng.standard_normal(p.N * p.N * p.nc + p.N * p.nf)) * s for s in (0.0, 0.5, 3.0, 10.0)]
    Qb, Rb, QbN = np.eye(p.nx), np.eye(p.nu), np.eye(p.nx)
    q = gsls.QP(p)
    r = q.sls_solve_batch(E, taus, Qb, Rb, QbN, rownorm=2, wbound=1.0)
    q.close()
    assert r["ms"] > 0
    for i, t in enumerate(taus):
        o = oracle.sls_solve(p, E, t, Qb, Rb, QbN, rownorm=2, wbound=1.0)
        assert _rel(r["h"][i], o["h"]) < 1e-4
        assert _rel(r["hf"][i], o["hf"]) < 1e-4


def test_sls_tau_matches_oracle():
    p, E, tau0 = _small(8, 4, 2, 5, 3, seed=21)
    Qb, Rb, QbN = np.eye(p.nx), np.eye(p.nu), np.eye(p.nx)
    o = oracle.sls_solve(p, E, tau0, Qb, Rb, QbN)
    lam = np.random.default_rng(5).standard_normal(p.m)
    q = gsls.QP(p)
    t = q.sls_tau(lam, o["Phi_x"], o["Phi_u"], eps=1e-8)
    q.close()
    to = oracle.sls_tau(p, lam, o["Phi_x"], o["Phi_u"], eps=1e-8)
    assert _rel(t, to) < 1e-4


def test_sls_with_appendix_b_tau_pipeline():
    """The SLS workload's pipeline on one quadruped-shaped instance (N=64):
    nominal ADMM multipliers, tau of App. B from the tau = 0 responses, then
    the tau-weighted SLS.  Each GPU stage is checked against the oracle fed
    the same inputs (tau reaches ~5e5 here, where the penalty of rows with no
    disturbance response is |lambda| / sqrt(eps))."""
    probs, E, wb = W.sls_batch(2)
    p = probs[0]
    Qb, Rb, QbN = np.eye(p.nx), np.eye(p.nu), np.eye(p.nx)
    zero = np.zeros(p.N * p.N * p.nc + p.N * p.nf)
    base = oracle.sls_solve(p, E, zero, Qb, Rb, QbN, rownorm=1, wbound=wb)
    nom = oracle.qp_solve(p, rho=1.0, tol=1e-5)
    tau_o = oracle.sls_tau(p, nom["lam"], base["Phi_x"], base["Phi_u"])
    q = gsls.QP(p)
    # tau on the GPU from the same multipliers and responses
    tau_g = q.sls_tau(nom["lam"], base["Phi_x"], base["Phi_u"])
    np.testing.assert_allclose(tau_g, tau_o, rtol=1e-3, atol=1e-6)
    # SLS on the GPU with the oracle's tau
    g = q.sls_solve(E, tau_o, Qb, Rb, QbN, rownorm=1, wbound=wb, want_phi=False)
    o = oracle.sls_solve(p, E, tau_o, Qb, Rb, QbN, rownorm=1, wbound=wb, want_phi=False)
    assert _rel(g["h"], o["h"]) < 1e-3, _rel(g["h"], o["h"])
    # the batched entry point with two instances' tau
    nom1 = oracle.qp_solve(probs[1], rho=1.0, tol=1e-5)
    tau1 = oracle.sls_tau(probs[1], nom1["lam"], base["Phi_x"], base["Phi_u"])
    r = q.sls_solve_batch(E, [tau_o, tau1], Qb, Rb, QbN, rownorm=1, wbound=wb)
    assert _rel(r["h"][0], o["h"]) < 1e-3
    o1 = oracle.sls_solve(probs[1], E, tau1, Qb, Rb, QbN, rownorm=1, wbound=wb, want_phi=False)
    assert _rel(r["h"][1], o1["h"]) < 1e-3
    q.close()
