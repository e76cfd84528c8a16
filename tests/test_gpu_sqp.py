"""GPU parity of the SQP on the analytic models (gsls_sqp_*, Sec. III-B, App. C
and D) and of one real-time-iteration update (gsls_rti_step, Sec. IV-C)
against the oracle.

Bars: the linearisation (FP64 on both sides, same formulas) to 1e-12; the SQP
in FP64 mode follows the oracle's iterations (same count, nominal to 1e-7);
in mixed mode it reaches the same fixed point to the QP tolerance (1e-3); one
RTI update (linearisation, one controller update, tightened nominal step) to
2e-3, the level of one App. B step.
"""
import numpy as np
import pytest

from oracle import robust as R
from oracle import sqp as S
from paper_2604_07644_amd import workloads as W

pytestmark = pytest.mark.gpu

from paper_2604_07644_amd import gsls  # noqa: E402  (fails loudly without libgsls.so)

# (scenario, QP tolerance, step tolerance)
CASES = {"dubins": (lambda: W.dubins_scenario(N=60, n_obs=3, seed=0), 1e-6, 1e-5),
         "quadrotor": (lambda: W.quadrotor_scenario(N=40, n_obs=1, seed=3), 1e-4, 1e-3)}


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("name", list(CASES))
def test_linearization_matches_oracle(name):
    sc = CASES[name][0]()
    md = S.from_scenario(sc)
    rng = np.random.default_rng(2)
    X = sc["X"] + 0.05 * rng.standard_normal(sc["X"].shape)
    U = sc["U"] + 0.05 * rng.standard_normal(sc["U"].shape)
    q = gsls.SQP(sc, gsls.default_settings(precision=gsls.FP64))
    g = q.linearize(X, U)
    q.close()
    o = S.linearize(md, X, U, sc["x0"])
    for k in ("A", "B", "b", "q", "r", "C", "D", "CN"):
        want = getattr(o, k)
        assert np.allclose(g[k], want, rtol=1e-12, atol=1e-12), k
    fin = np.isfinite(o.u)
    assert np.array_equal(np.isfinite(g["u"]), fin) and np.array_equal(np.isfinite(g["l"]), np.isfinite(o.l))
    assert np.allclose(g["u"][fin], o.u[fin], rtol=1e-12, atol=1e-12)
    fl = np.isfinite(o.l)
    assert np.allclose(g["l"][fl], o.l[fl], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("name", list(CASES))
def test_sqp_fp64_follows_oracle(name):
    make, tq, ts = CASES[name]
    sc = make()
    md = S.from_scenario(sc)
    o = S.sqp(md, sc["x0"], sc["X"], sc["U"], max_iter=40, alpha=1.0, tol_qp=tq, tol_step=ts)
    q = gsls.SQP(sc, gsls.default_settings(precision=gsls.FP64))
    X, U, r = q.solve(sc["x0"], sc["X"], sc["U"], max_iter=40, alpha=1.0, tol_qp=tq, tol_step=ts)
    q.close()
    assert o["status"] == 1 and r["status"] == 1, (o["status"], r)
    assert r["iterations"] == o["iterations"]
    assert _rel(X, o["X"]) <= 1e-7 and _rel(U, o["U"]) <= 1e-7


@pytest.mark.parametrize("name", list(CASES))
def test_sqp_mixed_reaches_the_fixed_point(name):
    make, tq, ts = CASES[name]
    sc = make()
    md = S.from_scenario(sc)
    o = S.sqp(md, sc["x0"], sc["X"], sc["U"], max_iter=40, alpha=1.0, tol_qp=tq, tol_step=ts)
    q = gsls.SQP(sc, gsls.default_settings(precision=gsls.MIXED))
    X, U, r = q.solve(sc["x0"], sc["X"], sc["U"], max_iter=40, alpha=1.0, tol_qp=tq, tol_step=ts)
    q.close()
    assert r["status"] == 1, r
    assert _rel(X, o["X"]) <= 1e-3 and _rel(U, o["U"]) <= 1e-3


@pytest.mark.parametrize("name", list(CASES))
def test_rti_step_matches_oracle(name):
    make, tol, _ = CASES[name]
    sc = make()
    md = S.from_scenario(sc)
    nx, nu = md.nx, md.nu
    Qb, Rb, QbN = np.eye(nx), np.eye(nu), np.eye(nx)
    # the Dubins margins grow along its 60 stages (heading disturbances integrate
    # into position): at |w|_inf <= 1 they exceed the free space, at 0.3 not
    wb = 0.3 if name == "dubins" else 1.0
    qp = S.linearize(md, sc["X"], sc["U"], sc["x0"])
    Es = np.stack([sc["E"]] * md.N)
    o = R.robust_alternation(qp, Es, Qb, Rb, QbN, rownorm=1, wbound=wb, tol=tol, max_passes=1, htol=0.0)
    q = gsls.SQP(sc, gsls.default_settings(precision=gsls.FP64))
    X, U, r = q.rti_step(sc["x0"], sc["X"], sc["U"], sc["E"], Qb, Rb, QbN, rownorm=1, wbound=wb, tol_qp=tol,
                         max_passes=1)
    q.close()
    assert r["status"] == o["status"] and r["passes"] == 1
    assert _rel(X, sc["X"] + o["X"]) <= 2e-3 and _rel(U, sc["U"] + o["U"]) <= 2e-3
    hg = np.concatenate([r["h"].ravel(), r["hf"]])
    ho = np.concatenate([o["h"].ravel(), o["hf"]])
    assert _rel(hg, ho) <= 2e-3
