"""ctypes front end of the C oracle (oracle.c).  Test infrastructure only.

Every function here returns plain numpy FP64 arrays.  The C code follows the
paper: the ADMM of Sec. III-C on eq. (admm_qp) with the Riccati solution of
the LQR subproblem eq. (primal_update) / eq. (controller_cache), and the SLS
recursions eq. (backward_prop) / eq. (forward_prop) with the margins of
Sec. III-D and the tau weights of App. B.
"""
from __future__ import annotations

import ctypes as ct
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(_HERE, "_oracle.so")
_lib = None

_dp = ct.POINTER(ct.c_double)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(lib_path):
            from .build import build
            build()
        _lib = ct.CDLL(lib_path)
        _lib.oracle_qp_solve.restype = ct.c_int
        _lib.oracle_qp_factor.restype = ct.c_int
        _lib.oracle_sls_solve.restype = ct.c_int
        _lib.oracle_sls_tau.restype = None
    return _lib


def _p(a):
    if a is None:
        return None
    return a.ctypes.data_as(_dp)


def _c(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


@dataclass
class Settings:
    """ADMM settings.  Defaults: cold start, rho adaptation every sigma=25
    iterations by the OSQP rule with tolerance factor 5, rho in [1e-6, 1e6],
    at most 10000 iterations."""
    max_iter: int = 10000
    adaptive: bool = True
    sigma: int = 25
    rho_min: float = 1e-6
    rho_max: float = 1e6
    rho_tol: float = 5.0


def qp_factor(prob, rho):
    """Riccati factor of the augmented LQR for a fixed rho: (P [N+1,nx,nx], K [N,nu,nx])."""
    lib = _load()
    N, nx, nu, nc, nf = prob.N, prob.nx, prob.nu, prob.nc, prob.nf
    P = np.zeros((N + 1, nx, nx)); K = np.zeros((N, nu, nx))
    arrs = [_c(prob.A), _c(prob.B), _c(prob.Q), _c(prob.R), _c(prob.S), _c(prob.C),
            _c(prob.D), _c(prob.CN, (nf, nx))]
    rc = lib.oracle_qp_factor(N, nx, nu, nc, nf, *[_p(a) for a in arrs], ct.c_double(rho),
                              _p(P), _p(K))
    if rc != 0:
        raise np.linalg.LinAlgError("oracle_qp_factor: matrix not positive definite")
    return P, K


def qp_solve(prob, rho=1.0, tol=1e-6, settings: Settings | None = None, z0=None, y0=None,
             x0=None):
    """Riccati ADMM.  Returns dict X, U, z, y, lam, iters, r_p, r_d, rho, rho_updates,
    status (1 solved, 2 max_iter, -4 not PD, -5 numerical), r_dyn, factorizations."""
    lib = _load()
    s = settings or Settings()
    N, nx, nu, nc, nf = prob.N, prob.nx, prob.nu, prob.nc, prob.nf
    m = N * nc + nf
    X = np.zeros((N + 1, nx)); U = np.zeros((N, nu)); z = np.zeros(m); y = np.zeros(m)
    info = np.zeros(8)
    x0 = prob.x0 if x0 is None else x0
    arrs = [_c(prob.A), _c(prob.B), _c(prob.b), _c(prob.Q), _c(prob.R), _c(prob.S),
            _c(prob.q), _c(prob.r), _c(prob.C), _c(prob.D), _c(prob.CN, (nf, nx)),
            _c(prob.l), _c(prob.u), _c(x0)]
    z0a = None if z0 is None else _c(z0)
    y0a = None if y0 is None else _c(y0)
    lib.oracle_qp_solve(N, nx, nu, nc, nf, *[_p(a) for a in arrs], ct.c_double(rho),
                        ct.c_double(tol), int(s.max_iter), int(bool(s.adaptive)), int(s.sigma),
                        ct.c_double(s.rho_min), ct.c_double(s.rho_max), ct.c_double(s.rho_tol),
                        _p(z0a), _p(y0a), _p(X), _p(U), _p(z), _p(y), _p(info))
    return dict(X=X, U=U, z=z, y=y, lam=info[3] * y, iters=int(info[0]), r_p=info[1],
                r_d=info[2], rho=info[3], rho_updates=int(info[4]), status=int(info[5]),
                r_dyn=info[6], factorizations=int(info[7]))


def sls_layout(N):
    """Block offsets of the packed Phi^x / Phi^u columns (see oracle_sls_solve)."""
    offx = [j * N - j * (j - 1) // 2 for j in range(N)]
    offu = [j * (N - 1) - j * (j - 1) // 2 for j in range(N)]
    return offx, offu


def sls_solve(prob, E, tau, Qbar, Rbar, QbarN, rownorm=2, wbound=1.0, want_phi=True,
              want_K=False):
    """Per-column Riccati SLS.  Returns dict Phi_x [N(N+1)/2, nx, nx],
    Phi_u [N(N-1)/2, nu, nx], h [N, nc], hf [nf] (and K [N, N, nu, nx] if asked)."""
    lib = _load()
    N, nx, nu, nc, nf = prob.N, prob.nx, prob.nu, prob.nc, prob.nf
    Px = np.zeros((N * (N + 1) // 2, nx, nx)) if want_phi else None
    Pu = np.zeros((N * (N - 1) // 2, nu, nx)) if want_phi else None
    h = np.zeros((N, nc)); hf = np.zeros(nf)
    K = np.zeros((N, N, nu, nx)) if want_K else None
    arrs = [_c(prob.A), _c(prob.B), _c(prob.C), _c(prob.D), _c(prob.CN, (nf, nx)), _c(E),
            _c(tau), _c(Qbar), _c(Rbar), _c(QbarN)]
    rc = lib.oracle_sls_solve(N, nx, nu, nc, nf, *[_p(a) for a in arrs], int(rownorm),
                              ct.c_double(wbound), _p(Px), _p(Pu), _p(h), _p(hf), _p(K))
    if rc != 0:
        raise np.linalg.LinAlgError("oracle_sls_solve: matrix not positive definite")
    return dict(Phi_x=Px, Phi_u=Pu, h=h, hf=hf, K=K)


def sls_tau(prob, lam, Phi_x, Phi_u, eps=1e-8):
    """tau weights of App. B, layout [N*N*nc] stage part then [N*nf] terminal part."""
    lib = _load()
    N, nx, nu, nc, nf = prob.N, prob.nx, prob.nu, prob.nc, prob.nf
    tau = np.zeros(N * N * nc + N * nf)
    arrs = [_c(prob.C), _c(prob.D), _c(prob.CN, (nf, nx)), _c(lam), _c(Phi_x), _c(Phi_u)]
    lib.oracle_sls_tau(N, nx, nu, nc, nf, *[_p(a) for a in arrs], ct.c_double(eps), _p(tau))
    return tau


def qp_solve_many(probs, rho=1.0, tol=1e-6, settings: Settings | None = None, lib=None):
    """Cold-start Riccati ADMM of every instance (oracle_qp_solve_many: OpenMP
    over the instances when the library was built with it).  lib: a ctypes
    library (e.g. from load_native); default the portable build.  Returns
    (iterations [count], threads)."""
    lib = lib or _load()
    s = settings or Settings()
    n = len(probs)
    dims = np.zeros(5 * n, dtype=np.int32)
    keep = []
    ptrs = (_dp * (14 * n))()
    for c, p in enumerate(probs):
        dims[5 * c:5 * c + 5] = (p.N, p.nx, p.nu, p.nc, p.nf)
        arrs = [_c(p.A), _c(p.B), _c(p.b), _c(p.Q), _c(p.R), _c(p.S), _c(p.q), _c(p.r), _c(p.C), _c(p.D),
                _c(p.CN, (p.nf, p.nx)), _c(p.l), _c(p.u), _c(p.x0)]
        keep.append(arrs)
        for k, a in enumerate(arrs):
            ptrs[14 * c + k] = _p(a)
    info = np.zeros(8 * n)
    lib.oracle_qp_solve_many.restype = ct.c_int
    th = lib.oracle_qp_solve_many(int(n), dims.ctypes.data_as(ct.POINTER(ct.c_int32)), ptrs, ct.c_double(rho),
                                  ct.c_double(tol), int(s.max_iter), int(bool(s.adaptive)), int(s.sigma),
                                  ct.c_double(s.rho_min), ct.c_double(s.rho_max), ct.c_double(s.rho_tol),
                                  _p(info))
    return info.reshape(n, 8)[:, 0].astype(int), int(th)


def load_native(outdir):
    """The oracle compiled for this host (-O3 -march=native, OpenMP) into
    outdir, as a ctypes library."""
    from .build import build_native
    return ct.CDLL(build_native(outdir))

