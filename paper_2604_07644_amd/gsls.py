"""ctypes binding of the C ABI in include/gsls.h (argument marshalling only).

Every computation happens in libgsls.so's HIP kernels.  Importing this module
loads the library and fails loudly if it has not been built; there is no CPU
fallback.
"""
from __future__ import annotations

import atexit
import ctypes as ct
import os
import sys
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgsls.so")

OK = 0
ERR_INVALID_ARG, ERR_DIM, ERR_NOT_PD, ERR_NUMERICAL, ERR_OOM, ERR_HIP, ERR_STATE = range(-1, -8, -1)
SOLVED, MAX_ITER, NUMERICAL_FAIL, INFEASIBLE_SUSPECTED = 1, 2, 3, 4
HOST, DEVICE = 0, 1
MIXED, FP64 = 0, 1

_dp = ct.POINTER(ct.c_double)
_fp = ct.POINTER(ct.c_float)


# outcomes of gsls_robust_solve
ROBUST_CONVERGED, ROBUST_PASS_LIMIT, ROBUST_INFEASIBLE, ROBUST_NOMINAL_FAILED = 1, 2, 4, 5


# parts of the learned warm start (gsls_qp_solve_batch_ws)
WS_RHO, WS_Z, WS_Y, WS_ALL = 1, 2, 4, 7


class QPDesc(ct.Structure):
    _fields_ = [("N", ct.c_int32), ("nx", ct.c_int32), ("nu", ct.c_int32), ("nc", ct.c_int32),
                ("nf", ct.c_int32), ("mem", ct.c_int32),
                ("A", _dp), ("B", _dp), ("b", _dp), ("Q", _dp), ("R", _dp), ("S", _dp),
                ("q", _dp), ("r", _dp), ("C", _dp), ("D", _dp), ("CN", _dp), ("l", _dp), ("u", _dp)]


class RobustResult(ct.Structure):
    _fields_ = [("status", ct.c_int32), ("passes", ct.c_int32), ("qp_solves", ct.c_int32),
                ("qp_iterations", ct.c_int32), ("qp_status", ct.c_int32), ("reserved", ct.c_int32),
                ("h_change", ct.c_double), ("ms_nominal", ct.c_double), ("ms_controller", ct.c_double)]

    def asdict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class ModelDesc(ct.Structure):
    _fields_ = [("model", ct.c_int32), ("N", ct.c_int32), ("n_obs", ct.c_int32), ("reserved", ct.c_int32),
                ("dt", ct.c_double), ("v", ct.c_double), ("mass", ct.c_double), ("gravity", ct.c_double),
                ("arm", ct.c_double), ("inertia", ct.c_double), ("obstacles", _dp), ("u_min", _dp),
                ("u_max", _dp), ("Q", _dp), ("R", _dp), ("QN", _dp), ("x_ref", _dp), ("u_ref", _dp)]


class SqpResult(ct.Structure):
    _fields_ = [("status", ct.c_int32), ("iterations", ct.c_int32), ("qp_iterations", ct.c_int32),
                ("qp_status", ct.c_int32), ("step", ct.c_double), ("ms_linearize", ct.c_double),
                ("ms_qp", ct.c_double)]

    def asdict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Settings(ct.Structure):
    _fields_ = [("precision", ct.c_int32), ("max_iter", ct.c_int32), ("adaptive_rho", ct.c_int32),
                ("sigma", ct.c_int32), ("rho_min", ct.c_double), ("rho_max", ct.c_double),
                ("rho_tol", ct.c_double), ("chunks_epoch", ct.c_int32), ("chunks_iter", ct.c_int32),
                ("refresh", ct.c_int32), ("fp64_fallback", ct.c_int32)]


class Result(ct.Structure):
    _fields_ = [("status", ct.c_int32), ("iterations", ct.c_int32), ("rho_updates", ct.c_int32),
                ("factorizations", ct.c_int32), ("r_p", ct.c_double), ("r_d", ct.c_double),
                ("rho", ct.c_double), ("ms_total", ct.c_double), ("ms_factor", ct.c_double),
                ("ms_iterate", ct.c_double), ("cold_restart", ct.c_int32), ("fallback", ct.c_int32),
                ("r_dyn", ct.c_double)]

    def asdict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class GslsError(RuntimeError):
    def __init__(self, code, where=""):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} ({code})")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libgsls.so not built at {LIB_PATH}; run paper_2604_07644_amd/build.py")
    # One HIP runtime per process: PyTorch ships its own libamdhip64 (soname
    # libamdhip64.so.7, loaded through an unversioned dependency).  Loading
    # torch first makes the library's libamdhip64.so.7 dependency resolve to
    # that same runtime, so streams and device pointers from torch are valid
    # here; loading the system runtime first would give the process two.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ct.CDLL(LIB_PATH)
    P = ct.c_void_p
    sig = {
        "gsls_default_settings": (None, [ct.POINTER(Settings)]),
        "gsls_strerror": (ct.c_char_p, [ct.c_int]),
        "gsls_validate_desc": (ct.c_int, [ct.POINTER(QPDesc)]),
        "gsls_qp_setup": (ct.c_int, [ct.POINTER(QPDesc), ct.POINTER(Settings), P, ct.POINTER(P)]),
        "gsls_qp_update_bounds": (ct.c_int, [P, _dp, _dp]),
        "gsls_qp_solve": (ct.c_int, [P, _dp, ct.c_double, ct.c_double, ct.POINTER(Result)]),
        "gsls_qp_solve_warm": (ct.c_int, [P, _dp, ct.c_double, ct.c_double, _dp, _dp, ct.POINTER(Result)]),
        "gsls_qp_get": (ct.c_int, [P, _dp, _dp, _dp, _dp]),
        "gsls_qp_free": (None, [P]),
        "gsls_sls_solve": (ct.c_int, [P, _dp, _dp, _dp, _dp, _dp, ct.c_int32, ct.c_double, _dp, _dp, _dp, _dp]),
        "gsls_sls_solve_batch": (ct.c_int, [P, ct.c_int32, _dp, _dp, _dp, _dp, _dp, ct.c_int32, ct.c_double,
                                            _dp, _dp, _dp]),
        "gsls_sls_tau": (ct.c_int, [P, _dp, _dp, _dp, ct.c_double, _dp]),
        "gsls_qp_update_data": (ct.c_int, [P, ct.POINTER(QPDesc)]),
        "gsls_sqp_setup": (ct.c_int, [ct.POINTER(ModelDesc), _dp, _dp, ct.POINTER(Settings), P, ct.POINTER(P)]),
        "gsls_sqp_linearize": (ct.c_int, [P, _dp, _dp] + [_dp] * 10),
        "gsls_sqp_solve": (ct.c_int, [P, _dp, _dp, _dp, ct.c_int32, ct.c_double, ct.c_double, ct.c_double,
                                      ct.POINTER(SqpResult)]),
        "gsls_rti_step": (ct.c_int, [P, _dp, _dp, _dp, _dp, _dp, _dp, _dp, ct.c_int32, ct.c_double, ct.c_double,
                                     ct.c_int32, ct.POINTER(RobustResult), _dp, _dp]),
        "gsls_sqp_free": (None, [P]),
        "gsls_robust_solve": (ct.c_int, [P, _dp, _dp, _dp, _dp, _dp, ct.c_int32, ct.c_double, ct.c_double,
                                         ct.c_double, ct.c_double, ct.c_int32, ct.c_double,
                                         ct.POINTER(RobustResult), _dp, _dp]),
        "gsls_debug_phase_cycles": (ct.c_int, [P, ct.c_int32, _dp, ct.POINTER(ct.c_int32)]),
        "gsls_qp_setup_batch": (ct.c_int, [ct.POINTER(QPDesc), ct.c_int32, ct.POINTER(Settings), P, ct.POINTER(P)]),
        "gsls_qp_solve_batch": (ct.c_int, [P, ct.POINTER(_dp), _dp, ct.c_double, ct.POINTER(_dp), ct.POINTER(_dp),
                                           ct.POINTER(Result), _dp]),
        "gsls_batch_get": (ct.c_int, [P, ct.c_int32, _dp, _dp, _dp, _dp]),
        "gsls_batch_free": (None, [P]),
        "gsls_batch_debug_phase_cycles": (ct.c_int, [P, ct.c_int32, _dp]),
        "gsls_batch_set_schedule": (ct.c_int, [P, ct.c_int32, ct.c_double]),
        "gsls_batch_get_schedule": (ct.c_int, [P, ct.POINTER(ct.c_int32), _dp, ct.POINTER(ct.c_int32)]),
        "gsls_ws_nparams": (ct.c_int64, []),
        "gsls_ws_create": (ct.c_int, [_fp, _fp, P, ct.POINTER(P)]),
        "gsls_ws_get_params": (ct.c_int, [P, _fp]),
        "gsls_ws_save": (ct.c_int, [P, ct.c_char_p]),
        "gsls_ws_load": (ct.c_int, [ct.c_char_p, P, ct.POINTER(P)]),
        "gsls_ws_forward": (ct.c_int, [P, P, ct.c_int32, P]),
        "gsls_ws_forward_static": (ct.c_int, [P, P, ct.c_int32, P]),
        "gsls_ws_loss_grad": (ct.c_int, [P, P, P, P, P, ct.c_int32, _fp, _fp]),
        "gsls_ws_train_step": (ct.c_int, [P, P, P, P, P, ct.c_int32, ct.c_float, _fp]),
        "gsls_ws_batch_rows": (ct.c_int32, [P]),
        "gsls_ws_features": (ct.c_int, [P, P, ct.POINTER(_dp), P]),
        "gsls_ws_targets": (ct.c_int, [P, P, P]),
        "gsls_qp_solve_batch_ws": (ct.c_int, [P, P, ct.POINTER(_dp), ct.c_double, ct.c_int32, ct.c_int32,
                                              ct.POINTER(Result),
                                              _dp, _dp]),
        "gsls_ws_free": (None, [P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()

# Handles still open when the interpreter exits are not freed: by then the
# HIP runtime (or a profiler attached to it) may already be shutting down, and
# a device call from a finaliser can crash the process after its work is
# done.  The process exit releases the device memory.
_exiting = False


def _mark_exiting():
    global _exiting
    _exiting = True


atexit.register(_mark_exiting)


def _can_free():
    return lib is not None and not _exiting and not sys.is_finalizing()


def strerror(code: int) -> str:
    return lib.gsls_strerror(int(code)).decode()


def default_settings(**kw) -> Settings:
    s = Settings()
    lib.gsls_default_settings(ct.byref(s))
    for k, v in kw.items():
        setattr(s, k, v)
    return s


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _check_len(a, n, what):
    """The C side reads exactly n doubles from a: refuse any other length."""
    if a is not None and a.size != n:
        raise ValueError(f"{what}: expected {n} values, got {a.size}")
    return a


def make_desc(prob):
    """QPDesc with host pointers for a workloads.QPProblem; returns (desc, keepalive)."""
    N, nx, nu, nc, nf = prob.N, prob.nx, prob.nu, prob.nc, prob.nf
    arrs = dict(A=_f64(prob.A), B=_f64(prob.B), b=_f64(prob.b), Q=_f64(prob.Q), R=_f64(prob.R),
                S=_f64(prob.S), q=_f64(prob.q), r=_f64(prob.r), C=_f64(prob.C), D=_f64(prob.D),
                CN=_f64(prob.CN, (nf, nx)) if nf else None, l=_f64(prob.l), u=_f64(prob.u))
    d = QPDesc(N=N, nx=nx, nu=nu, nc=nc, nf=nf, mem=HOST)
    for k, v in arrs.items():
        setattr(d, k, _ptr(v))
    return d, arrs


def validate_desc(prob) -> int:
    d, keep = make_desc(prob)
    return lib.gsls_validate_desc(ct.byref(d))


class QP:
    """One QP handle (gsls_qp_setup ... gsls_qp_free)."""

    def __init__(self, prob, settings: Optional[Settings] = None, stream=None, **kw):
        self.prob = prob
        self.settings = settings or default_settings(**kw)
        d, keep = make_desc(prob)
        h = ct.c_void_p()
        rc = lib.gsls_qp_setup(ct.byref(d), ct.byref(self.settings),
                               ct.c_void_p(stream) if stream else None, ct.byref(h))
        if rc != OK:
            raise GslsError(rc, "gsls_qp_setup")
        self.h = h
        self.result = None

    def close(self):
        if getattr(self, "h", None):
            if _can_free():
                lib.gsls_qp_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:   # interpreter teardown: the module's globals may already be gone
            pass

    def update_bounds(self, l, u):
        l = _f64(l); u = _f64(u)
        rc = lib.gsls_qp_update_bounds(self.h, _ptr(l), _ptr(u))
        if rc != OK:
            raise GslsError(rc, "gsls_qp_update_bounds")

    def solve(self, x0=None, rho=1.0, tol=1e-5, z0=None, y0=None) -> dict:
        p = self.prob
        x0 = _check_len(_f64(p.x0 if x0 is None else x0), p.nx, "x0")
        res = Result()
        if (z0 is None) != (y0 is None):
            raise ValueError("z0 and y0 go together")
        if z0 is None:
            rc = lib.gsls_qp_solve(self.h, _ptr(x0), rho, tol, ct.byref(res))
        else:
            z0 = _check_len(_f64(z0), p.m, "z0"); y0 = _check_len(_f64(y0), p.m, "y0")
            rc = lib.gsls_qp_solve_warm(self.h, _ptr(x0), rho, tol, _ptr(z0), _ptr(y0), ct.byref(res))
        if rc != OK:
            raise GslsError(rc, "gsls_qp_solve")
        self.result = res.asdict()
        return self.result

    def get(self) -> dict:
        p = self.prob
        X = np.zeros((p.N + 1, p.nx)); U = np.zeros((p.N, p.nu)); z = np.zeros(p.m); lam = np.zeros(p.m)
        rc = lib.gsls_qp_get(self.h, _ptr(X), _ptr(U), _ptr(z), _ptr(lam))
        if rc != OK:
            raise GslsError(rc, "gsls_qp_get")
        return dict(X=X, U=U, z=z, lam=lam)

    def phase_cycles(self, enable=-1):
        """Per-phase shader cycles of the iteration kernel (see gsls.h) and the
        chunk layout (Pe, Pi, resident, Lmax)."""
        out = np.zeros(16)
        lay = (ct.c_int32 * 4)()
        rc = lib.gsls_debug_phase_cycles(self.h, int(enable), _ptr(out), lay)
        if rc != OK:
            raise GslsError(rc, "gsls_debug_phase_cycles")
        return out, tuple(lay)

    def sls_solve(self, E, tau, Qbar, Rbar, QbarN, rownorm=2, wbound=1.0, want_phi=True):
        p = self.prob
        N, nx, nu, nc, nf = p.N, p.nx, p.nu, p.nc, p.nf
        Px = np.zeros((N * (N + 1) // 2, nx, nx)) if want_phi else None
        Pu = np.zeros((N * (N - 1) // 2, nu, nx)) if want_phi else None
        h = np.zeros((N, nc)); hf = np.zeros(nf)
        E = _f64(E); tau = _f64(tau); Qbar = _f64(Qbar); Rbar = _f64(Rbar); QbarN = _f64(QbarN)
        rc = lib.gsls_sls_solve(self.h, _ptr(E), _ptr(tau), _ptr(Qbar), _ptr(Rbar), _ptr(QbarN),
                                int(rownorm), float(wbound), _ptr(Px), _ptr(Pu), _ptr(h), _ptr(hf))
        if rc != OK:
            raise GslsError(rc, "gsls_sls_solve")
        return dict(Phi_x=Px, Phi_u=Pu, h=h, hf=hf)

    def sls_solve_batch(self, E, taus, Qbar, Rbar, QbarN, rownorm=2, wbound=1.0):
        p = self.prob
        cnt = len(taus)
        h = np.zeros((cnt, p.N, p.nc)); hf = np.zeros((cnt, p.nf)); ms = np.zeros(1)
        E = _f64(E); tau = _f64(np.concatenate([np.asarray(t).reshape(-1) for t in taus]))
        Qbar = _f64(Qbar); Rbar = _f64(Rbar); QbarN = _f64(QbarN)
        rc = lib.gsls_sls_solve_batch(self.h, cnt, _ptr(E), _ptr(tau), _ptr(Qbar), _ptr(Rbar), _ptr(QbarN),
                                      int(rownorm), float(wbound), _ptr(h), _ptr(hf), _ptr(ms))
        if rc != OK:
            raise GslsError(rc, "gsls_sls_solve_batch")
        return dict(h=h, hf=hf, ms=float(ms[0]))

    def sls_tau(self, lam, Phi_x, Phi_u, eps=1e-8):
        p = self.prob
        tau = np.zeros(p.N * p.N * p.nc + p.N * p.nf)
        lam = _f64(lam); Phi_x = _f64(Phi_x); Phi_u = _f64(Phi_u)
        rc = lib.gsls_sls_tau(self.h, _ptr(lam), _ptr(Phi_x), _ptr(Phi_u), float(eps), _ptr(tau))
        if rc != OK:
            raise GslsError(rc, "gsls_sls_tau")
        return tau

    def robust_solve(self, E, Qbar, Rbar, QbarN, rownorm=1, wbound=1.0, eps=1e-8, rho=1.0, tol=1e-6,
                     max_passes=10, htol=1e-3, x0=None):
        """FastSLS alternation (gsls_robust_solve).  Returns the outcome and the
        final margins; the final nominal trajectory is read with get()."""
        p = self.prob
        h = np.zeros((p.N, p.nc)); hf = np.zeros(p.nf)
        x0 = _check_len(_f64(p.x0 if x0 is None else x0), p.nx, "x0")
        E = _f64(E); Qbar = _f64(Qbar); Rbar = _f64(Rbar); QbarN = _f64(QbarN)
        res = RobustResult()
        rc = lib.gsls_robust_solve(self.h, _ptr(x0), _ptr(E), _ptr(Qbar), _ptr(Rbar), _ptr(QbarN), int(rownorm),
                                   float(wbound), float(eps), float(rho), float(tol), int(max_passes), float(htol),
                                   ct.byref(res), _ptr(h), _ptr(hf))
        if rc != OK:
            raise GslsError(rc, "gsls_robust_solve")
        out = res.asdict()
        out.update(h=h, hf=hf)
        return out


MODEL_DUBINS, MODEL_QUADROTOR = 1, 2


class SQP:
    """SQP and real-time iteration on an analytic model (gsls_sqp_*).  The
    scenario is a dict as produced by paper_2604_07644_amd.workloads
    (dubins_scenario / quadrotor_scenario)."""

    def __init__(self, sc, settings: Optional[Settings] = None, stream=None, **kw):
        self.kind = int(sc["kind"])
        self.N = int(sc["N"])
        self.nx, self.nu = (3, 1) if self.kind == MODEL_DUBINS else (6, 2)
        obst = np.asarray(sc.get("obstacles", np.zeros((0, 3))), dtype=np.float64).reshape(-1, 3)
        self.n_obs = obst.shape[0]
        self._keep = [_f64(obst.reshape(-1) if obst.size else np.zeros(3)), _f64(sc["u_min"]), _f64(sc["u_max"]),
                      _f64(sc["Q"]), _f64(sc["R"]), _f64(sc["QN"]), _f64(sc["x_ref"]), _f64(sc["u_ref"])]
        d = ModelDesc()
        d.model, d.N, d.n_obs = self.kind, self.N, self.n_obs
        d.dt = float(sc["dt"]); d.v = float(sc.get("v", 1.0)); d.mass = float(sc.get("mass", 1.0))
        d.gravity = float(sc.get("grav", 9.81)); d.arm = float(sc.get("arm", 0.0)); d.inertia = float(sc.get("inertia", 1.0))
        (d.obstacles, d.u_min, d.u_max, d.Q, d.R, d.QN, d.x_ref, d.u_ref) = [_ptr(a) for a in self._keep]
        self.desc = d
        s = settings or default_settings(**kw)
        X = _f64(sc["X"]); U = _f64(sc["U"])
        h = ct.c_void_p()
        rc = lib.gsls_sqp_setup(ct.byref(d), _ptr(X), _ptr(U), ct.byref(s), ct.c_void_p(stream or 0), ct.byref(h))
        if rc != OK:
            raise GslsError(rc, "gsls_sqp_setup")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            if _can_free():
                lib.gsls_sqp_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:   # interpreter teardown: the module's globals may already be gone
            pass

    def _check_traj(self, X, U, x0):
        X = np.array(X, dtype=np.float64); U = np.array(U, dtype=np.float64)
        _check_len(X, (self.N + 1) * self.nx, "X"); _check_len(U, self.N * self.nu, "U")
        return X, U, _check_len(_f64(x0), self.nx, "x0")

    @property
    def dims(self):
        nc = self.n_obs + self.nu
        return self.N, self.nx, self.nu, nc, self.n_obs

    def linearize(self, X, U):
        N, nx, nu, nc, nf = self.dims
        out = dict(A=np.zeros((N, nx, nx)), B=np.zeros((N, nx, nu)), b=np.zeros((N, nx)), q=np.zeros((N + 1, nx)),
                   r=np.zeros((N, nu)), C=np.zeros((N, nc, nx)), D=np.zeros((N, nc, nu)), CN=np.zeros((nf, nx)),
                   l=np.zeros(N * nc + nf), u=np.zeros(N * nc + nf))
        X = _f64(X); U = _f64(U)
        rc = lib.gsls_sqp_linearize(self.h, _ptr(X), _ptr(U), *[_ptr(out[k]) for k in
                                                              ("A", "B", "b", "q", "r", "C", "D", "CN", "l", "u")])
        if rc != OK:
            raise GslsError(rc, "gsls_sqp_linearize")
        return out

    def solve(self, x0, X, U, max_iter=20, alpha=1.0, tol_qp=1e-6, tol_step=1e-5):
        X, U, x0 = self._check_traj(X, U, x0)
        res = SqpResult()
        rc = lib.gsls_sqp_solve(self.h, _ptr(x0), _ptr(X), _ptr(U), int(max_iter), float(alpha), float(tol_qp),
                                float(tol_step), ct.byref(res))
        if rc != OK:
            raise GslsError(rc, "gsls_sqp_solve")
        return X, U, res.asdict()

    def rti_step(self, x0, X, U, E, Qbar, Rbar, QbarN, rownorm=1, wbound=1.0, tol_qp=1e-2, max_passes=0):
        N, nx, nu, nc, nf = self.dims
        X, U, x0 = self._check_traj(X, U, x0)
        h = np.zeros((N, nc)); hf = np.zeros(nf)
        E = _f64(E); Qbar = _f64(Qbar); Rbar = _f64(Rbar); QbarN = _f64(QbarN)
        res = RobustResult()
        rc = lib.gsls_rti_step(self.h, _ptr(x0), _ptr(X), _ptr(U), _ptr(E), _ptr(Qbar), _ptr(Rbar), _ptr(QbarN),
                               int(rownorm), float(wbound), float(tol_qp), int(max_passes), ct.byref(res),
                               _ptr(h), _ptr(hf))
        if rc != OK:
            raise GslsError(rc, "gsls_rti_step")
        out = res.asdict()
        out.update(h=h, hf=hf)
        return X, U, out


class Batch:
    """Many QPs solved in one persistent launch (gsls_qp_setup_batch ...)."""

    def __init__(self, probs, settings: Optional[Settings] = None, stream=None, **kw):
        self.probs = list(probs)
        self.settings = settings or default_settings(**kw)
        descs = (QPDesc * len(self.probs))()
        self._keep = []
        for i, p in enumerate(self.probs):
            d, keep = make_desc(p)
            descs[i] = d
            self._keep.append(keep)
        h = ct.c_void_p()
        rc = lib.gsls_qp_setup_batch(descs, len(self.probs), ct.byref(self.settings),
                                     ct.c_void_p(stream) if stream else None, ct.byref(h))
        self._keep = None
        if rc != OK:
            raise GslsError(rc, "gsls_qp_setup_batch")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            if _can_free():
                lib.gsls_batch_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:   # interpreter teardown: the module's globals may already be gone
            pass

    def solve(self, x0s=None, rhos=1.0, tol=1e-5, z0s=None, y0s=None):
        n = len(self.probs)
        x0s = self._x0_list(x0s)
        rh = _f64(np.broadcast_to(np.asarray(rhos, dtype=np.float64), (n,)).copy())
        xp = (_dp * n)(*[_ptr(x) for x in x0s])
        zp = yp = None
        keep = [x0s]
        if (z0s is None) != (y0s is None):
            raise ValueError("z0s and y0s go together")
        if z0s is not None:
            if len(z0s) != n or len(y0s) != n:
                raise ValueError(f"z0s, y0s: expected {n} entries")
            z0s = [None if z is None else _check_len(_f64(z), p.m, f"z0s[{i}]")
                   for i, (z, p) in enumerate(zip(z0s, self.probs))]
            y0s = [None if y is None else _check_len(_f64(y), p.m, f"y0s[{i}]")
                   for i, (y, p) in enumerate(zip(y0s, self.probs))]
            if any((z is None) != (y is None) for z, y in zip(z0s, y0s)):
                raise ValueError("z0s[i] and y0s[i] go together")
            keep += [z0s, y0s]
            zp = (_dp * n)(*[_ptr(z) for z in z0s])
            yp = (_dp * n)(*[_ptr(y) for y in y0s])
        res = (Result * n)()
        ms = np.zeros(1)
        rc = lib.gsls_qp_solve_batch(self.h, xp, _ptr(rh), float(tol), zp, yp, res, _ptr(ms))
        if rc != OK:
            raise GslsError(rc, "gsls_qp_solve_batch")
        self.results = [r.asdict() for r in res]
        return self.results, float(ms[0])

    def get(self, i):
        p = self.probs[i]
        X = np.zeros((p.N + 1, p.nx)); U = np.zeros((p.N, p.nu)); z = np.zeros(p.m); lam = np.zeros(p.m)
        rc = lib.gsls_batch_get(self.h, int(i), _ptr(X), _ptr(U), _ptr(z), _ptr(lam))
        if rc != OK:
            raise GslsError(rc, "gsls_batch_get")
        return dict(X=X, U=U, z=z, lam=lam)

    def _x0_list(self, x0s):
        n = len(self.probs)
        if x0s is None:
            return [_f64(p.x0) for p in self.probs]
        if len(x0s) != n:
            raise ValueError(f"x0s: expected {n} entries, got {len(x0s)}")
        return [_check_len(_f64(x), p.nx, f"x0s[{i}]") for i, (x, p) in enumerate(zip(x0s, self.probs))]

    def _x0_array(self, x0s):
        n = len(self.probs)
        x0s = self._x0_list(x0s)
        return x0s, (_dp * n)(*[_ptr(x) for x in x0s])

    def phase_cycles(self, enable=True):
        """Per-phase device clock counters of the iterations since the last
        call (gsls_batch_debug_phase_cycles); enable keeps counting."""
        out = np.zeros(16)
        rc = lib.gsls_batch_debug_phase_cycles(self.h, int(enable), _ptr(out))
        if rc != OK:
            raise GslsError(rc, "gsls_batch_debug_phase_cycles")
        return out

    def set_schedule(self, gang=0, park_share=0.0):
        """Gang schedule (gsls_batch_set_schedule): gang workgroups per
        handed-over instance (0 auto, 1 off), park_share the solo work budget."""
        rc = lib.gsls_batch_set_schedule(self.h, int(gang), float(park_share))
        if rc != OK:
            raise GslsError(rc, "gsls_batch_set_schedule")

    def schedule(self):
        """(gang, park_share, park_at[count]) of the current schedule."""
        g = ct.c_int32(0)
        sh = np.zeros(1)
        pa = np.zeros(len(self.probs), dtype=np.int32)
        rc = lib.gsls_batch_get_schedule(self.h, ct.byref(g), _ptr(sh),
                                         pa.ctypes.data_as(ct.POINTER(ct.c_int32)))
        if rc != OK:
            raise GslsError(rc, "gsls_batch_get_schedule")
        return int(g.value), float(sh[0]), pa

    def rows(self):
        """Number of warm-start feature rows (sum of N + 1)."""
        return int(lib.gsls_ws_batch_rows(self.h))

    def solve_ws(self, ws, x0s=None, tol=1e-5, warm_budget=0, parts=WS_ALL):
        """Learned warm start + solve (gsls_qp_solve_batch_ws).  Returns
        (results, ms_total, ms_predict)."""
        n = len(self.probs)
        keep, xp = self._x0_array(x0s)
        res = (Result * n)()
        ms = np.zeros(1); msp = np.zeros(1)
        rc = lib.gsls_qp_solve_batch_ws(self.h, ws.h, xp, float(tol), int(warm_budget), int(parts), res, _ptr(ms),
                                        _ptr(msp))
        if rc != OK:
            raise GslsError(rc, "gsls_qp_solve_batch_ws")
        self.results = [r.asdict() for r in res]
        return self.results, float(ms[0]), float(msp[0])


def _dev(t):
    return ct.c_void_p(t.data_ptr()) if t is not None else None


class WarmStart:
    """Learned warm-start model (gsls_ws_*).  Device arrays are torch tensors:
    features torch.bfloat16 [rows, 160], targets / mask / outputs float32
    [rows, 192], row indices int32."""

    D_IN, D_OUT = 160, 192

    def __init__(self, params=None, sketch=None, stream=None, path=None):
        h = ct.c_void_p()
        st = ct.c_void_p(stream) if stream else None
        if path is not None:
            rc = lib.gsls_ws_load(str(path).encode(), st, ct.byref(h))
            where = "gsls_ws_load"
        else:
            p = np.ascontiguousarray(params, dtype=np.float32)
            sk = np.ascontiguousarray(sketch, dtype=np.float32)
            if p.size != self.nparams() or sk.size != 64 * 94:
                raise GslsError(ERR_INVALID_ARG, "WarmStart: parameter or sketch size")
            rc = lib.gsls_ws_create(p.ctypes.data_as(_fp), sk.ctypes.data_as(_fp), st, ct.byref(h))
            where = "gsls_ws_create"
        if rc != OK:
            raise GslsError(rc, where)
        self.h = h

    @staticmethod
    def nparams():
        return int(lib.gsls_ws_nparams())

    def close(self):
        if getattr(self, "h", None):
            if _can_free():
                lib.gsls_ws_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:   # interpreter teardown: the module's globals may already be gone
            pass

    def params(self):
        p = np.zeros(self.nparams(), dtype=np.float32)
        rc = lib.gsls_ws_get_params(self.h, p.ctypes.data_as(_fp))
        if rc != OK:
            raise GslsError(rc, "gsls_ws_get_params")
        return p

    def save(self, path):
        rc = lib.gsls_ws_save(self.h, str(path).encode())
        if rc != OK:
            raise GslsError(rc, "gsls_ws_save")

    def forward(self, X):
        import torch
        Y = torch.empty((X.shape[0], self.D_OUT), dtype=torch.float32, device=X.device)
        rc = lib.gsls_ws_forward(self.h, _dev(X), int(X.shape[0]), _dev(Y))
        if rc != OK:
            raise GslsError(rc, "gsls_ws_forward")
        torch.cuda.synchronize()
        return Y

    def forward_static(self, X, Y=None):
        """gsls_ws_forward_static: the forward pass in the library's fixed
        workspace (no device allocation by the library; at most 2048 rows)."""
        import torch
        rows = int(X.shape[0])
        Y = torch.empty((rows, self.D_OUT), dtype=torch.float32, device=X.device) if Y is None else Y
        rc = lib.gsls_ws_forward_static(self.h, _dev(X), rows, _dev(Y))
        if rc != OK:
            raise GslsError(rc, "gsls_ws_forward_static")
        torch.cuda.synchronize()
        return Y

    def loss_grad(self, X, T, M, idx=None, rows=None):
        rows = int(idx.shape[0] if idx is not None else X.shape[0]) if rows is None else int(rows)
        g = np.zeros(self.nparams(), dtype=np.float32)
        loss = np.zeros(1, dtype=np.float32)
        rc = lib.gsls_ws_loss_grad(self.h, _dev(X), _dev(T), _dev(M), _dev(idx), rows, g.ctypes.data_as(_fp),
                                   loss.ctypes.data_as(_fp))
        if rc != OK:
            raise GslsError(rc, "gsls_ws_loss_grad")
        return float(loss[0]), g

    def train_step(self, X, T, M, idx=None, rows=None, lr=1e-3, want_loss=False):
        rows = int(idx.shape[0] if idx is not None else X.shape[0]) if rows is None else int(rows)
        loss = np.zeros(1, dtype=np.float32)
        rc = lib.gsls_ws_train_step(self.h, _dev(X), _dev(T), _dev(M), _dev(idx), rows, float(lr),
                                    loss.ctypes.data_as(_fp) if want_loss else None)
        if rc != OK:
            raise GslsError(rc, "gsls_ws_train_step")
        return float(loss[0]) if want_loss else None

    def features(self, batch, x0s=None):
        import torch
        X = torch.empty((batch.rows(), self.D_IN), dtype=torch.bfloat16, device="cuda")
        keep, xp = batch._x0_array(x0s)
        rc = lib.gsls_ws_features(self.h, batch.h, xp, _dev(X))
        if rc != OK:
            raise GslsError(rc, "gsls_ws_features")
        return X

    @staticmethod
    def targets(batch):
        import torch
        n = batch.rows()
        T = torch.empty((n, WarmStart.D_OUT), dtype=torch.float32, device="cuda")
        M = torch.empty_like(T)
        rc = lib.gsls_ws_targets(batch.h, _dev(T), _dev(M))
        if rc != OK:
            raise GslsError(rc, "gsls_ws_targets")
        return T, M
