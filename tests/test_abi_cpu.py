"""Host-side checks of the C ABI (no device calls): the library loads, exports
every entry point declared in include/gsls.h, and the host-side validation
returns the documented codes."""
import ctypes as ct
import os
import re

import numpy as np
import pytest

from paper_2604_07644_amd import gsls, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    txt = open(os.path.join(ROOT, "include", "gsls.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gsls_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    syms = _declared_symbols()
    assert len(syms) >= 10
    lib = ct.CDLL(gsls.LIB_PATH)
    missing = [s for s in syms if not hasattr(lib, s)]
    assert not missing, missing


def test_default_settings_and_strerror():
    s = gsls.default_settings()
    assert (s.precision, s.max_iter, s.adaptive_rho, s.sigma) == (gsls.MIXED, 10000, 1, 25)
    assert s.rho_min == 1e-6 and s.rho_max == 1e6 and s.rho_tol == 5.0
    for code in range(0, -8, -1):
        assert isinstance(gsls.strerror(code), str) and gsls.strerror(code) != "unknown error"


def test_validate_accepts_workloads():
    for p in (W.box_lq(), W.random_small(5, 3, 2, 2, 1, seed=0), W.polytopic_lq(8, 6, 2, 5)):
        assert gsls.validate_desc(p) == gsls.OK


@pytest.mark.parametrize("mutate, code", [
    (lambda p: p.A.__setitem__((0, 0, 0), np.nan), gsls.ERR_INVALID_ARG),
    (lambda p: p.q.__setitem__((1, 0), np.inf), gsls.ERR_INVALID_ARG),
    (lambda p: p.u.__setitem__(3, p.l[3] - 1.0), gsls.ERR_INVALID_ARG),
    (lambda p: p.l.__setitem__(2, np.inf), gsls.ERR_INVALID_ARG),
    (lambda p: setattr(p, "nx", 200), gsls.ERR_DIM),
    (lambda p: setattr(p, "nu", 0), gsls.ERR_DIM),
    (lambda p: setattr(p, "N", 0), gsls.ERR_DIM),
])
def test_validate_rejects(mutate, code):
    p = W.box_lq()
    mutate(p)
    if p.nx != 4 or p.nu != 2 or p.N != 32:
        d = gsls.QPDesc(N=p.N, nx=p.nx, nu=p.nu, nc=p.nc, nf=p.nf, mem=gsls.HOST)
        assert gsls.lib.gsls_validate_desc(ct.byref(d)) == code
    else:
        assert gsls.validate_desc(p) == code


def test_setup_rejects_bad_input_before_touching_the_device():
    p = W.box_lq(); p.B[3, 1, 0] = np.nan
    with pytest.raises(gsls.GslsError) as ei:
        gsls.QP(p)
    assert ei.value.code == gsls.ERR_INVALID_ARG
    with pytest.raises(gsls.GslsError) as ei:
        gsls.QP(W.box_lq(), gsls.default_settings(precision=7))
    assert ei.value.code == gsls.ERR_INVALID_ARG
    with pytest.raises(gsls.GslsError) as ei:
        gsls.QP(W.box_lq(), gsls.default_settings(fp64_fallback=2))
    assert ei.value.code == gsls.ERR_INVALID_ARG


def test_settings_struct_matches_the_header():
    s = gsls.default_settings()
    assert s.fp64_fallback == 0 and s.refresh == 0
    # 4 int32, 3 double, 4 int32 (the last one fp64_fallback): 56 bytes
    assert ct.sizeof(gsls.Settings) == 56
    assert gsls.Result.fallback.offset == gsls.Result.cold_restart.offset + 4


def test_null_handle_calls_fail_cleanly():
    r = gsls.Result()
    x0 = np.zeros(4)
    assert gsls.lib.gsls_qp_solve(None, x0.ctypes.data_as(gsls._dp), 1.0, 1e-5, ct.byref(r)) == gsls.ERR_INVALID_ARG
    assert gsls.lib.gsls_qp_get(None, None, None, None, None) == gsls.ERR_INVALID_ARG
    gsls.lib.gsls_qp_free(None)


def test_one_hip_runtime_per_process():
    """The binding loads PyTorch's HIP runtime before the library, so a process
    that uses both holds exactly one libamdhip64 (two runtimes cannot share
    streams or device pointers)."""
    import paper_2604_07644_amd.gsls  # noqa: F401
    import torch  # noqa: F401
    maps = open("/proc/self/maps").read().splitlines()
    libs = {ln.split()[-1] for ln in maps if "libamdhip64" in ln}
    assert len(libs) == 1, libs
