"""MI355X (gfx950) implementation of the GPU-SLS hot path: an ADMM solver for
stage-structured LTV-QPs whose LQR subproblem is solved by associative scans
over the horizon with cached rho-invariant factors, and the SLS controller
synthesis (system responses Phi^x / Phi^u and reachable-set margins) on the
same scan backend.

The compute runs in hand-written HIP kernels behind the C ABI of
``include/gsls.h`` (``libgsls.so``); ``gsls`` is a thin ctypes binding with the
same names (imported on first use: ``from paper_2604_07644_amd import gsls``
loads the library and raises ImportError if it is not built).  ``workloads``
holds the seeded synthetic problem generators (numpy only).
"""
import importlib


def __getattr__(name):
    if name == "gsls":
        return importlib.import_module(".gsls", __name__)
    raise AttributeError(name)
