"""FP64 CPU oracle for the GPU-SLS ADMM QP and SLS hot path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg import this package; the product library never does, and the
two share no code.  Inputs come from the seeded generators in
``paper_2604_07644_amd.workloads`` (which hold none of the method's arithmetic).

Modules
  oracle.c / native  sequential Riccati ADMM (timed baseline) and per-column
                     SLS Riccati, margins, tau (C, FP64)
  dense              dense-KKT ADMM, dense LQ solve, KKT residuals, active-set
                     brute force (numpy, FP64)
  scan               conditional value functions and their combination rules,
                     the affine forward composition (numpy, FP64)
  mlp                FP64 reference MLP forward / backward / Adam (numpy)
"""
from .native import (qp_solve, qp_factor, sls_solve, sls_tau, Settings,  # noqa: F401
                     lib_path)
