// Device-side description of an analytic model and the QP arrays its
// linearisation writes (see models.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/gsls.h"

namespace gsls {

struct ModelDev {
  int kind, N, nx, nu, no;          // no: obstacles
  double dt, v, mass, grav, arm, inertia;
  const double* obst;               // [no][3] (cx, cy, r)
  const double *umin, *umax;        // [nu]
  const double *Q, *R, *QN;         // [nx][nx], [nu][nu], [nx][nx]
  const double *xref, *uref;        // [N+1][nx], [N][nu]
};

// Device arrays of one linearised QP, in the gsls_qp_desc layout.
struct LinOut {
  double *A, *B, *b, *Q, *R, *S, *q, *r, *C, *D, *CN, *l, *u;
};

int launch_linearize(const ModelDev& m, const double* X, const double* U, const LinOut& o, hipStream_t st);

}  // namespace gsls
