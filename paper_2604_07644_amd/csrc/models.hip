// Linearisation of the paper's analytic models for the SQP iteration of
// Sec. III-B, eq. (sqp_qp): the Dubins car (App. C) and the planar quadrotor
// (App. D, one explicit Euler step of its continuous dynamics), with obstacle
// rows r^2 - |p - c|^2 <= 0 (eq. (obstacle_constraints)) at every stage and at
// the terminal state and an input box at every stage.
//
// One thread per stage k = 0..N writes the stage's part of the QP in the
// gsls_qp_desc layout (FP64, device memory), around the nominal (X, U):
//   A_k = df/dx, B_k = df/du, b_k = f(x_k, u_k) - x_{k+1},
//   rows (obstacles first, then inputs):  C_k dx_k <= -g(x_k),
//        u_min - u_k <= du_k <= u_max - u_k;  terminal obstacle rows on x_N,
//   Q_k = Q, R_k = R, S_k = 0 (Hessian of the tracking cost),
//   q_k = Q (x_k - x_ref_k), r_k = R (u_k - u_ref_k), q_N = Q_N (x_N - x_ref_N).
#include <cmath>

#include "models.hpp"

namespace gsls {

__global__ void k_linearize(ModelDev m, const double* __restrict__ X, const double* __restrict__ U, LinOut o) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int N = m.N, nx = m.nx, nu = m.nu, no = m.no, nc = no + nu;
  if (k > N) return;
  const double* x = X + (size_t)k * nx;
  // obstacle rows of state x (stage rows, or the terminal rows at k = N)
  double* Crow = k < N ? o.C + (size_t)k * nc * nx : o.CN;
  double* ub = o.u + (size_t)k * nc;
  double* lb = o.l + (size_t)k * nc;
  for (int i = 0; i < no; ++i) {
    const double dx = x[0] - m.obst[3 * i], dy = x[1] - m.obst[3 * i + 1], r = m.obst[3 * i + 2];
    double* c = Crow + (size_t)i * nx;
    for (int j = 0; j < nx; ++j) c[j] = 0.0;
    c[0] = -2.0 * dx;
    c[1] = -2.0 * dy;
    ub[i] = -(r * r - dx * dx - dy * dy);
    lb[i] = -INFINITY;
  }
  if (k == N) {
    for (int j = 0; j < nx; ++j) {
      double s = 0.0;
      for (int t = 0; t < nx; ++t) s += m.QN[j * nx + t] * (x[t] - m.xref[(size_t)N * nx + t]);
      o.q[(size_t)N * nx + j] = s;
      for (int t = 0; t < nx; ++t) o.Q[((size_t)N * nx + j) * nx + t] = m.QN[j * nx + t];
    }
    return;
  }
  const double* u = U + (size_t)k * nu;
  const double* xn = X + (size_t)(k + 1) * nx;
  double* A = o.A + (size_t)k * nx * nx;
  double* B = o.B + (size_t)k * nx * nu;
  double* b = o.b + (size_t)k * nx;
  for (int i = 0; i < nx * nx; ++i) A[i] = (i % (nx + 1)) == 0 ? 1.0 : 0.0;
  for (int i = 0; i < nx * nu; ++i) B[i] = 0.0;
  const double dt = m.dt;
  if (m.kind == GSLS_MODEL_DUBINS) {
    const double s = sin(x[2]), c = cos(x[2]);
    A[0 * 3 + 2] = -m.v * s * dt;
    A[1 * 3 + 2] = m.v * c * dt;
    B[2] = dt;
    b[0] = x[0] + m.v * c * dt - xn[0];
    b[1] = x[1] + m.v * s * dt - xn[1];
    b[2] = x[2] + u[0] * dt - xn[2];
  } else {
    const double s = sin(x[2]), c = cos(x[2]), T = u[0] + u[1];
    A[0 * 6 + 3] = dt;
    A[1 * 6 + 4] = dt;
    A[2 * 6 + 5] = dt;
    A[3 * 6 + 2] = -dt * T * c / m.mass;
    A[4 * 6 + 2] = -dt * T * s / m.mass;
    B[3 * 2 + 0] = B[3 * 2 + 1] = -dt * s / m.mass;
    B[4 * 2 + 0] = B[4 * 2 + 1] = dt * c / m.mass;
    B[5 * 2 + 0] = -dt * m.arm / m.inertia;
    B[5 * 2 + 1] = dt * m.arm / m.inertia;
    const double xdot[6] = {x[3], x[4], x[5], -T * s / m.mass, T * c / m.mass - m.grav,
                            m.arm * (u[1] - u[0]) / m.inertia};
    for (int j = 0; j < 6; ++j) b[j] = x[j] + dt * xdot[j] - xn[j];
  }
  // input rows
  double* D = o.D + (size_t)k * nc * nu;
  for (int i = 0; i < nc * nu; ++i) D[i] = 0.0;
  for (int i = 0; i < nu; ++i) {
    double* c = Crow + (size_t)(no + i) * nx;
    for (int j = 0; j < nx; ++j) c[j] = 0.0;
    D[(size_t)(no + i) * nu + i] = 1.0;
    lb[no + i] = m.umin[i] - u[i];
    ub[no + i] = m.umax[i] - u[i];
  }
  // cost
  for (int j = 0; j < nx; ++j) {
    double s = 0.0;
    for (int t = 0; t < nx; ++t) s += m.Q[j * nx + t] * (x[t] - m.xref[(size_t)k * nx + t]);
    o.q[(size_t)k * nx + j] = s;
    for (int t = 0; t < nx; ++t) o.Q[((size_t)k * nx + j) * nx + t] = m.Q[j * nx + t];
  }
  for (int j = 0; j < nu; ++j) {
    double s = 0.0;
    for (int t = 0; t < nu; ++t) s += m.R[j * nu + t] * (u[t] - m.uref[(size_t)k * nu + t]);
    o.r[(size_t)k * nu + j] = s;
    for (int t = 0; t < nu; ++t) o.R[((size_t)k * nu + j) * nu + t] = m.R[j * nu + t];
  }
  for (int i = 0; i < nu * nx; ++i) o.S[(size_t)k * nu * nx + i] = 0.0;
}

int launch_linearize(const ModelDev& m, const double* X, const double* U, const LinOut& o, hipStream_t st) {
  const int n = m.N + 1, bs = 64;
  k_linearize<<<(n + bs - 1) / bs, bs, 0, st>>>(m, X, U, o);
  return hipGetLastError() == hipSuccess ? GSLS_OK : GSLS_ERR_HIP;
}

}  // namespace gsls
