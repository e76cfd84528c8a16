/*
 * FP64 CPU oracle for the stage-structured ADMM QP solver and the SLS
 * controller synthesis of GPU-SLS (Fang & Chou, "Safe Large-Scale Robust
 * Nonlinear MPC in Milliseconds via Reachability-Constrained System Level
 * Synthesis on the GPU").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain, sequential
 * reference that the GPU path is checked against and the CPU baseline that the
 * benchmark times.  Nothing in the product library links or calls it; it
 * shares no code, header or table with the GPU path.
 *
 * Everything is double precision, row-major, single-threaded, with the
 * straightforward loop order of each definition.  No blocking, fusion or
 * reordering beyond what the definitions state.
 *
 * What it computes
 *  - oracle_qp_factor: the rho-dependent part of the ADMM primal update
 *    (Sec. IV-A): augmented costs of eq. (augmented_matrices) with the
 *    cross term read as S + rho D^T C (the printed C^T D has the wrong shape),
 *    then the textbook backward Riccati recursion of the LQR subproblem
 *    eq. (primal_update), whose P_i and gains K_i, Gamma_i are those of
 *    eq. (controller_cache).
 *  - oracle_qp_solve: ADMM of Sec. III-C applied to eq. (admm_qp):
 *    x-update = exact LQR solve (Riccati recursion), z-update = projection
 *    onto [l, u] (eq. after (augmented_linear); the paper's one-sided
 *    z <= f is the case l = -inf), scaled dual y = lambda / rho.  Penalty rho
 *    adapted every sigma iterations by the OSQP rule the paper adopts
 *    (Sec. IV-A, "Caching"): rho_new = rho * sqrt((r_p / max(|G xi|, |z|)) /
 *    (r_d / max(|H xi|, |G^T lambda|, |h|))), applied only when it moves rho
 *    by more than the factor rho_tol, clamped to [rho_min, rho_max], with y
 *    rescaled so lambda is unchanged.
 *    Residuals (the paper leaves them undefined): r_p = |G xi - z+|_inf and
 *    r_d = rho |G^T (z+ - z)|_inf; stop when both are <= tol.
 *  - oracle_sls_solve: the SLS controller problem eq. (fastsls_qp) solved by
 *    N independent Riccati recursions, eq. (backward_prop), and forward
 *    propagations, eq. (forward_prop), with the tau-weighted costs of
 *    eq. (sls_cost_matrices_tau); then the margins h_k, h^f of Sec. III-D.
 *    Column j's LQR runs over stages j+1..N-1 with terminal cost at N and
 *    starts from Phi^x_{j+1,j} = E_j.
 *  - oracle_sls_tau: the dual weights tau of App. B.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define IDX(i, j, ld) ((size_t)(i) * (size_t)(ld) + (size_t)(j))

/* ---------------------------------------------------------------- helpers */

/* C[m][n] = A[m][k] * B[k][n] */
static void mm(int m, int k, int n, const double* A, const double* B, double* C) {
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int t = 0; t < k; ++t) s += A[IDX(i, t, k)] * B[IDX(t, j, n)];
      C[IDX(i, j, n)] = s;
    }
}

/* C[m][n] = A[k][m]^T * B[k][n] */
static void mtm(int m, int k, int n, const double* A, const double* B, double* C) {
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int t = 0; t < k; ++t) s += A[IDX(t, i, m)] * B[IDX(t, j, n)];
      C[IDX(i, j, n)] = s;
    }
}

/* y[m] = A[m][n] x[n] */
static void mv(int m, int n, const double* A, const double* x, double* y) {
  for (int i = 0; i < m; ++i) {
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += A[IDX(i, j, n)] * x[j];
    y[i] = s;
  }
}

/* y[n] = A[m][n]^T x[m] */
static void mtv(int m, int n, const double* A, const double* x, double* y) {
  for (int j = 0; j < n; ++j) {
    double s = 0.0;
    for (int i = 0; i < m; ++i) s += A[IDX(i, j, n)] * x[i];
    y[j] = s;
  }
}

/* In-place lower Cholesky factor of the symmetric n x n matrix A (lower
 * triangle used).  Returns 0, or -1 when A is not positive definite. */
static int chol(int n, double* A) {
  for (int j = 0; j < n; ++j) {
    double d = A[IDX(j, j, n)];
    for (int t = 0; t < j; ++t) d -= A[IDX(j, t, n)] * A[IDX(j, t, n)];
    if (!(d > 0.0)) return -1;
    d = sqrt(d);
    A[IDX(j, j, n)] = d;
    for (int i = j + 1; i < n; ++i) {
      double s = A[IDX(i, j, n)];
      for (int t = 0; t < j; ++t) s -= A[IDX(i, t, n)] * A[IDX(j, t, n)];
      A[IDX(i, j, n)] = s / d;
    }
    for (int i = 0; i < j; ++i) A[IDX(i, j, n)] = 0.0;
  }
  return 0;
}

/* Solve (L L^T) X = Bm in place; Bm is n x k row-major. */
static void chol_solve(int n, int k, const double* L, double* Bm) {
  for (int c = 0; c < k; ++c) {
    for (int i = 0; i < n; ++i) {
      double s = Bm[IDX(i, c, k)];
      for (int t = 0; t < i; ++t) s -= L[IDX(i, t, n)] * Bm[IDX(t, c, k)];
      Bm[IDX(i, c, k)] = s / L[IDX(i, i, n)];
    }
    for (int i = n - 1; i >= 0; --i) {
      double s = Bm[IDX(i, c, k)];
      for (int t = i + 1; t < n; ++t) s -= L[IDX(t, i, n)] * Bm[IDX(t, c, k)];
      Bm[IDX(i, c, k)] = s / L[IDX(i, i, n)];
    }
  }
}

static double amax(size_t n, const double* x) {
  double m = 0.0;
  for (size_t i = 0; i < n; ++i) {
    double a = fabs(x[i]);
    if (a > m || a != a) m = a;
  }
  return m;
}

static void symmetrize(int n, double* P) {
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      double s = 0.5 * (P[IDX(i, j, n)] + P[IDX(j, i, n)]);
      P[IDX(i, j, n)] = s;
      P[IDX(j, i, n)] = s;
    }
}

/* ------------------------------------------------------ ADMM QP (Riccati) */

typedef struct {
  int N, nx, nu, nc, nf;
  const double *A, *B, *b, *Q, *R, *S, *q, *r, *C, *D, *CN, *l, *u;
} qp_t;

/* Factor for a fixed rho.  P: [N+1][nx][nx], K: [N][nu][nx],
 * L (Cholesky factor of H_i = Rhat_i + B_i^T P_{i+1} B_i): [N][nu][nu],
 * G (= Shat_i + B_i^T P_{i+1} A_i): [N][nu][nx].  Returns 0 or -1 (H not PD). */
static int factor(const qp_t* p, double rho, double* P, double* K, double* L, double* G) {
  const int N = p->N, nx = p->nx, nu = p->nu, nc = p->nc, nf = p->nf;
  double* CtC = malloc(sizeof(double) * nx * nx);
  double* PB = malloc(sizeof(double) * nx * (nu > 0 ? nu : 1));
  double* PA = malloc(sizeof(double) * nx * nx);
  double* tmp = malloc(sizeof(double) * nx * nx);
  double* Rh = malloc(sizeof(double) * (nu > 0 ? nu * nu : 1));
  double* Sh = malloc(sizeof(double) * (nu > 0 ? nu * nx : 1));
  double* DtD = malloc(sizeof(double) * (nu > 0 ? nu * nu : 1));
  double* DtC = malloc(sizeof(double) * (nu > 0 ? nu * nx : 1));
  int rc = 0;
  /* terminal: P_N = Q_N + rho C_N^T C_N */
  double* PN = P + (size_t)N * nx * nx;
  mtm(nx, nf, nx, p->CN, p->CN, CtC);
  for (int i = 0; i < nx * nx; ++i) PN[i] = p->Q[(size_t)N * nx * nx + i] + rho * CtC[i];
  for (int k = N - 1; k >= 0; --k) {
    const double* A = p->A + (size_t)k * nx * nx;
    const double* B = p->B + (size_t)k * nx * nu;
    const double* C = p->C + (size_t)k * nc * nx;
    const double* D = p->D + (size_t)k * nc * nu;
    const double* Pn = P + (size_t)(k + 1) * nx * nx;
    double* Pk = P + (size_t)k * nx * nx;
    double* Kk = K + (size_t)k * nu * nx;
    double* Lk = L + (size_t)k * nu * nu;
    double* Gk = G + (size_t)k * nu * nx;
    /* augmented costs */
    mtm(nx, nc, nx, C, C, CtC);
    mtm(nu, nc, nu, D, D, DtD);
    mtm(nu, nc, nx, D, C, DtC);
    for (int i = 0; i < nu * nu; ++i) Rh[i] = p->R[(size_t)k * nu * nu + i] + rho * DtD[i];
    for (int i = 0; i < nu * nx; ++i) Sh[i] = p->S[(size_t)k * nu * nx + i] + rho * DtC[i];
    /* H = Rhat + B^T P B, G = Shat + B^T P A */
    mm(nx, nx, nu, Pn, B, PB);
    mm(nx, nx, nx, Pn, A, PA);
    mtm(nu, nx, nu, B, PB, Lk);
    for (int i = 0; i < nu * nu; ++i) Lk[i] += Rh[i];
    mtm(nu, nx, nx, B, PA, Gk);
    for (int i = 0; i < nu * nx; ++i) Gk[i] += Sh[i];
    if (nu > 0 && chol(nu, Lk) != 0) { rc = -1; break; }
    /* K = -H^{-1} G */
    for (int i = 0; i < nu * nx; ++i) Kk[i] = -Gk[i];
    if (nu > 0) chol_solve(nu, nx, Lk, Kk);
    /* P_k = Qhat + A^T P A + G^T K */
    mtm(nx, nx, nx, A, PA, Pk);
    mtm(nx, nu, nx, Gk, Kk, tmp);
    for (int i = 0; i < nx * nx; ++i)
      Pk[i] += p->Q[(size_t)k * nx * nx + i] + rho * CtC[i] + tmp[i];
    symmetrize(nx, Pk);
  }
  free(CtC); free(PB); free(PA); free(tmp); free(Rh); free(Sh); free(DtD); free(DtC);
  return rc;
}

int oracle_qp_factor(int N, int nx, int nu, int nc, int nf,
                     const double* A, const double* B, const double* Q, const double* R,
                     const double* S, const double* C, const double* D, const double* CN,
                     double rho, double* P, double* K) {
  qp_t p = {N, nx, nu, nc, nf, A, B, NULL, Q, R, S, NULL, NULL, C, D, CN, NULL, NULL};
  double* L = malloc(sizeof(double) * (size_t)N * (nu > 0 ? nu * nu : 1));
  double* G = malloc(sizeof(double) * (size_t)N * (nu > 0 ? nu * nx : 1));
  int rc = factor(&p, rho, P, K, L, G);
  free(L); free(G);
  return rc;
}

/* Apply G (stage-block-diagonal constraint map) to (X, U): v [N*nc + nf]. */
static void gmap(const qp_t* p, const double* X, const double* U, double* v) {
  const int N = p->N, nx = p->nx, nu = p->nu, nc = p->nc;
  double* t = malloc(sizeof(double) * (nc > 0 ? nc : 1));
  for (int k = 0; k < N; ++k) {
    mv(nc, nx, p->C + (size_t)k * nc * nx, X + (size_t)k * nx, v + (size_t)k * nc);
    mv(nc, nu, p->D + (size_t)k * nc * nu, U + (size_t)k * nu, t);
    for (int i = 0; i < nc; ++i) v[(size_t)k * nc + i] += t[i];
  }
  mv(p->nf, nx, p->CN, X + (size_t)N * nx, v + (size_t)N * nc);
  free(t);
}

/* |G^T w|_inf for w [N*nc + nf] */
static double gtmax(const qp_t* p, const double* w) {
  const int N = p->N, nx = p->nx, nu = p->nu, nc = p->nc;
  double* tx = malloc(sizeof(double) * nx);
  double* tu = malloc(sizeof(double) * (nu > 0 ? nu : 1));
  double m = 0.0;
  for (int k = 0; k < N; ++k) {
    mtv(nc, nx, p->C + (size_t)k * nc * nx, w + (size_t)k * nc, tx);
    mtv(nc, nu, p->D + (size_t)k * nc * nu, w + (size_t)k * nc, tu);
    double a = amax(nx, tx), c = amax(nu, tu);
    if (a > m || a != a) m = a;
    if (c > m || c != c) m = c;
  }
  mtv(p->nf, nx, p->CN, w + (size_t)N * nc, tx);
  double a = amax(nx, tx);
  if (a > m || a != a) m = a;
  free(tx); free(tu);
  return m;
}

/* |H xi|_inf: stage blocks [[Q S^T],[S R]] (x_k, u_k) and Q_N x_N */
static double hmax(const qp_t* p, const double* X, const double* U) {
  const int N = p->N, nx = p->nx, nu = p->nu;
  double* tx = malloc(sizeof(double) * nx);
  double* tu = malloc(sizeof(double) * (nu > 0 ? nu : 1));
  double* t2 = malloc(sizeof(double) * nx);
  double m = 0.0;
  for (int k = 0; k <= N; ++k) {
    mv(nx, nx, p->Q + (size_t)k * nx * nx, X + (size_t)k * nx, tx);
    if (k < N) {
      mtv(nu, nx, p->S + (size_t)k * nu * nx, U + (size_t)k * nu, t2);
      for (int i = 0; i < nx; ++i) tx[i] += t2[i];
      mv(nu, nx, p->S + (size_t)k * nu * nx, X + (size_t)k * nx, tu);
      double* t3 = malloc(sizeof(double) * (nu > 0 ? nu : 1));
      mv(nu, nu, p->R + (size_t)k * nu * nu, U + (size_t)k * nu, t3);
      for (int i = 0; i < nu; ++i) tu[i] += t3[i];
      free(t3);
      double c = amax(nu, tu);
      if (c > m) m = c;
    }
    double a = amax(nx, tx);
    if (a > m) m = a;
  }
  free(tx); free(tu); free(t2);
  return m;
}

/*
 * ADMM on eq. (admm_qp).  Arrays as in the problem statement (row-major):
 *  A [N][nx][nx], B [N][nx][nu], b [N][nx], Q [N+1][nx][nx], R [N][nu][nu],
 *  S [N][nu][nx], q [N+1][nx], r [N][nu], C [N][nc][nx], D [N][nc][nu],
 *  CN [nf][nx], l, u [N*nc + nf], x0 [nx].
 *  z0, y0: warm-start iterate (both NULL: cold start z = y = 0).
 *  Outputs: X [N+1][nx], U [N][nu], z, y [N*nc+nf] (scaled dual, lambda = rho*y).
 *  info[0..7] = iterations, r_p, r_d, final rho, rho updates, status
 *  (1 solved, 2 max_iter, -4 not PD, -5 numerical), r_dyn, factorizations.
 */
int oracle_qp_solve(int N, int nx, int nu, int nc, int nf,
                    const double* A, const double* B, const double* b,
                    const double* Q, const double* R, const double* S,
                    const double* q, const double* r,
                    const double* C, const double* D, const double* CN,
                    const double* l, const double* u, const double* x0,
                    double rho0, double tol, int max_iter, int adaptive, int sigma,
                    double rho_min, double rho_max, double rho_tol,
                    const double* z0, const double* y0,
                    double* X, double* U, double* z, double* y, double* info) {
  qp_t p = {N, nx, nu, nc, nf, A, B, b, Q, R, S, q, r, C, D, CN, l, u};
  const size_t m = (size_t)N * nc + nf;
  double* P = malloc(sizeof(double) * (size_t)(N + 1) * nx * nx);
  double* K = malloc(sizeof(double) * (size_t)N * (nu > 0 ? nu * nx : 1));
  double* L = malloc(sizeof(double) * (size_t)N * (nu > 0 ? nu * nu : 1));
  double* G = malloc(sizeof(double) * (size_t)N * (nu > 0 ? nu * nx : 1));
  double* kff = malloc(sizeof(double) * (size_t)N * (nu > 0 ? nu : 1));
  double* w = malloc(sizeof(double) * (m > 0 ? m : 1));
  double* v = malloc(sizeof(double) * (m > 0 ? m : 1));
  double* zn = malloc(sizeof(double) * (m > 0 ? m : 1));
  double* dz = malloc(sizeof(double) * (m > 0 ? m : 1));
  double* pn = malloc(sizeof(double) * nx);
  double* pk = malloc(sizeof(double) * nx);
  double* s = malloc(sizeof(double) * nx);
  double* tx = malloc(sizeof(double) * nx);
  double* tx2 = malloc(sizeof(double) * nx);
  double* tu = malloc(sizeof(double) * (nu > 0 ? nu : 1));
  double* g = malloc(sizeof(double) * (nu > 0 ? nu : 1));
  double rho = rho0;
  int status = 2, it = 0, nupd = 0, nfact = 0;
  double rp = INFINITY, rd = INFINITY;

  for (size_t i = 0; i < m; ++i) {
    z[i] = z0 ? z0[i] : 0.0;
    y[i] = y0 ? y0[i] : 0.0;
  }
  double hnorm = fmax(amax((size_t)(N + 1) * nx, q), amax((size_t)N * nu, r));

  if (factor(&p, rho, P, K, L, G) != 0) { status = -4; goto done; }
  nfact = 1;
  for (it = 1; it <= max_iter; ++it) {
    /* linear terms, eq. (augmented_linear), with w = y - z */
    for (size_t i = 0; i < m; ++i) w[i] = y[i] - z[i];
    /* backward pass: p_N = qhat_N */
    mtv(nf, nx, CN, w + (size_t)N * nc, tx);
    for (int i = 0; i < nx; ++i) pn[i] = q[(size_t)N * nx + i] + rho * tx[i];
    for (int k = N - 1; k >= 0; --k) {
      const double* Ak = A + (size_t)k * nx * nx;
      const double* Bk = B + (size_t)k * nx * nu;
      const double* Pn = P + (size_t)(k + 1) * nx * nx;
      /* s = p_{k+1} + P_{k+1} b_k */
      mv(nx, nx, Pn, b + (size_t)k * nx, s);
      for (int i = 0; i < nx; ++i) s[i] += pn[i];
      /* rhat_k, qhat_k */
      mtv(nc, nu, D + (size_t)k * nc * nu, w + (size_t)k * nc, tu);
      mtv(nc, nx, C + (size_t)k * nc * nx, w + (size_t)k * nc, tx);
      /* g = rhat + B^T s;  k_k = -H^{-1} g */
      mtv(nx, nu, Bk, s, g);
      for (int i = 0; i < nu; ++i) g[i] += r[(size_t)k * nu + i] + rho * tu[i];
      double* kk = kff + (size_t)k * nu;
      for (int i = 0; i < nu; ++i) kk[i] = -g[i];
      if (nu > 0) chol_solve(nu, 1, L + (size_t)k * nu * nu, kk);
      /* p_k = qhat + A^T s + G^T k */
      mtv(nx, nx, Ak, s, pk);
      mtv(nu, nx, G + (size_t)k * nu * nx, kk, tx2);
      for (int i = 0; i < nx; ++i) pk[i] += q[(size_t)k * nx + i] + rho * tx[i] + tx2[i];
      memcpy(pn, pk, sizeof(double) * nx);
    }
    /* forward roll-out from x0 */
    memcpy(X, x0, sizeof(double) * nx);
    for (int k = 0; k < N; ++k) {
      double* xk = X + (size_t)k * nx;
      double* uk = U + (size_t)k * nu;
      mv(nu, nx, K + (size_t)k * nu * nx, xk, uk);
      for (int i = 0; i < nu; ++i) uk[i] += kff[(size_t)k * nu + i];
      double* xn = X + (size_t)(k + 1) * nx;
      mv(nx, nx, A + (size_t)k * nx * nx, xk, xn);
      mv(nx, nu, B + (size_t)k * nx * nu, uk, tx);
      for (int i = 0; i < nx; ++i) xn[i] += tx[i] + b[(size_t)k * nx + i];
    }
    /* z- and dual update */
    gmap(&p, X, U, v);
    rp = 0.0;
    for (size_t i = 0; i < m; ++i) {
      double t = v[i] + y[i];
      double zz = t < l[i] ? l[i] : (t > u[i] ? u[i] : t);
      zn[i] = zz;
      dz[i] = zz - z[i];
      y[i] = y[i] + v[i] - zz;
      double a = fabs(v[i] - zz);
      if (a > rp || a != a) rp = a;
    }
    rd = rho * gtmax(&p, dz);
    memcpy(z, zn, sizeof(double) * m);
    if (!(rp == rp) || !(rd == rd) || isinf(rp) || isinf(rd)) { status = -5; break; }
    if (rp <= tol && rd <= tol) { status = 1; break; }
    if (it == max_iter) { status = 2; break; }
    if (adaptive && sigma > 0 && it % sigma == 0) {
      double pscale = fmax(amax(m, v), amax(m, z));
      for (size_t i = 0; i < m; ++i) w[i] = rho * y[i];
      double dscale = fmax(fmax(hmax(&p, X, U), gtmax(&p, w)), hnorm);
      const double eps = 1e-10;
      double ratio = (rp / (pscale + eps)) / (rd / (dscale + eps) + eps);
      double rn = rho * sqrt(ratio);
      if (rn < rho_min) rn = rho_min;
      if (rn > rho_max) rn = rho_max;
      if (rn > rho * rho_tol || rn < rho / rho_tol) {
        for (size_t i = 0; i < m; ++i) y[i] *= rho / rn;
        rho = rn;
        ++nupd;
        if (factor(&p, rho, P, K, L, G) != 0) { status = -4; break; }
        ++nfact;
      }
    }
  }
  if (it > max_iter) it = max_iter;
done:;
  /* dynamics residual of the returned trajectory */
  double rdyn = 0.0;
  if (status != -4) {
    for (int k = 0; k < N; ++k) {
      mv(nx, nx, A + (size_t)k * nx * nx, X + (size_t)k * nx, tx);
      mv(nx, nu, B + (size_t)k * nx * nu, U + (size_t)k * nu, tx2);
      for (int i = 0; i < nx; ++i) {
        double e = fabs(X[(size_t)(k + 1) * nx + i] - tx[i] - tx2[i] - b[(size_t)k * nx + i]);
        if (e > rdyn) rdyn = e;
      }
    }
  }
  info[0] = it; info[1] = rp; info[2] = rd; info[3] = rho; info[4] = nupd;
  info[5] = status; info[6] = rdyn; info[7] = nfact;
  free(P); free(K); free(L); free(G); free(kff); free(w); free(v); free(zn); free(dz);
  free(pn); free(pk); free(s); free(tx); free(tx2); free(tu); free(g);
  return status;
}

/*
 * Batch driver of the CPU baseline: `count` independent instances solved by
 * oracle_qp_solve from a cold start, in parallel over the host cores when
 * compiled with OpenMP (one instance per thread at a time, dynamic schedule;
 * each solve stays sequential).  dims[5c..5c+4] = N, nx, nu, nc, nf of
 * instance c; ptrs[14c..14c+13] = A, B, b, Q, R, S, q, r, C, D, CN, l, u, x0;
 * info[8c..8c+7] as for oracle_qp_solve.  The solutions are not returned.
 * Returns the number of threads that ran.
 */
#ifdef _OPENMP
#include <omp.h>
#endif
int oracle_qp_solve_many(int count, const int* dims, const double* const* ptrs, double rho0, double tol,
                         int max_iter, int adaptive, int sigma, double rho_min, double rho_max, double rho_tol,
                         double* info) {
  int threads = 1;
#ifdef _OPENMP
#pragma omp parallel
  {
#pragma omp single
    threads = omp_get_num_threads();
  }
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (int c = 0; c < count; ++c) {
    const int* d = dims + 5 * (size_t)c;
    const double* const* a = ptrs + 14 * (size_t)c;
    const int N = d[0], nx = d[1], nu = d[2], nc = d[3], nf = d[4];
    const size_t m = (size_t)N * nc + nf;
    double* X = malloc(sizeof(double) * (size_t)(N + 1) * nx);
    double* U = malloc(sizeof(double) * ((size_t)N * nu + 1));
    double* z = malloc(sizeof(double) * (m + 1));
    double* y = malloc(sizeof(double) * (m + 1));
    oracle_qp_solve(N, nx, nu, nc, nf, a[0], a[1], a[2], a[3], a[4], a[5], a[6], a[7], a[8], a[9], a[10], a[11],
                    a[12], a[13], rho0, tol, max_iter, adaptive, sigma, rho_min, rho_max, rho_tol, NULL, NULL, X, U,
                    z, y, info + 8 * (size_t)c);
    free(X); free(U); free(z); free(y);
  }
  return threads;
}

/* ------------------------------------------------------------------- SLS */

static size_t offx(int N, int j) { return (size_t)j * N - (size_t)j * (j - 1) / 2; }
static size_t offu(int N, int j) { return (size_t)j * (N - 1) - (size_t)j * (j - 1) / 2; }

/*
 * SLS controller synthesis, eq. (fastsls_qp), one column j at a time.
 *  A [N][nx][nx], B [N][nx][nu], C [N][nc][nx], D [N][nc][nu], CN [nf][nx],
 *  E [N][nx][nx]; tau = [N][N][nc] stage weights tau[k][j][.] (used for
 *  j < k <= N-1) followed by [N][nf] terminal weights tau_N[j][.].
 *  Qbar [nx][nx], Rbar [nu][nu], QbarN [nx][nx] (symmetric positive definite).
 *  Phi_x: column j holds blocks k = j+1..N (each nx x nx) at offset
 *  (j*N - j(j-1)/2) blocks; Phi_u: blocks k = j+1..N-1 (each nu x nx) at
 *  offset (j*(N-1) - j(j-1)/2) blocks.  Either may be NULL.
 *  h [N][nc], hf [nf]: margins with row norm `rownorm` (2 or 1) scaled by wbound.
 *  Kout (optional) [N][N][nu][nx]: gains K^{(j)}_k at [k][j].
 */
int oracle_sls_solve(int N, int nx, int nu, int nc, int nf,
                     const double* A, const double* B, const double* C, const double* D,
                     const double* CN, const double* E, const double* tau,
                     const double* Qbar, const double* Rbar, const double* QbarN,
                     int rownorm, double wbound,
                     double* Phi_x, double* Phi_u, double* h, double* hf, double* Kout) {
  double* P = malloc(sizeof(double) * nx * nx);
  double* Pn = malloc(sizeof(double) * nx * nx);
  double* Kc = malloc(sizeof(double) * (size_t)N * nu * nx);
  double* PA = malloc(sizeof(double) * nx * nx);
  double* PB = malloc(sizeof(double) * nx * nu);
  double* H = malloc(sizeof(double) * nu * nu);
  double* G = malloc(sizeof(double) * nu * nx);
  double* Qx = malloc(sizeof(double) * nx * nx);
  double* Qu = malloc(sizeof(double) * nu * nu);
  double* Qux = malloc(sizeof(double) * nu * nx);
  double* TC = malloc(sizeof(double) * (size_t)(nc > nf ? nc : nf) * nx);
  double* TD = malloc(sizeof(double) * (size_t)(nc > 0 ? nc : 1) * nu);
  double* tmp = malloc(sizeof(double) * nx * nx);
  double* Fx = malloc(sizeof(double) * nx * nx);
  double* Fxn = malloc(sizeof(double) * nx * nx);
  double* Fu = malloc(sizeof(double) * nu * nx);
  double* Acl = malloc(sizeof(double) * nx * nx);
  double* M = malloc(sizeof(double) * (size_t)(nc > nf ? nc : nf) * nx);
  double* M2 = malloc(sizeof(double) * (size_t)(nc > 0 ? nc : 1) * nx);
  int rc = 0;
  for (size_t i = 0; i < (size_t)N * nc; ++i) h[i] = 0.0;
  for (int i = 0; i < nf; ++i) hf[i] = 0.0;
  for (int j = 0; j < N && rc == 0; ++j) {
    /* terminal: P_N = C_N^T T_N C_N + Qbar_N */
    const double* tN = tau + (size_t)N * N * nc + (size_t)j * nf;
    for (int i = 0; i < nf; ++i)
      for (int c = 0; c < nx; ++c) TC[IDX(i, c, nx)] = tN[i] * CN[IDX(i, c, nx)];
    mtm(nx, nf, nx, CN, TC, P);
    for (int i = 0; i < nx * nx; ++i) P[i] += QbarN[i];
    /* backward Riccati over k = N-1..j+1 */
    for (int k = N - 1; k >= j + 1; --k) {
      const double* Ak = A + (size_t)k * nx * nx;
      const double* Bk = B + (size_t)k * nx * nu;
      const double* Ck = C + (size_t)k * nc * nx;
      const double* Dk = D + (size_t)k * nc * nu;
      const double* tk = tau + ((size_t)k * N + j) * nc;
      for (int i = 0; i < nc; ++i) {
        for (int c = 0; c < nx; ++c) TC[IDX(i, c, nx)] = tk[i] * Ck[IDX(i, c, nx)];
        for (int c = 0; c < nu; ++c) TD[IDX(i, c, nu)] = tk[i] * Dk[IDX(i, c, nu)];
      }
      mtm(nx, nc, nx, Ck, TC, Qx);
      for (int i = 0; i < nx * nx; ++i) Qx[i] += Qbar[i];
      mtm(nu, nc, nu, Dk, TD, Qu);
      for (int i = 0; i < nu * nu; ++i) Qu[i] += Rbar[i];
      mtm(nu, nc, nx, Dk, TC, Qux);
      mm(nx, nx, nx, P, Ak, PA);
      mm(nx, nx, nu, P, Bk, PB);
      mtm(nu, nx, nu, Bk, PB, H);
      for (int i = 0; i < nu * nu; ++i) H[i] += Qu[i];
      mtm(nu, nx, nx, Bk, PA, G);
      for (int i = 0; i < nu * nx; ++i) G[i] += Qux[i];
      if (chol(nu, H) != 0) { rc = -4; break; }
      double* Kk = Kc + (size_t)k * nu * nx;
      for (int i = 0; i < nu * nx; ++i) Kk[i] = -G[i];
      chol_solve(nu, nx, H, Kk);
      mtm(nx, nx, nx, Ak, PA, Pn);
      mtm(nx, nu, nx, G, Kk, tmp);
      for (int i = 0; i < nx * nx; ++i) Pn[i] += Qx[i] + tmp[i];
      symmetrize(nx, Pn);
      memcpy(P, Pn, sizeof(double) * nx * nx);
      if (Kout) memcpy(Kout + ((size_t)k * N + j) * nu * nx, Kk, sizeof(double) * nu * nx);
    }
    if (rc) break;
    /* forward propagation from Phi^x_{j+1,j} = E_j */
    memcpy(Fx, E + (size_t)j * nx * nx, sizeof(double) * nx * nx);
    for (int k = j + 1; k <= N; ++k) {
      if (Phi_x) memcpy(Phi_x + (offx(N, j) + (size_t)(k - j - 1)) * nx * nx, Fx, sizeof(double) * nx * nx);
      if (k == N) {
        mm(nf, nx, nx, CN, Fx, M);
        for (int i = 0; i < nf; ++i) {
          double s = 0.0;
          for (int c = 0; c < nx; ++c) {
            double a = M[IDX(i, c, nx)];
            s += rownorm == 1 ? fabs(a) : a * a;
          }
          hf[i] += wbound * (rownorm == 1 ? s : sqrt(s));
        }
        break;
      }
      const double* Kk = Kc + (size_t)k * nu * nx;
      mm(nu, nx, nx, Kk, Fx, Fu);
      if (Phi_u) memcpy(Phi_u + (offu(N, j) + (size_t)(k - j - 1)) * nu * nx, Fu, sizeof(double) * nu * nx);
      /* margins: rows of C_k Phi^x + D_k Phi^u */
      mm(nc, nx, nx, C + (size_t)k * nc * nx, Fx, M);
      mm(nc, nu, nx, D + (size_t)k * nc * nu, Fu, M2);
      for (int i = 0; i < nc; ++i) {
        double s = 0.0;
        for (int c = 0; c < nx; ++c) {
          double a = M[IDX(i, c, nx)] + M2[IDX(i, c, nx)];
          s += rownorm == 1 ? fabs(a) : a * a;
        }
        h[(size_t)k * nc + i] += wbound * (rownorm == 1 ? s : sqrt(s));
      }
      /* Phi^x_{k+1} = A_k Phi^x_k + B_k Phi^u_k */
      mm(nx, nx, nx, A + (size_t)k * nx * nx, Fx, Fxn);
      mm(nx, nu, nx, B + (size_t)k * nx * nu, Fu, tmp);
      for (int i = 0; i < nx * nx; ++i) Fx[i] = Fxn[i] + tmp[i];
    }
  }
  free(P); free(Pn); free(Kc); free(PA); free(PB); free(H); free(G); free(Qx); free(Qu);
  free(Qux); free(TC); free(TD); free(tmp); free(Fx); free(Fxn); free(Fu); free(Acl);
  free(M); free(M2);
  return rc;
}

/*
 * Dual weights of App. B: beta_{k,j} = |C_k Phi^x_{k,j} + D_k Phi^u_{k,j}|^2 per
 * row, tau_{k,j} = |lambda_k| / sqrt(beta_{k,j} + eps) for j < k <= N-1, and
 * the terminal analogue with C_N.  |lambda| is used so that a row whose lower
 * bound is active (lambda < 0) weighs the same as one whose upper bound is.
 * Layout of tau as in oracle_sls_solve; entries with k <= j are set to 0.
 */
void oracle_sls_tau(int N, int nx, int nu, int nc, int nf, const double* C, const double* D,
                    const double* CN, const double* lambda, const double* Phi_x,
                    const double* Phi_u, double eps, double* tau) {
  double* M = malloc(sizeof(double) * (size_t)(nc > nf ? nc : nf) * nx + 8);
  double* M2 = malloc(sizeof(double) * (size_t)(nc > 0 ? nc : 1) * nx + 8);
  for (size_t i = 0; i < (size_t)N * N * nc + (size_t)N * nf; ++i) tau[i] = 0.0;
  for (int j = 0; j < N; ++j) {
    for (int k = j + 1; k <= N; ++k) {
      const double* Fx = Phi_x + (offx(N, j) + (size_t)(k - j - 1)) * nx * nx;
      if (k == N) {
        mm(nf, nx, nx, CN, Fx, M);
        for (int i = 0; i < nf; ++i) {
          double s = 0.0;
          for (int c = 0; c < nx; ++c) s += M[IDX(i, c, nx)] * M[IDX(i, c, nx)];
          tau[(size_t)N * N * nc + (size_t)j * nf + i] = fabs(lambda[(size_t)N * nc + i]) / sqrt(s + eps);
        }
      } else {
        const double* Fu = Phi_u + (offu(N, j) + (size_t)(k - j - 1)) * nu * nx;
        mm(nc, nx, nx, C + (size_t)k * nc * nx, Fx, M);
        mm(nc, nu, nx, D + (size_t)k * nc * nu, Fu, M2);
        for (int i = 0; i < nc; ++i) {
          double s = 0.0;
          for (int c = 0; c < nx; ++c) {
            double a = M[IDX(i, c, nx)] + M2[IDX(i, c, nx)];
            s += a * a;
          }
          tau[((size_t)k * N + j) * nc + i] = fabs(lambda[(size_t)k * nc + i]) / sqrt(s + eps);
        }
      }
    }
  }
  free(M); free(M2);
}
