// Internal declarations of the gfx950 ADMM / associative-scan QP solver.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <vector>

#include "../../include/gsls.h"

namespace gsls {

// Device copies of one LTV-QP in the working precision T (row-major, the
// layout of the C ABI).
template <typename T>
struct DevProblem {
  int N, nx, nu, nc, nf, m;
  T *A, *B, *b, *Q, *R, *S, *q, *r, *C, *D, *CN;
  T *G;              // [N][nc][nx+nu]  stage constraint map [C | D]
};

// Factor-epoch outputs (rho fixed) consumed by the ADMM iteration kernel.
template <typename T>
struct DevFactor {
  T *F;              // [N][nx+nu][nx+nu]  [[Abar, B], [K, I]] with Abar = A + B K
  T *Gam;            // [N][nu][nu]   (R_hat + B^T P_{k+1} B)^{-1}
  T *ev;             // [N][nx]       Abar^T P_{k+1} b
  T *fv;             // [N][nu]       B^T P_{k+1} b
  T *Phi;            // [nlev][P][nx][nx] chunk transfer maps (see iteration kernel)
};

// Scratch of the factor epoch.
template <typename T>
struct DevEpochWork {
  T *eP, *eA, *eC;          // [N+1][nx][nx] scan elements (P~, A~, C~)
  T *Qh, *Rh, *Sh;          // [N+1][nx][nx], [N][nu][nu], [N][nu][nx]
  T *fP, *fA, *fC;          // [Pe][nx][nx] chunk folds / suffix levels (ping)
  T *gP, *gA, *gC;          // [Pe][nx][nx] suffix levels (pong)
  T *Pend;                  // [Pe][nx][nx] P at each chunk's right end
  T *scratch;               // [max(Pe,Pi)][8][slot] per-workgroup scratch
  size_t slot;              // max(nx, nu)^2
  int* status;              // [1] 0 ok, 1 not positive definite
};

// Per-launch control block shared by the iteration kernel and the host.
struct IterCtl {
  int32_t it;          // iterations completed (cumulative)
  int32_t status;      // 0 running, 1 solved, 2 max_iter, 3 numerical, 4 rho change, 5 wait timeout
  double r_p, r_d;
  double rho_new;      // proposed rho when status == 4
  double r_dyn;        // max_k |x_{k+1} - A_k x_k - B_k u_k - b_k|_inf of the last iterate
};

struct IterParams {
  int P;               // workgroups (horizon chunks)
  int nlev;            // ceil(log2 P)
  double rho, tol;
  int it0, max_iter;   // iteration counter at launch, global limit
  int adaptive, sigma;
  double rho_min, rho_max, rho_tol;
  double hnorm;        // |(q, r)|_inf
  uint32_t stamp0;     // stamps of this launch start after stamp0
  int refresh;         // full evaluation at iteration counts divisible by refresh (0: none)
};

struct LLBufs {
  unsigned long long* bwd;   // [nlev+1][P][nx*W]  packed words, W = words per value
  unsigned long long* fwd;   // [nlev+1][P][nx*W]
  unsigned long long* red;   // [P][kRed*W]
  int* abort;                // set when any wait gives up
};
constexpr int kRed = 6;      // r_p, r_d, |v|, |z|, |H xi|, |G^T lambda|

template <typename T>
struct IterArgs {
  DevProblem<T> pb;
  DevFactor<T> fc;
  double *z, *y;             // [m] ADMM state (scaled dual y = lambda / rho), FP64
  const double *l, *u;       // [m] bounds, FP64
  double *X, *U;             // [N+1][nx], [N][nu] last primal iterate (FP64)
  const T* x0;               // [nx]
  LLBufs ll;
  IterParams ip;
  IterCtl* ctl;
  int Lmax;                  // max stages per chunk
  int resident;              // chunk operators kept in LDS
  unsigned long long* prof;  // optional [16] cycle counts per phase (workgroup 0)
};

template <typename T> int epoch_set_attributes();
template <typename T>
int launch_epoch(const DevProblem<T>& pb, const DevEpochWork<T>& ew, const DevFactor<T>& fc,
                 double rho, int Pe, int Pi, int nlev, hipStream_t st);
template <typename T> size_t admm_lds_bytes(int nx, int nu, int nc, int nf, int Lmax, int P, bool resident);
template <typename T> int launch_admm(const IterArgs<T>& args, hipStream_t st);
template <typename T>
int launch_rdyn(const DevProblem<T>& pb, const double* X, const double* U, IterCtl* ctl, hipStream_t st);

struct SlsArgs {
  int N, nx, nu, nc, nf, count;
  const float *A, *B, *G, *CN;     // problem (FP32): [N][nx][nx], [N][nx][nu], [N][nc][nx+nu], [nf][nx]
  const float *E;                  // [N][nx][nx]
  const float *tau;                // [count][N*N*nc + N*nf]
  const float *Qb, *Rb, *QbN;      // [nx][nx], [nu][nu], [nx][nx]
  int rownorm;                     // 2 or 1
  int squared;                     // store squared row norms (beta of App. B) instead
  float* Kst;                      // [grid][N][nu][nx] per-workgroup gain store
  float* hj;                       // [count][N][N][nc]: row norms for (k, j), k > j
  float* hfj;                      // [count][N][nf]
  float *Phx, *Phu;                // optional Phi^x / Phi^u of instance 0 (packed as in gsls.h)
  unsigned* counter;               // work queue head
  int* status;                     // 1 if a Z_uu block was not positive definite
};
int sls_grid(int nx, int nu, int nc, int nf);
int launch_sls(const SlsArgs& args, int grid, hipStream_t st);
int launch_sls_sum(int N, int nc, int nf, int count, float wbound, const float* hj, const float* hfj, double* h,
                   double* hf, hipStream_t st);
int launch_sls_beta(const SlsArgs& args, hipStream_t st);
int launch_sls_tau(int N, int nc, int nf, const float* betaj, const float* betafj, const double* lam, double eps,
                   double* tau, hipStream_t st);

// One-wavefront solver of tiny problems (nx, nu <= 4, nc, nf <= 8, N <= 63):
// a whole solve in FP64 in one launch.
struct TinyOut {
  int32_t it, status, nupd, nfact;   // status: 1 solved, 2 max_iter, 3 numerical, 6 not positive definite
  double r_p, r_d, rho, r_dyn;
  unsigned long long t_factor, t_iter;   // 100 MHz counter ticks
  unsigned long long c_load, c_factor, c_iter;   // shader clock cycles: load, factors, iterations
};
struct TinyArgs {
  int N, nx, nu, nc, nf, nlev;       // nlev: smallest L with 2^L > N
  int box;                           // rows are [I 0; 0 I] per stage and I at the terminal stage (nf == nx)
  const double *A, *B, *b, *Q, *R, *S, *q, *r, *C, *D, *CN, *l, *u;   // FP64, layout of the C ABI
  double x0v[4];                     // initial state (first nx entries)
  int cold;                          // 1: start from z = y = 0 (z, y are not read)
  double *z, *y;                     // [m] in: start iterate (cold == 0), out: last iterate
  double *X, *U;                     // [N+1][nx], [N][nu]
  double rho0, tol, rho_min, rho_max, rho_tol, hnorm;
  int max_iter, adaptive, sigma;
  TinyOut* out;
};
bool tiny_fits(int N, int nx, int nu, int nc, int nf);
int launch_tiny(const TinyArgs& args, hipStream_t st);

// Settings check shared by the entry points; descriptor validation with a
// row limit of max_rows per stage (host descriptors only).
int check_settings(const gsls_settings* s);
int validate_host_desc(const gsls_qp_desc* desc, int max_rows);

}  // namespace gsls
