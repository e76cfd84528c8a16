// Batched solver state shared by the batched ADMM kernel (batch.hip) and the
// learned warm start (mlp.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/gsls.h"

namespace gsls {

struct BInst {
  int N, nx, nu, nc, nf, box, m;
  long long oA, oB, ob, oQ, oR, oS, oq, orr, oG, oCN, ox0;  // float pool: problem
  long long oPk, okff;                                     // float pool: stage packets, feed-forward k
  long long ol, ou, oz, oy, ov, owp, oX, oU;                // double pool
};

struct BResult {
  int status, iterations, rho_updates, factorizations, restarted;
  double r_p, r_d, rho;
  long long t_epoch, t_iter;   // device clock ticks (100 MHz real-time counter)
};

struct BatchArgs {
  const BInst* inst;
  const int* order;            // instance order (largest first)
  int count;
  float* fp;                   // float pool
  double* dp;                  // double pool
  const double* rho0;          // [count]
  double tol;
  int max_iter, adaptive, sigma;
  double rho_min, rho_max, rho_tol;
  BResult* res;                // [count]
  unsigned* counter;
  int* warm;                   // [count] 1: start from the given z, y
  int warm_budget;             // > 0: a warm start that has not converged after
                               // this many iterations restarts cold
  double rho_cold;             // rho of such a cold restart
  unsigned long long* prof;    // [16] phase clock counters, or null
};

struct BatchSolver {
  hipStream_t stream = nullptr;
  gsls_settings st;
  int count = 0;
  std::vector<BInst> inst;
  std::vector<int> order;
  std::vector<int> nx_of;
  size_t nfp = 0, ndp = 0, lds = 0;
  float* fp = nullptr;
  double* dp = nullptr;
  BInst* d_inst = nullptr;
  int* d_order = nullptr;
  double* d_rho = nullptr;
  int* d_warm = nullptr;
  BResult* d_res = nullptr;
  unsigned* d_counter = nullptr;
  BatchArgs* d_args = nullptr;    // kernel arguments (the graph keeps this pointer)
  int grid = 0;
  // feature rows of the learned warm start: one per stage k = 0..N of every
  // instance, instance c owning rows row_off[c] .. row_off[c+1]-1
  unsigned long long* d_prof = nullptr;   // phase counters when profiling is on
  std::vector<int> row_off;
  int* d_row_inst = nullptr;   // [rows] owning instance
  int* d_row_off = nullptr;    // [count + 1]
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  double graph_key[3] = {-1, -1, -1};   // (tol, warm budget, profiling) of the captured graph
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ~BatchSolver() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    for (void* p : {(void*)fp, (void*)dp, (void*)d_inst, (void*)d_order, (void*)d_rho, (void*)d_warm,
                    (void*)d_res, (void*)d_counter, (void*)d_row_inst, (void*)d_row_off, (void*)d_prof,
                    (void*)d_args})
      if (p) (void)hipFree(p);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
};

// Set-up, solve and read-back of a batch (batch.hip).
int batch_setup(const gsls_qp_desc* descs, int count, const gsls_settings* s, hipStream_t stream, BatchSolver* B);
int batch_solve(BatchSolver* B, const double* const* x0, const double* rho, double tol, const double* const* z0,
                const double* const* y0, gsls_result* out, double* ms);
int batch_get(BatchSolver* B, int idx, double* X, double* U, double* z, double* lam, double rho_final);
// Uploads the instances' initial states (FP32 copies in the float pool).
int batch_upload_x0(BatchSolver* B, const double* const* x0);
// Launches the captured solve graph with the start (rho, warm flags, z, y)
// already in device memory, waits, and fills out / ms.
int batch_run(BatchSolver* B, double tol, int warm_budget, gsls_result* out, double* ms);

}  // namespace gsls

// C-ABI handle of a batch.
struct gsls_batch {
  gsls::BatchSolver s;
  std::vector<double> rho_final;
};
