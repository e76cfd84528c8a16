// Batched solver state shared by the batched ADMM kernel (batch.hip) and the
// learned warm start (mlp.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/gsls.h"

namespace gsls {

struct BInst {
  int N, nx, nu, nc, nf, box, m;
  int park_at;                                             // solo iterations before a gang takes over
  long long ogw, ogm;                                      // gang exchange words / transfer maps
  long long oE, oQN, ob, oq, orr, oG, oCN, ox0;           // float pool: problem
  long long oPk, okff;                                     // float pool: stage packets, feed-forward k
  long long ol, ou, oz, oy, ov, owp, oX, oU;                // double pool
};

// Per-stage input of the factor epoch in the float pool, laid out as the
// epoch's LDS blocks so that it moves to LDS by linear DMA: [A_k | B_k]
// (nx rows) and the symmetric part of the stage cost [[Q_k, S_k^T], [S_k, R_k]]
// (nx + nu rows), both with the odd leading dimension ld = (nx + nu) | 1 and
// zero padding, each block a multiple of 4 floats.
struct EpLayout {
  int ld, AB, Z, stride;
};
__host__ __device__ inline EpLayout ep_layout(int nx, int nu) {
  EpLayout L;
  const int nxu = nx + nu;
  L.ld = nxu | 1;
  L.AB = 0;
  L.Z = (nx * L.ld + 3) & ~3;
  L.stride = L.Z + ((nxu * L.ld + 3) & ~3);
  return L;
}

struct BResult {
  int status, iterations, rho_updates, factorizations, restarted;
  double r_p, r_d, rho;
  long long t_epoch, t_iter;   // device clock ticks (100 MHz real-time counter)
  double r_dyn;                // dynamics residual of the returned iterate
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
  int refresh;                 // full evaluation at iteration counts divisible by refresh (0: none)
  double rho_min, rho_max, rho_tol;
  BResult* res;                // [count]
  int* warm;                   // [count] 1: start from the given z, y
  int warm_budget;             // > 0: a warm start that has not converged after
                               // this many iterations restarts cold
  double rho_cold;             // rho of such a cold restart
  unsigned long long* prof;    // [16] phase clock counters, or null
  // gangs (continuation of instances over several workgroups)
  int gang;                    // workgroups per gang (<= 1: no gangs)
  struct BSync* sync;          // launch counters (cleared by the prologue)
  int* cont_list;              // [count] instances handed to gangs: priority list from the front, the other from the back
  unsigned* join;              // [count] gang join counters
  struct BPark* park;          // [count] control state at hand-over
  unsigned long long* gwords;  // exchange words (per instance at BInst::ogw)
  float* gmaps;                // transfer maps (per instance at BInst::ogm)
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
  BatchArgs* d_args = nullptr;    // kernel arguments (the graph keeps this pointer)
  int grid = 0;
  // gang schedule: workgroups per gang and the solo work (as a share of one
  // workgroup's share of an estimated batch) after which an instance is handed over
  int gang = 0;
  double park_share = 0.0;
  void* d_sync = nullptr;
  int* d_cont = nullptr;
  unsigned* d_join = nullptr;
  void* d_park = nullptr;
  unsigned long long* d_gwords = nullptr;
  float* d_gmaps = nullptr;
  // feature rows of the learned warm start: one per stage k = 0..N of every
  // instance, instance c owning rows row_off[c] .. row_off[c+1]-1
  unsigned long long* d_prof = nullptr;   // phase counters when profiling is on
  std::vector<int> row_off;
  int* d_row_inst = nullptr;   // [rows] owning instance
  int* d_row_off = nullptr;    // [count + 1]
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  double graph_key[4] = {-1, -1, -1, -1};   // (tol, warm budget, profiling, schedule) of the captured graph
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ~BatchSolver() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    for (void* p : {(void*)fp, (void*)dp, (void*)d_inst, (void*)d_order, (void*)d_rho, (void*)d_warm,
                    (void*)d_res, (void*)d_row_inst, (void*)d_row_off, (void*)d_prof, (void*)d_args,
                    d_sync, (void*)d_cont, (void*)d_join, d_park, (void*)d_gwords, (void*)d_gmaps})
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
// Sets the gang schedule (gang <= 1: every instance on one workgroup) and the
// per-instance hand-over points.
int batch_set_schedule(BatchSolver* B, int gang, double park_share);

}  // namespace gsls

// C-ABI handle of a batch.
struct gsls_batch {
  gsls::BatchSolver s;
  std::vector<double> rho_final;
};
