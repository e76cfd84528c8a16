// System level synthesis on the MI355X (Sec. III-D and IV-B of the paper).
//
// For every instance and disturbance column j the controller problem
// eq. (fastsls_qp) is an LQR over stages j+1..N-1 with terminal cost at N,
// whose tau-weighted costs are the blocks of Q^T Q of
// eq. (sls_cost_matrices_tau):
//   [[Qx, Qxu], [Qux, Qu]] = blkdiag(Qbar, Rbar) + G_k^T diag(tau_{k,j}) G_k,
// with G_k = [C_k | D_k];  terminal Qx_N = Qbar_N + C_N^T diag(tau_{N,j}) C_N.
// The batch supplies count x N independent columns, enough to fill the GPU,
// so each column is scanned by one workgroup as a single chunk: the chunk
// fix-up of the factor scan, i.e. the Riccati recursion eq. (backward_prop),
//   Z = [A | B]^T P [A | B] + blkdiag(Qbar, Rbar) + G^T diag(tau) G,
//   K = -Z_uu^{-1} Z_ux (Z_uu inverted in FP64),   P <- Z_xx + Z_ux^T K,
// followed by the forward propagation eq. (forward_prop) from Phi^x_{j+1,j} = E_j:
//   Phi^u_k = K_k Phi^x_k,   Phi^x_{k+1} = [A | B] [Phi^x_k; Phi^u_k],
// and the row norms of G_k [Phi^x_k; Phi^u_k] (C_N Phi^x_N at the terminal
// stage), whose sum over j < k is the margin h_k (Sec. III-D).
//
// The kernel is persistent: a grid sized to the machine pulls (instance,
// column) items from a device counter, longest columns first.  All products
// run on the matrix cores (FP32 MFMA) with operands in LDS.
#include <algorithm>

#include "dev_common.hpp"
#include "solver.hpp"

namespace gsls {

__host__ __device__ inline int sls_odd(int x) { return x | 1; }

// Row slots per wave and pass of the block copies (16 loads in flight per
// thread: rows wave + 4q of the pass, columns lane and lane + 64).
constexpr int kSlsRowSlots = 8;

struct SlsLayout {
  int ldP, ldW, ldZ, ldAB, ldG, ldY;
  size_t P, W, Z, AB, G, Y, M, T, aug, bytes;
};
__host__ __device__ inline SlsLayout sls_layout(int nx, int nu, int nc, int nf) {
  SlsLayout L;
  const int nxu = nx + nu;
  const int rows = nc > nf ? nc : nf;
  L.ldP = sls_odd(nx); L.ldW = sls_odd(nxu); L.ldZ = sls_odd(nxu); L.ldAB = sls_odd(nxu);
  L.ldG = sls_odd(nxu); L.ldY = sls_odd(nx);
  size_t o = 0;
  L.P = o; o += (size_t)nx * L.ldP;                      // P, later Phi^x
  L.W = o; o += (size_t)(nx > rows ? nx : rows) * L.ldW;  // P [A|B], diag(tau) G, G Y
  L.Z = o; o += (size_t)nxu * L.ldZ;                     // Z, later Phi^x_{k+1}
  L.AB = o; o += (size_t)nx * L.ldAB;                    // [A_k | B_k]
  L.G = o; o += (size_t)rows * L.ldG;                    // G_k (or C_N)
  L.Y = o; o += (size_t)nxu * L.ldY;                     // [Phi^x; Phi^u]
  L.M = o; o += 0;
  L.T = o; o += (size_t)(rows + 3) & ~(size_t)3;         // tau column / row norms
  o = (o + 3) & ~(size_t)3;
  L.aug = o * 4;                                         // bytes: FP64 [Z_uu | Z_ux]
  L.bytes = L.aug + sizeof(double) * ((size_t)nu * (nu + nx) + 2 * nu) + 2 * sizeof(int) * nu + 64;
  return L;
}

__global__ void __launch_bounds__(kWG) k_sls(SlsArgs a) {
  extern __shared__ __align__(16) char lds_generic[];
  LDS char* base = (LDS char*)lds_generic;
  const int N = a.N, nx = a.nx, nu = a.nu, nc = a.nc, nf = a.nf, nxu = nx + nu;
  const SlsLayout lay = sls_layout(nx, nu, nc, nf);
  LDS float* F = (LDS float*)base;
  LDS float* P = F + lay.P;
  LDS float* W = F + lay.W;
  LDS float* Z = F + lay.Z;
  LDS float* AB = F + lay.AB;
  LDS float* G = F + lay.G;
  LDS float* Y = F + lay.Y;
  LDS float* Tv = F + lay.T;
  LDS double* aug = (LDS double*)(base + lay.aug);
  LDS double* dg = aug + nu * (nu + nx);
  LDS int* perm = (LDS int*)(dg + 2 * nu);
  LDS int* used = perm + nu;
  __shared__ unsigned s_item;
  float* Kst = a.Kst + (size_t)blockIdx.x * N * nu * nx;
  const size_t tau_stride = (size_t)N * N * nc + (size_t)N * nf;
  const unsigned total = (unsigned)a.count * N;

  // Block copies global -> LDS in passes of 32 rows, each issuing all of a
  // thread's loads before its first LDS store (one memory latency per pass).
  auto load_block = [&](int m, int n, auto src, LDS float* dst, int ldd) {
    for (int q0 = 0; 4 * q0 < m; q0 += kSlsRowSlots) {
      float v[kSlsRowSlots][2];
#pragma unroll
      for (int q = 0; q < kSlsRowSlots; ++q)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const int r = wave() + 4 * (q0 + q), c = lane() + 64 * b;
          v[q][b] = (r < m && c < n) ? src(r, c) : 0.f;
        }
#pragma unroll
      for (int q = 0; q < kSlsRowSlots; ++q)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const int r = wave() + 4 * (q0 + q), c = lane() + 64 * b;
          if (r < m && c < n) dst[r * ldd + c] = v[q][b];
        }
    }
  };
  auto load_stage = [&](int k) {   // AB <- [A_k | B_k], G <- G_k
    const float* Ak = a.A + (size_t)k * nx * nx;
    const float* Bk = a.B + (size_t)k * nx * nu;
    const float* Gk = a.G + (size_t)k * nc * nxu;
    load_block(nx, nxu, [&](int r, int c) { return c < nx ? Ak[(size_t)r * nx + c] : Bk[(size_t)r * nu + (c - nx)]; },
               AB, lay.ldAB);
    load_block(nc, nxu, [&](int r, int c) { return Gk[(size_t)r * nxu + c]; }, G, lay.ldG);
  };

  while (true) {
    if (tid() == 0) s_item = atomicAdd(a.counter, 1u);
    __syncthreads();
    const unsigned item = s_item;
    __syncthreads();
    if (item >= total) break;
    // longest columns first: items are ordered by column, then instance
    const int j = (int)(item / a.count), inst = (int)(item % a.count);
    const float* tau = a.tau + (size_t)inst * tau_stride;
    // ------------------------------------------- terminal: P = Qbar_N + C_N^T T C_N
    for (int r = wave(); r < nx; r += 4)
      for (int c = lane(); c < nx; c += 64) P[r * lay.ldP + c] = a.QbN[(size_t)r * nx + c];
    if (nf > 0) {
      const float* tN = tau + (size_t)N * N * nc + (size_t)j * nf;
      for (int r = wave(); r < nf; r += 4)
        for (int c = lane(); c < nx; c += 64) {
          const float cv = a.CN[(size_t)r * nx + c];
          G[r * lay.ldG + c] = cv;
          W[r * lay.ldW + c] = tN[r] * cv;
        }
      __syncthreads();
      wg_mm_f32(nx, nx, nf, 1.f, G, lay.ldG, true, W, lay.ldW, false, 1.f, P, lay.ldP);
    }
    __syncthreads();
    // ------------------------------------------------ backward Riccati
    for (int k = N - 1; k >= j + 1; --k) {
      load_stage(k);
      const float* tk = tau + ((size_t)k * N + j) * nc;
      for (int r = tid(); r < nc; r += kWG) Tv[r] = tk[r];
      __syncthreads();
      // W = P [A | B];  Z = [A | B]^T W + blkdiag(Qbar, Rbar)
      wg_mm_f32(nx, nxu, nx, 1.f, P, lay.ldP, false, AB, lay.ldAB, false, 0.f, W, lay.ldW);
      load_block(nxu, nxu, [&](int r, int c) {
        if (r < nx && c < nx) return a.Qb[(size_t)r * nx + c];
        if (r >= nx && c >= nx) return a.Rb[(size_t)(r - nx) * nu + (c - nx)];
        return 0.f;
      }, Z, lay.ldZ);
      __syncthreads();
      wg_mm_f32(nxu, nxu, nx, 1.f, AB, lay.ldAB, true, W, lay.ldW, false, 1.f, Z, lay.ldZ);
      // Z += G^T diag(tau) G
      for (int r = wave(); r < nc; r += 4)
        for (int c = lane(); c < nxu; c += 64) W[r * lay.ldW + c] = Tv[r] * G[r * lay.ldG + c];
      __syncthreads();
      wg_mm_f32(nxu, nxu, nc, 1.f, G, lay.ldG, true, W, lay.ldW, false, 1.f, Z, lay.ldZ);
      // K = -Z_uu^{-1} Z_ux by FP64 elimination of [Z_uu | Z_ux] (Z_uu symmetric
      // positive definite).  Solving for K directly keeps P = Z_xx + Z_ux^T K
      // accurate when the tau-weighted terms are large: a K formed from a
      // rounded inverse carries cond(Z_uu) times its rounding into P.
      const int lda = nu + nx;
      for (int r = wave(); r < nu; r += 4)
        for (int c = lane(); c < lda; c += 64) {
          double v;
          if (c < nu) {
            v = 0.5 * ((double)Z[(nx + r) * lay.ldZ + nx + c] + (double)Z[(nx + c) * lay.ldZ + nx + r]);
          } else {
            v = (double)Z[(nx + r) * lay.ldZ + (c - nu)];
          }
          aug[r * lda + c] = v;
        }
      __syncthreads();
      if (!wg_gj_eliminate(nu, lda, aug, false, perm, used, dg)) {
        if (tid() == 0) atomicMax(a.status, 1);
        break;
      }
      wg_gj_extract<float>(nu, lda, aug, perm, dg, 0, nx, -1.0, (float*)Y, lay.ldY);
      // K (in Y) and its copy in this workgroup's gain store for the forward pass
      float* Kk = Kst + (size_t)k * nu * nx;
      for (int r = wave(); r < nu; r += 4)
        for (int c = lane(); c < nx; c += 64) Kk[(size_t)r * nx + c] = Y[r * lay.ldY + c];
      // P = Z_xx + Z_ux^T K
      for (int r = wave(); r < nx; r += 4)
        for (int c = lane(); c < nx; c += 64) P[r * lay.ldP + c] = Z[r * lay.ldZ + c];
      __syncthreads();
      wg_mm_f32(nx, nx, nu, 1.f, Z + nx * lay.ldZ, lay.ldZ, true, Y, lay.ldY, false, 1.f, P, lay.ldP);
      // symmetrise
      for (int r = wave(); r < nx; r += 4)
        for (int c = r + 1 + lane(); c < nx; c += 64) {
          const float s = 0.5f * (P[r * lay.ldP + c] + P[c * lay.ldP + r]);
          P[r * lay.ldP + c] = s;
          P[c * lay.ldP + r] = s;
        }
      __syncthreads();
    }
    // ------------------------------------------------ forward propagation
    // Y = [Phi^x; Phi^u]; Phi^x starts at E_j (rows 0..nx-1 of Y)
    const float* Ej = a.E + (size_t)j * nx * nx;
    for (int r = wave(); r < nx; r += 4)
      for (int c = lane(); c < nx; c += 64) Y[r * lay.ldY + c] = Ej[(size_t)r * nx + c];
    __syncthreads();
    const size_t offx = (size_t)j * N - (size_t)j * (j - 1) / 2;
    const size_t offu = (size_t)j * (N - 1) - (size_t)j * (j - 1) / 2;
    for (int k = j + 1; k <= N; ++k) {
      if (a.Phx && inst == 0) {
        float* dst = a.Phx + (offx + (size_t)(k - j - 1)) * nx * nx;
        for (int r = wave(); r < nx; r += 4)
          for (int c = lane(); c < nx; c += 64) dst[(size_t)r * nx + c] = Y[r * lay.ldY + c];
      }
      if (k == N) {
        if (nf > 0) {
          for (int r = wave(); r < nf; r += 4)
            for (int c = lane(); c < nx; c += 64) G[r * lay.ldG + c] = a.CN[(size_t)r * nx + c];
          __syncthreads();
          wg_mm_f32(nf, nx, nx, 1.f, G, lay.ldG, false, Y, lay.ldY, false, 0.f, W, lay.ldW);
          wg_row_norms(nf, nx, W, lay.ldW, a.rownorm, a.hfj + ((size_t)inst * N + j) * nf, a.squared);
        }
        __syncthreads();
        break;
      }
      load_stage(k);
      __syncthreads();
      // Phi^u = K_k Phi^x  (rows nx.. of Y)
      const float* Kk = Kst + (size_t)k * nu * nx;
      load_block(nu, nx, [&](int r, int c) { return Kk[(size_t)r * nx + c]; }, Z, lay.ldZ);
      __syncthreads();
      wg_mm_f32(nu, nx, nx, 1.f, Z, lay.ldZ, false, Y, lay.ldY, false, 0.f, Y + nx * lay.ldY, lay.ldY);
      if (a.Phu && inst == 0) {
        float* dst = a.Phu + (offu + (size_t)(k - j - 1)) * nu * nx;
        for (int r = wave(); r < nu; r += 4)
          for (int c = lane(); c < nx; c += 64) dst[(size_t)r * nx + c] = Y[(nx + r) * lay.ldY + c];
      }
      // margins: rows of G_k [Phi^x; Phi^u]
      wg_mm_f32(nc, nx, nxu, 1.f, G, lay.ldG, false, Y, lay.ldY, false, 0.f, W, lay.ldW);
      wg_row_norms(nc, nx, W, lay.ldW, a.rownorm, a.hj + (((size_t)inst * N + k) * N + j) * nc, a.squared);
      // Phi^x_{k+1} = [A | B] Y
      wg_mm_f32(nx, nx, nxu, 1.f, AB, lay.ldAB, false, Y, lay.ldY, false, 0.f, Z, lay.ldZ);
      for (int r = wave(); r < nx; r += 4)
        for (int c = lane(); c < nx; c += 64) Y[r * lay.ldY + c] = Z[r * lay.ldZ + c];
      __syncthreads();
    }
  }
}

// h[inst][k][r] = wbound * sum_{j<k} hj[inst][k][j][r];  hf[inst][r] = wbound * sum_j hfj[inst][j][r]
// (fixed summation order: deterministic).
__global__ void k_sls_sum(int N, int nc, int nf, int count, float wbound, const float* hj, const float* hfj,
                          double* h, double* hf) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t nh = (size_t)count * N * nc;
  if (t < nh) {
    const size_t inst = t / ((size_t)N * nc), rem = t % ((size_t)N * nc);
    const int k = (int)(rem / nc), r = (int)(rem % nc);
    double s = 0.0;
    for (int j = 0; j < k; ++j) s += (double)hj[((inst * N + k) * N + j) * nc + r];
    h[t] = wbound * s;
  } else if (t < nh + (size_t)count * nf) {
    const size_t u = t - nh;
    const size_t inst = u / nf;
    const int r = (int)(u % nf);
    double s = 0.0;
    for (int j = 0; j < N; ++j) s += (double)hfj[(inst * N + j) * nf + r];
    hf[u] = wbound * s;
  }
}

// tau_{k,j} = |lambda_k| / sqrt(beta_{k,j} + eps)  (App. B), entries k <= j zero.
__global__ void k_sls_tau(int N, int nc, int nf, const float* betaj, const float* betafj, const double* lam,
                          double eps, double* tau) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t ns = (size_t)N * N * nc;
  if (t < ns) {
    const int k = (int)(t / ((size_t)N * nc));
    const int j = (int)((t / nc) % N), r = (int)(t % nc);
    tau[t] = k > j ? fabs(lam[(size_t)k * nc + r]) / sqrt((double)betaj[((size_t)k * N + j) * nc + r] + eps) : 0.0;
  } else if (t < ns + (size_t)N * nf) {
    const size_t u = t - ns;
    const int j = (int)(u / nf), r = (int)(u % nf);
    tau[t] = fabs(lam[(size_t)N * nc + r]) / sqrt((double)betafj[(size_t)j * nf + r] + eps);
  }
}

// beta_{k,j}: squared row norms of G_k [Phi^x_{k,j}; Phi^u_{k,j}] (C_N Phi^x_{N,j}
// at k = N) for given responses (packed as in gsls.h), one workgroup per (k, j).
__global__ void __launch_bounds__(kWG) k_sls_beta(SlsArgs a) {
  extern __shared__ __align__(16) char lds_generic[];
  LDS char* base = (LDS char*)lds_generic;
  const int N = a.N, nx = a.nx, nu = a.nu, nc = a.nc, nf = a.nf, nxu = nx + nu;
  const SlsLayout lay = sls_layout(nx, nu, nc, nf);
  LDS float* F = (LDS float*)base;
  LDS float* W = F + lay.W;
  LDS float* G = F + lay.G;
  LDS float* Y = F + lay.Y;
  const int k = blockIdx.x / N + 1, j = blockIdx.x % N;   // k in 1..N
  if (k <= j) return;
  const size_t offx = (size_t)j * N - (size_t)j * (j - 1) / 2;
  const size_t offu = (size_t)j * (N - 1) - (size_t)j * (j - 1) / 2;
  const float* Fx = a.Phx + (offx + (size_t)(k - j - 1)) * nx * nx;
  for (int r = wave(); r < nx; r += 4)
    for (int c = lane(); c < nx; c += 64) Y[r * lay.ldY + c] = Fx[(size_t)r * nx + c];
  if (k == N) {
    if (nf == 0) return;
    for (int r = wave(); r < nf; r += 4)
      for (int c = lane(); c < nx; c += 64) G[r * lay.ldG + c] = a.CN[(size_t)r * nx + c];
    __syncthreads();
    wg_mm_f32(nf, nx, nx, 1.f, G, lay.ldG, false, Y, lay.ldY, false, 0.f, W, lay.ldW);
    wg_row_norms(nf, nx, W, lay.ldW, 2, a.hfj + (size_t)j * nf, true);
    return;
  }
  const float* Fu = a.Phu + (offu + (size_t)(k - j - 1)) * nu * nx;
  const float* Gk = a.G + (size_t)k * nc * nxu;
  for (int r = wave(); r < nu; r += 4)
    for (int c = lane(); c < nx; c += 64) Y[(nx + r) * lay.ldY + c] = Fu[(size_t)r * nx + c];
  for (int r = wave(); r < nc; r += 4)
    for (int c = lane(); c < nxu; c += 64) G[r * lay.ldG + c] = Gk[(size_t)r * nxu + c];
  __syncthreads();
  wg_mm_f32(nc, nx, nxu, 1.f, G, lay.ldG, false, Y, lay.ldY, false, 0.f, W, lay.ldW);
  wg_row_norms(nc, nx, W, lay.ldW, 2, a.hj + ((size_t)k * N + j) * nc, true);
}

int launch_sls_beta(const SlsArgs& args, hipStream_t st) {
  const size_t sh = sls_layout(args.nx, args.nu, args.nc, args.nf).bytes;
  if (hipFuncSetAttribute((const void*)k_sls_beta, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh) != hipSuccess)
    return GSLS_ERR_HIP;
  k_sls_beta<<<args.N * args.N, kWG, sh, st>>>(args);
  return hipGetLastError() == hipSuccess ? GSLS_OK : GSLS_ERR_HIP;
}

size_t sls_lds_bytes(int nx, int nu, int nc, int nf) { return sls_layout(nx, nu, nc, nf).bytes; }

int launch_sls(const SlsArgs& args, int grid, hipStream_t st) {
  const size_t sh = sls_lds_bytes(args.nx, args.nu, args.nc, args.nf);
  if (hipFuncSetAttribute((const void*)k_sls, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh) != hipSuccess)
    return GSLS_ERR_HIP;
  k_sls<<<grid, kWG, sh, st>>>(args);
  return hipGetLastError() == hipSuccess ? GSLS_OK : GSLS_ERR_HIP;
}

int sls_grid(int nx, int nu, int nc, int nf) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  const size_t sh = sls_lds_bytes(nx, nu, nc, nf);
  if (hipFuncSetAttribute((const void*)k_sls, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void*)k_sls, kWG, sh) != hipSuccess) per = 1;
  return cus * std::max(per, 1);
}

int launch_sls_sum(int N, int nc, int nf, int count, float wbound, const float* hj, const float* hfj, double* h,
                   double* hf, hipStream_t st) {
  const size_t tot = (size_t)count * N * nc + (size_t)count * nf;
  k_sls_sum<<<(unsigned)((tot + 255) / 256), 256, 0, st>>>(N, nc, nf, count, wbound, hj, hfj, h, hf);
  return hipGetLastError() == hipSuccess ? GSLS_OK : GSLS_ERR_HIP;
}

int launch_sls_tau(int N, int nc, int nf, const float* betaj, const float* betafj, const double* lam, double eps,
                   double* tau, hipStream_t st) {
  const size_t tot = (size_t)N * N * nc + (size_t)N * nf;
  k_sls_tau<<<(unsigned)((tot + 255) / 256), 256, 0, st>>>(N, nc, nf, betaj, betafj, lam, eps, tau);
  return hipGetLastError() == hipSuccess ? GSLS_OK : GSLS_ERR_HIP;
}

}  // namespace gsls
