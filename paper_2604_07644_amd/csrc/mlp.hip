// Learned warm start for the batched solver: feature rows, a 4-layer MLP in
// BF16 on the matrix cores (forward, backward, Adam), and the scatter of its
// prediction into the batch's starting iterate.
//
// The warm start is an extension of the ADMM start of Sec. IV-A: instead of
// z = y = 0 at rho = 1, each instance starts from a predicted (z, lambda) and a
// predicted rho.  One feature row per stage k = 0..N of a box-constrained
// instance (d_in = 160: x0 / x_max, the bound scales, a 64-d sketch of the
// stage's linearisation (A_k - I) x0, B_k^T x0, and k/N, N/512, nx/75, nu/19);
// one output row (d_out = 192: z and lambda of the stage's rows, log10 rho).
//
// GEMMs: C = op(A) op(B) on 64 x 64 output tiles, four waves with 32 x 32
// each, K in steps of 32 through LDS, v_mfma_f32_16x16x32_bf16 with FP32
// accumulation.  Lane l of a wave supplies A[i0 + l%16][8(l/16) .. 8(l/16)+7]
// and B[8(l/16) .. +7][j0 + l%16] of the 32-wide K slice and holds
// C[i0 + 4(l/16) + r][j0 + l%16] in accumulator r.  Weight gradients reduce
// over the rows in K chunks (one partial per chunk, summed in a fixed order:
// deterministic).
//
// Hidden activations are kept as a pair of BF16 arrays, h = hi + lo with
// hi = bf16(h) and lo = bf16(h - hi) (about 16 significant bits), and every
// product that consumes them (the next layer's forward GEMM and the weight
// gradient h^T delta) runs the matrix cores on both halves.  Rounding the
// activations to a single BF16 moves ReLU decisions downstream and costs a
// few per cent on the first layer's weight gradient; with the pair the
// gradients follow the FP64 definition to the BF16 rounding of the weights,
// inputs and back-propagated deltas (a few 1e-3).  Deltas stay single BF16.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "batch.hpp"
#include "dev_common.hpp"

namespace gsls {

typedef unsigned short u16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef u16 u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kDin = 160, kDh = 512, kDout = 192, kLayers = 4;
constexpr int kSketch = 64, kSlots = 94, kXs = 75, kUs = 19, kRhoCol = 188;
constexpr float kRhoWeight = 25.f;   // loss weight of the rho entry of a row
constexpr int kSizes[kLayers + 1] = {kDin, kDh, kDh, kDh, kDout};

// round to nearest even (NaN kept quiet)
__device__ __forceinline__ u16 f2bf(float f) {
  unsigned u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;
  u += 0x7fffu + ((u >> 16) & 1u);
  return (u16)(u >> 16);
}
__device__ __forceinline__ float bf2f(u16 h) { return __uint_as_float((unsigned)h << 16); }

// ------------------------------------------------------------------ GEMM
enum { EPI_BIAS_RELU = 0, EPI_BIAS = 1, EPI_RELU_MASK = 2, EPI_PARTIAL = 3 };

struct GemmArgs {
  int M, N, K;
  const u16* A; int lda; int ta; const int* ridx;   // ridx: gather of A's stored rows
  const u16* Alo;                                   // nullable: low BF16 half of A (A = A + Alo)
  const u16* B; int ldb; int tb;
  const float* bias;                                // EPI_BIAS*
  const u16* act; int ldact;                        // EPI_RELU_MASK: mask [act > 0]
  u16* Cb; float* Cf; int ldc;
  u16* Clo;                                         // EPI_BIAS_RELU, nullable: low half of the output
  int kc;                                           // K chunk per blockIdx.z
};

constexpr int BM = 64, BN = 64, BK = 32, BKP = BK + 8;

// Stages a 64 x 32 slice of op(X) into S[r][k] (r over the 64 output rows or
// columns, k over the slice).  kmaj: X is stored with k contiguous
// (element (r, k) at X[row(r) * ld + k]); else r contiguous (X[row(k) * ld + r]).
__device__ __forceinline__ void stage_tile(LDS u16 (*S)[BKP], const u16* X, int ld, bool kmaj, const int* ridx,
                                           int r0, int R, int k0, int kend) {
  const int t = tid();
  if (kmaj) {
    const int r = t >> 2, ks = (t & 3) * 8;
    const int rr = min(r0 + r, R - 1);
    const long long row = ridx ? ridx[rr] : rr;
    const u16* src = X + row * ld + k0 + ks;
    u16x8 v;
    if (k0 + ks + 8 <= kend) {
      v = *(const u16x8*)src;
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = (k0 + ks + e < kend) ? src[e] : (u16)0;
    }
    *(LDS u16x8*)&S[r][ks] = v;
  } else {
    const int kk = t >> 3, rs = (t & 7) * 8;
    const bool kin = k0 + kk < kend;
    const int kr = min(k0 + kk, kend - 1);
    const long long row = ridx ? ridx[kr] : kr;
    const u16* src = X + row * ld + r0 + rs;
    u16x8 v;
    if (kin && r0 + rs + 8 <= R) {
      v = *(const u16x8*)src;
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = (kin && r0 + rs + e < R) ? src[e] : (u16)0;
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) S[rs + e][kk] = v[e];
  }
}

__global__ void __launch_bounds__(256) k_gemm(GemmArgs g, int epi) {
  __shared__ __align__(16) u16 As_[BM][BKP];
  __shared__ __align__(16) u16 Al_[BM][BKP];
  __shared__ __align__(16) u16 Bs_[BN][BKP];
  LDS u16 (*As)[BKP] = (LDS u16 (*)[BKP])As_;
  LDS u16 (*Al)[BKP] = (LDS u16 (*)[BKP])Al_;
  LDS u16 (*Bs)[BKP] = (LDS u16 (*)[BKP])Bs_;
  const bool split = g.Alo != nullptr;
  const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN, kz = blockIdx.z;
  const int kbeg = kz * g.kc, kend = min(g.K, kbeg + g.kc);
  const int l = lane(), w = wave();
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  const int r16 = l & 15, q = l >> 4;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    // A(m, k): ta -> stored [K][M] (m contiguous); else [M][K]
    stage_tile(As, g.A, g.lda, !g.ta, g.ridx, m0, g.M, k0, kend);
    if (split) stage_tile(Al, g.Alo, g.lda, !g.ta, g.ridx, m0, g.M, k0, kend);
    // B(k, n): tb -> stored [N][K] (k contiguous); else [K][N]
    stage_tile(Bs, g.B, g.ldb, g.tb, nullptr, n0, g.N, k0, kend);
    __syncthreads();
    bf16x8 a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) a[i] = __builtin_bit_cast(bf16x8, *(const LDS u16x8*)&As[wm + i * 16 + r16][q * 8]);
#pragma unroll
    for (int j = 0; j < 2; ++j) b[j] = __builtin_bit_cast(bf16x8, *(const LDS u16x8*)&Bs[wn + j * 16 + r16][q * 8]);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    if (split) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
        a[i] = __builtin_bit_cast(bf16x8, *(const LDS u16x8*)&Al[wm + i * 16 + r16][q * 8]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm + i * 16 + 4 * q + r, col = n0 + wn + j * 16 + r16;
        if (row >= g.M || col >= g.N) continue;
        float v = acc[i][j][r];
        const long long o = (long long)row * g.ldc + col;
        if (epi == EPI_BIAS_RELU) {
          const float h = fmaxf(v + g.bias[col], 0.f);
          const u16 hi = f2bf(h);
          g.Cb[o] = hi;
          if (g.Clo) g.Clo[o] = f2bf(h - bf2f(hi));
        } else if (epi == EPI_BIAS) {
          g.Cf[o] = v + g.bias[col];
        } else if (epi == EPI_RELU_MASK) {
          const float h = bf2f(g.act[(long long)row * g.ldact + col]);
          g.Cb[o] = f2bf(h > 0.f ? v : 0.f);
        } else {
          g.Cf[(long long)kz * g.M * g.N + o] = v;
        }
      }
}

// ------------------------------------------------------- loss and reductions
// dY = 2 M (Y - T) (unscaled; the gradient is divided by sum(M) in the
// reduction), per-block partial sums of M (Y - T)^2 and M.
__global__ void __launch_bounds__(256) k_loss(const float* Y, const float* T, const float* Mk, const int* idx,
                                              int rows, u16* dY, float* part) {
  __shared__ float s1[256], s2[256];
  float a1 = 0.f, a2 = 0.f;
  const long long n = (long long)rows * kDout;
  for (long long e = (long long)blockIdx.x * 256 + tid(); e < n; e += (long long)gridDim.x * 256) {
    const int r = (int)(e / kDout), c = (int)(e - (long long)r * kDout);
    const long long src = (long long)(idx ? idx[r] : r) * kDout + c;
    const float m = Mk[src], d = Y[e] - T[src];
    a1 += m * d * d;
    a2 += m;
    dY[e] = f2bf(2.f * m * d);
  }
  s1[tid()] = a1; s2[tid()] = a2;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid() < st) { s1[tid()] += s1[tid() + st]; s2[tid()] += s2[tid() + st]; }
    __syncthreads();
  }
  if (tid() == 0) { part[2 * blockIdx.x] = s1[0]; part[2 * blockIdx.x + 1] = s2[0]; }
}

// scal[0] = loss, scal[1] = sum(M), from nb block partials (fixed order).
__global__ void k_loss_final(const float* part, int nb, float* scal) {
  if (tid() == 0) {
    double a = 0, b = 0;
    for (int i = 0; i < nb; ++i) { a += part[2 * i]; b += part[2 * i + 1]; }
    scal[0] = (float)(b > 0 ? a / b : 0.0);
    scal[1] = (float)b;
  }
}

// Column sums of an R x n BF16 matrix over row chunks: part[z][c].
__global__ void __launch_bounds__(256) k_colsum(const u16* X, int R, int n, int rc, float* part) {
  const int c = blockIdx.x * 256 + tid();
  const int z = blockIdx.y;
  if (c >= n) return;
  const int r1 = min(R, (z + 1) * rc);
  float s = 0.f;
  for (int r = z * rc; r < r1; ++r) s += bf2f(X[(long long)r * n + c]);
  part[(long long)z * n + c] = s;
}

// out[i] = (sum_z part[z * len + i]) / scal[1]  (fixed order)
__global__ void __launch_bounds__(256) k_reduce_scale(const float* part, int nz, long long len, const float* scal,
                                                      float* out) {
  const long long i = (long long)blockIdx.x * 256 + tid();
  if (i >= len) return;
  float s = 0.f;
  for (int z = 0; z < nz; ++z) s += part[(long long)z * len + i];
  const float cnt = scal[1];
  out[i] = cnt > 0.f ? s / cnt : 0.f;
}

// Adam with bias correction c1 = 1 / (1 - b1^t), c2 = 1 / (1 - b2^t);
// writes the FP32 master weights and their BF16 copy.
__global__ void __launch_bounds__(256) k_adam(float* p, float* m, float* v, const float* g, u16* pb, long long n,
                                              float lr, float b1, float b2, float eps, float c1, float c2) {
  const long long i = (long long)blockIdx.x * 256 + tid();
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
  p[i] = pi;
  pb[i] = f2bf(pi);
}

__global__ void __launch_bounds__(256) k_to_bf16(const float* p, u16* pb, long long n) {
  const long long i = (long long)blockIdx.x * 256 + tid();
  if (i < n) pb[i] = f2bf(p[i]);
}

// ------------------------------------------------------------ feature rows
// One wave per row (four rows per workgroup).  Row r belongs to instance
// c = row_inst[r], stage k = r - row_off[c]; x_max = u of the first state
// row, u_max = u of the first input row.
__global__ void __launch_bounds__(256) k_ws_features(const BInst* inst, const float* fp, const double* dp,
                                                     const int* row_inst, const int* row_off, int rows,
                                                     const float* sketch, u16* X) {
  __shared__ float dsh[4][96];
  __shared__ float xsh[4][80];
  const int w = wave(), l = lane();
  const int r = blockIdx.x * 4 + w;
  const bool valid = r < rows;
  const int rr = valid ? r : rows - 1;
  const int c = row_inst[rr];
  const BInst I = inst[c];
  const int k = rr - row_off[c];
  const int nx = I.nx, nu = I.nu, N = I.N;
  const EpLayout ep = ep_layout(nx, nu);
  const float xm = (float)dp[I.ou], um = (float)dp[I.ou + nx];
  const float* x0 = fp + I.ox0;
  for (int j = l; j < 80; j += 64) xsh[w][j] = j < nx ? x0[j] : 0.f;
  __syncthreads();
  for (int j = l; j < 96; j += 64) {
    float d = 0.f;
    if (k < N) {
      if (j < nx) {
        // row j of A_k in the epoch input packet ([A_k | B_k], leading dimension ep.ld)
        const float* Ar = fp + I.oE + (long long)k * ep.stride + ep.AB + (long long)j * ep.ld;
        float s = 0.f;
        for (int cc = 0; cc < nx; ++cc) s += Ar[cc] * xsh[w][cc];
        d = (s - xsh[w][j]) / xm;
      } else if (j >= kXs && j < kXs + nu) {
        const int jj = j - kXs;
        const float* Bk = fp + I.oE + (long long)k * ep.stride + ep.AB + nx;
        float s = 0.f;
        for (int rr2 = 0; rr2 < nx; ++rr2) s += Bk[(long long)rr2 * ep.ld + jj] * xsh[w][rr2];
        d = s / xm;
      }
    }
    dsh[w][j] = d;
  }
  __syncthreads();
  if (!valid) return;
  u16* out = X + (long long)r * kDin;
  {
    const float* Sr = sketch + (long long)l * kSlots;
    float s = 0.f;
    for (int e = 0; e < kSlots; ++e) s += Sr[e] * dsh[w][e];
    out[77 + l] = f2bf(s);
  }
  for (int j = l; j < kDin; j += 64) {
    if (j >= 77 && j < 141) continue;
    float f = 0.f;
    if (j < nx) f = xsh[w][j] / xm;
    else if (j == 75) f = xm / 5.f;
    else if (j == 76) f = um;
    else if (j == 141) f = (float)k / (float)N;
    else if (j == 142) f = (float)N / 512.f;
    else if (j == 143) f = (float)nx / 75.f;
    else if (j == 144) f = (float)nu / 19.f;
    out[j] = f2bf(f);
  }
}

// Prediction -> start of instance c (one workgroup per instance): rho0 =
// 10^(mean over its rows of Y[., 188]) clamped to [rho_min, rho_max];
// z0 = clip(prediction * scale, l, u); y0 = lambda prediction / rho0.
// parts selects what the prediction sets (bit 0: rho0, bit 1: z0, bit 2: y0);
// the rest keeps the cold start (rho0 = 1, z0 = 0, y0 = 0).
__global__ void __launch_bounds__(256) k_ws_scatter(const BInst* inst, double* dp, const int* row_off,
                                                    const float* Y, double rho_min, double rho_max, double* rho0,
                                                    int* warm, int parts) {
  __shared__ double red[256];
  const int c = blockIdx.x;
  const BInst I = inst[c];
  const int nx = I.nx, nu = I.nu, N = I.N, nc = I.nc;
  const int r0 = row_off[c];
  double s = 0.0;
  for (int k = tid(); k <= N; k += 256) s += (double)Y[(long long)(r0 + k) * kDout + kRhoCol];
  red[tid()] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid() < st) red[tid()] += red[tid() + st];
    __syncthreads();
  }
  double rho = pow(10.0, red[0] / (double)(N + 1));
  rho = fmin(fmax(rho, rho_min), rho_max);
  if (!(rho > 0.0) || !(parts & 1)) rho = 1.0;
  const double xm = dp[I.ou], um = dp[I.ou + nx];
  for (int e = tid(); e < I.m; e += 256) {
    int k, j;
    if (e < N * nc) { k = e / nc; j = e - k * nc; } else { k = N; j = e - N * nc; }
    const float* Yr = Y + (long long)(r0 + k) * kDout;
    const bool isx = j < nx;
    const double zp = isx ? (double)Yr[j] * xm : (double)Yr[kXs + (j - nx)] * um;
    const double lp = isx ? (double)Yr[94 + j] : (double)Yr[169 + (j - nx)];
    const double lo = dp[I.ol + e], hi = dp[I.ou + e];
    dp[I.oz + e] = (parts & 2) ? (zp < lo ? lo : (zp > hi ? hi : zp)) : 0.0;
    dp[I.oy + e] = (parts & 4) ? lp / rho : 0.0;
  }
  if (tid() == 0) { rho0[c] = rho; warm[c] = 1; }
}

// Target and weight rows of instance c from its solution (z, y) and final
// rho: weight 1 on the z and lambda entries, kRhoWeight on the rho entry.
__global__ void __launch_bounds__(256) k_ws_targets(const BInst* inst, const double* dp, const int* row_off,
                                                    const BResult* res, float* T, float* Mk) {
  const int c = blockIdx.x;
  const BInst I = inst[c];
  const int nx = I.nx, nu = I.nu, N = I.N, nc = I.nc, nf = I.nf;
  const int r0 = row_off[c];
  const double rho = res[c].rho;
  const double xm = dp[I.ou], um = dp[I.ou + nx];
  const float lr = (float)log10(rho);
  for (long long e = tid(); e < (long long)(N + 1) * kDout; e += 256) {
    const int k = (int)(e / kDout), col = (int)(e - (long long)k * kDout);
    float t = 0.f, m = 0.f;
    const int rows_k = k < N ? nc : nf;
    const long long base = (long long)k * nc;
    int j = -1;
    bool lam = false;
    if (col < nx) j = col;
    else if (col >= kXs && col < kXs + nu && k < N) j = nx + (col - kXs);
    else if (col >= 94 && col < 94 + nx) { j = col - 94; lam = true; }
    else if (col >= 169 && col < 169 + nu && k < N) { j = nx + (col - 169); lam = true; }
    if (j >= 0 && j < rows_k) {
      const double zv = dp[I.oz + base + j], yv = dp[I.oy + base + j];
      t = lam ? (float)(rho * yv) : (float)(zv / (j < nx ? xm : um));
      m = 1.f;
    }
    if (col == kRhoCol) { t = lr; m = kRhoWeight; }
    T[(long long)(r0 + k) * kDout + col] = t;
    Mk[(long long)(r0 + k) * kDout + col] = m;
  }
}

// ------------------------------------------------------------------ host
struct WsModel {
  hipStream_t stream = nullptr;
  long long np = 0;
  long long woff[kLayers], boff[kLayers];
  float *p = nullptr, *m = nullptr, *v = nullptr, *g = nullptr, *sketch = nullptr, *scal = nullptr;
  u16* pb = nullptr;
  int step = 0;
  // workspace (grown on demand)
  int cap = 0;
  u16 *H[3] = {nullptr, nullptr, nullptr}, *Hl[3] = {nullptr, nullptr, nullptr};   // activations, hi / lo
  u16 *dY = nullptr, *dA[2] = {nullptr, nullptr}, *Xw = nullptr;
  float *Y = nullptr, *part = nullptr, *lpart = nullptr, *cpart = nullptr;
  size_t part_len = 0;
  ~WsModel() {
    for (void* q : {(void*)p, (void*)m, (void*)v, (void*)g, (void*)sketch, (void*)scal, (void*)pb})
      if (q) (void)hipFree(q);
    free_ws();
  }
  void free_ws() {
    for (void* q : {(void*)H[0], (void*)H[1], (void*)H[2], (void*)Hl[0], (void*)Hl[1], (void*)Hl[2], (void*)dY,
                    (void*)dA[0], (void*)dA[1], (void*)Xw, (void*)Y, (void*)part, (void*)lpart, (void*)cpart})
      if (q) (void)hipFree(q);
    H[0] = H[1] = H[2] = Hl[0] = Hl[1] = Hl[2] = dY = dA[0] = dA[1] = Xw = nullptr;
    Y = part = lpart = cpart = nullptr;
    cap = 0;
  }
};

constexpr int kSplitRows = 512;    // rows per K chunk of a weight-gradient GEMM
constexpr int kLossBlocks = 512;

static long long ws_nparams() {
  long long n = 0;
  for (int i = 0; i < kLayers; ++i) n += (long long)kSizes[i] * kSizes[i + 1] + kSizes[i + 1];
  return n;
}

static int ws_reserve(WsModel* W, int rows, bool train) {
  if (rows <= W->cap && (!train || W->part)) return GSLS_OK;
  const int cap = rows > W->cap ? rows : W->cap;
  W->free_ws();
  const size_t R = (size_t)cap;
  for (int i = 0; i < 3; ++i)
    if (hipMalloc(&W->H[i], R * kDh * 2) != hipSuccess || hipMalloc(&W->Hl[i], R * kDh * 2) != hipSuccess)
      return GSLS_ERR_OOM;
  if (hipMalloc(&W->Y, R * kDout * 4) != hipSuccess) return GSLS_ERR_OOM;
  if (hipMalloc(&W->Xw, R * kDin * 2) != hipSuccess) return GSLS_ERR_OOM;
  if (train) {
    if (hipMalloc(&W->dY, R * kDout * 2) != hipSuccess) return GSLS_ERR_OOM;
    for (int i = 0; i < 2; ++i)
      if (hipMalloc(&W->dA[i], R * kDh * 2) != hipSuccess) return GSLS_ERR_OOM;
    const size_t nz = (R + kSplitRows - 1) / kSplitRows;
    W->part_len = nz * (size_t)kDh * kDh;
    if (hipMalloc(&W->part, W->part_len * 4) != hipSuccess) return GSLS_ERR_OOM;
    if (hipMalloc(&W->cpart, nz * kDh * 4) != hipSuccess) return GSLS_ERR_OOM;
    if (hipMalloc(&W->lpart, 2 * kLossBlocks * 4) != hipSuccess) return GSLS_ERR_OOM;
  }
  W->cap = cap;
  return GSLS_OK;
}

static void gemm(hipStream_t s, int M, int N, int K, const u16* A, const u16* Alo, int lda, bool ta, const int* ridx,
                 const u16* B, int ldb, bool tb, int epi, const float* bias, const u16* act, int ldact, u16* Cb,
                 u16* Clo, float* Cf, int ldc, int kc) {
  GemmArgs g{};
  g.M = M; g.N = N; g.K = K;
  g.A = A; g.Alo = Alo; g.lda = lda; g.ta = ta ? 1 : 0; g.ridx = ridx;
  g.B = B; g.ldb = ldb; g.tb = tb ? 1 : 0;
  g.bias = bias; g.act = act; g.ldact = ldact; g.Cb = Cb; g.Clo = Clo; g.Cf = Cf; g.ldc = ldc;
  g.kc = kc > 0 ? kc : K;
  const int nz = (K + g.kc - 1) / g.kc;
  dim3 grid((M + BM - 1) / BM, (N + BN - 1) / BN, nz);
  k_gemm<<<grid, 256, 0, s>>>(g, epi);
}

// Forward pass of rows X (gathered through idx if given) with the hidden
// activations in H[0..2] (hi) and Hl[0..2] (lo), each [rows][512], and the
// output in Y.
static void ws_forward_into(WsModel* W, const u16* X, const int* idx, int rows, float* Y, u16* const* H,
                            u16* const* Hl) {
  const u16* in = X;
  const u16* inlo = nullptr;   // the feature rows are BF16 by definition
  const int* ri = idx;
  int din = kDin;
  for (int L = 0; L < kLayers; ++L) {
    const int dout = kSizes[L + 1];
    const u16* Wl = W->pb + W->woff[L];
    const float* bl = W->p + W->boff[L];
    if (L + 1 < kLayers)
      gemm(W->stream, rows, dout, din, in, inlo, din, false, ri, Wl, dout, false, EPI_BIAS_RELU, bl, nullptr, 0,
           H[L], Hl[L], nullptr, dout, 0);
    else
      gemm(W->stream, rows, dout, din, in, inlo, din, false, ri, Wl, dout, false, EPI_BIAS, bl, nullptr, 0, nullptr,
           nullptr, Y, dout, 0);
    in = H[L];
    inlo = Hl[L];
    ri = nullptr;
    din = dout;
  }
}

// Forward pass with the model's own workspace (H1..H3 as BF16 hi / lo pairs).
static void ws_forward(WsModel* W, const u16* X, const int* idx, int rows, float* Y) {
  ws_forward_into(W, X, idx, rows, Y, W->H, W->Hl);
}

// ------------------------------------------- forward without allocation
// Workspace of gsls_ws_forward_static: the six [kStaticRows][512] BF16
// activation arrays (hi and lo of the three hidden layers) in one
// file-scope device array, 12 MiB on every GPU the library runs on, held
// until the process ends.  Every layer writes its activations before the
// next layer reads them, so nothing needs clearing between calls.
constexpr int kStaticRows = 2048;
constexpr size_t kStaticElems = (size_t)6 * kStaticRows * kDh;
static __device__ __align__(256) u16 scratch[kStaticElems];
constexpr int kMaxDevices = 64;
static u16* g_scratch_dev[kMaxDevices];     // device address of scratch, per device
static std::mutex g_scratch_mu;

// Device address of the static workspace on the current device, looked up
// once per device (the array's host-side name is not a device address).
static int static_scratch(u16** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return GSLS_ERR_HIP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return GSLS_ERR_HIP;
    g_scratch_dev[dev] = (u16*)p;
  }
  *out = g_scratch_dev[dev];
  return GSLS_OK;
}

// Forward + backward: the flat gradient (W1, b1, ..., divided by sum(M)) in
// W->g and (loss, sum(M)) in W->scal.
static void ws_backward(WsModel* W, const u16* X, const float* T, const float* Mk, const int* idx, int rows) {
  hipStream_t s = W->stream;
  ws_forward(W, X, idx, rows, W->Y);
  k_loss<<<kLossBlocks, 256, 0, s>>>(W->Y, T, Mk, idx, rows, W->dY, W->lpart);
  k_loss_final<<<1, 64, 0, s>>>(W->lpart, kLossBlocks, W->scal);
  const int nz = (rows + kSplitRows - 1) / kSplitRows;
  const u16* dcur = W->dY;
  for (int L = kLayers - 1; L >= 0; --L) {
    const int din = kSizes[L], dout = kSizes[L + 1];
    const u16* hin = L > 0 ? W->H[L - 1] : X;
    const u16* hlo = L > 0 ? W->Hl[L - 1] : nullptr;
    const int* ri = L > 0 ? nullptr : idx;
    // dW_L = h_in^T dcur  (K = rows, chunked)
    gemm(s, din, dout, rows, hin, hlo, din, true, ri, dcur, dout, false, EPI_PARTIAL, nullptr, nullptr, 0, nullptr,
         nullptr, W->part, dout, kSplitRows);
    const long long wl = (long long)din * dout;
    k_reduce_scale<<<(unsigned)((wl + 255) / 256), 256, 0, s>>>(W->part, nz, wl, W->scal, W->g + W->woff[L]);
    k_colsum<<<dim3((dout + 255) / 256, nz), 256, 0, s>>>(dcur, rows, dout, kSplitRows, W->cpart);
    k_reduce_scale<<<(dout + 255) / 256, 256, 0, s>>>(W->cpart, nz, dout, W->scal, W->g + W->boff[L]);
    if (L > 0) {
      // d(pre-activation of layer L-1) = (dcur W_L^T) * [h_in > 0]
      u16* dn = W->dA[L & 1];
      gemm(s, rows, din, dout, dcur, nullptr, dout, false, nullptr, W->pb + W->woff[L], dout, true, EPI_RELU_MASK,
           nullptr, hin, din, dn, nullptr, nullptr, din, 0);
      dcur = dn;
    }
  }
}

static int ws_alloc_params(WsModel* W, const float* params_host, const float* sketch_host) {
  W->np = ws_nparams();
  long long o = 0;
  for (int i = 0; i < kLayers; ++i) {
    W->woff[i] = o; o += (long long)kSizes[i] * kSizes[i + 1];
    W->boff[i] = o; o += kSizes[i + 1];
  }
  const size_t n = (size_t)W->np;
  if (hipMalloc(&W->p, n * 4) != hipSuccess || hipMalloc(&W->m, n * 4) != hipSuccess ||
      hipMalloc(&W->v, n * 4) != hipSuccess || hipMalloc(&W->g, n * 4) != hipSuccess ||
      hipMalloc(&W->pb, n * 2) != hipSuccess || hipMalloc(&W->sketch, kSketch * kSlots * 4) != hipSuccess ||
      hipMalloc(&W->scal, 4 * 4) != hipSuccess)
    return GSLS_ERR_OOM;
  if (hipMemcpy(W->p, params_host, n * 4, hipMemcpyHostToDevice) != hipSuccess) return GSLS_ERR_HIP;
  if (hipMemcpy(W->sketch, sketch_host, kSketch * kSlots * 4, hipMemcpyHostToDevice) != hipSuccess)
    return GSLS_ERR_HIP;
  if (hipMemset(W->m, 0, n * 4) != hipSuccess || hipMemset(W->v, 0, n * 4) != hipSuccess) return GSLS_ERR_HIP;
  k_to_bf16<<<(unsigned)((n + 255) / 256), 256, 0, W->stream>>>(W->p, W->pb, (long long)n);
  if (hipStreamSynchronize(W->stream) != hipSuccess) return GSLS_ERR_HIP;
  return GSLS_OK;
}

static bool finite_host(const float* x, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(x[i])) return false;
  return true;
}

static const char kMagic[8] = {'G', 'S', 'L', 'S', 'W', 'S', '0', '1'};

}  // namespace gsls

struct gsls_ws {
  gsls::WsModel w;
};

extern "C" {

int64_t gsls_ws_nparams(void) { return gsls::ws_nparams(); }

int gsls_ws_create(const float* params, const float* sketch, void* stream, gsls_ws** out) {
  if (!params || !sketch || !out) return GSLS_ERR_INVALID_ARG;
  *out = nullptr;
  if (!gsls::finite_host(params, (size_t)gsls::ws_nparams()) ||
      !gsls::finite_host(sketch, gsls::kSketch * gsls::kSlots))
    return GSLS_ERR_INVALID_ARG;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return GSLS_ERR_HIP;
  gsls_ws* h = new (std::nothrow) gsls_ws;
  if (!h) return GSLS_ERR_OOM;
  h->w.stream = (hipStream_t)stream;
  int rc = gsls::ws_alloc_params(&h->w, params, sketch);
  if (rc) { delete h; return rc; }
  *out = h;
  return GSLS_OK;
}

int gsls_ws_get_params(gsls_ws* h, float* params) {
  if (!h || !params) return GSLS_ERR_INVALID_ARG;
  if (hipStreamSynchronize(h->w.stream) != hipSuccess) return GSLS_ERR_HIP;
  if (hipMemcpy(params, h->w.p, (size_t)h->w.np * 4, hipMemcpyDeviceToHost) != hipSuccess) return GSLS_ERR_HIP;
  return GSLS_OK;
}

int gsls_ws_save(gsls_ws* h, const char* path) {
  if (!h || !path) return GSLS_ERR_INVALID_ARG;
  std::vector<float> p((size_t)h->w.np), sk(gsls::kSketch * gsls::kSlots);
  int rc = gsls_ws_get_params(h, p.data());
  if (rc) return rc;
  if (hipMemcpy(sk.data(), h->w.sketch, sk.size() * 4, hipMemcpyDeviceToHost) != hipSuccess) return GSLS_ERR_HIP;
  FILE* f = fopen(path, "wb");
  if (!f) return GSLS_ERR_INVALID_ARG;
  const int64_t n = h->w.np;
  bool ok = fwrite(gsls::kMagic, 1, 8, f) == 8 && fwrite(&n, 8, 1, f) == 1 &&
            fwrite(p.data(), 4, p.size(), f) == p.size() && fwrite(sk.data(), 4, sk.size(), f) == sk.size();
  ok = (fclose(f) == 0) && ok;
  return ok ? GSLS_OK : GSLS_ERR_INVALID_ARG;
}

int gsls_ws_load(const char* path, void* stream, gsls_ws** out) {
  if (!path || !out) return GSLS_ERR_INVALID_ARG;
  *out = nullptr;
  FILE* f = fopen(path, "rb");
  if (!f) return GSLS_ERR_INVALID_ARG;
  char mg[8];
  int64_t n = 0;
  std::vector<float> p((size_t)gsls::ws_nparams()), sk(gsls::kSketch * gsls::kSlots);
  bool ok = fread(mg, 1, 8, f) == 8 && memcmp(mg, gsls::kMagic, 8) == 0 && fread(&n, 8, 1, f) == 1 &&
            n == gsls::ws_nparams() && fread(p.data(), 4, p.size(), f) == p.size() &&
            fread(sk.data(), 4, sk.size(), f) == sk.size();
  fclose(f);
  if (!ok) return GSLS_ERR_INVALID_ARG;
  return gsls_ws_create(p.data(), sk.data(), stream, out);
}

int gsls_ws_forward(gsls_ws* h, const uint16_t* X, int32_t rows, float* Y) {
  if (!h || !X || !Y || rows < 1) return GSLS_ERR_INVALID_ARG;
  int rc = gsls::ws_reserve(&h->w, rows, false);
  if (rc) return rc;
  gsls::ws_forward(&h->w, X, nullptr, rows, Y);
  if (hipGetLastError() != hipSuccess) return GSLS_ERR_HIP;
  return GSLS_OK;
}

int gsls_ws_forward_static(gsls_ws* h, const uint16_t* X, int32_t rows, float* Y) {
  if (!h || !X || !Y || rows < 1) return GSLS_ERR_INVALID_ARG;
  if (rows > gsls::kStaticRows) return GSLS_ERR_DIM;
  gsls::u16* base = nullptr;
  int rc = gsls::static_scratch(&base);
  if (rc) return rc;
  const size_t stride = (size_t)gsls::kStaticRows * gsls::kDh;
  gsls::u16* H[3] = {base, base + stride, base + 2 * stride};
  gsls::u16* Hl[3] = {base + 3 * stride, base + 4 * stride, base + 5 * stride};
  gsls::ws_forward_into(&h->w, X, nullptr, rows, Y, H, Hl);
  if (hipGetLastError() != hipSuccess) return GSLS_ERR_HIP;
  return GSLS_OK;
}

int gsls_ws_loss_grad(gsls_ws* h, const uint16_t* X, const float* T, const float* M, const int32_t* idx,
                      int32_t rows, float* grad, float* loss) {
  if (!h || !X || !T || !M || rows < 1) return GSLS_ERR_INVALID_ARG;
  int rc = gsls::ws_reserve(&h->w, rows, true);
  if (rc) return rc;
  gsls::ws_backward(&h->w, X, T, M, idx, rows);
  if (hipGetLastError() != hipSuccess) return GSLS_ERR_HIP;
  if (hipStreamSynchronize(h->w.stream) != hipSuccess) return GSLS_ERR_HIP;
  if (grad && hipMemcpy(grad, h->w.g, (size_t)h->w.np * 4, hipMemcpyDeviceToHost) != hipSuccess) return GSLS_ERR_HIP;
  if (loss && hipMemcpy(loss, h->w.scal, 4, hipMemcpyDeviceToHost) != hipSuccess) return GSLS_ERR_HIP;
  return GSLS_OK;
}

int gsls_ws_train_step(gsls_ws* h, const uint16_t* X, const float* T, const float* M, const int32_t* idx,
                       int32_t rows, float lr, float* loss) {
  if (!h || !X || !T || !M || rows < 1 || !(lr > 0.f)) return GSLS_ERR_INVALID_ARG;
  int rc = gsls::ws_reserve(&h->w, rows, true);
  if (rc) return rc;
  gsls::WsModel* W = &h->w;
  gsls::ws_backward(W, X, T, M, idx, rows);
  W->step += 1;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = (float)(1.0 / (1.0 - std::pow(0.9, W->step)));
  const float c2 = (float)(1.0 / (1.0 - std::pow(0.999, W->step)));
  gsls::k_adam<<<(unsigned)((W->np + 255) / 256), 256, 0, W->stream>>>(W->p, W->m, W->v, W->g, W->pb, W->np, lr, b1,
                                                                       b2, eps, c1, c2);
  if (hipGetLastError() != hipSuccess) return GSLS_ERR_HIP;
  if (loss) {
    if (hipStreamSynchronize(W->stream) != hipSuccess) return GSLS_ERR_HIP;
    if (hipMemcpy(loss, W->scal, 4, hipMemcpyDeviceToHost) != hipSuccess) return GSLS_ERR_HIP;
  }
  return GSLS_OK;
}

int32_t gsls_ws_batch_rows(gsls_batch* b) {
  if (!b) return GSLS_ERR_INVALID_ARG;
  return b->s.row_off.empty() ? 0 : b->s.row_off.back();
}

static int ws_check_batch(gsls_batch* b) {
  for (const gsls::BInst& I : b->s.inst)
    if (!I.box || I.nx > gsls::kXs || I.nu > gsls::kUs) return GSLS_ERR_INVALID_ARG;
  return GSLS_OK;
}

int gsls_ws_features(gsls_ws* h, gsls_batch* b, const double* const* x0, uint16_t* X) {
  if (!h || !b || !X) return GSLS_ERR_INVALID_ARG;
  int rc = ws_check_batch(b);
  if (rc) return rc;
  if (x0 && (rc = gsls::batch_upload_x0(&b->s, x0))) return rc;
  const int rows = gsls_ws_batch_rows(b);
  gsls::k_ws_features<<<(rows + 3) / 4, 256, 0, b->s.stream>>>(b->s.d_inst, b->s.fp, b->s.dp, b->s.d_row_inst,
                                                               b->s.d_row_off, rows, h->w.sketch, X);
  if (hipGetLastError() != hipSuccess) return GSLS_ERR_HIP;
  if (hipStreamSynchronize(b->s.stream) != hipSuccess) return GSLS_ERR_HIP;
  return GSLS_OK;
}

int gsls_ws_targets(gsls_batch* b, float* T, float* M) {
  if (!b || !T || !M) return GSLS_ERR_INVALID_ARG;
  int rc = ws_check_batch(b);
  if (rc) return rc;
  gsls::k_ws_targets<<<b->s.count, 256, 0, b->s.stream>>>(b->s.d_inst, b->s.dp, b->s.d_row_off, b->s.d_res, T, M);
  if (hipGetLastError() != hipSuccess) return GSLS_ERR_HIP;
  if (hipStreamSynchronize(b->s.stream) != hipSuccess) return GSLS_ERR_HIP;
  return GSLS_OK;
}

int gsls_qp_solve_batch_ws(gsls_batch* b, gsls_ws* h, const double* const* x0, double tol, int32_t warm_budget,
                           int32_t parts, gsls_result* out, double* ms, double* ms_predict) {
  if (!b || !h || !x0 || !out || !(tol >= 0) || warm_budget < 0 || parts < 1 || parts > 7)
    return GSLS_ERR_INVALID_ARG;
  int rc = ws_check_batch(b);
  if (rc) return rc;
  gsls::BatchSolver* B = &b->s;
  if ((rc = gsls::batch_upload_x0(B, x0))) return rc;
  const int rows = gsls_ws_batch_rows(b);
  if ((rc = gsls::ws_reserve(&h->w, rows, false))) return rc;
  hipStream_t saved = h->w.stream;
  h->w.stream = B->stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return GSLS_ERR_HIP;
  (void)hipEventRecord(e0, B->stream);
  gsls::k_ws_features<<<(rows + 3) / 4, 256, 0, B->stream>>>(B->d_inst, B->fp, B->dp, B->d_row_inst, B->d_row_off,
                                                             rows, h->w.sketch, h->w.Xw);
  gsls::ws_forward(&h->w, h->w.Xw, nullptr, rows, h->w.Y);
  gsls::k_ws_scatter<<<B->count, 256, 0, B->stream>>>(B->d_inst, B->dp, B->d_row_off, h->w.Y, B->st.rho_min,
                                                      B->st.rho_max, B->d_rho, B->d_warm, parts);
  (void)hipEventRecord(e1, B->stream);
  h->w.stream = saved;
  if (hipGetLastError() != hipSuccess) return GSLS_ERR_HIP;
  double ms_solve = 0.0;
  rc = gsls::batch_run(B, tol, warm_budget, out, &ms_solve);
  float tp = 0.f;
  (void)hipEventElapsedTime(&tp, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (ms_predict) *ms_predict = tp;
  if (ms) *ms = ms_solve + tp;
  for (int c = 0; c < B->count; ++c) {
    out[c].ms_total = ms_solve + tp;
    b->rho_final[c] = out[c].rho;
  }
  return rc;
}

void gsls_ws_free(gsls_ws* h) { delete h; }

}  // extern "C"
