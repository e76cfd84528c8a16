// Batched ADMM QP solver: many independent LTV-QPs of uneven shape in one
// persistent launch (Sec. III-C / IV-A of the paper applied per instance).
//
// A workgroup pulls whole instances from a device work queue (largest first)
// and runs for each: the factor epoch (backward Riccati recursion with the
// augmented costs of eq. (augmented_matrices); stage inputs moved to LDS by
// DMA, products on the FP32 matrix cores, the nu x nu inverse in FP64), then
// ADMM iterations whose x-update evaluates the cached affine map of
// eq. (gains_cache) (backward pass for p, forward roll-out, sequential over
// the horizon inside the workgroup), the projection / dual update and the
// residuals, with the OSQP-style rho adaptation re-running the epoch when rho
// changes.  An instance that outlasts its solo budget is handed to a gang of
// workgroups that split its horizon into chunks combined by associative scans
// (the gangs section below).  State, projection and residuals are FP64; after the first
// iteration of each epoch the affine map is applied to the increment of
// w = y - z with FP64 accumulation (see iterate.hip).
//
// Box fast path: when every stage's rows are exactly [x; u] (C = [I; 0],
// D = [0; I]) and the terminal rows are x_N or absent, G = I and the
// products with G and G^T are skipped.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "dev_common.hpp"
#include "solver.hpp"
#include "batch.hpp"

namespace gsls {

constexpr int kBV = 128;       // work-vector length (>= nx + nu, >= nc)
constexpr int kBatchMaxNxu = 96;
constexpr int kGangMax = 32;          // workgroups per gang (6 kGangMax <= kWG: residual exchange)
constexpr int kGangAuto = 32;
constexpr double kParkShareAuto = 1.0;
// No hand-over once r_p, r_d <= kParkResid * tol: at the solo budget the
// residual's distance from the stopping test tracks the iterations still to
// run, and an instance this close finishes solo in fewer workgroup-seconds
// (and sooner) than a gang that must first assemble.
constexpr double kParkResid = 30.0;
// A hand-over whose rho is at least kPrioRho and has grown at least
// kPrioGrowth-fold since the start, with a residual still at least
// kPrioResid * tol, goes to the priority list, whose gangs are filled first:
// a penalty parameter driven up by the residual balance together with a
// residual far from the stopping test marks the ill-conditioned instances
// that run for many more iterations than the rest of the batch (its
// makespan).  A high rho that was the start value (a learned start) says less
// about the remaining iterations.
constexpr double kPrioRho = 50.0;
constexpr double kPrioGrowth = 4.0;
constexpr double kPrioResid = 300.0;

__host__ __device__ inline int bodd(int x) { return x | 1; }

// Per-stage packet of the cached iteration operators, one contiguous block per
// stage in the float pool: F = [[Abar, B], [K, I]] (odd leading dimension, so
// that both F x and F^T x read LDS without bank conflicts), Gamma, ev =
// Abar^T P b, fv = B^T P b, and the stage's constant data q, r, b.  The
// iterations stream these packets through LDS.
struct PkLayout {
  int ldF, F, Gam, ev, fv, q, r, b, stride;
};
__host__ __device__ inline PkLayout pk_layout(int nx, int nu) {
  PkLayout L;
  const int nxu = nx + nu;
  L.ldF = bodd(nxu);
  int o = 0;
  L.F = o; o += nxu * L.ldF;
  L.Gam = o; o += nu * nu;
  L.ev = o; o += nx;
  L.fv = o; o += nu;
  L.q = o; o += nx;
  L.r = o; o += nu;
  L.b = o; o += nx;
  L.stride = (o + 3) & ~3;
  return L;
}
constexpr int kPkVec = 11;      // 16-byte packet slices per thread (stride <= 44 * kWG)

struct BLayout {
  int ldP, ldW, ldZ, ldAB, ldG, ldY;
  size_t P, W, Z, AB, G, Y, pk0, pk1, vec, bytes;
  size_t aug, dg, perm, red;   // byte offsets: FP64 / int scratch of the epoch (in the
                               // W region) and the reduction buffer of the iterations
  size_t prof;                 // byte offset: 16 phase counters (profiling only)
};
// nc: rows held in the G buffer (0 on the box fast path, else max(nc, nf)).
// Float regions start on 16-byte boundaries.  The Gauss-Jordan block
// ([Z_uu | Z_ux | I] in FP64, pivots) lives in the W region, which is dead
// while it is in use.  The two packet buffers of the iterations alias the
// epoch's regions (the epoch and the iterations never overlap in time).
__host__ __device__ inline BLayout batch_layout(int nx, int nu, int nc) {
  BLayout L;
  const int nxu = nx + nu;
  L.ldP = bodd(nx); L.ldW = bodd(nxu); L.ldZ = bodd(nxu); L.ldAB = bodd(nxu); L.ldG = bodd(nxu);
  L.ldY = bodd(nx);
  auto r4 = [](size_t v) { return (v + 3) & ~(size_t)3; };
  const size_t aug_d = (size_t)nu * (2 * nu + nx), dg_d = 32, perm_d = 32;
  const size_t wfl = r4((size_t)(nx > nc ? nx : nc) * L.ldW);
  // the W region also holds the FP64 work space of the gain (nu^2 + 64 doubles and a flag)
  const size_t afl = 2 * std::max(aug_d + dg_d + perm_d, (size_t)nu * nu + 66);
  size_t o = 0;
  L.P = o; o += r4((size_t)nx * L.ldP);
  L.W = o; o += wfl > afl ? wfl : afl;
  L.Z = o; o += r4((size_t)nxu * L.ldZ);
  L.AB = o; o += r4((size_t)nx * L.ldAB);
  L.G = o; o += r4((size_t)nc * L.ldG);
  L.Y = o; o += r4((size_t)nu * L.ldY);
  const size_t pkf = (size_t)kPkVec * 4 * kWG;   // a packet buffer holds a full prefetch
  L.pk0 = 0;
  L.pk1 = pkf;
  if (o < 2 * pkf) o = 2 * pkf;
  L.vec = o; o += 8 * kBV + 512;   // the epoch uses [0, 384) for vectors and [1024, 1536) for partial sums
  o = r4(o);
  const size_t redf = o; o += 2 * (kWG + 8);
  const size_t proff = o; o += 2 * 16;
  L.bytes = o * 4;
  L.aug = L.W * 4;
  L.dg = L.aug + aug_d * 8;
  L.perm = L.dg + dg_d * 8;
  L.red = redf * 4;
  L.prof = proff * 4;
  return L;
}

// Dynamic LDS available to one workgroup of the batched kernel.
constexpr size_t kBatchLdsMax = 160 * 1024 - 512;

// Workgroup barrier for loops that keep a buffer-to-LDS copy in flight: waits
// for the thread's own LDS reads and writes only (lgkmcnt), then s_barrier.
// An LDS release fence (lds_barrier) would also wait for every outstanding
// copy into LDS (those count as LDS writes, tracked by vmcnt), i.e. for the
// prefetch this barrier is meant to overlap.  The copies only target the
// packet buffer that no thread reads before pk_dma_wait() and the barrier
// after it.  The signal fences keep the compiler from moving memory accesses
// across the barrier.
__device__ __forceinline__ void dma_barrier() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0); vmcnt, expcnt unconstrained
  __builtin_amdgcn_s_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Barrier of one wave over its own LDS accesses: waits for its LDS
// operations and keeps the compiler from moving LDS accesses across.
__device__ __forceinline__ void wave_lds_sync() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0)
  __builtin_amdgcn_wave_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

__device__ inline double wg_max_d(double v, LDS double* s) {
  s[tid()] = v;
  dma_barrier();
  for (int st = kWG / 2; st > 0; st >>= 1) {
    if (tid() < st) {
      double a = s[tid()], b = s[tid() + st];
      s[tid()] = (b > a || b != b) ? b : a;
    }
    dma_barrier();
  }
  double r = s[0];
  dma_barrier();
  return r;
}

// Work vectors of the iterations in LDS.
struct IterVecs {
  LDS float *g, *g2, *xz, *tv, *tu, *wv, *wv2, *part;
  LDS double* red;
  LDS unsigned long long* pc;
  LDS float *buf0, *buf1;   // the two packet buffers (selected, never indexed: an
                            // indexed pair would live in scratch memory, and
                            // reading it back waits for every outstanding
                            // memory operation of the wave)
  __device__ __forceinline__ LDS float* buf(int c) const { return c ? buf1 : buf0; }
};
__device__ __forceinline__ IterVecs iter_vecs(const BLayout& lay, LDS char* base) {
  IterVecs v;
  LDS float* F0 = (LDS float*)base;
  v.buf0 = F0 + lay.pk0;
  v.buf1 = F0 + lay.pk1;
  v.g = F0 + lay.vec;
  v.g2 = v.g + kBV;
  v.xz = v.g2 + kBV;
  v.tv = v.xz + kBV;
  v.tu = v.tv + kBV;
  v.wv = v.tu + kBV;
  v.wv2 = v.wv + kBV;
  v.part = v.wv2 + 2 * kBV;
  v.red = (LDS double*)(base + lay.red);
  v.pc = (LDS unsigned long long*)(base + lay.prof);
  return v;
}

// Optional phase profile: device clock between marks, summed per phase (LDS
// counters, thread 0).
struct PhaseMark {
  LDS unsigned long long* pc;
  bool on;
  unsigned long long last = 0;
  __device__ __forceinline__ void operator()(int ph) {
    if (on) {
      dma_barrier();
      const unsigned long long tn = __builtin_amdgcn_s_memtime();
      if (tid() == 0 && last) pc[ph] += tn - last;
      last = tn;
    }
  }
};

// Light GEMVs for operands already in LDS (or read rarely): the reduction is
// split over the four waves (row w + 4k), each thread keeping only a running
// sum, so they add little register pressure next to the packet prefetch.
// y = M^T x for M m x n (m any, n <= 128), y = M x for M m x n (m <= 128).
template <typename PM, typename PX, typename PY>
__device__ __forceinline__ void lite_gemv_t(int m, int n, PM M, int ld, PX x, PY y, LDS float* part) {
  // keep the per-call index arithmetic inside the caller's loops (hoisting it
  // out of a stage loop would hold many registers for the whole loop)
  asm volatile("" : "+v"(ld));
  const int lane = tid() & 63, w = tid() >> 6;
  for (int jb = 0; jb * 64 < n; ++jb) {
    const int j = jb * 64 + lane;
    const int jc = min(j, n - 1);
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    int i = w;
    for (; i + 12 < m; i += 16) {
      s0 += float(M[i * ld + jc]) * float(x[i]);
      s1 += float(M[(i + 4) * ld + jc]) * float(x[i + 4]);
      s2 += float(M[(i + 8) * ld + jc]) * float(x[i + 8]);
      s3 += float(M[(i + 12) * ld + jc]) * float(x[i + 12]);
    }
    for (; i < m; i += 4) s0 += float(M[i * ld + jc]) * float(x[i]);
    part[w * 128 + j] = (s0 + s1) + (s2 + s3);
  }
  dma_barrier();
  for (int j = tid(); j < n; j += kWG) y[j] = part[j] + part[128 + j] + part[256 + j] + part[384 + j];
  dma_barrier();
}
template <typename PM, typename PX, typename PY>
__device__ __forceinline__ void lite_gemv_n(int m, int n, PM M, int ld, PX x, PY y, LDS float* part, bool acc) {
  asm volatile("" : "+v"(ld));
  const int lane = tid() & 63, w = tid() >> 6;
  for (int ib = 0; ib * 64 < m; ++ib) {
    const int i = ib * 64 + lane;
    const int ic = min(i, m - 1);
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    int k = w;
    for (; k + 12 < n; k += 16) {
      s0 += float(M[ic * ld + k]) * float(x[k]);
      s1 += float(M[ic * ld + k + 4]) * float(x[k + 4]);
      s2 += float(M[ic * ld + k + 8]) * float(x[k + 8]);
      s3 += float(M[ic * ld + k + 12]) * float(x[k + 12]);
    }
    for (; k < n; k += 4) s0 += float(M[ic * ld + k]) * float(x[k]);
    part[w * 128 + i] = (s0 + s1) + (s2 + s3);
  }
  dma_barrier();
  for (int i = tid(); i < m; i += kWG) {
    const float v = part[i] + part[128 + i] + part[256 + i] + part[384 + i];
    y[i] = acc ? float(y[i]) + v : v;
  }
  dma_barrier();
}

// The same products for an LDS operand with every load of a thread issued
// before its first multiply (R = rows per wave, m <= 4R): one LDS latency per
// product instead of one per group of four rows.  y = M^T x (n <= 128 columns
// over the lanes, rows over the waves) and y = M x (m <= 128 rows over the
// lanes, columns over the waves).  Out-of-range terms load a clamped element
// and are masked to zero.
template <int R, bool TWO, bool SYNC, typename PM>
__device__ __forceinline__ void fgemv_t_r(int m, int n, PM M, int ld, const LDS float* x, LDS float* y,
                                          LDS float* part) {
  const int lane = tid() & 63, w = tid() >> 6;
  const int j0 = min(lane, n - 1), j1 = min(64 + lane, n - 1);
  float a0[R], a1[R], xv[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int i = min(w + 4 * q, m - 1);
    a0[q] = M[i * ld + j0];
    if (TWO) a1[q] = M[i * ld + j1];
    xv[q] = x[i];
  }
  float s0 = 0.f, s1 = 0.f;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const float xx = (w + 4 * q < m) ? xv[q] : 0.f;
    s0 += a0[q] * xx;
    if (TWO) s1 += a1[q] * xx;
  }
  part[w * 128 + lane] = s0;
  if (TWO) part[w * 128 + 64 + lane] = s1;
  dma_barrier();
  for (int j = tid(); j < n; j += kWG) y[j] = part[j] + part[128 + j] + part[256 + j] + part[384 + j];
  if (SYNC) dma_barrier();
}
template <bool SYNC = true, typename PM>
__device__ __forceinline__ void fgemv_t(int m, int n, PM M, int ld, const LDS float* x, LDS float* y,
                                        LDS float* part) {
  if (n > 64) {
    if (m <= 16) fgemv_t_r<4, true, SYNC>(m, n, M, ld, x, y, part);
    else if (m <= 32) fgemv_t_r<8, true, SYNC>(m, n, M, ld, x, y, part);
    else if (m <= 64) fgemv_t_r<16, true, SYNC>(m, n, M, ld, x, y, part);
    else fgemv_t_r<24, true, SYNC>(m, n, M, ld, x, y, part);
  } else {
    if (m <= 16) fgemv_t_r<4, false, SYNC>(m, n, M, ld, x, y, part);
    else if (m <= 32) fgemv_t_r<8, false, SYNC>(m, n, M, ld, x, y, part);
    else if (m <= 64) fgemv_t_r<16, false, SYNC>(m, n, M, ld, x, y, part);
    else fgemv_t_r<24, false, SYNC>(m, n, M, ld, x, y, part);
  }
}
template <int R, bool TWO, bool SYNC, typename PM>
__device__ __forceinline__ void fgemv_n_r(int m, int n, PM M, int ld, const LDS float* x, LDS float* y,
                                          LDS float* part) {
  const int lane = tid() & 63, w = tid() >> 6;
  const int i0 = min(lane, m - 1), i1 = min(64 + lane, m - 1);
  float a0[R], a1[R], xv[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int k = min(w + 4 * q, n - 1);
    a0[q] = M[i0 * ld + k];
    if (TWO) a1[q] = M[i1 * ld + k];
    xv[q] = x[k];
  }
  float s0 = 0.f, s1 = 0.f;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const float xx = (w + 4 * q < n) ? xv[q] : 0.f;
    s0 += a0[q] * xx;
    if (TWO) s1 += a1[q] * xx;
  }
  part[w * 128 + lane] = s0;
  if (TWO) part[w * 128 + 64 + lane] = s1;
  dma_barrier();
  for (int i = tid(); i < m; i += kWG) y[i] = part[i] + part[128 + i] + part[256 + i] + part[384 + i];
  if (SYNC) dma_barrier();
}
template <bool SYNC = true, typename PM>
__device__ __forceinline__ void fgemv_n(int m, int n, PM M, int ld, const LDS float* x, LDS float* y,
                                        LDS float* part) {
  if (m > 64) {
    if (n <= 16) fgemv_n_r<4, true, SYNC>(m, n, M, ld, x, y, part);
    else if (n <= 32) fgemv_n_r<8, true, SYNC>(m, n, M, ld, x, y, part);
    else if (n <= 64) fgemv_n_r<16, true, SYNC>(m, n, M, ld, x, y, part);
    else fgemv_n_r<24, true, SYNC>(m, n, M, ld, x, y, part);
  } else {
    if (n <= 16) fgemv_n_r<4, false, SYNC>(m, n, M, ld, x, y, part);
    else if (n <= 32) fgemv_n_r<8, false, SYNC>(m, n, M, ld, x, y, part);
    else if (n <= 64) fgemv_n_r<16, false, SYNC>(m, n, M, ld, x, y, part);
    else fgemv_n_r<24, false, SYNC>(m, n, M, ld, x, y, part);
  }
}

// One 16 x 16 output tile of op(A) op(B) on the matrix cores
// (v_mfma_f32_16x16x4f32: lane l supplies A[ic][k0 + l/16] and
// B[k0 + l/16][jc], ic / jc the lane's row / column clamped into range --
// rows and columns past the matrix are computed but never stored).  K runs in
// slabs of 4 KS steps whose LDS reads are all issued before the slab's
// products (one LDS latency per slab); full slabs read at fixed offsets from
// two base addresses with no masking, the last partial slab clamps its K
// index, zeroes the terms past k and skips its empty steps.
template <int KS, bool TA, bool TB>
__device__ __forceinline__ mfma_f4 tile_mm(int k, const LDS float* A, int lda, const LDS float* B, int ldb, int ic,
                                           int jc, int q) {
  const int sa = TA ? lda : 1, sb = TB ? 1 : ldb;   // strides along K
  const LDS float* pa = TA ? A + q * lda + ic : A + ic * lda + q;
  const LDS float* pb = TB ? B + jc * ldb + q : B + q * ldb + jc;
  mfma_f4 acc = {0.f, 0.f, 0.f, 0.f};
  int k0 = 0;
  for (; k0 + 4 * KS <= k; k0 += 4 * KS) {
    float av[KS], bv[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      av[s] = pa[(k0 + 4 * s) * sa];
      bv[s] = pb[(k0 + 4 * s) * sb];
    }
    // keep the slab's reads together: without this fence the scheduler
    // interleaves them with the products (one LDS round trip per product)
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int s = 0; s < KS; ++s) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s], bv[s], acc, 0, 0, 0);
  }
  if (k0 < k) {
    // the complete 4-steps left at fixed offsets, the last partial step
    // (k % 4 != 0) clamped and zeroed past k
    const int gfull = (k - k0) >> 2;   // < KS
    const int kp = k0 + 4 * gfull;
    float av[KS], bv[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s)
      if (s < gfull) {
        av[s] = pa[(k0 + 4 * s) * sa];
        bv[s] = pb[(k0 + 4 * s) * sb];
      }
    float ap = 0.f, bp = 0.f;
    if (kp < k) {
      const int kc = min(kp + q, k - 1);
      const bool in = kp + q < k;
      const float va = TA ? A[kc * lda + ic] : A[ic * lda + kc];
      const float vb = TB ? B[jc * ldb + kc] : B[kc * ldb + jc];
      ap = in ? va : 0.f;
      bp = in ? vb : 0.f;
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int s = 0; s < KS; ++s)
      if (s < gfull) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s], bv[s], acc, 0, 0, 0);
    if (kp < k) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ap, bp, acc, 0, 0, 0);
  }
  return acc;
}

// Two output tiles at once (tile_mm's scheme): their products alternate, so
// the two accumulation chains overlap on the matrix core (a dependent
// 16x16x4 product waits for its predecessor; two chains issue back to back).
template <int KS, bool TA, bool TB>
__device__ __forceinline__ void tile_mm2(int k, const LDS float* A, int lda, const LDS float* B, int ldb, int ic0,
                                         int jc0, int ic1, int jc1, int q, mfma_f4& acc0, mfma_f4& acc1) {
  const int sa = TA ? lda : 1, sb = TB ? 1 : ldb;
  const LDS float* pa0 = TA ? A + q * lda + ic0 : A + ic0 * lda + q;
  const LDS float* pb0 = TB ? B + jc0 * ldb + q : B + q * ldb + jc0;
  const LDS float* pa1 = TA ? A + q * lda + ic1 : A + ic1 * lda + q;
  const LDS float* pb1 = TB ? B + jc1 * ldb + q : B + q * ldb + jc1;
  acc0 = mfma_f4{0.f, 0.f, 0.f, 0.f};
  acc1 = mfma_f4{0.f, 0.f, 0.f, 0.f};
  int k0 = 0;
  for (; k0 + 4 * KS <= k; k0 += 4 * KS) {
    float a0[KS], b0[KS], a1[KS], b1[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      a0[s] = pa0[(k0 + 4 * s) * sa];
      b0[s] = pb0[(k0 + 4 * s) * sb];
      a1[s] = pa1[(k0 + 4 * s) * sa];
      b1[s] = pb1[(k0 + 4 * s) * sb];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[s], b0[s], acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[s], b1[s], acc1, 0, 0, 0);
    }
  }
  if (k0 < k) {
    const int gfull = (k - k0) >> 2;
    const int kp = k0 + 4 * gfull;
    float a0[KS], b0[KS], a1[KS], b1[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s)
      if (s < gfull) {
        a0[s] = pa0[(k0 + 4 * s) * sa];
        b0[s] = pb0[(k0 + 4 * s) * sb];
        a1[s] = pa1[(k0 + 4 * s) * sa];
        b1[s] = pb1[(k0 + 4 * s) * sb];
      }
    float ap0 = 0.f, bp0 = 0.f, ap1 = 0.f, bp1 = 0.f;
    if (kp < k) {
      const int kc = min(kp + q, k - 1);
      const bool in = kp + q < k;
      const float va0 = TA ? A[kc * lda + ic0] : A[ic0 * lda + kc];
      const float vb0 = TB ? B[jc0 * ldb + kc] : B[kc * ldb + jc0];
      const float va1 = TA ? A[kc * lda + ic1] : A[ic1 * lda + kc];
      const float vb1 = TB ? B[jc1 * ldb + kc] : B[kc * ldb + jc1];
      ap0 = in ? va0 : 0.f;
      bp0 = in ? vb0 : 0.f;
      ap1 = in ? va1 : 0.f;
      bp1 = in ? vb1 : 0.f;
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int s = 0; s < KS; ++s)
      if (s < gfull) {
        acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[s], b0[s], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[s], b1[s], acc1, 0, 0, 0);
      }
    if (kp < k) {
      acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(ap0, bp0, acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(ap1, bp1, acc1, 0, 0, 0);
    }
  }
}

// C = alpha op(A) op(B) + beta C on the matrix cores for LDS operands with
// k <= 96: 16 x 16 output tiles round-robin over the waves (tile_mm).  C may
// share an array with A or B but not their elements.  Ends with a barrier.
template <int KS, bool TA, bool TB, typename PC>
__device__ __forceinline__ void mm_pl_k(int m, int n, int k, float alpha, const LDS float* A, int lda,
                                        const LDS float* B, int ldb, float beta, PC C, int ldc) {
  const int l = lane(), w = wave();
  const int tn = (n + 15) >> 4, tm = (m + 15) >> 4;
  const int r16 = l & 15, q = l >> 4;
  const int T = tm * tn;
  auto store = [&](int ti, int tj, const mfma_f4& acc) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int ii = ti * 16 + 4 * q + r, jj = tj * 16 + r16;
      if (ii < m && jj < n) {
        float v = alpha * acc[r];
        if (beta != 0.f) v += beta * C[ii * ldc + jj];
        C[ii * ldc + jj] = v;
      }
    }
  };
  // the wave's tiles w, w + 4, ... in pairs
  for (int t = w; t < T; t += 8) {
    const int ti0 = t / tn, tj0 = t - ti0 * tn;
    const int ic0 = min(ti0 * 16 + r16, m - 1), jc0 = min(tj0 * 16 + r16, n - 1);
    if (t + 4 < T) {
      const int ti1 = (t + 4) / tn, tj1 = (t + 4) - ti1 * tn;
      const int ic1 = min(ti1 * 16 + r16, m - 1), jc1 = min(tj1 * 16 + r16, n - 1);
      mfma_f4 acc0, acc1;
      tile_mm2<KS, TA, TB>(k, A, lda, B, ldb, ic0, jc0, ic1, jc1, q, acc0, acc1);
      store(ti0, tj0, acc0);
      store(ti1, tj1, acc1);
    } else {
      store(ti0, tj0, tile_mm<KS, TA, TB>(k, A, lda, B, ldb, ic0, jc0, q));
    }
  }
  __syncthreads();
}
template <bool TA, bool TB, typename PC>
__device__ __forceinline__ void mm_pl(int m, int n, int k, float alpha, const LDS float* A, int lda,
                                      const LDS float* B, int ldb, float beta, PC C, int ldc) {
  if (k <= 4) mm_pl_k<1, TA, TB>(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc);
  else if (k <= 16) mm_pl_k<4, TA, TB>(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc);
  else mm_pl_k<10, TA, TB>(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc);
}

// Symmetric product C_out = alpha op(A) op(B) + beta C_in for a result known
// to be symmetric (n x n): only the tiles on and above the diagonal are
// formed, and each value is written to both (i, j) and (j, i), so the result
// is exactly symmetric.  C_in may be C_out (every thread reads only the
// elements on and above the diagonal it then writes).
template <int KS, bool TA, bool TB, typename PC>
__device__ __forceinline__ void mm_sym_pl_k(int n, int k, float alpha, const LDS float* A, int lda,
                                            const LDS float* B, int ldb, float beta, const LDS float* Cin,
                                            int ldi, PC Cout, int ldo) {
  const int l = lane(), w = wave();
  const int tn = (n + 15) >> 4;
  const int r16 = l & 15, q = l >> 4;
  const int tiles = tn * (tn + 1) / 2;
  auto tile_of = [&](int t, int& ti, int& tj) {   // upper tile t in row-major order of the upper triangle
    ti = 0;
    int rem = t;
    while (rem >= tn - ti) {
      rem -= tn - ti;
      ++ti;
    }
    tj = ti + rem;
  };
  auto store = [&](int ti, int tj, const mfma_f4& acc) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int ii = ti * 16 + 4 * q + r, jj = tj * 16 + r16;
      if (ii < n && jj < n && ii <= jj) {
        float v = alpha * acc[r];
        if (beta != 0.f) v += beta * Cin[ii * ldi + jj];
        Cout[ii * ldo + jj] = v;
        Cout[jj * ldo + ii] = v;
      }
    }
  };
  for (int t = w; t < tiles; t += 8) {
    int ti0, tj0;
    tile_of(t, ti0, tj0);
    const int ic0 = min(ti0 * 16 + r16, n - 1), jc0 = min(tj0 * 16 + r16, n - 1);
    if (t + 4 < tiles) {
      int ti1, tj1;
      tile_of(t + 4, ti1, tj1);
      const int ic1 = min(ti1 * 16 + r16, n - 1), jc1 = min(tj1 * 16 + r16, n - 1);
      mfma_f4 acc0, acc1;
      tile_mm2<KS, TA, TB>(k, A, lda, B, ldb, ic0, jc0, ic1, jc1, q, acc0, acc1);
      store(ti0, tj0, acc0);
      store(ti1, tj1, acc1);
    } else {
      store(ti0, tj0, tile_mm<KS, TA, TB>(k, A, lda, B, ldb, ic0, jc0, q));
    }
  }
  __syncthreads();
}
template <bool TA, bool TB, typename PC>
__device__ __forceinline__ void mm_sym_pl(int n, int k, float alpha, const LDS float* A, int lda, const LDS float* B,
                                          int ldb, float beta, const LDS float* Cin, int ldi, PC Cout, int ldo) {
  if (k <= 4) mm_sym_pl_k<1, TA, TB>(n, k, alpha, A, lda, B, ldb, beta, Cin, ldi, Cout, ldo);
  else if (k <= 16) mm_sym_pl_k<4, TA, TB>(n, k, alpha, A, lda, B, ldb, beta, Cin, ldi, Cout, ldo);
  else mm_sym_pl_k<10, TA, TB>(n, k, alpha, A, lda, B, ldb, beta, Cin, ldi, Cout, ldo);
}

__device__ __forceinline__ void pk_dma_wait() { __builtin_amdgcn_s_waitcnt(0); }

// Linear global -> LDS copy by DMA of n floats (n a multiple of 4, both ends
// 16-byte aligned): float e lands at dst[e].  Lanes past n issue nothing.
// Completion: pk_dma_wait() (all of the wave's vector memory operations),
// then a barrier.
__device__ __forceinline__ void lds_dma_issue(const float* src, int n, LDS float* dst) {
  src = uniform_ptr(src);
  n = __builtin_amdgcn_readfirstlane(n);
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void*)src, (short)0, n * 4, 0x00020000);
  // the LDS destination (M0) computed on the scalar unit: a wave-uniform
  // wave index, so no vector -> scalar round trip per copy
  dst = uniform_lds(dst);
  const int w = __builtin_amdgcn_readfirstlane((int)tid() >> 6);
  const int vo = (int)tid() * 16;
#pragma unroll
  for (int q = 0; q < 10; ++q)
    if (q * kWG * 4 + (int)tid() * 4 < n)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (LDS void*)(dst + q * kWG * 4 + w * 256), 16, vo, q * kWG * 16, 0,
                                               0);
}

// Gain of one Riccati stage for a small control dimension (n = nu <= 2 TM):
//   Gamma = Z_uu^{-1} in FP64 by wave 0 -- Gauss-Jordan steps without pivot
//   search, every pivot of the symmetric positive definite Z_uu being a
//   positive Schur complement (a non-positive or non-finite pivot reports
//   "not positive definite").  Lane l holds the elements (2t + l/32, l%32),
//   t < TM.  Before step p, the pivot row equals the pivot column with the
//   sign flipped on the columns already eliminated, so only the column is
//   exchanged (through LDS), and the iterate keeps that (anti)symmetry
//   exactly; Gamma comes out exactly symmetric.
//   K = -Gamma Z_ux, summed in FP64 by all waves, rounded once to FP32.
// Z holds the stage's Z = [[Z_xx, Z_xu], [Z_ux, Z_uu]] (FP32, leading
// dimension ldz); ws: FP64 LDS work space of n^2 + 64 doubles + a flag.
// Outputs: K (n x nx, ldk) in LDS and Gamma (n x n) in the packet.  Returns
// false (uniformly) if Z_uu is not positive definite.  Ends with a barrier.
template <int TM>
__device__ __forceinline__ bool stage_gain(int nx, int n, const LDS float* Z, int ldz, LDS double* ws, LDS float* K,
                                           int ldk, float* Gam) {
  LDS double* gam = ws;
  LDS double* cb = ws + n * n;
  LDS int* flag = (LDS int*)(cb + 64);
  const int l = lane(), kk = l & 31, h = l >> 5;
  const LDS float* Zuu = Z + nx * ldz + nx;
  if (wave() == 0) {
    double a[TM];
#pragma unroll
    for (int t = 0; t < TM; ++t) {
      const int i = 2 * t + h;
      a[t] = (i < n && kk < n) ? 0.5 * ((double)Zuu[i * ldz + kk] + (double)Zuu[kk * ldz + i]) : 0.0;
    }
    int ok = 1;
    for (int p = 0; p < n; ++p) {
      LDS double* col = cb + (p & 1) * 32;
      if (kk == p) {
#pragma unroll
        for (int t = 0; t < TM; ++t) col[2 * t + h] = a[t];   // entries past n are never used
      }
      wave_lds_sync();
      const double d = col[p];
      if (!(d > 0.0) || !isfinite(d)) {
        ok = 0;
        break;
      }
      const double r = 1.0 / d;
      const double ck = col[min(kk, n - 1)];
      const double rowk = kk < p ? -ck : ck;   // the pivot row's element in column kk
      const bool kp = kk == p;
      const double rowv = rowk * r;
#pragma unroll
      for (int t = 0; t < TM; ++t) {
        // branch-free: the general update, then the pivot column, row and element
        const int i = 2 * t + h;
        const bool ip = i == p;
        const double ci = col[min(i, n - 1)];
        double v = a[t] - (ci * rowk) * r;
        v = kp ? -ci * r : v;
        v = ip ? rowv : v;
        v = (ip && kp) ? r : v;
        a[t] = v;
      }
    }
    if (ok) {
#pragma unroll
      for (int t = 0; t < TM; ++t) {
        const int i = 2 * t + h;
        if (i < n && kk < n) gam[i * n + kk] = a[t];
      }
    }
    if (l == 0) *flag = ok;
  }
  __syncthreads();
  if (!*flag) return false;
  // K = -Gamma Z_ux: thread (wave w, lane l) takes columns l, l + 64 and rows w, w + 4, ...
  for (int cb0 = 0; cb0 < nx; cb0 += 64) {
    const int c = cb0 + l, cc = min(c, nx - 1);
    float z[2 * TM];
#pragma unroll
    for (int j = 0; j < 2 * TM; ++j) z[j] = Z[(nx + min(j, n - 1)) * ldz + cc];   // Z_ux column c
    for (int r = wave(); r < n; r += 4) {
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < 2 * TM; ++j)
        if (j < n) s += gam[r * n + j] * (double)z[j];
      if (c < nx) K[r * ldk + c] = (float)(-s);
    }
  }
  for (int e = tid(); e < n * n; e += kWG) Gam[e] = (float)gam[e];
  __syncthreads();
  return true;
}

// Factor epoch of one instance for penalty rho.  Returns false if a Z_uu block
// is not positive definite.
__device__ __attribute__((noinline)) bool batch_epoch(const BInst* __restrict__ Ip, const BatchArgs* __restrict__ ag,
                                                     double rho, LDS char* base) {
  Ip = uniform_ptr(Ip);
  ag = uniform_ptr(ag);
  const BInst& I = *Ip;
  const BatchArgs& a = *ag;
  const int N = I.N, nx = I.nx, nu = I.nu, nc = I.nc, nf = I.nf, nxu = nx + nu;
  const BLayout lay = batch_layout(nx, nu, I.box ? 0 : (nc > nf ? nc : nf));
  LDS float* F0 = (LDS float*)base;
  LDS float* P = F0 + lay.P;
  LDS float* W = F0 + lay.W;
  LDS float* Z = F0 + lay.Z;
  LDS float* AB = F0 + lay.AB;
  LDS float* G = F0 + lay.G;
  LDS float* Y = F0 + lay.Y;
  LDS float* vec = F0 + lay.vec;
  LDS double* aug = (LDS double*)(base + lay.aug);
  LDS double* dg = (LDS double*)(base + lay.dg);
  LDS int* perm = (LDS int*)(base + lay.perm);
  LDS int* used = perm + 32;
  float* fp = a.fp;
  const float fr = (float)rho;
  const IterVecs V = iter_vecs(lay, base);
  PhaseMark mark{V.pc, a.prof != nullptr};
  if (a.prof && tid() < 4) V.pc[12 + tid()] = 0ull;
  // P_N = Q_N + rho C_N^T C_N
  const float* QN = fp + I.oQN;
  for (int r = wave(); r < nx; r += 4)
    for (int c = lane(); c < nx; c += 64) P[r * lay.ldP + c] = QN[(size_t)r * nx + c];
  __syncthreads();
  if (nf > 0) {
    if (I.box) {
      for (int r = tid(); r < nx; r += kWG) P[r * lay.ldP + r] += fr;
    } else {
      const float* CN = fp + I.oCN;
      for (int r = wave(); r < nf; r += 4)
        for (int c = lane(); c < nx; c += 64) G[r * lay.ldG + c] = CN[(size_t)r * nx + c];
      __syncthreads();
      wg_mm_f32(nx, nx, nf, fr, G, lay.ldG, true, G, lay.ldG, false, 1.f, P, lay.ldP);
    }
  }
  __syncthreads();
  const EpLayout ein = ep_layout(nx, nu);
  const int ld = ein.ld;   // = lay.ldAB = lay.ldZ = lay.ldW
  const PkLayout pk = pk_layout(nx, nu);
  LDS double* ws = (LDS double*)(base + lay.aug);   // FP64 work space of the gain (W is dead then)
  for (int k = N - 1; k >= 0; --k) {
    // stage input into LDS: [A | B] and the cost block by DMA (one memory
    // latency for both), G and b by plain loads
    const float* Ek = fp + I.oE + (size_t)k * ein.stride;
    lds_dma_issue(Ek + ein.AB, ein.Z - ein.AB, AB);
    lds_dma_issue(Ek + ein.Z, ein.stride - ein.Z, Z);
    if (!I.box) {
      const float* Gk = fp + I.oG + (size_t)k * nc * nxu;
      wg_block_pass<float>(nc, nxu, [&](int r, int c) { return Gk[(size_t)r * nxu + c]; },
                           [&](int r, int c, float v) { G[r * lay.ldG + c] = v; });
    }
    const float* bk = fp + I.ob + (size_t)k * nx;
    for (int c = tid(); c < nx; c += kWG) vec[128 + c] = bk[c];
    pk_dma_wait();
    __syncthreads();
    if (I.box)
      for (int r = tid(); r < nxu; r += kWG) Z[r * ld + r] += fr;   // + rho on the box rows
    mark(15);
    // Pb = P b_k (vec[0..nx))
    fgemv_n(nx, nx, P, lay.ldP, vec + 128, vec, vec + 1024);   // partial sums in vec[1024..1536)
    mark(12);
    // W = P [A | B];  Z = [A | B]^T W + [[Q, S^T], [S, R]] (+ rho I or rho G^T G), symmetric
    mm_pl<false, false>(nx, nxu, nx, 1.f, P, lay.ldP, AB, ld, 0.f, W, ld);
    mm_sym_pl<true, false>(nxu, nx, 1.f, AB, ld, W, ld, 1.f, Z, ld, Z, ld);
    if (!I.box && nc > 0) mm_sym_pl<true, false>(nxu, nc, fr, G, lay.ldG, G, lay.ldG, 1.f, Z, ld, Z, ld);
    mark(13);
    float* pkt = fp + I.oPk + (size_t)k * pk.stride;
    float* Gam = pkt + pk.Gam;
    // K = -Z_uu^{-1} Z_ux into Y, Gamma = Z_uu^{-1} into the packet
    bool ok;
    if (nu <= 4) ok = stage_gain<2>(nx, nu, Z, ld, ws, (LDS float*)Y, lay.ldY, Gam);
    else if (nu <= 8) ok = stage_gain<4>(nx, nu, Z, ld, ws, (LDS float*)Y, lay.ldY, Gam);
    else if (nu <= 12) ok = stage_gain<6>(nx, nu, Z, ld, ws, (LDS float*)Y, lay.ldY, Gam);
    else if (nu <= 16) ok = stage_gain<8>(nx, nu, Z, ld, ws, (LDS float*)Y, lay.ldY, Gam);
    else if (nu <= 20) ok = stage_gain<10>(nx, nu, Z, ld, ws, (LDS float*)Y, lay.ldY, Gam);
    else if (nu <= 32) ok = stage_gain<16>(nx, nu, Z, ld, ws, (LDS float*)Y, lay.ldY, Gam);
    else {
      // larger control dimensions: FP64 elimination of [Z_uu | Z_ux | I]
      const int lda = 2 * nu + nx;
      for (int r = wave(); r < nu; r += 4)
        for (int c = lane(); c < lda; c += 64) {
          double v;
          if (c < nu) v = 0.5 * ((double)Z[(nx + r) * ld + nx + c] + (double)Z[(nx + c) * ld + nx + r]);
          else if (c < nu + nx) v = (double)Z[(nx + r) * ld + (c - nu)];
          else v = (c - nu - nx == r) ? 1.0 : 0.0;
          aug[r * lda + c] = v;
        }
      __syncthreads();
      ok = wg_gj_eliminate(nu, lda, aug, false, perm, used, dg);
      if (ok) {
        wg_gj_extract<float>(nu, lda, aug, perm, dg, 0, nx, -1.0, (float*)Y, lay.ldY);
        wg_gj_extract<float>(nu, lda, aug, perm, dg, nx, nu, 1.0, Gam, nu);
      }
    }
    if (!ok) return false;
    mark(14);
    // Abar = A + B K in place in the A block of [A | B] (the B block is kept)
    mm_pl<false, false>(nx, nx, nu, 1.f, AB + nx, ld, Y, lay.ldY, 1.f, AB, ld);
    // F = [[A + B K, B], [K, I]]
    float* Fk = pkt + pk.F;
    wg_block_pass<float>(nxu, nxu, [&](int r, int c) {
                           if (r < nx) return AB[r * ld + c];
                           return c < nx ? Y[(r - nx) * lay.ldY + c] : (c - nx == r - nx ? 1.f : 0.f);
                         },
                         [&](int r, int c, float v) { Fk[(size_t)r * pk.ldF + c] = v; });
    // [ev; fv] = [Abar | B]^T P b
    fgemv_t(nx, nxu, AB, ld, vec, vec + 256, vec + 1024);
    float* ev = pkt + pk.ev;
    float* fv = pkt + pk.fv;
    for (int c = tid(); c < nxu; c += kWG) {
      if (c < nx) ev[c] = vec[256 + c];
      else fv[c - nx] = vec[256 + c];
    }
    // P = Z_xx + Z_ux^T K (symmetric)
    mm_sym_pl<true, false>(nx, nu, 1.f, Z + nx * ld, ld, Y, lay.ldY, 1.f, Z, ld, P, lay.ldP);
  }
  mark(15);
  if (a.prof && tid() < 4) atomicAdd(a.prof + 12 + tid(), V.pc[12 + tid()]);
  return true;
}

// Stage packets move global -> LDS by DMA (buffer loads with the LDS
// destination): no registers hold the data, so the copy of the next stage's
// packet runs while the current stage is processed.  Each 16-byte slice of
// wave w lands at M0 + 16 * lane with M0 = dst + slice * 1024 floats + w * 256
// floats, i.e. at the same offset as in global memory; reads past n floats
// return 0.  Completion: pk_dma_wait() (all of the wave's vector memory
// operations), then a barrier.
__device__ __forceinline__ void pk_dma_issue(const float* src, int n, LDS float* dst) {
  src = uniform_ptr(src);
  n = __builtin_amdgcn_readfirstlane(n);
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void*)src, (short)0, n * 4, 0x00020000);
  // the LDS destination (M0) computed on the scalar unit: a wave-uniform
  // wave index, so no vector -> scalar round trip per copy
  dst = uniform_lds(dst);
  const int w = __builtin_amdgcn_readfirstlane((int)tid() >> 6);
  const int vo = (int)tid() * 16;
#pragma unroll
  for (int q = 0; q < kPkVec; ++q)
    if (q * kWG * 4 < n)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (LDS void*)(dst + q * kWG * 4 + w * 256), 16, vo, q * kWG * 16, 0,
                                               0);
}


// Backward pass of one cached iteration (Sec. IV-A) over the stages [s, e):
// p_N = cst q_N + rho C_N^T dw_N when e = N (else p_e is the caller's entry
// in V.g, or zero in fold mode), then per stage k = e-1..s, from the stage
// packet in LDS,
//   F^T [p; r_hat] = [Abar^T p + K^T r_hat; B^T p + r_hat]  (F = [[Abar, B], [K, I]]),
//   p_k = Abar^T p + K^T r_hat + cst (q_k + ev_k) + rho C_k^T dw,
//   k_k = -Gamma (B^T p + r_hat + cst fv_k),  r_hat = cst r_k + rho D_k^T dw,
// with dw the increment of w = y - z (w itself on a full evaluation, cst = 1).
// Writes k_k to the feed-forward store and w to the previous-w store.  Fold
// mode (a chunk of a horizon shared by several workgroups) runs the p
// recurrence alone from a zero entry and writes nothing; p_s is left in V.g.
// Thread r handles constraint row r of every stage (so its global reads are
// its own writes: LDS-only barriers).
template <bool BOX>
__device__ __attribute__((noinline)) void batch_backward(const BInst* __restrict__ Ip,
                                                         const BatchArgs* __restrict__ ag, float fr, bool full,
                                                         LDS char* base, int s, int e, bool fold) {
  Ip = uniform_ptr(Ip);
  ag = uniform_ptr(ag);
  s = uniform_int(s);
  e = uniform_int(e);
  fold = uniform_int(fold ? 1 : 0) != 0;
  const BInst& I = *Ip;
  const BatchArgs& a = *ag;
  const int N = I.N, nx = I.nx, nu = I.nu, nc = I.nc, nf = I.nf, nxu = nx + nu;
  const BLayout lay = batch_layout(nx, nu, BOX ? 0 : (nc > nf ? nc : nf));
  const PkLayout pk = pk_layout(nx, nu);
  const int pst = pk.stride;
  const IterVecs V = iter_vecs(lay, base);
  const float* fp = a.fp;
  double* dp = a.dp;
  const float* pkt = fp + I.oPk;
  const GLB double* ys = (const GLB double*)(dp + I.oy);
  const GLB double* zs = (const GLB double*)(dp + I.oz);
  GLB double* wprev = (GLB double*)(dp + I.owp);
  GLB float* kff = (GLB float*)(a.fp + I.okff);
  const float cst = full ? 1.f : 0.f;
  const int t = tid();
  PhaseMark mark{V.pc, a.prof != nullptr};
  if (e == N) {
    for (int r = t; r < nf; r += kWG) {
      const size_t gr = (size_t)N * nc + r;
      const double w = ys[gr] - zs[gr];
      V.wv[r] = (float)(full ? w : w - wprev[gr]);
      if (!fold) wprev[gr] = w;
    }
    dma_barrier();
    if (nf > 0 && !BOX) lite_gemv_t(nf, nx, (const float*)(fp + I.oCN), nx, V.wv, V.tv, V.part);
    for (int j = t; j < nx; j += kWG) {
      const float cw = nf > 0 ? (BOX ? V.wv[j] : V.tv[j]) : 0.f;
      V.g[j] = cst * fp[I.oq + (size_t)N * nx + j] + fr * cw;
    }
  } else if (fold) {
    for (int j = t; j < nx; j += kWG) V.g[j] = 0.f;
  }
  if (s >= e) {
    dma_barrier();
    return;
  }
  pk_dma_issue(pkt + (size_t)(e - 1) * pst, pst, V.buf0);
  double ry = 0.0, rz = 0.0, rw = 0.0;
  if (t < nc) {
    const size_t gr = (size_t)(e - 1) * nc + t;
    ry = ys[gr]; rz = zs[gr]; rw = wprev[gr];
  }
  pk_dma_wait();
  dma_barrier();
  int cb = 0;
  for (int i = e - 1; i >= s; --i) {
    LDS float* P = V.buf(cb);
    double ny = 0.0, nz = 0.0, nw = 0.0;
    if (i > s) {
      pk_dma_issue(pkt + (size_t)(i - 1) * pst, pst, V.buf(cb ^ 1));
      if (t < nc) {
        const size_t gr = (size_t)(i - 1) * nc + t;
        ny = ys[gr]; nz = zs[gr]; nw = wprev[gr];
      }
    }
    mark(0);
    if (t < nc) {
      const double w = ry - rz;
      V.wv[t] = (float)(full ? w : w - rw);
      if (!fold) wprev[(size_t)i * nc + t] = w;
    }
    dma_barrier();
    mark(1);
    if (!BOX) {
      if (nc > 0) {
        lite_gemv_t(nc, nxu, (const float*)(fp + I.oG + (size_t)i * nc * nxu), nxu, V.wv, V.tv, V.part);
      } else {
        for (int j = t; j < nxu; j += kWG) V.tv[j] = 0.f;
        dma_barrier();
      }
    }
    // xz = [p; r_hat],  wv2 = q_hat + ev (state part of c_k without K^T r_hat)
    for (int j = t; j < nxu; j += kWG) {
      const float gw = BOX ? V.wv[j] : V.tv[j];
      if (j < nx) {
        V.xz[j] = V.g[j];
        V.wv2[j] = cst * (P[pk.q + j] + P[pk.ev + j]) + fr * gw;
      } else {
        V.xz[j] = cst * P[pk.r + (j - nx)] + fr * gw;
      }
    }
    dma_barrier();
    mark(2);
    fgemv_t(nxu, fold ? nx : nxu, (const LDS float*)(P + pk.F), pk.ldF, V.xz, V.g2, V.part);
    mark(3);
    if (fold) {
      for (int j = t; j < nx; j += kWG) V.g[j] = V.g2[j] + V.wv2[j];
    } else {
      for (int j = t; j < nxu; j += kWG) {
        if (j < nx) V.g[j] = V.g2[j] + V.wv2[j];
        else V.tu[j - nx] = V.g2[j] + cst * P[pk.fv + (j - nx)];
      }
      dma_barrier();
      lite_gemv_t(nu, nu, (const LDS float*)(P + pk.Gam), nu, V.tu, V.g2, V.part);
      for (int j = t; j < nu; j += kWG) kff[(size_t)i * nu + j] = -V.g2[j];
    }
    mark(4);
    ry = ny; rz = nz; rw = nw;
    pk_dma_wait();
    dma_barrier();
    mark(5);
    cb ^= 1;
  }
}

// |H xi| on the accumulated iterate (rho rule's dual scale): max over the
// stages [s, e) of |Q x + S^T u| and |S x + R u| (and Q_N x_N when e = N).
// Returns the workgroup maximum.
__device__ __attribute__((noinline)) double batch_hxi(const BInst* __restrict__ Ip,
                                                      const BatchArgs* __restrict__ ag, LDS char* base, int s,
                                                      int e) {
  Ip = uniform_ptr(Ip);
  ag = uniform_ptr(ag);
  s = uniform_int(s);
  e = uniform_int(e);
  const BInst& I = *Ip;
  const BatchArgs& a = *ag;
  const int N = I.N, nx = I.nx, nu = I.nu, nc = I.nc, nf = I.nf;
  const BLayout lay = batch_layout(nx, nu, I.box ? 0 : (nc > nf ? nc : nf));
  const IterVecs V = iter_vecs(lay, base);
  const EpLayout ep = ep_layout(nx, nu);
  const float* fp = a.fp;
  const GLB double* X = (const GLB double*)(a.dp + I.oX);
  const GLB double* U = (const GLB double*)(a.dp + I.oU);
  const int t = tid();
  double hx = 0.0;
  const int last = e == N ? N : e - 1;
  for (int i = s; i <= last; ++i) {
  const bool term = i == N;
  for (int j = t; j < nx; j += kWG) V.tv[j] = (float)X[(size_t)i * nx + j];
  if (!term)
    for (int j = t; j < nu; j += kWG) V.tu[j] = (float)U[(size_t)i * nu + j];
  dma_barrier();
  // stage cost blocks from the epoch input packet (Q_N on its own)
  const float* Zc = fp + I.oE + (size_t)(term ? 0 : i) * ep.stride + ep.Z;
  const float* Qi = term ? (const float*)(fp + I.oQN) : Zc;
  lite_gemv_n(nx, nx, Qi, term ? nx : ep.ld, V.tv, V.wv2, V.part, false);
  if (!term) {
    const float* Si = Zc + (size_t)nx * ep.ld;   // S_i: rows nx.. of the cost block, columns 0..nx-1
    lite_gemv_t(nu, nx, Si, ep.ld, V.tu, V.wv, V.part);
    for (int j = t; j < nx; j += kWG) V.wv2[j] += V.wv[j];
    lite_gemv_n(nu, nu, Si + nx, ep.ld, V.tu, V.g, V.part, false);
    lite_gemv_n(nu, nx, Si, ep.ld, V.tv, V.g, V.part, true);
    for (int j = t; j < nu; j += kWG) hx = fmax(hx, fabs((double)V.g[j]));
  }
  for (int j = t; j < nx; j += kWG) hx = fmax(hx, fabs((double)V.wv2[j]));
  dma_barrier();
  }
  return wg_max_d(hx, V.red);
}

// ----------------------------------------------------------------------
// Box-row stage passes.  When every stage's rows are exactly [x; u] the
// iteration needs no constraint products, and each stage's other work can be
// arranged so that every thread reads back only what it wrote itself or what
// the stage product's own closing barrier published: a backward stage then
// needs four workgroup barriers and a forward stage four (two of them inside
// the product), about half of the general path's.


// sum_q Gm[q][t] u[q] over q < nu <= QM, in order of q: every read issued
// before the first product (clamped indices, terms past nu dropped).
template <int QM>
__device__ __forceinline__ float gam_dot(const LDS float* Gm, const LDS float* u, int nu, int t) {
  float g[QM], v[QM];
#pragma unroll
  for (int q = 0; q < QM; ++q) {
    const int qq = min(q, nu - 1);
    g[q] = Gm[qq * nu + t];
    v[q] = u[qq];
  }
  float s = 0.f;
#pragma unroll
  for (int q = 0; q < QM; ++q)
    if (q < nu) s += g[q] * v[q];
  return s;
}

// Backward pass of box-row instances over [s, e) (semantics of
// batch_backward<true>).
__device__ __attribute__((noinline)) void box_backward(const BInst* __restrict__ Ip,
                                                       const BatchArgs* __restrict__ ag, float fr, bool full,
                                                       LDS char* base, int s, int e, bool fold) {
  Ip = uniform_ptr(Ip);
  ag = uniform_ptr(ag);
  s = uniform_int(s);
  e = uniform_int(e);
  fold = uniform_int(fold ? 1 : 0) != 0;
  const BInst& I = *Ip;
  const BatchArgs& a = *ag;
  const int N = I.N, nx = I.nx, nu = I.nu, nc = I.nc, nf = I.nf, nxu = nx + nu;
  const BLayout lay = batch_layout(nx, nu, 0);
  const PkLayout pk = pk_layout(nx, nu);
  const int pst = pk.stride;
  const IterVecs V = iter_vecs(lay, base);
  const float* fp = a.fp;
  double* dp = a.dp;
  const float* pkt = fp + I.oPk;
  const GLB double* ys = (const GLB double*)(dp + I.oy);
  const GLB double* zs = (const GLB double*)(dp + I.oz);
  GLB double* wprev = (GLB double*)(dp + I.owp);
  GLB float* kff = (GLB float*)(a.fp + I.okff);
  const float cst = full ? 1.f : 0.f;
  const int t = tid(), w = wave();
  PhaseMark mark{V.pc, a.prof != nullptr};
  if (e == N) {
    // p_N = cst q_N + rho dw_N on the terminal rows x_N (if any)
    for (int j = t; j < nx; j += kWG) {
      float cw = 0.f;
      if (j < nf) {
        const size_t gr = (size_t)N * nc + j;
        const double wn = ys[gr] - zs[gr];
        cw = (float)(full ? wn : wn - wprev[gr]);
        if (!fold) wprev[gr] = wn;
      }
      V.g[j] = cst * fp[I.oq + (size_t)N * nx + j] + fr * cw;
    }
  } else if (fold) {
    for (int j = t; j < nx; j += kWG) V.g[j] = 0.f;
  }
  if (s >= e) {
    dma_barrier();
    return;
  }
  pk_dma_issue(pkt + (size_t)(e - 1) * pst, pst, V.buf0);
  double ry = 0.0, rz = 0.0, rw = 0.0;
  if (t < nc) {
    const size_t gr = (size_t)(e - 1) * nc + t;
    ry = ys[gr]; rz = zs[gr]; rw = wprev[gr];
  }
  // r_k of input row t (the packet holds the same values; reading it from the
  // problem data lets the input vector of a stage be formed before its packet
  // has arrived)
  const float* rk = fp + I.orr;
  auto dw_of = [&](double y_, double z_, double w_) {
    const double wt = y_ - z_;
    return (float)(full ? wt : wt - w_);
  };
  // input vector [p; r_hat] of the first stage, own entries
  if (t < nx) V.xz[t] = V.g[t];
  else if (t < nc) V.xz[t] = cst * rk[(size_t)(e - 1) * nu + (t - nx)] + fr * dw_of(ry, rz, rw);
  pk_dma_wait();
  dma_barrier();
  int cb = 0;
  for (int i = e - 1; i >= s; --i) {
    LDS float* P = V.buf(cb);
    double ny = 0.0, nz = 0.0, nw = 0.0;
    float nr = 0.f;
    if (i > s) {
      pk_dma_issue(pkt + (size_t)(i - 1) * pst, pst, V.buf(cb ^ 1));
      if (t < nc) {
        const size_t gr = (size_t)(i - 1) * nc + t;
        ny = ys[gr]; nz = zs[gr]; nw = wprev[gr];
      }
      if (t >= nx && t < nc) nr = rk[(size_t)(i - 1) * nu + (t - nx)];
    }
    mark(0);
    // row t of the stage: state row t < nx (its own terms, read back by the
    // same thread below), input row t - nx (already in the input vector)
    if (t < nc) {
      const double wt = ry - rz;
      if (!fold) wprev[(size_t)i * nc + t] = wt;
      if (t < nx) V.wv2[t] = cst * (P[pk.q + t] + P[pk.ev + t]) + fr * dw_of(ry, rz, rw);
    }
    mark(3);
    // F^T [p; r_hat] over all four waves; then thread j forms p_k[j] and, in
    // wave 0, k_k = -Gamma^T (B^T p + r_hat + cst fv) with only that wave's
    // own LDS ordering
    // (no closing barrier: thread j reads only its own output entry below, and
    // wave 0 sums the input rows' partial sums itself; the stage-end barrier
    // orders everything else)
    fgemv_t<false>(nxu, fold ? nx : nxu, (const LDS float*)(P + pk.F), pk.ldF, V.xz, V.g2, V.part);
    if (t < nx) V.g[t] = V.g2[t] + V.wv2[t];
    if (!fold && w == 0) {
      if (t < nu) {
        const int j = nx + t;
        V.tu[t] = V.part[j] + V.part[128 + j] + V.part[256 + j] + V.part[384 + j] + cst * P[pk.fv + t];
      }
      wave_lds_sync();
      if (t < nu) {
        const LDS float* Gm = P + pk.Gam;
        float kk;
        if (nu <= 4) kk = gam_dot<4>(Gm, V.tu, nu, t);
        else if (nu <= 8) kk = gam_dot<8>(Gm, V.tu, nu, t);
        else if (nu <= 16) kk = gam_dot<16>(Gm, V.tu, nu, t);
        else if (nu <= 24) kk = gam_dot<24>(Gm, V.tu, nu, t);
        else if (nu <= 32) kk = gam_dot<32>(Gm, V.tu, nu, t);
        else {
          kk = 0.f;
          for (int q = 0; q < nu; ++q) kk += Gm[q * nu + t] * V.tu[q];
        }
        kff[(size_t)i * nu + t] = -kk;
      }
    }
    // input vector of the next stage, own entries (every read of V.xz in this
    // stage precedes the GEMV's internal barrier)
    if (i > s) {
      if (t < nx) V.xz[t] = V.g[t];
      else if (t < nc) V.xz[t] = cst * nr + fr * dw_of(ny, nz, nw);
    }
    mark(4);
    ry = ny; rz = nz; rw = nw;
    pk_dma_wait();
    dma_barrier();
    mark(5);
    cb ^= 1;
  }
}

// Forward pass of box-row instances over [s, e) (semantics of
// batch_forward<true>): the entry in V.xz[0..nx); thread j replaces its own
// state entry after its projection has read it; x_e ends in V.xz for a chunk
// with e < N.
__device__ __attribute__((noinline)) void box_forward(const BInst* __restrict__ Ip,
                                                      const BatchArgs* __restrict__ ag, double rho, bool full,
                                                      bool sigma_it, LDS char* base, int s, int e, bool fold) {
  Ip = uniform_ptr(Ip);
  ag = uniform_ptr(ag);
  s = uniform_int(s);
  e = uniform_int(e);
  fold = uniform_int(fold ? 1 : 0) != 0;
  const BInst& I = *Ip;
  const BatchArgs& a = *ag;
  const int N = I.N, nx = I.nx, nu = I.nu, nc = I.nc, nf = I.nf, nxu = nx + nu;
  const BLayout lay = batch_layout(nx, nu, 0);
  const PkLayout pk = pk_layout(nx, nu);
  const int pst = pk.stride;
  const IterVecs V = iter_vecs(lay, base);
  const float* fp = a.fp;
  double* dp = a.dp;
  const float* pkt = fp + I.oPk;
  const GLB float* kff = (const GLB float*)(fp + I.okff);
  const float cst = full ? 1.f : 0.f;
  const int t = tid(), w = wave();
  LDS float* xa = V.xz;
  if (fold) {
    if (s < e) pk_dma_issue(pkt + (size_t)s * pst, pst, V.buf0);
    float kf = (s < e && t < nu) ? kff[(size_t)s * nu + t] : 0.f;
    if (s < e && t < nu) xa[nx + t] = kf;   // the first stage's feed-forward entry
    pk_dma_wait();
    dma_barrier();
    int cb = 0;
    for (int i = s; i < e; ++i) {
      LDS float* P = V.buf(cb);
      if (i + 1 < e) {
        pk_dma_issue(pkt + (size_t)(i + 1) * pst, pst, V.buf(cb ^ 1));
        if (t < nu) kf = kff[(size_t)(i + 1) * nu + t];
      }
      // [x; k] complete since the previous barrier; own entries only below
      fgemv_n<false>(nx, nxu, (const LDS float*)(P + pk.F), pk.ldF, xa, V.tu, V.part);
      if (t < nx) xa[t] = V.tu[t] + cst * P[pk.b + t];
      if (i + 1 < e && t < nu) xa[nx + t] = kf;   // the next stage's feed-forward entry
      pk_dma_wait();
      dma_barrier();
      cb ^= 1;
    }
    return;
  }
  GLB double* ys = (GLB double*)(dp + I.oy);
  GLB double* zs = (GLB double*)(dp + I.oz);
  GLB double* vacc = (GLB double*)(dp + I.ov);
  const GLB double* ls = (const GLB double*)(dp + I.ol);
  const GLB double* us = (const GLB double*)(dp + I.ou);
  GLB double* X = (GLB double*)(dp + I.oX);
  GLB double* U = (GLB double*)(dp + I.oU);
  PhaseMark mark{V.pc, a.prof != nullptr};
  double rp = 0.0, rd = 0.0, vmax = 0.0, zmax = 0.0, hx = 0.0, gl = 0.0;
  const int last = e == N ? N : e - 1;
  if (s < e) pk_dma_issue(pkt + (size_t)s * pst, pst, V.buf0);
  double sv = 0.0, sy = 0.0, sz = 0.0, sl = 0.0, su = 0.0, sX = 0.0, sU = 0.0;
  {
    const int nr0 = (s == N) ? nf : nc;
    if (t < nr0) {
      const size_t gr = (size_t)s * nc + t;
      sv = vacc[gr]; sy = ys[gr]; sz = zs[gr]; sl = ls[gr]; su = us[gr];
    }
    if (t < nx) sX = X[(size_t)s * nx + t];
    if (s < N && t >= nx && t < nxu) sU = U[(size_t)s * nu + (t - nx)];   // u entry of thread t = nx + j
  }
  float sK = (s < N && t < nu) ? kff[(size_t)s * nu + t] : 0.f;
  if (s < N && t < nu) xa[nx + t] = sK;   // the first stage's feed-forward entry
  pk_dma_wait();
  dma_barrier();
  int cb = 0;
  for (int i = s; i <= last; ++i) {
    const bool term = (i == N);
    const int nr = term ? nf : nc;
    LDS float* P = V.buf(cb);
    double nv = 0.0, ny = 0.0, nz = 0.0, nl = 0.0, nu_ = 0.0, nX = 0.0, nU = 0.0;
    if (i + 1 < e) pk_dma_issue(pkt + (size_t)(i + 1) * pst, pst, V.buf(cb ^ 1));
    float nK = 0.f;
    if (i + 1 < N && i + 1 <= last && t < nu) nK = kff[(size_t)(i + 1) * nu + t];
    if (i + 1 <= last) {
      const int nr1 = (i + 1 == N) ? nf : nc;
      if (t < nr1) {
        const size_t gr = (size_t)(i + 1) * nc + t;
        nv = vacc[gr]; ny = ys[gr]; nz = zs[gr]; nl = ls[gr]; nu_ = us[gr];
      }
      if (t < nx) nX = X[(size_t)(i + 1) * nx + t];
      if (i + 1 < N && t >= nx && t < nxu) nU = U[(size_t)(i + 1) * nu + (t - nx)];
    }
    if (t < nx) X[(size_t)i * nx + t] = full ? (double)xa[t] : sX + (double)xa[t];
    mark(6);
    if (!term) {
      // [x; k] is complete since the previous barrier
      mark(7);
      // F [x; k] = [Abar x + B k; K x + k] over all four waves (ends with a barrier)
      // (no closing barrier: every reader below reads its own entry of V.tu)
      fgemv_n<false>(nxu, nxu, (const LDS float*)(P + pk.F), pk.ldF, xa, V.tu, V.part);
      mark(8);
      if (t >= nx && t < nxu) U[(size_t)i * nu + (t - nx)] = full ? (double)V.tu[t] : sU + (double)V.tu[t];
    }
    mark(9);
    if (t < nr) {
      // v = [x; u] (terminal: x_N)
      const float vf = t < nx ? xa[t] : V.tu[t];
      const size_t gr = (size_t)i * nc + t;
      const double v = full ? (double)vf : sv + (double)vf;
      vacc[gr] = v;
      const double tt = v + sy;
      const double zn = tt < sl ? sl : (tt > su ? su : tt);
      const double yn = sy + v - zn;
      zs[gr] = zn;
      ys[gr] = yn;
      const double er = fabs(v - zn);
      rp = (er > rp || er != er) ? er : rp;
      vmax = fmax(vmax, fabs(v));
      zmax = fmax(zmax, fabs(zn));
      const double q = rho * fabs((double)(float)(zn - sz));
      rd = (q > rd || q != q) ? q : rd;
      if (sigma_it) gl = fmax(gl, rho * fabs((double)(float)yn));
    }
    mark(10);
    if (term) break;
    // next state: thread j replaces its own entry (it has read it above)
    if (t < nx) xa[t] = V.tu[t] + cst * P[pk.b + t];
    if (i == last) {   // a chunk that ends before the horizon: x_e stays in V.xz
      dma_barrier();
      break;
    }
    // the next stage's feed-forward entry (every read of xa[nx..] in this
    // stage precedes the GEMV's internal barrier)
    if (i + 1 < N && t < nu) xa[nx + t] = nK;
    sv = nv; sy = ny; sz = nz; sl = nl; su = nu_; sX = nX; sU = nU; sK = nK;
    pk_dma_wait();
    dma_barrier();
    mark(11);
    cb ^= 1;
  }
  rp = wg_max_d(rp, V.red);
  rd = wg_max_d(rd, V.red);
  if (sigma_it) {
    vmax = wg_max_d(vmax, V.red);
    zmax = wg_max_d(zmax, V.red);
    gl = wg_max_d(gl, V.red);
    hx = batch_hxi(Ip, ag, base, s, e);   // on the x, u just accumulated
  }
  LDS double* out = V.red + kWG;
  if (t == 0) { out[0] = rp; out[1] = rd; out[2] = vmax; out[3] = zmax; out[4] = hx; out[5] = gl; }
  dma_barrier();
}

// Stage passes by row structure: box rows take the wave-owned products.
template <bool BOX>
__device__ __forceinline__ void stage_backward(const BInst* Ip, const BatchArgs* ag, float fr, bool full,
                                               LDS char* base, int s, int e, bool fold);
template <bool BOX>
__device__ __forceinline__ void stage_forward(const BInst* Ip, const BatchArgs* ag, double rho, bool full,
                                              bool sigma_it, LDS char* base, int s, int e, bool fold);

// Forward pass of one cached iteration over the stages [s, e) (and the
// terminal stage when e = N) from the entry x_s in V.xz[0..nx) (set by the
// caller: cst x0 for s = 0): per stage F [x; k] = [Abar x + B k; K x + k]
// gives u_k and x_{k+1} (+ cst b_k), the constraint values v = G [x; u] (box
// rows: v = [x; u]), then the projection z+ = clip(v + y, l, u), the scaled
// dual y+ = y + v - z+, and the residual terms.  x, u, v accumulate in FP64
// (increments after the first evaluation).  Returns, reduced over the
// workgroup, r_p, r_d and (rho-rule iterations) |v|, |z|, |H xi|,
// |G^T lambda| / rho of its stages in out[0..5] (LDS).
// A chunk that ends before the horizon (e < N) leaves x_e in V.xz[0..nx).
// Fold mode runs the x recurrence alone and writes nothing: x_e is left in
// V.xz[0..nx).
template <bool BOX>
__device__ __attribute__((noinline)) void batch_forward(const BInst* __restrict__ Ip,
                                                        const BatchArgs* __restrict__ ag, double rho, bool full,
                                                        bool sigma_it, LDS char* base, int s, int e, bool fold) {
  Ip = uniform_ptr(Ip);
  ag = uniform_ptr(ag);
  s = uniform_int(s);
  e = uniform_int(e);
  fold = uniform_int(fold ? 1 : 0) != 0;
  const BInst& I = *Ip;
  const BatchArgs& a = *ag;
  const int N = I.N, nx = I.nx, nu = I.nu, nc = I.nc, nf = I.nf, nxu = nx + nu;
  const BLayout lay = batch_layout(nx, nu, BOX ? 0 : (nc > nf ? nc : nf));
  const PkLayout pk = pk_layout(nx, nu);
  const int pst = pk.stride;
  const IterVecs V = iter_vecs(lay, base);
  const float* fp = a.fp;
  double* dp = a.dp;
  const float* pkt = fp + I.oPk;
  const GLB float* kff = (const GLB float*)(fp + I.okff);
  const float cst = full ? 1.f : 0.f;
  const int t = tid();
  if (fold) {
    // (each stage's feed-forward term is read one stage ahead, with the
    // next packet's copy)
    if (s < e) pk_dma_issue(pkt + (size_t)s * pst, pst, V.buf0);
    float kf = (s < e && t < nu) ? kff[(size_t)s * nu + t] : 0.f;
    pk_dma_wait();
    dma_barrier();
    int cb = 0;
    for (int i = s; i < e; ++i) {
      LDS float* P = V.buf(cb);
      if (t < nu) V.xz[nx + t] = kf;
      if (i + 1 < e) {
        pk_dma_issue(pkt + (size_t)(i + 1) * pst, pst, V.buf(cb ^ 1));
        if (t < nu) kf = kff[(size_t)(i + 1) * nu + t];
      }
      dma_barrier();
      fgemv_n(nx, nxu, (const LDS float*)(P + pk.F), pk.ldF, V.xz, V.g2, V.part);
      for (int j = t; j < nx; j += kWG) V.xz[j] = V.g2[j] + cst * P[pk.b + j];
      pk_dma_wait();
      dma_barrier();
      cb ^= 1;
    }
    return;
  }
  GLB double* ys = (GLB double*)(dp + I.oy);
  GLB double* zs = (GLB double*)(dp + I.oz);
  GLB double* vacc = (GLB double*)(dp + I.ov);
  const GLB double* ls = (const GLB double*)(dp + I.ol);
  const GLB double* us = (const GLB double*)(dp + I.ou);
  GLB double* X = (GLB double*)(dp + I.oX);
  GLB double* U = (GLB double*)(dp + I.oU);
  PhaseMark mark{V.pc, a.prof != nullptr};
  double rp = 0.0, rd = 0.0, vmax = 0.0, zmax = 0.0, hx = 0.0, gl = 0.0;
  const int last = e == N ? N : e - 1;   // last stage processed
  if (s < e) pk_dma_issue(pkt + (size_t)s * pst, pst, V.buf0);
  double sv = 0.0, sy = 0.0, sz = 0.0, sl = 0.0, su = 0.0, sX = 0.0, sU = 0.0;
  {
    const int nr0 = (s == N) ? nf : nc;
    if (t < nr0) {
      const size_t gr = (size_t)s * nc + t;
      sv = vacc[gr]; sy = ys[gr]; sz = zs[gr]; sl = ls[gr]; su = us[gr];
    }
    if (t < nx) sX = X[(size_t)s * nx + t];
    if (s < N && t < nu) sU = U[(size_t)s * nu + t];
  }
  float sK = (s < N && t < nu) ? kff[(size_t)s * nu + t] : 0.f;
  pk_dma_wait();
  dma_barrier();
  int cb = 0;
  for (int i = s; i <= last; ++i) {
    const bool term = (i == N);
    const int nr = term ? nf : nc;
    LDS float* P = V.buf(cb);
    double nv = 0.0, ny = 0.0, nz = 0.0, nl = 0.0, nu_ = 0.0, nX = 0.0, nU = 0.0;
    // the stage's feed-forward term was read one stage ahead
    if (!term && t < nu) V.xz[nx + t] = sK;
    if (i + 1 < e) pk_dma_issue(pkt + (size_t)(i + 1) * pst, pst, V.buf(cb ^ 1));
    float nK = 0.f;
    if (i + 1 < N && i + 1 <= last && t < nu) nK = kff[(size_t)(i + 1) * nu + t];
    if (i + 1 <= last) {
      const int nr1 = (i + 1 == N) ? nf : nc;
      if (t < nr1) {
        const size_t gr = (size_t)(i + 1) * nc + t;
        nv = vacc[gr]; ny = ys[gr]; nz = zs[gr]; nl = ls[gr]; nu_ = us[gr];
      }
      if (t < nx) nX = X[(size_t)(i + 1) * nx + t];
      if (i + 1 < N && t < nu) nU = U[(size_t)(i + 1) * nu + t];
    }
    if (t < nx) X[(size_t)i * nx + t] = full ? (double)V.xz[t] : sX + (double)V.xz[t];
    mark(6);
    if (!term) {
      dma_barrier();
      mark(7);
      fgemv_n(nxu, nxu, (const LDS float*)(P + pk.F), pk.ldF, V.xz, V.g2, V.part);
      mark(8);
      if (t < nu) {
        const float uu = V.g2[nx + t];
        V.xz[nx + t] = uu;
        U[(size_t)i * nu + t] = full ? (double)uu : sU + (double)uu;
      }
      dma_barrier();
      if (BOX) {
        for (int r = t; r < nc; r += kWG) V.wv[r] = V.xz[r];
      } else if (nc > 0) {
        lite_gemv_n(nc, nxu, (const float*)(fp + I.oG + (size_t)i * nc * nxu), nxu, V.xz, V.wv, V.part, false);
      }
    } else if (nr > 0) {
      if (BOX) {
        for (int r = t; r < nf; r += kWG) V.wv[r] = V.xz[r];
      } else {
        lite_gemv_n(nf, nx, (const float*)(fp + I.oCN), nx, V.xz, V.wv, V.part, false);
      }
    }
    dma_barrier();
    mark(9);
    if (t < nr) {
      const size_t gr = (size_t)i * nc + t;
      const double v = full ? (double)V.wv[t] : sv + (double)V.wv[t];
      vacc[gr] = v;
      const double tt = v + sy;
      const double zn = tt < sl ? sl : (tt > su ? su : tt);
      const double yn = sy + v - zn;
      zs[gr] = zn;
      ys[gr] = yn;
      const double er = fabs(v - zn);
      rp = (er > rp || er != er) ? er : rp;
      vmax = fmax(vmax, fabs(v));
      zmax = fmax(zmax, fabs(zn));
      V.wv[t] = (float)(zn - sz);
      V.wv2[t] = (float)yn;
    }
    dma_barrier();
    if (nr > 0) {
      if (BOX) {
        if (t < nr) {
          const double q = rho * fabs((double)V.wv[t]);
          rd = (q > rd || q != q) ? q : rd;
          if (sigma_it) gl = fmax(gl, rho * fabs((double)V.wv2[t]));
        }
      } else {
        const int ncol = term ? nx : nxu;
        const float* Gm = term ? fp + I.oCN : fp + I.oG + (size_t)i * nc * nxu;
        const int ldm = term ? nx : nxu;
        lite_gemv_t(nr, ncol, Gm, ldm, V.wv, V.tv, V.part);
        for (int j = t; j < ncol; j += kWG) {
          const double q = rho * fabs((double)V.tv[j]);
          rd = (q > rd || q != q) ? q : rd;
        }
        if (sigma_it) {
          lite_gemv_t(nr, ncol, Gm, ldm, V.wv2, V.tv, V.part);
          for (int j = t; j < ncol; j += kWG) gl = fmax(gl, rho * fabs((double)V.tv[j]));
        }
      }
      dma_barrier();
    }
    mark(10);
    if (term) break;
    for (int j = t; j < nx; j += kWG) V.xz[j] = V.g2[j] + cst * P[pk.b + j];
    if (i == last) {   // a chunk that ends before the horizon: x_e stays in V.xz
      dma_barrier();
      break;
    }
    sv = nv; sy = ny; sz = nz; sl = nl; su = nu_; sX = nX; sU = nU; sK = nK;
    pk_dma_wait();
    dma_barrier();
    mark(11);
    cb ^= 1;
  }
  rp = wg_max_d(rp, V.red);
  rd = wg_max_d(rd, V.red);
  if (sigma_it) {
    vmax = wg_max_d(vmax, V.red);
    zmax = wg_max_d(zmax, V.red);
    gl = wg_max_d(gl, V.red);
    hx = batch_hxi(Ip, ag, base, s, e);   // on the x, u just accumulated
  }
  LDS double* out = V.red + kWG;   // the reduction buffer holds kWG + 8 doubles
  if (t == 0) { out[0] = rp; out[1] = rd; out[2] = vmax; out[3] = zmax; out[4] = hx; out[5] = gl; }
  dma_barrier();
}

template <bool BOX>
__device__ __forceinline__ void stage_backward(const BInst* Ip, const BatchArgs* ag, float fr, bool full,
                                               LDS char* base, int s, int e, bool fold) {
  if constexpr (BOX) box_backward(Ip, ag, fr, full, base, s, e, fold);
  else batch_backward<false>(Ip, ag, fr, full, base, s, e, fold);
}
template <bool BOX>
__device__ __forceinline__ void stage_forward(const BInst* Ip, const BatchArgs* ag, double rho, bool full,
                                              bool sigma_it, LDS char* base, int s, int e, bool fold) {
  if constexpr (BOX) box_forward(Ip, ag, rho, full, sigma_it, base, s, e, fold);
  else batch_forward<false>(Ip, ag, rho, full, sigma_it, base, s, e, fold);
}

// Decision after one ADMM iteration from the reduced residual terms
// o = (r_p, r_d, |v|, |z|, |H xi|, |G^T lambda| / rho): 0 continue, 1 solved,
// 2 iteration limit, 3 numerical, 4 rho change (OSQP rule every sigma
// iterations, new rho in *rn).
__device__ inline int admm_decide(const BatchArgs& a, double rho, int it, int max_iter, bool sigma_it,
                                  double hnorm, const double o[6], double* rn) {
  const double rp = o[0], rd = o[1];
  if (rp != rp || rd != rd || isinf(rp) || isinf(rd)) return 3;
  if (rp <= a.tol && rd <= a.tol) return 1;
  if (it >= max_iter) return 2;
  if (sigma_it) {
    const double ps = fmax(o[2], o[3]), ds = fmax(fmax(o[4], o[5]), hnorm);
    const double ratio = (rp / (ps + 1e-10)) / (rd / (ds + 1e-10) + 1e-10);
    const double r = fmin(fmax(rho * sqrt(ratio), a.rho_min), a.rho_max);
    if (r > rho * a.rho_tol || r < rho / a.rho_tol) {
      *rn = r;
      return 4;
    }
  }
  return 0;
}

// max(|q|, |r|) over the instance (the rho rule's dual scale floor).
__device__ inline double batch_hnorm(const BInst& I, const float* fp, LDS double* red) {
  double h = 0.0;
  for (int e = tid(); e < (I.N + 1) * I.nx; e += kWG) h = fmax(h, fabs((double)fp[I.oq + e]));
  for (int e = tid(); e < I.N * I.nu; e += kWG) h = fmax(h, fabs((double)fp[I.orr + e]));
  return wg_max_d(h, red);
}

// ADMM iterations of one instance at fixed rho on one workgroup.  Returns 1
// solved, 2 max_iter, 3 numerical, 4 rho change (new rho in *rho_new), 6 the
// iteration count reached park_at with none of these (the instance is handed
// to a gang of workgroups; its state is complete in global memory).
// it0: iteration count when this attempt (cold or warm start) began; the rho
// rule runs every sigma iterations of the attempt.
__device__ __attribute__((noinline)) int batch_iterate(const BInst* __restrict__ Ip,
                                                       const BatchArgs* __restrict__ ag, double rho, int it0,
                                                       int max_iter, int park_at, int* it, double* rho_new,
                                                       double* rp_out, double* rd_out, LDS char* base) {
  Ip = uniform_ptr(Ip);
  ag = uniform_ptr(ag);
  const BInst& I = *Ip;
  const BatchArgs& a = *ag;
  const int N = I.N, nx = I.nx, nu = I.nu, nc = I.nc, nf = I.nf;
  const BLayout lay = batch_layout(nx, nu, I.box ? 0 : (nc > nf ? nc : nf));
  const IterVecs V = iter_vecs(lay, base);
  const float* fp = a.fp;
  double* ys = a.dp + I.oy;
  const int t = tid();
  if (a.prof && t < 12) V.pc[t] = 0ull;
  const double hnorm = batch_hnorm(I, fp, V.red);
  bool first = true;
  while (true) {
    ++*it;
    const bool full = first || (a.refresh > 0 && *it % a.refresh == 0);
    const bool sigma_it = a.adaptive && ((*it - it0) % a.sigma == 0) && *it < max_iter;
    if (I.box) stage_backward<true>(Ip, ag, (float)rho, full, base, 0, N, false);
    else stage_backward<false>(Ip, ag, (float)rho, full, base, 0, N, false);
    // forward entry x_0 (the backward pass uses V.xz as scratch)
    for (int j = t; j < nx; j += kWG) V.xz[j] = full ? fp[I.ox0 + j] : 0.f;
    if (I.box) stage_forward<true>(Ip, ag, rho, full, sigma_it, base, 0, N, false);
    else stage_forward<false>(Ip, ag, rho, full, sigma_it, base, 0, N, false);
    first = false;
    LDS double* out = V.red + kWG;
    double o[6];
    for (int q = 0; q < 6; ++q) o[q] = out[q];
    dma_barrier();
    *rp_out = o[0];
    *rd_out = o[1];
    if (a.prof && t < 12) { atomicAdd(a.prof + t, V.pc[t]); V.pc[t] = 0ull; }
    double rn = rho;
    const int st = admm_decide(a, rho, *it, max_iter, sigma_it, hnorm, o, &rn);
    if (st == 4) {
      const double f = rho / rn;
      for (int r = t; r < I.m; r += kWG) ys[r] *= f;
      __syncthreads();   // cross-thread global update: full fence
      *rho_new = rn;
      return 4;
    }
    if (st) return st;
    // hand-over: not for an instance already close to the stopping test (a
    // gang costs its members' waiting and a factor epoch; a few more solo
    // iterations cost less)
    if (*it >= park_at && !(o[0] <= kParkResid * a.tol && o[1] <= kParkResid * a.tol)) return 6;
  }
}

// ----------------------------------------------------------------- gangs
// An instance that has not converged within its solo budget (park_at
// iterations, a function of its size only) and is not yet within kParkResid
// of the stopping test is continued by a gang of G
// workgroups that split its horizon into G chunks (Sec. IV-A: the affine maps
// of the backward and forward recurrences are composed by associative scans
// over the horizon).  Per iteration each member
//   1. folds its chunk's backward recurrence from a zero entry,
//   2. combines the chunk results across the gang by recursive doubling with
//      the cached chunk transfer maps Phi[d][r] = Abar_{e-1} ... Abar_s over
//      2^d chunks (p_s = Phi^T p_e + fold),
//   3. re-runs its chunk from the exact entry p_e (feed-forward gains k),
//   4.-6. the same for the forward recurrence (x_e = Phi x_s + fold), the
//      re-run doing the projection, dual update and residual terms,
//   7. exchanges the residual terms; every member takes the same decision.
// The chunk ending at N needs no backward fold (its entry is the terminal
// value) and the chunk starting at 0 no forward fold.  A rho change runs the
// factor epoch on member 0 (the others wait), then the transfer maps again.
// Members exchange through packed (payload, stamp) words; every wait is
// bounded and a failed wait raises the launch's abort flag.

struct GangLayout {
  int nlev;
  size_t bwd, fwd, res, mflag, eword, words;   // 64-bit word offsets
};
__host__ __device__ inline int gang_levels(int G) {
  int l = 0;
  while ((1 << l) < G) ++l;
  return l;
}
__host__ __device__ inline GangLayout gang_layout(int nx, int G) {
  GangLayout L;
  L.nlev = gang_levels(G);
  size_t o = 0;
  L.bwd = o; o += (size_t)(L.nlev + 1) * G * nx;
  L.fwd = o; o += (size_t)(L.nlev + 1) * G * nx;
  L.res = o; o += (size_t)G * 12;
  L.mflag = o; o += (size_t)(L.nlev > 0 ? L.nlev : 1) * G;
  L.eword = o; o += 1;
  L.words = o;
  return L;
}
// Transfer maps of one instance: [nlev][G][nx][nx] floats.
__host__ __device__ inline size_t gang_map_floats(int nx, int G) {
  const int nl = gang_levels(G);
  return (size_t)(nl > 0 ? nl : 1) * G * nx * nx;
}

// Control state of an instance handed from its solo workgroup to a gang.
struct BPark {
  int it, nupd, nfact, it0, limit, warm, budgeted, restarted;
  double rho;
  long long te, ti;
};

// Device-wide counters of one launch (cleared by the prologue kernel).
struct BSync {
  unsigned counter;     // solo work queue
  unsigned ticket;      // gang tickets
  unsigned cont;        // instances handed to gangs (slots reserved)
  unsigned done;        // solo items finished (solved or handed over)
  int abort;            // a bounded wait gave up
  unsigned pticket;     // gang tickets of the priority list
  unsigned pcont;       // instances handed to the priority list
};

__device__ inline void g_publish(unsigned long long* w, uint32_t stamp, const LDS float* v, int n) {
  for (int j = tid(); j < n; j += kWG) ll_put(w + j, stamp, __float_as_uint(v[j]));
}
// Reads n stamped values into v (all threads call); false (uniformly) if a
// wait gave up, after raising the abort flag.
__device__ inline bool g_fetch(const unsigned long long* w, uint32_t stamp, LDS float* v, int n, int* abort,
                               int* flag) {
  bool ok = true;
  for (int j = tid(); j < n; j += kWG) {
    uint32_t b = 0;
    if (!ll_get(w + j, stamp, &b, abort)) ok = false;
    v[j] = __uint_as_float(b);
  }
  if (!ok) {
    *flag = 1;
    __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  const bool r = *flag == 0;
  __syncthreads();
  return r;
}
// One stamped word waited for by thread 0 and broadcast (payload in *bits).
__device__ inline bool g_wait_word(const unsigned long long* w, uint32_t stamp, uint32_t* bits, int* abort,
                                   int* flag, uint32_t* sbits) {
  if (tid() == 0) {
    uint32_t b = 0;
    if (!ll_get(w, stamp, &b, abort)) {
      *flag = 1;
      __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    *sbits = b;
  }
  __syncthreads();
  const bool r = *flag == 0;
  *bits = *sbits;
  __syncthreads();
  return r;
}

// Chunk [s, e) of member r of G over a horizon of N stages.
__host__ __device__ inline int gang_cbeg(int r, int N, int G) { return (int)(((long long)r * N) / G); }

// Transfer maps of member r after a factor epoch: Phi[0][r] = product of
// Abar over its chunk (later stages on the left), Phi[d][r] =
// Phi[d-1][r + 2^(d-1)] Phi[d-1][r] for r + 2^d <= G.  Each map is published
// (flag word mflag[d][r], stamp) after it is stored.
__device__ __attribute__((noinline)) bool gang_maps(const BInst* __restrict__ Ip, const BatchArgs* __restrict__ ag,
                                                    int r, int G, uint32_t stamp, LDS char* base, int* flag,
                                                    uint32_t* sbits) {
  Ip = uniform_ptr(Ip);
  ag = uniform_ptr(ag);
  r = uniform_int(r);
  G = uniform_int(G);
  const BInst& I = *Ip;
  const BatchArgs& a = *ag;
  const int N = I.N, nx = I.nx, nu = I.nu, nc = I.nc, nf = I.nf;
  const BLayout lay = batch_layout(nx, nu, I.box ? 0 : (nc > nf ? nc : nf));
  const PkLayout pk = pk_layout(nx, nu);
  const GangLayout gl = gang_layout(nx, G);
  LDS float* F0 = (LDS float*)base;
  LDS float* Pm = F0 + lay.P;    // running product (ld ldP)
  LDS float* Am = F0 + lay.AB;   // multiplier (ld ldAB)
  LDS float* Wm = F0 + lay.W;    // product (ld ldW)
  const int ldP = lay.ldP, ldA = lay.ldAB, ldW = lay.ldW;
  const float* pkt = a.fp + I.oPk;
  float* maps = a.gmaps + I.ogm;
  unsigned long long* words = a.gwords + I.ogw;
  const size_t xx = (size_t)nx * nx;
  const int s = gang_cbeg(r, N, G), e = gang_cbeg(r + 1, N, G);
  for (int i = s; i < e; ++i) {
    const float* Fi = pkt + (size_t)i * pk.stride + pk.F;
    LDS float* dst = (i == s) ? Pm : Am;
    const int ldd = (i == s) ? ldP : ldA;
    for (int q = wave(); q < nx; q += 4)
      for (int c = lane(); c < nx; c += 64) dst[q * ldd + c] = Fi[q * pk.ldF + c];
    __syncthreads();
    if (i > s) {
      mm_pl<false, false>(nx, nx, nx, 1.f, Am, ldA, Pm, ldP, 0.f, Wm, ldW);
      for (int q = wave(); q < nx; q += 4)
        for (int c = lane(); c < nx; c += 64) Pm[q * ldP + c] = Wm[q * ldW + c];
      __syncthreads();
    }
  }
  for (int d = 0; d < gl.nlev; ++d) {
    if (r + (1 << d) > G) break;
    if (d > 0) {
      const int pr = r + (1 << (d - 1));
      uint32_t bits;
      if (!g_wait_word(words + gl.mflag + (size_t)(d - 1) * G + pr, stamp, &bits, &a.sync->abort, flag, sbits))
        return false;
      __threadfence();
      const float* src = maps + ((size_t)(d - 1) * G + pr) * xx;
      for (int q = wave(); q < nx; q += 4)
        for (int c = lane(); c < nx; c += 64) Am[q * ldA + c] = src[(size_t)q * nx + c];
      __syncthreads();
      mm_pl<false, false>(nx, nx, nx, 1.f, Am, ldA, Pm, ldP, 0.f, Wm, ldW);
      for (int q = wave(); q < nx; q += 4)
        for (int c = lane(); c < nx; c += 64) Pm[q * ldP + c] = Wm[q * ldW + c];
      __syncthreads();
    }
    float* dstg = maps + ((size_t)d * G + r) * xx;
    for (int q = wave(); q < nx; q += 4)
      for (int c = lane(); c < nx; c += 64) dstg[(size_t)q * nx + c] = Pm[q * ldP + c];
    __threadfence();
    __syncthreads();
    if (tid() == 0) ll_put(words + gl.mflag + (size_t)d * G + r, stamp, 1u);
  }
  // the forward combination of level d reads Phi[d][r - 2^d + 1], a map of
  // another member: wait until each of those is stored
  for (int d = 1; d < gl.nlev; ++d) {
    const int q = r - (1 << d) + 1;
    if (q < 1) break;
    uint32_t bits;
    if (!g_wait_word(words + gl.mflag + (size_t)d * G + q, stamp, &bits, &a.sync->abort, flag, sbits))
      return false;
  }
  __threadfence();
  return true;
}

// One gang member's part of an instance's continuation.
template <bool BOX>
__device__ __attribute__((noinline)) void gang_run(const BInst* __restrict__ Ip, const BatchArgs* __restrict__ ag,
                                                   int idx, int r, int G, LDS char* base) {
  Ip = uniform_ptr(Ip);
  ag = uniform_ptr(ag);
  idx = uniform_int(idx);
  r = uniform_int(r);
  G = uniform_int(G);
  const BInst& I = *Ip;
  const BatchArgs& a = *ag;
  const int N = I.N, nx = I.nx, nu = I.nu, nc = I.nc, nf = I.nf;
  const BLayout lay = batch_layout(nx, nu, BOX ? 0 : (nc > nf ? nc : nf));
  const IterVecs V = iter_vecs(lay, base);
  const GangLayout gl = gang_layout(nx, G);
  const int nlev = gl.nlev;
  unsigned long long* words = a.gwords + I.ogw;
  const float* maps = a.gmaps + I.ogm;
  const size_t xx = (size_t)nx * nx;
  const int s = gang_cbeg(r, N, G), e = gang_cbeg(r + 1, N, G);
  const int row0 = s * nc, row1 = e * nc + (e == N ? nf : 0);   // rows owned by this member
  double* ys = a.dp + I.oy;
  double* zs = a.dp + I.oz;
  const int t = tid();
  __shared__ int s_flag;
  __shared__ uint32_t s_bits;
  if (t == 0) s_flag = 0;
  // clear this member's exchange words, then join
  for (int d = 0; d <= nlev; ++d)
    for (int j = t; j < nx; j += kWG) {
      words[gl.bwd + ((size_t)d * G + r) * nx + j] = 0ull;
      words[gl.fwd + ((size_t)d * G + r) * nx + j] = 0ull;
    }
  for (int j = t; j < 12; j += kWG) words[gl.res + (size_t)r * 12 + j] = 0ull;
  for (int d = t; d < (nlev > 0 ? nlev : 1); d += kWG) words[gl.mflag + (size_t)d * G + r] = 0ull;
  if (r == 0 && t == 0) words[gl.eword] = 0ull;
  __threadfence();
  __syncthreads();
  if (t == 0) {
    atomicAdd(a.join + idx, 1u);
    unsigned n = 0;
    while (__hip_atomic_load(a.join + idx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < (unsigned)G) {
      if (++n > kSpinLimit || __hip_atomic_load(&a.sync->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        s_flag = 1;
        __hip_atomic_store(&a.sync->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
  }
  __syncthreads();
  __threadfence();
  BPark pkd = a.park[idx];
  int it = pkd.it, nupd = pkd.nupd, nfact = pkd.nfact, it0 = pkd.it0, limit = pkd.limit;
  bool warm = pkd.warm != 0, restarted = pkd.restarted != 0;
  const bool budgeted = pkd.budgeted != 0;
  double rho = pkd.rho;
  long long te = pkd.te, ti = pkd.ti;
  int st = 5;
  double rp = 0.0, rd = 0.0;
  bool ok = s_flag == 0;
  const double hnorm = batch_hnorm(I, a.fp, V.red);
  if (ok) ok = gang_maps(Ip, ag, r, G, (uint32_t)nfact, base, &s_flag, &s_bits);
  bool first = false;
  long long tc = wall_clock64();
  while (ok) {
    ++it;
    const uint32_t stamp = (uint32_t)it;
    const bool full = first || (a.refresh > 0 && it % a.refresh == 0);
    const float cst = full ? 1.f : 0.f;
    const bool sigma_it = a.adaptive && ((it - it0) % a.sigma == 0) && it < limit;
    // ---- backward: fold, doubling, re-run from the exact entry.  The last
    // member's entry is exact already; it folds too (its fold is its chunk's
    // exact p_s) and re-runs after publishing, off the doubling's critical path
    if (r > 0) stage_backward<BOX>(Ip, ag, (float)rho, full, base, s, e, true);
    if (r > 0) {
      g_publish(words + gl.bwd + (size_t)r * nx, stamp, V.g, nx);
      for (int d = 0; d < nlev; ++d) {
        const int pr = r + (1 << d);
        if (pr < G) {
          if (!g_fetch(words + gl.bwd + ((size_t)d * G + pr) * nx, stamp, V.g2, nx, &a.sync->abort, &s_flag)) {
            ok = false; break;
          }
          // map from global memory: every load of a thread issued before its
          // first product (one memory latency per level)
          fgemv_t(nx, nx, maps + ((size_t)d * G + r) * xx, nx, V.g2, V.tv, V.part);
          for (int j = t; j < nx; j += kWG) V.g[j] += V.tv[j];
          dma_barrier();
        }
        g_publish(words + gl.bwd + ((size_t)(d + 1) * G + r) * nx, stamp, V.g, nx);
      }
      if (!ok) break;
    }
    if (r < G - 1) {
      if (!g_fetch(words + gl.bwd + ((size_t)nlev * G + r + 1) * nx, stamp, V.g, nx, &a.sync->abort, &s_flag)) {
        ok = false; break;
      }
    }
    stage_backward<BOX>(Ip, ag, (float)rho, full, base, s, e, false);   // (the last chunk starts from p_N)
    // ---- forward: fold, doubling, re-run with projection and residuals.
    // The first member's entry x_0 is exact: its fold is its chunk's exact
    // x_e, published before its re-run
    for (int j = t; j < nx; j += kWG) V.xz[j] = (r == 0) ? cst * a.fp[I.ox0 + j] : 0.f;
    if (r < G - 1) stage_forward<BOX>(Ip, ag, rho, full, sigma_it, base, s, e, true);
    if (r < G - 1) {
      for (int j = t; j < nx; j += kWG) V.g[j] = V.xz[j];
      dma_barrier();
      g_publish(words + gl.fwd + (size_t)r * nx, stamp, V.g, nx);
      for (int d = 0; d < nlev; ++d) {
        const int pr = r - (1 << d);
        if (pr >= 0) {
          if (!g_fetch(words + gl.fwd + ((size_t)d * G + pr) * nx, stamp, V.g2, nx, &a.sync->abort, &s_flag)) {
            ok = false; break;
          }
          fgemv_n(nx, nx, maps + ((size_t)d * G + pr + 1) * xx, nx, V.g2, V.tv, V.part);
          for (int j = t; j < nx; j += kWG) V.g[j] += V.tv[j];
          dma_barrier();
        }
        g_publish(words + gl.fwd + ((size_t)(d + 1) * G + r) * nx, stamp, V.g, nx);
      }
      if (!ok) break;
    }
    if (r > 0) {
      if (!g_fetch(words + gl.fwd + ((size_t)nlev * G + r - 1) * nx, stamp, V.xz, nx, &a.sync->abort, &s_flag)) {
        ok = false; break;
      }
    } else {
      for (int j = t; j < nx; j += kWG) V.xz[j] = cst * a.fp[I.ox0 + j];
    }
    stage_forward<BOX>(Ip, ag, rho, full, sigma_it, base, s, e, false);
    first = false;
    // ---- residual terms of the whole instance (same order on every member)
    LDS double* out = V.red + kWG;
    if (t < 6) {
      const unsigned long long b = (unsigned long long)__double_as_longlong(out[t]);
      ll_put(words + gl.res + (size_t)r * 12 + 2 * t, stamp, (uint32_t)b);
      ll_put(words + gl.res + (size_t)r * 12 + 2 * t + 1, stamp, (uint32_t)(b >> 32));
    }
    double o[6] = {0, 0, 0, 0, 0, 0};
    {
      bool good = true;
      double mine = 0.0;
      if (t < 6 * G) {
        const int q = t % 6, mr = t / 6;
        uint32_t b[2] = {0, 0};
        const unsigned long long* w0 = words + gl.res + (size_t)mr * 12 + 2 * q;
        good = ll_get_batch<2>([&](int k) { return w0 + k; }, 2, stamp, b, &a.sync->abort);
        mine = __longlong_as_double((long long)(((unsigned long long)b[1] << 32) | b[0]));
      }
      if (!good) {
        s_flag = 1;
        __hip_atomic_store(&a.sync->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      dma_barrier();
      if (t < 6 * G) V.red[t] = mine;   // V.red holds kWG + 8 doubles; 6 G <= kWG
      __syncthreads();
      if (s_flag) { ok = false; break; }
      for (int mr = 0; mr < G; ++mr)
        for (int q = 0; q < 6; ++q) {
          const double v = V.red[mr * 6 + q];
          o[q] = (v > o[q] || v != v) ? v : o[q];
        }
      __syncthreads();
    }
    rp = o[0];
    rd = o[1];
    double rn = rho;
    const int dec = admm_decide(a, rho, it, limit, sigma_it, hnorm, o, &rn);
    bool epoch = false;
    if (dec == 4) {
      const double f = rho / rn;
      for (int q = row0 + t; q < row1; q += kWG) ys[q] *= f;
      rho = rn;
      ++nupd;
      epoch = true;
    } else if (warm && budgeted && (dec == 2 || dec == 3)) {
      // the warm start did not pay off: restart from z = y = 0
      warm = false;
      restarted = true;
      it0 = it;
      limit = it + a.max_iter;
      rho = a.rho_cold;
      for (int q = row0 + t; q < row1; q += kWG) { zs[q] = 0.0; ys[q] = 0.0; }
      epoch = true;
    } else if (dec != 0) {
      st = dec;
      break;
    }
    if (epoch) {
      __syncthreads();
      ++nfact;
      const long long c0 = wall_clock64();
      ti += c0 - tc;
      uint32_t bits = 1;
      if (r == 0) {
        const bool pd = batch_epoch(Ip, ag, rho, base);
        __threadfence();
        __syncthreads();
        if (t == 0) ll_put(words + gl.eword, (uint32_t)nfact, pd ? 1u : 2u);
        bits = pd ? 1u : 2u;
      } else {
        if (!g_wait_word(words + gl.eword, (uint32_t)nfact, &bits, &a.sync->abort, &s_flag, &s_bits)) {
          ok = false; break;
        }
        __threadfence();
      }
      if (bits != 1u) { st = -1; break; }
      if (!gang_maps(Ip, ag, r, G, (uint32_t)nfact, base, &s_flag, &s_bits)) { ok = false; break; }
      tc = wall_clock64();
      te += tc - c0;
      first = true;
    }
  }
  ti += wall_clock64() - tc;
  if (!ok) st = 5;
  if (r == 0 && t == 0) {
    BResult res;
    res.status = st; res.iterations = it; res.rho_updates = nupd; res.factorizations = nfact;
    res.restarted = restarted ? 1 : 0;
    res.r_p = rp; res.r_d = rd; res.rho = rho;
    res.t_epoch = te; res.t_iter = ti;
    res.r_dyn = 0.0;
    a.res[idx] = res;
  }
  __syncthreads();
}

// Solo part of one instance on this workgroup (cold or warm start, epochs,
// iterations); hands the instance over to a gang when its iteration count
// reaches park_at.
__device__ __attribute__((noinline)) void batch_solo(const BatchArgs* __restrict__ ag, int idx, LDS char* base) {
  ag = uniform_ptr(ag);
  idx = uniform_int(idx);
  const BatchArgs& a = *ag;
  BSync* sy = a.sync;
  const BInst* Ip = a.inst + idx;
  const int m = Ip->m;
  const long long oz = Ip->oz, oy = Ip->oy;
  bool warm = a.warm[idx] != 0;
  if (!warm)
    for (int r = tid(); r < m; r += kWG) { a.dp[oz + r] = 0.0; a.dp[oy + r] = 0.0; }
  __syncthreads();
  double rho = a.rho0[idx];
  double rho_start = rho;
  int it = 0, nupd = 0, nfact = 0, st = 0, restarted = 0;
  double rp = 0.0, rd = 0.0;
  const bool budgeted = warm && a.warm_budget > 0 && a.warm_budget < a.max_iter;
  int limit = budgeted ? a.warm_budget : a.max_iter, it0 = 0;
  const int park_at = a.gang > 1 ? Ip->park_at : 0x7fffffff;
  long long te = 0, ti = 0;
  while (true) {
    ++nfact;
    const long long c0 = wall_clock64();
    if (!batch_epoch(Ip, ag, rho, base)) { st = -1; break; }
    const long long c1 = wall_clock64();
    double rn = rho;
    st = batch_iterate(Ip, ag, rho, it0, limit, park_at, &it, &rn, &rp, &rd, base);
    te += c1 - c0;
    ti += wall_clock64() - c1;
    if (st == 4) { rho = rn; ++nupd; continue; }
    if (warm && budgeted && (st == 2 || st == 3)) {
      // the warm start did not pay off: restart from z = y = 0 with a
      // full iteration budget of its own
      warm = false;
      restarted = 1;
      it0 = it;
      limit = it + a.max_iter;
      rho = rho_start = a.rho_cold;
      for (int r = tid(); r < m; r += kWG) { a.dp[oz + r] = 0.0; a.dp[oy + r] = 0.0; }
      __syncthreads();
      continue;
    }
    break;
  }
  if (st == 6) {
    // hand over: state to global memory, then the slot (release)
    __syncthreads();
    if (tid() == 0) {
      BPark pk;
      pk.it = it; pk.nupd = nupd; pk.nfact = nfact; pk.it0 = it0; pk.limit = limit;
      pk.warm = warm ? 1 : 0; pk.budgeted = budgeted ? 1 : 0; pk.restarted = restarted;
      pk.rho = rho; pk.te = te; pk.ti = ti;
      a.park[idx] = pk;
      __threadfence();
      // priority slots fill cont_list from the front, the others from the
      // back (an instance is handed over at most once per launch)
      const bool prio = rho >= kPrioRho && rho >= kPrioGrowth * rho_start &&
                        (rp >= kPrioResid * a.tol || rd >= kPrioResid * a.tol);
      const unsigned slot = atomicAdd(prio ? &sy->pcont : &sy->cont, 1u);
      atomicExch(a.cont_list + (prio ? slot : (unsigned)a.count - 1u - slot), idx);
    }
  } else if (tid() == 0) {
    BResult r;
    r.status = st; r.iterations = it; r.rho_updates = nupd; r.factorizations = nfact;
    r.restarted = restarted;
    r.r_p = rp; r.r_d = rd; r.rho = rho;
    r.t_epoch = te; r.t_iter = ti;
    r.r_dyn = 0.0;
    a.res[idx] = r;
  }
  if (tid() == 0) {
    __threadfence();
    atomicAdd(&sy->done, 1u);
  }
  __syncthreads();
}

// Thread 0: a seat in the gang of a handed-over instance of one hand-over
// list, if one is open (a ticket below cont * G).  Tickets are consecutive
// per listed instance (G per instance, in hand-over order), so a gang's seats
// are all taken before any seat of a later gang of the same list.  The list's
// slot i is cont_list[i] (front) or cont_list[count - 1 - i].  True if a
// ticket was taken; *code is then the seat (instance << 8 | rank), or left as
// it was after raising the abort flag if the slot's entry never appeared.
__device__ inline bool take_seat(const BatchArgs& a, unsigned* ticket, const unsigned* cont, bool front, int G,
                                 int* code) {
  unsigned tk = __hip_atomic_load(ticket, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  while (true) {
    const unsigned cn = __hip_atomic_load(cont, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (tk >= cn * (unsigned)G) return false;
    if (__hip_atomic_compare_exchange_strong(ticket, &tk, tk + 1u, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT)) {
      const unsigned slot = tk / (unsigned)G;
      const int* e = a.cont_list + (front ? slot : (unsigned)a.count - 1u - slot);
      int v = -1;
      unsigned n = 0;
      // the slot is reserved: its entry is being written
      while ((v = __hip_atomic_load(e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) < 0 && ++n < kSpinLimit)
        __builtin_amdgcn_s_sleep(1);
      if (v < 0) __hip_atomic_store(&a.sync->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      else *code = (v << 8) | (int)(tk % (unsigned)G);
      return true;
    }
  }
}

// Persistent batched solver.  A free workgroup first takes an open seat in
// the gang of a handed-over instance (priority list first, then the other),
// else the next solo instance from the work queue (largest first), else it
// waits for a seat to open until every solo item has finished.  A seat is
// taken only once its instance has been handed over, so no workgroup waits on
// an instance that may never come.  At most one gang per list has seats both
// taken and open (tickets are consecutive per list), every other workgroup
// runs work that ends, and G <= grid / 2, so both partial gangs fill.
__global__ void __launch_bounds__(kWG) k_batch(const BatchArgs* __restrict__ ag) {
  extern __shared__ __align__(16) char lds_generic[];
  LDS char* base = (LDS char*)lds_generic;
  __shared__ int s_code;
  const BatchArgs& a = *ag;
  BSync* sy = a.sync;
  const int G = a.gang > 1 ? a.gang : 1;
  const unsigned count = (unsigned)a.count;
  while (true) {
    // code >= 0: gang member (instance << 8 | rank); -1 - item: solo item; -1 - count: exit
    if (tid() == 0) {
      int code = -1 - (int)count;
      bool decided = false;
      // 1. an open seat in a handed-over instance's gang
      if (G > 1)
        decided = take_seat(a, &sy->pticket, &sy->pcont, true, G, &code) ||
                  take_seat(a, &sy->ticket, &sy->cont, false, G, &code);
      if (!decided) {
        // 2. the next solo item
        const unsigned item = atomicAdd(&sy->counter, 1u);
        if (item < count) {
          code = -1 - (int)item;
          decided = true;
        }
      }
      if (!decided && G > 1) {
        // 3. no solo work left: wait for a seat, or for the end.  A hand-over
        // reserves its slot before its solo item counts as done, so once every
        // solo item is done the lists read after that are final.
        unsigned n = 0;
        while (true) {
          const unsigned dn = __hip_atomic_load(&sy->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __threadfence();
          if (take_seat(a, &sy->pticket, &sy->pcont, true, G, &code) ||
              take_seat(a, &sy->ticket, &sy->cont, false, G, &code))
            break;
          if (dn >= count) break;
          if (__hip_atomic_load(&sy->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
          if (++n > 64u * kSpinLimit) {
            __hip_atomic_store(&sy->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
          }
          __builtin_amdgcn_s_sleep(8);
        }
      }
      s_code = code;
    }
    __syncthreads();
    const int code = s_code;
    __syncthreads();
    if (code == -1 - (int)count) break;
    if (code < 0) {
      batch_solo(ag, a.order[-1 - code], base);
    } else {
      __threadfence();
      const int idx = code >> 8, r = code & 255;
      const BInst* Ip = a.inst + idx;
      if (Ip->box) gang_run<true>(Ip, ag, idx, r, G, base);
      else gang_run<false>(Ip, ag, idx, r, G, base);
    }
  }
}

// Dynamics residual of each instance's returned iterate: one workgroup per
// stage row of the warm-start row table (instance c = row_inst[b], stage
// k = b - row_off[c]; the terminal row has no stage), each wave taking state
// rows i and its lanes the columns of [A_k | B_k] (coalesced loads), the
// maximum over the stage merged into the instance's result by an atomic max
// of the bit pattern (non-negative doubles order as their bits).
// res[c].r_dyn must start at zero (the solver writes it so).
__global__ void __launch_bounds__(kWG) k_batch_rdyn(const BInst* __restrict__ inst, const float* __restrict__ fp,
                                                    const double* __restrict__ dp, const int* __restrict__ row_inst,
                                                    const int* __restrict__ row_off, BResult* res) {
  __shared__ double red[4];
  const int c = row_inst[blockIdx.x];
  const BInst I = inst[c];
  const int k = (int)blockIdx.x - row_off[c];
  if (k >= I.N) return;   // terminal row: uniform exit
  const int nx = I.nx, nu = I.nu, w = wave(), l = lane();
  const EpLayout ep = ep_layout(nx, nu);
  const double* xk = dp + I.oX + (size_t)k * nx;
  const double* uk = dp + I.oU + (size_t)k * nu;
  double m = 0.0;
  for (int i = w; i < nx; i += 4) {
    // row i of [A_k | B_k] in the epoch input packet
    const float* ABr = fp + I.oE + (size_t)k * ep.stride + ep.AB + (size_t)i * ep.ld;
    double a = 0.0;
    for (int j = l; j < nx + nu; j += 64) a += (double)ABr[j] * (j < nx ? xk[j] : uk[j - nx]);
    for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
    const double e = fabs(dp[I.oX + (size_t)(k + 1) * nx + i] - (double)fp[I.ob + (size_t)k * nx + i] - a);
    m = (e > m || e != e) ? e : m;
  }
  if (l == 0) red[w] = m;
  __syncthreads();
  if (tid() == 0) {
    double r = red[0];
    for (int q = 1; q < 4; ++q) r = (red[q] > r || red[q] != red[q]) ? red[q] : r;
    atomicMax((unsigned long long*)&res[c].r_dyn, (unsigned long long)__double_as_longlong(r));
  }
}

// Clears the launch's counters, the hand-over list and the gang join counters.
__global__ void k_batch_prologue(BSync* sync, int* cont_list, unsigned* join, int count) {
  const int i = blockIdx.x * blockDim.x + tid();
  if (i == 0) {
    sync->counter = 0u; sync->ticket = 0u; sync->cont = 0u; sync->done = 0u; sync->abort = 0;
    sync->pticket = 0u; sync->pcont = 0u;
  }
  if (i < count) { cont_list[i] = -1; join[i] = 0u; }
}

// ------------------------------------------------------------------ host
static bool is_box(const gsls_qp_desc& d, const std::vector<double>& C, const std::vector<double>& D,
                   const std::vector<double>& CN) {
  const int nx = d.nx, nu = d.nu, nc = d.nc, nf = d.nf;
  if (nc != nx + nu) return false;
  if (nf != 0 && nf != nx) return false;
  for (int k = 0; k < d.N; ++k)
    for (int r = 0; r < nc; ++r) {
      for (int j = 0; j < nx; ++j)
        if (C[((size_t)k * nc + r) * nx + j] != (r == j ? 1.0 : 0.0)) return false;
      for (int j = 0; j < nu; ++j)
        if (D[((size_t)k * nc + r) * nu + j] != (r == nx + j ? 1.0 : 0.0)) return false;
    }
  for (int r = 0; r < nf; ++r)
    for (int j = 0; j < nx; ++j)
      if (CN[(size_t)r * nx + j] != (r == j ? 1.0 : 0.0)) return false;
  return true;
}

int batch_setup(const gsls_qp_desc* descs, int count, const gsls_settings* s, hipStream_t stream, BatchSolver* B) {
  B->stream = stream;
  B->st = *s;
  B->count = count;
  B->inst.resize(count);
  std::vector<float> fpool;
  std::vector<double> dpool;
  auto pushf = [&](const double* p, size_t n) {
    long long o = (long long)fpool.size();
    for (size_t i = 0; i < n; ++i) fpool.push_back(p ? (float)p[i] : 0.f);
    while (fpool.size() % 4) fpool.push_back(0.f);
    return o;
  };
  auto reservef = [&](size_t n) {
    long long o = (long long)fpool.size();
    fpool.resize(fpool.size() + ((n + 3) & ~(size_t)3), 0.f);
    return o;
  };
  auto pushd = [&](const double* p, size_t n) {
    long long o = (long long)dpool.size();
    for (size_t i = 0; i < n; ++i) dpool.push_back(p ? p[i] : 0.0);
    while (dpool.size() % 2) dpool.push_back(0.0);
    return o;
  };
  auto reserved = [&](size_t n) {
    long long o = (long long)dpool.size();
    dpool.resize(dpool.size() + ((n + 1) & ~(size_t)1), 0.0);
    return o;
  };
  size_t lds = 0;
  std::vector<double> cost(count);
  for (int c = 0; c < count; ++c) {
    const gsls_qp_desc& d = descs[c];
    if (d.mem != GSLS_HOST) return GSLS_ERR_INVALID_ARG;
    const size_t N = d.N, nx = d.nx, nu = d.nu, nc = d.nc, nf = d.nf, nxu = nx + nu;
    if (nx + nu > kBatchMaxNxu) return GSLS_ERR_DIM;
    std::vector<double> C(d.C ? d.C : (const double*)nullptr, d.C ? d.C + N * nc * nx : nullptr);
    std::vector<double> D(d.D ? d.D : (const double*)nullptr, d.D ? d.D + N * nc * nu : nullptr);
    std::vector<double> CN(d.CN ? d.CN : (const double*)nullptr, d.CN ? d.CN + nf * nx : nullptr);
    BInst& I = B->inst[c];
    I.N = d.N; I.nx = d.nx; I.nu = d.nu; I.nc = d.nc; I.nf = d.nf; I.m = (int)(N * nc + nf);
    I.box = is_box(d, C, D, CN) ? 1 : 0;
    // general rows go through the GEMV helpers (at most 64 reduction rows)
    if (!I.box && (nc > (size_t)GSLS_MAX_NC || nf > (size_t)GSLS_MAX_NC)) return GSLS_ERR_DIM;
    I.ob = pushf(d.b, N * nx);
    {   // terminal cost, symmetric part
      std::vector<double> QN(nx * nx, 0.0);
      if (d.Q)
        for (size_t r = 0; r < nx; ++r)
          for (size_t c = 0; c < nx; ++c)
            QN[r * nx + c] = 0.5 * (d.Q[(N * nx + r) * nx + c] + d.Q[(N * nx + c) * nx + r]);
      I.oQN = pushf(QN.data(), nx * nx);
    }
    {   // epoch input packets
      const EpLayout ep = ep_layout(d.nx, d.nu);
      const size_t ld = ep.ld;
      I.oE = reservef(N * (size_t)ep.stride);
      for (size_t k = 0; k < N; ++k) {
        float* e = fpool.data() + I.oE + k * ep.stride;
        for (size_t r = 0; r < nx; ++r) {
          for (size_t c = 0; c < nx; ++c) e[ep.AB + r * ld + c] = d.A ? (float)d.A[(k * nx + r) * nx + c] : 0.f;
          for (size_t c = 0; c < nu; ++c) e[ep.AB + r * ld + nx + c] = d.B ? (float)d.B[(k * nx + r) * nu + c] : 0.f;
        }
        // cost block, symmetric part (only it enters the quadratic form)
        auto cost = [&](size_t r, size_t c) -> double {
          if (r < nx && c < nx) return d.Q ? d.Q[k * nx * nx + r * nx + c] : 0.0;
          if (r >= nx && c >= nx) return d.R ? d.R[k * nu * nu + (r - nx) * nu + (c - nx)] : 0.0;
          if (r >= nx) return d.S ? d.S[k * nu * nx + (r - nx) * nx + c] : 0.0;
          return d.S ? d.S[k * nu * nx + (c - nx) * nx + r] : 0.0;
        };
        for (size_t r = 0; r < nxu; ++r)
          for (size_t c = r; c < nxu; ++c) {
            const float v = (float)(0.5 * (cost(r, c) + cost(c, r)));
            e[ep.Z + r * ld + c] = v;
            e[ep.Z + c * ld + r] = v;
          }
      }
    }
    I.oq = pushf(d.q, (N + 1) * nx); I.orr = pushf(d.r, N * nu);
    if (!I.box) {
      std::vector<double> G(N * nc * nxu);
      for (size_t k = 0; k < N; ++k)
        for (size_t r = 0; r < nc; ++r) {
          for (size_t j = 0; j < nx; ++j) G[(k * nc + r) * nxu + j] = C[(k * nc + r) * nx + j];
          for (size_t j = 0; j < nu; ++j) G[(k * nc + r) * nxu + nx + j] = D[(k * nc + r) * nu + j];
        }
      I.oG = pushf(G.data(), G.size());
      I.oCN = pushf(CN.data(), CN.size());
    } else {
      I.oG = 0; I.oCN = 0;
    }
    I.ox0 = reservef(nx);
    const PkLayout pk = pk_layout(d.nx, d.nu);
    if (pk.stride > kPkVec * 4 * kWG) return GSLS_ERR_DIM;
    I.oPk = reservef(N * (size_t)pk.stride);
    for (size_t k = 0; k < N; ++k) {   // constant stage data of the packets
      float* pp = fpool.data() + I.oPk + k * pk.stride;
      for (size_t j = 0; j < nx; ++j) pp[pk.q + j] = d.q ? (float)d.q[k * nx + j] : 0.f;
      for (size_t j = 0; j < nu; ++j) pp[pk.r + j] = d.r ? (float)d.r[k * nu + j] : 0.f;
      for (size_t j = 0; j < nx; ++j) pp[pk.b + j] = d.b ? (float)d.b[k * nx + j] : 0.f;
    }
    I.okff = reservef(N * nu);
    I.ol = pushd(d.l, I.m); I.ou = pushd(d.u, I.m);
    I.oz = reserved(I.m); I.oy = reserved(I.m); I.ov = reserved(I.m); I.owp = reserved(I.m);
    I.oX = reserved((N + 1) * nx); I.oU = reserved(N * nu);
    lds = std::max(lds, batch_layout(d.nx, d.nu, I.box ? 0 : std::max(d.nc, d.nf)).bytes);
    cost[c] = (double)N * nxu * nxu;
  }
  B->order.resize(count);
  for (int c = 0; c < count; ++c) B->order[c] = c;
  std::stable_sort(B->order.begin(), B->order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
  if (lds > kBatchLdsMax) return GSLS_ERR_DIM;
  B->lds = lds;
  B->nfp = fpool.size(); B->ndp = dpool.size();
  if (hipMalloc(&B->fp, B->nfp * 4) != hipSuccess) return GSLS_ERR_OOM;
  if (hipMalloc(&B->dp, B->ndp * 8) != hipSuccess) return GSLS_ERR_OOM;
  if (hipMalloc(&B->d_inst, count * sizeof(BInst)) != hipSuccess) return GSLS_ERR_OOM;
  if (hipMalloc(&B->d_order, count * sizeof(int)) != hipSuccess) return GSLS_ERR_OOM;
  if (hipMalloc(&B->d_rho, count * sizeof(double)) != hipSuccess) return GSLS_ERR_OOM;
  if (hipMalloc(&B->d_warm, count * sizeof(int)) != hipSuccess) return GSLS_ERR_OOM;
  if (hipMalloc(&B->d_res, count * sizeof(BResult)) != hipSuccess) return GSLS_ERR_OOM;
  if (hipMalloc(&B->d_args, sizeof(BatchArgs)) != hipSuccess) return GSLS_ERR_OOM;
  if (hipMalloc(&B->d_sync, sizeof(BSync)) != hipSuccess) return GSLS_ERR_OOM;
  if (hipMalloc(&B->d_cont, count * sizeof(int)) != hipSuccess) return GSLS_ERR_OOM;
  if (hipMalloc(&B->d_join, count * sizeof(unsigned)) != hipSuccess) return GSLS_ERR_OOM;
  if (hipMalloc(&B->d_park, count * sizeof(BPark)) != hipSuccess) return GSLS_ERR_OOM;
  if (hipMemcpy(B->fp, fpool.data(), B->nfp * 4, hipMemcpyHostToDevice) != hipSuccess) return GSLS_ERR_HIP;
  if (hipMemcpy(B->dp, dpool.data(), B->ndp * 8, hipMemcpyHostToDevice) != hipSuccess) return GSLS_ERR_HIP;
  if (hipMemcpy(B->d_inst, B->inst.data(), count * sizeof(BInst), hipMemcpyHostToDevice) != hipSuccess)
    return GSLS_ERR_HIP;
  if (hipMemcpy(B->d_order, B->order.data(), count * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
    return GSLS_ERR_HIP;
  if (hipFuncSetAttribute((const void*)k_batch, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return GSLS_ERR_HIP;
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return GSLS_ERR_HIP;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return GSLS_ERR_HIP;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void*)k_batch, kWG, lds) != hipSuccess) per = 1;
  B->grid = cus * std::max(per, 1);
  if (hipEventCreate(&B->e0) != hipSuccess || hipEventCreate(&B->e1) != hipSuccess) return GSLS_ERR_HIP;
  if (int rc = batch_set_schedule(B, 0, 0.0)) return rc;
  B->row_off.assign(count + 1, 0);
  for (int c = 0; c < count; ++c) B->row_off[c + 1] = B->row_off[c] + B->inst[c].N + 1;
  const int rows = B->row_off[count];
  std::vector<int> row_inst(rows);
  for (int c = 0; c < count; ++c)
    for (int r = B->row_off[c]; r < B->row_off[c + 1]; ++r) row_inst[r] = c;
  if (hipMalloc(&B->d_row_inst, rows * sizeof(int)) != hipSuccess) return GSLS_ERR_OOM;
  if (hipMalloc(&B->d_row_off, (count + 1) * sizeof(int)) != hipSuccess) return GSLS_ERR_OOM;
  if (hipMemcpy(B->d_row_inst, row_inst.data(), rows * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
    return GSLS_ERR_HIP;
  if (hipMemcpy(B->d_row_off, B->row_off.data(), (count + 1) * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
    return GSLS_ERR_HIP;
  return GSLS_OK;
}

// Solo cost model of one stage of one iteration on one workgroup (us): a
// fixed latency per stage and direction plus a part growing with the packet
// (fitted to the per-instance device times of the uneven benchmark batch).
static double solo_stage_us(int nx, int nu) { return 2.9 + 0.068 * (nx + nu); }

int batch_set_schedule(BatchSolver* B, int gang, double park_share) {
  if (gang < 0 || gang > kGangMax || !(park_share >= 0.0) || !std::isfinite(park_share)) return GSLS_ERR_INVALID_ARG;
  if (gang == 0) gang = kGangAuto;
  if (park_share == 0.0) park_share = kParkShareAuto;
  gang = std::min(gang, B->grid / 2);
  if (gang < 2) gang = 1;
  const int count = B->count;
  // hand-over points: an instance long enough to split (N >= 2 G) leaves
  // its solo workgroup once its estimated solo work exceeds park_share times
  // one workgroup's share of the batch (every instance at 100 iterations)
  double total = 0.0;
  for (const BInst& I : B->inst) total += (double)I.N * solo_stage_us(I.nx, I.nu);
  const double wb = park_share * total * 100.0 / (double)B->grid;
  size_t nw = 0, nm = 0;
  for (BInst& I : B->inst) {
    I.park_at = 0x7fffffff;
    I.ogw = 0; I.ogm = 0;
    if (gang > 1 && I.N >= 2 * gang) {
      const double w = (double)I.N * solo_stage_us(I.nx, I.nu);
      I.park_at = (int)std::max(10.0, std::ceil(wb / w));
      I.ogw = (long long)nw; I.ogm = (long long)nm;
      nw += gang_layout(I.nx, gang).words;
      nm += (gang_map_floats(I.nx, gang) + 63) & ~(size_t)63;
    }
  }
  if (B->d_gwords) { (void)hipFree(B->d_gwords); B->d_gwords = nullptr; }
  if (B->d_gmaps) { (void)hipFree(B->d_gmaps); B->d_gmaps = nullptr; }
  if (nw > 0) {
    if (hipMalloc(&B->d_gwords, nw * 8) != hipSuccess) return GSLS_ERR_OOM;
    if (hipMalloc(&B->d_gmaps, nm * 4) != hipSuccess) return GSLS_ERR_OOM;
  } else {
    gang = 1;
  }
  if (hipMemcpy(B->d_inst, B->inst.data(), count * sizeof(BInst), hipMemcpyHostToDevice) != hipSuccess)
    return GSLS_ERR_HIP;
  B->gang = gang;
  B->park_share = park_share;
  // the captured launch depends on the schedule
  if (B->gexec) { (void)hipGraphExecDestroy(B->gexec); B->gexec = nullptr; }
  if (B->graph) { (void)hipGraphDestroy(B->graph); B->graph = nullptr; }
  return GSLS_OK;
}

int batch_upload_x0(BatchSolver* B, const double* const* x0) {
  const int count = B->count;
  if (!x0) return GSLS_ERR_INVALID_ARG;
  for (int c = 0; c < count; ++c) {
    if (!x0[c]) return GSLS_ERR_INVALID_ARG;
    for (int j = 0; j < B->inst[c].nx; ++j)
      if (!std::isfinite(x0[c][j])) return GSLS_ERR_INVALID_ARG;
  }
  // host staging in pinned-free pageable memory: the copies are synchronous
  // with respect to the host before this function returns
  std::vector<float> xf;
  std::vector<size_t> xoff(count);
  for (int c = 0; c < count; ++c) {
    xoff[c] = xf.size();
    for (int j = 0; j < B->inst[c].nx; ++j) xf.push_back((float)x0[c][j]);
  }
  for (int c = 0; c < count; ++c) {
    const BInst& I = B->inst[c];
    if (hipMemcpyAsync(B->fp + I.ox0, xf.data() + xoff[c], I.nx * 4, hipMemcpyHostToDevice, B->stream) !=
        hipSuccess)
      return GSLS_ERR_HIP;
  }
  if (hipStreamSynchronize(B->stream) != hipSuccess) return GSLS_ERR_HIP;
  return GSLS_OK;
}

int batch_run(BatchSolver* B, double tol, int warm_budget, gsls_result* out, double* ms) {
  const int count = B->count;
  BatchArgs a{};
  a.inst = B->d_inst; a.order = B->d_order; a.count = count; a.fp = B->fp; a.dp = B->dp; a.rho0 = B->d_rho;
  a.tol = tol; a.max_iter = B->st.max_iter; a.adaptive = B->st.adaptive_rho; a.sigma = B->st.sigma;
  a.refresh = B->st.refresh;
  a.rho_min = B->st.rho_min; a.rho_max = B->st.rho_max; a.rho_tol = B->st.rho_tol;
  a.res = B->d_res; a.warm = B->d_warm;
  a.gang = B->gang; a.sync = (BSync*)B->d_sync; a.cont_list = B->d_cont; a.join = B->d_join;
  a.park = (BPark*)B->d_park; a.gwords = B->d_gwords; a.gmaps = B->d_gmaps;
  a.warm_budget = warm_budget; a.rho_cold = 1.0;
  a.prof = B->d_prof;
  if (hipMemcpyAsync(B->d_args, &a, sizeof(a), hipMemcpyHostToDevice, B->stream) != hipSuccess) return GSLS_ERR_HIP;
  // the launch (counter reset by a fill kernel, then the persistent solver) is
  // captured once per (tol, warm budget) into a graph and replayed
  const double pkey = B->d_prof ? 1.0 : 0.0;
  if (!B->gexec || B->graph_key[0] != tol || B->graph_key[1] != (double)warm_budget || B->graph_key[2] != pkey) {
    if (B->gexec) { (void)hipGraphExecDestroy(B->gexec); B->gexec = nullptr; }
    if (B->graph) { (void)hipGraphDestroy(B->graph); B->graph = nullptr; }
    hipStream_t cs;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return GSLS_ERR_HIP;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) return GSLS_ERR_HIP;
    k_batch_prologue<<<(count + 255) / 256, 256, 0, cs>>>((BSync*)B->d_sync, B->d_cont, B->d_join, count);
    k_batch<<<B->grid, kWG, B->lds, cs>>>(B->d_args);
    k_batch_rdyn<<<B->row_off[count], kWG, 0, cs>>>(B->d_inst, B->fp, B->dp, B->d_row_inst, B->d_row_off,
                                                      B->d_res);
    if (hipStreamEndCapture(cs, &B->graph) != hipSuccess) return GSLS_ERR_HIP;
    (void)hipStreamDestroy(cs);
    if (hipGraphInstantiate(&B->gexec, B->graph, nullptr, nullptr, 0) != hipSuccess) return GSLS_ERR_HIP;
    B->graph_key[0] = tol;
    B->graph_key[1] = (double)warm_budget;
    B->graph_key[2] = pkey;
  }
  if (hipEventRecord(B->e0, B->stream) != hipSuccess) return GSLS_ERR_HIP;
  if (hipGraphLaunch(B->gexec, B->stream) != hipSuccess) return GSLS_ERR_HIP;
  if (hipEventRecord(B->e1, B->stream) != hipSuccess) return GSLS_ERR_HIP;
  std::vector<BResult> res(count);
  if (hipMemcpyAsync(res.data(), B->d_res, count * sizeof(BResult), hipMemcpyDeviceToHost, B->stream) != hipSuccess)
    return GSLS_ERR_HIP;
  if (hipStreamSynchronize(B->stream) != hipSuccess) return GSLS_ERR_HIP;
  float t = 0.f;
  (void)hipEventElapsedTime(&t, B->e0, B->e1);
  if (ms) *ms = t;
  int rc = GSLS_OK;
  for (int c = 0; c < count; ++c) {
    gsls_result r{};
    const BResult& b = res[c];
    if (b.status == -1) rc = GSLS_ERR_NOT_PD;
    if (b.status == 5 && rc == GSLS_OK) rc = GSLS_ERR_HIP;   // a gang's bounded wait gave up
    r.status = b.status == 1 ? GSLS_SOLVED : (b.status == 2 ? GSLS_MAX_ITER : GSLS_NUMERICAL_FAIL);
    r.iterations = b.iterations; r.rho_updates = b.rho_updates; r.factorizations = b.factorizations;
    r.r_p = b.r_p; r.r_d = b.r_d; r.rho = b.rho; r.ms_total = t; r.r_dyn = b.r_dyn;
    r.ms_factor = (double)b.t_epoch * 1e-5;    // 100 MHz counter -> ms (this instance's workgroup)
    r.ms_iterate = (double)b.t_iter * 1e-5;
    r.cold_restart = b.restarted;
    out[c] = r;
  }
  return rc;
}

int batch_solve(BatchSolver* B, const double* const* x0, const double* rho, double tol, const double* const* z0,
                const double* const* y0, gsls_result* out, double* ms) {
  const int count = B->count;
  if (!x0 || !rho || !out || !(tol >= 0)) return GSLS_ERR_INVALID_ARG;
  for (int c = 0; c < count; ++c)
    if (!(rho[c] > 0) || !std::isfinite(rho[c])) return GSLS_ERR_INVALID_ARG;
  int rc = batch_upload_x0(B, x0);
  if (rc) return rc;
  std::vector<int> warm(count, 0);
  for (int c = 0; c < count; ++c) {
    const BInst& I = B->inst[c];
    if (z0 && y0 && z0[c] && y0[c]) {
      warm[c] = 1;
      if (hipMemcpyAsync(B->dp + I.oz, z0[c], I.m * 8, hipMemcpyHostToDevice, B->stream) != hipSuccess)
        return GSLS_ERR_HIP;
      if (hipMemcpyAsync(B->dp + I.oy, y0[c], I.m * 8, hipMemcpyHostToDevice, B->stream) != hipSuccess)
        return GSLS_ERR_HIP;
    }
  }
  if (hipMemcpyAsync(B->d_rho, rho, count * 8, hipMemcpyHostToDevice, B->stream) != hipSuccess) return GSLS_ERR_HIP;
  if (hipMemcpyAsync(B->d_warm, warm.data(), count * 4, hipMemcpyHostToDevice, B->stream) != hipSuccess)
    return GSLS_ERR_HIP;
  return batch_run(B, tol, 0, out, ms);
}

int batch_get(BatchSolver* B, int idx, double* X, double* U, double* z, double* lam, double rho_final) {
  if (idx < 0 || idx >= B->count) return GSLS_ERR_INVALID_ARG;
  const BInst& I = B->inst[idx];
  auto cp = [&](double* dst, long long off, size_t n, double sc) -> int {
    if (!dst) return GSLS_OK;
    if (hipMemcpy(dst, B->dp + off, n * 8, hipMemcpyDeviceToHost) != hipSuccess) return GSLS_ERR_HIP;
    if (sc != 1.0)
      for (size_t i = 0; i < n; ++i) dst[i] *= sc;
    return GSLS_OK;
  };
  int rc;
  if ((rc = cp(X, I.oX, (size_t)(I.N + 1) * I.nx, 1.0))) return rc;
  if ((rc = cp(U, I.oU, (size_t)I.N * I.nu, 1.0))) return rc;
  if ((rc = cp(z, I.oz, I.m, 1.0))) return rc;
  if ((rc = cp(lam, I.oy, I.m, rho_final))) return rc;
  return GSLS_OK;
}

}  // namespace gsls

// ================================================================ C ABI
extern "C" {

int gsls_qp_setup_batch(const gsls_qp_desc* descs, int32_t count, const gsls_settings* settings, void* stream,
                        gsls_batch** out) {
  if (!descs || count < 1 || !out) return GSLS_ERR_INVALID_ARG;
  *out = nullptr;
  gsls_settings s;
  gsls_default_settings(&s);
  if (settings) s = *settings;
  if (int rc = gsls::check_settings(&s)) return rc;
  for (int c = 0; c < count; ++c) {
    // box rows ([x; u] per stage) may number up to nx + nu <= 96; general
    // rows are limited in batch_setup
    int rc = gsls::validate_host_desc(&descs[c], gsls::kBatchMaxNxu);
    if (rc) return rc;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return GSLS_ERR_HIP;
  gsls_batch* b = new (std::nothrow) gsls_batch;
  if (!b) return GSLS_ERR_OOM;
  int rc = gsls::batch_setup(descs, count, &s, (hipStream_t)stream, &b->s);
  if (rc) { delete b; return rc; }
  b->rho_final.assign(count, 1.0);
  *out = b;
  return GSLS_OK;
}

int gsls_qp_solve_batch(gsls_batch* b, const double* const* x0, const double* rho, double tol,
                        const double* const* z0, const double* const* y0, gsls_result* out, double* ms) {
  if (!b) return GSLS_ERR_INVALID_ARG;
  int rc = gsls::batch_solve(&b->s, x0, rho, tol, z0, y0, out, ms);
  if (out)
    for (int c = 0; c < b->s.count; ++c) b->rho_final[c] = out[c].rho;
  return rc;
}

int gsls_batch_get(gsls_batch* b, int32_t index, double* X, double* U, double* z, double* lambda) {
  if (!b || index < 0 || index >= b->s.count) return GSLS_ERR_INVALID_ARG;
  return gsls::batch_get(&b->s, index, X, U, z, lambda, b->rho_final[index]);
}

void gsls_batch_free(gsls_batch* b) { delete b; }

int gsls_batch_set_schedule(gsls_batch* b, int32_t gang, double park_share) {
  if (!b) return GSLS_ERR_INVALID_ARG;
  return gsls::batch_set_schedule(&b->s, gang, park_share);
}

int gsls_batch_get_schedule(gsls_batch* b, int32_t* gang, double* park_share, int32_t* park_at) {
  if (!b) return GSLS_ERR_INVALID_ARG;
  if (gang) *gang = b->s.gang;
  if (park_share) *park_share = b->s.park_share;
  if (park_at)
    for (int c = 0; c < b->s.count; ++c) park_at[c] = b->s.inst[c].park_at;
  return GSLS_OK;
}

int gsls_batch_debug_phase_cycles(gsls_batch* b, int32_t enable, double* cycles16) {
  if (!b) return GSLS_ERR_INVALID_ARG;
  gsls::BatchSolver* B = &b->s;
  if (cycles16) {
    for (int i = 0; i < 16; ++i) cycles16[i] = 0.0;
    if (B->d_prof) {
      unsigned long long h[16];
      if (hipMemcpy(h, B->d_prof, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) return GSLS_ERR_HIP;
      for (int i = 0; i < 16; ++i) cycles16[i] = (double)h[i];
    }
  }
  if (enable && !B->d_prof) {
    if (hipMalloc(&B->d_prof, 16 * sizeof(unsigned long long)) != hipSuccess) return GSLS_ERR_OOM;
  } else if (!enable && B->d_prof) {
    (void)hipFree(B->d_prof);
    B->d_prof = nullptr;
  }
  if (B->d_prof && hipMemset(B->d_prof, 0, 16 * sizeof(unsigned long long)) != hipSuccess) return GSLS_ERR_HIP;
  return GSLS_OK;
}

}  // extern "C"
