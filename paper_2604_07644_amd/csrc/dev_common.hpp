// Device building blocks shared by the gfx950 kernels: workgroup GEMM on
// register micro-tiles, FP32 MFMA products of LDS operands, FP64 Gauss-Jordan
// elimination held in registers (partial pivoting, or none for symmetric
// positive definite systems), workgroup matrix-vector products, and the
// packed (payload, stamp) words used for low-latency exchange between
// workgroups of a persistent kernel.
//
// All routines with the prefix wg_ must be called by every thread of the
// workgroup (they contain __syncthreads); the workgroup size is kWG threads.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// Pointer qualifier for the local data share: accesses through it compile to
// ds_read / ds_write (a generic pointer would take the flat path).
#define LDS __attribute__((address_space(3)))

namespace gsls {

constexpr int kWG = 256;          // threads per workgroup
constexpr int kMaxNx = 80;        // largest state dimension handled
constexpr int kMaxNu = 32;        // largest control dimension
constexpr int kMaxNc = 64;        // largest number of stage rows
constexpr int kKT = 16;           // K-slab depth of the workgroup GEMM
constexpr unsigned kSpinLimit = 1u << 22;   // bounded waits (a few seconds): give up and flag an error

__device__ __forceinline__ int tid() { return threadIdx.x; }

// Global-memory address space: loads and stores through such pointers are
// global_* instructions (counted by vmcnt only), not flat ones (which also
// count against lgkmcnt and so make every LDS wait wait for them too).
#define GLB __attribute__((address_space(1)))

// A pointer known to be the same in every lane (e.g. a device function
// argument derived from kernel arguments) moved to scalar registers, so that
// address arithmetic on it stays scalar and buffer descriptors built from it
// need no per-lane loop.
template <typename T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
  const unsigned long long v = (unsigned long long)p;
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
  return (T*)(((unsigned long long)hi << 32) | lo);
}

// The same for an LDS pointer, an int and a scalar of 4 or 8 bytes.  Device
// functions that are not inlined receive their arguments in vector registers;
// these calls tell the compiler that workgroup-uniform arguments are uniform,
// so loops over them stay scalar branches and address arithmetic stays scalar.
template <typename T>
__device__ __forceinline__ LDS T* uniform_lds(LDS T* p) {
  return (LDS T*)(uintptr_t)__builtin_amdgcn_readfirstlane((unsigned)(uintptr_t)p);
}
__device__ __forceinline__ int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float uniform_val(float v) {
  return __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(v)));
}
__device__ __forceinline__ double uniform_val(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Workgroup barrier that orders LDS only: waits for the thread's own LDS
// operations, then s_barrier.  Unlike __syncthreads() it does not wait for
// outstanding global loads and stores, so prefetches stay in flight and
// stores drain in the background.  Valid only where every global location a
// thread reads after the barrier was written by that same thread (or before
// the kernel began); cross-thread global data needs __syncthreads().
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ------------------------------------------------------------------ GEMM
// Reductions up to this many K-slabs have all their loads issued at once.
constexpr int kGemmSlabsInFlight = 5;

// C = alpha * op(A) * op(B) + beta * C, with op(A) m x k and op(B) k x n.
//   A element (i, t) = ta ? A[t*lda + i] : A[i*lda + t]
//   B element (t, j) = tb ? B[j*ldb + t] : B[t*ldb + j]
// Thread (ty, tx) of a 16 x 16 grid owns rows ty + 16a and columns tx + 16b of
// C (a, b < TT).  op(A) and op(B) pass through LDS in K-slabs of kKT; each
// thread holds TT elements of each slab in registers.  For k up to
// kGemmSlabsInFlight slabs all loads are issued before the first product (a
// single global latency per product); beyond that the next slab's loads
// overlap the current product.  Indices are clamped into range (loads never leave
// the operand) and out-of-range terms masked to zero.  beta == 0 never reads
// C.  All reads of A and B complete before C is written, so C may alias them.
// smem: 2 * 16*TT * kKT elements.
template <typename T, int TT>
__device__ void wg_gemm_tt(int m, int n, int k, T alpha, const T* A, int lda, bool ta,
                           const T* B, int ldb, bool tb, T beta, T* C, int ldc, LDS T* smem) {
  constexpr int MM = 16 * TT;
  constexpr int NS = kGemmSlabsInFlight;
  LDS T* As = smem;              // [MM][kKT]
  LDS T* Bs = smem + MM * kKT;   // [kKT][MM]
  const int tx = tid() & 15, ty = tid() >> 4;
  T acc[TT][TT];
#pragma unroll
  for (int a = 0; a < TT; ++a)
#pragma unroll
    for (int b = 0; b < TT; ++b) acc[a][b] = T(0);
  auto load = [&](int t0, T* ra, T* rb) {
#pragma unroll
    for (int q = 0; q < TT; ++q) {
      const int e = tid() + q * kWG;
      const int i = e / kKT, t = e % kKT;
      const int ic = min(i, m - 1), tc = min(t0 + t, k - 1);
      T v = ta ? A[(size_t)tc * lda + ic] : A[(size_t)ic * lda + tc];
      ra[q] = (i < m && t0 + t < k) ? v : T(0);
    }
#pragma unroll
    for (int q = 0; q < TT; ++q) {
      const int e = tid() + q * kWG;
      const int t = e / MM, j = e % MM;
      const int jc = min(j, n - 1), tc = min(t0 + t, k - 1);
      T v = tb ? B[(size_t)jc * ldb + tc] : B[(size_t)tc * ldb + jc];
      rb[q] = (j < n && t0 + t < k) ? v : T(0);
    }
  };
  auto multiply = [&](const T* ra, const T* rb) {
#pragma unroll
    for (int q = 0; q < TT; ++q) {
      const int e = tid() + q * kWG;
      As[(e / kKT) * kKT + e % kKT] = ra[q];
      Bs[e] = rb[q];
    }
    __syncthreads();
    // slabs are zero-padded past k, so the slab loop has a fixed trip count
#pragma unroll
    for (int t = 0; t < kKT; ++t) {
      T av[TT], bv[TT];
#pragma unroll
      for (int a = 0; a < TT; ++a) av[a] = As[(ty + 16 * a) * kKT + t];
#pragma unroll
      for (int b = 0; b < TT; ++b) bv[b] = Bs[t * MM + tx + 16 * b];
#pragma unroll
      for (int a = 0; a < TT; ++a)
#pragma unroll
        for (int b = 0; b < TT; ++b) acc[a][b] += av[a] * bv[b];
    }
    __syncthreads();
  };
  if (k <= NS * kKT) {
    // every slab's loads are issued up front: one global latency per product
    T ra[NS][TT], rb[NS][TT];
#pragma unroll
    for (int sl = 0; sl < NS; ++sl)
      if (sl * kKT < k) load(sl * kKT, ra[sl], rb[sl]);
#pragma unroll
    for (int sl = 0; sl < NS; ++sl)
      if (sl * kKT < k) multiply(ra[sl], rb[sl]);
  } else {
    // longer reductions: the next slab's loads overlap the current product
    T ra[TT], rb[TT], na[TT], nb[TT];
    load(0, ra, rb);
    for (int t0 = 0; t0 < k; t0 += kKT) {
      if (t0 + kKT < k) load(t0 + kKT, na, nb);
      multiply(ra, rb);
#pragma unroll
      for (int q = 0; q < TT; ++q) { ra[q] = na[q]; rb[q] = nb[q]; }
    }
  }
#pragma unroll
  for (int a = 0; a < TT; ++a) {
    int i = ty + 16 * a;
    if (i >= m) continue;
#pragma unroll
    for (int b = 0; b < TT; ++b) {
      int j = tx + 16 * b;
      if (j >= n) continue;
      T v = alpha * acc[a][b];
      if (beta != T(0)) v += beta * C[(size_t)i * ldc + j];
      C[(size_t)i * ldc + j] = v;
    }
  }
  __syncthreads();
}

template <typename T>
__device__ void wg_gemm(int m, int n, int k, T alpha, const T* A, int lda, bool ta, const T* B,
                        int ldb, bool tb, T beta, T* C, int ldc, LDS T* smem) {
  m = uniform_int(m); n = uniform_int(n); k = uniform_int(k);
  lda = uniform_int(lda); ldb = uniform_int(ldb); ldc = uniform_int(ldc);
  ta = uniform_int(ta) != 0; tb = uniform_int(tb) != 0;
  alpha = uniform_val(alpha); beta = uniform_val(beta);
  A = uniform_ptr(A); B = uniform_ptr(B); C = uniform_ptr(C); smem = uniform_lds(smem);
  int mx = max(m, n);
  if (mx <= 16) wg_gemm_tt<T, 1>(m, n, k, alpha, A, lda, ta, B, ldb, tb, beta, C, ldc, smem);
  else if (mx <= 32) wg_gemm_tt<T, 2>(m, n, k, alpha, A, lda, ta, B, ldb, tb, beta, C, ldc, smem);
  else if (mx <= 48) wg_gemm_tt<T, 3>(m, n, k, alpha, A, lda, ta, B, ldb, tb, beta, C, ldc, smem);
  else if (mx <= 64) wg_gemm_tt<T, 4>(m, n, k, alpha, A, lda, ta, B, ldb, tb, beta, C, ldc, smem);
  else wg_gemm_tt<T, 5>(m, n, k, alpha, A, lda, ta, B, ldb, tb, beta, C, ldc, smem);
}
constexpr int kGemmSmem = 2 * 16 * 5 * kKT;   // elements of T needed by wg_gemm

// Element loops of the workgroup helpers are two-dimensional: the four waves
// take rows w, w+4, ... and the 64 lanes take columns lane, lane+64, ..., so
// no index is ever divided at run time.
__device__ __forceinline__ int wave() { return threadIdx.x >> 6; }
__device__ __forceinline__ int lane() { return threadIdx.x & 63; }

// Element loops over an m x n block in passes of 32 rows: wave w and lane l
// take rows w + 4q (q < 8) and columns l, l + 64 (n <= 128) of the pass, and
// every load of a thread in a pass is issued before its first store, so a
// pass costs one memory latency instead of one per row.
constexpr int kPassRows = 8;
template <typename TV, typename Load, typename Store>
__device__ __forceinline__ void wg_block_pass(int m, int n, Load load, Store store) {
  for (int q0 = 0; 4 * q0 < m; q0 += kPassRows) {
    TV v[kPassRows][2];
#pragma unroll
    for (int q = 0; q < kPassRows; ++q)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int i = wave() + 4 * (q0 + q), j = lane() + 64 * b;
        if (i < m && j < n) v[q][b] = load(i, j);
      }
#pragma unroll
    for (int q = 0; q < kPassRows; ++q)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int i = wave() + 4 * (q0 + q), j = lane() + 64 * b;
        if (i < m && j < n) store(i, j, v[q][b]);
      }
  }
}

// Copy / convert a matrix block: dst[i*ldd + j] = src[i*lds + j] (or transposed), n <= 128.
template <typename TD, typename TS>
__device__ void wg_copy(int m, int n, TD* dst, int ldd, const TS* src, int lds, bool trans = false) {
  wg_block_pass<TD>(m, n, [&](int i, int j) { return TD(trans ? src[(size_t)j * lds + i] : src[(size_t)i * lds + j]); },
                    [&](int i, int j, TD v) { dst[(size_t)i * ldd + j] = v; });
}

// Symmetrise a square matrix in place: P = (P + P^T) / 2 (n <= 128).  Every
// thread reads both halves of its pairs before any write; the result is
// written to both triangles.
template <typename T>
__device__ void wg_symmetrize(int n, T* P, int ld) {
  __syncthreads();
  wg_block_pass<T>(n, n, [&](int i, int j) { return j > i ? T(0.5) * (P[(size_t)i * ld + j] + P[(size_t)j * ld + i]) : T(0); },
                   [&](int i, int j, T v) {
                     if (j > i) {
                       P[(size_t)i * ld + j] = v;
                       P[(size_t)j * ld + i] = v;
                     }
                   });
  __syncthreads();
}


// ------------------------------------------------------- MFMA GEMM (FP32)
// C = alpha * op(A) * op(B) + beta * C on the matrix cores, op(A) m x k and
// op(B) k x n with A and B in LDS (op = transpose when ta / tb), C anywhere.
// The output is cut into 16 x 16 tiles handed round-robin to the four waves;
// a wave accumulates its tile with v_mfma_f32_16x16x4f32, lane l supplying
// A[i0 + l%16][k0 + l/16] and B[k0 + l/16][j0 + l%16], and holding
// C[i0 + 4(l/16) + r][j0 + l%16] in accumulator r.  Out-of-range operands are
// clamped into range and zeroed.  Ends with a barrier.  C must not alias A/B.
typedef float mfma_f4 __attribute__((ext_vector_type(4)));

template <typename PC>
__device__ inline void wg_mm_f32(int m, int n, int k, float alpha, const LDS float* A, int lda, bool ta,
                                 const LDS float* B, int ldb, bool tb, float beta, PC C, int ldc) {
  const int l = lane(), w = wave();
  const int tn = (n + 15) >> 4, tm = (m + 15) >> 4;
  const int r16 = l & 15, q = l >> 4;
  for (int t = w; t < tm * tn; t += 4) {
    const int ti = t / tn, tj = t - ti * tn;
    const int i = ti * 16 + r16, j = tj * 16 + r16;
    const int ic = min(i, m - 1), jc = min(j, n - 1);
    const float ma = i < m ? 1.f : 0.f, mb = j < n ? 1.f : 0.f;
    mfma_f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
    for (int k0 = 0; k0 < k; k0 += 4) {
      const int kk = k0 + q;
      const int kc = min(kk, k - 1);
      const float mk = kk < k ? 1.f : 0.f;
      const float av = ta ? A[kc * lda + ic] : A[ic * lda + kc];
      const float bv = tb ? B[jc * ldb + kc] : B[kc * ldb + jc];
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av * ma * mk, bv * mb, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int ii = ti * 16 + 4 * q + r, jj = tj * 16 + r16;
      if (ii < m && jj < n) {
        float v = alpha * acc[r];
        if (beta != 0.f) v += beta * C[ii * ldc + jj];
        C[ii * ldc + jj] = v;
      }
    }
  }
  __syncthreads();
}

// Sum (2-norm or 1-norm) of each row of the m x n matrix M (LDS): out[r] for
// r < m, one wave per row at a time.
__device__ inline void wg_row_norms(int m, int n, const LDS float* M, int ld, int rownorm, float* out,
                                    bool squared) {
  const int l = lane(), w = wave();
  for (int r = w; r < m; r += 4) {
    float s = 0.f;
    for (int c = l; c < n; c += 64) {
      const float v = M[r * ld + c];
      s += rownorm == 1 ? fabsf(v) : v * v;
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (l == 0) out[r] = (rownorm == 1 || squared) ? s : sqrtf(s);
  }
}

// -------------------------------------------------- FP64 Gauss-Jordan elimination
// Gauss-Jordan elimination of Aug = [M | R] (LDS, FP64, n x ld row-major,
// ld = n + r, the caller fills both parts): on success the right part holds
// M^{-1} R up to the row permutation perm and the row scales dg, i.e.
// (M^{-1} R)[j][c] = Aug[perm[j]][n + c] * dg[j] (read with wg_gj_extract).
// Column j's pivot is the largest |entry| among rows not used as pivots yet,
// the lowest such row on ties (pivot = true), or simply row j (pivot = false:
// for symmetric positive definite M, where every pivot must then be
// positive).  Rows are never swapped and the pivot rows are normalised at the
// end (elimination and row scaling commute).  Returns false uniformly on a
// zero, negative (SPD mode) or non-finite pivot.  perm: LDS int[n];
// dg: LDS double[n]; used: unused (kept for the callers' layouts).
//
// The matrix lives in registers for the whole elimination: lane l holds rows
// l and l + 64 (RS slots), wave w holds columns w + 4k (KC slots).  Column j
// is owned by one wave; while step j - 1 updates it, that wave also copies it
// into an LDS vector (double-buffered by step parity), so the owner can pick
// the pivot from it and every thread reads its row's multiplier from it after
// the step's single (LDS-only) barrier.  The pivot row is broadcast inside
// each wave with readlane, and the update is one FMA per register:
//   a[r][c] -= (a[r][j] / a[p][j]) * a[p][c]   for r != p
// (applied to every column: those up to j are dead and never read again).
// The pivot search compares |a[r][j]| rounded to FP32 (a monotone key), so
// among candidates equal at that precision the lowest row is taken.
__device__ __forceinline__ double readlane_f64(double v, int l) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Maximum of an unsigned key over the 64 lanes of the wave: a butterfly
// inside each row of 16 lanes (quad swaps 1 and 2, half-row and row mirrors),
// then the four row results combined on the scalar unit.
__device__ __forceinline__ unsigned wave_max_u32(unsigned k) {
  k = max(k, (unsigned)__builtin_amdgcn_update_dpp(0, (int)k, 0xB1, 0xF, 0xF, true));
  k = max(k, (unsigned)__builtin_amdgcn_update_dpp(0, (int)k, 0x4E, 0xF, 0xF, true));
  k = max(k, (unsigned)__builtin_amdgcn_update_dpp(0, (int)k, 0x141, 0xF, 0xF, true));
  k = max(k, (unsigned)__builtin_amdgcn_update_dpp(0, (int)k, 0x140, 0xF, 0xF, true));
  const unsigned r0 = (unsigned)__builtin_amdgcn_readlane((int)k, 0);
  const unsigned r1 = (unsigned)__builtin_amdgcn_readlane((int)k, 16);
  const unsigned r2 = (unsigned)__builtin_amdgcn_readlane((int)k, 32);
  const unsigned r3 = (unsigned)__builtin_amdgcn_readlane((int)k, 48);
  return max(max(r0, r1), max(r2, r3));
}

template <int RS, int KC>
__device__ __forceinline__ bool gj_eliminate_regs(int n, int ld, LDS double* Aug, bool pivot, LDS int* perm,
                                                  LDS double* dg, LDS int* s_piv, LDS double* s_inv) {
  const int l = lane();
  const int w = __builtin_amdgcn_readfirstlane(wave());
  double a[RS][KC];
  __syncthreads();   // the caller's fill of Aug
#pragma unroll
  for (int s = 0; s < RS; ++s)
#pragma unroll
    for (int k = 0; k < KC; ++k) {
      const int r = l + 64 * s, c = w + 4 * k;
      a[s][k] = (r < n && c < ld) ? Aug[r * ld + c] : 0.0;
    }
  // Aug is dead until the write-back: its first 2n entries hold the column
  // copies of even and odd steps (ld > n, so n * ld >= 2n)
  LDS double* col[2] = {Aug, Aug + n};
  lds_barrier();
  if (w == 0) {
#pragma unroll
    for (int s = 0; s < RS; ++s)
      if (l + 64 * s < n) col[0][l + 64 * s] = a[s][0];
  }
  unsigned used = 0;   // bit s: row l + 64 s has been a pivot row
  for (int j = 0; j < n; ++j) {
    const int b = j & 1;
    LDS double* cj = col[b];
    if (w == (j & 3)) {
      // the owner of column j selects the pivot from its LDS copy
      int p = j;
      if (pivot) {
        unsigned key[RS];
        unsigned kmax = 0;
#pragma unroll
        for (int s = 0; s < RS; ++s) {
          const int r = l + 64 * s;
          const double av = r < n ? fabs(cj[r]) : -1.0;
          key[s] = (!((used >> s) & 1u) && av >= 0.0) ? __float_as_uint((float)av) : 0u;
          kmax = max(kmax, key[s]);
        }
        kmax = wave_max_u32(kmax);
        p = n;   // no candidate, or all zero: singular
        if (kmax != 0u) {
#pragma unroll
          for (int s = RS - 1; s >= 0; --s) {
            const unsigned long long m = __ballot(key[s] == kmax);
            if (m) p = 64 * s + __builtin_ctzll(m);
          }
        }
      }
      if (l == 0) {
        const double pv = p < n ? cj[p] : 0.0;
        const bool bad = p >= n || !(pivot ? fabs(pv) > 0.0 : pv > 0.0) || !isfinite(pv);
        s_piv[b] = bad ? -1 : p;
        if (!bad) {
          const double iv = 1.0 / pv;
          s_inv[b] = iv;
          perm[j] = p;
          dg[j] = iv;
        }
      }
    }
    lds_barrier();
    const int p = s_piv[b];
    if (p < 0) return false;
    const double inv = s_inv[b];
    double mult[RS];
#pragma unroll
    for (int s = 0; s < RS; ++s) {
      const int r = l + 64 * s;
      mult[s] = (r == p || r >= n) ? 0.0 : cj[r] * inv;
    }
    if (l == (p & 63)) used |= 1u << (p >> 6);
    const int pl = p & 63;
    const bool hi_slot = RS > 1 && p >= 64;
    LDS double* cn = col[b ^ 1];
    const int kn = (j + 1 - w) >> 2;   // the next column's slot, if this wave owns it
    const bool owner_next = ((j + 1) & 3) == w && j + 1 < n;
#pragma unroll
    for (int k = 0; k < KC; ++k) {
      const double pr = readlane_f64(hi_slot ? a[RS - 1][k] : a[0][k], pl);
#pragma unroll
      for (int s = 0; s < RS; ++s) a[s][k] = fma(-mult[s], pr, a[s][k]);
      if (owner_next && k == kn) {
#pragma unroll
        for (int s = 0; s < RS; ++s)
          if (l + 64 * s < n) cn[l + 64 * s] = a[s][k];
      }
    }
  }
  lds_barrier();   // last step's reads of the column copy
  // the right part back to LDS (the left part is dead)
#pragma unroll
  for (int s = 0; s < RS; ++s)
#pragma unroll
    for (int k = 0; k < KC; ++k) {
      const int r = l + 64 * s, c = w + 4 * k;
      if (r < n && c >= n && c < ld) Aug[r * ld + c] = a[s][k];
    }
  __syncthreads();
  return true;
}

// n <= 128 rows, n < ld <= 160 columns.
__device__ inline bool wg_gj_eliminate(int n, int ld, LDS double* Aug, bool pivot, LDS int* perm, LDS int* used,
                                       LDS double* dg) {
  __shared__ int s_piv_[2];
  __shared__ double s_inv_[2];
  LDS int* s_piv = (LDS int*)s_piv_;
  LDS double* s_inv = (LDS double*)s_inv_;
  (void)used;
  n = uniform_int(n); ld = uniform_int(ld); pivot = uniform_int(pivot) != 0;
  Aug = uniform_lds(Aug); perm = uniform_lds(perm); dg = uniform_lds(dg);
  if (n <= 64) {
    if (ld <= 32) return gj_eliminate_regs<1, 8>(n, ld, Aug, pivot, perm, dg, s_piv, s_inv);
    if (ld <= 64) return gj_eliminate_regs<1, 16>(n, ld, Aug, pivot, perm, dg, s_piv, s_inv);
    if (ld <= 96) return gj_eliminate_regs<1, 24>(n, ld, Aug, pivot, perm, dg, s_piv, s_inv);
    if (ld <= 128) return gj_eliminate_regs<1, 32>(n, ld, Aug, pivot, perm, dg, s_piv, s_inv);
    return gj_eliminate_regs<1, 40>(n, ld, Aug, pivot, perm, dg, s_piv, s_inv);
  }
  if (ld <= 128) return gj_eliminate_regs<2, 32>(n, ld, Aug, pivot, perm, dg, s_piv, s_inv);
  return gj_eliminate_regs<2, 40>(n, ld, Aug, pivot, perm, dg, s_piv, s_inv);
}

// Out[j][c] = scale * (M^{-1} R)[j][c0 + c] for c < m, after wg_gj_eliminate,
// converted to TO (any memory, leading dimension ldo).  Ends with a barrier.
template <typename TO>
__device__ inline void wg_gj_extract(int n, int ld, const LDS double* Aug, const LDS int* perm,
                                     const LDS double* dg, int c0, int m, double scale, TO* Out, int ldo) {
  const int lane = tid() & 63, w = tid() >> 6;
  for (int r = w; r < n; r += 4) {
    const LDS double* row = Aug + perm[r] * ld + n + c0;
    const double sc = dg[r] * scale;
    for (int c = lane; c < m; c += 64) Out[(size_t)r * ldo + c] = TO(row[c] * sc);
  }
  __syncthreads();
}

// Inverse of M held in the left half of Aug = [M | I] (n x 2n): Minv (ldm).
template <typename TO>
__device__ inline bool wg_gj_inverse(int n, LDS double* Aug, bool pivot, LDS int* perm, LDS int* used,
                                     LDS double* dg, TO* Minv, int ldm) {
  if (!wg_gj_eliminate(n, 2 * n, Aug, pivot, perm, used, dg)) return false;
  wg_gj_extract<TO>(n, 2 * n, Aug, perm, dg, 0, n, 1.0, Minv, ldm);
  return true;
}

// ------------------------------------------------ batched-load GEMV (WG)
// Reduction dimension up to 4 * KR, output dimension up to 128.  All loads of
// a thread are issued before its first multiply (indices are clamped into
// range and out-of-range terms multiplied by zero), so one memory latency
// covers the whole product and the body has no branch.  PM / PX / PY are
// pointer types (LDS-qualified or global).  part: LDS scratch [4][128].  Both
// end with a barrier.

// y[j] = sum_i M[i*ld + j] x[i]  (M^T x) for M m x n;  y += ... if acc.
template <typename T, int KR, typename PM, typename PX, typename PY>
__device__ __forceinline__ void wg_gemv_t(int m, int n, PM M, int ld, PX x, PY y, LDS T* part, bool acc) {
  const int lane = tid() & 63, w = tid() >> 6;
  T xv[KR];
#pragma unroll
  for (int k = 0; k < KR; ++k) {
    const int i = w + 4 * k;
    const T xi = T(x[min(i, m - 1)]);
    xv[k] = i < m ? xi : T(0);
  }
  for (int jb = 0; jb * 64 < n; ++jb) {
    const int jc = min(jb * 64 + lane, n - 1);
    T v[KR];
#pragma unroll
    for (int k = 0; k < KR; ++k) v[k] = T(M[min(w + 4 * k, m - 1) * ld + jc]);
    T s = T(0);
#pragma unroll
    for (int k = 0; k < KR; ++k) s += v[k] * xv[k];
    part[w * 128 + jb * 64 + lane] = s;
  }
  __syncthreads();
  for (int j = tid(); j < n; j += kWG) {
    T s = part[j] + part[128 + j] + part[256 + j] + part[384 + j];
    y[j] = acc ? T(y[j]) + s : s;
  }
  __syncthreads();
}

// y[i] = sum_j M[i*ld + j] x[j]  (M x) for M m x n (m <= 128, n <= 4 KR).
template <typename T, int KR, typename PM, typename PX, typename PY>
__device__ __forceinline__ void wg_gemv_n(int m, int n, PM M, int ld, PX x, PY y, LDS T* part, bool acc) {
  const int lane = tid() & 63, w = tid() >> 6;
  T xv[KR];
#pragma unroll
  for (int k = 0; k < KR; ++k) {
    const int j = w + 4 * k;
    const T xj = T(x[min(j, n - 1)]);
    xv[k] = j < n ? xj : T(0);
  }
  for (int ib = 0; ib * 64 < m; ++ib) {
    const int ic = min(ib * 64 + lane, m - 1);
    T v[KR];
#pragma unroll
    for (int k = 0; k < KR; ++k) v[k] = T(M[ic * ld + min(w + 4 * k, n - 1)]);
    T s = T(0);
#pragma unroll
    for (int k = 0; k < KR; ++k) s += v[k] * xv[k];
    part[w * 128 + ib * 64 + lane] = s;
  }
  __syncthreads();
  for (int i = tid(); i < m; i += kWG) {
    T s = part[i] + part[128 + i] + part[256 + i] + part[384 + i];
    y[i] = acc ? T(y[i]) + s : s;
  }
  __syncthreads();
}

// Square n x n products (n <= 64) split in two so the matrix loads can be
// issued before a wait for x: _pre loads this thread's entries of M into v,
// _fin multiplies them with x (TR: M^T x, else M x).
template <typename T, int KR, bool TR, typename PM>
__device__ __forceinline__ void wg_gemv_sq_pre(int n, PM M, int ld, T v[KR]) {
  const int lane = tid() & 63, w = tid() >> 6;
  const int jc = min(lane, n - 1);
#pragma unroll
  for (int k = 0; k < KR; ++k) {
    const int r = min(w + 4 * k, n - 1);
    v[k] = TR ? T(M[r * ld + jc]) : T(M[jc * ld + r]);
  }
}
template <typename T, int KR, typename PX, typename PY>
__device__ __forceinline__ void wg_gemv_sq_fin(int n, const T v[KR], PX x, PY y, LDS T* part, bool acc) {
  const int lane = tid() & 63, w = tid() >> 6;
  T s = T(0);
#pragma unroll
  for (int k = 0; k < KR; ++k) {
    const int i = w + 4 * k;
    const T xi = T(x[min(i, n - 1)]);
    s += v[k] * (i < n ? xi : T(0));
  }
  part[w * 128 + lane] = s;
  __syncthreads();
  for (int j = tid(); j < n; j += kWG) {
    T t = part[j] + part[128 + j] + part[256 + j] + part[384 + j];
    y[j] = acc ? T(y[j]) + t : t;
  }
  __syncthreads();
}

// ------------------------------------------- inter-workgroup packed words
// A 64-bit word carries 32 payload bits (low) and a 32-bit stamp (high).  Words
// are written and polled with relaxed device-scope atomics, which the gfx950
// backend emits as cache-coherent (sc1) stores and loads with no cache
// write-back or invalidate; the payload and its stamp arrive together because
// an aligned 64-bit access is single-copy atomic.  A reader waits until the
// stamp equals the one it expects.  Waits are bounded by kSpinLimit polls.
__device__ __forceinline__ void ll_put(unsigned long long* p, uint32_t stamp, uint32_t bits) {
  __hip_atomic_store(p, ((unsigned long long)stamp << 32) | bits, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
// Returns false if the wait gave up (poll limit, or another workgroup raised
// the abort flag, which is checked every 256 polls).
__device__ __forceinline__ bool ll_get(const unsigned long long* p, uint32_t stamp, uint32_t* bits,
                                       const int* abort) {
  unsigned n = 0;
  while (true) {
    unsigned long long w = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if ((uint32_t)(w >> 32) == stamp) { *bits = (uint32_t)w; return true; }
    if (++n > kSpinLimit) return false;
    if ((n & 255) == 0 && __hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
    __builtin_amdgcn_s_sleep(1);
  }
}

// Words per value of type T.
template <typename T> struct LLWords;
template <> struct LLWords<float> { static constexpr int n = 1; };
template <> struct LLWords<double> { static constexpr int n = 2; };

template <typename T>
__device__ __forceinline__ void ll_put_val(unsigned long long* p, uint32_t stamp, T v);
template <>
__device__ __forceinline__ void ll_put_val<float>(unsigned long long* p, uint32_t stamp, float v) {
  ll_put(p, stamp, __float_as_uint(v));
}
template <>
__device__ __forceinline__ void ll_put_val<double>(unsigned long long* p, uint32_t stamp, double v) {
  unsigned long long b = (unsigned long long)__double_as_longlong(v);
  ll_put(p, stamp, (uint32_t)b);
  ll_put(p + 1, stamp, (uint32_t)(b >> 32));
}
template <typename T>
__device__ __forceinline__ bool ll_get_val(const unsigned long long* p, uint32_t stamp, T* v,
                                           const int* abort);
template <>
__device__ __forceinline__ bool ll_get_val<float>(const unsigned long long* p, uint32_t stamp, float* v,
                                                  const int* abort) {
  uint32_t b = 0;
  bool ok = ll_get(p, stamp, &b, abort);
  *v = __uint_as_float(b);
  return ok;
}
// Poll cnt <= K words addr(0..cnt) in one round trip per round: every load of a
// round is issued before any stamp is checked.  Same bounds as ll_get.
template <int K, typename F>
__device__ __forceinline__ bool ll_get_batch(F addr, int cnt, uint32_t stamp, uint32_t bits[K], const int* abort) {
  unsigned n = 0;
  while (true) {
    unsigned long long w[K];
#pragma unroll
    for (int k = 0; k < K; ++k)
      w[k] = k < cnt ? __hip_atomic_load(addr(k), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                     : (unsigned long long)stamp << 32;
    bool all = true;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      all = all && (uint32_t)(w[k] >> 32) == stamp;
      bits[k] = (uint32_t)w[k];
    }
    if (all) return true;
    if (++n > kSpinLimit) return false;
    if ((n & 255) == 0 && __hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
    __builtin_amdgcn_s_sleep(1);
  }
}

template <>
__device__ __forceinline__ bool ll_get_val<double>(const unsigned long long* p, uint32_t stamp, double* v,
                                                   const int* abort) {
  uint32_t b[2] = {0, 0};
  bool ok = ll_get_batch<2>([&](int k) { return p + k; }, 2, stamp, b, abort);
  *v = __longlong_as_double((long long)(((unsigned long long)b[1] << 32) | b[0]));
  return ok;
}

}  // namespace gsls
