// Persistent ADMM iteration kernel (Sec. III-C / IV-A of the paper).
//
// With rho fixed the factors of the LQR subproblem eq. (primal_update) are
// cached (eq. (gains_cache)), so each ADMM x-update is an affine function of
// w = y - z (scaled dual minus split variable):
//   backward   p_k = Abar_k^T p_{k+1} + c_k,
//              c_k = q_hat_k + K_k^T r_hat_k + Abar_k^T P_{k+1} b_k,   p_N = q_hat_N
//              k_k = -Gamma_k (B_k^T p_{k+1} + B_k^T P_{k+1} b_k + r_hat_k)
//   forward    x_{k+1} = Abar_k x_k + B_k k_k + b_k,  u_k = K_k x_k + k_k
// with q_hat, r_hat the linear terms of eq. (augmented_linear).  Both
// recurrences are affine maps composed by associative scans over the horizon:
// the horizon is cut into P chunks, one workgroup each; a workgroup folds its
// chunk, the chunk results are combined across workgroups by recursive
// doubling with the cached transfer maps Phi[d][c] (the product of Abar over
// 2^d consecutive chunks), and each workgroup finishes its own stages.  Then
// the z-projection and scaled dual update and the residuals
// r_p = |G xi - z+|_inf, r_d = rho |G^T (z+ - z)|_inf, reduced over all
// workgroups.
//
// Precision.  Operators and scans run in T.  The ADMM state (z, y), the
// constraint values v = G xi, the projection, the dual update and the
// residuals are FP64.  In mixed mode (T = float) the first iteration after a
// factor epoch evaluates the affine map in full; every later iteration
// evaluates only its linear part on the increment dw = w_t - w_{t-1} and adds
// the result to FP64 accumulators of x, u and v.  FP32 rounding then scales
// with the step rather than with the iterate, so the residuals are not held
// at FP32 resolution.  In FP64 mode every iteration is a full evaluation.
//
// Operators.  Per stage F = [[Abar, B], [K, I]] and G = [C | D] (plus
// Gamma), so that one product gives [Abar^T p; B^T p], [Abar x + B k; K x + k],
// [C^T w; D^T w] or C x + D u.
//
// Residency.  A workgroup keeps its chunk's vectors, bounds, state and
// accumulators in LDS for the whole launch, and its operators (with odd
// leading dimensions so that both M x and M^T x read LDS without bank
// conflicts) when they fit; otherwise the operators are read from global
// memory (L2 / Infinity Cache) with batched loads.  Global memory is written
// only at exit.
//
// Workgroups exchange vectors through packed (payload, stamp) words (see
// dev_common.hpp); every wait is bounded and an abort flag ends all waits.
// The kernel runs until convergence, the iteration limit, or a rho change
// (OSQP rule, every sigma iterations), which needs a new factor epoch.
#include <algorithm>

#include "dev_common.hpp"
#include "solver.hpp"

namespace gsls {

__device__ __forceinline__ int cbeg(int c, int N, int P) { return (int)(((long long)c * N) / P); }

// WG-wide max (NaN propagates) of the first nq of kRed per-thread values: a
// butterfly inside each wave, then one combine of the four wave results.
// s: LDS [4][kRed]; out[0..nq) is valid after the call.
__device__ __forceinline__ double nanmax(double a, double b) { return (b > a || b != b) ? b : a; }
__device__ inline void wg_max_red(const double v[kRed], int nq, LDS double* s, LDS double* out) {
#pragma unroll
  for (int q = 0; q < kRed; ++q) {
    if (q < nq) {
      double m = v[q];
      for (int off = 32; off > 0; off >>= 1) m = nanmax(m, __shfl_xor(m, off));
      if (lane() == 0) s[wave() * kRed + q] = m;
    }
  }
  __syncthreads();
  if (tid() < nq) {
    double m = s[tid()];
    for (int w = 1; w < 4; ++w) m = nanmax(m, s[w * kRed + tid()]);
    out[tid()] = m;
  }
  __syncthreads();
}

template <typename T>
__device__ inline void publish_vec(unsigned long long* w, uint32_t stamp, const LDS T* v, int n) {
  constexpr int W = LLWords<T>::n;
  for (int j = tid(); j < n; j += kWG) ll_put_val<T>(w + (size_t)j * W, stamp, v[j]);
}

// Read n values (all threads call; returns false uniformly if a wait failed).
template <typename T>
__device__ inline bool fetch_vec(const unsigned long long* w, uint32_t stamp, LDS T* v, int n, int* abort,
                                 int* s_flag) {
  constexpr int W = LLWords<T>::n;
  bool ok = true;
  for (int j = tid(); j < n; j += kWG) {
    T val;
    bool g = ll_get_val<T>(w + (size_t)j * W, stamp, &val, abort);
    if (!g) ok = false;
    v[j] = val;
  }
  if (!ok) {
    atomicExch(s_flag, 1);
    __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  bool res = (*s_flag == 0);
  __syncthreads();
  return res;
}

__host__ __device__ inline int odd(int x) { return x | 1; }

// Elements of one LDS-resident stage block: F = [[Abar, B], [K, I]]
// ((nx+nu) x (nx+nu)), G = [C | D] (nc x (nx+nu)) and Gamma (nu x nu), each
// with an odd leading dimension.
__host__ __device__ inline int stage_block_elems(int nx, int nu, int nc) {
  const int nxu = nx + nu;
  int e = nxu * odd(nxu) + nc * odd(nxu) + nu * odd(nu);
  return (e + 3) & ~3;
}

// LDS layout of one workgroup (element counts), shared by host sizing and
// the kernel carve.
constexpr int kVec = 112;   // work-vector length (>= nx + nu)
struct AdmmLayout {
  size_t ops;       // T    [Lmax][sbe]  (0 if not resident)
  size_t tvec;      // T    per-chunk vectors
  size_t work;      // T    work vectors
  size_t dvec;      // double per-chunk state
  size_t dwork;     // double reductions
  size_t bytes;
};

template <typename T>
__host__ __device__ inline AdmmLayout admm_layout(int nx, int nu, int nc, int nf, int Lmax, int P, bool resident) {
  AdmmLayout L;
  const size_t rows = (size_t)Lmax * nc + nf;  // rows of the chunk (terminal rows for the last one)
  L.ops = resident ? (size_t)Lmax * stage_block_elems(nx, nu, nc) : 0;
  // cvec, qv, bv, evv: [Lmax][nx]; hh, kff, rv, fvv: [Lmax][nu]; qN: [nx]
  L.tvec = (size_t)Lmax * (4 * nx + 4 * nu) + nx;
  L.work = 6 * kVec + 2 * kMaxNc + 512;
  // ys, zs, ls, us, vacc, wprev: [rows]; x accumulator [Lmax+1][nx]; u accumulator [Lmax][nu]
  L.dvec = 6 * rows + (size_t)(Lmax + 1) * nx + (size_t)Lmax * nu;
  L.dwork = 4 * kRed + 2 * kRed;
  size_t tbytes = sizeof(T) * (L.ops + L.tvec + L.work);
  tbytes = (tbytes + 15) & ~(size_t)15;
  L.bytes = tbytes + sizeof(double) * (L.dvec + L.dwork);
  return L;
}

// Operator access of one stage: LDS-resident copies or global memory.
template <typename T, bool RES>
struct OpPtr;
template <typename T>
struct OpPtr<T, true> { typedef const LDS T* type; };
template <typename T>
struct OpPtr<T, false> { typedef const T* type; };

template <typename T, bool RES, int KR>
__global__ void __launch_bounds__(kWG) k_admm(IterArgs<T> a) {
  extern __shared__ __align__(16) char lds_generic[];
  LDS char* lds_raw = (LDS char*)lds_generic;
  typedef typename OpPtr<T, RES>::type OP;
  const DevProblem<T>& pb = a.pb;
  const DevFactor<T>& fc = a.fc;
  const int N = pb.N, nx = pb.nx, nu = pb.nu, nc = pb.nc, nf = pb.nf, nxu = nx + nu;
  const int P = a.ip.P, nlev = a.ip.nlev, c = blockIdx.x;
  const int s = cbeg(c, N, P), e = cbeg(c + 1, N, P), L = e - s;
  const bool last = (c == P - 1);
  const int rows = L * nc + (last ? nf : 0);       // constraint rows owned by this chunk
  const size_t row0 = (size_t)s * nc;              // first global row
  const size_t xx = (size_t)nx * nx, ff = (size_t)nxu * nxu;
  constexpr int W = LLWords<T>::n;
  const size_t vstride = (size_t)nx * W;
  const T rho = T(a.ip.rho);
  const double rhod = a.ip.rho;
  const int sbe = stage_block_elems(nx, nu, nc);
  constexpr bool kIncremental = sizeof(T) < sizeof(double);
  // transfer-map loads issued before the partner wait: KR registers per thread,
  // kept to the narrower variants (the wider ones spill less without them)
  constexpr bool kPrefetchMaps = KR <= 20;
  unsigned long long* prof = (a.prof && c == 0) ? a.prof : nullptr;
  unsigned long long t_last = 0;
  auto mark = [&](int ph) {
    if (prof) {
      __syncthreads();
      unsigned long long t = __builtin_amdgcn_s_memtime();
      if (tid() == 0 && t_last) prof[ph] += t - t_last;
      t_last = t;
    }
  };

  // ------------------------------------------------------------ LDS carve
  const AdmmLayout lay = admm_layout<T>(nx, nu, nc, nf, a.Lmax, P, RES);
  const int Lm = a.Lmax;
  LDS T* ops = (LDS T*)lds_raw;
  LDS T* cvec = ops + lay.ops;                      // [Lmax][nx]
  LDS T* qv = cvec + Lm * nx;                       // [Lmax][nx]
  LDS T* bv = qv + Lm * nx;                         // [Lmax][nx]
  LDS T* evv = bv + Lm * nx;                        // [Lmax][nx]
  LDS T* hh = evv + Lm * nx;                        // [Lmax][nu]
  LDS T* kff = hh + Lm * nu;                        // [Lmax][nu]
  LDS T* rv = kff + Lm * nu;                        // [Lmax][nu]
  LDS T* fvv = rv + Lm * nu;                        // [Lmax][nu]
  LDS T* qN = fvv + Lm * nu;                        // [nx]
  LDS T* g = ops + lay.ops + lay.tvec;              // [kVec] running vector
  LDS T* g2 = g + kVec;                             // [kVec]
  LDS T* xz = g2 + kVec;                            // [kVec] stacked [x; k] / [x; u]
  LDS T* tvu = xz + kVec;                           // [kVec]
  LDS T* tu = tvu + kVec;                           // [kVec]
  LDS T* tu2 = tu + kVec;                           // [kVec]
  LDS T* wv = tu2 + kVec;                           // [kMaxNc]
  LDS T* wv2 = wv + kMaxNc;                         // [kMaxNc]
  LDS T* part = wv2 + kMaxNc;                       // [4][128]
  size_t tb = sizeof(T) * (lay.ops + lay.tvec + lay.work);
  tb = (tb + 15) & ~(size_t)15;
  LDS double* dv = (LDS double*)(lds_raw + tb);
  const int rmax = Lm * nc + nf;
  LDS double* ys = dv;                              // [rows]
  LDS double* zs = ys + rmax;
  LDS double* ls = zs + rmax;
  LDS double* us = ls + rmax;
  LDS double* vacc = us + rmax;
  LDS double* wprev = vacc + rmax;
  LDS double* xacc = wprev + rmax;                  // [Lmax+1][nx]  x of the chunk's stages (+ x_N)
  LDS double* uacc = xacc + (size_t)(Lm + 1) * nx;  // [Lmax][nu]
  LDS double* redv = uacc + (size_t)Lm * nu;        // [4][kRed]
  LDS double* res = redv + 4 * kRed;                // [2*kRed]
  __shared__ int s_flag;
  if (tid() == 0) s_flag = 0;

  const int ldF = RES ? odd(nxu) : nxu, ldG = RES ? odd(nxu) : nxu, ldGm = RES ? odd(nu) : nu;
  auto opF = [&](int i) -> OP {
    if constexpr (RES) return (OP)(ops + (size_t)(i - s) * sbe);
    else return fc.F + (size_t)i * ff;
  };
  auto opG = [&](int i) -> OP {
    if constexpr (RES) return (OP)(ops + (size_t)(i - s) * sbe + nxu * odd(nxu));
    else return pb.G + (size_t)i * nc * nxu;
  };
  auto opGm = [&](int i) -> OP {
    if constexpr (RES) return (OP)(ops + (size_t)(i - s) * sbe + nxu * odd(nxu) + nc * odd(nxu));
    else return fc.Gam + (size_t)i * nu * nu;
  };
  // ------------------------------------------------------- load residents
  if constexpr (RES) {
    for (int i = s; i < e; ++i) {
      LDS T* F = (LDS T*)opF(i);
      LDS T* Gc = (LDS T*)opG(i);
      LDS T* Gm = (LDS T*)opGm(i);
      const T* Fg = fc.F + (size_t)i * ff;
      const T* Gg = pb.G + (size_t)i * nc * nxu;
      const T* Gmg = fc.Gam + (size_t)i * nu * nu;
      for (int r = wave(); r < nxu; r += 4)
        for (int cc = lane(); cc < nxu; cc += 64) F[r * ldF + cc] = Fg[(size_t)r * nxu + cc];
      for (int r = wave(); r < nc; r += 4)
        for (int cc = lane(); cc < nxu; cc += 64) Gc[r * ldG + cc] = Gg[(size_t)r * nxu + cc];
      for (int r = wave(); r < nu; r += 4)
        for (int cc = lane(); cc < nu; cc += 64) Gm[r * ldGm + cc] = Gmg[(size_t)r * nu + cc];
    }
  }
  for (int t = tid(); t < L * nx; t += kWG) {
    const size_t gi = (size_t)s * nx + t;
    qv[t] = pb.q[gi]; bv[t] = pb.b[gi]; evv[t] = fc.ev[gi];
  }
  for (int t = tid(); t < L * nu; t += kWG) {
    const size_t gi = (size_t)s * nu + t;
    rv[t] = pb.r[gi]; fvv[t] = fc.fv[gi];
  }
  for (int t = tid(); t < nx; t += kWG) qN[t] = pb.q[(size_t)N * nx + t];
  for (int t = tid(); t < rows; t += kWG) {
    ys[t] = a.y[row0 + t]; zs[t] = a.z[row0 + t];
    ls[t] = a.l[row0 + t]; us[t] = a.u[row0 + t];
    vacc[t] = 0.0; wprev[t] = 0.0;
  }
  const int nxs = (L + (last ? 1 : 0)) * nx;       // states owned by this chunk
  for (int t = tid(); t < nxs; t += kWG) xacc[t] = a.X[(size_t)s * nx + t];
  for (int t = tid(); t < L * nu; t += kWG) uacc[t] = a.U[(size_t)s * nu + t];
  __syncthreads();

  int it = a.ip.it0;
  uint32_t stamp = a.ip.stamp0;
  int status = 0;
  double rho_new = a.ip.rho;
  double fin_rp = 0.0, fin_rd = 0.0;
  bool first = true;
  mark(0);

  while (true) {
    ++it;
    ++stamp;
    const bool sigma_it = a.ip.adaptive && a.ip.sigma > 0 && (it % a.ip.sigma == 0) && it < a.ip.max_iter;
    // evaluate the affine map in full (FP64; mixed after an epoch and at refresh points)
    const bool full = first || !kIncremental || (a.ip.refresh > 0 && it % a.ip.refresh == 0);
    const T cst = full ? T(1) : T(0);           // weight of the w-independent terms
    // ---------------------------------------------------- 1. linear terms
    for (int i = s; i < e; ++i) {
      const int li = i - s;
      for (int r = tid(); r < nc; r += kWG) {
        const double w = ys[li * nc + r] - zs[li * nc + r];
        wv[r] = T(full ? w : w - wprev[li * nc + r]);
        wprev[li * nc + r] = w;
      }
      __syncthreads();
      wg_gemv_t<T, KR>(nc, nxu, opG(i), ldG, wv, tvu, part, false);       // [C^T w; D^T w]
      for (int j = tid(); j < nu; j += kWG) {
        T rh = cst * rv[li * nu + j] + rho * tvu[nx + j];
        tu[j] = rh;
        hh[li * nu + j] = cst * fvv[li * nu + j] + rh;
      }
      for (int j = tid(); j < nx; j += kWG)
        cvec[li * nx + j] = cst * (qv[li * nx + j] + evv[li * nx + j]) + rho * tvu[j];
      __syncthreads();
      wg_gemv_t<T, KR>(nu, nx, opF(i) + nx * ldF, ldF, tu, cvec + li * nx, part, true);  // + K^T r_hat
    }
    // rho C_N^T w_N  (last chunk; kept in tvu for the terminal value)
    if (last) {
      for (int r = tid(); r < nf; r += kWG) {
        const int lr = L * nc + r;
        const double w = ys[lr] - zs[lr];
        wv[r] = T(full ? w : w - wprev[lr]);
        wprev[lr] = w;
      }
      __syncthreads();
      if (nf > 0) wg_gemv_t<T, KR>(nf, nx, (const T*)pb.CN, nx, wv, tvu, part, false);
    }
    auto terminal_p = [&](LDS T* dst) {
      for (int j = tid(); j < nx; j += kWG) dst[j] = cst * qN[j] + (nf > 0 ? rho * tvu[j] : T(0));
      __syncthreads();
    };
    mark(1);
    // ----------------------------------------------- 2. backward local fold
    if (last) {
      terminal_p(g);
    } else {
      for (int j = tid(); j < nx; j += kWG) g[j] = T(0);
      __syncthreads();
    }
    for (int i = e - 1; i >= s; --i) {
      wg_gemv_t<T, KR>(nx, nx, opF(i), ldF, g, g2, part, false);           // Abar^T g
      for (int j = tid(); j < nx; j += kWG) g[j] = g2[j] + cvec[(i - s) * nx + j];
      __syncthreads();
    }
    mark(2);
    // --------------------------------------- 3. backward doubling across chunks
    publish_vec<T>(a.ll.bwd + (size_t)c * vstride, stamp, g, nx);
    for (int d = 0; d < nlev; ++d) {
      const int pc = c + (1 << d);
      if (pc < P) {
        const T* Phi = fc.Phi + ((size_t)d * P + c) * xx;
        if (kPrefetchMaps && nx <= 64) {
          // issue the transfer-map loads, then wait for the partner's vector
          T pv[KR];
          wg_gemv_sq_pre<T, KR, true>(nx, Phi, nx, pv);
          if (!fetch_vec<T>(a.ll.bwd + ((size_t)d * P + pc) * vstride, stamp, g2, nx, a.ll.abort, &s_flag)) {
            status = 5; break;
          }
          wg_gemv_sq_fin<T, KR>(nx, pv, g2, g, part, true);
        } else {
          if (!fetch_vec<T>(a.ll.bwd + ((size_t)d * P + pc) * vstride, stamp, g2, nx, a.ll.abort, &s_flag)) {
            status = 5; break;
          }
          wg_gemv_t<T, KR>(nx, nx, Phi, nx, g2, g, part, true);
        }
      }
      publish_vec<T>(a.ll.bwd + ((size_t)(d + 1) * P + c) * vstride, stamp, g, nx);
    }
    if (status) break;
    // p at the chunk's right end (tvu still holds C_N^T w_N for the last chunk)
    if (!last) {
      if (!fetch_vec<T>(a.ll.bwd + ((size_t)nlev * P + c + 1) * vstride, stamp, g, nx, a.ll.abort, &s_flag)) {
        status = 5; break;
      }
    } else {
      terminal_p(g);
    }
    mark(3);
    // ------------------------------------------------ 4. backward fix-up
    for (int i = e - 1; i >= s; --i) {
      const int li = i - s;
      wg_gemv_t<T, KR>(nx, nxu, opF(i), ldF, g, g2, part, false);          // [Abar^T p; B^T p]
      for (int j = tid(); j < nu; j += kWG) tu[j] = g2[nx + j] + hh[li * nu + j];
      if (i > s)
        for (int j = tid(); j < nx; j += kWG) g[j] = g2[j] + cvec[li * nx + j];
      __syncthreads();
      wg_gemv_t<T, KR>(nu, nu, opGm(i), ldGm, tu, tu2, part, false);      // Gamma (...)
      for (int j = tid(); j < nu; j += kWG) kff[li * nu + j] = -tu2[j];
      __syncthreads();
    }
    mark(4);
    // ------------------------------------------------ 5. forward local fold
    for (int j = tid(); j < nx; j += kWG) xz[j] = (c == 0) ? cst * a.x0[j] : T(0);
    for (int i = s; i < e; ++i) {
      const int li = i - s;
      for (int j = tid(); j < nu; j += kWG) xz[nx + j] = kff[li * nu + j];
      __syncthreads();
      wg_gemv_n<T, KR>(nx, nxu, opF(i), ldF, xz, g2, part, false);         // Abar x + B k
      for (int j = tid(); j < nx; j += kWG) xz[j] = g2[j] + cst * bv[li * nx + j];
    }
    for (int j = tid(); j < nx; j += kWG) g[j] = xz[j];
    __syncthreads();
    mark(5);
    // -------------------------------------- 6. forward doubling across chunks
    publish_vec<T>(a.ll.fwd + (size_t)c * vstride, stamp, g, nx);
    for (int d = 0; d < nlev; ++d) {
      const int pc = c - (1 << d);
      if (pc >= 0) {
        // g += Phi[d][c - 2^d + 1] g2; the map's loads are issued before the wait
        const T* Phi = fc.Phi + ((size_t)d * P + (c - (1 << d) + 1)) * xx;
        if (kPrefetchMaps && nx <= 64) {
          T pv[KR];
          wg_gemv_sq_pre<T, KR, false>(nx, Phi, nx, pv);
          if (!fetch_vec<T>(a.ll.fwd + ((size_t)d * P + pc) * vstride, stamp, g2, nx, a.ll.abort, &s_flag)) {
            status = 5; break;
          }
          wg_gemv_sq_fin<T, KR>(nx, pv, g2, g, part, true);
        } else {
          if (!fetch_vec<T>(a.ll.fwd + ((size_t)d * P + pc) * vstride, stamp, g2, nx, a.ll.abort, &s_flag)) {
            status = 5; break;
          }
          wg_gemv_n<T, KR>(nx, nx, Phi, nx, g2, g, part, true);
        }
      }
      publish_vec<T>(a.ll.fwd + ((size_t)(d + 1) * P + c) * vstride, stamp, g, nx);
    }
    if (status) break;
    if (c > 0) {
      if (!fetch_vec<T>(a.ll.fwd + ((size_t)nlev * P + c - 1) * vstride, stamp, g, nx, a.ll.abort, &s_flag)) {
        status = 5; break;
      }
    } else {
      for (int j = tid(); j < nx; j += kWG) g[j] = cst * a.x0[j];
      __syncthreads();
    }
    mark(6);
    // ------------------- 7. forward fix-up, constraint map, projection, duals
    double loc[kRed];
    for (int q = 0; q < kRed; ++q) loc[q] = 0.0;
    for (int j = tid(); j < nx; j += kWG) xz[j] = g[j];
    for (int i = s; i <= e; ++i) {
      if (i == e && !(last && i == N)) break;
      const bool term = (i == N);
      const int li = i - s;
      const int nr = term ? nf : nc;
      const int lr0 = li * nc;                     // local row offset (terminal rows follow)
      // xacc (and uacc) hold the last iterate: full value or increment added
      for (int j = tid(); j < nx; j += kWG) {
        LDS double* xa = xacc + li * nx + j;
        *xa = full ? (double)xz[j] : *xa + (double)xz[j];
      }
      if (!term) {
        for (int j = tid(); j < nu; j += kWG) xz[nx + j] = kff[li * nu + j];
        __syncthreads();
        wg_gemv_n<T, KR>(nxu, nxu, opF(i), ldF, xz, g2, part, false);      // [Abar x + B k; K x + k]
        for (int j = tid(); j < nu; j += kWG) {
          const T uu = g2[nx + j];
          xz[nx + j] = uu;                                              // xz = [x; u]
          LDS double* ua = uacc + li * nu + j;
          *ua = full ? (double)uu : *ua + (double)uu;
        }
        __syncthreads();
        wg_gemv_n<T, KR>(nc, nxu, opG(i), ldG, xz, wv, part, false);       // v = C x + D u
      } else {
        __syncthreads();
        if (nr > 0) wg_gemv_n<T, KR>(nf, nx, (const T*)pb.CN, nx, xz, wv, part, false);
      }
      // projection and dual update in FP64; wv <- dz, wv2 <- y+
      for (int r = tid(); r < nr; r += kWG) {
        const int lr = lr0 + r;
        const double v = full ? (double)wv[r] : vacc[lr] + (double)wv[r];
        vacc[lr] = v;
        const double yo = ys[lr], zo = zs[lr];
        const double t = v + yo;
        const double lo = ls[lr], hi = us[lr];
        const double zn = t < lo ? lo : (t > hi ? hi : t);
        const double yn = yo + v - zn;
        zs[lr] = zn;
        ys[lr] = yn;
        const double rp = fabs(v - zn);
        loc[0] = (rp > loc[0] || rp != rp) ? rp : loc[0];
        loc[2] = fmax(loc[2], fabs(v));
        loc[3] = fmax(loc[3], fabs(zn));
        wv[r] = T(zn - zo);
        wv2[r] = T(yn);
      }
      __syncthreads();
      // r_d contribution: rho |[C D]^T dz|
      const int ncol = term ? nx : nxu;
      if (nr > 0) {
        if (term) wg_gemv_t<T, KR>(nr, nx, (const T*)pb.CN, nx, wv, tvu, part, false);
        else wg_gemv_t<T, KR>(nr, nxu, opG(i), ldG, wv, tvu, part, false);
        for (int j = tid(); j < ncol; j += kWG) loc[1] = nanmax(loc[1], rhod * fabs((double)tvu[j]));
        if (!sigma_it && !term) {
          // next state (g2 still holds Abar x + B k); one barrier covers both
          for (int j = tid(); j < nx; j += kWG) xz[j] = g2[j] + cst * bv[li * nx + j];
          __syncthreads();
          continue;
        }
        __syncthreads();
      }
      if (sigma_it) {
        // |G^T lambda| with lambda = rho y+
        if (nr > 0) {
          if (term) wg_gemv_t<T, KR>(nr, nx, (const T*)pb.CN, nx, wv2, tvu, part, false);
          else wg_gemv_t<T, KR>(nr, nxu, opG(i), ldG, wv2, tvu, part, false);
          for (int j = tid(); j < ncol; j += kWG) loc[5] = fmax(loc[5], rhod * fabs((double)tvu[j]));
          __syncthreads();
        }
        // |H xi|: Q x + S^T u and S x + R u (only Q_N x_N at the terminal stage),
        // on the accumulated iterate
        for (int j = tid(); j < nx; j += kWG) tu2[j] = T(xacc[li * nx + j]);
        if (!term)
          for (int j = tid(); j < nu; j += kWG) tu[j] = T(uacc[li * nu + j]);
        __syncthreads();
        wg_gemv_n<T, KR>(nx, nx, (const T*)(pb.Q + i * xx), nx, tu2, tvu, part, false);
        if (!term) {
          wg_gemv_t<T, KR>(nu, nx, (const T*)(pb.S + (size_t)i * nu * nx), nx, tu, tvu, part, true);   // + S^T u
          wg_gemv_n<T, KR>(nu, nu, (const T*)(pb.R + (size_t)i * nu * nu), nu, tu, wv2, part, false); // R u
          wg_gemv_n<T, KR>(nu, nx, (const T*)(pb.S + (size_t)i * nu * nx), nx, tu2, wv2, part, true); // + S x
          for (int j = tid(); j < nu; j += kWG) loc[4] = fmax(loc[4], fabs((double)wv2[j]));
        }
        for (int j = tid(); j < nx; j += kWG) loc[4] = fmax(loc[4], fabs((double)tvu[j]));
        __syncthreads();
      }
      if (term) break;
      // next state: x_{i+1} = Abar x + B k + b
      for (int j = tid(); j < nx; j += kWG) xz[j] = g2[j] + cst * bv[li * nx + j];
      __syncthreads();
    }
    mark(7);
    // ---------------------------------------------- 8. global reductions
    const int nq = sigma_it ? kRed : 2;            // the scale terms only feed the rho rule
    wg_max_red(loc, nq, redv, res);
    for (int q = tid(); q < nq; q += kWG)
      ll_put_val<double>(a.ll.red + ((size_t)c * kRed + q) * 2, stamp, res[q]);
    {
      // thread -> (q, workgroups pp = tid / nqp + (kWG / nqp) k); each thread
      // folds its values, then lanes of equal q combine (q = lane mod nqp)
      const int nqp = nq == 2 ? 2 : 8, q = tid() % nqp, pstep = kWG / nqp;
      double m = 0.0;
      bool ok = true;
      if (q < nq) {
        for (int p0 = tid() / nqp; p0 < P; p0 += 2 * pstep) {
          const int cnt = p0 + pstep < P ? 4 : 2;      // words: one or two values
          uint32_t b[4];
          ok = ok && ll_get_batch<4>(
                         [&](int k) { return a.ll.red + ((size_t)(p0 + (k >> 1) * pstep) * kRed + q) * 2 + (k & 1); },
                         cnt, stamp, b, a.ll.abort);
          m = nanmax(m, __longlong_as_double((long long)(((unsigned long long)b[1] << 32) | b[0])));
          if (cnt == 4) m = nanmax(m, __longlong_as_double((long long)(((unsigned long long)b[3] << 32) | b[2])));
        }
      }
      for (int off = 32; off >= nqp; off >>= 1) m = nanmax(m, __shfl_xor(m, off));
      if (lane() < nq) redv[wave() * kRed + lane()] = m;
      if (!ok) {
        atomicExch(&s_flag, 1);
        __hip_atomic_store(a.ll.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      __syncthreads();
      if (s_flag) { status = 5; break; }
    }
    if (tid() < nq) {
      double m = redv[tid()];
      for (int w = 1; w < 4; ++w) m = nanmax(m, redv[w * kRed + tid()]);
      res[kRed + tid()] = m;
    }
    __syncthreads();
    mark(8);
    first = false;
    const double rp = res[kRed + 0], rd = res[kRed + 1];
    fin_rp = rp; fin_rd = rd;
    // ---------------------------------------------- 9. decisions (uniform)
    if (rp != rp || rd != rd || isinf(rp) || isinf(rd)) { status = 3; break; }
    if (rp <= a.ip.tol && rd <= a.ip.tol) { status = 1; break; }
    if (it >= a.ip.max_iter) { status = 2; break; }
    if (sigma_it) {
      const double ps = fmax(res[kRed + 2], res[kRed + 3]);
      const double ds = fmax(fmax(res[kRed + 4], res[kRed + 5]), a.ip.hnorm);
      const double eps = 1e-10;
      const double ratio = (rp / (ps + eps)) / (rd / (ds + eps) + eps);
      double rn = a.ip.rho * sqrt(ratio);
      rn = fmin(fmax(rn, a.ip.rho_min), a.ip.rho_max);
      if (rn > a.ip.rho * a.ip.rho_tol || rn < a.ip.rho / a.ip.rho_tol) {
        // rescale the scaled dual so lambda is unchanged
        const double f = a.ip.rho / rn;
        for (int r = tid(); r < rows; r += kWG) ys[r] *= f;
        __syncthreads();
        rho_new = rn;
        status = 4;
        break;
      }
    }
  }
  // ----------------------------------------------------- write state back
  __syncthreads();
  for (int t = tid(); t < rows; t += kWG) {
    a.y[row0 + t] = ys[t];
    a.z[row0 + t] = zs[t];
  }
  for (int t = tid(); t < nxs; t += kWG) a.X[(size_t)s * nx + t] = xacc[t];
  for (int t = tid(); t < L * nu; t += kWG) a.U[(size_t)s * nu + t] = uacc[t];
  // status is merged with atomicMax by every writer (the host zeroes it before
  // the launch): a timeout (5) seen by any workgroup outranks the uniform
  // decision (1-4) that workgroup 0 reports, whatever the order of the writes
  if (c == 0 && tid() == 0) {
    a.ctl->it = it;
    a.ctl->r_p = fin_rp;
    a.ctl->r_d = fin_rd;
    a.ctl->rho_new = rho_new;
    atomicMax(&a.ctl->status, status);
  }
  if (c != 0 && status == 5 && tid() == 0) atomicMax(&a.ctl->status, 5);
}

template <typename T>
size_t admm_lds_bytes(int nx, int nu, int nc, int nf, int Lmax, int P, bool resident) {
  return admm_layout<T>(nx, nu, nc, nf, Lmax, P, resident).bytes;
}

template <typename T>
int launch_admm(const IterArgs<T>& args, hipStream_t st) {
  const auto& pb = args.pb;
  const size_t sh = admm_lds_bytes<T>(pb.nx, pb.nu, pb.nc, pb.nf, args.Lmax, args.ip.P, args.resident);
  // KR: reduction entries per wave of the GEMVs, 4 KR >= max(nx + nu, nc)
  const int dim = std::max(pb.nx + pb.nu, pb.nc);
  const void* fn;
  if (dim <= 32) fn = args.resident ? (const void*)k_admm<T, true, 8> : (const void*)k_admm<T, false, 8>;
  else if (dim <= 64) fn = args.resident ? (const void*)k_admm<T, true, 16> : (const void*)k_admm<T, false, 16>;
  else if (dim <= 80) fn = args.resident ? (const void*)k_admm<T, true, 20> : (const void*)k_admm<T, false, 20>;
  else if (dim <= 96) fn = args.resident ? (const void*)k_admm<T, true, 24> : (const void*)k_admm<T, false, 24>;
  else fn = args.resident ? (const void*)k_admm<T, true, 28> : (const void*)k_admm<T, false, 28>;
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh) != hipSuccess)
    return GSLS_ERR_HIP;
  IterArgs<T> a = args;
  void* params[] = {&a};
  hipError_t e = hipLaunchCooperativeKernel(fn, dim3(args.ip.P), dim3(kWG), params, (unsigned)sh, st);
  if (e != hipSuccess) return GSLS_ERR_HIP;
  return GSLS_OK;
}

// Dynamics residual of the FP64 iterate (X, U) against the working-precision
// stage data: one workgroup per stage, ctl->r_dyn = max over stages and rows
// of |x_{k+1} - A_k x_k - B_k u_k - b_k| (a max of non-negative doubles, so
// the maximum of their bit patterns).
template <typename T>
__global__ void __launch_bounds__(kWG) k_rdyn(DevProblem<T> pb, const double* X, const double* U, IterCtl* ctl) {
  __shared__ double red[kWG];
  const int nx = pb.nx, nu = pb.nu;
  double m = 0.0;
  for (int k = blockIdx.x; k < pb.N; k += gridDim.x) {
    const double* xk = X + (size_t)k * nx;
    const double* uk = U + (size_t)k * nu;
    for (int i = tid(); i < nx; i += kWG) {
      const T* Ar = pb.A + ((size_t)k * nx + i) * nx;
      const T* Br = pb.B + ((size_t)k * nx + i) * nu;
      double v = X[(size_t)(k + 1) * nx + i] - (double)pb.b[(size_t)k * nx + i];
      for (int j = 0; j < nx; ++j) v -= (double)Ar[j] * xk[j];
      for (int j = 0; j < nu; ++j) v -= (double)Br[j] * uk[j];
      const double a = fabs(v);
      m = (a > m || a != a) ? a : m;
    }
  }
  red[tid()] = m;
  __syncthreads();
  for (int st = kWG / 2; st > 0; st >>= 1) {
    if (tid() < st) red[tid()] = nanmax(red[tid()], red[tid() + st]);
    __syncthreads();
  }
  if (tid() == 0)
    atomicMax((unsigned long long*)&ctl->r_dyn, (unsigned long long)__double_as_longlong(red[0]));
}

template <typename T>
int launch_rdyn(const DevProblem<T>& pb, const double* X, const double* U, IterCtl* ctl, hipStream_t st) {
  if (pb.N < 1) return GSLS_OK;
  k_rdyn<T><<<std::min(pb.N, 1024), kWG, 0, st>>>(pb, X, U, ctl);
  return hipGetLastError() == hipSuccess ? GSLS_OK : GSLS_ERR_HIP;
}
template int launch_rdyn<float>(const DevProblem<float>&, const double*, const double*, IterCtl*, hipStream_t);
template int launch_rdyn<double>(const DevProblem<double>&, const double*, const double*, IterCtl*, hipStream_t);

template size_t admm_lds_bytes<float>(int, int, int, int, int, int, bool);
template size_t admm_lds_bytes<double>(int, int, int, int, int, int, bool);
template int launch_admm<float>(const IterArgs<float>&, hipStream_t);
template int launch_admm<double>(const IterArgs<double>&, hipStream_t);

}  // namespace gsls
