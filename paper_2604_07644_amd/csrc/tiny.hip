// One-wavefront solver for tiny stage-structured QPs (nx <= 4, nu <= 4, at
// most 8 rows per stage and 8 terminal rows, N <= 63).
//
// The whole ADMM solve of Sec. III-C applied to eq. (admm_qp) -- the factor
// for each rho, every iteration, the residual test and the rho adaptation of
// Sec. IV-A ("Caching") -- runs in one launch of one 64-lane wavefront, in
// FP64, with everything held in registers and the local data share.  At these
// sizes the multi-workgroup solver spends its time in launches, host round
// trips and cross-workgroup exchanges, not in arithmetic.
//
// Lane k owns stage k (lane N the terminal stage).  Per iteration:
//  * the linear terms of eq. (augmented_linear) enter the constant of the
//    backward affine recursion p_k = c_k + Abar_k^T p_{k+1}
//    (Abar_k = A_k + B_k K_k, c_k = qhat_k + K_k^T rhat_k + Abar_k^T P_{k+1} b_k),
//    which is solved by a Kogge-Stone suffix scan over the lanes (the reverse
//    associative scan of eq. (combination_rules), with the rho-invariant
//    transfer maps of every doubling level cached per factor, eq.
//    (controller_cache));
//  * the feed-forward terms, then the forward recursion
//    x_{k+1} = Abar_k x_k + B_k k_k + b_k by a prefix scan that reuses the
//    same cached maps transposed (eq. (nom_recovery));
//  * constraint map, projection, dual update and the residual maxima by
//    wavefront reductions.
// The factor itself (the backward Riccati recursion of eq. (primal_update),
// gains of eq. (controller_cache)) runs stage by stage with the 4 x 4 products
// spread over lanes; it is re-run only when rho changes.
//
// Blocks are 4 x 4 (zero padded) at a stride of 17 doubles per stage, so both
// access patterns -- one stage's 16 entries (factor) and one entry of every
// stage (iteration, lane = stage) -- are free of bank conflicts.
#include <hip/hip_runtime.h>

#include "solver.hpp"

namespace gsls {
namespace {

constexpr int kTW = 64;    // lanes: stages 0..N
constexpr int kTS = 17;    // stride of a padded 4 x 4 block
constexpr int kTL = 6;     // doubling levels: offsets 1..32 cover N <= 63
constexpr int kTC = 8;     // rows per stage (padded)

struct TinyLds {
  double A[kTW * kTS], B[kTW * kTS], Q[kTW * kTS], S[kTW * kTS], R[kTW * kTS];
  double CC[kTW * kTS], DD[kTW * kTS], DC[kTW * kTS];   // C^T C, D^T D, D^T C per stage
  double P[kTW * kTS], K[kTW * kTS], Hm[kTW * kTS];      // P_k, K_k, -(Rhat + B^T P B)^{-1}
  double M[kTL][kTW * kTS];                              // suffix-scan maps per level
  double lo[kTC * kTW], hi[kTC * kTW];                   // row bounds, slot-major (lane fastest)
  double sc[6][16];                                      // factor-step scratch
  int flag;
};

__device__ __forceinline__ double amax_acc(double m, double x) {
  const double a = fabs(x);
  return (a > m || a != a) ? a : m;
}

// Max over the wavefront; a NaN anywhere is the result.
__device__ __forceinline__ double wave_max(double a) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const double b = __shfl_xor(a, o);
    a = (b > a || b != b) ? b : a;
  }
  return a;
}

// Max over the wavefront of non-NaN values through DPP lane moves (quad
// swaps, half-row and row mirrors, then the row broadcasts of lanes 15 and 31);
// lane 63 ends with the maximum, which is returned to every lane.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_max(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const int lo2 = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROWS, 0xF, false);
  const int hi2 = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROWS, 0xF, false);
  return fmax(v, __hiloint2double(hi2, lo2));
}
__device__ __forceinline__ double wave_max_dpp(double v) {
  v = dpp_max<0xB1, 0xF>(v);    // quad_perm [1, 0, 3, 2]
  v = dpp_max<0x4E, 0xF>(v);    // quad_perm [2, 3, 0, 1]
  v = dpp_max<0x141, 0xF>(v);   // row_half_mirror
  v = dpp_max<0x140, 0xF>(v);   // row_mirror
  v = dpp_max<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
  v = dpp_max<0x143, 0xC>(v);   // row_bcast:31 into rows 2 and 3
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 63),
                          __builtin_amdgcn_readlane(__double2loint(v), 63));
}

// Column (lane & 3) of K = -H^{-1} G (lanes 0-3) or of -H^{-1} (lanes 4-7) for
// H = sc[1] whose block past NU is the identity, by Cholesky (reciprocals of
// the pivots); writes K or -H^{-1} of stage k and K to sc[3].  False if a pivot
// of the NU x NU block is not positive.
template <int NU>
__device__ __forceinline__ bool tiny_gain_cols(TinyLds& L, int k, int lane) {
  double l[NU][NU], il[NU];
  bool ok = true;
#pragma unroll
  for (int c = 0; c < NU; ++c) {
    double d = L.sc[1][c * 4 + c];
#pragma unroll
    for (int t = 0; t < c; ++t) d -= l[c][t] * l[c][t];
    if (!(d > 0.0)) { ok = false; d = 1.0; }
    d = sqrt(d);
    il[c] = 1.0 / d;
#pragma unroll
    for (int r = c + 1; r < NU; ++r) {
      double s = L.sc[1][r * 4 + c];
#pragma unroll
      for (int t = 0; t < c; ++t) s -= l[r][t] * l[c][t];
      l[r][c] = s * il[c];
    }
  }
  const int col = lane & 3;
  double x[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) x[r] = lane < 4 ? -L.sc[0][r * 4 + col] : (r == col ? -1.0 : 0.0);
#pragma unroll
  for (int r = 0; r < NU; ++r) {
    double s = x[r];
#pragma unroll
    for (int t = 0; t < r; ++t) s -= l[r][t] * x[t];
    x[r] = s * il[r];
  }
#pragma unroll
  for (int r = NU - 1; r >= 0; --r) {
    double s = x[r];
#pragma unroll
    for (int t = r + 1; t < NU; ++t) s -= l[t][r] * x[t];
    x[r] = s * il[r];
  }
  double* dst = lane < 4 ? L.K : L.Hm;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    dst[k * kTS + r * 4 + col] = x[r];
    if (lane < 4) L.sc[3][r * 4 + col] = x[r];
  }
  return ok;
}

// Riccati recursion for penalty rho (stages N-1..0) and the per-lane cached
// quantities of the iteration.  Returns false if some H_k is not positive
// definite.  Every lane calls it.
__device__ bool tiny_factor(TinyLds& L, const TinyArgs& a, double rho, int nlev, double (&c0)[4],
                            double (&pbk)[4], const double (&qv)[4], const double (&rv)[4], const double (&bv)[4]) {
  const int lane = threadIdx.x, N = a.N, nu = a.nu;
  if (lane == 0) L.flag = 0;
  if (lane < 16) {
    const int e = N * kTS + lane;
    L.P[e] = L.Q[e] + rho * L.CC[e];
  }
  __syncthreads();
  for (int k = N - 1; k >= 0; --k) {
    const double* Pn = L.P + (k + 1) * kTS;
    const double* Ak = L.A + k * kTS;
    const double* Bk = L.B + k * kTS;
    const int e = lane & 15, i = e >> 2, j = e & 3, g = lane >> 4;
    // G = Shat + B^T P A (lanes 0-15), H = Rhat + B^T P B (16-31),
    // A^T P A (32-47), each entry as one double sum
    if (g < 3) {
      const double* X = g == 2 ? Ak : Bk;   // left factor (transposed)
      const double* Y = g == 1 ? Bk : Ak;   // right factor
      double s = 0.0;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        double w = 0.0;
#pragma unroll
        for (int t = 0; t < 4; ++t) w += Pn[a * 4 + t] * Y[t * 4 + j];
        s += X[a * 4 + i] * w;
      }
      if (g == 0) s += L.S[k * kTS + e] + rho * L.DC[k * kTS + e];
      if (g == 1) {
        s += L.R[k * kTS + e] + rho * L.DD[k * kTS + e];
        if (i >= nu) s = i == j ? 1.0 : 0.0;   // padded controls: identity block
      }
      L.sc[g][e] = s;   // sc[0] = G, sc[1] = H, sc[2] = A^T P A
    }
    __syncthreads();
    // Cholesky of the nu x nu block of H (the padded rest is the identity) in
    // every lane of 0-7; lanes 0-3 solve for column c of K = -H^{-1} G, lanes
    // 4-7 for column c of -H^{-1}.
    if (lane < 8) {
      bool ok;
      switch (nu) {
        case 0: case 1: ok = tiny_gain_cols<1>(L, k, lane); break;
        case 2: ok = tiny_gain_cols<2>(L, k, lane); break;
        case 3: ok = tiny_gain_cols<3>(L, k, lane); break;
        default: ok = tiny_gain_cols<4>(L, k, lane); break;
      }
      if (!ok) L.flag = 1;
    }
    __syncthreads();
    // P_k = Qhat + A^T P A + G^T K, symmetrised: 0.5 (P_ij + P_ji) off the diagonal
    if (g == 0) {
      double s1 = L.sc[2][i * 4 + j] + L.Q[k * kTS + i * 4 + j] + rho * L.CC[k * kTS + i * 4 + j];
      double s2 = L.sc[2][j * 4 + i] + L.Q[k * kTS + j * 4 + i] + rho * L.CC[k * kTS + j * 4 + i];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        s1 += L.sc[0][t * 4 + i] * L.sc[3][t * 4 + j];
        s2 += L.sc[0][t * 4 + j] * L.sc[3][t * 4 + i];
      }
      L.P[k * kTS + e] = i == j ? s1 : 0.5 * (s1 + s2);
    }
    __syncthreads();
  }
  if (L.flag) return false;
  // per-lane cached terms: Abar_k, P_{k+1} b_k, the constant of c_k, level-0 map
  const int k = lane;
  if (k < N) {
    const double* Ak = L.A + k * kTS;
    const double* Bk = L.B + k * kTS;
    const double* Kk = L.K + k * kTS;
    const double* Pn = L.P + (k + 1) * kTS;
    double ab[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        double s = Ak[r * 4 + c];
#pragma unroll
        for (int t = 0; t < 4; ++t) s += Bk[r * 4 + t] * Kk[t * 4 + c];
        ab[r][c] = s;
      }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double s = 0.0;
#pragma unroll
      for (int c = 0; c < 4; ++c) s += Pn[r * 4 + c] * bv[c];
      pbk[r] = s;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      double s = qv[c];
#pragma unroll
      for (int t = 0; t < 4; ++t) s += Kk[t * 4 + c] * rv[t] + ab[t][c] * pbk[t];
      c0[c] = s;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) L.M[0][k * kTS + r * 4 + c] = ab[c][r];
  } else {
#pragma unroll
    for (int r = 0; r < 4; ++r) { pbk[r] = 0.0; c0[r] = k == N ? qv[r] : 0.0; }
  }
  // M^(d)_k = M^(d-1)_k M^(d-1)_{k + 2^(d-1)}, kept where k + 2^d <= N
  for (int d = 1; d < nlev; ++d) {
    __syncthreads();
    const int o = 1 << d;
    if (k + o <= N) {
      const double* M1 = L.M[d - 1] + k * kTS;
      const double* M2 = L.M[d - 1] + (k + o / 2) * kTS;
      double out[16];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          double s = 0.0;
#pragma unroll
          for (int t = 0; t < 4; ++t) s += M1[r * 4 + t] * M2[t * 4 + c];
          out[r * 4 + c] = s;
        }
#pragma unroll
      for (int r = 0; r < 16; ++r) L.M[d][k * kTS + r] = out[r];
    }
  }
  __syncthreads();
  return true;
}

// Row slot i of lane k -> index into l, u, z, y (-1: padding).  General rows:
// slot i is row i of the stage (or terminal) block.  Box rows ([I 0; 0 I] per
// stage, I at the terminal stage): slots 0-3 are the state rows, slots 4-7 the
// input rows, so that a row's value is x_i or u_{i-4}.
template <bool BOX>
__device__ __forceinline__ int tiny_row(int i, int k, int N, int nx, int nu, int nc, int nf) {
  if (k > N) return -1;
  const int base = k < N ? k * nc : N * nc;
  if (!BOX) return i < (k < N ? nc : nf) ? base + i : -1;
  if (i < 4) return i < nx ? base + i : -1;
  return (k < N && i - 4 < nu) ? base + nx + (i - 4) : -1;
}

template <bool BOX>
__global__ void __launch_bounds__(kTW) k_tiny(TinyArgs a) {
  extern __shared__ __align__(16) char lds_tiny[];
  TinyLds& L = *reinterpret_cast<TinyLds*>(lds_tiny);
  const int k = threadIdx.x;
  const int N = a.N, nx = a.nx, nu = a.nu, nc = a.nc, nf = a.nf;
  const bool stage = k < N;
  long long t0 = wall_clock64(), tf = 0, ti = 0;
  long long cc0 = clock64(), cl = 0, cf = 0, ci = 0;

  // ---------------------------------------------------------------- load
  {
    double* all = reinterpret_cast<double*>(&L);
    const int nd = (int)(sizeof(TinyLds) / sizeof(double));
    for (int i = k; i < nd; i += kTW) all[i] = 0.0;
  }
  __syncthreads();
  // general rows: C and D rows in registers (box rows need none)
  double Cr[kTC][4], Dr[kTC][4], z[kTC], y[kTC];
  double qv[4], rv[4], bv[4], xz[4];
#pragma unroll
  for (int i = 0; i < kTC; ++i) {
    const int row = tiny_row<BOX>(i, k, N, nx, nu, nc, nf);
    const bool on = row >= 0;
    if (!BOX) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        Cr[i][j] = (on && j < nx) ? (stage ? a.C[((size_t)k * nc + i) * nx + j] : a.CN[(size_t)i * nx + j]) : 0.0;
        Dr[i][j] = (on && stage && j < nu) ? a.D[((size_t)k * nc + i) * nu + j] : 0.0;
      }
    }
    L.lo[i * kTW + k] = on ? a.l[row] : 0.0;
    L.hi[i * kTW + k] = on ? a.u[row] : 0.0;
    z[i] = (on && !a.cold) ? a.z[row] : 0.0;
    y[i] = (on && !a.cold) ? a.y[row] : 0.0;
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    qv[j] = (k <= N && j < nx) ? a.q[(size_t)k * nx + j] : 0.0;
    rv[j] = (stage && j < nu) ? a.r[(size_t)k * nu + j] : 0.0;
    bv[j] = (stage && j < nx) ? a.b[(size_t)k * nx + j] : 0.0;
    xz[j] = (k == 0 && j < nx) ? a.x0v[j] : 0.0;
  }
  if (k <= N) {
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int e = k * kTS + r * 4 + c;
        if (r < nx && c < nx) L.Q[e] = a.Q[((size_t)k * nx + r) * nx + c];
        if (stage) {
          if (r < nx && c < nx) L.A[e] = a.A[((size_t)k * nx + r) * nx + c];
          if (r < nx && c < nu) L.B[e] = a.B[((size_t)k * nx + r) * nu + c];
          if (r < nu && c < nx) L.S[e] = a.S[((size_t)k * nu + r) * nx + c];
          if (r < nu && c < nu) L.R[e] = a.R[((size_t)k * nu + r) * nu + c];
        }
        double cc = 0.0, dd = 0.0, dc = 0.0;
        if (BOX) {
          cc = (r == c && r < nx) ? 1.0 : 0.0;
          dd = (stage && r == c && r < nu) ? 1.0 : 0.0;
        } else {
#pragma unroll
          for (int i = 0; i < kTC; ++i) {
            cc += Cr[i][r] * Cr[i][c];
            dd += Dr[i][r] * Dr[i][c];
            dc += Dr[i][r] * Cr[i][c];
          }
        }
        L.CC[e] = cc; L.DD[e] = dd; L.DC[e] = dc;
      }
  }
  __syncthreads();

  // ---------------------------------------------------------------- solve
  double rho = a.rho0, rp = INFINITY, rd = INFINITY;
  int it = 0, nupd = 0, nfact = 0, status = 2;
  double c0[4], pbk[4];
  double x[4] = {0.0, 0.0, 0.0, 0.0}, u[4] = {0.0, 0.0, 0.0, 0.0};
  {
    const long long c1 = clock64();
    cl = c1 - cc0;
    cc0 = c1;
  }
  if (!tiny_factor(L, a, rho, a.nlev, c0, pbk, qv, rv, bv)) {
    status = 6;
  } else {
    nfact = 1;
    long long t1 = wall_clock64();
    tf += t1 - t0;
    t0 = t1;
    long long c1 = clock64();
    cf += c1 - cc0;
    cc0 = c1;
    // Lanes past the horizon hold zero data (zero-filled blocks, no rows),
    // so every quantity they compute is exactly zero and the loop needs no
    // per-lane branches.
    for (it = 1; it <= a.max_iter; ++it) {
      // linear terms: G^T w per stage, w = y - z
      double tx[4] = {0.0, 0.0, 0.0, 0.0}, tu[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int i = 0; i < kTC; ++i) {
        const double w = y[i] - z[i];
        if (BOX) {
          if (i < 4) tx[i] = w; else tu[i - 4] = w;
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j) { tx[j] += Cr[i][j] * w; tu[j] += Dr[i][j] * w; }
        }
      }
      const double* Kk = L.K + k * kTS;
      double cv[4], rh[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        double s = tx[j];
#pragma unroll
        for (int t = 0; t < 4; ++t) s += Kk[t * 4 + j] * tu[t];
        cv[j] = c0[j] + rho * s;
        rh[j] = rv[j] + rho * tu[j];
      }
      // backward suffix scan p_k = c_k + Abar_k^T p_{k+1}; the map of a lane
      // whose partner lies past the terminal stage is zero
#pragma unroll
      for (int d = 0; d < kTL; ++d) {
        if (d < a.nlev) {
          const double* Md = L.M[d] + k * kTS;
          double pc[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) pc[j] = __shfl_down(cv[j], 1 << d);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            double s = cv[r];
#pragma unroll
            for (int t = 0; t < 4; ++t) s += Md[r * 4 + t] * pc[t];
            cv[r] = s;
          }
        }
      }
      // feed-forward k_k = -H^{-1} (rhat + B^T (p_{k+1} + P_{k+1} b_k)) and the
      // forward offset B_k k_k + b_k
      const double* Bk = L.B + k * kTS;
      const double* Hk = L.Hm + k * kTS;
      double kff[4], dv[4];
      {
        double sv[4], g[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) sv[j] = __shfl_down(cv[j], 1) + pbk[j];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          double acc = rh[t];
#pragma unroll
          for (int j = 0; j < 4; ++j) acc += Bk[j * 4 + t] * sv[j];
          g[t] = acc;
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          double acc = 0.0;
#pragma unroll
          for (int v = 0; v < 4; ++v) acc += Hk[t * 4 + v] * g[v];
          kff[t] = acc;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          double acc = bv[r];
#pragma unroll
          for (int t = 0; t < 4; ++t) acc += Bk[r * 4 + t] * kff[t];
          dv[r] = acc;
        }
      }
      // forward prefix scan x_{k+1} = Abar_k x_k + d_k from x_0; lane k - 2^d's
      // level-d map, transposed, is Abar_{k-1} ... Abar_{k-2^d} (zero where
      // that product would pass the terminal stage)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const double up = __shfl_up(dv[j], 1);
        x[j] = k == 0 ? xz[j] : up;
      }
#pragma unroll
      for (int d = 0; d < kTL; ++d) {
        if (d < a.nlev) {
          const int o = 1 << d;
          const double* Md = L.M[d] + (k >= o ? k - o : 0) * kTS;
          const double on = k >= o ? 1.0 : 0.0;
          double pe[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) pe[j] = on * __shfl_up(x[j], o);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            double s = x[r];
#pragma unroll
            for (int t = 0; t < 4; ++t) s += Md[t * 4 + r] * pe[t];
            x[r] = s;
          }
        }
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        double acc = kff[t];
#pragma unroll
        for (int j = 0; j < 4; ++j) acc += Kk[t * 4 + j] * x[j];
        u[t] = acc;
      }
      // constraint map, projection, dual update; residual maxima, with any
      // NaN or infinity carried by `bad`
      double rpl = 0.0, bad = 0.0, dzx[4] = {0.0, 0.0, 0.0, 0.0}, dzu[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int i = 0; i < kTC; ++i) {
        double v = 0.0;
        if (BOX) {
          v = i < 4 ? x[i] : u[i - 4];
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j) v += Cr[i][j] * x[j] + Dr[i][j] * u[j];
        }
        const double t = v + y[i];
        const double zn = fmin(fmax(t, L.lo[i * kTW + k]), L.hi[i * kTW + k]);
        const double dz = zn - z[i];
        const double rr = v - zn;
        y[i] += rr;
        rpl = fmax(rpl, fabs(rr));
        bad = fma(0.0, rr, bad);
        z[i] = zn;
        if (BOX) {
          if (i < 4) dzx[i] = dz; else dzu[i - 4] = dz;
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j) { dzx[j] += Cr[i][j] * dz; dzu[j] += Dr[i][j] * dz; }
        }
      }
      double rdl = 0.0;
#pragma unroll
      for (int j = 0; j < 4; ++j) rdl = fmax(rdl, fmax(fabs(dzx[j]), fabs(dzu[j])));
      if (bad != bad) { rpl = INFINITY; rdl = INFINITY; }
      // both residuals <= tol  <=>  max(r_p, r_d) <= tol: one reduction per
      // iteration; the two separate maxima only when they are used
      const double cm = wave_max_dpp(fmax(rpl, rho * rdl));
      const bool sig = a.adaptive && a.sigma > 0 && it % a.sigma == 0;
      if (cm <= a.tol || isinf(cm) || it == a.max_iter || sig) {
        rp = wave_max_dpp(rpl);
        rd = rho * wave_max_dpp(rdl);
      }
      if (isinf(cm)) { status = 3; break; }
      if (cm <= a.tol) { status = 1; break; }
      if (it == a.max_iter) { status = 2; break; }
      if (sig) {
        // max(|G xi|, |z|), |H xi| with [[Q S^T], [S R]] per stage and Q_N x_N,
        // |G^T (rho y)|
        double pl = 0.0, hl = 0.0, gl = 0.0;
        double gx[4] = {0.0, 0.0, 0.0, 0.0}, gu[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int i = 0; i < kTC; ++i) {
          double v = 0.0;
          const double w = rho * y[i];
          if (BOX) {
            v = i < 4 ? x[i] : u[i - 4];
            if (i < 4) gx[i] = w; else gu[i - 4] = w;
          } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              v += Cr[i][j] * x[j] + Dr[i][j] * u[j];
              gx[j] += Cr[i][j] * w;
              gu[j] += Dr[i][j] * w;
            }
          }
          pl = fmax(pl, fmax(fabs(v), fabs(z[i])));
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) gl = fmax(gl, fmax(fabs(gx[j]), fabs(gu[j])));
        const double* Qk = L.Q + k * kTS;
        const double* Sk = L.S + k * kTS;
        const double* Rk = L.R + k * kTS;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          double s = 0.0, s2 = 0.0;
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            s += Qk[r * 4 + t] * x[t] + Sk[t * 4 + r] * u[t];
            s2 += Sk[r * 4 + t] * x[t] + Rk[r * 4 + t] * u[t];
          }
          hl = fmax(hl, fmax(fabs(s), fabs(s2)));
        }
        const double pscale = wave_max_dpp(pl);
        const double dscale = fmax(fmax(wave_max_dpp(hl), wave_max_dpp(gl)), a.hnorm);
        const double eps = 1e-10;
        const double ratio = (rp / (pscale + eps)) / (rd / (dscale + eps) + eps);
        double rn = rho * sqrt(ratio);
        rn = fmin(fmax(rn, a.rho_min), a.rho_max);
        if (rn > rho * a.rho_tol || rn < rho / a.rho_tol) {
#pragma unroll
          for (int i = 0; i < kTC; ++i) y[i] *= rho / rn;
          rho = rn;
          ++nupd;
          long long t1 = wall_clock64(), c2 = clock64();
          ti += t1 - t0;
          t0 = t1;
          ci += c2 - cc0;
          cc0 = c2;
          if (!tiny_factor(L, a, rho, a.nlev, c0, pbk, qv, rv, bv)) { status = 6; break; }
          ++nfact;
          t1 = wall_clock64();
          tf += t1 - t0;
          t0 = t1;
          c2 = clock64();
          cf += c2 - cc0;
          cc0 = c2;
        }
      }
    }
    if (it > a.max_iter) it = a.max_iter;
    ti += wall_clock64() - t0;
    ci += clock64() - cc0;
  }

  // ---------------------------------------------------------------- store
  double rdl = 0.0;
  {
    double xn[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) xn[j] = __shfl_down(x[j], 1);
    if (stage && status != 6) {
      const double* Ak = L.A + k * kTS;
      const double* Bk = L.B + k * kTS;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        double s = xn[r] - bv[r];
#pragma unroll
        for (int t = 0; t < 4; ++t) s -= Ak[r * 4 + t] * x[t] + Bk[r * 4 + t] * u[t];
        rdl = fmax(rdl, fabs(s));
      }
    }
  }
  const double rdyn = wave_max(rdl);
  if (status != 6) {
    if (k <= N)
      for (int j = 0; j < nx; ++j) a.X[(size_t)k * nx + j] = x[j];
    if (stage)
      for (int t = 0; t < nu; ++t) a.U[(size_t)k * nu + t] = u[t];
  }
  // the iterate (z, y) is written also when a factor failed: a cold start
  // leaves zeros, as the solver state before the first iteration
#pragma unroll
  for (int i = 0; i < kTC; ++i) {
    const int row = tiny_row<BOX>(i, k, N, nx, nu, nc, nf);
    if (row >= 0) {
      a.z[row] = z[i];
      a.y[row] = y[i];
    }
  }
  if (k == 0) {
    TinyOut o;
    o.it = it; o.status = status; o.nupd = nupd; o.nfact = nfact;
    o.r_p = rp; o.r_d = rd; o.rho = rho; o.r_dyn = rdyn;
    o.t_factor = (unsigned long long)tf; o.t_iter = (unsigned long long)ti;
    o.c_load = (unsigned long long)cl; o.c_factor = (unsigned long long)cf; o.c_iter = (unsigned long long)ci;
    *a.out = o;
  }
}

}  // namespace

bool tiny_fits(int N, int nx, int nu, int nc, int nf) {
  return N >= 1 && N < kTW && nx >= 1 && nx <= 4 && nu >= 0 && nu <= 4 && nc >= 0 && nc <= kTC && nf >= 0 &&
         nf <= kTC;
}

int launch_tiny(const TinyArgs& args, hipStream_t st) {
  if (!tiny_fits(args.N, args.nx, args.nu, args.nc, args.nf) || args.nlev < 1 || args.nlev > kTL ||
      (1 << (args.nlev - 1)) > args.N || (1 << args.nlev) <= args.N)
    return GSLS_ERR_DIM;
  static bool attr = false;
  if (!attr) {
    if (hipFuncSetAttribute((const void*)k_tiny<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)sizeof(TinyLds)) != hipSuccess ||
        hipFuncSetAttribute((const void*)k_tiny<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)sizeof(TinyLds)) != hipSuccess)
      return GSLS_ERR_HIP;
    attr = true;
  }
  if (args.box)
    hipLaunchKernelGGL(k_tiny<true>, dim3(1), dim3(kTW), sizeof(TinyLds), st, args);
  else
    hipLaunchKernelGGL(k_tiny<false>, dim3(1), dim3(kTW), sizeof(TinyLds), st, args);
  return hipGetLastError() == hipSuccess ? GSLS_OK : GSLS_ERR_HIP;
}

}  // namespace gsls
