// Factor epoch of the ADMM QP solver (everything that depends on rho but not
// on the ADMM iterate), Sec. IV-A of the paper:
//   1. augmented costs, eq. (augmented_matrices), cross term S + rho D^T C;
//   2. scan elements (P~, A~, C~) of eq. (assoc_init), FP64 Cholesky of R_hat;
//   3. reverse associative scan over the horizon with the combination rules of
//      eq. (combination_rules), organised as chunk folds (one workgroup per
//      chunk), a recursive-doubling suffix scan over the chunk results (one
//      launch per level), and one application of each suffix to the terminal
//      value function, which yields P at every chunk boundary; the inverse of
//      M = I + C~ P~ is formed in FP64 (Gauss-Jordan with partial pivoting);
//   4. Riccati fix-up inside each chunk giving P_k, the gains of
//      eq. (controller_cache) (Gamma inverted in FP64), Abar = A + B K;
//   5. transfer maps of the iteration's chunked affine scans: products of
//      consecutive Abar and their doubling levels.
#include "dev_common.hpp"
#include "solver.hpp"

namespace gsls {

// LDS layout shared by the epoch kernels (bytes): GEMM slabs, the FP64
// augmented matrix [M | I] of the Gauss-Jordan inverse, and its bookkeeping.
template <typename T>
struct EpochLds {
  static constexpr size_t gemm = sizeof(T) * kGemmSmem;
  static constexpr size_t aug = sizeof(double) * kMaxNx * 2 * kMaxNx;
  static constexpr size_t book = sizeof(double) * kMaxNx + 2 * sizeof(int) * kMaxNx;
  static constexpr size_t total = gemm + aug + book;
};

struct LdsPtrs {
  LDS char* gsm; LDS double* Aug; LDS double* dg; LDS int* perm; LDS int* used;
};
template <typename T>
__device__ inline LdsPtrs carve(char* base_generic) {
  LDS char* base = (LDS char*)base_generic;
  LdsPtrs p;
  p.gsm = base;
  p.Aug = (LDS double*)(base + EpochLds<T>::gemm);
  p.dg = (LDS double*)(base + EpochLds<T>::gemm + EpochLds<T>::aug);
  p.perm = (LDS int*)(p.dg + kMaxNx);
  p.used = p.perm + kMaxNx;
  return p;
}

// Aug <- [shift I + X | I] for the n x n matrix X (T, any memory), FP64; the
// loads of X are batched (wg_block_pass).
template <typename T>
__device__ inline void fill_aug_shift(int n, LDS double* Aug, const T* X, double shift) {
  const int ld = 2 * n;
  wg_block_pass<double>(n, n, [&](int i, int c) { return double(X[(size_t)i * n + c]) + (i == c ? shift : 0.0); },
                        [&](int i, int c, double v) { Aug[i * ld + c] = v; });
  for (int i = wave(); i < n; i += 4)
    for (int c = lane(); c < n; c += 64) Aug[i * ld + n + c] = c == i ? 1.0 : 0.0;
  __syncthreads();
}
// Aug <- [I + X | I].
template <typename T>
__device__ inline void fill_aug_ipx(int n, LDS double* Aug, const T* X) { fill_aug_shift(n, Aug, X, 1.0); }
// Aug <- [X | I] for the symmetric n x n matrix X (T, ld n).
template <typename T>
__device__ inline void fill_aug(int n, LDS double* Aug, const T* X) { fill_aug_shift(n, Aug, X, 0.0); }

__device__ inline void flag_fail(int* status) {
  if (tid() == 0) atomicMax(status, 1);
}

// -------------------------------------------------------------- elements
template <typename T>
__global__ void __launch_bounds__(kWG) k_elements(DevProblem<T> pb, DevEpochWork<T> ew, double rho) {
  extern __shared__ __align__(16) char lds[];
  LdsPtrs L = carve<T>(lds);
  LDS T* gsm = (LDS T*)L.gsm;
  const int i = blockIdx.x;
  const int nx = pb.nx, nu = pb.nu, nc = pb.nc, N = pb.N;
  const size_t xx = (size_t)nx * nx;
  T* Qh = ew.Qh + i * xx;
  const T r = T(rho);
  if (i == N) {
    wg_copy(nx, nx, Qh, nx, pb.Q + N * xx, nx);
    __syncthreads();
    if (pb.nf > 0) wg_gemm<T>(nx, nx, pb.nf, r, pb.CN, nx, true, pb.CN, nx, false, T(1), Qh, nx, gsm);
    wg_symmetrize(nx, Qh, nx);
    wg_copy(nx, nx, ew.eP + N * xx, nx, Qh, nx);
    for (int t = tid(); t < (int)xx; t += kWG) { ew.eA[N * xx + t] = T(0); ew.eC[N * xx + t] = T(0); }
    return;
  }
  const T* C = pb.C + (size_t)i * nc * nx;
  const T* D = pb.D + (size_t)i * nc * nu;
  const T* A = pb.A + i * xx;
  const T* B = pb.B + (size_t)i * nx * nu;
  T* Rh = ew.Rh + (size_t)i * nu * nu;
  T* Sh = ew.Sh + (size_t)i * nu * nx;
  wg_copy(nx, nx, Qh, nx, pb.Q + i * xx, nx);
  wg_copy(nu, nu, Rh, nu, pb.R + (size_t)i * nu * nu, nu);
  wg_copy(nu, nx, Sh, nx, pb.S + (size_t)i * nu * nx, nx);
  __syncthreads();
  wg_gemm<T>(nx, nx, nc, r, C, nx, true, C, nx, false, T(1), Qh, nx, gsm);
  wg_gemm<T>(nu, nu, nc, r, D, nu, true, D, nu, false, T(1), Rh, nu, gsm);
  wg_gemm<T>(nu, nx, nc, r, D, nu, true, C, nx, false, T(1), Sh, nx, gsm);
  wg_symmetrize(nx, Qh, nx);
  wg_symmetrize(nu, Rh, nu);
  // FP64 inverse of R_hat (symmetric positive definite: no pivoting, positive
  // pivots required), then W1 = R_hat^{-1} S_hat and W2 = R_hat^{-1} B^T.
  fill_aug(nu, L.Aug, Rh);
  T* Rinv = ew.eC + i * xx;      // staging in this stage's element slots, rewritten below
  T* W1s = ew.eA + i * xx;
  T* W2s = ew.eP + i * xx;
  if (!wg_gj_inverse<T>(nu, L.Aug, false, L.perm, L.used, L.dg, Rinv, nu)) {
    flag_fail(ew.status);
    return;
  }
  // W1 = R_hat^{-1} S_hat, W2 = R_hat^{-1} B^T (nu x nx each) kept in LDS (as T)
  // while the element slots are overwritten
  LDS T* W1l = (LDS T*)L.Aug;
  LDS T* W2l = W1l + nu * nx;
  T* W1g = ew.eA + i * xx;
  T* W2g = ew.eP + i * xx;
  wg_gemm<T>(nu, nx, nu, T(1), Rinv, nu, false, Sh, nx, false, T(0), W1g, nx, gsm);
  wg_gemm<T>(nu, nx, nu, T(1), Rinv, nu, false, B, nu, true, T(0), W2g, nx, gsm);
  for (int r = wave(); r < nu; r += 4)
    for (int c = lane(); c < nx; c += 64) { W1l[r * nx + c] = W1g[r * nx + c]; W2l[r * nx + c] = W2g[r * nx + c]; }
  __syncthreads();
  T* eP = ew.eP + i * xx;
  T* eA = ew.eA + i * xx;
  T* eC = ew.eC + i * xx;
  wg_copy(nx, nx, eA, nx, A, nx);
  wg_copy(nx, nx, eP, nx, Qh, nx);
  __syncthreads();
  // A~ = A - B W1,  C~ = B W2 = B R_hat^{-1} B^T,  P~ = Q_hat - S_hat^T W1  (W in LDS:
  // staged to T scratch views for the GEMM operand loads)
  T* W1 = (T*)W1l;
  T* W2 = (T*)W2l;
  wg_gemm<T>(nx, nx, nu, T(-1), B, nu, false, W1, nx, false, T(1), eA, nx, gsm);
  wg_gemm<T>(nx, nx, nu, T(1), B, nu, false, W2, nx, false, T(0), eC, nx, gsm);
  wg_gemm<T>(nx, nx, nu, T(-1), Sh, nx, true, W1, nx, false, T(1), eP, nx, gsm);
  wg_symmetrize(nx, eP, nx);
  wg_symmetrize(nx, eC, nx);
}

// e_out = e1 (x) e2 (matrix part of eq. (combination_rules)), with
//   M = I + C1 P2 inverted in FP64 (Gauss-Jordan, partial pivoting),
//   Y1 = M^{-1} A1,  Y2 = M^{-1} C1,
//   A = A2 Y1,  C = A2 Y2 A2^T + C2,  P = Y1^T (P2 A1) + P1.
// (Upsilon = A1^T (I + P2 C1)^{-1} = (M^{-1} A1)^T because P2, C1 are symmetric,
//  and Psi = A2 M^{-1}.)  S0..S2: n x n global scratch.  Returns false if M is
// singular.
// role < 0 computes all three outputs.  Two workgroups can share one combination
// instead: both invert M (identical arithmetic), role 0 then forms C (Y2, A2 Y2,
// C) and role 1 forms A and P (P2 A1 first, then Y1, A, P), so neither waits for
// the other and the critical path is five products and one inverse, not eight.
// The outputs equal the one-workgroup combination bit for bit.
template <typename T>
__device__ bool wg_combine(int n, const T* P1, const T* A1, const T* C1, const T* P2, const T* A2,
                           const T* C2, T* P, T* A, T* C, T* S0, T* S1, T* S2, const LdsPtrs& L,
                           int role = -1) {
  LDS T* gsm = (LDS T*)L.gsm;
  const bool do_c = role != 1, do_ap = role != 0;
  if (do_ap && role == 1)
    wg_gemm<T>(n, n, n, T(1), P2, n, false, A1, n, false, T(0), S2, n, gsm);   // P2 A1 (needs no inverse)
  wg_gemm<T>(n, n, n, T(1), C1, n, false, P2, n, false, T(0), S0, n, gsm);
  fill_aug_ipx(n, L.Aug, S0);
  if (!wg_gj_inverse<T>(n, L.Aug, true, L.perm, L.used, L.dg, S0, n)) return false;
  if (role < 0) {
    wg_gemm<T>(n, n, n, T(1), S0, n, false, A1, n, false, T(0), S1, n, gsm);   // Y1
    wg_gemm<T>(n, n, n, T(1), S0, n, false, C1, n, false, T(0), S2, n, gsm);   // Y2
    wg_gemm<T>(n, n, n, T(1), A2, n, false, S1, n, false, T(0), A, n, gsm);
    wg_gemm<T>(n, n, n, T(1), A2, n, false, S2, n, false, T(0), S0, n, gsm);
    wg_copy(n, n, C, n, C2, n);
    __syncthreads();
    wg_gemm<T>(n, n, n, T(1), S0, n, false, A2, n, true, T(1), C, n, gsm);
    wg_gemm<T>(n, n, n, T(1), P2, n, false, A1, n, false, T(0), S0, n, gsm);
    wg_copy(n, n, P, n, P1, n);
    __syncthreads();
    wg_gemm<T>(n, n, n, T(1), S1, n, true, S0, n, false, T(1), P, n, gsm);
    wg_symmetrize(n, P, n);
    wg_symmetrize(n, C, n);
    return true;
  }
  if (do_c) {
    wg_gemm<T>(n, n, n, T(1), S0, n, false, C1, n, false, T(0), S2, n, gsm);   // Y2
    wg_gemm<T>(n, n, n, T(1), A2, n, false, S2, n, false, T(0), S0, n, gsm);   // A2 Y2
    wg_copy(n, n, C, n, C2, n);
    __syncthreads();
    wg_gemm<T>(n, n, n, T(1), S0, n, false, A2, n, true, T(1), C, n, gsm);
    wg_symmetrize(n, C, n);
  } else {
    wg_gemm<T>(n, n, n, T(1), S0, n, false, A1, n, false, T(0), S1, n, gsm);   // Y1
    wg_gemm<T>(n, n, n, T(1), A2, n, false, S1, n, false, T(0), A, n, gsm);
    wg_copy(n, n, P, n, P1, n);
    __syncthreads();
    wg_gemm<T>(n, n, n, T(1), S1, n, true, S2, n, false, T(1), P, n, gsm);   // + Y1^T (P2 A1)
    wg_symmetrize(n, P, n);
  }
  return true;
}

__device__ __forceinline__ int chunk_begin(int c, int N, int P) { return (int)(((long long)c * N) / P); }

// ------------------------------------------------------------ chunk fold
template <typename T>
__global__ void __launch_bounds__(kWG) k_fold(DevProblem<T> pb, DevEpochWork<T> ew, int Pe) {
  extern __shared__ __align__(16) char lds[];
  LdsPtrs L = carve<T>(lds);
  const int c = blockIdx.x, nx = pb.nx;
  const size_t xx = (size_t)nx * nx;
  const int s = chunk_begin(c, pb.N, Pe), e = chunk_begin(c + 1, pb.N, Pe);
  T* fP = ew.fP + c * xx; T* fA = ew.fA + c * xx; T* fC = ew.fC + c * xx;
  const size_t sl = ew.slot;
  T* sc = ew.scratch + (size_t)c * 8 * sl;
  wg_copy(nx, nx, fP, nx, ew.eP + (e - 1) * xx, nx);
  wg_copy(nx, nx, fA, nx, ew.eA + (e - 1) * xx, nx);
  wg_copy(nx, nx, fC, nx, ew.eC + (e - 1) * xx, nx);
  __syncthreads();
  for (int i = e - 2; i >= s; --i) {
    if (!wg_combine<T>(nx, ew.eP + i * xx, ew.eA + i * xx, ew.eC + i * xx, fP, fA, fC,
                       sc + 3 * sl, sc + 4 * sl, sc + 5 * sl, sc, sc + sl, sc + 2 * sl, L)) {
      flag_fail(ew.status);
      return;
    }
    wg_copy(nx, nx, fP, nx, sc + 3 * sl, nx);
    wg_copy(nx, nx, fA, nx, sc + 4 * sl, nx);
    wg_copy(nx, nx, fC, nx, sc + 5 * sl, nx);
    __syncthreads();
  }
}

// ---------------------------------------------------- cross-chunk suffix
// Suffix products of the chunk elements by recursive doubling, one launch per
// level: S_c <- S_c (x) S_{c + 2^d} (or unchanged when c + 2^d >= Pe).  After
// ceil(log2 Pe) levels S_c = E_c (x) E_{c+1} (x) ... (x) E_{Pe-1}.  With
// split, two workgroups share each chunk's combination (blockIdx.x = 2c + role,
// each with its own half of the chunk's scratch slots).
template <typename T>
__global__ void __launch_bounds__(kWG) k_suffix_level(DevProblem<T> pb, DevEpochWork<T> ew, int Pe, int d,
                                                      int split) {
  extern __shared__ __align__(16) char lds[];
  LdsPtrs L = carve<T>(lds);
  const int c = split ? (int)blockIdx.x >> 1 : (int)blockIdx.x, nx = pb.nx;
  const int role = split ? (int)(blockIdx.x & 1) : -1;
  const size_t xx = (size_t)nx * nx;
  const bool even = (d % 2) == 0;
  const T* sP = even ? ew.fP : ew.gP; const T* sA = even ? ew.fA : ew.gA; const T* sC = even ? ew.fC : ew.gC;
  T* dP = even ? ew.gP : ew.fP; T* dA = even ? ew.gA : ew.fA; T* dC = even ? ew.gC : ew.fC;
  const int h = 1 << d;
  if (c + h < Pe) {
    T* sc = ew.scratch + (size_t)c * 8 * ew.slot + (role == 1 ? 4 * ew.slot : 0);
    if (!wg_combine<T>(nx, sP + c * xx, sA + c * xx, sC + c * xx, sP + (c + h) * xx, sA + (c + h) * xx,
                       sC + (c + h) * xx, dP + c * xx, dA + c * xx, dC + c * xx, sc, sc + ew.slot,
                       sc + 2 * ew.slot, L, role))
      flag_fail(ew.status);
  } else {
    if (role != 1) wg_copy(nx, nx, dC + c * xx, nx, sC + c * xx, nx);
    if (role != 0) {
      wg_copy(nx, nx, dP + c * xx, nx, sP + c * xx, nx);
      wg_copy(nx, nx, dA + c * xx, nx, sA + c * xx, nx);
    }
  }
}

// P at each chunk's right end: the terminal value function Q_hat_N carried
// back through the suffix product of the following chunks.  Applying an
// element (P~, A~, C~) to a value function P (the combination with an element
// whose A~ = C~ = 0) gives A~^T (I + P C~)^{-1} P A~ + P~.
template <typename T>
__global__ void __launch_bounds__(kWG) k_pend(DevProblem<T> pb, DevEpochWork<T> ew, int Pe, int final_in_g) {
  extern __shared__ __align__(16) char lds[];
  LdsPtrs L = carve<T>(lds);
  LDS T* gsm = (LDS T*)L.gsm;
  const int c = blockIdx.x, nx = pb.nx;
  const size_t xx = (size_t)nx * nx;
  const T* PN = ew.eP + (size_t)pb.N * xx;
  T* out = ew.Pend + c * xx;
  if (c == Pe - 1) {
    wg_copy(nx, nx, out, nx, PN, nx);
    return;
  }
  const T* fP = (final_in_g ? ew.gP : ew.fP) + (c + 1) * xx;
  const T* fA = (final_in_g ? ew.gA : ew.fA) + (c + 1) * xx;
  const T* fC = (final_in_g ? ew.gC : ew.fC) + (c + 1) * xx;
  T* S0 = ew.scratch + (size_t)c * 8 * ew.slot;
  T* S1 = S0 + ew.slot;
  wg_gemm<T>(nx, nx, nx, T(1), fC, nx, false, PN, nx, false, T(0), S0, nx, gsm);
  fill_aug_ipx(nx, L.Aug, S0);
  if (!wg_gj_inverse<T>(nx, L.Aug, true, L.perm, L.used, L.dg, S0, nx)) { flag_fail(ew.status); return; }
  wg_gemm<T>(nx, nx, nx, T(1), S0, nx, false, fA, nx, false, T(0), S1, nx, gsm);   // Y = M^{-1} A~
  wg_gemm<T>(nx, nx, nx, T(1), PN, nx, false, fA, nx, false, T(0), S0, nx, gsm);   // P A~
  wg_copy(nx, nx, out, nx, fP, nx);
  __syncthreads();
  wg_gemm<T>(nx, nx, nx, T(1), S1, nx, true, S0, nx, false, T(1), out, nx, gsm);
  wg_symmetrize(nx, out, nx);
}

// ------------------------------------------------------- Riccati fix-up
// Backward Riccati recursion over the chunk from P at its right end:
//   H = R_hat + B^T P B,  G = S_hat + B^T P A,  Gamma = H^{-1} (FP64, SPD),
//   K = -Gamma G,  P <- Q_hat + A^T P A + G^T K,
// writing the iteration operator F = [[Abar, B], [K, I]] (Abar = A + B K),
// Gamma, ev = Abar^T P b and fv = B^T P b of every stage (eq. (controller_cache)).
template <typename T>
__global__ void __launch_bounds__(kWG) k_fixup(DevProblem<T> pb, DevEpochWork<T> ew, DevFactor<T> fc,
                                               int Pe) {
  extern __shared__ __align__(16) char lds[];
  LdsPtrs L = carve<T>(lds);
  LDS T* gsm = (LDS T*)L.gsm;
  const int c = blockIdx.x, nx = pb.nx, nu = pb.nu, nxu = nx + nu;
  const size_t xx = (size_t)nx * nx, ux = (size_t)nu * nx;
  const int s = chunk_begin(c, pb.N, Pe), e = chunk_begin(c + 1, pb.N, Pe);
  const size_t sl = ew.slot;
  T* sc = ew.scratch + (size_t)c * 8 * sl;
  T* Pc = sc; T* PB = sc + sl; T* PA = sc + 2 * sl; T* Pb = sc + 3 * sl; T* Hs = sc + 4 * sl;
  T* G = sc + 5 * sl; T* Pn = sc + 6 * sl;
  wg_copy(nx, nx, Pc, nx, ew.Pend + c * xx, nx);
  __syncthreads();
  for (int i = e - 1; i >= s; --i) {
    const T* A = pb.A + i * xx;
    const T* B = pb.B + (size_t)i * nx * nu;
    const T* b = pb.b + (size_t)i * nx;
    T* F = fc.F + (size_t)i * nxu * nxu;
    wg_gemm<T>(nx, nu, nx, T(1), Pc, nx, false, B, nu, false, T(0), PB, nu, gsm);
    wg_gemm<T>(nx, nx, nx, T(1), Pc, nx, false, A, nx, false, T(0), PA, nx, gsm);
    wg_gemm<T>(nx, 1, nx, T(1), Pc, nx, false, b, 1, false, T(0), Pb, 1, gsm);
    wg_copy(nu, nu, Hs, nu, ew.Rh + (size_t)i * nu * nu, nu);
    wg_copy(nu, nx, G, nx, ew.Sh + i * ux, nx);
    // F's B block and identity block
    for (int r = wave(); r < nxu; r += 4)
      for (int cc = nx + lane(); cc < nxu; cc += 64)
        F[(size_t)r * nxu + cc] = r < nx ? B[(size_t)r * nu + (cc - nx)] : (r - nx == cc - nx ? T(1) : T(0));
    __syncthreads();
    wg_gemm<T>(nu, nu, nx, T(1), B, nu, true, PB, nu, false, T(1), Hs, nu, gsm);
    wg_gemm<T>(nu, nx, nx, T(1), B, nu, true, PA, nx, false, T(1), G, nx, gsm);
    wg_symmetrize(nu, Hs, nu);
    // FP64 elimination of [H | G | I] for the symmetric positive definite H:
    // K = -H^{-1} G and Gamma = H^{-1}.  K is read from the elimination, not
    // formed from a rounded Gamma (that would carry cond(H) times Gamma's
    // rounding into K and from there into P).
    T* K = F + (size_t)nx * nxu;         // K block: rows nx.., columns 0..nx-1
    T* Gam = fc.Gam + (size_t)i * nu * nu;
    const int lda = 2 * nu + nx;
    for (int r = wave(); r < nu; r += 4)
      for (int cc = lane(); cc < lda; cc += 64) {
        double v;
        if (cc < nu) v = double(Hs[(size_t)r * nu + cc]);
        else if (cc < nu + nx) v = double(G[(size_t)r * nx + (cc - nu)]);
        else v = (cc - nu - nx == r) ? 1.0 : 0.0;
        L.Aug[r * lda + cc] = v;
      }
    __syncthreads();
    if (!wg_gj_eliminate(nu, lda, L.Aug, false, L.perm, L.used, L.dg)) { flag_fail(ew.status); return; }
    wg_gj_extract<T>(nu, lda, L.Aug, L.perm, L.dg, 0, nx, -1.0, K, nxu);
    wg_gj_extract<T>(nu, lda, L.Aug, L.perm, L.dg, nx, nu, 1.0, Gam, nu);
    // Abar = A + B K  (block rows 0..nx-1, columns 0..nx-1 of F)
    wg_copy(nx, nx, F, nxu, A, nx);
    __syncthreads();
    wg_gemm<T>(nx, nx, nu, T(1), B, nu, false, K, nxu, false, T(1), F, nxu, gsm);
    // ev = Abar^T P b, fv = B^T P b
    wg_gemm<T>(nx, 1, nx, T(1), F, nxu, true, Pb, 1, false, T(0), fc.ev + (size_t)i * nx, 1, gsm);
    wg_gemm<T>(nu, 1, nx, T(1), B, nu, true, Pb, 1, false, T(0), fc.fv + (size_t)i * nu, 1, gsm);
    if (i == s) break;   // the chunk's first stage: its P is not needed
    // P_i = Q_hat + A^T P A + G^T K
    wg_copy(nx, nx, Pn, nx, ew.Qh + i * xx, nx);
    __syncthreads();
    wg_gemm<T>(nx, nx, nx, T(1), A, nx, true, PA, nx, false, T(1), Pn, nx, gsm);
    wg_gemm<T>(nx, nx, nu, T(1), G, nx, true, K, nxu, false, T(1), Pn, nx, gsm);
    wg_symmetrize(nx, Pn, nx);
    wg_copy(nx, nx, Pc, nx, Pn, nx);
    __syncthreads();
  }
}

// -------------------------------------- transfer maps of the iteration scan
// Phi[0][c] = Abar_{e-1} ... Abar_s over iteration chunk c.
template <typename T>
__global__ void __launch_bounds__(kWG) k_chunkmap(DevProblem<T> pb, DevEpochWork<T> ew, DevFactor<T> fc,
                                                  int Pi) {
  extern __shared__ __align__(16) char lds[];
  LdsPtrs L = carve<T>(lds);
  LDS T* gsm = (LDS T*)L.gsm;
  const int c = blockIdx.x, nx = pb.nx, nxu = nx + pb.nu;
  const size_t xx = (size_t)nx * nx, ff = (size_t)nxu * nxu;
  const int s = chunk_begin(c, pb.N, Pi), e = chunk_begin(c + 1, pb.N, Pi);
  T* out = fc.Phi + c * xx;
  T* sc = ew.scratch + (size_t)c * 8 * ew.slot;
  wg_copy(nx, nx, out, nx, fc.F + s * ff, nxu);
  __syncthreads();
  for (int i = s + 1; i < e; ++i) {
    wg_gemm<T>(nx, nx, nx, T(1), fc.F + i * ff, nxu, false, out, nx, false, T(0), sc, nx, gsm);
    wg_copy(nx, nx, out, nx, sc, nx);
    __syncthreads();
  }
}

// Phi[d+1][c] = Phi[d][c + 2^d] Phi[d][c]  for c + 2^{d+1} <= Pi.
template <typename T>
__global__ void __launch_bounds__(kWG) k_level(DevProblem<T> pb, DevFactor<T> fc, int Pi, int d) {
  extern __shared__ __align__(16) char lds[];
  LdsPtrs L = carve<T>(lds);
  LDS T* gsm = (LDS T*)L.gsm;
  const int c = blockIdx.x, nx = pb.nx;
  const size_t xx = (size_t)nx * nx;
  const int h = 1 << d;
  if (c + 2 * h > Pi) return;
  const T* lo = fc.Phi + ((size_t)d * Pi + c) * xx;
  const T* hi = fc.Phi + ((size_t)d * Pi + c + h) * xx;
  T* out = fc.Phi + ((size_t)(d + 1) * Pi + c) * xx;
  wg_gemm<T>(nx, nx, nx, T(1), hi, nx, false, lo, nx, false, T(0), out, nx, gsm);
}

// ----------------------------------------------------------------- host
#define GSLS_LAUNCH_CHECK()                                  \
  do {                                                       \
    hipError_t e_ = hipGetLastError();                       \
    if (e_ != hipSuccess) return GSLS_ERR_HIP;               \
  } while (0)

template <typename T>
int epoch_set_attributes() {
  const int bytes = (int)EpochLds<T>::total;
  if (hipFuncSetAttribute((const void*)k_elements<T>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) != hipSuccess) return GSLS_ERR_HIP;
  if (hipFuncSetAttribute((const void*)k_fold<T>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) != hipSuccess) return GSLS_ERR_HIP;
  if (hipFuncSetAttribute((const void*)k_suffix_level<T>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) != hipSuccess) return GSLS_ERR_HIP;
  if (hipFuncSetAttribute((const void*)k_pend<T>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) != hipSuccess) return GSLS_ERR_HIP;
  if (hipFuncSetAttribute((const void*)k_fixup<T>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) != hipSuccess) return GSLS_ERR_HIP;
  if (hipFuncSetAttribute((const void*)k_chunkmap<T>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) != hipSuccess) return GSLS_ERR_HIP;
  if (hipFuncSetAttribute((const void*)k_level<T>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) != hipSuccess) return GSLS_ERR_HIP;
  return GSLS_OK;
}

// Enqueue one factor epoch on `st`.  Pe: chunks of the factor scan, Pi: chunks
// (workgroups) of the iteration kernel, nlev = ceil(log2 Pi).
constexpr int kEpochSplitMaxWG = 256;   // compute units of the device

template <typename T>
int launch_epoch(const DevProblem<T>& pb, const DevEpochWork<T>& ew, const DevFactor<T>& fc,
                 double rho, int Pe, int Pi, int nlev, hipStream_t st) {
  const size_t sh = EpochLds<T>::total;
  k_elements<T><<<pb.N + 1, kWG, sh, st>>>(pb, ew, rho);
  GSLS_LAUNCH_CHECK();
  k_fold<T><<<Pe, kWG, sh, st>>>(pb, ew, Pe);
  GSLS_LAUNCH_CHECK();
  int nle = 0;
  while ((1 << nle) < Pe) ++nle;
  // two workgroups per combination while that still fits one per compute unit
  const int split = 2 * Pe <= kEpochSplitMaxWG ? 1 : 0;
  for (int d = 0; d < nle; ++d) {
    k_suffix_level<T><<<split ? 2 * Pe : Pe, kWG, sh, st>>>(pb, ew, Pe, d, split);
    GSLS_LAUNCH_CHECK();
  }
  k_pend<T><<<Pe, kWG, sh, st>>>(pb, ew, Pe, nle % 2);
  GSLS_LAUNCH_CHECK();
  k_fixup<T><<<Pe, kWG, sh, st>>>(pb, ew, fc, Pe);
  GSLS_LAUNCH_CHECK();
  k_chunkmap<T><<<Pi, kWG, sh, st>>>(pb, ew, fc, Pi);
  GSLS_LAUNCH_CHECK();
  for (int d = 0; d + 1 < nlev; ++d) {
    k_level<T><<<Pi, kWG, sh, st>>>(pb, fc, Pi, d);
    GSLS_LAUNCH_CHECK();
  }
  return GSLS_OK;
}

template int epoch_set_attributes<float>();
template int epoch_set_attributes<double>();
template int launch_epoch<float>(const DevProblem<float>&, const DevEpochWork<float>&, const DevFactor<float>&,
                                 double, int, int, int, hipStream_t);
template int launch_epoch<double>(const DevProblem<double>&, const DevEpochWork<double>&, const DevFactor<double>&,
                                  double, int, int, int, hipStream_t);

}  // namespace gsls
