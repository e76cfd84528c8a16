// Host side of the C ABI declared in include/gsls.h: argument validation,
// handle lifetime, device buffers, the rho / factor-epoch driver around the
// persistent ADMM iteration kernel, and the result struct.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <limits>
#include <type_traits>
#include <vector>

#include "dev_common.hpp"
#include "models.hpp"
#include "solver.hpp"

namespace gsls {

// ------------------------------------------------------------- allocation
struct DevArena {
  std::vector<void*> ptrs;
  bool ok = true;
  template <typename T>
  T* alloc(size_t n) {
    if (n == 0) n = 1;
    void* p = nullptr;
    if (hipMalloc(&p, n * sizeof(T)) != hipSuccess) { ok = false; return nullptr; }
    ptrs.push_back(p);
    return (T*)p;
  }
  ~DevArena() {
    for (void* p : ptrs) (void)hipFree(p);
  }
};

static int ceil_log2(int x) {
  int l = 0;
  while ((1 << l) < x) ++l;
  return l;
}

// Host-side view of a description with host pointers (device inputs are
// staged to host first).
struct HostDesc {
  int N, nx, nu, nc, nf, m;
  std::vector<double> A, B, b, Q, R, S, q, r, C, D, CN, l, u;
};

static bool finite_all(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

static int check_dims(const gsls_qp_desc* d, int max_rows = GSLS_MAX_NC) {
  if (!d) return GSLS_ERR_INVALID_ARG;
  if (d->N < 1 || d->N > GSLS_MAX_N || d->nx < 1 || d->nx > GSLS_MAX_NX || d->nu < 1 ||
      d->nu > GSLS_MAX_NU || d->nc < 0 || d->nc > max_rows || d->nf < 0 || d->nf > max_rows)
    return GSLS_ERR_DIM;
  if (d->mem != GSLS_HOST && d->mem != GSLS_DEVICE) return GSLS_ERR_INVALID_ARG;
  if (!d->A || !d->B || !d->Q || !d->R || !d->l || !d->u) return GSLS_ERR_INVALID_ARG;
  if (d->nc > 0 && (!d->C || !d->D)) return GSLS_ERR_INVALID_ARG;
  if (d->nf > 0 && !d->CN) return GSLS_ERR_INVALID_ARG;
  return GSLS_OK;
}

static int validate_host(const HostDesc& h) {
  const size_t N = h.N, nx = h.nx, nu = h.nu, nc = h.nc, nf = h.nf;
  if (!finite_all(h.A.data(), N * nx * nx) || !finite_all(h.B.data(), N * nx * nu) ||
      !finite_all(h.b.data(), N * nx) || !finite_all(h.Q.data(), (N + 1) * nx * nx) ||
      !finite_all(h.R.data(), N * nu * nu) || !finite_all(h.S.data(), N * nu * nx) ||
      !finite_all(h.q.data(), (N + 1) * nx) || !finite_all(h.r.data(), N * nu) ||
      !finite_all(h.C.data(), N * nc * nx) || !finite_all(h.D.data(), N * nc * nu) ||
      !finite_all(h.CN.data(), nf * nx))
    return GSLS_ERR_INVALID_ARG;
  for (size_t i = 0; i < h.l.size(); ++i) {
    if (std::isnan(h.l[i]) || std::isnan(h.u[i]) || h.l[i] > h.u[i] || h.l[i] == INFINITY ||
        h.u[i] == -INFINITY)
      return GSLS_ERR_INVALID_ARG;
  }
  return GSLS_OK;
}

static int stage_to_host(const gsls_qp_desc* d, HostDesc* h) {
  const size_t N = d->N, nx = d->nx, nu = d->nu, nc = d->nc, nf = d->nf;
  h->N = d->N; h->nx = d->nx; h->nu = d->nu; h->nc = d->nc; h->nf = d->nf;
  h->m = (int)(N * nc + nf);
  auto get = [&](std::vector<double>& v, const double* p, size_t n) -> int {
    v.assign(n, 0.0);
    if (!p || n == 0) return GSLS_OK;
    if (d->mem == GSLS_HOST) {
      std::memcpy(v.data(), p, n * sizeof(double));
    } else {
      if (hipMemcpy(v.data(), p, n * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) return GSLS_ERR_HIP;
    }
    return GSLS_OK;
  };
  int rc = GSLS_OK;
  if ((rc = get(h->A, d->A, N * nx * nx))) return rc;
  if ((rc = get(h->B, d->B, N * nx * nu))) return rc;
  if ((rc = get(h->b, d->b, N * nx))) return rc;
  if ((rc = get(h->Q, d->Q, (N + 1) * nx * nx))) return rc;
  if ((rc = get(h->R, d->R, N * nu * nu))) return rc;
  if ((rc = get(h->S, d->S, N * nu * nx))) return rc;
  if ((rc = get(h->q, d->q, (N + 1) * nx))) return rc;
  if ((rc = get(h->r, d->r, N * nu))) return rc;
  if ((rc = get(h->C, d->C, N * nc * nx))) return rc;
  if ((rc = get(h->D, d->D, N * nc * nu))) return rc;
  if ((rc = get(h->CN, d->CN, nf * nx))) return rc;
  if ((rc = get(h->l, d->l, N * nc + nf))) return rc;
  if ((rc = get(h->u, d->u, N * nc + nf))) return rc;
  return GSLS_OK;
}

// ------------------------------------------------------------ the solver
struct SolverBase {
  virtual ~SolverBase() {}
  virtual int solve(const double* x0, int x0_dev, double rho, double tol, const double* z0,
                    const double* y0, int warm_dev, gsls_result* res) = 0;
  virtual int get(double* X, double* U, double* z, double* lam) = 0;
  virtual int update_bounds(const double* l, const double* u, int dev) = 0;
  virtual int sls(const double* E, const double* tau, const double* Qb, const double* Rb,
                  const double* QbN, int rownorm, double wbound, double* Phx, double* Phu,
                  double* h, double* hf) = 0;
  virtual int sls_batch(int count, const double* E, const double* tau, const double* Qb,
                        const double* Rb, const double* QbN, int rownorm, double wbound, double* h,
                        double* hf, double* ms) = 0;
  virtual int phase_cycles(int enable, double* out, int* chunks) = 0;
  virtual int sls_tau(const double* lam, const double* Phx, const double* Phu, double eps, double* tau) = 0;
  virtual int robust(const double* x0, const double* E, const double* Qb, const double* Rb, const double* QbN,
                     int rownorm, double wbound, double eps, double rho, double tol, int max_passes, double htol,
                     gsls_robust_result* res, double* h, double* hf) = 0;
  virtual int update_data(const HostDesc& h) = 0;
};

template <typename T>
static void convert(std::vector<T>& out, const std::vector<double>& in) {
  out.resize(in.size());
  for (size_t i = 0; i < in.size(); ++i) out[i] = T(in[i]);
}

// batched transpose: [cnt][r][c] -> [cnt][c][r]
template <typename T>
static std::vector<T> transpose_blocks(const std::vector<double>& in, size_t cnt, size_t r, size_t c) {
  std::vector<T> out(cnt * r * c);
  for (size_t k = 0; k < cnt; ++k)
    for (size_t i = 0; i < r; ++i)
      for (size_t j = 0; j < c; ++j) out[k * r * c + j * r + i] = T(in[k * r * c + i * c + j]);
  return out;
}


template <typename T>
struct Solver : SolverBase {
  HostDesc hd;
  gsls_settings st;
  hipStream_t stream = nullptr;
  DevArena arena;
  DevProblem<T> pb{};
  DevFactor<T> fc{};
  DevEpochWork<T> ew{};
  double *z = nullptr, *y = nullptr, *ld_ = nullptr, *ud_ = nullptr;
  double *X = nullptr, *U = nullptr;
  T* x0d = nullptr;
  unsigned long long* prof = nullptr;
  int resident = 0;
  LLBufs ll{};
  IterCtl* ctl = nullptr;       // device
  IterCtl* ctl_h = nullptr;     // pinned host copy
  int* status_h = nullptr;      // pinned
  int Pe = 1, Pi = 1, nlev = 0, Lmax = 1;
  bool profile_on = false;
  uint32_t stamp = 1;
  double hnorm = 0.0;
  double last_rho = 1.0;
  bool solved_once = false;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  // one-wavefront path for tiny problems (auto chunking, nx, nu <= 4, rows <= 8, N <= 63):
  // FP64 copies of the problem and its result block
  bool tiny = false;
  TinyArgs ta{};
  TinyOut* tout = nullptr;      // device
  TinyOut* tout_h = nullptr;    // pinned
  double tiny_prof[16] = {};    // phase counters of the one-wavefront path (see phase_cycles)
  std::unique_ptr<SolverBase> fb;   // FP64 solver of the same problem (fp64_fallback), created on first use

  ~Solver() override {
    if (tout_h) (void)hipHostFree(tout_h);
    if (ctl_h) (void)hipHostFree(ctl_h);
    if (status_h) (void)hipHostFree(status_h);
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
  }

  template <typename U_>
  U_* up(const std::vector<U_>& v) {
    U_* p = arena.alloc<U_>(v.size());
    if (p && !v.empty()) {
      if (hipMemcpyAsync(p, v.data(), v.size() * sizeof(U_), hipMemcpyHostToDevice, stream) != hipSuccess)
        arena.ok = false;
    }
    return p;
  }

  // Iteration chunking: the workgroup count P (<= 256, all co-resident) and
  // whether each chunk's operators fit in LDS.
  void choose_chunks(const gsls_settings& s) {
    const int N = hd.N, nx = hd.nx, nu = hd.nu, nc = hd.nc;
    if (s.chunks_iter > 0) {
      Pi = std::min(s.chunks_iter, N);
    } else {
      // one stage per workgroup while the horizon fits the co-resident grid:
      // an iteration's critical path is the chunk-local stage chain (about ten
      // workgroup barriers per stage) plus a few cross-workgroup hops per
      // doubling level, and one extra level costs less than one extra stage
      Pi = N;
    }
    Pi = std::max(1, std::min(Pi, 256));
    Lmax = (N + Pi - 1) / Pi;
    if (Lmax > 64) { Pi = std::min(256, (N + 63) / 64); Lmax = (N + Pi - 1) / Pi; }
    nlev = ceil_log2(Pi);
    resident = admm_lds_bytes<T>(nx, nu, nc, hd.nf, Lmax, Pi, true) <= 156 * 1024 ? 1 : 0;
    Pe = s.chunks_epoch > 0 ? s.chunks_epoch : std::min(256, N);   // epoch: one stage per chunk too
    Pe = std::max(1, std::min(std::min(Pe, N), 256));
  }

  int init(const HostDesc& h, const gsls_settings& s, hipStream_t strm) {
    hd = h; st = s; stream = strm;
    const int N = h.N, nx = h.nx, nu = h.nu, nc = h.nc, nf = h.nf;
    const size_t xx = (size_t)nx * nx;
    choose_chunks(s);
    if (Lmax > 64) return GSLS_ERR_DIM;
    // a chunking whose per-workgroup state does not fit the local data share
    // (long chunks of wide stages) is refused here rather than at launch
    if (admm_lds_bytes<T>(nx, nu, nc, nf, Lmax, Pi, resident != 0) > 160 * 1024 - 512) return GSLS_ERR_DIM;
    // problem copies
    std::vector<T> tmp;
    pb.N = N; pb.nx = nx; pb.nu = nu; pb.nc = nc; pb.nf = nf; pb.m = h.m;
    convert(tmp, h.A); pb.A = up(tmp);
    convert(tmp, h.B); pb.B = up(tmp);
    convert(tmp, h.b); pb.b = up(tmp);
    convert(tmp, h.Q); pb.Q = up(tmp);
    convert(tmp, h.R); pb.R = up(tmp);
    convert(tmp, h.S); pb.S = up(tmp);
    convert(tmp, h.q); pb.q = up(tmp);
    convert(tmp, h.r); pb.r = up(tmp);
    convert(tmp, h.C); pb.C = up(tmp);
    convert(tmp, h.D); pb.D = up(tmp);
    convert(tmp, h.CN); pb.CN = up(tmp);
    {  // G = [C | D] per stage
      const int nxu = nx + nu;
      std::vector<T> G((size_t)N * nc * nxu);
      for (int k = 0; k < N; ++k)
        for (int r = 0; r < nc; ++r) {
          for (int j = 0; j < nx; ++j) G[((size_t)k * nc + r) * nxu + j] = T(h.C[((size_t)k * nc + r) * nx + j]);
          for (int j = 0; j < nu; ++j) G[((size_t)k * nc + r) * nxu + nx + j] = T(h.D[((size_t)k * nc + r) * nu + j]);
        }
      pb.G = up(G);
    }
    ld_ = up(h.l); ud_ = up(h.u);
    // factor outputs
    fc.F = arena.alloc<T>((size_t)N * (nx + nu) * (nx + nu));
    fc.Gam = arena.alloc<T>((size_t)N * nu * nu);
    fc.ev = arena.alloc<T>((size_t)N * nx); fc.fv = arena.alloc<T>((size_t)N * nu);
    fc.Phi = arena.alloc<T>((size_t)std::max(nlev, 1) * Pi * xx);
    // epoch scratch
    ew.eP = arena.alloc<T>((N + 1) * xx); ew.eA = arena.alloc<T>((N + 1) * xx); ew.eC = arena.alloc<T>((N + 1) * xx);
    ew.Qh = arena.alloc<T>((N + 1) * xx); ew.Rh = arena.alloc<T>((size_t)N * nu * nu);
    ew.Sh = arena.alloc<T>((size_t)N * nu * nx);
    ew.fP = arena.alloc<T>(Pe * xx); ew.fA = arena.alloc<T>(Pe * xx); ew.fC = arena.alloc<T>(Pe * xx);
    ew.gP = arena.alloc<T>(Pe * xx); ew.gA = arena.alloc<T>(Pe * xx); ew.gC = arena.alloc<T>(Pe * xx);
    ew.Pend = arena.alloc<T>(Pe * xx);
    ew.slot = (size_t)std::max(nx, nu) * std::max(nx, nu);
    ew.scratch = arena.alloc<T>((size_t)std::max(Pe, Pi) * 8 * ew.slot);
    ew.status = arena.alloc<int>(1);
    // state
    z = arena.alloc<double>(h.m); y = arena.alloc<double>(h.m);
    X = arena.alloc<double>((size_t)(N + 1) * nx); U = arena.alloc<double>((size_t)N * nu);
    prof = arena.alloc<unsigned long long>(16);
    x0d = arena.alloc<T>(nx);
    constexpr int W = LLWords<T>::n;
    const size_t vw = (size_t)(nlev + 1) * Pi * nx * W;
    ll.bwd = arena.alloc<unsigned long long>(vw);
    ll.fwd = arena.alloc<unsigned long long>(vw);
    ll.red = arena.alloc<unsigned long long>((size_t)Pi * kRed * 2);
    ll.abort = arena.alloc<int>(1);
    ctl = arena.alloc<IterCtl>(1);
    if (!arena.ok) return GSLS_ERR_OOM;
    if (hipMemsetAsync(ll.bwd, 0, vw * 8, stream) != hipSuccess) return GSLS_ERR_HIP;
    if (hipMemsetAsync(ll.fwd, 0, vw * 8, stream) != hipSuccess) return GSLS_ERR_HIP;
    if (hipMemsetAsync(ll.red, 0, (size_t)Pi * kRed * 2 * 8, stream) != hipSuccess) return GSLS_ERR_HIP;
    if (hipMemsetAsync(X, 0, sizeof(double) * (N + 1) * nx, stream) != hipSuccess) return GSLS_ERR_HIP;
    if (hipMemsetAsync(U, 0, sizeof(double) * N * nu, stream) != hipSuccess) return GSLS_ERR_HIP;
    if (hipMemsetAsync(prof, 0, sizeof(unsigned long long) * 16, stream) != hipSuccess) return GSLS_ERR_HIP;
    if (hipHostMalloc((void**)&ctl_h, sizeof(IterCtl)) != hipSuccess) return GSLS_ERR_OOM;
    if (hipHostMalloc((void**)&status_h, sizeof(int)) != hipSuccess) return GSLS_ERR_OOM;
    for (auto& e : ev)
      if (hipEventCreate(&e) != hipSuccess) return GSLS_ERR_HIP;
    double hn = 0.0;
    for (double v : h.q) hn = std::max(hn, std::fabs(v));
    for (double v : h.r) hn = std::max(hn, std::fabs(v));
    hnorm = hn;
    tiny = s.chunks_epoch == 0 && s.chunks_iter == 0 && tiny_fits(N, nx, nu, nc, nf);
    if (tiny) {
      ta.box = box_rows(h);
      ta.A = up(h.A); ta.B = up(h.B); ta.b = up(h.b); ta.Q = up(h.Q); ta.R = up(h.R); ta.S = up(h.S);
      ta.q = up(h.q); ta.r = up(h.r); ta.C = up(h.C); ta.D = up(h.D); ta.CN = up(h.CN);
      tout = arena.alloc<TinyOut>(1);
      if (!arena.ok) return GSLS_ERR_OOM;
      if (hipHostMalloc((void**)&tout_h, sizeof(TinyOut)) != hipSuccess) return GSLS_ERR_OOM;
    }
    if (epoch_set_attributes<T>() != GSLS_OK) return GSLS_ERR_HIP;
    if (hipStreamSynchronize(stream) != hipSuccess) return GSLS_ERR_HIP;
    return GSLS_OK;
  }

  int run_epoch(double rho, float* ms) {
    if (hipMemsetAsync(ew.status, 0, sizeof(int), stream) != hipSuccess) return GSLS_ERR_HIP;
    if (hipEventRecord(ev[0], stream) != hipSuccess) return GSLS_ERR_HIP;
    int rc = launch_epoch<T>(pb, ew, fc, rho, Pe, Pi, nlev, stream);
    if (rc) return rc;
    if (hipEventRecord(ev[1], stream) != hipSuccess) return GSLS_ERR_HIP;
    if (hipMemcpyAsync(status_h, ew.status, sizeof(int), hipMemcpyDeviceToHost, stream) != hipSuccess)
      return GSLS_ERR_HIP;
    if (hipStreamSynchronize(stream) != hipSuccess) return GSLS_ERR_HIP;
    if (*status_h != 0) return GSLS_ERR_NOT_PD;
    float t = 0.f;
    (void)hipEventElapsedTime(&t, ev[0], ev[1]);
    *ms += t;
    return GSLS_OK;
  }

  template <typename D_>
  int load_vec(D_* dst, const double* src, size_t n, int dev) {
    std::vector<double> hv(n);
    if (dev) {
      if (hipMemcpy(hv.data(), src, n * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) return GSLS_ERR_HIP;
    } else {
      std::memcpy(hv.data(), src, n * sizeof(double));
    }
    for (double v : hv)
      if (!std::isfinite(v)) return GSLS_ERR_INVALID_ARG;
    std::vector<D_> tv(n);
    for (size_t i = 0; i < n; ++i) tv[i] = D_(hv[i]);
    if (hipMemcpyAsync(dst, tv.data(), n * sizeof(D_), hipMemcpyHostToDevice, stream) != hipSuccess) return GSLS_ERR_HIP;
    if (hipStreamSynchronize(stream) != hipSuccess) return GSLS_ERR_HIP;
    return GSLS_OK;
  }

  // A solve, then the outcome's post-processing.  A solve that reaches the
  // iteration limit with the primal residual above tol after the rho rule has
  // raised rho to rho_max is reported as GSLS_INFEASIBLE_SUSPECTED: on an
  // infeasible QP r_p settles at the distance between the sets and the rule
  // keeps raising rho to its clamp.  Otherwise a mixed-precision solve that
  // reached the limit is continued in FP64 from its last iterate when
  // settings.fp64_fallback is set.
  int solve(const double* x0, int x0_dev, double rho, double tol, const double* z0, const double* y0,
            int warm_dev, gsls_result* res) override {
    gsls_result r{};
    int rc = solve_core(x0, x0_dev, rho, tol, z0, y0, warm_dev, &r);
    if (rc) return rc;
    auto suspect = [&](const gsls_result& q) {
      return q.status == GSLS_MAX_ITER && st.adaptive_rho && q.rho >= st.rho_max && q.r_p > tol;
    };
    if (!suspect(r) && r.status == GSLS_MAX_ITER && !std::is_same<T, double>::value && !tiny && st.fp64_fallback) {
      if ((rc = fallback_fp64(x0, x0_dev, tol, &r))) return rc;
    }
    if (suspect(r)) r.status = GSLS_INFEASIBLE_SUSPECTED;
    if (res) *res = r;
    return GSLS_OK;
  }

  // FP64 continuation of a stalled mixed-precision solve: an FP64 solver of the
  // same problem (created on first use), warm-started from the mixed iterate
  // (z, y at the final rho); its iterate replaces this handle's.
  int fallback_fp64(const double* x0, int x0_dev, double tol, gsls_result* r) {
    int rc;
    if (!fb) {
      gsls_settings s2 = st;
      s2.precision = GSLS_FP64;
      s2.fp64_fallback = 0;
      auto* p = new (std::nothrow) Solver<double>();
      if (!p) return GSLS_ERR_OOM;
      fb.reset(p);
      if ((rc = p->init(hd, s2, stream))) { fb.reset(); return rc; }
    }
    auto* f = static_cast<Solver<double>*>(fb.get());
    gsls_result r2{};
    if ((rc = f->solve_core(x0, x0_dev, r->rho, tol, z, y, 1, &r2))) return rc;
    const size_t N = hd.N, nx = hd.nx, nu = hd.nu, m = hd.m;
    if (hipMemcpyAsync(X, f->X, (N + 1) * nx * sizeof(double), hipMemcpyDeviceToDevice, stream) != hipSuccess ||
        (N * nu > 0 && hipMemcpyAsync(U, f->U, N * nu * sizeof(double), hipMemcpyDeviceToDevice, stream) != hipSuccess) ||
        (m > 0 && hipMemcpyAsync(z, f->z, m * sizeof(double), hipMemcpyDeviceToDevice, stream) != hipSuccess) ||
        (m > 0 && hipMemcpyAsync(y, f->y, m * sizeof(double), hipMemcpyDeviceToDevice, stream) != hipSuccess) ||
        hipStreamSynchronize(stream) != hipSuccess)
      return GSLS_ERR_HIP;
    last_rho = r2.rho;
    r->status = r2.status;
    r->iterations += r2.iterations; r->rho_updates += r2.rho_updates; r->factorizations += r2.factorizations;
    r->r_p = r2.r_p; r->r_d = r2.r_d; r->rho = r2.rho; r->r_dyn = r2.r_dyn;
    r->ms_total += r2.ms_total; r->ms_factor += r2.ms_factor; r->ms_iterate += r2.ms_iterate;
    r->fallback = 1;
    return GSLS_OK;
  }

  int solve_core(const double* x0, int x0_dev, double rho, double tol, const double* z0, const double* y0,
                 int warm_dev, gsls_result* res) {
    if (!x0 || !(rho > 0.0) || !std::isfinite(rho) || !(tol >= 0.0)) return GSLS_ERR_INVALID_ARG;
    int rc;
    if (tiny) return solve_tiny(x0, x0_dev, rho, tol, z0, y0, warm_dev, res);
    if ((rc = load_vec(x0d, x0, hd.nx, x0_dev))) return rc;
    if (z0 && y0) {
      if ((rc = load_vec(z, z0, hd.m, warm_dev))) return rc;
      if ((rc = load_vec(y, y0, hd.m, warm_dev))) return rc;
    } else {
      if (hipMemsetAsync(z, 0, sizeof(double) * hd.m, stream) != hipSuccess) return GSLS_ERR_HIP;
      if (hipMemsetAsync(y, 0, sizeof(double) * hd.m, stream) != hipSuccess) return GSLS_ERR_HIP;
    }
    float ms_f = 0.f, ms_i = 0.f;
    int it = 0, nfact = 0, nupd = 0;
    double cur = rho;
    gsls_result r{};
    while (true) {
      if ((rc = run_epoch(cur, &ms_f))) return rc;
      ++nfact;
      IterArgs<T> a{};
      a.pb = pb; a.fc = fc; a.z = z; a.y = y; a.l = ld_; a.u = ud_; a.X = X; a.U = U; a.x0 = x0d;
      a.ll = ll; a.ctl = ctl; a.Lmax = Lmax; a.resident = resident;
      a.prof = profile_on ? prof : nullptr;
      a.ip.P = Pi; a.ip.nlev = nlev; a.ip.rho = cur; a.ip.tol = tol; a.ip.it0 = it;
      a.ip.max_iter = st.max_iter; a.ip.adaptive = st.adaptive_rho; a.ip.sigma = st.sigma;
      a.ip.rho_min = st.rho_min; a.ip.rho_max = st.rho_max; a.ip.rho_tol = st.rho_tol;
      a.ip.hnorm = hnorm; a.ip.stamp0 = stamp; a.ip.refresh = st.refresh;
      if (hipMemsetAsync(ll.abort, 0, sizeof(int), stream) != hipSuccess) return GSLS_ERR_HIP;
      if (hipMemsetAsync(ctl, 0, sizeof(IterCtl), stream) != hipSuccess) return GSLS_ERR_HIP;
      if (hipEventRecord(ev[2], stream) != hipSuccess) return GSLS_ERR_HIP;
      if ((rc = launch_admm<T>(a, stream))) return rc;
      if (hipEventRecord(ev[3], stream) != hipSuccess) return GSLS_ERR_HIP;
      if ((rc = launch_rdyn<T>(pb, X, U, ctl, stream))) return rc;
      if (hipMemcpyAsync(ctl_h, ctl, sizeof(IterCtl), hipMemcpyDeviceToHost, stream) != hipSuccess) return GSLS_ERR_HIP;
      if (hipStreamSynchronize(stream) != hipSuccess) return GSLS_ERR_HIP;
      float t = 0.f;
      (void)hipEventElapsedTime(&t, ev[2], ev[3]);
      ms_i += t;
      stamp += (uint32_t)(ctl_h->it - it) + 2;
      it = ctl_h->it;
      r.r_p = ctl_h->r_p; r.r_d = ctl_h->r_d; r.r_dyn = ctl_h->r_dyn;
      const int s = ctl_h->status;
      if (s == 5) return GSLS_ERR_HIP;
      if (s == 4) {
        cur = ctl_h->rho_new;
        ++nupd;
        continue;
      }
      r.status = s == 1 ? GSLS_SOLVED : (s == 2 ? GSLS_MAX_ITER : GSLS_NUMERICAL_FAIL);
      break;
    }
    r.iterations = it; r.rho_updates = nupd; r.factorizations = nfact; r.rho = cur;
    r.ms_factor = ms_f; r.ms_iterate = ms_i; r.ms_total = ms_f + ms_i;
    last_rho = cur;
    solved_once = true;
    if (res) *res = r;
    return GSLS_OK;
  }

  // Rows exactly [I 0; 0 I] at every stage and I at the terminal stage.
  static int box_rows(const HostDesc& h) {
    const int nx = h.nx, nu = h.nu, nc = h.nc;
    if (nc != nx + nu || h.nf != nx) return 0;
    for (int k = 0; k < h.N; ++k)
      for (int r = 0; r < nc; ++r) {
        for (int j = 0; j < nx; ++j)
          if (h.C[((size_t)k * nc + r) * nx + j] != (r == j ? 1.0 : 0.0)) return 0;
        for (int j = 0; j < nu; ++j)
          if (h.D[((size_t)k * nc + r) * nu + j] != (r == nx + j ? 1.0 : 0.0)) return 0;
      }
    for (int r = 0; r < nx; ++r)
      for (int j = 0; j < nx; ++j)
        if (h.CN[(size_t)r * nx + j] != (r == j ? 1.0 : 0.0)) return 0;
    return 1;
  }

  // The whole solve in one launch of the one-wavefront kernel (FP64).
  int solve_tiny(const double* x0, int x0_dev, double rho, double tol, const double* z0, const double* y0,
                 int warm_dev, gsls_result* res) {
    int rc;
    TinyArgs a = ta;
    // x0 travels in the kernel arguments; a cold start is cleared in the kernel
    double xh[4] = {0.0, 0.0, 0.0, 0.0};
    if (x0_dev) {
      if (hipMemcpy(xh, x0, hd.nx * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) return GSLS_ERR_HIP;
    } else {
      std::memcpy(xh, x0, hd.nx * sizeof(double));
    }
    for (int j = 0; j < hd.nx; ++j) {
      if (!std::isfinite(xh[j])) return GSLS_ERR_INVALID_ARG;
      a.x0v[j] = xh[j];
    }
    a.cold = (z0 && y0) ? 0 : 1;
    if (!a.cold) {
      if ((rc = load_vec(z, z0, hd.m, warm_dev))) return rc;
      if ((rc = load_vec(y, y0, hd.m, warm_dev))) return rc;
    }
    a.N = hd.N; a.nx = hd.nx; a.nu = hd.nu; a.nc = hd.nc; a.nf = hd.nf;
    a.nlev = 1;
    while ((1 << a.nlev) <= hd.N) ++a.nlev;
    a.l = ld_; a.u = ud_; a.z = z; a.y = y; a.X = X; a.U = U;
    a.rho0 = rho; a.tol = tol; a.rho_min = st.rho_min; a.rho_max = st.rho_max; a.rho_tol = st.rho_tol;
    a.hnorm = hnorm; a.max_iter = st.max_iter; a.adaptive = st.adaptive_rho; a.sigma = st.sigma;
    a.out = tout;
    if (hipEventRecord(ev[0], stream) != hipSuccess) return GSLS_ERR_HIP;
    if ((rc = launch_tiny(a, stream))) return rc;
    if (hipEventRecord(ev[1], stream) != hipSuccess) return GSLS_ERR_HIP;
    if (hipMemcpyAsync(tout_h, tout, sizeof(TinyOut), hipMemcpyDeviceToHost, stream) != hipSuccess) return GSLS_ERR_HIP;
    if (hipStreamSynchronize(stream) != hipSuccess) return GSLS_ERR_HIP;
    const TinyOut o = *tout_h;
    if (profile_on) {
      tiny_prof[0] += 1.0;
      tiny_prof[1] += (double)o.c_load;
      tiny_prof[2] += (double)o.c_factor;
      tiny_prof[3] += (double)o.c_iter;
      tiny_prof[4] += (double)o.t_factor + (double)o.t_iter;
      tiny_prof[5] += (double)o.nfact;
      tiny_prof[6] += (double)o.it;
    }
    if (o.status == 6) return GSLS_ERR_NOT_PD;
    float t = 0.f;
    (void)hipEventElapsedTime(&t, ev[0], ev[1]);
    gsls_result r{};
    r.status = o.status == 1 ? GSLS_SOLVED : (o.status == 2 ? GSLS_MAX_ITER : GSLS_NUMERICAL_FAIL);
    r.iterations = o.it; r.rho_updates = o.nupd; r.factorizations = o.nfact;
    r.r_p = o.r_p; r.r_d = o.r_d; r.rho = o.rho; r.r_dyn = o.r_dyn;
    r.ms_total = t;
    r.ms_factor = (double)o.t_factor * 1e-5;   // 100 MHz counter -> ms
    r.ms_iterate = (double)o.t_iter * 1e-5;
    last_rho = o.rho;
    solved_once = true;
    if (res) *res = r;
    return GSLS_OK;
  }

  int get(double* Xo, double* Uo, double* zo, double* lo) override {
    if (!solved_once) return GSLS_ERR_STATE;
    auto dl = [&](double* out, auto* src, size_t n, double scale) -> int {
      if (!out) return GSLS_OK;
      using S_ = std::remove_pointer_t<decltype(src)>;
      std::vector<S_> t(n);
      if (hipMemcpyAsync(t.data(), src, n * sizeof(S_), hipMemcpyDeviceToHost, stream) != hipSuccess) return GSLS_ERR_HIP;
      if (hipStreamSynchronize(stream) != hipSuccess) return GSLS_ERR_HIP;
      for (size_t i = 0; i < n; ++i) out[i] = scale * double(t[i]);
      return GSLS_OK;
    };
    int rc;
    if ((rc = dl(Xo, X, (size_t)(hd.N + 1) * hd.nx, 1.0))) return rc;
    if ((rc = dl(Uo, U, (size_t)hd.N * hd.nu, 1.0))) return rc;
    if ((rc = dl(zo, z, hd.m, 1.0))) return rc;
    if ((rc = dl(lo, y, hd.m, last_rho))) return rc;
    return GSLS_OK;
  }

  // Replace every stage datum (same dimensions) in place: device copies,
  // G = [C | D], bounds and the host description; the SLS copies are
  // refreshed on their next use.
  int update_data(const HostDesc& h) override {
    fb.reset();
    if (h.N != hd.N || h.nx != hd.nx || h.nu != hd.nu || h.nc != hd.nc || h.nf != hd.nf) return GSLS_ERR_DIM;
    const int N = h.N, nx = h.nx, nu = h.nu, nc = h.nc, nxu = nx + nu;
    std::vector<std::vector<T>> keep;   // host sources of the asynchronous copies
    keep.reserve(16);
    bool ok = true;
    auto put = [&](T* dst, const std::vector<double>& src) {
      keep.emplace_back();
      convert(keep.back(), src);
      if (!keep.back().empty() &&
          hipMemcpyAsync(dst, keep.back().data(), keep.back().size() * sizeof(T), hipMemcpyHostToDevice, stream) !=
              hipSuccess)
        ok = false;
    };
    put(pb.A, h.A); put(pb.B, h.B); put(pb.b, h.b); put(pb.Q, h.Q); put(pb.R, h.R); put(pb.S, h.S);
    put(pb.q, h.q); put(pb.r, h.r); put(pb.C, h.C); put(pb.D, h.D); put(pb.CN, h.CN);
    keep.emplace_back((size_t)N * nc * nxu);
    std::vector<T>& G = keep.back();
    for (int k = 0; k < N; ++k)
      for (int r = 0; r < nc; ++r) {
        for (int j = 0; j < nx; ++j) G[((size_t)k * nc + r) * nxu + j] = T(h.C[((size_t)k * nc + r) * nx + j]);
        for (int j = 0; j < nu; ++j) G[((size_t)k * nc + r) * nxu + nx + j] = T(h.D[((size_t)k * nc + r) * nu + j]);
      }
    if (!G.empty() && hipMemcpyAsync(pb.G, G.data(), G.size() * sizeof(T), hipMemcpyHostToDevice, stream) != hipSuccess)
      ok = false;
    if (h.m > 0) {
      if (hipMemcpyAsync(ld_, h.l.data(), h.m * sizeof(double), hipMemcpyHostToDevice, stream) != hipSuccess) ok = false;
      if (hipMemcpyAsync(ud_, h.u.data(), h.m * sizeof(double), hipMemcpyHostToDevice, stream) != hipSuccess) ok = false;
    }
    if (tiny) {   // the one-wavefront path's FP64 copies
      auto putd = [&](const double* dst, const std::vector<double>& src) {
        if (!src.empty() && hipMemcpyAsync(const_cast<double*>(dst), src.data(), src.size() * sizeof(double),
                                           hipMemcpyHostToDevice, stream) != hipSuccess)
          ok = false;
      };
      putd(ta.A, h.A); putd(ta.B, h.B); putd(ta.b, h.b); putd(ta.Q, h.Q); putd(ta.R, h.R); putd(ta.S, h.S);
      putd(ta.q, h.q); putd(ta.r, h.r); putd(ta.C, h.C); putd(ta.D, h.D); putd(ta.CN, h.CN);
      ta.box = box_rows(h);
    }
    if (hipStreamSynchronize(stream) != hipSuccess || !ok) return GSLS_ERR_HIP;
    hd = h;
    double hn = 0.0;
    for (double v : h.q) hn = std::max(hn, std::fabs(v));
    for (double v : h.r) hn = std::max(hn, std::fabs(v));
    hnorm = hn;
    sls_dirty = true;
    return GSLS_OK;
  }

  int update_bounds(const double* l, const double* u, int dev) override {
    fb.reset();
    if (!l || !u) return GSLS_ERR_INVALID_ARG;
    std::vector<double> lh(hd.m), uh(hd.m);
    if (dev) {
      if (hipMemcpy(lh.data(), l, hd.m * 8, hipMemcpyDeviceToHost) != hipSuccess) return GSLS_ERR_HIP;
      if (hipMemcpy(uh.data(), u, hd.m * 8, hipMemcpyDeviceToHost) != hipSuccess) return GSLS_ERR_HIP;
    } else {
      std::memcpy(lh.data(), l, hd.m * 8);
      std::memcpy(uh.data(), u, hd.m * 8);
    }
    for (int i = 0; i < hd.m; ++i)
      if (std::isnan(lh[i]) || std::isnan(uh[i]) || lh[i] > uh[i]) return GSLS_ERR_INVALID_ARG;
    hd.l = lh; hd.u = uh;
    if (hipMemcpyAsync(ld_, lh.data(), hd.m * sizeof(double), hipMemcpyHostToDevice, stream) != hipSuccess) return GSLS_ERR_HIP;
    if (hipMemcpyAsync(ud_, uh.data(), hd.m * sizeof(double), hipMemcpyHostToDevice, stream) != hipSuccess) return GSLS_ERR_HIP;
    if (hipStreamSynchronize(stream) != hipSuccess) return GSLS_ERR_HIP;
    return GSLS_OK;
  }

  int phase_cycles(int enable, double* out, int* chunks) override {
    if (enable >= 0) profile_on = enable != 0;
    if (chunks) {
      if (tiny) { chunks[0] = 1; chunks[1] = 1; chunks[2] = 1; chunks[3] = hd.N; }
      else { chunks[0] = Pe; chunks[1] = Pi; chunks[2] = resident; chunks[3] = Lmax; }
    }
    if (out && tiny) {
      for (int i = 0; i < 16; ++i) { out[i] = tiny_prof[i]; tiny_prof[i] = 0.0; }
      return GSLS_OK;
    }
    if (out) {
      unsigned long long h[16];
      if (hipMemcpy(h, prof, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) return GSLS_ERR_HIP;
      for (int i = 0; i < 16; ++i) out[i] = (double)h[i];
      if (hipMemset(prof, 0, sizeof(h)) != hipSuccess) return GSLS_ERR_HIP;
    }
    return GSLS_OK;
  }

  // ------------------------------------------------------------ SLS
  struct SlsBuf {
    bool ready = false;
    int grid = 0, cap = 0;                  // work-queue grid, instance capacity
    float *A = nullptr, *B = nullptr, *G = nullptr, *CN = nullptr;
    float *E = nullptr, *Qb = nullptr, *Rb = nullptr, *QbN = nullptr;
    float *tau = nullptr, *Kst = nullptr, *hj = nullptr, *hfj = nullptr, *Phx = nullptr, *Phu = nullptr;
    double *h = nullptr, *hf = nullptr, *lam = nullptr, *taud = nullptr;
    unsigned* counter = nullptr;
    int* status = nullptr;
  } sb;
  DevArena sls_arena;
  bool sls_dirty = false;   // stage data replaced since the SLS copies were made

  int sls_prepare(int count) {
    const int N = hd.N, nx = hd.nx, nu = hd.nu, nc = hd.nc, nf = hd.nf, nxu = nx + nu;
    auto cvt = [&](const std::vector<double>& v) {
      std::vector<float> t(v.size());
      for (size_t i = 0; i < v.size(); ++i) t[i] = (float)v[i];
      return t;
    };
    auto upf = [&](const std::vector<float>& v) {
      float* p = sls_arena.alloc<float>(v.size());
      if (p && hipMemcpyAsync(p, v.data(), v.size() * 4, hipMemcpyHostToDevice, stream) != hipSuccess)
        sls_arena.ok = false;
      return p;
    };
    auto stage_floats = [&]() {
      std::vector<float> G((size_t)N * nc * nxu);
      for (int k = 0; k < N; ++k)
        for (int r = 0; r < nc; ++r) {
          for (int j = 0; j < nx; ++j) G[((size_t)k * nc + r) * nxu + j] = (float)hd.C[((size_t)k * nc + r) * nx + j];
          for (int j = 0; j < nu; ++j) G[((size_t)k * nc + r) * nxu + nx + j] = (float)hd.D[((size_t)k * nc + r) * nu + j];
        }
      return G;
    };
    if (sb.ready && sls_dirty) {   // same shapes: refresh the copies in place
      const std::vector<float> A = cvt(hd.A), B = cvt(hd.B), G = stage_floats(), CN = cvt(hd.CN);
      bool ok = hipMemcpy(sb.A, A.data(), A.size() * 4, hipMemcpyHostToDevice) == hipSuccess &&
                hipMemcpy(sb.B, B.data(), B.size() * 4, hipMemcpyHostToDevice) == hipSuccess &&
                (G.empty() || hipMemcpy(sb.G, G.data(), G.size() * 4, hipMemcpyHostToDevice) == hipSuccess) &&
                (CN.empty() || hipMemcpy(sb.CN, CN.data(), CN.size() * 4, hipMemcpyHostToDevice) == hipSuccess);
      if (!ok) return GSLS_ERR_HIP;
    }
    sls_dirty = false;
    if (!sb.ready) {
      sb.A = upf(cvt(hd.A));
      sb.B = upf(cvt(hd.B));
      sb.G = upf(stage_floats());
      sb.CN = upf(cvt(hd.CN));
      sb.E = sls_arena.alloc<float>((size_t)N * nx * nx);
      sb.Qb = sls_arena.alloc<float>((size_t)nx * nx);
      sb.Rb = sls_arena.alloc<float>((size_t)nu * nu);
      sb.QbN = sls_arena.alloc<float>((size_t)nx * nx);
      sb.grid = sls_grid(nx, nu, nc, nf);
      if (sb.grid <= 0) return GSLS_ERR_HIP;
      sb.Kst = sls_arena.alloc<float>((size_t)sb.grid * N * nu * nx);
      sb.Phx = sls_arena.alloc<float>((size_t)N * (N + 1) / 2 * nx * nx);
      sb.Phu = sls_arena.alloc<float>((size_t)std::max(1, N * (N - 1) / 2) * nu * nx);
      sb.lam = sls_arena.alloc<double>((size_t)hd.m);
      sb.taud = sls_arena.alloc<double>((size_t)N * N * nc + (size_t)N * nf);
      sb.counter = sls_arena.alloc<unsigned>(1);
      sb.status = sls_arena.alloc<int>(1);
      if (!sls_arena.ok) return GSLS_ERR_OOM;
      sb.ready = true;
    }
    if (count > sb.cap) {
      const size_t ts = (size_t)N * N * nc + (size_t)N * nf;
      sb.tau = sls_arena.alloc<float>((size_t)count * ts);
      sb.hj = sls_arena.alloc<float>((size_t)count * N * N * nc);
      sb.hfj = sls_arena.alloc<float>((size_t)count * N * std::max(nf, 1));
      sb.h = sls_arena.alloc<double>((size_t)count * N * std::max(nc, 1));
      sb.hf = sls_arena.alloc<double>((size_t)count * std::max(nf, 1));
      if (!sls_arena.ok) return GSLS_ERR_OOM;
      sb.cap = count;
    }
    return GSLS_OK;
  }

  int sls_common(int count, const double* E, const double* tau, const double* Qb, const double* Rb,
                 const double* QbN, int rownorm, double wbound, bool want_phi, float* ms) {
    const int N = hd.N, nx = hd.nx, nu = hd.nu, nc = hd.nc, nf = hd.nf;
    if (!E || !Qb || !Rb || !QbN || count < 1) return GSLS_ERR_INVALID_ARG;
    if (rownorm != 1 && rownorm != 2) return GSLS_ERR_INVALID_ARG;
    if (!std::isfinite(wbound) || wbound < 0) return GSLS_ERR_INVALID_ARG;
    int rc;
    if ((rc = sls_prepare(count))) return rc;
    const size_t ts = (size_t)N * N * nc + (size_t)N * nf;
    auto h2d = [&](float* dst, const double* src, size_t n) -> int {
      std::vector<float> t(n);
      for (size_t i = 0; i < n; ++i) {
        if (!std::isfinite(src[i])) return GSLS_ERR_INVALID_ARG;
        t[i] = (float)src[i];
      }
      if (hipMemcpyAsync(dst, t.data(), n * 4, hipMemcpyHostToDevice, stream) != hipSuccess) return GSLS_ERR_HIP;
      return hipStreamSynchronize(stream) == hipSuccess ? GSLS_OK : GSLS_ERR_HIP;
    };
    if ((rc = h2d(sb.E, E, (size_t)N * nx * nx))) return rc;
    if ((rc = h2d(sb.Qb, Qb, (size_t)nx * nx))) return rc;
    if ((rc = h2d(sb.Rb, Rb, (size_t)nu * nu))) return rc;
    if ((rc = h2d(sb.QbN, QbN, (size_t)nx * nx))) return rc;
    if (tau) {
      if ((rc = h2d(sb.tau, tau, (size_t)count * ts))) return rc;
    } else if (hipMemsetAsync(sb.tau, 0, (size_t)count * ts * 4, stream) != hipSuccess) {
      return GSLS_ERR_HIP;
    }
    if (hipMemsetAsync(sb.counter, 0, 4, stream) != hipSuccess) return GSLS_ERR_HIP;
    if (hipMemsetAsync(sb.status, 0, 4, stream) != hipSuccess) return GSLS_ERR_HIP;
    SlsArgs sa{};
    sa.N = N; sa.nx = nx; sa.nu = nu; sa.nc = nc; sa.nf = nf; sa.count = count;
    sa.A = sb.A; sa.B = sb.B; sa.G = sb.G; sa.CN = sb.CN; sa.E = sb.E; sa.tau = sb.tau;
    sa.Qb = sb.Qb; sa.Rb = sb.Rb; sa.QbN = sb.QbN; sa.rownorm = rownorm; sa.squared = 0;
    sa.Kst = sb.Kst; sa.hj = sb.hj; sa.hfj = sb.hfj;
    sa.Phx = want_phi ? sb.Phx : nullptr; sa.Phu = want_phi ? sb.Phu : nullptr;
    sa.counter = sb.counter; sa.status = sb.status;
    if (hipEventRecord(ev[0], stream) != hipSuccess) return GSLS_ERR_HIP;
    if ((rc = launch_sls(sa, sb.grid, stream))) return rc;
    if ((rc = launch_sls_sum(N, nc, nf, count, (float)wbound, sb.hj, sb.hfj, sb.h, sb.hf, stream))) return rc;
    if (hipEventRecord(ev[1], stream) != hipSuccess) return GSLS_ERR_HIP;
    if (hipMemcpyAsync(status_h, sb.status, sizeof(int), hipMemcpyDeviceToHost, stream) != hipSuccess)
      return GSLS_ERR_HIP;
    if (hipStreamSynchronize(stream) != hipSuccess) return GSLS_ERR_HIP;
    if (*status_h) return GSLS_ERR_NOT_PD;
    if (ms) (void)hipEventElapsedTime(ms, ev[0], ev[1]);
    return GSLS_OK;
  }

  int d2h(double* dst, const double* src, size_t n) {
    if (!dst || n == 0) return GSLS_OK;
    return hipMemcpy(dst, src, n * sizeof(double), hipMemcpyDeviceToHost) == hipSuccess ? GSLS_OK : GSLS_ERR_HIP;
  }
  int d2h_f(double* dst, const float* src, size_t n) {
    if (!dst || n == 0) return GSLS_OK;
    std::vector<float> t(n);
    if (hipMemcpy(t.data(), src, n * 4, hipMemcpyDeviceToHost) != hipSuccess) return GSLS_ERR_HIP;
    for (size_t i = 0; i < n; ++i) dst[i] = t[i];
    return GSLS_OK;
  }

  int sls(const double* E, const double* tau, const double* Qb, const double* Rb, const double* QbN,
          int rownorm, double wbound, double* Phx, double* Phu, double* h, double* hf) override {
    const int N = hd.N, nx = hd.nx, nu = hd.nu, nc = hd.nc, nf = hd.nf;
    int rc = sls_common(1, E, tau, Qb, Rb, QbN, rownorm, wbound, Phx || Phu, nullptr);
    if (rc) return rc;
    if ((rc = d2h_f(Phx, sb.Phx, (size_t)N * (N + 1) / 2 * nx * nx))) return rc;
    if ((rc = d2h_f(Phu, sb.Phu, (size_t)N * (N - 1) / 2 * nu * nx))) return rc;
    if ((rc = d2h(h, sb.h, (size_t)N * nc))) return rc;
    if ((rc = d2h(hf, sb.hf, (size_t)nf))) return rc;
    return GSLS_OK;
  }

  int sls_batch(int count, const double* E, const double* tau, const double* Qb, const double* Rb,
                const double* QbN, int rownorm, double wbound, double* h, double* hf, double* ms) override {
    const int N = hd.N, nc = hd.nc, nf = hd.nf;
    float t = 0.f;
    int rc = sls_common(count, E, tau, Qb, Rb, QbN, rownorm, wbound, false, &t);
    if (rc) return rc;
    if (ms) *ms = t;
    if ((rc = d2h(h, sb.h, (size_t)count * N * nc))) return rc;
    if ((rc = d2h(hf, sb.hf, (size_t)count * nf))) return rc;
    return GSLS_OK;
  }

  int sls_tau(const double* lam, const double* Phx, const double* Phu, double eps, double* tau) override {
    const int N = hd.N, nx = hd.nx, nu = hd.nu, nc = hd.nc, nf = hd.nf;
    if (!lam || !Phx || !tau || (N > 1 && !Phu) || !(eps > 0.0)) return GSLS_ERR_INVALID_ARG;
    int rc;
    if ((rc = sls_prepare(1))) return rc;
    auto h2d = [&](float* dst, const double* src, size_t n) -> int {
      std::vector<float> t(n);
      for (size_t i = 0; i < n; ++i) t[i] = (float)src[i];
      return hipMemcpy(dst, t.data(), n * 4, hipMemcpyHostToDevice) == hipSuccess ? GSLS_OK : GSLS_ERR_HIP;
    };
    if ((rc = h2d(sb.Phx, Phx, (size_t)N * (N + 1) / 2 * nx * nx))) return rc;
    if (N > 1 && (rc = h2d(sb.Phu, Phu, (size_t)N * (N - 1) / 2 * nu * nx))) return rc;
    if (hipMemcpy(sb.lam, lam, (size_t)hd.m * 8, hipMemcpyHostToDevice) != hipSuccess) return GSLS_ERR_HIP;
    SlsArgs sa{};
    sa.N = N; sa.nx = nx; sa.nu = nu; sa.nc = nc; sa.nf = nf; sa.count = 1;
    sa.G = sb.G; sa.CN = sb.CN; sa.Phx = sb.Phx; sa.Phu = sb.Phu; sa.hj = sb.hj; sa.hfj = sb.hfj;
    if ((rc = launch_sls_beta(sa, stream))) return rc;
    if ((rc = launch_sls_tau(N, nc, nf, sb.hj, sb.hfj, sb.lam, eps, sb.taud, stream))) return rc;
    if (hipStreamSynchronize(stream) != hipSuccess) return GSLS_ERR_HIP;
    return d2h(tau, sb.taud, (size_t)N * N * nc + (size_t)N * nf);
  }

  // App. B weights from the multipliers lam (host) and the responses that the
  // last sls_common(want_phi) left in device memory; tau to host.
  int tau_from_last_phi(const double* lam, double eps, double* tau, float* ms) {
    const int N = hd.N, nc = hd.nc, nf = hd.nf;
    if (hipMemcpyAsync(sb.lam, lam, (size_t)hd.m * 8, hipMemcpyHostToDevice, stream) != hipSuccess) return GSLS_ERR_HIP;
    SlsArgs sa{};
    sa.N = N; sa.nx = hd.nx; sa.nu = hd.nu; sa.nc = nc; sa.nf = nf; sa.count = 1;
    sa.G = sb.G; sa.CN = sb.CN; sa.Phx = sb.Phx; sa.Phu = sb.Phu; sa.hj = sb.hj; sa.hfj = sb.hfj;
    int rc;
    if (hipEventRecord(ev[0], stream) != hipSuccess) return GSLS_ERR_HIP;
    if ((rc = launch_sls_beta(sa, stream))) return rc;
    if ((rc = launch_sls_tau(N, nc, nf, sb.hj, sb.hfj, sb.lam, eps, sb.taud, stream))) return rc;
    if (hipEventRecord(ev[1], stream) != hipSuccess) return GSLS_ERR_HIP;
    if (hipStreamSynchronize(stream) != hipSuccess) return GSLS_ERR_HIP;
    if (ms) (void)hipEventElapsedTime(ms, ev[0], ev[1]);
    return d2h(tau, sb.taud, (size_t)N * N * nc + (size_t)N * nf);
  }

  // The alternation of Sec. III-D (see gsls_robust_solve in gsls.h).
  int robust(const double* x0, const double* E, const double* Qb, const double* Rb, const double* QbN,
             int rownorm, double wbound, double eps, double rho, double tol, int max_passes, double htol,
             gsls_robust_result* res, double* hout, double* hfout) override {
    const int N = hd.N, nc = hd.nc, nf = hd.nf, m = hd.m;
    if (!x0 || max_passes < 0 || !(htol >= 0.0) || !(eps > 0.0) || !(rho > 0.0) || !(tol >= 0.0))
      return GSLS_ERR_INVALID_ARG;
    const size_t ts = (size_t)N * N * nc + (size_t)N * nf;
    const std::vector<double> l0 = hd.l, u0 = hd.u;
    std::vector<double> hrow(m), hnew(m), lt(m), ut(m), lam(m), tau(ts);
    gsls_robust_result out{};
    auto read_h = [&](std::vector<double>& dst) -> int {
      int e = d2h(dst.data(), sb.h, (size_t)N * nc);
      return e ? e : d2h(dst.data() + (size_t)N * nc, sb.hf, (size_t)nf);
    };
    float t = 0.f;
    int rc = sls_common(1, E, nullptr, Qb, Rb, QbN, rownorm, wbound, true, &t);   // tau = 0
    if (rc || (rc = read_h(hrow))) return rc;
    out.ms_controller += t;
    double change = std::numeric_limits<double>::infinity();
    int status = GSLS_ROBUST_PASS_LIMIT;
    while (true) {
      bool cross = false;
      for (int i = 0; i < m; ++i) {
        lt[i] = std::isfinite(l0[i]) ? l0[i] + hrow[i] : l0[i];
        ut[i] = std::isfinite(u0[i]) ? u0[i] - hrow[i] : u0[i];
        cross = cross || lt[i] > ut[i];
      }
      if (cross) { status = GSLS_ROBUST_INFEASIBLE; break; }
      if ((rc = update_bounds(lt.data(), ut.data(), 0))) break;
      gsls_result r{};
      if ((rc = solve(x0, 0, rho, tol, nullptr, nullptr, 0, &r))) break;
      ++out.qp_solves;
      out.qp_iterations += r.iterations;
      out.qp_status = r.status;
      out.ms_nominal += r.ms_total;
      if (r.status != GSLS_SOLVED) { status = GSLS_ROBUST_NOMINAL_FAILED; break; }
      if (status == GSLS_ROBUST_CONVERGED || out.passes >= max_passes) break;
      if ((rc = get(nullptr, nullptr, nullptr, lam.data()))) break;
      if ((rc = tau_from_last_phi(lam.data(), eps, tau.data(), &t))) break;
      out.ms_controller += t;
      if ((rc = sls_common(1, E, tau.data(), Qb, Rb, QbN, rownorm, wbound, true, &t))) break;
      out.ms_controller += t;
      if ((rc = read_h(hnew))) break;
      change = 0.0;
      double hmax = 0.0;
      for (int i = 0; i < m; ++i) {
        change = std::max(change, std::fabs(hnew[i] - hrow[i]));
        hmax = std::max(hmax, std::fabs(hnew[i]));
      }
      hrow.swap(hnew);
      ++out.passes;
      if (change <= htol * std::max(1.0, hmax)) status = GSLS_ROBUST_CONVERGED;
    }
    const int rc_restore = update_bounds(l0.data(), u0.data(), 0);
    if (rc) return rc;
    if (rc_restore) return rc_restore;
    out.status = status;
    out.h_change = change;
    if (hout) std::copy(hrow.begin(), hrow.begin() + (size_t)N * nc, hout);
    if (hfout) std::copy(hrow.begin() + (size_t)N * nc, hrow.end(), hfout);
    if (res) *res = out;
    return GSLS_OK;
  }
};

}  // namespace gsls

// ================================================================ C ABI
struct gsls_qp {
  std::unique_ptr<gsls::SolverBase> impl;
  int mem;
};

extern "C" {

void gsls_default_settings(gsls_settings* s) {
  if (!s) return;
  s->precision = GSLS_MIXED;
  s->max_iter = 10000;
  s->adaptive_rho = 1;
  s->sigma = 25;
  s->rho_min = 1e-6;
  s->rho_max = 1e6;
  s->rho_tol = 5.0;
  s->chunks_epoch = 0;
  s->chunks_iter = 0;
  s->refresh = 0;
  s->fp64_fallback = 0;
}

const char* gsls_strerror(int code) {
  switch (code) {
    case GSLS_OK: return "ok";
    case GSLS_ERR_INVALID_ARG: return "invalid argument";
    case GSLS_ERR_DIM: return "dimension out of the supported range";
    case GSLS_ERR_NOT_PD: return "matrix not positive definite";
    case GSLS_ERR_NUMERICAL: return "numerical failure (NaN/Inf)";
    case GSLS_ERR_OOM: return "device allocation failed";
    case GSLS_ERR_HIP: return "HIP runtime error";
    case GSLS_ERR_STATE: return "call out of order";
    default: return "unknown error";
  }
}

}  // extern "C"

namespace gsls {
int check_settings(const gsls_settings* s) {
  if (s->precision != GSLS_MIXED && s->precision != GSLS_FP64) return GSLS_ERR_INVALID_ARG;
  if (s->max_iter < 1 || s->sigma < 1 || !(s->rho_min > 0) || !(s->rho_max >= s->rho_min) ||
      !(s->rho_tol > 1.0) || s->chunks_epoch < 0 || s->chunks_iter < 0 || s->chunks_iter > 256 || s->refresh < 0 ||
      (s->fp64_fallback != 0 && s->fp64_fallback != 1))
    return GSLS_ERR_INVALID_ARG;
  return GSLS_OK;
}

int validate_host_desc(const gsls_qp_desc* desc, int max_rows) {
  int rc = check_dims(desc, max_rows);
  if (rc) return rc;
  if (desc->mem != GSLS_HOST) return GSLS_ERR_INVALID_ARG;
  HostDesc h;
  if ((rc = stage_to_host(desc, &h))) return rc;
  return validate_host(h);
}
}  // namespace gsls

extern "C" {

int gsls_validate_desc(const gsls_qp_desc* desc) {
  int rc = gsls::check_dims(desc);
  if (rc) return rc;
  if (desc->mem != GSLS_HOST) return GSLS_ERR_INVALID_ARG;
  gsls::HostDesc h;
  if ((rc = gsls::stage_to_host(desc, &h))) return rc;
  return gsls::validate_host(h);
}

int gsls_qp_setup(const gsls_qp_desc* desc, const gsls_settings* settings, void* stream, gsls_qp** out) {
  if (!out) return GSLS_ERR_INVALID_ARG;
  *out = nullptr;
  int rc = gsls::check_dims(desc);
  if (rc) return rc;
  gsls_settings s;
  gsls_default_settings(&s);
  if (settings) s = *settings;
  if ((rc = gsls::check_settings(&s))) return rc;
  gsls::HostDesc h;
  if ((rc = gsls::stage_to_host(desc, &h))) return rc;
  if ((rc = gsls::validate_host(h))) return rc;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return GSLS_ERR_HIP;
  gsls_qp* q = new (std::nothrow) gsls_qp;
  if (!q) return GSLS_ERR_OOM;
  q->mem = desc->mem;
  try {
    if (s.precision == GSLS_FP64) {
      auto* p = new gsls::Solver<double>();
      q->impl.reset(p);
      rc = p->init(h, s, (hipStream_t)stream);
    } else {
      auto* p = new gsls::Solver<float>();
      q->impl.reset(p);
      rc = p->init(h, s, (hipStream_t)stream);
    }
  } catch (...) {
    rc = GSLS_ERR_OOM;
  }
  if (rc) {
    delete q;
    return rc;
  }
  *out = q;
  return GSLS_OK;
}

int gsls_qp_update_bounds(gsls_qp* h, const double* l, const double* u) {
  if (!h) return GSLS_ERR_INVALID_ARG;
  return h->impl->update_bounds(l, u, h->mem == GSLS_DEVICE);
}

int gsls_qp_update_data(gsls_qp* h, const gsls_qp_desc* desc) {
  if (!h) return GSLS_ERR_INVALID_ARG;
  int rc = gsls::check_dims(desc);
  if (rc) return rc;
  gsls::HostDesc hd;
  if ((rc = gsls::stage_to_host(desc, &hd))) return rc;
  if ((rc = gsls::validate_host(hd))) return rc;
  return h->impl->update_data(hd);
}

int gsls_qp_solve(gsls_qp* h, const double* x0, double rho, double tol, gsls_result* result) {
  if (!h) return GSLS_ERR_INVALID_ARG;
  return h->impl->solve(x0, h->mem == GSLS_DEVICE, rho, tol, nullptr, nullptr, 0, result);
}

int gsls_qp_solve_warm(gsls_qp* h, const double* x0, double rho, double tol, const double* z0,
                       const double* y0, gsls_result* result) {
  if (!h || !z0 || !y0) return GSLS_ERR_INVALID_ARG;
  return h->impl->solve(x0, h->mem == GSLS_DEVICE, rho, tol, z0, y0, h->mem == GSLS_DEVICE, result);
}

int gsls_qp_get(gsls_qp* h, double* X, double* U, double* z, double* lambda) {
  if (!h) return GSLS_ERR_INVALID_ARG;
  return h->impl->get(X, U, z, lambda);
}

void gsls_qp_free(gsls_qp* h) { delete h; }

int gsls_debug_phase_cycles(gsls_qp* h, int32_t enable, double* cycles16, int32_t* layout4) {
  if (!h) return GSLS_ERR_INVALID_ARG;
  return h->impl->phase_cycles(enable, cycles16, layout4);
}

int gsls_sls_solve(gsls_qp* h, const double* E, const double* tau, const double* Qbar, const double* Rbar,
                   const double* QbarN, int32_t rownorm, double wbound, double* Phi_x, double* Phi_u,
                   double* hmarg, double* hf) {
  if (!h) return GSLS_ERR_INVALID_ARG;
  return h->impl->sls(E, tau, Qbar, Rbar, QbarN, rownorm, wbound, Phi_x, Phi_u, hmarg, hf);
}

int gsls_sls_solve_batch(gsls_qp* h, int32_t count, const double* E, const double* tau, const double* Qbar,
                         const double* Rbar, const double* QbarN, int32_t rownorm, double wbound, double* hmarg,
                         double* hf, double* ms) {
  if (!h) return GSLS_ERR_INVALID_ARG;
  return h->impl->sls_batch(count, E, tau, Qbar, Rbar, QbarN, rownorm, wbound, hmarg, hf, ms);
}

int gsls_sls_tau(gsls_qp* h, const double* lambda, const double* Phi_x, const double* Phi_u, double eps,
                 double* tau) {
  if (!h) return GSLS_ERR_INVALID_ARG;
  return h->impl->sls_tau(lambda, Phi_x, Phi_u, eps, tau);
}

int gsls_robust_solve(gsls_qp* h, const double* x0, const double* E, const double* Qbar, const double* Rbar,
                      const double* QbarN, int32_t rownorm, double wbound, double eps, double rho, double tol,
                      int32_t max_passes, double htol, gsls_robust_result* result, double* hmarg, double* hf) {
  if (!h) return GSLS_ERR_INVALID_ARG;
  return h->impl->robust(x0, E, Qbar, Rbar, QbarN, rownorm, wbound, eps, rho, tol, max_passes, htol, result,
                         hmarg, hf);
}

}  // extern "C"

// ===================================================== analytic models: SQP
namespace gsls {

struct SqpState {
  int N = 0, nx = 0, nu = 0, no = 0, nc = 0, nf = 0, m = 0;
  hipStream_t stream = nullptr;
  DevArena arena;
  ModelDev md{};
  double *Xd = nullptr, *Ud = nullptr;
  LinOut lo{};
  gsls_qp* qp = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  ~SqpState() {
    if (qp) gsls_qp_free(qp);
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
  }
  gsls_qp_desc desc(int mem, const HostDesc* h) const {
    gsls_qp_desc d{};
    d.N = N; d.nx = nx; d.nu = nu; d.nc = nc; d.nf = nf; d.mem = mem;
    if (h) {
      d.A = h->A.data(); d.B = h->B.data(); d.b = h->b.data(); d.Q = h->Q.data(); d.R = h->R.data();
      d.S = h->S.data(); d.q = h->q.data(); d.r = h->r.data(); d.C = h->C.data(); d.D = h->D.data();
      d.CN = nf ? h->CN.data() : nullptr; d.l = h->l.data(); d.u = h->u.data();
    } else {
      d.A = lo.A; d.B = lo.B; d.b = lo.b; d.Q = lo.Q; d.R = lo.R; d.S = lo.S; d.q = lo.q; d.r = lo.r;
      d.C = lo.C; d.D = lo.D; d.CN = nf ? lo.CN : nullptr; d.l = lo.l; d.u = lo.u;
    }
    return d;
  }
  // linearise around the host nominal (X, U); device time to *ms
  int linearize(const double* X, const double* U, float* ms) {
    if (hipMemcpyAsync(Xd, X, sizeof(double) * (N + 1) * nx, hipMemcpyHostToDevice, stream) != hipSuccess ||
        hipMemcpyAsync(Ud, U, sizeof(double) * N * nu, hipMemcpyHostToDevice, stream) != hipSuccess)
      return GSLS_ERR_HIP;
    if (hipEventRecord(ev[0], stream) != hipSuccess) return GSLS_ERR_HIP;
    int rc = launch_linearize(md, Xd, Ud, lo, stream);
    if (rc) return rc;
    if (hipEventRecord(ev[1], stream) != hipSuccess || hipStreamSynchronize(stream) != hipSuccess)
      return GSLS_ERR_HIP;
    float t = 0.f;
    (void)hipEventElapsedTime(&t, ev[0], ev[1]);
    if (ms) *ms += t;
    return GSLS_OK;
  }
  int to_host(HostDesc* h) const {
    gsls_qp_desc d = desc(GSLS_DEVICE, nullptr);
    return stage_to_host(&d, h);
  }
};

static int model_dims(int kind, int* nx, int* nu) {
  if (kind == GSLS_MODEL_DUBINS) { *nx = 3; *nu = 1; return GSLS_OK; }
  if (kind == GSLS_MODEL_QUADROTOR) { *nx = 6; *nu = 2; return GSLS_OK; }
  return GSLS_ERR_INVALID_ARG;
}

}  // namespace gsls

struct gsls_sqp {
  gsls::SqpState s;
};

extern "C" {

int gsls_sqp_setup(const gsls_model_desc* md, const double* X, const double* U, const gsls_settings* settings,
                   void* stream, gsls_sqp** out) {
  using namespace gsls;
  if (!out) return GSLS_ERR_INVALID_ARG;
  *out = nullptr;
  if (!md || !X || !U) return GSLS_ERR_INVALID_ARG;
  int nx = 0, nu = 0;
  int rc = model_dims(md->model, &nx, &nu);
  if (rc) return rc;
  if (md->N < 1 || md->N > GSLS_MAX_N || md->n_obs < 0 || md->n_obs + nu > GSLS_MAX_NC) return GSLS_ERR_DIM;
  if (!(md->dt > 0.0) || !md->u_min || !md->u_max || !md->Q || !md->R || !md->QN || !md->x_ref || !md->u_ref ||
      (md->n_obs > 0 && !md->obstacles))
    return GSLS_ERR_INVALID_ARG;
  if (md->model == GSLS_MODEL_QUADROTOR && (!(md->mass > 0.0) || !(md->inertia > 0.0))) return GSLS_ERR_INVALID_ARG;
  gsls_sqp* h = new (std::nothrow) gsls_sqp;
  if (!h) return GSLS_ERR_OOM;
  SqpState& S = h->s;
  const int N = md->N, no = md->n_obs;
  S.N = N; S.nx = nx; S.nu = nu; S.no = no; S.nc = no + nu; S.nf = no; S.m = N * S.nc + no;
  S.stream = (hipStream_t)stream;
  auto upd = [&](const double* src, size_t n) -> const double* {
    double* p = S.arena.alloc<double>(std::max<size_t>(n, 1));
    if (p && n && hipMemcpy(p, src, n * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) S.arena.ok = false;
    return p;
  };
  ModelDev& m = S.md;
  m.kind = md->model; m.N = N; m.nx = nx; m.nu = nu; m.no = no;
  m.dt = md->dt; m.v = md->v; m.mass = md->mass; m.grav = md->gravity; m.arm = md->arm; m.inertia = md->inertia;
  m.obst = upd(md->obstacles, (size_t)no * 3);
  m.umin = upd(md->u_min, nu); m.umax = upd(md->u_max, nu);
  m.Q = upd(md->Q, (size_t)nx * nx); m.R = upd(md->R, (size_t)nu * nu); m.QN = upd(md->QN, (size_t)nx * nx);
  m.xref = upd(md->x_ref, (size_t)(N + 1) * nx); m.uref = upd(md->u_ref, (size_t)N * nu);
  S.Xd = S.arena.alloc<double>((size_t)(N + 1) * nx);
  S.Ud = S.arena.alloc<double>((size_t)N * nu);
  LinOut& o = S.lo;
  o.A = S.arena.alloc<double>((size_t)N * nx * nx); o.B = S.arena.alloc<double>((size_t)N * nx * nu);
  o.b = S.arena.alloc<double>((size_t)N * nx); o.Q = S.arena.alloc<double>((size_t)(N + 1) * nx * nx);
  o.R = S.arena.alloc<double>((size_t)N * nu * nu); o.S = S.arena.alloc<double>((size_t)N * nu * nx);
  o.q = S.arena.alloc<double>((size_t)(N + 1) * nx); o.r = S.arena.alloc<double>((size_t)N * nu);
  o.C = S.arena.alloc<double>((size_t)N * S.nc * nx); o.D = S.arena.alloc<double>((size_t)N * S.nc * nu);
  o.CN = S.arena.alloc<double>((size_t)std::max(no, 1) * nx);
  o.l = S.arena.alloc<double>((size_t)S.m); o.u = S.arena.alloc<double>((size_t)S.m);
  if (!S.arena.ok) { delete h; return GSLS_ERR_OOM; }
  for (auto& e : S.ev)
    if (hipEventCreate(&e) != hipSuccess) { delete h; return GSLS_ERR_HIP; }
  HostDesc hd;
  if ((rc = S.linearize(X, U, nullptr)) || (rc = S.to_host(&hd))) { delete h; return rc; }
  gsls_qp_desc d = S.desc(GSLS_HOST, &hd);
  if ((rc = gsls_qp_setup(&d, settings, stream, &S.qp))) { delete h; return rc; }
  *out = h;
  return GSLS_OK;
}

int gsls_sqp_linearize(gsls_sqp* h, const double* X, const double* U, double* A, double* B, double* b, double* q,
                       double* r, double* C, double* D, double* CN, double* l, double* u) {
  using namespace gsls;
  if (!h || !X || !U) return GSLS_ERR_INVALID_ARG;
  SqpState& S = h->s;
  int rc = S.linearize(X, U, nullptr);
  if (rc) return rc;
  const size_t N = S.N, nx = S.nx, nu = S.nu, nc = S.nc, nf = S.nf;
  auto d2h = [&](double* dst, const double* src, size_t n) -> int {
    if (!dst || !n) return GSLS_OK;
    return hipMemcpy(dst, src, n * sizeof(double), hipMemcpyDeviceToHost) == hipSuccess ? GSLS_OK : GSLS_ERR_HIP;
  };
  if ((rc = d2h(A, S.lo.A, N * nx * nx)) || (rc = d2h(B, S.lo.B, N * nx * nu)) || (rc = d2h(b, S.lo.b, N * nx)) ||
      (rc = d2h(q, S.lo.q, (N + 1) * nx)) || (rc = d2h(r, S.lo.r, N * nu)) || (rc = d2h(C, S.lo.C, N * nc * nx)) ||
      (rc = d2h(D, S.lo.D, N * nc * nu)) || (rc = d2h(CN, S.lo.CN, nf * nx)) || (rc = d2h(l, S.lo.l, S.m)) ||
      (rc = d2h(u, S.lo.u, S.m)))
    return rc;
  return GSLS_OK;
}

int gsls_sqp_solve(gsls_sqp* h, const double* x0, double* X, double* U, int32_t max_iter, double alpha,
                   double tol_qp, double tol_step, gsls_sqp_result* result) {
  using namespace gsls;
  if (!h || !x0 || !X || !U || max_iter < 0 || !(alpha > 0.0) || !(alpha <= 1.0) || !(tol_qp >= 0.0) ||
      !(tol_step >= 0.0))
    return GSLS_ERR_INVALID_ARG;
  SqpState& S = h->s;
  const int N = S.N, nx = S.nx, nu = S.nu;
  std::vector<double> dX((size_t)(N + 1) * nx), dU((size_t)N * nu), dx0(nx);
  gsls_sqp_result out{};
  out.status = 2;
  float ms_lin = 0.f;
  int rc = GSLS_OK;
  for (int it = 0; it < max_iter; ++it) {
    if ((rc = S.linearize(X, U, &ms_lin))) break;
    gsls_qp_desc d = S.desc(GSLS_DEVICE, nullptr);
    if ((rc = gsls_qp_update_data(S.qp, &d))) break;
    for (int j = 0; j < nx; ++j) dx0[j] = x0[j] - X[j];
    gsls_result r{};
    if ((rc = gsls_qp_solve(S.qp, dx0.data(), 1.0, tol_qp, &r))) break;
    out.qp_iterations += r.iterations;
    out.qp_status = r.status;
    out.ms_qp += r.ms_total;
    if (r.status != GSLS_SOLVED) { out.status = 5; break; }
    if ((rc = gsls_qp_get(S.qp, dX.data(), dU.data(), nullptr, nullptr))) break;
    double st = 0.0;
    for (size_t i = 0; i < dX.size(); ++i) { X[i] += alpha * dX[i]; st = std::max(st, std::fabs(dX[i])); }
    for (size_t i = 0; i < dU.size(); ++i) { U[i] += alpha * dU[i]; st = std::max(st, std::fabs(dU[i])); }
    ++out.iterations;
    out.step = st;
    if (st <= tol_step) { out.status = 1; break; }
  }
  out.ms_linearize = ms_lin;
  if (rc) return rc;
  if (result) *result = out;
  return GSLS_OK;
}

int gsls_rti_step(gsls_sqp* h, const double* x0, double* X, double* U, const double* E, const double* Qbar,
                  const double* Rbar, const double* QbarN, int32_t rownorm, double wbound, double tol_qp,
                  int32_t max_passes, gsls_robust_result* result, double* hmarg, double* hf) {
  using namespace gsls;
  if (!h || !x0 || !X || !U || !E) return GSLS_ERR_INVALID_ARG;
  SqpState& S = h->s;
  const int N = S.N, nx = S.nx, nu = S.nu;
  int rc = S.linearize(X, U, nullptr);
  if (rc) return rc;
  gsls_qp_desc d = S.desc(GSLS_DEVICE, nullptr);
  if ((rc = gsls_qp_update_data(S.qp, &d))) return rc;
  std::vector<double> Es((size_t)N * nx * nx), dx0(nx), dX((size_t)(N + 1) * nx), dU((size_t)N * nu);
  for (int k = 0; k < N; ++k) std::memcpy(Es.data() + (size_t)k * nx * nx, E, sizeof(double) * nx * nx);
  for (int j = 0; j < nx; ++j) dx0[j] = x0[j] - X[j];
  gsls_robust_result rr{};
  if ((rc = gsls_robust_solve(S.qp, dx0.data(), Es.data(), Qbar, Rbar, QbarN, rownorm, wbound, 1e-8, 1.0, tol_qp,
                              max_passes, 0.0, &rr, hmarg, hf)))
    return rc;
  if (rr.qp_status == GSLS_SOLVED) {
    if ((rc = gsls_qp_get(S.qp, dX.data(), dU.data(), nullptr, nullptr))) return rc;
    for (size_t i = 0; i < dX.size(); ++i) X[i] += dX[i];
    for (size_t i = 0; i < dU.size(); ++i) U[i] += dU[i];
  }
  if (result) *result = rr;
  return GSLS_OK;
}

void gsls_sqp_free(gsls_sqp* h) { delete h; }

}  // extern "C"
