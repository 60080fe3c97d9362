// Cell-wise geometric multigrid V-cycle and primal-dual preconditioned CG.
//
// V-cycle: Algorithm 1 with a zero initial guess (Sec. 5: the preconditioner
// skips the first operator application), residual restriction fused with
// the residual formation (Sec. 5), coarse solve by a dense FP64 inverse.
// Smoothers:
//   Jacobi:  the fused sweep of Algorithm 9 (apply, raw per-copy update with
//            the valence-baked masked inverse diagonal, averaging DSS);
//   Cheb-FDM: Chebyshev semi-iteration of degree d preconditioned by the
//            vertex-patch inverse, an admissible smoother of the form
//            G P_CG G^T (eq. precond_consistency).
// PCG: Sec. 4.4, all inner products pair a dual with a primal vector and are
// therefore local (eq. pairing_global); the stopping test uses the assembled
// residual ||G^T r||_2.  The V-cycle may run in FP32 inside the FP64
// iteration; the flexible (Polak-Ribiere) beta then keeps the iteration
// robust to the small nonlinearity of the rounded preconditioner.
#include <chrono>
#include <cmath>

#include "fe_internal.h"

namespace fe {

fe_status ensure_dinv_level(fe_problem* p, int li, hipStream_t s);
fe_status ensure_coarse_inverse(fe_problem* p, hipStream_t s);

struct Solver {
  fe_pcg_opts opts{};
  bool ready = false;
  int inner = FE_F64;
  DeviceBuf r, z, pv, q, zf;  // finest-level FP64 PCG vectors
  DeviceBuf dscal;             // device doubles for reductions
  // HIP graph of the preconditioner application (see apply_precond)
  hipStream_t cs = nullptr;    // pcg_solve's own stream (capture needs a non-null stream)
  int64_t gen = 0;             // bumped by every full setup
  int64_t eager_gen = -1;      // generation of the last eager application
  fe_pcg_opts eager_opts{};
  hipGraphExec_t graph = nullptr;
  int64_t graph_gen = -1;
  fe_pcg_opts graph_opts{};
  const void* graph_r = nullptr;
  void* graph_z = nullptr;
  // level work buffers (e, t of the inner dtype, per level) as they were at
  // capture: the Jacobi sweeps alternate e and t by swapping these pointers, so
  // a call outside the graph (fe_vcycle with an odd sweep count) can leave
  // them swapped, and the graph would then write where pcg_solve no longer reads
  std::vector<void*> graph_bufs;
  void drop_graph() {
    if (graph) (void)hipGraphExecDestroy(graph);
    graph = nullptr;
    graph_gen = -1;
  }
  ~Solver() {
    drop_graph();
    if (cs) (void)hipStreamDestroy(cs);
  }
};

static bool same_setup(const fe_pcg_opts& a, const fe_pcg_opts& b) {
  return a.smoother == b.smoother && a.cheb_degree == b.cheb_degree && a.cheb_ratio == b.cheb_ratio &&
         a.cheb_lmax == b.cheb_lmax && a.inner == b.inner && a.factors == b.factors && a.precond == b.precond &&
         a.omega == b.omega;
}

static double* dev_scalar(fe_problem* p, int i) { return p->solver->dscal.as<double>() + i; }

// device scalars 0..2 in one copy and one wait
static fe_status read_scalars3(fe_problem* p, double* out, hipStream_t s) {
  FE_HIP_CHECK(hipMemcpyAsync(out, dev_scalar(p, 0), 3 * sizeof(double), hipMemcpyDeviceToHost, s));
  FE_HIP_CHECK(hipStreamSynchronize(s));
  return FE_OK;
}

static fe_status read_scalar(fe_problem* p, int i, double* out, hipStream_t s) {
  FE_HIP_CHECK(hipMemcpyAsync(out, dev_scalar(p, i), sizeof(double), hipMemcpyDeviceToHost, s));
  FE_HIP_CHECK(hipStreamSynchronize(s));
  return FE_OK;
}

// The patch inverse's scratch and factors are prepared at solver setup
// (prepare_patch_inverse), so the V-cycle's launches allocate nothing.
static fe_status patch_apply(fe_problem* p, int l, const void* r, void* z, fe_dtype dt, int factors, hipStream_t s) {
  return launch_patch_inverse(p, l, r, z, p->levels[l].fdm_scratch[dt == FE_F64 ? 0 : 1].p, dt, factors, s);
}

// v = P r, then w = a v + c w and e = w (e_zero) or e += w
static fe_status patch_cheb(fe_problem* p, int l, const void* r, void* v, fe_dtype dt, int factors, double a, double c,
                            void* w, void* e, int e_zero, hipStream_t s) {
  return launch_patch_cheb(p, l, r, v, p->levels[l].fdm_scratch[dt == FE_F64 ? 0 : 1].p, dt, factors, a, c, w, e,
                           e_zero, s);
}

// lambda_max of P A on level l by CG-Lanczos from a fixed start vector; P is the
// patch inverse (smoother = FE_SMOOTH_CHEB_FDM) or the Jacobi preconditioner
// G D^{-1} G^T = S_bar(K_cell D_cell^{-1} .) (smoother = FE_SMOOTH_JACOBI).
static fe_status estimate_lmax(fe_problem* p, int l, int smoother, int factors, int steps, double* out,
                               hipStream_t s) {
  Level& L = p->levels[l];
  const int64_t n = L.len;
  if (smoother == FE_SMOOTH_JACOBI) FE_CHECK(ensure_dinv_level(p, l, s));
  if (smoother == FE_SMOOTH_CHEB_FDM) FE_CHECK(prepare_patch_inverse(p, l, FE_F64, factors, s));
  auto precond = [&](const void* rr, void* zz) -> fe_status {
    if (smoother == FE_SMOOTH_JACOBI)
      return launch_jacobi_avg(p, l, rr, rr, rr, L.dinv64.p, zz, 1.0, 1, FE_F64, s);
    return patch_apply(p, l, rr, zz, FE_F64, factors, s);
  };
  DeviceBuf x, r, z, pp, q;
  for (DeviceBuf* b : {&x, &r, &z, &pp, &q}) FE_CHECK(b->alloc(n * sizeof(double)));
  // start vector: deterministic hash of the index (counter based), dual
  std::vector<double> h(n);
  for (int64_t i = 0; i < n; ++i) {
    uint64_t zq = (uint64_t)i * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
    zq = (zq ^ (zq >> 30)) * 0xBF58476D1CE4E5B9ull;
    zq = (zq ^ (zq >> 27)) * 0x94D049BB133111EBull;
    zq ^= zq >> 31;
    h[i] = (double)(zq >> 11) * (1.0 / 9007199254740992.0) - 0.5;
  }
  FE_HIP_CHECK(hipMemcpyAsync(r.p, h.data(), n * sizeof(double), hipMemcpyHostToDevice, s));
  std::vector<double> alpha, beta;
  FE_CHECK(precond(r.p, z.p));
  FE_CHECK(launch_cast(n, z.p, FE_F64, pp.p, FE_F64, s));
  FE_CHECK(dot_async(p, n, r.p, z.p, FE_F64, dev_scalar(p, 0), s));
  double rho;
  FE_CHECK(read_scalar(p, 0, &rho, s));
  for (int it = 0; it < steps; ++it) {
    FE_CHECK(launch_apply(p, l, pp.p, q.p, FE_F64, s));
    FE_CHECK(dot_async(p, n, pp.p, q.p, FE_F64, dev_scalar(p, 0), s));
    double pq;
    FE_CHECK(read_scalar(p, 0, &pq, s));
    if (!(pq > 0.0) || !(rho > 0.0)) break;
    const double a = rho / pq;
    alpha.push_back(a);
    FE_CHECK(launch_axpby(n, -a, q.p, 1.0, r.p, FE_F64, s));
    FE_CHECK(precond(r.p, z.p));
    FE_CHECK(dot_async(p, n, r.p, z.p, FE_F64, dev_scalar(p, 0), s));
    double rho2;
    FE_CHECK(read_scalar(p, 0, &rho2, s));
    const double b = rho2 / rho;
    beta.push_back(b);
    rho = rho2;
    FE_CHECK(launch_axpby(n, 1.0, z.p, b, pp.p, FE_F64, s));
  }
  const int m = (int)alpha.size();
  if (m == 0) return fail(FE_EBREAKDOWN, "Lanczos estimate broke down");
  // Lanczos tridiagonal from the CG coefficients
  std::vector<double> T(m * m, 0.0), I(m * m, 0.0), S, lam;
  for (int i = 0; i < m; ++i) {
    I[i * m + i] = 1.0;
    T[i * m + i] = 1.0 / alpha[i] + (i > 0 ? beta[i - 1] / alpha[i - 1] : 0.0);
    if (i + 1 < m) T[i * m + i + 1] = T[(i + 1) * m + i] = std::sqrt(beta[i]) / alpha[i];
  }
  if (!sym_generalized_eig(m, T, I, S, lam)) return fail(FE_EBREAKDOWN, "tridiagonal eigensolve failed");
  *out = lam[m - 1];
  return FE_OK;
}

fe_status solver_setup(fe_problem* p, const fe_pcg_opts* o, hipStream_t s) {
  if (p->dim != 3) return fail(FE_EUNSUPPORTED, "the multigrid solver is implemented for d = 3");
  if (p->bc != 1) return fail(FE_EINVAL, "the solver needs homogeneous Dirichlet conditions (bc = 1)");
  FE_CHECK(ensure_coarse_inverse(p, s));
  if (!p->solver) p->solver = new Solver();
  Solver& S = *p->solver;
  // the per-level data the options need (patch factors, Chebyshev bounds) can
  // be invalidated between calls, e.g. when the factor model is retrained
  bool levels_ready = true;
  if (o->smoother == FE_SMOOTH_CHEB_FDM) {
    const int key = o->factors * 1000 + 15;
    for (size_t l = 1; l < p->levels.size(); ++l) {
      const Level& L = p->levels[l];
      if ((o->factors != 0 && !L.patch_eig_ready[o->factors]) || (o->cheb_lmax <= 0.0 && L.lmax_key != key))
        levels_ready = false;
    }
  }
  if (S.ready && levels_ready && same_setup(S.opts, *o)) {
    S.opts = *o;
    return FE_OK;
  }
  const int nl = (int)p->levels.size();
  const int64_t nfine = p->levels.back().len;
  FE_CHECK(S.dscal.alloc(64 * sizeof(double)));
  for (DeviceBuf* b : {&S.r, &S.z, &S.pv, &S.q}) FE_CHECK(b->alloc(nfine * sizeof(double)));
  const int di = o->inner == FE_F64 ? 0 : 1;
  const size_t es = o->inner == FE_F64 ? 8 : 4;
  for (int l = 0; l < nl; ++l) {
    Level& L = p->levels[l];
    for (DeviceBuf* b : {&L.e[di], &L.b[di], &L.v[di], &L.t[di], &L.w[di]}) FE_CHECK(b->alloc(L.len * es));
    if (l > 0 && o->smoother == FE_SMOOTH_JACOBI) {
      FE_CHECK(ensure_dinv_level(p, l, s));
      if (o->omega != 0.0) {
        L.omega = o->omega;   // taken literally (a negative value is allowed and diverges)
      } else if (L.omega_auto <= 0.0) {
        // automatic damping 4 / (3 lambda_max(D^{-1} A)): 2/3 of the stability limit
        double lm;
        FE_CHECK(estimate_lmax(p, l, FE_SMOOTH_JACOBI, 0, 15, &lm, s));
        L.omega_auto = 4.0 / (3.0 * lm);
        L.omega = L.omega_auto;
      } else {
        L.omega = L.omega_auto;
      }
    }
    if (l > 0 && o->smoother == FE_SMOOTH_CHEB_FDM) {
      FE_CHECK(prepare_patch_inverse(p, l, (fe_dtype)o->inner, o->factors, s));
      const int key = o->factors * 1000 + 15;
      // L.lmax is the top of the Chebyshev interval: a caller's value as given,
      // a Lanczos estimate (which approaches lambda_max from below) times 1.2
      if (o->cheb_lmax > 0.0) {
        L.lmax = o->cheb_lmax;
        L.lmax_key = -1;
      } else if (L.lmax_key != key) {
        double lm;
        FE_CHECK(estimate_lmax(p, l, FE_SMOOTH_CHEB_FDM, o->factors, 15, &lm, s));
        L.lmax = 1.2 * lm;
        L.lmax_key = key;
      }
    }
  }
  FE_HIP_CHECK(hipStreamSynchronize(s));
  S.opts = *o;
  S.ready = true;
  ++S.gen;   // level data may have changed: a captured preconditioner is stale
  S.drop_graph();
  return FE_OK;
}

void solver_destroy(fe_problem* p) {
  delete p->solver;
  p->solver = nullptr;
}

// ---------------------------------------------------------------- smoothers
static fe_status jacobi_smooth(fe_problem* p, int l, int sweeps, bool u_zero, fe_dtype dt, hipStream_t s) {
  Level& L = p->levels[l];
  const int di = dt == FE_F64 ? 0 : 1;
  const void* dinv = dt == FE_F64 ? L.dinv64.p : L.dinv32.p;
  const double omega = L.omega;
  for (int it = 0; it < sweeps; ++it) {
    const bool z = u_zero && it == 0;
    if (!z) FE_CHECK(launch_apply(p, l, L.e[di].p, L.v[di].p, dt, s));
    // fused update + averaging DSS into t, then t becomes the iterate
    FE_CHECK(launch_jacobi_avg(p, l, L.e[di].p, L.b[di].p, L.v[di].p, dinv, L.t[di].p, omega, z ? 1 : 0, dt, s));
    std::swap(L.e[di].p, L.t[di].p);
    std::swap(L.e[di].bytes, L.t[di].bytes);
  }
  return FE_OK;
}

// Chebyshev semi-iteration on [lmax/ratio, lmax] preconditioned by the patch inverse.
// Buffers: e = iterate, b = rhs, t = residual (dual), w = direction (primal),
// v = P t (primal) where the step does not run inside the patch inverse.
static fe_status cheb_smooth(fe_problem* p, int l, int sweeps, bool u_zero, fe_dtype dt, hipStream_t s) {
  Level& L = p->levels[l];
  const int di = dt == FE_F64 ? 0 : 1;
  const fe_pcg_opts& o = p->solver->opts;
  const double lmax = L.lmax, lmin = lmax / o.cheb_ratio;
  const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin), sigma = theta / delta;
  void *e = L.e[di].p, *b = L.b[di].p, *t = L.t[di].p, *w = L.w[di].p, *v = L.v[di].p;
  for (int sw = 0; sw < sweeps; ++sw) {
    const bool z = u_zero && sw == 0;
    double rho = 1.0 / sigma;
    // t = b - A e (the residual fused into the operator's store); from a zero
    // start the residual is b itself and is read in place
    if (!z) FE_CHECK(launch_apply_ep(p, l, e, t, -1.0, 1.0, b, dt, s));
    // w = P t / theta; e += w
    FE_CHECK(patch_cheb(p, l, z ? b : t, w, dt, o.factors, 1.0 / theta, 0.0, w, e, z ? 1 : 0, s));
    for (int it = 1; it < o.cheb_degree; ++it) {
      // t -= A w (t = b - A w after a zero start: nothing was copied into t)
      FE_CHECK(launch_apply_ep(p, l, w, t, -1.0, 1.0, z && it == 1 ? b : t, dt, s));
      const double rho_new = 1.0 / (2.0 * sigma - rho);
      // v = P t (primal), w = 2 rho_new / delta v + rho_new rho w, e += w
      FE_CHECK(patch_cheb(p, l, t, v, dt, o.factors, 2.0 * rho_new / delta, rho_new * rho, w, e, 0, s));
      rho = rho_new;
    }
  }
  return FE_OK;
}

static fe_status smooth(fe_problem* p, int l, bool pre, bool u_zero, fe_dtype dt, hipStream_t s) {
  const fe_pcg_opts& o = p->solver->opts;
  const int sweeps = pre ? o.nu_pre : o.nu_post;
  if (sweeps <= 0) {
    if (u_zero) FE_CHECK(launch_fill(p->levels[l].len, p->levels[l].e[dt == FE_F64 ? 0 : 1].p, 0.0, dt, s));
    return FE_OK;
  }
  if (o.smoother == FE_SMOOTH_JACOBI) return jacobi_smooth(p, l, sweeps, u_zero, dt, s);
  return cheb_smooth(p, l, sweeps, u_zero, dt, s);
}

// e_l = MG(b_l) with zero initial guess; b_l, e_l live in the level buffers.
static fe_status vcycle_level(fe_problem* p, int l, fe_dtype dt, hipStream_t s) {
  Level& L = p->levels[l];
  const int di = dt == FE_F64 ? 0 : 1;
  if (l == 0) return launch_coarse_solve(p, L.b[di].p, L.e[di].p, dt, s);
  FE_CHECK(smooth(p, l, true, true, dt, s));
  FE_CHECK(launch_apply(p, l, L.e[di].p, L.v[di].p, dt, s));
  Level& C = p->levels[l - 1];
  FE_CHECK(launch_restrict(p, l, L.b[di].p, L.v[di].p, C.b[di].p, dt, s));
  FE_CHECK(vcycle_level(p, l - 1, dt, s));
  FE_CHECK(launch_prolongate_add(p, l, C.e[di].p, L.e[di].p, dt, s));
  return smooth(p, l, false, false, dt, s);
}

fe_status solver_vcycle(fe_problem* p, const fe_pcg_opts* o, fe_dtype dt, hipStream_t s) {
  (void)o;
  return vcycle_level(p, (int)p->levels.size() - 1, dt, s);
}

// z = M r (finest level): r, z FP64 (with a preconditioner, z may be null)
static fe_status precondition(fe_problem* p, const void* r, void* z, hipStream_t s) {
  Solver& S = *p->solver;
  Level& F = p->levels.back();
  const fe_dtype dt = (fe_dtype)S.opts.inner;
  const int di = dt == FE_F64 ? 0 : 1;
  if (!S.opts.precond) return launch_cast(F.len, r, FE_F64, z, FE_F64, s);
  // The preconditioner reads r only through G^T r, so an FP32 V-cycle is fed
  // the averaged copies S_bar r (formed in FP64): the raw copies of a residual
  // near convergence are far larger than their sum, and rounding them to FP32
  // first would bury G^T r.
  if (dt == FE_F32) FE_CHECK(launch_average_convert(p, -1, (const double*)r, F.b[di].p, dt, s));
  else FE_CHECK(launch_cast(F.len, r, FE_F64, F.b[di].p, dt, s));
  FE_CHECK(vcycle_level(p, (int)p->levels.size() - 1, dt, s));
  // z null: the result stays in the finest level's iterate, in the inner precision
  return z ? launch_cast(F.len, F.e[di].p, dt, z, FE_F64, s) : FE_OK;
}

// Options that shape the V-cycle's launch sequence (and the values baked into
// its kernel arguments, together with the setup generation).
static bool same_vcycle(const fe_pcg_opts& a, const fe_pcg_opts& b) {
  return same_setup(a, b) && a.nu_pre == b.nu_pre && a.nu_post == b.nu_post;
}

static std::vector<void*> level_bufs(fe_problem* p) {
  const int di = p->solver->opts.inner == FE_F64 ? 0 : 1;
  std::vector<void*> v;
  for (const Level& L : p->levels) {
    v.push_back(L.e[di].p);
    v.push_back(L.t[di].p);
  }
  return v;
}

// z = M r, replayed as a HIP graph once the same application has run eagerly
// with the current setup (the eager run performs any first-use allocation,
// which capture would reject).  A V-cycle is a fixed sequence of launches on
// fixed buffers with coefficients fixed at setup, and launch latency dominates
// its coarse levels.  No fill or copy in it is a memset (those do not replay
// reliably in graphs here).  Falls back to the eager path when capture fails.
static fe_status apply_precond(fe_problem* p, const void* r, void* z, hipStream_t s) {
  Solver& S = *p->solver;
  const fe_pcg_opts& o = S.opts;
  const bool safe = graphs_enabled() && !prof_enabled() && o.precond &&
                    !(o.smoother == FE_SMOOTH_JACOBI && ((o.nu_pre & 1) || (o.nu_post & 1)));
  if (!safe) {
    S.drop_graph();
    return precondition(p, r, z, s);
  }
  if (S.graph && S.graph_gen == S.gen && same_vcycle(S.graph_opts, o) && S.graph_r == r && S.graph_z == z &&
      S.graph_bufs == level_bufs(p)) {
    FE_HIP_CHECK(hipGraphLaunch(S.graph, s));
    return FE_OK;
  }
  S.drop_graph();
  if (S.eager_gen != S.gen || !same_vcycle(S.eager_opts, o)) {
    S.eager_gen = S.gen;
    S.eager_opts = o;
    return precondition(p, r, z, s);
  }
  hipGraph_t g = nullptr;
  const std::vector<void*> bufs = level_bufs(p);
  if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return precondition(p, r, z, s);
  const fe_status st = precondition(p, r, z, s);
  const hipError_t ec = hipStreamEndCapture(s, &g);
  hipGraphExec_t ex = nullptr;
  if (st != FE_OK || ec != hipSuccess || !g || hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    S.eager_gen = -1;   // capture again only after another eager run
    return precondition(p, r, z, s);   // nothing captured was executed
  }
  (void)hipGraphDestroy(g);
  S.graph = ex;
  S.graph_gen = S.gen;
  S.graph_opts = o;
  S.graph_r = r;
  S.graph_z = z;
  S.graph_bufs = bufs;
  FE_HIP_CHECK(hipGraphLaunch(ex, s));
  return FE_OK;
}

}  // namespace fe

using namespace fe;

extern "C" {

void fe_pcg_default_opts(fe_pcg_opts* o) {
  if (!o) return;
  o->tol = 1e-10;
  o->maxit = 200;
  o->nu_pre = 2;
  o->nu_post = 2;
  o->smoother = FE_SMOOTH_JACOBI;
  o->cheb_degree = 3;
  o->cheb_ratio = 20.0;
  o->cheb_lmax = 0.0;
  o->omega = 0.7;
  o->inner = FE_F64;
  o->factors = 0;
  o->flexible = 0;
  o->precond = 1;
  o->stop = 0;
}

static fe_status check_opts(const fe_problem* p, const fe_pcg_opts* o) {
  if (!o) return fail(FE_EINVAL, "null opts");
  if (o->inner != FE_F64 && o->inner != FE_F32) return fail(FE_EINVAL, "bad inner precision");
  if (o->smoother != FE_SMOOTH_JACOBI && o->smoother != FE_SMOOTH_CHEB_FDM) return fail(FE_EINVAL, "bad smoother");
  if (o->smoother == FE_SMOOTH_CHEB_FDM && (o->cheb_degree < 1 || o->cheb_ratio <= 1.0))
    return fail(FE_EINVAL, "bad Chebyshev parameters");
  if (o->smoother == FE_SMOOTH_CHEB_FDM && o->factors == 0 && p->desc.geometry != FE_GEOM_CARTESIAN)
    return fail(FE_EINVAL, "exact separable factors need the Cartesian mesh");
  if (o->smoother == FE_SMOOTH_CHEB_FDM && o->factors != 0 && p->desc.geometry != FE_GEOM_DEFORMED)
    return fail(FE_EINVAL, "per-patch factors need the deformed geometry");
  if (o->factors < 0 || o->factors > 3) return fail(FE_EINVAL, "bad factors");
  if (o->nu_pre < 0 || o->nu_post < 0 || o->maxit < 0) return fail(FE_EINVAL, "negative counts");
  if (!(o->tol >= 0.0)) return fail(FE_EINVAL, "bad tolerance");
  if (o->stop != 0 && o->stop != 1) return fail(FE_EINVAL, "stop must be 0 or 1");
  if (o->stop == 1 && !o->precond) return fail(FE_EINVAL, "the energy stopping test needs the preconditioner");
  return FE_OK;
}

fe_status fe_vcycle(fe_problem* p, const void* b, void* e, const fe_pcg_opts* o, fe_dtype dt, void* stream) {
  if (!p) return fail(FE_EINVAL, "null problem");
  FE_CHECK(check_opts(p, o));
  if (dt != (fe_dtype)o->inner) return fail(FE_EINVAL, "dtype must equal opts->inner");
  FE_CHECK(check_ptr(b, "b"));
  FE_CHECK(check_ptr(e, "e"));
  hipStream_t s = (hipStream_t)stream;
  FE_CHECK(solver_setup(p, o, s));
  Level& F = p->levels.back();
  const int di = dt == FE_F64 ? 0 : 1;
  FE_CHECK(launch_cast(F.len, b, dt, F.b[di].p, dt, s));
  FE_CHECK(vcycle_level(p, (int)p->levels.size() - 1, dt, s));
  return launch_cast(F.len, F.e[di].p, dt, e, dt, s);
}

fe_status fe_estimate_lmax(fe_problem* p, int level, int smoother, int factors, int steps, double* out,
                           void* stream) {
  if (!p || !out) return fail(FE_EINVAL, "null argument");
  FE_CHECK(check_level(p, level));
  if (smoother != FE_SMOOTH_CHEB_FDM && smoother != FE_SMOOTH_JACOBI) return fail(FE_EINVAL, "unknown smoother");
  if (steps < 1 || steps > 200) return fail(FE_EINVAL, "steps out of range");
  hipStream_t s = (hipStream_t)stream;
  const int l = level < 0 ? (int)p->levels.size() - 1 : level;
  if (factors != 0 && !p->levels[l].patch_eig_ready[factors]) FE_CHECK(setup_patch_factors(p, l, factors, s));
  if (!p->solver) p->solver = new Solver();
  FE_CHECK(p->solver->dscal.alloc(64 * sizeof(double)));
  return estimate_lmax(p, l, smoother, factors, steps, out, s);
}

fe_status pcg_solve(fe_problem* p, const void* b, void* x, const fe_pcg_opts* o, fe_pcg_report* rep, void* stream) {
  using clk = std::chrono::steady_clock;
  if (!p) return fail(FE_EINVAL, "null problem");
  FE_CHECK(check_opts(p, o));
  FE_CHECK(check_ptr(b, "b_cell"));
  FE_CHECK(check_ptr(x, "x_cell"));
  hipStream_t s = (hipStream_t)stream;
  auto t0 = clk::now();
  FE_CHECK(solver_setup(p, o, s));
  FE_HIP_CHECK(hipStreamSynchronize(s));   // the caller's stream has drained
  auto t1 = clk::now();
  Solver& S = *p->solver;
  if (!S.cs) FE_HIP_CHECK(hipStreamCreateWithFlags(&S.cs, hipStreamNonBlocking));
  s = S.cs;
  Level& F = p->levels.back();
  const int64_t n = F.len;
  void *r = S.r.p, *z = S.z.p, *pv = S.pv.p, *q = S.q.p;
  // z = M r: with a preconditioner the V-cycle's result is read where it lies,
  // the finest level's iterate in the inner precision (FP32 values enter the
  // FP64 dot products and direction update exactly), so no FP64 copy is made.
  // It stays intact until the next application, past the flexible <r, z_old>.
  const void* zc = z;
  fe_dtype zdt = FE_F64;
  auto precond = [&]() -> fe_status {
    if (!S.opts.precond) return apply_precond(p, r, z, s);
    FE_CHECK(apply_precond(p, r, nullptr, s));
    zdt = (fe_dtype)S.opts.inner;
    zc = F.e[zdt == FE_F64 ? 0 : 1].p;
    return FE_OK;
  };
  double nb2, rr2;
  // Dirichlet problem: the residual lives in the dual of the interior space, so
  // the boundary copies of b are masked out (they carry no equation).
  FE_CHECK(launch_cast(n, b, FE_F64, r, FE_F64, s));
  FE_CHECK(launch_mask_boundary(p, -1, r, FE_F64, s));
  FE_CHECK(assembled_norm2_async(p, -1, r, FE_F64, dev_scalar(p, 1), s));
  FE_CHECK(read_scalar(p, 1, &nb2, s));
  // r = M (b - A x)
  FE_CHECK(launch_mask_boundary(p, -1, x, FE_F64, s));
  FE_CHECK(launch_apply(p, -1, x, q, FE_F64, s));
  FE_CHECK(launch_axpby(n, -1.0, q, 1.0, r, FE_F64, s));
  FE_CHECK(assembled_norm2_async(p, -1, r, FE_F64, dev_scalar(p, 1), s));
  FE_CHECK(read_scalar(p, 1, &rr2, s));
  const double nb = std::sqrt(nb2);
  double relres = nb > 0 ? std::sqrt(rr2) / nb : 0.0;
  fe_pcg_report R{};
  fe_status result = FE_OK;
  int it = 0;
  bool energy_done = false;
  if (!std::isfinite(nb2) || !std::isfinite(relres))
    result = fail(FE_EBREAKDOWN, "non-finite right-hand side or initial residual");
  if (result == FE_OK && relres > o->tol) {
    FE_CHECK(precond());
    FE_CHECK(launch_cast(n, zc, zdt, pv, FE_F64, s));
    double rho;
    FE_CHECK(dot_async_x(p, n, (const double*)r, zc, zdt, dev_scalar(p, 0), s));
    FE_CHECK(read_scalar(p, 0, &rho, s));
    R.energy0 = rho;
    R.energy = rho;
    const double rho0 = rho;
    const bool energy_stop = o->stop == 1;
    if (!(rho > 0.0)) result = fail(FE_EBREAKDOWN, "<r, z> <= 0 at start: preconditioner not positive");
    while (result == FE_OK && it < o->maxit) {
      ++it;
      FE_CHECK(launch_apply(p, -1, pv, q, FE_F64, s));
      // <p, A p> stays on the device: the update forms alpha there, and the
      // host reads it with the residual norm and <r_new, z_old> in one copy
      FE_CHECK(dot_async(p, n, pv, q, FE_F64, dev_scalar(p, 0), s));
      FE_CHECK(launch_cg_update(n, rho, dev_scalar(p, 0), (const double*)pv, (const double*)q, (double*)x, (double*)r,
                                s));
      if (o->flexible) FE_CHECK(dot_async_x(p, n, (const double*)r, zc, zdt, dev_scalar(p, 2), s));
      // the residual test needs one assembled norm per iteration; the energy
      // test reads <r, z> that the next direction needs anyway
      if (!energy_stop) FE_CHECK(assembled_norm2_async(p, -1, r, FE_F64, dev_scalar(p, 1), s));
      double sc[3];
      FE_CHECK(read_scalars3(p, sc, s));
      const double pq = sc[0], rz_old = o->flexible ? sc[2] : 0.0;
      if (!(pq > 0.0) || !std::isfinite(pq)) {
        result = fail(FE_EBREAKDOWN, "<p, A p> <= 0");
        break;
      }
      if (!energy_stop) {
        rr2 = sc[1];
        relres = std::sqrt(rr2) / nb;
        if (!std::isfinite(relres)) {
          result = fail(FE_EBREAKDOWN, "non-finite residual");
          break;
        }
        if (relres <= o->tol) break;
      }
      FE_CHECK(precond());
      double rho_new;
      FE_CHECK(dot_async_x(p, n, (const double*)r, zc, zdt, dev_scalar(p, 0), s));
      FE_CHECK(read_scalar(p, 0, &rho_new, s));
      R.energy = rho_new;
      if (energy_stop && std::isfinite(rho_new) && rho_new >= 0.0 && rho_new <= o->tol * rho0) {
        energy_done = true;
        break;
      }
      if (!(rho_new > 0.0)) {
        result = fail(FE_EBREAKDOWN, "<r, z> <= 0: preconditioner not positive");
        break;
      }
      const double beta = o->flexible ? (rho_new - rz_old) / rho : rho_new / rho;
      FE_CHECK(launch_axpby_x(n, 1.0, zc, zdt, beta, (double*)pv, s));
      rho = rho_new;
    }
    if (energy_stop) {
      // the assembled residual of the final iterate, for the report
      FE_CHECK(assembled_norm2_async(p, -1, r, FE_F64, dev_scalar(p, 1), s));
      FE_CHECK(read_scalar(p, 1, &rr2, s));
      relres = std::sqrt(rr2) / nb;
      if (result == FE_OK && !energy_done) result = fail(FE_ENOTCONV, "maximum number of iterations reached");
    } else if (result == FE_OK && relres > o->tol) {
      result = fail(FE_ENOTCONV, "maximum number of iterations reached");
    }
  }
  FE_HIP_CHECK(hipStreamSynchronize(s));
  auto t2 = clk::now();
  R.iters = it;
  R.relres = relres;
  R.converged = (o->stop == 1 ? energy_done : relres <= o->tol) ? 1 : 0;
  R.t_setup = std::chrono::duration<double>(t1 - t0).count();
  R.t_solve = std::chrono::duration<double>(t2 - t1).count();
  if (rep) *rep = R;
  return result;
}


fe_status fe_mg_iterate(fe_problem* p, const void* b, void* x, const fe_pcg_opts* o, int cycles, double* eta,
                        double* res, void* stream) {
  if (!p) return fail(FE_EINVAL, "null problem");
  FE_CHECK(check_opts(p, o));
  if (!o->precond) return fail(FE_EINVAL, "the multigrid iteration needs the V-cycle (precond = 1)");
  if (cycles < 0 || cycles > 100000) return fail(FE_EINVAL, "cycles out of range");
  FE_CHECK(check_ptr(b, "b_cell"));
  FE_CHECK(check_ptr(x, "x_cell"));
  hipStream_t s = (hipStream_t)stream;
  FE_CHECK(solver_setup(p, o, s));
  FE_HIP_CHECK(hipStreamSynchronize(s));
  Solver& S = *p->solver;
  if (!S.cs) FE_HIP_CHECK(hipStreamCreateWithFlags(&S.cs, hipStreamNonBlocking));
  s = S.cs;
  Level& F = p->levels.back();
  const int64_t n = F.len;
  void *bm = S.pv.p, *r = S.r.p, *z = S.z.p, *q = S.q.p;
  // b with its boundary copies masked (they carry no equation), kept in pv
  FE_CHECK(launch_cast(n, b, FE_F64, bm, FE_F64, s));
  FE_CHECK(launch_mask_boundary(p, -1, bm, FE_F64, s));
  FE_CHECK(launch_mask_boundary(p, -1, x, FE_F64, s));
  for (int c = 0; c < cycles; ++c) {
    // r = b - A x, z = MG(r), x += z
    FE_CHECK(launch_apply_ep(p, -1, x, r, -1.0, 1.0, bm, FE_F64, s));
    FE_CHECK(apply_precond(p, r, z, s));
    FE_CHECK(launch_axpby(n, 1.0, z, 1.0, x, FE_F64, s));
    if (!eta && !res) continue;
    FE_CHECK(launch_apply_ep(p, -1, x, q, -1.0, 1.0, bm, FE_F64, s));
    if (eta) FE_CHECK(dot_async(p, n, q, x, FE_F64, dev_scalar(p, 0), s));
    if (res) FE_CHECK(assembled_norm2_async(p, -1, q, FE_F64, dev_scalar(p, 1), s));
    double v = 0.0;
    if (eta) {
      FE_CHECK(read_scalar(p, 0, &v, s));
      eta[c] = v;
    }
    if (res) {
      FE_CHECK(read_scalar(p, 1, &v, s));
      res[c] = std::sqrt(v);
    }
  }
  FE_HIP_CHECK(hipStreamSynchronize(s));
  return FE_OK;
}

}  // extern "C"
