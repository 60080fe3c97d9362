// C ABI entry points: problem setup, argument validation, dispatch to the
// kernel launchers, error state and per-kernel event timing.
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>

#include "fe_internal.h"

namespace fe {

// ---------------------------------------------------------------- errors
static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }
fe_status fail(fe_status st, const std::string& msg) {
  set_error(msg);
  return st;
}

fe_status check_level(const fe_problem* p, int l) {
  if (l < -1 || l >= (int)p->levels.size()) return fail(FE_EINVAL, "level out of range");
  return FE_OK;
}

fe_status check_ptr(const void* ptr, const char* name) {
  if (!ptr) return fail(FE_EINVAL, std::string("null pointer: ") + name);
  if (reinterpret_cast<uintptr_t>(ptr) % 16 != 0) return fail(FE_EINVAL, std::string("misaligned buffer: ") + name);
  return FE_OK;
}

// ---------------------------------------------------------------- device buffers
DeviceBuf::~DeviceBuf() { release(); }
void DeviceBuf::release() {
  if (p) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
}
fe_status DeviceBuf::alloc(size_t b) {
  if (p && bytes >= b) return FE_OK;
  release();
  if (b == 0) b = 16;
  hipError_t e = hipMalloc(&p, b);
  if (e != hipSuccess) {
    p = nullptr;
    return fail(FE_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
  }
  bytes = b;
  return FE_OK;
}

// ---------------------------------------------------------------- profiling
namespace {
struct ProfRecord {
  std::string name;
  hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRecord> g_prof;
bool g_graphs_on = true;
}  // namespace

bool prof_enabled() { return g_prof_on; }
bool graphs_enabled() { return g_graphs_on; }
void set_graphs_enabled(bool on) { g_graphs_on = on; }

ProfScope::ProfScope(const char* name, hipStream_t s) : slot(-1), stream(s) {
  if (!g_prof_on) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  ProfRecord r;
  r.name = name;
  if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) return;
  (void)hipEventRecord(r.a, s);
  slot = (int)g_prof.size();
  g_prof.push_back(r);
}

ProfScope::~ProfScope() {
  if (slot < 0) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  (void)hipEventRecord(g_prof[slot].b, stream);
}

}  // namespace fe

using namespace fe;

static fe_status build_coarse_inverse(fe_problem* p, hipStream_t s);
static fe_status ensure_dinv(fe_problem* p, int li, hipStream_t s);

extern "C" {

const char* fe_last_error(void) { return g_last_error.c_str(); }

void fe_prof_enable(int enable) { g_prof_on = enable != 0; }
void fe_set_graphs(int enable) { fe::set_graphs_enabled(enable != 0); }

void fe_prof_reset(void) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto& r : g_prof) {
    (void)hipEventSynchronize(r.b);
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  g_prof.clear();
}

fe_status fe_prof_query(const char* name, int* count, double* total_ms) {
  if (!name || !count || !total_ms) return fail(FE_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(g_prof_mu);
  int c = 0;
  double t = 0.0;
  for (auto& r : g_prof) {
    if (r.name != name) continue;
    FE_HIP_CHECK(hipEventSynchronize(r.b));
    float ms = 0.f;
    FE_HIP_CHECK(hipEventElapsedTime(&ms, r.a, r.b));
    ++c;
    t += ms;
  }
  *count = c;
  *total_ms = t;
  return FE_OK;
}

// ---------------------------------------------------------------- problem
fe_status fe_problem_create(const fe_problem_desc* desc, void* stream, fe_problem** out) {
  if (!desc || !out) return fail(FE_EINVAL, "null argument");
  *out = nullptr;
  if (desc->dim != 2 && desc->dim != 3) return fail(FE_EINVAL, "dim must be 2 or 3");
  if (desc->degree < 1 || desc->degree > kMaxDegree) return fail(FE_EINVAL, "degree must be in 1..8");
  if (desc->n < 1 || desc->n > 4096) return fail(FE_EINVAL, "n out of range");
  if (desc->geometry != FE_GEOM_CARTESIAN && desc->geometry != FE_GEOM_DEFORMED)
    return fail(FE_EINVAL, "unknown geometry");
  if (desc->geometry == FE_GEOM_DEFORMED && desc->dim != 3)
    return fail(FE_EUNSUPPORTED, "deformed geometry is implemented for d = 3");
  if (desc->bc != 0 && desc->bc != 1) return fail(FE_EINVAL, "bc must be 0 or 1");
  // det of x + amp prod sin(2 pi x_b) (1,1,1) is 1 + 2 pi amp (c s s + s c s + s s c), whose
  // bracket ranges over [-2/sqrt(3), 2/sqrt(3)]: the map folds for |amp| >= sqrt(3) / (4 pi)
  if (desc->geometry == FE_GEOM_DEFORMED && !(std::fabs(desc->deform_amp) < std::sqrt(3.0) / (4.0 * M_PI)))
    return fail(FE_EINVAL, "deformation amplitude folds the mesh (|amp| must be < sqrt(3)/(4 pi))");
  {
    const int64_t K = desc->degree + 1;
    int64_t len = K * K * (int64_t)desc->n * desc->n;
    if (desc->dim == 3) len *= K * desc->n;
    if (len > (int64_t)1 << 33) return fail(FE_EINVAL, "problem too large");
  }
  hipStream_t s = (hipStream_t)stream;
  fe_problem* p = new fe_problem();
  p->desc = *desc;
  p->dim = desc->dim;
  p->k = desc->degree;
  p->K = desc->degree + 1;
  p->bc = desc->bc;
  p->setup_stream = s;

  // level hierarchy by uniform bisection: n_l = n0 * 2^l
  int n0 = desc->n_coarse;
  if (n0 <= 0) {
    n0 = desc->n;
    while (n0 % 2 == 0 && n0 > 1) n0 /= 2;
  }
  {
    int m = desc->n;
    while (m > n0 && m % 2 == 0) m /= 2;
    if (m != n0) {
      delete p;
      return fail(FE_EINVAL, "n must equal n_coarse * 2^L");
    }
  }
  std::vector<int> ns;
  for (int m = desc->n; m >= n0; m /= 2) {
    ns.push_back(m);
    if (m == n0) break;
  }
  p->levels.resize(ns.size());
  for (size_t i = 0; i < ns.size(); ++i) {
    Level& L = p->levels[ns.size() - 1 - i];
    L.n = ns[i];
    L.h = 1.0 / ns[i];
    L.n_cells = p->dim == 3 ? (int64_t)L.n * L.n * L.n : (int64_t)L.n * L.n;
    L.len = L.n_cells * (p->dim == 3 ? (int64_t)p->K * p->K * p->K : (int64_t)p->K * p->K);
  }

  // 1D reference data
  const int K = p->K, k = p->k, M = 2 * k - 1;
  p->B = mass_1d(k);
  p->D = stiffness_1d(k);
  p->P0 = prolongation_1d(k, 0);
  p->P1 = prolongation_1d(k, 1);
  {
    // two-interval patch on [0, 2] with unit cells, interior nodes only
    const int NP = 2 * k + 1;
    std::vector<double> Kp(NP * NP, 0.0), Mp(NP * NP, 0.0);
    for (int e = 0; e < 2; ++e)
      for (int i = 0; i < K; ++i)
        for (int j = 0; j < K; ++j) {
          Kp[(k * e + i) * NP + k * e + j] += p->D[i * K + j];
          Mp[(k * e + i) * NP + k * e + j] += p->B[i * K + j];
        }
    std::vector<double> Ki(M * M), Mi(M * M);
    for (int i = 0; i < M; ++i)
      for (int j = 0; j < M; ++j) {
        Ki[i * M + j] = Kp[(i + 1) * NP + j + 1];
        Mi[i * M + j] = Mp[(i + 1) * NP + j + 1];
      }
    if (!sym_generalized_eig(M, Ki, Mi, p->S, p->lam)) {
      delete p;
      return fail(FE_EINVAL, "patch eigenproblem failed");
    }
  }
  std::vector<double> host;
  auto put = [&](const std::vector<double>& v) {
    int off = (int)host.size();
    host.insert(host.end(), v.begin(), v.end());
    while (host.size() % 4) host.push_back(0.0);
    return off;
  };
  p->co.off_B = put(p->B);
  p->co.off_D = put(p->D);
  p->co.off_P0 = put(p->P0);
  p->co.off_P1 = put(p->P1);
  {
    std::vector<double> t0(p->P0.size()), t1(p->P1.size());
    for (int i = 0; i < K; ++i)
      for (int j = 0; j < K; ++j) {
        t0[i * K + j] = p->P0[j * K + i];
        t1[i * K + j] = p->P1[j * K + i];
      }
    p->co.off_P0T = put(t0);
    p->co.off_P1T = put(t1);
  }
  {
    // the patch kernel reads the eigenvalues right after S (M*M entries)
    std::vector<double> sl(p->S);
    sl.insert(sl.end(), p->lam.begin(), p->lam.end());
    p->co.off_S = put(sl);
    p->co.off_lam = p->co.off_S + M * M;
  }
  if (p->dim == 3 && k >= 2) {
    // The two-cell patch is mirror symmetric, so every 1D eigenvector is even
    // or odd about the middle node c = k-1.  Modes are reordered evens first;
    // SE[je][a] (a = 0..c) and SO[jo][a] (a = 0..c-1) hold the left half of
    // the even and odd eigenvectors, followed by the M eigenvalues in that
    // order.  The patch kernels apply them to sums and differences of
    // mirrored nodes.
    const int c = k - 1, ne = c + 1, no = c;
    std::vector<int> even, odd;
    for (int j = 0; j < M; ++j) {
      double sym = 0.0;
      for (int a = 0; a < M; ++a) sym += p->S[a * M + j] * p->S[(M - 1 - a) * M + j];
      (sym > 0.0 ? even : odd).push_back(j);
    }
    if ((int)even.size() == ne && (int)odd.size() == no) {
      std::vector<double> seo, lm(M);
      for (int je = 0; je < ne; ++je)
        for (int a = 0; a <= c; ++a) seo.push_back(p->S[a * M + even[je]]);
      for (int jo = 0; jo < no; ++jo)
        for (int a = 0; a < c; ++a) seo.push_back(p->S[a * M + odd[jo]]);
      for (int je = 0; je < ne; ++je) lm[je] = p->lam[even[je]];
      for (int jo = 0; jo < no; ++jo) lm[ne + jo] = p->lam[odd[jo]];
      seo.insert(seo.end(), lm.begin(), lm.end());
      p->co.off_Seo = put(seo);
      {
        // inverse eigenvalue sums in that mode order, scaled by h^{2-d} per level
        std::vector<double> il;
        for (const Level& L : p->levels) {
          const double scale = 1.0 / L.h;
          for (int mz = 0; mz < M; ++mz)
            for (int my = 0; my < M; ++my)
              for (int mx = 0; mx < M; ++mx) il.push_back(scale / (lm[mx] + lm[my] + lm[mz]));
        }
        p->co.off_il = put(il);
      }
    }
  }
  std::vector<float> host32(host.begin(), host.end());
  fe_status st = p->coef64.alloc(host.size() * sizeof(double));
  if (st == FE_OK) st = p->coef32.alloc(host32.size() * sizeof(float));
  if (st == FE_OK) st = p->red_scratch.alloc(2048 * sizeof(double));
  if (st != FE_OK) {
    delete p;
    return st;
  }
  if (hipMemcpyAsync(p->coef64.p, host.data(), host.size() * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(p->coef32.p, host32.data(), host32.size() * sizeof(float), hipMemcpyHostToDevice, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    delete p;
    return fail(FE_EHIP, "copy of reference data failed");
  }

  if (desc->geometry == FE_GEOM_DEFORMED) {
    if (desc->coef.n_modes > 0) {
      if (!desc->coef.modes || !desc->coef.amp || !desc->coef.phase) {
        delete p;
        return fail(FE_EINVAL, "coefficient arrays missing");
      }
      p->modes.assign(desc->coef.modes, desc->coef.modes + 3 * desc->coef.n_modes);
      p->amp.assign(desc->coef.amp, desc->coef.amp + desc->coef.n_modes);
      p->phase.assign(desc->coef.phase, desc->coef.phase + desc->coef.n_modes);
    }
    st = setup_geometry(p, s);
    if (st != FE_OK) {
      delete p;
      return st;
    }
  }
  *out = p;
  return FE_OK;
}

void fe_problem_destroy(fe_problem* p) {
  if (!p) return;
  (void)hipDeviceSynchronize();
  solver_destroy(p);
  delete p;
}

int64_t fe_num_cells(const fe_problem* p) { return p ? p->levels.back().n_cells : 0; }
int64_t fe_cellvec_len(const fe_problem* p) { return p ? p->levels.back().len : 0; }
int64_t fe_num_dofs(const fe_problem* p) {
  if (!p) return 0;
  const int64_t N = (int64_t)p->k * p->levels.back().n + 1;
  return p->dim == 3 ? N * N * N : N * N;
}
int fe_num_levels(const fe_problem* p) { return p ? (int)p->levels.size() : 0; }
int fe_level_cells_1d(const fe_problem* p, int level) {
  if (!p || level < 0 || level >= (int)p->levels.size()) return -1;
  return p->levels[level].n;
}

static fe_status check_dt(fe_dtype dt) {
  if (dt != FE_F64 && dt != FE_F32) return fail(FE_EINVAL, "unknown dtype");
  return FE_OK;
}

fe_status fe_gather(const fe_problem* p, const void* xg, void* xc, fe_dtype dt, void* stream) {
  if (!p) return fail(FE_EINVAL, "null problem");
  FE_CHECK(check_dt(dt));
  FE_CHECK(check_ptr(xg, "x_glob"));
  FE_CHECK(check_ptr(xc, "x_cell"));
  return launch_gather(p, xg, xc, dt, (hipStream_t)stream);
}

fe_status fe_assemble(const fe_problem* p, const void* yc, void* yg, fe_dtype dt, void* stream) {
  if (!p) return fail(FE_EINVAL, "null problem");
  FE_CHECK(check_dt(dt));
  FE_CHECK(check_ptr(yc, "y_cell"));
  FE_CHECK(check_ptr(yg, "y_glob"));
  return launch_assemble(p, yc, yg, dt, (hipStream_t)stream);
}

fe_status fe_dss(const fe_problem* p, int level, void* v, int averaging, fe_dtype dt, void* stream) {
  if (!p) return fail(FE_EINVAL, "null problem");
  FE_CHECK(check_dt(dt));
  FE_CHECK(check_level(p, level));
  FE_CHECK(check_ptr(v, "v_cell"));
  return launch_dss(p, level, v, averaging ? 1 : 0, dt, (hipStream_t)stream);
}

fe_status fe_apply_level(const fe_problem* p, int level, const void* x, void* y, fe_dtype dt, void* stream) {
  if (!p) return fail(FE_EINVAL, "null problem");
  FE_CHECK(check_dt(dt));
  FE_CHECK(check_level(p, level));
  FE_CHECK(check_ptr(x, "x_cell"));
  FE_CHECK(check_ptr(y, "y_cell"));
  if (x == y) return fail(FE_EINVAL, "x and y must not alias");
  return launch_apply(p, level, x, y, dt, (hipStream_t)stream);
}

fe_status fe_apply(const fe_problem* p, const void* x, void* y, fe_dtype dt, void* stream) {
  return fe_apply_level(p, -1, x, y, dt, stream);
}

fe_status patch_fdm_inverse_level(const fe_problem* cp, int level, const void* r, void* z, fe_dtype dt, int factors,
                                  void* stream) {
  if (!cp) return fail(FE_EINVAL, "null problem");
  fe_problem* p = const_cast<fe_problem*>(cp);
  FE_CHECK(check_dt(dt));
  FE_CHECK(check_level(p, level));
  FE_CHECK(check_ptr(r, "r_cell"));
  FE_CHECK(check_ptr(z, "z_cell"));
  if (r == z) return fail(FE_EINVAL, "r and z must not alias");
  if (factors < 0 || factors > 3) return fail(FE_EINVAL, "factors must be 0, 1, 2 or 3");
  if (factors == 0 && p->desc.geometry != FE_GEOM_CARTESIAN)
    return fail(FE_EINVAL, "exact separable factors need the Cartesian mesh");
  if (factors != 0 && p->desc.geometry != FE_GEOM_DEFORMED)
    return fail(FE_EINVAL, "per-patch factors need the deformed geometry");
  hipStream_t s = (hipStream_t)stream;
  const int li = level < 0 ? (int)p->levels.size() - 1 : level;
  FE_CHECK(prepare_patch_inverse(p, li, dt, factors, s));   // no-op once prepared
  return launch_patch_inverse(p, li, r, z, p->levels[li].fdm_scratch[dt == FE_F64 ? 0 : 1].p, dt, factors, s);
}

fe_status fe_patch_prepare(fe_problem* p, int level, fe_dtype dt, int factors, void* stream) {
  if (!p) return fail(FE_EINVAL, "null problem");
  FE_CHECK(check_dt(dt));
  FE_CHECK(check_level(p, level));
  if (factors < 0 || factors > 3) return fail(FE_EINVAL, "factors must be 0, 1, 2 or 3");
  if (factors == 0 && p->desc.geometry != FE_GEOM_CARTESIAN)
    return fail(FE_EINVAL, "exact separable factors need the Cartesian mesh");
  if (factors != 0 && p->desc.geometry != FE_GEOM_DEFORMED)
    return fail(FE_EINVAL, "per-patch factors need the deformed geometry");
  const int li = level < 0 ? (int)p->levels.size() - 1 : level;
  return prepare_patch_inverse(p, li, dt, factors, (hipStream_t)stream);
}

fe_status patch_fdm_inverse(const fe_problem* p, const void* r, void* z, fe_dtype dt, int factors, void* stream) {
  return patch_fdm_inverse_level(p, -1, r, z, dt, factors, stream);
}

fe_status fe_prolongate_add(const fe_problem* p, int fl, const void* ec, void* ef, fe_dtype dt, void* stream) {
  if (!p) return fail(FE_EINVAL, "null problem");
  FE_CHECK(check_dt(dt));
  if (fl < 1 || fl >= (int)p->levels.size()) return fail(FE_EINVAL, "fine_level out of range");
  FE_CHECK(check_ptr(ec, "e_coarse"));
  FE_CHECK(check_ptr(ef, "e_fine"));
  return launch_prolongate_add(p, fl, ec, ef, dt, (hipStream_t)stream);
}

fe_status fe_restrict_residual(const fe_problem* p, int fl, const void* bf, const void* vf, void* bc, fe_dtype dt,
                               void* stream) {
  if (!p) return fail(FE_EINVAL, "null problem");
  FE_CHECK(check_dt(dt));
  if (fl < 1 || fl >= (int)p->levels.size()) return fail(FE_EINVAL, "fine_level out of range");
  FE_CHECK(check_ptr(bf, "b_fine"));
  if (vf) FE_CHECK(check_ptr(vf, "v_fine"));
  FE_CHECK(check_ptr(bc, "b_coarse"));
  return launch_restrict(p, fl, bf, vf, bc, dt, (hipStream_t)stream);
}

fe_status fe_jacobi_sweep(const fe_problem* cp, int level, const void* b, void* u, void* v, double omega,
                          int u_is_zero, fe_dtype dt, void* stream) {
  if (!cp) return fail(FE_EINVAL, "null problem");
  fe_problem* p = const_cast<fe_problem*>(cp);
  FE_CHECK(check_dt(dt));
  FE_CHECK(check_level(p, level));
  FE_CHECK(check_ptr(b, "b"));
  FE_CHECK(check_ptr(u, "u"));
  FE_CHECK(check_ptr(v, "v"));
  hipStream_t s = (hipStream_t)stream;
  const int li = level < 0 ? (int)p->levels.size() - 1 : level;
  FE_CHECK(ensure_dinv(p, li, s));
  Level& L = p->levels[li];
  if (!u_is_zero) FE_CHECK(launch_apply(p, li, u, v, dt, s));
  FE_CHECK(launch_jacobi_update(p, li, b, v, u, dt == FE_F64 ? L.dinv64.p : L.dinv32.p, omega, u_is_zero, dt, s));
  return launch_dss(p, li, u, 1, dt, s);
}

fe_status fe_rhs_manufactured(const fe_problem* p, void* b, void* stream) {
  if (!p) return fail(FE_EINVAL, "null problem");
  FE_CHECK(check_ptr(b, "b_cell"));
  if (p->desc.geometry == FE_GEOM_DEFORMED) return launch_rhs_general(p, b, (hipStream_t)stream);
  return launch_rhs_cartesian(p, b, (hipStream_t)stream);
}

fe_status fe_dot(const fe_problem* p, const void* a, const void* b, fe_dtype dt, double* out, void* stream) {
  if (!p || !out) return fail(FE_EINVAL, "null argument");
  FE_CHECK(check_dt(dt));
  FE_CHECK(check_ptr(a, "a"));
  FE_CHECK(check_ptr(b, "b"));
  hipStream_t s = (hipStream_t)stream;
  double* dev = p->red_scratch.as<double>() + 2040;
  FE_CHECK(dot_async(p, p->levels.back().len, a, b, dt, dev, s));
  FE_HIP_CHECK(hipMemcpyAsync(out, dev, sizeof(double), hipMemcpyDeviceToHost, s));
  FE_HIP_CHECK(hipStreamSynchronize(s));
  return FE_OK;
}

fe_status fe_assembled_norm2(const fe_problem* p, const void* r, fe_dtype dt, double* out, void* stream) {
  if (!p || !out) return fail(FE_EINVAL, "null argument");
  FE_CHECK(check_dt(dt));
  FE_CHECK(check_ptr(r, "r_cell"));
  hipStream_t s = (hipStream_t)stream;
  double* dev = p->red_scratch.as<double>() + 2040;
  FE_CHECK(assembled_norm2_async(p, -1, r, dt, dev, s));
  FE_HIP_CHECK(hipMemcpyAsync(out, dev, sizeof(double), hipMemcpyDeviceToHost, s));
  FE_HIP_CHECK(hipStreamSynchronize(s));
  return FE_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- setup helpers
namespace fe {

// Inverse of the interior block of the level-0 operator, by probing the cell-wise
// operator with unit vectors of the interior coarse nodes (one column at a time)
// and a dense Cholesky factorization.  FP64.
static fe_status build_coarse_inverse_impl(fe_problem* p, hipStream_t s) {
  const Level& L0 = p->levels[0];
  const int k = p->k, K = p->K, n0 = L0.n;
  const int N = k * n0 + 1, Ni = N - 2;
  const int ni = Ni * Ni * Ni;
  if (ni <= 0) { p->coarse_n = 0; return FE_OK; }
  if (ni > 3000) return fail(FE_EUNSUPPORTED, "coarse level too large for the dense coarse solve");
  const int64_t len = L0.len;
  const int K3 = K * K * K;
  // copies of every interior node: list of cell-wise indices
  std::vector<std::vector<int64_t>> copies(ni);
  for (int64_t e = 0; e < len; ++e) {
    const int64_t cell = e / K3;
    const int loc = (int)(e % K3);
    const int ix = loc % K, iy = (loc / K) % K, iz = loc / (K * K);
    const int cx = (int)(cell % n0), cy = (int)((cell / n0) % n0), cz = (int)(cell / ((int64_t)n0 * n0));
    const int gx = k * cx + ix, gy = k * cy + iy, gz = k * cz + iz;
    if (gx == 0 || gy == 0 || gz == 0 || gx == N - 1 || gy == N - 1 || gz == N - 1) continue;
    copies[(gx - 1) + Ni * ((gy - 1) + Ni * (gz - 1))].push_back(e);
  }
  const int batch = 64;
  DeviceBuf xin, yout;
  FE_CHECK(xin.alloc((size_t)batch * len * sizeof(double)));
  FE_CHECK(yout.alloc((size_t)batch * len * sizeof(double)));
  std::vector<double> hx((size_t)batch * len), hy((size_t)batch * len);
  std::vector<double> A((size_t)ni * ni, 0.0);
  for (int j0 = 0; j0 < ni; j0 += batch) {
    const int nb = std::min(batch, ni - j0);
    std::fill(hx.begin(), hx.end(), 0.0);
    for (int b = 0; b < nb; ++b)
      for (int64_t e : copies[j0 + b]) hx[(size_t)b * len + e] = 1.0;
    FE_HIP_CHECK(hipMemcpyAsync(xin.p, hx.data(), (size_t)nb * len * sizeof(double), hipMemcpyHostToDevice, s));
    for (int b = 0; b < nb; ++b)
      FE_CHECK(launch_apply(p, 0, xin.as<double>() + (size_t)b * len, yout.as<double>() + (size_t)b * len, FE_F64, s));
    FE_HIP_CHECK(hipMemcpyAsync(hy.data(), yout.p, (size_t)nb * len * sizeof(double), hipMemcpyDeviceToHost, s));
    FE_HIP_CHECK(hipStreamSynchronize(s));
    for (int b = 0; b < nb; ++b)
      for (int i = 0; i < ni; ++i) {
        double sum = 0.0;
        for (int64_t e : copies[i]) sum += hy[(size_t)b * len + e];
        A[(size_t)i * ni + j0 + b] = sum;
      }
  }
  // symmetrize, Cholesky, explicit inverse
  for (int i = 0; i < ni; ++i)
    for (int j = i + 1; j < ni; ++j) A[(size_t)i * ni + j] = A[(size_t)j * ni + i] = 0.5 * (A[(size_t)i * ni + j] + A[(size_t)j * ni + i]);
  std::vector<double>& Lc = A;  // in place lower Cholesky factor
  for (int j = 0; j < ni; ++j) {
    double d = Lc[(size_t)j * ni + j];
    for (int q = 0; q < j; ++q) d -= Lc[(size_t)j * ni + q] * Lc[(size_t)j * ni + q];
    if (!(d > 0.0)) return fail(FE_EINVAL, "coarse operator is not positive definite");
    d = std::sqrt(d);
    Lc[(size_t)j * ni + j] = d;
    for (int i = j + 1; i < ni; ++i) {
      double v = Lc[(size_t)i * ni + j];
      for (int q = 0; q < j; ++q) v -= Lc[(size_t)i * ni + q] * Lc[(size_t)j * ni + q];
      Lc[(size_t)i * ni + j] = v / d;
    }
  }
  std::vector<double> inv((size_t)ni * ni, 0.0), col(ni);
  for (int c = 0; c < ni; ++c) {
    // solve L L^T x = e_c
    for (int i = 0; i < ni; ++i) {
      double v = (i == c) ? 1.0 : 0.0;
      for (int q = 0; q < i; ++q) v -= Lc[(size_t)i * ni + q] * col[q];
      col[i] = v / Lc[(size_t)i * ni + i];
    }
    for (int i = ni - 1; i >= 0; --i) {
      double v = col[i];
      for (int q = i + 1; q < ni; ++q) v -= Lc[(size_t)q * ni + i] * col[q];
      col[i] = v / Lc[(size_t)i * ni + i];
    }
    for (int i = 0; i < ni; ++i) inv[(size_t)i * ni + c] = col[i];
  }
  FE_CHECK(p->coarse_inv.alloc(inv.size() * sizeof(double)));
  FE_HIP_CHECK(hipMemcpyAsync(p->coarse_inv.p, inv.data(), inv.size() * sizeof(double), hipMemcpyHostToDevice, s));
  FE_HIP_CHECK(hipStreamSynchronize(s));
  p->coarse_n = ni;
  return FE_OK;
}

}  // namespace fe

static fe_status build_coarse_inverse(fe_problem* p, hipStream_t s) { return fe::build_coarse_inverse_impl(p, s); }

static fe_status ensure_dinv(fe_problem* p, int li, hipStream_t s) {
  Level& L = p->levels[li];
  if (L.dinv_ready) return FE_OK;
  DeviceBuf d;
  FE_CHECK(d.alloc(L.len * sizeof(double)));
  if (p->desc.geometry == FE_GEOM_DEFORMED) FE_CHECK(launch_diag_general(p, li, d.p, FE_F64, s));
  else FE_CHECK(launch_diag_cartesian(p, li, d.p, FE_F64, s));
  FE_CHECK(launch_dss(p, li, d.p, 0, FE_F64, s));
  FE_CHECK(L.dinv64.alloc(L.len * sizeof(double)));
  FE_CHECK(L.dinv32.alloc(L.len * sizeof(float)));
  FE_CHECK(launch_make_dinv(p, li, d.as<double>(), L.dinv64.p, FE_F64, s));
  FE_CHECK(launch_make_dinv(p, li, d.as<double>(), L.dinv32.p, FE_F32, s));
  FE_HIP_CHECK(hipStreamSynchronize(s));
  L.dinv_ready = true;
  return FE_OK;
}

namespace fe {
// Set-up of the patch inverse on level li: the per-patch factors of a factor
// mode (deformed mesh) and the scratch of the two-pass kernels in dtype dt
// (allocated once, kept until the problem is destroyed).
fe_status prepare_patch_inverse(fe_problem* p, int li, fe_dtype dt, int factors, hipStream_t s) {
  Level& L = p->levels[li];
  if (factors != 0 && !L.patch_eig_ready[factors]) FE_CHECK(setup_patch_factors(p, li, factors, s));
  if (!fused_patch_supported(p, factors != 0))
    FE_CHECK(L.fdm_scratch[dt == FE_F64 ? 0 : 1].alloc(patch_scratch_bytes(p, li, dt)));
  return FE_OK;
}
fe_status ensure_dinv_level(fe_problem* p, int li, hipStream_t s) { return ::ensure_dinv(p, li, s); }
fe_status ensure_coarse_inverse(fe_problem* p, hipStream_t s) {
  if (p->coarse_ready) return FE_OK;
  FE_CHECK(::build_coarse_inverse(p, s));
  p->coarse_ready = true;
  return FE_OK;
}
}  // namespace fe
