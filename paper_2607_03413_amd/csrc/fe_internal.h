// Internal declarations shared by the host side and the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fe.h"

namespace fe {

constexpr int kMaxDegree = 8;
constexpr int kMaxK = kMaxDegree + 1;

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
fe_status fail(fe_status st, const std::string& msg);

#define FE_HIP_CHECK(expr)                                                              \
  do {                                                                                  \
    hipError_t _e = (expr);                                                             \
    if (_e != hipSuccess)                                                               \
      return ::fe::fail(FE_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e));    \
  } while (0)

#define FE_CHECK(expr)                  \
  do {                                  \
    fe_status _s = (expr);              \
    if (_s != FE_OK) return _s;         \
  } while (0)

// ---------------------------------------------------------------- profiling
// Kernel launches go through prof_begin/prof_end so that per-family durations
// can be measured with events on the launch stream.
bool prof_enabled();     // per-kernel event timing switched on (fe_prof_enable)
bool graphs_enabled();   // the MG-PCG preconditioner may be replayed as a HIP graph (fe_set_graphs)
void set_graphs_enabled(bool on);

struct ProfScope {
  ProfScope(const char* name, hipStream_t s);
  ~ProfScope();
  int slot;
  hipStream_t stream;
};

// ---------------------------------------------------------------- 1D basis (host, FP64)
std::vector<double> gll_nodes(int k);
void gauss_rule(int n, std::vector<double>& x, std::vector<double>& w);
double lagrange_value(const std::vector<double>& nodes, int j, double x);
double lagrange_deriv(const std::vector<double>& nodes, int j, double x);
// K x K row-major, K = k+1
std::vector<double> mass_1d(int k);
std::vector<double> stiffness_1d(int k);
std::vector<double> prolongation_1d(int k, int c);
// Symmetric generalized eigenproblem A S = M S diag(lam), S^T M S = I (n x n row-major,
// eigenvalues ascending).  Cholesky of M then cyclic Jacobi rotations.
bool sym_generalized_eig(int n, const std::vector<double>& A, const std::vector<double>& M,
                         std::vector<double>& S, std::vector<double>& lam);

// ---------------------------------------------------------------- problem data
struct DeviceBuf {
  void* p = nullptr;
  size_t bytes = 0;
  ~DeviceBuf();
  fe_status alloc(size_t b);
  void release();
  template <typename T> T* as() const { return static_cast<T*>(p); }
};

// Constant 1D data for one dtype, laid out contiguously in one device buffer.
struct Coef1D {
  // offsets (in elements) into the buffer
  int off_B = 0, off_D = 0, off_P0 = 0, off_P1 = 0, off_diag = 0;
  int off_P0T = 0, off_P1T = 0;  // transposes of P0, P1 (the restriction reads their rows)
  int off_S = 0, off_lam = 0;   // Cartesian patch eigen-data, scaled for h = 1
  // 3D Cartesian, k >= 2: even/odd halves of the 1D patch eigenvectors,
  // SE[(k)][k] then SO[(k-1)][k-1], then the M eigenvalues in that mode order
  // (evens first); then per level l the M^3 entries h_l^{-1} / (lam_x + lam_y
  // + lam_z) in that mode order, index (mz*M + my)*M + mx, at off_il + l*M^3
  // (-1: not built)
  int off_Seo = -1, off_il = -1;
};

struct Level {
  int n = 0;              // cells per direction
  int64_t n_cells = 0;
  int64_t len = 0;        // cell-wise entries
  double h = 0.0;
  // deformed geometry: per-cell quadrature metric (6 per point), per dtype
  DeviceBuf metric64, metric32;
  // deformed geometry, metric formed in the apply kernel: coefficient per point, per dtype
  DeviceBuf kappa64, kappa32;
  // deformed geometry: per-patch 1D eigen-data, per factor mode and dtype
  DeviceBuf patch_eig64[4], patch_eig32[4];
  bool patch_eig_ready[4] = {false, false, false, false};
  // inverse assembled diagonal with valence and Dirichlet mask baked in
  DeviceBuf dinv64, dinv32;
  bool dinv_ready = false;
  // multigrid work vectors (allocated at solver setup), per dtype
  DeviceBuf e[2], b[2], v[2], t[2], w[2];
  DeviceBuf fdm_scratch[2];   // patch-major scratch of the patch inverse
  double lmax = 0.0;
  int lmax_key = -1;
  double omega = 0.7;          // Jacobi damping in use on this level
  double omega_auto = 0.0;     // cached automatic damping (0: not estimated)
};

struct Solver;

}  // namespace fe

struct fe_problem {
  fe_problem_desc desc{};
  int dim = 3, k = 1, K = 2;
  int bc = 1;
  std::vector<fe::Level> levels;     // 0 = coarsest
  hipStream_t setup_stream = nullptr;
  fe::DeviceBuf coef64, coef32;      // 1D reference matrices (see Coef1D)
  fe::DeviceBuf geo_tab64, geo_tab32;  // deformed geometry: basis values/derivatives at Gauss points
  fe::DeviceBuf geo_tabT64, geo_tabT32;  // their transposes PHI^T, DPHI^T (rows for the backward contractions)
  fe::Coef1D co;
  // host copies of the 1D data (FP64)
  std::vector<double> B, D, P0, P1, S, lam;
  // coefficient-field parameters (deformed geometry)
  std::vector<int32_t> modes;
  std::vector<double> amp, phase;
  double coef_scale = 1.0;
  // coarse dense inverse (FP64), over interior DoFs of level 0
  fe::DeviceBuf coarse_inv;
  int coarse_n = 0;
  bool coarse_ready = false;
  fe::DeviceBuf coarse_idx;          // (n_int) global index per interior coarse DoF
  fe::DeviceBuf red_scratch;         // reduction partials
  fe::DeviceBuf red_host_dummy;
  fe::Solver* solver = nullptr;
  // learned-factor MLP (see fe_mlp_*)
  fe::DeviceBuf mlp_params, mlp_adam_m, mlp_adam_v;
  int mlp_ready = 0;
  int64_t mlp_step = 0;
  // deformed geometry: 1 = the general apply forms the metric from the map
  // (reads kappa only), 0 = it streams the stored metric (fe_set_metric_mode)
  int metric_otf = 0;
};

namespace fe {

inline int ipow(int b, int e) { int r = 1; while (e-- > 0) r *= b; return r; }
inline const Level& level_of(const fe_problem* p, int l) {
  return p->levels[l < 0 ? p->levels.size() - 1 : l];
}
inline Level& level_of(fe_problem* p, int l) {
  return p->levels[l < 0 ? p->levels.size() - 1 : l];
}
fe_status check_level(const fe_problem* p, int l);
fe_status check_ptr(const void* ptr, const char* name);

// ---------------------------------------------------------------- kernel launchers
// Each returns FE_OK or a HIP error; arguments are validated by the caller.
fe_status launch_gather(const fe_problem* p, const void* xg, void* xc, fe_dtype dt, hipStream_t s);
fe_status launch_assemble(const fe_problem* p, const void* yc, void* yg, fe_dtype dt, hipStream_t s);
fe_status launch_dss(const fe_problem* p, int level, void* v, int averaging, fe_dtype dt, hipStream_t s);
fe_status launch_apply(const fe_problem* p, int level, const void* x, void* y, fe_dtype dt, hipStream_t s);
// y = alpha A x + beta b (b may be null: y = alpha A x; b may alias y)
fe_status launch_apply_ep(const fe_problem* p, int level, const void* x, void* y, double alpha, double beta,
                          const void* b, fe_dtype dt, hipStream_t s);
// Chebyshev step on cell-wise vectors: w = a v + c w (v may alias w); e = w (e_zero) or e + w
fe_status launch_cheb_update(int64_t n, double a, const void* v, double c, void* w, void* e, int e_zero,
                             fe_dtype dt, hipStream_t s);
fe_status launch_patch_inverse(const fe_problem* p, int level, const void* r, void* z, void* scratch,
                               fe_dtype dt, int factors, hipStream_t s);
// v = P r followed by the Chebyshev step of launch_cheb_update (w = a v + c w;
// e = w or e += w).  On 3D meshes served by the two-pass inverse the step runs
// inside the summing pass and v is neither written nor read (v may be null
// there); elsewhere v receives P r (it may alias w) and the update follows.
fe_status launch_patch_cheb(const fe_problem* p, int level, const void* r, void* v, void* scratch, fe_dtype dt,
                            int factors, double a, double c, void* w, void* e, int e_zero, hipStream_t s);
size_t patch_scratch_bytes(const fe_problem* p, int level, fe_dtype dt);
// the one-pass (scratch-free) patch inverse serves this problem and factor kind
bool fused_patch_supported(const fe_problem* p, bool per_patch);
// per-patch factors of `factors` and the patch scratch in dtype dt on level li
fe_status prepare_patch_inverse(fe_problem* p, int li, fe_dtype dt, int factors, hipStream_t s);
fe_status launch_prolongate_add(const fe_problem* p, int fine_level, const void* ec, void* ef,
                                fe_dtype dt, hipStream_t s);
fe_status launch_restrict(const fe_problem* p, int fine_level, const void* bf, const void* vf, void* bc,
                          fe_dtype dt, hipStream_t s);
fe_status launch_diag(const fe_problem* p, int level, void* d, fe_dtype dt, hipStream_t s);
fe_status launch_jacobi_update(const fe_problem* p, int level, const void* b, const void* v, void* u,
                               const void* dinv, double omega, int u_is_zero, fe_dtype dt, hipStream_t s);
fe_status launch_rhs(const fe_problem* p, void* b, hipStream_t s);
// blas-1 on cell-wise vectors (n entries)
fe_status launch_axpby(int64_t n, double a, const void* x, double b, void* y, fe_dtype dt, hipStream_t s);
// y = a x + b y, y FP64, x FP64 or FP32 (xdt)
fe_status launch_axpby_x(int64_t n, double a, const void* x, fe_dtype xdt, double b, double* y, hipStream_t s);
fe_status launch_cg_update(int64_t n, double rho, const double* pq, const double* p, const double* q, double* x,
                           double* r, hipStream_t s);
fe_status launch_cast(int64_t n, const void* src, fe_dtype st, void* dst, fe_dtype dtt, hipStream_t s);
fe_status launch_fill(int64_t n, void* x, double v, fe_dtype dt, hipStream_t s);
fe_status dot_async(const fe_problem* p, int64_t n, const void* a, const void* b, fe_dtype dt,
                    double* dev_out, hipStream_t s);
// <a, b> with a FP64 and b FP64 or FP32 (bdt), into *dev_out (device)
fe_status dot_async_x(const fe_problem* p, int64_t n, const double* a, const void* b, fe_dtype bdt, double* dev_out,
                      hipStream_t s);
fe_status assembled_norm2_async(const fe_problem* p, int level, const void* r, fe_dtype dt,
                                double* dev_out, hipStream_t s);
fe_status launch_coarse_solve(const fe_problem* p, const void* b0, void* e0, fe_dtype dt, hipStream_t s);
fe_status launch_average_convert(const fe_problem* p, int level, const double* r, void* out, fe_dtype dt,
                                 hipStream_t s);
fe_status launch_mask_boundary(const fe_problem* p, int level, void* v, fe_dtype dt, hipStream_t s);
fe_status launch_jacobi_avg(const fe_problem* p, int level, const void* u, const void* b, const void* v,
                            const void* dinv, void* out, double omega, int u_is_zero, fe_dtype dt, hipStream_t s);
fe_status launch_make_dinv(const fe_problem* p, int level, const double* d, void* dinv, fe_dtype dt, hipStream_t s);
fe_status launch_diag_cartesian(const fe_problem* p, int level, void* d, fe_dtype dt, hipStream_t s);
fe_status launch_diag_general(const fe_problem* p, int level, void* d, fe_dtype dt, hipStream_t s);
fe_status launch_rhs_cartesian(const fe_problem* p, void* b, hipStream_t s);
fe_status launch_rhs_general(const fe_problem* p, void* b, hipStream_t s);
fe_status launch_apply_general(const fe_problem* p, int level, const void* x, void* y, double alpha, double beta,
                               const void* b, fe_dtype dt, hipStream_t s);
fe_status finish_reduction(const fe_problem* p, int nparts, double* dev_out, hipStream_t s);
// deformed geometry setup (metric per level) and per-patch factors
fe_status setup_geometry(fe_problem* p, hipStream_t s);
fe_status setup_patch_factors(fe_problem* p, int level, int mode, hipStream_t s);
// solver
fe_status solver_setup(fe_problem* p, const fe_pcg_opts* o, hipStream_t s);
fe_status solver_vcycle(fe_problem* p, const fe_pcg_opts* o, fe_dtype dt, hipStream_t s);
void solver_destroy(fe_problem* p);

}  // namespace fe
