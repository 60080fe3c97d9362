// Locally refined hierarchy and the cell-wise local multigrid (paper, Sec. 3.2,
// Algorithms 4 and 5; Sec. 4.2-4.3; Sec. 5).
//
// The refinement tree is built on the host from a description (uniform levels,
// then levels refined toward a feature), made 2:1 balanced across faces, edges
// and vertices, and stored level by level in bricks of 8 children (see
// k_adapt.hip for the layout).  Active-mesh vectors live in "level layout":
// the level blocks concatenated, each level's cells in brick order, zeros on
// refined cells.  No hanging-node constraint appears anywhere: the smoother
// runs the structured DSS cascade on the level meshes, masking the
// refinement edge on both sides (the edge set is found at setup by one DSS of
// a face marker, Sec. 5), and the transfers act on unassembled residuals
// (lemma on the residual transfer).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <unordered_map>
#include <unordered_set>

#include "fe_internal.h"

namespace fe {

fe_status ensure_coarse_inverse(fe_problem* p, hipStream_t s);
fe_status launch_apply_cells(const fe_problem* p, int64_t n_cells, double h, const double* x, double* y, double alpha,
                             double beta, const double* b, hipStream_t s);
fe_status launch_diag_cells(const fe_problem* p, int64_t n_cells, double h, double* d, hipStream_t s);
fe_status launch_adss(int K, double* v, const int32_t* nbr, int64_t n_bricks, int averaging, hipStream_t s);
fe_status launch_aedge_flags(int K, double* m, const int32_t* coords, const int32_t* nbr, int64_t n_cells, int n_l,
                             hipStream_t s);
fe_status launch_amake_dinv(int K, double* dinv, const double* d, const double* kap, const double* em,
                            const int32_t* coords, int64_t n_cells, int n_l, hipStream_t s);
fe_status launch_ajacobi(double* u, const double* b, const double* v, const double* dinv, double omega, int64_t n,
                         int u_zero, hipStream_t s);
fe_status launch_aactive(double* dst, const double* src, const uint8_t* refined, int K3, int64_t n, int mode,
                         hipStream_t s);
fe_status launch_amask(int K, double* x, const uint8_t* refined, const int32_t* coords, int64_t n_cells, int n_l,
                       hipStream_t s);
fe_status launch_arhs(int K, double* b, const int32_t* coords, const uint8_t* refined, const double* tab, int nq,
                      int64_t n_cells, double h, hipStream_t s);
fe_status launch_aprolong(int K, const double* ec, double* ef, const int32_t* parent, int64_t n_bricks,
                          const double* P0, const double* P1, hipStream_t s);
fe_status launch_arestrict(int K, const double* bf, const double* vf, double* bc, const int32_t* parent,
                           int64_t n_bricks, const double* P0, const double* P1, hipStream_t s);

struct ALevel {
  int64_t n_cells = 0, n_bricks = 0;   // level 0: one cell, no bricks
  int n1 = 1;                          // 2^l cells per direction of the full level-l grid
  double h = 1.0;
  int64_t off = 0, len = 0;            // entry offset and length in level layout
  std::vector<int32_t> coords;         // 3 per cell
  std::vector<uint8_t> refined;        // per cell
  std::vector<int32_t> parent, nbr;    // per brick: parent cell on level l-1; 6 face-neighbour bricks
  DeviceBuf d_coords, d_refined, d_parent, d_nbr;
  DeviceBuf dinv, e, b, v;             // FP64
};

}  // namespace fe

struct fe_adaptive {
  fe_adaptive_desc desc{};
  int k = 1, K = 2;
  fe_problem* base = nullptr;          // one-cell problem: 1D data, coarse solve, reductions
  std::vector<fe::ALevel> levels;
  int64_t total_len = 0;
  int64_t active_cells = 0;
  fe::DeviceBuf rhs_tab;
  int rhs_nq = 0;
  // outer CG vectors (level layout) and device scalars
  fe::DeviceBuf r, z, pv, q, dscal;
  hipStream_t cs = nullptr;
  ~fe_adaptive() {
    if (cs) (void)hipStreamDestroy(cs);
    if (base) fe_problem_destroy(base);
  }
};

namespace fe {
namespace {

using Key = uint64_t;
inline Key pack(int64_t x, int64_t y, int64_t z) { return ((Key)x << 42) | ((Key)y << 21) | (Key)z; }

// Refinement predicate: the cell centre within band * h of the feature
// (squared distances; exact for dyadic centres, radii and bands).
bool feature_mark(const fe_adaptive_desc& d, int l, int64_t cx, int64_t cy, int64_t cz) {
  const double h = std::ldexp(1.0, -l);
  const double c[3] = {(cx + 0.5) * h, (cy + 0.5) * h, (cz + 0.5) * h};
  double d2 = 0.0;
  for (int a = 0; a < 3; ++a) {
    const double t = c[a] - d.center[a];
    d2 += t * t;
  }
  const double bh = d.band * h;
  if (d.feature == FE_FEATURE_SPHERE) {
    const double lo = std::max(d.radius - bh, 0.0), hi = d.radius + bh;
    return d2 >= lo * lo && d2 <= hi * hi;
  }
  return d2 <= bh * bh;
}

fe_status build_tree(fe_adaptive* A) {
  const fe_adaptive_desc& d = A->desc;
  const int L = d.global_refinements + d.adaptive_refinements;
  std::vector<std::unordered_set<Key>> present(L + 1), refined(L + 1);
  present[0].insert(pack(0, 0, 0));
  auto unpack = [](Key k, int64_t& x, int64_t& y, int64_t& z) {
    x = (int64_t)(k >> 42);
    y = (int64_t)((k >> 21) & ((1u << 21) - 1));
    z = (int64_t)(k & ((1u << 21) - 1));
  };
  for (int l = 0; l < L; ++l) {
    for (Key c : present[l]) {
      int64_t x, y, z;
      unpack(c, x, y, z);
      if (l < d.global_refinements || feature_mark(d, l, x, y, z)) refined[l].insert(c);
    }
    for (Key c : refined[l]) {
      int64_t x, y, z;
      unpack(c, x, y, z);
      for (int ch = 0; ch < 8; ++ch) present[l + 1].insert(pack(2 * x + (ch & 1), 2 * y + ((ch >> 1) & 1), 2 * z + (ch >> 2)));
    }
  }
  // 2:1 balance: a refined level-l cell needs its 26 level-l neighbours to exist
  for (int l = L - 1; l >= 1; --l) {
    const int64_t n_l = (int64_t)1 << l;
    std::vector<Key> todo(refined[l].begin(), refined[l].end());
    for (Key c : todo) {
      int64_t x, y, z;
      unpack(c, x, y, z);
      for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx) {
            const int64_t nx = x + dx, ny = y + dy, nz = z + dz;
            if (nx < 0 || ny < 0 || nz < 0 || nx >= n_l || ny >= n_l || nz >= n_l) continue;
            if (present[l].count(pack(nx, ny, nz))) continue;
            const Key par = pack(nx / 2, ny / 2, nz / 2);
            refined[l - 1].insert(par);
            for (int ch = 0; ch < 8; ++ch)
              present[l].insert(pack(2 * (nx / 2) + (ch & 1), 2 * (ny / 2) + ((ch >> 1) & 1), 2 * (nz / 2) + (ch >> 2)));
          }
    }
  }
  int Lt = L;
  while (Lt > 0 && refined[Lt - 1].empty()) --Lt;
  // canonical order: level 0 = (0,0,0); level l = children (child order) of the
  // refined cells of level l-1 in their order
  A->levels.assign(Lt + 1, ALevel());
  ALevel& L0 = A->levels[0];
  L0.n_cells = 1;
  L0.coords = {0, 0, 0};
  for (int l = 0; l <= Lt; ++l) {
    ALevel& V = A->levels[l];
    V.n1 = 1 << l;
    V.h = std::ldexp(1.0, -l);
    if (l > 0) {
      const ALevel& P = A->levels[l - 1];
      V.n_bricks = 0;
      for (int64_t e = 0; e < P.n_cells; ++e) {
        if (!P.refined[e]) continue;
        V.parent.push_back((int32_t)e);
        for (int ch = 0; ch < 8; ++ch) {
          V.coords.push_back(2 * P.coords[3 * e] + (ch & 1));
          V.coords.push_back(2 * P.coords[3 * e + 1] + ((ch >> 1) & 1));
          V.coords.push_back(2 * P.coords[3 * e + 2] + (ch >> 2));
        }
        ++V.n_bricks;
      }
      V.n_cells = 8 * V.n_bricks;
      if ((int64_t)present[l].size() != V.n_cells) return fail(FE_EINVAL, "refinement tree is not closed");
    }
    V.refined.resize(V.n_cells);
    for (int64_t e = 0; e < V.n_cells; ++e)
      V.refined[e] = refined[l].count(pack(V.coords[3 * e], V.coords[3 * e + 1], V.coords[3 * e + 2])) ? 1 : 0;
    if (l > 0) {
      // brick face neighbours: the brick of the parent's face neighbour (if refined)
      const ALevel& P = A->levels[l - 1];
      std::unordered_map<Key, int32_t> brick_of;   // parent cell coords -> brick
      for (int64_t b = 0; b < V.n_bricks; ++b) {
        const int64_t e = V.parent[b];
        brick_of[pack(P.coords[3 * e], P.coords[3 * e + 1], P.coords[3 * e + 2])] = (int32_t)b;
      }
      V.nbr.assign(6 * V.n_bricks, -1);
      for (int64_t b = 0; b < V.n_bricks; ++b) {
        const int64_t e = V.parent[b];
        for (int a = 0; a < 3; ++a)
          for (int sgn = 0; sgn < 2; ++sgn) {
            int64_t c[3] = {P.coords[3 * e], P.coords[3 * e + 1], P.coords[3 * e + 2]};
            c[a] += sgn ? 1 : -1;
            if (c[a] < 0 || c[a] >= P.n1) continue;
            auto it = brick_of.find(pack(c[0], c[1], c[2]));
            if (it != brick_of.end()) V.nbr[6 * b + 2 * a + sgn] = it->second;
          }
      }
    }
    for (uint8_t r : V.refined) A->active_cells += r ? 0 : 1;
  }
  return FE_OK;
}

template <typename V>
fe_status upload(DeviceBuf& buf, const std::vector<V>& h, hipStream_t s) {
  FE_CHECK(buf.alloc(std::max<size_t>(h.size(), 1) * sizeof(V)));
  if (!h.empty()) FE_HIP_CHECK(hipMemcpyAsync(buf.p, h.data(), h.size() * sizeof(V), hipMemcpyHostToDevice, s));
  return FE_OK;
}

const double* P0(const fe_adaptive* A) { return A->base->coef64.as<double>() + A->base->co.off_P0; }
const double* P1(const fe_adaptive* A) { return A->base->coef64.as<double>() + A->base->co.off_P1; }
int K3(const fe_adaptive* A) { return A->K * A->K * A->K; }

// Edge marker of level l (1 on the refinement edge E_l, per copy), into m:
// flags on faces without a level-l neighbour, one summing DSS, support.
fe_status edge_marker(fe_adaptive* A, int l, double* m, hipStream_t s) {
  ALevel& V = A->levels[l];
  if (l == 0) return launch_fill(V.len, m, 0.0, FE_F64, s);
  FE_CHECK(launch_aedge_flags(A->K, m, V.d_coords.as<int32_t>(), V.d_nbr.as<int32_t>(), V.n_cells, V.n1, s));
  return launch_adss(A->K, m, V.d_nbr.as<int32_t>(), V.n_bricks, 0, s);
}

fe_status setup_levels(fe_adaptive* A, hipStream_t s) {
  int64_t off = 0;
  for (ALevel& V : A->levels) {
    V.off = off;
    V.len = V.n_cells * K3(A);
    off += V.len;
  }
  A->total_len = off;
  for (size_t l = 0; l < A->levels.size(); ++l) {
    ALevel& V = A->levels[l];
    FE_CHECK(upload(V.d_coords, V.coords, s));
    FE_CHECK(upload(V.d_refined, V.refined, s));
    FE_CHECK(upload(V.d_parent, V.parent, s));
    FE_CHECK(upload(V.d_nbr, V.nbr, s));
    for (DeviceBuf* b : {&V.e, &V.b, &V.v}) FE_CHECK(b->alloc(V.len * sizeof(double)));
    if (l == 0) continue;
    // masked, valence-baked inverse diagonal (Algorithm 9): diagonal and copy
    // count summed by the cascade, the edge marker summed by the same cascade
    FE_CHECK(V.dinv.alloc(V.len * sizeof(double)));
    double* d = V.e.as<double>();
    double* kap = V.b.as<double>();
    double* em = V.v.as<double>();
    FE_CHECK(launch_diag_cells(A->base, V.n_cells, V.h, d, s));
    FE_CHECK(launch_adss(A->K, d, V.d_nbr.as<int32_t>(), V.n_bricks, 0, s));
    FE_CHECK(launch_fill(V.len, kap, 1.0, FE_F64, s));
    FE_CHECK(launch_adss(A->K, kap, V.d_nbr.as<int32_t>(), V.n_bricks, 0, s));
    FE_CHECK(edge_marker(A, (int)l, em, s));
    FE_CHECK(launch_amake_dinv(A->K, V.dinv.as<double>(), d, kap, em, V.d_coords.as<int32_t>(), V.n_cells, V.n1, s));
  }
  for (DeviceBuf* b : {&A->r, &A->z, &A->pv, &A->q}) FE_CHECK(b->alloc(std::max<int64_t>(A->total_len, 1) * sizeof(double)));
  FE_CHECK(A->dscal.alloc(64 * sizeof(double)));
  // load-vector tables: (k+2)-point Gauss rule, basis values at its points
  {
    const int nq = A->k + 2;
    std::vector<double> xq, wq;
    gauss_rule(nq, xq, wq);
    const std::vector<double> nodes = gll_nodes(A->k);
    std::vector<double> tab;
    for (int q = 0; q < nq; ++q)
      for (int i = 0; i < A->K; ++i) tab.push_back(lagrange_value(nodes, i, xq[q]));
    tab.insert(tab.end(), xq.begin(), xq.end());
    tab.insert(tab.end(), wq.begin(), wq.end());
    FE_CHECK(upload(A->rhs_tab, tab, s));
    A->rhs_nq = nq;
  }
  FE_CHECK(ensure_coarse_inverse(A->base, s));
  FE_HIP_CHECK(hipStreamSynchronize(s));
  return FE_OK;
}

// ---------------------------------------------------------------- local V-cycle (Algorithm 5)
struct MgParams {
  double omega;
  int nu_pre, nu_post;
};

// One fused masked Jacobi sweep (Algorithm 9) on level l: v = A u; u += omega
// dinv (b - v) per copy (dinv zero on the refinement edge and the boundary);
// u = S_bar u by the averaging cascade.
fe_status asweep(fe_adaptive* A, int l, bool u_zero, double omega, hipStream_t s) {
  ALevel& V = A->levels[l];
  double *u = V.e.as<double>(), *b = V.b.as<double>(), *v = V.v.as<double>();
  if (!u_zero) FE_CHECK(launch_apply_cells(A->base, V.n_cells, V.h, u, v, 1.0, 0.0, nullptr, s));
  FE_CHECK(launch_ajacobi(u, b, v, V.dinv.as<double>(), omega, V.len, u_zero ? 1 : 0, s));
  return launch_adss(A->K, u, V.d_nbr.as<int32_t>(), V.n_bricks, 1, s);
}

fe_status avcycle(fe_adaptive* A, int l, const MgParams& m, hipStream_t s) {
  ALevel& V = A->levels[l];
  if (l == 0) return launch_coarse_solve(A->base, V.b.p, V.e.p, FE_F64, s);
  for (int it = 0; it < m.nu_pre; ++it) FE_CHECK(asweep(A, l, it == 0, m.omega, s));
  if (m.nu_pre == 0) FE_CHECK(launch_fill(V.len, V.e.p, 0.0, FE_F64, s));
  // residual of the unmasked operator, restricted and accumulated into level l-1
  FE_CHECK(launch_apply_cells(A->base, V.n_cells, V.h, V.e.as<double>(), V.v.as<double>(), 1.0, 0.0, nullptr, s));
  ALevel& C = A->levels[l - 1];
  FE_CHECK(launch_arestrict(A->K, V.b.as<double>(), V.v.as<double>(), C.b.as<double>(), V.d_parent.as<int32_t>(),
                            V.n_bricks, P0(A), P1(A), s));
  FE_CHECK(avcycle(A, l - 1, m, s));
  FE_CHECK(launch_aprolong(A->K, C.e.as<double>(), V.e.as<double>(), V.d_parent.as<int32_t>(), V.n_bricks, P0(A),
                           P1(A), s));
  for (int it = 0; it < m.nu_post; ++it) FE_CHECK(asweep(A, l, false, m.omega, s));
  return FE_OK;
}

// Algorithm 4 from a zero iterate: level distribution of r, V-cycle, reassembly into z.
fe_status aprecondition(fe_adaptive* A, const double* r, double* z, const MgParams& m, hipStream_t s) {
  for (ALevel& V : A->levels)
    FE_CHECK(launch_aactive(V.b.as<double>(), r + V.off, V.d_refined.as<uint8_t>(), K3(A), V.len, 0, s));
  FE_CHECK(avcycle(A, (int)A->levels.size() - 1, m, s));
  for (ALevel& V : A->levels)
    FE_CHECK(launch_aactive(z + V.off, V.e.as<double>(), V.d_refined.as<uint8_t>(), K3(A), V.len, 0, s));
  return FE_OK;
}

// y = A_act x over the level layout (each level's operator on its cells; refined
// cells hold zeros in x, so their output is zero).
fe_status aapply(fe_adaptive* A, const double* x, double* y, hipStream_t s) {
  for (ALevel& V : A->levels) FE_CHECK(launch_apply_cells(A->base, V.n_cells, V.h, x + V.off, y + V.off, 1.0, 0.0, nullptr, s));
  return FE_OK;
}

fe_status amask(fe_adaptive* A, double* x, hipStream_t s) {
  for (ALevel& V : A->levels)
    FE_CHECK(launch_amask(A->K, x + V.off, V.d_refined.as<uint8_t>(), V.d_coords.as<int32_t>(), V.n_cells, V.n1, s));
  return FE_OK;
}

fe_status read_dev(fe_adaptive* A, int i, double* out, hipStream_t s) {
  FE_HIP_CHECK(hipMemcpyAsync(out, A->dscal.as<double>() + i, sizeof(double), hipMemcpyDeviceToHost, s));
  FE_HIP_CHECK(hipStreamSynchronize(s));
  return FE_OK;
}

fe_status check_mg_opts(const fe_pcg_opts* o) {
  if (!o) return fail(FE_EINVAL, "null opts");
  if (o->smoother != FE_SMOOTH_JACOBI) return fail(FE_EUNSUPPORTED, "the adaptive hierarchy smooths with Jacobi");
  if (o->inner != FE_F64) return fail(FE_EUNSUPPORTED, "the adaptive hierarchy runs in FP64");
  if (o->nu_pre < 0 || o->nu_post < 0 || o->maxit < 0 || !(o->tol >= 0.0) || !(o->omega > 0.0))
    return fail(FE_EINVAL, "bad multigrid options");
  return FE_OK;
}

fe_status check_vec(const void* p, const char* name) { return check_ptr(p, name); }

}  // namespace
}  // namespace fe

using namespace fe;

extern "C" {

fe_status fe_adaptive_create(const fe_adaptive_desc* d, void* stream, fe_adaptive** out) {
  if (!d || !out) return fail(FE_EINVAL, "null argument");
  *out = nullptr;
  if (d->degree < 1 || d->degree > 5) return fail(FE_EINVAL, "the adaptive hierarchy supports degrees 1..5");
  if (d->global_refinements < 0 || d->adaptive_refinements < 0 || d->global_refinements + d->adaptive_refinements > 12)
    return fail(FE_EINVAL, "refinement counts out of range (total at most 12)");
  if (d->feature != FE_FEATURE_SPHERE && d->feature != FE_FEATURE_POINT) return fail(FE_EINVAL, "unknown feature");
  if (!(d->band >= 0.0) || !(d->radius >= 0.0)) return fail(FE_EINVAL, "band and radius must be non-negative");
  hipStream_t s = (hipStream_t)stream;
  fe_adaptive* A = new fe_adaptive();
  A->desc = *d;
  A->k = d->degree;
  A->K = d->degree + 1;
  fe_problem_desc bd{};
  bd.dim = 3;
  bd.degree = d->degree;
  bd.n = 1;
  bd.geometry = FE_GEOM_CARTESIAN;
  bd.bc = 1;
  fe_status st = fe_problem_create(&bd, stream, &A->base);
  if (st == FE_OK) st = build_tree(A);
  if (st == FE_OK) st = setup_levels(A, s);
  if (st != FE_OK) {
    delete A;
    return st;
  }
  *out = A;
  return FE_OK;
}

void fe_adaptive_destroy(fe_adaptive* A) {
  if (!A) return;
  (void)hipDeviceSynchronize();
  delete A;
}

int fe_adaptive_num_levels(const fe_adaptive* A) { return A ? (int)A->levels.size() : 0; }
int64_t fe_adaptive_level_cells(const fe_adaptive* A, int l) {
  if (!A || l < 0 || l >= (int)A->levels.size()) return -1;
  return A->levels[l].n_cells;
}
int64_t fe_adaptive_level_offset(const fe_adaptive* A, int l) {
  if (!A || l < 0 || l > (int)A->levels.size()) return -1;
  return l == (int)A->levels.size() ? A->total_len : A->levels[l].off;
}
int64_t fe_adaptive_active_cells(const fe_adaptive* A) { return A ? A->active_cells : 0; }

fe_status fe_adaptive_level_info(const fe_adaptive* A, int l, int32_t* coords, uint8_t* refined) {
  if (!A) return fail(FE_EINVAL, "null hierarchy");
  if (l < 0 || l >= (int)A->levels.size()) return fail(FE_EINVAL, "level out of range");
  const ALevel& V = A->levels[l];
  if (coords) std::copy(V.coords.begin(), V.coords.end(), coords);
  if (refined) std::copy(V.refined.begin(), V.refined.end(), refined);
  return FE_OK;
}

fe_status fe_adaptive_brick_neighbors(const fe_adaptive* A, int l, int32_t* nbr, int32_t* parent) {
  if (!A) return fail(FE_EINVAL, "null hierarchy");
  if (l < 1 || l >= (int)A->levels.size()) return fail(FE_EINVAL, "level out of range (bricks exist on levels >= 1)");
  const ALevel& V = A->levels[l];
  if (nbr) std::copy(V.nbr.begin(), V.nbr.end(), nbr);
  if (parent) std::copy(V.parent.begin(), V.parent.end(), parent);
  return FE_OK;
}

fe_status fe_adaptive_edge_mask(fe_adaptive* A, int l, double* m, void* stream) {
  if (!A) return fail(FE_EINVAL, "null hierarchy");
  if (l < 0 || l >= (int)A->levels.size()) return fail(FE_EINVAL, "level out of range");
  FE_CHECK(check_vec(m, "mask"));
  return edge_marker(A, l, m, (hipStream_t)stream);
}

fe_status fe_adaptive_dss(fe_adaptive* A, int l, double* v, int averaging, void* stream) {
  if (!A) return fail(FE_EINVAL, "null hierarchy");
  if (l < 0 || l >= (int)A->levels.size()) return fail(FE_EINVAL, "level out of range");
  FE_CHECK(check_vec(v, "v"));
  return launch_adss(A->K, v, A->levels[l].d_nbr.as<int32_t>(), A->levels[l].n_bricks, averaging ? 1 : 0,
                     (hipStream_t)stream);
}

fe_status fe_adaptive_dinv(const fe_adaptive* A, int l, double* dinv, void* stream) {
  if (!A) return fail(FE_EINVAL, "null hierarchy");
  if (l < 1 || l >= (int)A->levels.size()) return fail(FE_EINVAL, "level out of range (smoothed levels are >= 1)");
  FE_CHECK(check_vec(dinv, "dinv"));
  const ALevel& V = A->levels[l];
  FE_HIP_CHECK(hipMemcpyAsync(dinv, V.dinv.p, V.len * sizeof(double), hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return FE_OK;
}

fe_status fe_adaptive_apply(fe_adaptive* A, const double* x, double* y, void* stream) {
  if (!A) return fail(FE_EINVAL, "null hierarchy");
  FE_CHECK(check_vec(x, "x"));
  FE_CHECK(check_vec(y, "y"));
  if (x == y) return fail(FE_EINVAL, "x and y must not alias");
  return aapply(A, x, y, (hipStream_t)stream);
}

fe_status fe_adaptive_prolongate_add(fe_adaptive* A, int fl, const double* ec, double* ef, void* stream) {
  if (!A) return fail(FE_EINVAL, "null hierarchy");
  if (fl < 1 || fl >= (int)A->levels.size()) return fail(FE_EINVAL, "fine_level out of range");
  FE_CHECK(check_vec(ec, "e_coarse"));
  FE_CHECK(check_vec(ef, "e_fine"));
  const ALevel& V = A->levels[fl];
  return launch_aprolong(A->K, ec, ef, V.d_parent.as<int32_t>(), V.n_bricks, P0(A), P1(A), (hipStream_t)stream);
}

fe_status fe_adaptive_restrict_add(fe_adaptive* A, int fl, const double* bf, const double* vf, double* bc,
                                   void* stream) {
  if (!A) return fail(FE_EINVAL, "null hierarchy");
  if (fl < 1 || fl >= (int)A->levels.size()) return fail(FE_EINVAL, "fine_level out of range");
  FE_CHECK(check_vec(bf, "b_fine"));
  FE_CHECK(check_vec(vf, "v_fine"));
  FE_CHECK(check_vec(bc, "b_coarse"));
  const ALevel& V = A->levels[fl];
  return launch_arestrict(A->K, bf, vf, bc, V.d_parent.as<int32_t>(), V.n_bricks, P0(A), P1(A), (hipStream_t)stream);
}

fe_status fe_adaptive_rhs_manufactured(fe_adaptive* A, double* b, void* stream) {
  if (!A) return fail(FE_EINVAL, "null hierarchy");
  FE_CHECK(check_vec(b, "b"));
  hipStream_t s = (hipStream_t)stream;
  for (ALevel& V : A->levels)
    FE_CHECK(launch_arhs(A->K, b + V.off, V.d_coords.as<int32_t>(), V.d_refined.as<uint8_t>(), A->rhs_tab.as<double>(),
                         A->rhs_nq, V.n_cells, V.h, s));
  return FE_OK;
}

fe_status fe_adaptive_precondition(fe_adaptive* A, const double* r, double* z, const fe_pcg_opts* o, void* stream) {
  if (!A) return fail(FE_EINVAL, "null hierarchy");
  FE_CHECK(check_mg_opts(o));
  FE_CHECK(check_vec(r, "r"));
  FE_CHECK(check_vec(z, "z"));
  if (r == z) return fail(FE_EINVAL, "r and z must not alias");
  return aprecondition(A, r, z, MgParams{o->omega, o->nu_pre, o->nu_post}, (hipStream_t)stream);
}

fe_status fe_adaptive_pcg(fe_adaptive* A, const double* b, double* x, const fe_pcg_opts* o, fe_pcg_report* rep,
                          void* stream) {
  using clk = std::chrono::steady_clock;
  if (!A) return fail(FE_EINVAL, "null hierarchy");
  FE_CHECK(check_mg_opts(o));
  if (o->stop != 1) return fail(FE_EUNSUPPORTED, "the adaptive solver stops on the energy measure (stop = 1)");
  FE_CHECK(check_vec(b, "b"));
  FE_CHECK(check_vec(x, "x"));
  hipStream_t s0 = (hipStream_t)stream;
  auto t0 = clk::now();
  FE_HIP_CHECK(hipStreamSynchronize(s0));
  if (!A->cs) FE_HIP_CHECK(hipStreamCreateWithFlags(&A->cs, hipStreamNonBlocking));
  hipStream_t s = A->cs;
  auto t1 = clk::now();
  const int64_t n = A->total_len;
  double *r = A->r.as<double>(), *z = A->z.as<double>(), *p = A->pv.as<double>(), *q = A->q.as<double>();
  double* dev = A->dscal.as<double>();
  const MgParams m{o->omega, o->nu_pre, o->nu_post};
  // r = b - A x with b and x masked on refined cells and Dirichlet copies
  FE_CHECK(amask(A, x, s));
  FE_CHECK(aapply(A, x, q, s));
  FE_CHECK(launch_cast(n, b, FE_F64, r, FE_F64, s));
  FE_CHECK(amask(A, r, s));
  FE_CHECK(launch_axpby(n, -1.0, q, 1.0, r, FE_F64, s));
  FE_CHECK(amask(A, r, s));
  FE_CHECK(aprecondition(A, r, z, m, s));
  FE_CHECK(launch_cast(n, z, FE_F64, p, FE_F64, s));
  double rho, rho0;
  FE_CHECK(dot_async(A->base, n, r, z, FE_F64, dev, s));
  FE_CHECK(read_dev(A, 0, &rho, s));
  rho0 = rho;
  fe_pcg_report R{};
  R.energy0 = rho0;
  R.energy = rho;
  fe_status result = FE_OK;
  int it = 0;
  bool done = !(rho0 > 0.0) ? (rho0 == 0.0) : false;
  if (!std::isfinite(rho0) || rho0 < 0.0) result = fail(FE_EBREAKDOWN, "<r, z> not positive at start");
  while (result == FE_OK && !done && it < o->maxit) {
    ++it;
    FE_CHECK(aapply(A, p, q, s));
    double pq;
    FE_CHECK(dot_async(A->base, n, p, q, FE_F64, dev, s));
    FE_CHECK(read_dev(A, 0, &pq, s));
    if (!(pq > 0.0) || !std::isfinite(pq)) {
      result = fail(FE_EBREAKDOWN, "<p, A p> <= 0");
      break;
    }
    const double alpha = rho / pq;
    FE_CHECK(launch_axpby(n, alpha, p, 1.0, x, FE_F64, s));
    FE_CHECK(launch_axpby(n, -alpha, q, 1.0, r, FE_F64, s));
    FE_CHECK(aprecondition(A, r, z, m, s));
    double rho_new;
    FE_CHECK(dot_async(A->base, n, r, z, FE_F64, dev, s));
    FE_CHECK(read_dev(A, 0, &rho_new, s));
    R.energy = rho_new;
    if (std::isfinite(rho_new) && rho_new >= 0.0 && rho_new <= o->tol * rho0) {
      done = true;
      break;
    }
    if (!(rho_new > 0.0)) {
      result = fail(FE_EBREAKDOWN, "<r, z> <= 0");
      break;
    }
    FE_CHECK(launch_axpby(n, 1.0, z, rho_new / rho, p, FE_F64, s));
    rho = rho_new;
  }
  if (result == FE_OK && !done) result = fail(FE_ENOTCONV, "maximum number of iterations reached");
  FE_HIP_CHECK(hipStreamSynchronize(s));
  auto t2 = clk::now();
  R.iters = it;
  R.converged = done ? 1 : 0;
  R.relres = rho0 > 0.0 ? std::sqrt(std::max(R.energy, 0.0) / rho0) : 0.0;
  R.t_setup = std::chrono::duration<double>(t1 - t0).count();
  R.t_solve = std::chrono::duration<double>(t2 - t1).count();
  if (rep) *rep = R;
  return result;
}

}  // extern "C"
