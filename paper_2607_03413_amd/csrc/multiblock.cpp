// Multi-block direct stiffness summation (paper, Sec. 4.3, Algorithm 8) on a
// 7-block atlas: a centre cube and six caps between its faces and the faces
// of the cube of twice its size, each block an n^3 grid of Q_k cells with its
// own orientation (axis permutation and flips).  Macro-faces join 2 blocks,
// macro-lines 2 or 3, macro-vertices 3 or 4.
//
// DSS runs in two phases.  Phase 1: the structured cascade inside every block
// (the single-block DSS kernel; after it every copy of a node holds the sum of
// that node's copies in its own block).  Phase 2: three disjoint sets of
// inter-block DoFs, one launch each: macro-face DoFs (not on a block edge) as a
// fixed pairwise exchange between the two blocks' copies; macro-line DoFs (on
// a block edge, not a corner) and macro-vertex DoFs (block corners) gather one
// representative copy per sharing block -- the blocks' copies already agree,
// so adding every copy would count a block's sum several times -- and scatter
// the total to every copy.  The tables of phase 2 are built once from integer
// position keys of the block lattices (no floating point), so orientation is
// resolved at setup; the kernels only follow index lists.
#include <algorithm>
#include <array>
#include <unordered_map>

#include "fe_internal.h"

namespace fe {

fe_status launch_mb_pairs(void* v, const int32_t* pairs, int64_t n_pairs, fe_dtype dt, hipStream_t s);
fe_status launch_mb_gather_scatter(void* v, const int32_t* rep_ptr, const int32_t* rep, const int32_t* all_ptr,
                                   const int32_t* all, int64_t n_ent, fe_dtype dt, hipStream_t s);
fe_status launch_mb_scale(void* v, const double* w, int64_t n, fe_dtype dt, hipStream_t s);

namespace {

struct BlockSpec {
  int kind, axis, sign, perm[3], flips[3];
};
// (kind 0: centre; 1: cap of the given axis and sign), axis permutation, flips
const BlockSpec kBlocks[7] = {
    {0, 0, 0, {0, 1, 2}, {0, 0, 0}},  {1, 0, +1, {0, 1, 2}, {0, 0, 0}}, {1, 0, -1, {1, 0, 2}, {0, 1, 0}},
    {1, 1, +1, {2, 0, 1}, {0, 0, 1}}, {1, 1, -1, {0, 2, 1}, {1, 0, 0}}, {1, 2, +1, {1, 2, 0}, {0, 1, 1}},
    {1, 2, -1, {2, 1, 0}, {1, 1, 0}},
};

// Integer position of block-lattice point a (each a_d in [0, m]) in the
// cube-in-cube frame, scaled by m^2 / 2: centre X = (2 t - m) m; cap of axis e
// and sign s: X_e = s (m + t_0) m, X_f = (m + t_0)(2 t_1 - m), X_g = (m + t_0)(2 t_2 - m).
void block_key(int b, const int64_t a[3], int64_t m, int64_t X[3]) {
  const BlockSpec& B = kBlocks[b];
  int64_t t[3];
  for (int d = 0; d < 3; ++d) t[d] = B.flips[d] ? m - a[B.perm[d]] : a[B.perm[d]];
  if (B.kind == 0) {
    for (int d = 0; d < 3; ++d) X[d] = (2 * t[d] - m) * m;
    return;
  }
  int f = -1, g = -1;
  for (int d = 0; d < 3; ++d)
    if (d != B.axis) (f < 0 ? f : g) = d;
  const int64_t rad = m + t[0];
  X[B.axis] = B.sign * rad * m;
  X[f] = rad * (2 * t[1] - m);
  X[g] = rad * (2 * t[2] - m);
}

struct KeyHash {
  size_t operator()(const std::array<int64_t, 3>& k) const {
    uint64_t h = (uint64_t)k[0] * 0x9E3779B97F4A7C15ull;
    h ^= (uint64_t)k[1] + 0x632BE59BD9B4E019ull + (h << 6) + (h >> 2);
    h ^= (uint64_t)k[2] + 0x94D049BB133111EBull + (h << 6) + (h >> 2);
    return (size_t)h;
  }
};

}  // namespace
}  // namespace fe

struct fe_multiblock {
  int k = 1, K = 2, n = 1;
  int64_t block_len = 0, len = 0, n_nodes = 0;
  fe_problem* block = nullptr;   // one block's structured mesh: phase 1
  fe::DeviceBuf pairs, line_rep_ptr, line_rep, line_all_ptr, line_all, vert_rep_ptr, vert_rep, vert_all_ptr, vert_all;
  int64_t n_pairs = 0, n_lines = 0, n_verts = 0;
  fe::DeviceBuf inv_valence;     // 1 / (copies of the node) per entry, FP64
  ~fe_multiblock() {
    if (block) fe_problem_destroy(block);
  }
};

namespace fe {
namespace {

template <typename V>
fe_status upload_vec(DeviceBuf& buf, const std::vector<V>& h, hipStream_t s) {
  FE_CHECK(buf.alloc(std::max<size_t>(h.size(), 1) * sizeof(V)));
  if (!h.empty()) FE_HIP_CHECK(hipMemcpyAsync(buf.p, h.data(), h.size() * sizeof(V), hipMemcpyHostToDevice, s));
  return FE_OK;
}

fe_status mb_dss(fe_multiblock* M, void* v, int averaging, fe_dtype dt, hipStream_t s);

fe_status build_tables(fe_multiblock* M, hipStream_t s) {
  const int k = M->k, K = M->K, n = M->n;
  const int64_t m = (int64_t)k * n, K3 = (int64_t)K * K * K, ncell = (int64_t)n * n * n;
  // copies of every block-boundary lattice node, by position key
  struct Copy {
    int32_t entry;
    int8_t block, nbnd;
  };
  std::unordered_map<std::array<int64_t, 3>, std::vector<Copy>, KeyHash> nodes;
  int64_t interior_nodes = 0;
  for (int b = 0; b < 7; ++b)
    for (int64_t e = 0; e < ncell; ++e) {
      const int64_t c[3] = {e % n, (e / n) % n, e / ((int64_t)n * n)};
      for (int64_t i = 0; i < K3; ++i) {
        const int64_t a[3] = {k * c[0] + i % K, k * c[1] + (i / K) % K, k * c[2] + i / (K * K)};
        int nb = 0;
        for (int d = 0; d < 3; ++d) nb += (a[d] == 0 || a[d] == m);
        if (nb == 0) continue;
        std::array<int64_t, 3> X;
        block_key(b, a, m, X.data());
        nodes[X].push_back(Copy{(int32_t)(b * M->block_len + e * K3 + i), (int8_t)b, (int8_t)nb});
      }
    }
  // interior lattice nodes of a block (not on its boundary): (m - 1)^3 each
  interior_nodes = 7 * (m - 1) * (m - 1) * (m - 1);
  M->n_nodes = interior_nodes + (int64_t)nodes.size();
  std::vector<int32_t> pairs, lrp{0}, lr, lap{0}, la, vrp{0}, vr, vap{0}, va;
  // deterministic order: sort the shared keys
  std::vector<const std::array<int64_t, 3>*> keys;
  for (auto& kv : nodes) keys.push_back(&kv.first);
  std::sort(keys.begin(), keys.end(), [](const std::array<int64_t, 3>* x, const std::array<int64_t, 3>* y) {
    return *x < *y;
  });
  for (const auto* key : keys) {
    std::vector<Copy>& cp = nodes[*key];
    std::sort(cp.begin(), cp.end(), [](const Copy& x, const Copy& y) { return x.entry < y.entry; });
    int nblk = 0;
    for (size_t j = 0; j < cp.size(); ++j)
      if (j == 0 || cp[j].block != cp[j - 1].block) ++nblk;
    if (nblk < 2) continue;   // on the outer boundary of one block only
    const int ent = cp[0].nbnd;   // 1: macro-face, 2: macro-line, 3: macro-vertex
    if (ent == 1) {
      if (nblk != 2) return fail(FE_EINVAL, "a macro-face node is shared by more than two blocks");
      std::vector<int32_t> A, B;
      for (const Copy& c : cp) (c.block == cp[0].block ? A : B).push_back(c.entry);
      if (A.size() != B.size()) return fail(FE_EINVAL, "non-conforming macro-face");
      for (size_t j = 0; j < A.size(); ++j) {
        pairs.push_back(A[j]);
        pairs.push_back(B[j]);
      }
      continue;
    }
    std::vector<int32_t>& rp = ent == 2 ? lrp : vrp;
    std::vector<int32_t>& r = ent == 2 ? lr : vr;
    std::vector<int32_t>& ap = ent == 2 ? lap : vap;
    std::vector<int32_t>& al = ent == 2 ? la : va;
    for (size_t j = 0; j < cp.size(); ++j) {
      if (j == 0 || cp[j].block != cp[j - 1].block) r.push_back(cp[j].entry);   // one representative per block
      al.push_back(cp[j].entry);
    }
    rp.push_back((int32_t)r.size());
    ap.push_back((int32_t)al.size());
  }
  M->n_pairs = (int64_t)pairs.size() / 2;
  M->n_lines = (int64_t)lrp.size() - 1;
  M->n_verts = (int64_t)vrp.size() - 1;
  FE_CHECK(upload_vec(M->pairs, pairs, s));
  FE_CHECK(upload_vec(M->line_rep_ptr, lrp, s));
  FE_CHECK(upload_vec(M->line_rep, lr, s));
  FE_CHECK(upload_vec(M->line_all_ptr, lap, s));
  FE_CHECK(upload_vec(M->line_all, la, s));
  FE_CHECK(upload_vec(M->vert_rep_ptr, vrp, s));
  FE_CHECK(upload_vec(M->vert_rep, vr, s));
  FE_CHECK(upload_vec(M->vert_all_ptr, vap, s));
  FE_CHECK(upload_vec(M->vert_all, va, s));
  // copies per node, by the summing DSS of a vector of ones
  FE_CHECK(M->inv_valence.alloc(M->len * sizeof(double)));
  FE_CHECK(launch_fill(M->len, M->inv_valence.p, 1.0, FE_F64, s));
  FE_CHECK(mb_dss(M, M->inv_valence.p, 0, FE_F64, s));
  std::vector<double> h(M->len);
  FE_HIP_CHECK(hipMemcpyAsync(h.data(), M->inv_valence.p, M->len * sizeof(double), hipMemcpyDeviceToHost, s));
  FE_HIP_CHECK(hipStreamSynchronize(s));
  for (double& x : h) x = 1.0 / x;
  FE_HIP_CHECK(hipMemcpyAsync(M->inv_valence.p, h.data(), M->len * sizeof(double), hipMemcpyHostToDevice, s));
  FE_HIP_CHECK(hipStreamSynchronize(s));
  return FE_OK;
}

fe_status mb_dss(fe_multiblock* M, void* v, int averaging, fe_dtype dt, hipStream_t s) {
  const size_t es = dt == FE_F64 ? 8 : 4;
  // phase 1: the structured cascade inside every block
  for (int b = 0; b < 7; ++b)
    FE_CHECK(launch_dss(M->block, -1, (char*)v + (size_t)b * M->block_len * es, 0, dt, s));
  // phase 2: macro-faces (pairs), macro-lines, macro-vertices
  {
    ProfScope ps("mb_interblock", s);
    FE_CHECK(launch_mb_pairs(v, M->pairs.as<int32_t>(), M->n_pairs, dt, s));
    FE_CHECK(launch_mb_gather_scatter(v, M->line_rep_ptr.as<int32_t>(), M->line_rep.as<int32_t>(),
                                      M->line_all_ptr.as<int32_t>(), M->line_all.as<int32_t>(), M->n_lines, dt, s));
    FE_CHECK(launch_mb_gather_scatter(v, M->vert_rep_ptr.as<int32_t>(), M->vert_rep.as<int32_t>(),
                                      M->vert_all_ptr.as<int32_t>(), M->vert_all.as<int32_t>(), M->n_verts, dt, s));
  }
  if (averaging) FE_CHECK(launch_mb_scale(v, M->inv_valence.as<double>(), M->len, dt, s));
  return FE_OK;
}

}  // namespace
}  // namespace fe

using namespace fe;

extern "C" {

fe_status fe_multiblock_create(int degree, int n, void* stream, fe_multiblock** out) {
  if (!out) return fail(FE_EINVAL, "null argument");
  *out = nullptr;
  if (degree < 1 || degree > kMaxDegree) return fail(FE_EINVAL, "degree must be in 1..8");
  if (n < 1 || n > 256) return fail(FE_EINVAL, "n out of range");
  const int64_t K = degree + 1;
  if (7 * K * K * K * (int64_t)n * n * n >= ((int64_t)1 << 31))
    return fail(FE_EINVAL, "multi-block vector too long for 32-bit entry tables");
  hipStream_t s = (hipStream_t)stream;
  fe_multiblock* M = new fe_multiblock();
  M->k = degree;
  M->K = degree + 1;
  M->n = n;
  M->block_len = K * K * K * (int64_t)n * n * n;
  M->len = 7 * M->block_len;
  fe_problem_desc bd{};
  bd.dim = 3;
  bd.degree = degree;
  bd.n = n;
  bd.geometry = FE_GEOM_CARTESIAN;
  bd.bc = 0;
  bd.n_coarse = n;
  fe_status st = fe_problem_create(&bd, stream, &M->block);
  if (st == FE_OK) st = build_tables(M, s);
  if (st != FE_OK) {
    delete M;
    return st;
  }
  *out = M;
  return FE_OK;
}

void fe_multiblock_destroy(fe_multiblock* M) {
  if (!M) return;
  (void)hipDeviceSynchronize();
  delete M;
}

int64_t fe_multiblock_len(const fe_multiblock* M) { return M ? M->len : 0; }
int64_t fe_multiblock_num_nodes(const fe_multiblock* M) { return M ? M->n_nodes : 0; }

fe_status fe_multiblock_counts(const fe_multiblock* M, int64_t* counts) {
  if (!M || !counts) return fail(FE_EINVAL, "null argument");
  counts[0] = M->n_pairs;
  counts[1] = M->n_lines;
  counts[2] = M->n_verts;
  return FE_OK;
}

fe_status fe_multiblock_dss(fe_multiblock* M, void* v, int averaging, fe_dtype dt, void* stream) {
  if (!M) return fail(FE_EINVAL, "null multi-block mesh");
  if (dt != FE_F64 && dt != FE_F32) return fail(FE_EINVAL, "unknown dtype");
  FE_CHECK(check_ptr(v, "v"));
  return mb_dss(M, v, averaging ? 1 : 0, dt, (hipStream_t)stream);
}

}  // extern "C"
