// Kernels of the locally refined hierarchy (paper, Sec. 3.2: adaptive
// multigrid with local smoothing; Sec. 4.3: the structured DSS cascade on
// refinement edges; Sec. 5: refinement-edge detection by one DSS).
//
// Storage: level l >= 1 holds all level-l cells (active or refined further),
// grouped in bricks of 8 -- the children of one refined level-(l-1) cell --
// brick b's child c = bx + 2 by + 4 bz at cell index 8 b + c; each cell keeps
// its (k+1)^3 values contiguously (local index x fastest).  Per brick the
// library keeps the parent cell index on level l-1 and the brick indices of
// the six face neighbours on level l (-1: no level-l cells there).  Every
// inter-cell address is therefore brick arithmetic plus at most one neighbour
// lookup per brick face; the transfers couple each brick with its parent
// only, through contiguous blocks.
#include "fe_internal.h"
#include "kernel_common.h"

namespace fe {

// ---------------------------------------------------------------- DSS cascade
// One axis pass of Algorithm 7 over a brick level: every interface pair normal
// to axis AX is summed and the sum written to both copies (halved when
// averaging: the averaging DSS S_bar).  Pairs inside a brick (children with
// bit AX = 0 and 1) and pairs between a brick and its +AX neighbour brick are
// handled by one thread per face entry; when the neighbour brick is absent the
// pair has no partner and is skipped.  Those skipped copies all lie on the
// refinement edge or on the domain boundary; their sums are wrong (the
// situation of the paper's L-shaped corner), and the smoother masks them on
// both sides, so they never reach an iterate.
template <typename T, int K, int AX>
__global__ void __launch_bounds__(256) k_adss_pass(T* __restrict__ v, const int32_t* __restrict__ nbr,
                                                   int64_t n_bricks, int averaging) {
  constexpr int K2 = K * K, K3 = K2 * K, k = K - 1;
  constexpr int A1 = AX == 0 ? 1 : 0, A2 = AX == 2 ? 1 : 2;   // the other two axes, ascending
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= n_bricks * 8 * K2) return;
  const int j = (int)(gid % K2);
  const int64_t t = gid / K2;
  const int s = (int)(t % 8);
  const int64_t b = t / 8;
  const int c_other = ((s & 1) << A1) | (((s >> 1) & 1) << A2);
  const int c_lo = c_other, c_hi = c_other | (1 << AX);
  int64_t bl = b, br = b;
  int cl = c_lo, cr = c_hi;
  if (s >= 4) {   // across the +AX brick face: high child of b with low child of the neighbour
    const int nb = nbr[b * 6 + 2 * AX + 1];
    if (nb < 0) return;
    cl = c_hi;
    br = nb;
    cr = c_lo;
  }
  int il[3], ir[3];
  il[A1] = ir[A1] = j % K;
  il[A2] = ir[A2] = j / K;
  il[AX] = k;
  ir[AX] = 0;
  const int64_t pl = (bl * 8 + cl) * K3 + il[0] + K * (il[1] + K * il[2]);
  const int64_t pr = (br * 8 + cr) * K3 + ir[0] + K * (ir[1] + K * ir[2]);
  T sum = v[pl] + v[pr];
  if (averaging) sum *= T(0.5);
  v[pl] = sum;
  v[pr] = sum;
}

// ---------------------------------------------------------------- refinement edge
// Marker of the edge detection of Sec. 5: 1 on every entry of a cell face that
// is interior to the cube and has no level-l cell behind it, 0 elsewhere.
template <typename T, int K>
__global__ void __launch_bounds__(256) k_aedge_flags(T* __restrict__ m, const int32_t* __restrict__ coords,
                                                     const int32_t* __restrict__ nbr, int64_t n_cells, int n_l) {
  constexpr int K3 = K * K * K, k = K - 1;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= n_cells * K3) return;
  const int64_t e = gid / K3;
  const int loc = (int)(gid - e * K3);
  const int i[3] = {loc % K, (loc / K) % K, loc / (K * K)};
  const int64_t b = e >> 3;
  const int c = (int)(e & 7);
  T flag = T(0);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int bit = (c >> a) & 1;
    const int ca = coords[e * 3 + a];
    // low face (s = 0) and high face (s = 1) of the cell along a
    if (i[a] == 0 && ca > 0 && bit == 0 && nbr[b * 6 + 2 * a] < 0) flag = T(1);
    if (i[a] == k && ca < n_l - 1 && bit == 1 && nbr[b * 6 + 2 * a + 1] < 0) flag = T(1);
  }
  m[gid] = flag;
}

// Masked, valence-baked inverse diagonal of Algorithm 9 on a brick level:
// dinv = kappa / d from the DSS-summed cell diagonals d and copy counts kappa,
// 0 on the refinement edge (summed edge marker > 0) and on the Dirichlet
// boundary of the cube (lattice coordinate 0 or k 2^l on some axis).
template <int K>
__global__ void __launch_bounds__(256) k_amake_dinv(double* __restrict__ dinv, const double* __restrict__ d,
                                                    const double* __restrict__ kap, const double* __restrict__ em,
                                                    const int32_t* __restrict__ coords, int64_t n_cells, int n_l) {
  constexpr int K3 = K * K * K, k = K - 1;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= n_cells * K3) return;
  const int64_t e = gid / K3;
  const int loc = (int)(gid - e * K3);
  const int i[3] = {loc % K, (loc / K) % K, loc / (K * K)};
  bool bnd = false;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int g = k * coords[e * 3 + a] + i[a];
    bnd = bnd || g == 0 || g == k * n_l;
  }
  dinv[gid] = (bnd || em[gid] != 0.0) ? 0.0 : kap[gid] / d[gid];
}

// ---------------------------------------------------------------- cell-wise updates
// Raw per-copy Jacobi update (the update step of Algorithm 9): u = u + omega dinv (b - v),
// or u = omega dinv b from a zero iterate.
__global__ void __launch_bounds__(256) k_ajacobi(double* __restrict__ u, const double* __restrict__ b,
                                                 const double* __restrict__ v, const double* __restrict__ dinv,
                                                 double omega, int64_t n, int u_zero) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double w = omega * dinv[i];
  u[i] = u_zero ? w * b[i] : u[i] + w * (b[i] - v[i]);
}

// Level distribution / reassembly (eqs. level_distribution, level_gather):
// dst = active ? src : 0 (mode 0), dst += active ? src : 0 (mode 1).
__global__ void __launch_bounds__(256) k_aactive(double* __restrict__ dst, const double* __restrict__ src,
                                                 const uint8_t* __restrict__ refined, int K3, int64_t n, int mode) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double s = refined[i / K3] ? 0.0 : src[i];
  dst[i] = mode ? dst[i] + s : s;
}

// Zero the copies on refined cells and on the Dirichlet boundary (in place).
template <int K>
__global__ void __launch_bounds__(256) k_amask(double* __restrict__ x, const uint8_t* __restrict__ refined,
                                               const int32_t* __restrict__ coords, int64_t n_cells, int n_l) {
  constexpr int K3 = K * K * K, k = K - 1;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= n_cells * K3) return;
  const int64_t e = gid / K3;
  const int loc = (int)(gid - e * K3);
  const int i[3] = {loc % K, (loc / K) % K, loc / (K * K)};
  bool z = refined[e] != 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int g = k * coords[e * 3 + a] + i[a];
    z = z || g == 0 || g == k * n_l;
  }
  if (z) x[gid] = 0.0;
}

// Manufactured load vector on the active cells of one level (refined cells 0):
// b_K,i = 3 pi^2 prod_a int_0^h sin(pi (c_a h + s)) phi_{i_a}(s / h) ds by a
// Gauss rule of NQ points (tables V[q][i] = phi_i(x_q), x_q, w_q on [0, 1]).
template <int K>
__global__ void __launch_bounds__(256) k_arhs(double* __restrict__ b, const int32_t* __restrict__ coords,
                                              const uint8_t* __restrict__ refined, const double* __restrict__ tab,
                                              int nq, int64_t n_cells, double h) {
  constexpr int K3 = K * K * K;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= n_cells * K3) return;
  const int64_t e = gid / K3;
  const int loc = (int)(gid - e * K3);
  if (refined[e]) {
    b[gid] = 0.0;
    return;
  }
  const int i[3] = {loc % K, (loc / K) % K, loc / (K * K)};
  const double* V = tab;                 // nq x K
  const double* xq = tab + nq * K;
  const double* wq = xq + nq;
  double prod = 3.0 * M_PI * M_PI;
  for (int a = 0; a < 3; ++a) {
    const double c = coords[e * 3 + a];
    double s = 0.0;
    for (int q = 0; q < nq; ++q) s += wq[q] * h * sin(M_PI * (c + xq[q]) * h) * V[q * K + i[a]];
    prod *= s;
  }
  b[gid] = prod;
}

// ---------------------------------------------------------------- transfers
// Algorithm 2 on a brick level: ef(8 b + c) += (P_cx x P_cy x P_cz) ec(parent(b))
// for the 8 children c of each brick, by three sum-factorized stages staged in
// LDS (z, then y, then x; the children share the stages of equal bits).
// P_c[i][j] = phi_j((xi_i + c) / 2), row-major K x K.
template <int K>
__global__ void __launch_bounds__(256) k_aprolong(const double* __restrict__ ec, double* __restrict__ ef,
                                                  const int32_t* __restrict__ parent, const double* __restrict__ P0,
                                                  const double* __restrict__ P1) {
  constexpr int K2 = K * K, K3 = K2 * K;
  __shared__ double u[K3], t1[2 * K3], t2[4 * K3], Pm[2][K2];
  const int64_t b = blockIdx.x;
  const int tid = threadIdx.x;
  const double* src = ec + (int64_t)parent[b] * K3;
  for (int q = tid; q < K3; q += blockDim.x) u[q] = src[q];
  for (int q = tid; q < K2; q += blockDim.x) {
    Pm[0][q] = P0[q];
    Pm[1][q] = P1[q];
  }
  __syncthreads();
  // t1[cz][iz][jy][jx] = sum_jz P_cz[iz][jz] u[jz][jy][jx]
  for (int q = tid; q < 2 * K3; q += blockDim.x) {
    const int cz = q / K3, r = q - cz * K3, iz = r / K2, jyx = r - iz * K2;
    double s = 0.0;
    for (int jz = 0; jz < K; ++jz) s += Pm[cz][iz * K + jz] * u[jz * K2 + jyx];
    t1[q] = s;
  }
  __syncthreads();
  // t2[cz][cy][iz][iy][jx] = sum_jy P_cy[iy][jy] t1[cz][iz][jy][jx]
  for (int q = tid; q < 4 * K3; q += blockDim.x) {
    const int czy = q / K3, r = q - czy * K3, cz = czy >> 1, cy = czy & 1;
    const int iz = r / K2, iy = (r / K) % K, jx = r % K;
    double s = 0.0;
    for (int jy = 0; jy < K; ++jy) s += Pm[cy][iy * K + jy] * t1[cz * K3 + iz * K2 + jy * K + jx];
    t2[q] = s;
  }
  __syncthreads();
  // ef[8 b + c][iz][iy][ix] += sum_jx P_cx[ix][jx] t2[cz][cy][iz][iy][jx]
  for (int q = tid; q < 8 * K3; q += blockDim.x) {
    const int c = q / K3, r = q - c * K3;
    const int cx = c & 1, cy = (c >> 1) & 1, cz = c >> 2;
    const int iz = r / K2, iy = (r / K) % K, ix = r % K;
    const double* row = t2 + ((cz * 2 + cy) * K3 + iz * K2 + iy * K);
    double s = 0.0;
    for (int jx = 0; jx < K; ++jx) s += Pm[cx][ix * K + jx] * row[jx];
    ef[(b * 8) * K3 + q] += s;
  }
}

// Algorithm 3 with the fused residual of Sec. 5 on a brick level:
// bc(parent(b)) += sum_c (P_cx^T x P_cy^T x P_cz^T) (bf - vf)(8 b + c),
// accumulating into the coarse level's right-hand side (Algorithm 5:
// the coarse level already carries its own share of the active residual).
template <int K>
__global__ void __launch_bounds__(256) k_arestrict(const double* __restrict__ bf, const double* __restrict__ vf,
                                                   double* __restrict__ bc, const int32_t* __restrict__ parent,
                                                   const double* __restrict__ P0, const double* __restrict__ P1) {
  constexpr int K2 = K * K, K3 = K2 * K;
  __shared__ double d[8 * K3], t[4 * K3], Pm[2][K2];
  double* t2 = d;   // the third stage's input reuses the residual area
  const int64_t b = blockIdx.x;
  const int tid = threadIdx.x;
  const int64_t base = b * 8 * K3;
  for (int q = tid; q < 8 * K3; q += blockDim.x) d[q] = bf[base + q] - vf[base + q];
  for (int q = tid; q < K2; q += blockDim.x) {
    Pm[0][q] = P0[q];
    Pm[1][q] = P1[q];
  }
  __syncthreads();
  // x: t[cz][cy][iz][iy][jx] = sum_cx sum_ix P_cx[ix][jx] d[c][iz][iy][ix]
  for (int q = tid; q < 4 * K3; q += blockDim.x) {
    const int czy = q / K3, r = q - czy * K3;
    const int iz = r / K2, iy = (r / K) % K, jx = r % K;
    double s = 0.0;
    for (int cx = 0; cx < 2; ++cx) {
      const double* row = d + (czy * 2 + cx) * K3 + iz * K2 + iy * K;
      for (int ix = 0; ix < K; ++ix) s += Pm[cx][ix * K + jx] * row[ix];
    }
    t[q] = s;
  }
  __syncthreads();
  // y: t2[cz][iz][jy][jx] = sum_cy sum_iy P_cy[iy][jy] t[cz][cy][iz][iy][jx]
  for (int q = tid; q < 2 * K3; q += blockDim.x) {
    const int cz = q / K3, r = q - cz * K3;
    const int iz = r / K2, jy = (r / K) % K, jx = r % K;
    double s = 0.0;
    for (int cy = 0; cy < 2; ++cy)
      for (int iy = 0; iy < K; ++iy) s += Pm[cy][iy * K + jy] * t[(cz * 2 + cy) * K3 + iz * K2 + iy * K + jx];
    t2[q] = s;
  }
  __syncthreads();
  // z: bc[parent][jz][jy][jx] += sum_cz sum_iz P_cz[iz][jz] t2[cz][iz][jy][jx]
  double* dst = bc + (int64_t)parent[b] * K3;
  for (int q = tid; q < K3; q += blockDim.x) {
    const int jz = q / K2, jyx = q - jz * K2;
    double s = 0.0;
    for (int cz = 0; cz < 2; ++cz)
      for (int iz = 0; iz < K; ++iz) s += Pm[cz][iz * K + jz] * t2[cz * K3 + iz * K2 + jyx];
    dst[q] += s;
  }
}

// ---------------------------------------------------------------- launchers

#define FE_DISPATCH_K_ADAPT(KVAL, CALL)   \
  switch (KVAL) {                          \
    case 2: { constexpr int KK = 2; CALL; } \
    case 3: { constexpr int KK = 3; CALL; } \
    case 4: { constexpr int KK = 4; CALL; } \
    case 5: { constexpr int KK = 5; CALL; } \
    case 6: { constexpr int KK = 6; CALL; } \
    default: return fail(FE_EINVAL, "the adaptive hierarchy supports degrees 1..5"); \
  }

static unsigned blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

template <int K>
static fe_status adss_typed(double* v, const int32_t* nbr, int64_t n_bricks, int averaging, hipStream_t s) {
  const int64_t n = n_bricks * 8 * K * K;
  if (n == 0) return FE_OK;
  ProfScope ps(averaging ? "adss_avg" : "adss_sum", s);
  hipLaunchKernelGGL((k_adss_pass<double, K, 0>), dim3(blocks(n)), dim3(256), 0, s, v, nbr, n_bricks, averaging);
  hipLaunchKernelGGL((k_adss_pass<double, K, 1>), dim3(blocks(n)), dim3(256), 0, s, v, nbr, n_bricks, averaging);
  hipLaunchKernelGGL((k_adss_pass<double, K, 2>), dim3(blocks(n)), dim3(256), 0, s, v, nbr, n_bricks, averaging);
  FE_HIP_CHECK(hipGetLastError());
  return FE_OK;
}

fe_status launch_adss(int K, double* v, const int32_t* nbr, int64_t n_bricks, int averaging, hipStream_t s) {
  FE_DISPATCH_K_ADAPT(K, return adss_typed<KK>(v, nbr, n_bricks, averaging, s));
}

fe_status launch_aedge_flags(int K, double* m, const int32_t* coords, const int32_t* nbr, int64_t n_cells, int n_l,
                             hipStream_t s) {
  FE_DISPATCH_K_ADAPT(K, {
    const int64_t n = n_cells * KK * KK * KK;
    hipLaunchKernelGGL((k_aedge_flags<double, KK>), dim3(blocks(n)), dim3(256), 0, s, m, coords, nbr, n_cells, n_l);
    FE_HIP_CHECK(hipGetLastError());
    return FE_OK;
  });
}

fe_status launch_amake_dinv(int K, double* dinv, const double* d, const double* kap, const double* em,
                            const int32_t* coords, int64_t n_cells, int n_l, hipStream_t s) {
  FE_DISPATCH_K_ADAPT(K, {
    const int64_t n = n_cells * KK * KK * KK;
    hipLaunchKernelGGL((k_amake_dinv<KK>), dim3(blocks(n)), dim3(256), 0, s, dinv, d, kap, em, coords, n_cells, n_l);
    FE_HIP_CHECK(hipGetLastError());
    return FE_OK;
  });
}

fe_status launch_ajacobi(double* u, const double* b, const double* v, const double* dinv, double omega, int64_t n,
                         int u_zero, hipStream_t s) {
  if (n == 0) return FE_OK;
  ProfScope ps("ajacobi", s);
  hipLaunchKernelGGL(k_ajacobi, dim3(blocks(n)), dim3(256), 0, s, u, b, v, dinv, omega, n, u_zero);
  FE_HIP_CHECK(hipGetLastError());
  return FE_OK;
}

fe_status launch_aactive(double* dst, const double* src, const uint8_t* refined, int K3, int64_t n, int mode,
                         hipStream_t s) {
  if (n == 0) return FE_OK;
  hipLaunchKernelGGL(k_aactive, dim3(blocks(n)), dim3(256), 0, s, dst, src, refined, K3, n, mode);
  FE_HIP_CHECK(hipGetLastError());
  return FE_OK;
}

fe_status launch_amask(int K, double* x, const uint8_t* refined, const int32_t* coords, int64_t n_cells, int n_l,
                       hipStream_t s) {
  FE_DISPATCH_K_ADAPT(K, {
    const int64_t n = n_cells * KK * KK * KK;
    if (n == 0) return FE_OK;
    hipLaunchKernelGGL((k_amask<KK>), dim3(blocks(n)), dim3(256), 0, s, x, refined, coords, n_cells, n_l);
    FE_HIP_CHECK(hipGetLastError());
    return FE_OK;
  });
}

fe_status launch_arhs(int K, double* b, const int32_t* coords, const uint8_t* refined, const double* tab, int nq,
                      int64_t n_cells, double h, hipStream_t s) {
  FE_DISPATCH_K_ADAPT(K, {
    const int64_t n = n_cells * KK * KK * KK;
    hipLaunchKernelGGL((k_arhs<KK>), dim3(blocks(n)), dim3(256), 0, s, b, coords, refined, tab, nq, n_cells, h);
    FE_HIP_CHECK(hipGetLastError());
    return FE_OK;
  });
}

fe_status launch_aprolong(int K, const double* ec, double* ef, const int32_t* parent, int64_t n_bricks,
                          const double* P0, const double* P1, hipStream_t s) {
  if (n_bricks == 0) return FE_OK;
  ProfScope ps("aprolong", s);
  FE_DISPATCH_K_ADAPT(K, {
    hipLaunchKernelGGL((k_aprolong<KK>), dim3((unsigned)n_bricks), dim3(256), 0, s, ec, ef, parent, P0, P1);
    FE_HIP_CHECK(hipGetLastError());
    return FE_OK;
  });
}

fe_status launch_arestrict(int K, const double* bf, const double* vf, double* bc, const int32_t* parent,
                           int64_t n_bricks, const double* P0, const double* P1, hipStream_t s) {
  if (n_bricks == 0) return FE_OK;
  ProfScope ps("arestrict", s);
  FE_DISPATCH_K_ADAPT(K, {
    hipLaunchKernelGGL((k_arestrict<KK>), dim3((unsigned)n_bricks), dim3(256), 0, s, bf, vf, bc, parent, P0, P1);
    FE_HIP_CHECK(hipGetLastError());
    return FE_OK;
  });
}

}  // namespace fe
