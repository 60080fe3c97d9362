// General-geometry operator on the deformed, variable-coefficient mesh.
//
// Paper, Sec. 6 (the curved case): the cell-wise Laplacian is applied in
// three stages -- reference gradients at the quadrature points, the
// physics (here the metric G_q = kappa w_q det(J_q) J_q^{-1} J_q^{-T}), and
// integration against the reference gradients -- with a per-quadrature-point
// Q_k mapping.  The mapping here is the Q_k interpolant of
// x = xh + amp * prod_b sin(2 pi xh_b) (1, 1, 1) through every cell's
// Gauss-Lobatto nodes; the coefficient is kappa = exp(s g(x)), g a Fourier
// sum, s scaling max |s g| to 1 over the Gauss points of the finest mesh.
//
// Setup stores the 6 unique metric entries at the (k+1)^3 Gauss points of
// every cell (component-major within a cell, point index x fastest).  The
// apply kernel streams u, the metric and y once: 16 sum-factorized 1D
// contractions per cell with the pencils re-oriented through LDS.
#include <cmath>

#include "fe_internal.h"
#include "kernel_common.h"

namespace fe {

// 1D tables in one device buffer (FP64, each K x K, row = quadrature point):
//   PHI[q][i] = phi_i(xq_q), DPHI[q][i] = phi_i'(xq_q)  (Gauss rule with K points)
//   WQ[q] (weights), XQ[q] (points), XN[i] (GLL nodes)
struct GeoTables {
  int off_phi, off_dphi, off_wq, off_xq, off_xn;
};

__host__ __device__ static inline GeoTables geo_layout(int K) {
  GeoTables t;
  t.off_phi = 0;
  t.off_dphi = K * K;
  t.off_wq = 2 * K * K;
  t.off_xq = 2 * K * K + K;
  t.off_xn = 2 * K * K + 2 * K;
  return t;
}

__device__ __forceinline__ double deform_shift(double x, double y, double z, double amp) {
  return amp * sin(2.0 * M_PI * x) * sin(2.0 * M_PI * y) * sin(2.0 * M_PI * z);
}

// Physical coordinates and Jacobian of the Q_k interpolated map at the
// reference point with 1D basis values (v, d) per axis; X = node coords in LDS.
template <int K>
__device__ __forceinline__ void eval_map(const double* __restrict__ X, const double* vx, const double* dx,
                                         const double* vy, const double* dy, const double* vz, const double* dz,
                                         double x[3], double J[3][3]) {
  for (int a = 0; a < 3; ++a) {
    x[a] = 0.0;
    J[a][0] = J[a][1] = J[a][2] = 0.0;
  }
  for (int iz = 0; iz < K; ++iz)
    for (int iy = 0; iy < K; ++iy) {
      const double vyz = vy[iy] * vz[iz], dyz = dy[iy] * vz[iz], vdz = vy[iy] * dz[iz];
      for (int ix = 0; ix < K; ++ix) {
        const int j = ix + K * (iy + K * iz);
        const double w = vx[ix] * vyz, wx = dx[ix] * vyz, wy = vx[ix] * dyz, wz = vx[ix] * vdz;
        for (int a = 0; a < 3; ++a) {
          const double Xa = X[3 * j + a];
          x[a] = fma(Xa, w, x[a]);
          J[a][0] = fma(Xa, wx, J[a][0]);
          J[a][1] = fma(Xa, wy, J[a][1]);
          J[a][2] = fma(Xa, wz, J[a][2]);
        }
      }
    }
}

__device__ __forceinline__ double coefficient_raw(const double x[3], const int* __restrict__ modes,
                                                  const double* __restrict__ amp, const double* __restrict__ ph,
                                                  int n_modes) {
  double g = 0.0;
  for (int j = 0; j < n_modes; ++j) {
    const double arg = M_PI * (modes[3 * j] * x[0] + modes[3 * j + 1] * x[1] + modes[3 * j + 2] * x[2]) + ph[j];
    g = fma(amp[j], cos(arg), g);
  }
  return g;
}

// Node coordinates of a cell into LDS: X[3 j + a].
template <int K>
__device__ __forceinline__ void load_cell_nodes(double* X, const double* __restrict__ xn, int cx, int cy, int cz,
                                                int n, double amp) {
  for (int j = threadIdx.x; j < K * K * K; j += blockDim.x) {
    const int ix = j % K, iy = (j / K) % K, iz = j / (K * K);
    const double x = (cx + xn[ix]) / n, y = (cy + xn[iy]) / n, z = (cz + xn[iz]) / n;
    const double s = deform_shift(x, y, z, amp);
    X[3 * j] = x + s;
    X[3 * j + 1] = y + s;
    X[3 * j + 2] = z + s;
  }
}

// mode 0: write the raw coefficient exponent g at every Gauss point (for the max);
// mode 1: write the 6 metric entries (xx, yy, zz, xy, xz, yz) with kappa = exp(scale g).
template <int K>
__global__ void __launch_bounds__(1024) k_geometry(const double* __restrict__ tab, int n, double amp,
                                                   const int* __restrict__ modes, const double* __restrict__ mamp,
                                                   const double* __restrict__ mph, int n_modes, double scale,
                                                   int mode, double* __restrict__ out) {
  constexpr int K3 = K * K * K;
  __shared__ double X[3 * K3];
  const int64_t cell = blockIdx.x;
  const int cx = (int)(cell % n), cy = (int)((cell / n) % n), cz = (int)(cell / ((int64_t)n * n));
  const GeoTables T = geo_layout(K);
  load_cell_nodes<K>(X, tab + T.off_xn, cx, cy, cz, n, amp);
  __syncthreads();
  const int q = threadIdx.x;
  if (q >= K3) return;
  const int qx = q % K, qy = (q / K) % K, qz = q / (K * K);
  const double* PHI = tab + T.off_phi;
  const double* DPHI = tab + T.off_dphi;
  double x[3], J[3][3];
  eval_map<K>(X, PHI + qx * K, DPHI + qx * K, PHI + qy * K, DPHI + qy * K, PHI + qz * K, DPHI + qz * K, x, J);
  const double g = n_modes > 0 ? coefficient_raw(x, modes, mamp, mph, n_modes) : 0.0;
  if (mode == 0) {
    out[cell * K3 + q] = g;
    return;
  }
  if (mode == 2) {   // the coefficient alone, for the apply that forms the metric itself
    out[cell * K3 + q] = exp(scale * g);
    return;
  }
  // inverse and determinant by cofactors: Jinv = adj(J) / det
  const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
  double Ji[3][3];
  Ji[0][0] = c00 / det;
  Ji[1][0] = c01 / det;
  Ji[2][0] = c02 / det;
  Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
  Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
  Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
  Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
  Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
  Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
  const double* WQ = tab + T.off_wq;
  const double f = exp(scale * g) * WQ[qx] * WQ[qy] * WQ[qz] * det;
  double G[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) G[a][b] = f * (Ji[a][0] * Ji[b][0] + Ji[a][1] * Ji[b][1] + Ji[a][2] * Ji[b][2]);
  double* o = out + cell * 6 * K3 + q;
  o[0] = G[0][0];
  o[K3] = G[1][1];
  o[2 * K3] = G[2][2];
  o[3 * K3] = G[0][1];
  o[4 * K3] = G[0][2];
  o[5 * K3] = G[1][2];
}

__global__ void __launch_bounds__(256) k_absmax_partial(const double* __restrict__ v, int64_t n,
                                                        double* __restrict__ part) {
  double m = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    m = fmax(m, fabs(v[e]));
  __shared__ double red[256];
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

template <typename T>
__global__ void k_convert_metric(const double* __restrict__ a, T* __restrict__ b, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) b[e] = (T)a[e];
}

// General cell-wise apply: y = sum_q grad(phi)^T G_q grad(u) (reference gradients).
// K^2 threads per cell; forward: z (PHI, DPHI), y (3), x (3) contractions;
// metric; backward: x (3), y (2 accumulating into 2), z (2 into 1).
//
// OTF = false: G holds the 6 metric entries per point (setup output).
// OTF = true (geometry traffic reduced to the coefficient): G holds only
// kappa at the points, and the metric is formed in the kernel.  The map is
// X_a = Q_k interpolant of xh_a + S, with the same shift S = amp sx sy sz
// (s_a = sin(2 pi xh_a)) in every coordinate, so on a cell of side 1/n
//   J = I / n + 1 v^T,  v_b = dS/dxi_b = amp (products of 1D interpolants of s_a),
// a rank-one update of a multiple of the identity.  With sigma = 1 + n sum_b v_b:
// det J = sigma / n^3, J^{-1} = n (I - (n / sigma) 1 v^T), and
//   G_ab = kappa w_q sigma / n (delta_ab - c (v_a + v_b) + c^2 |v|^2),  c = n / sigma.
// Per cell the 1D interpolants of s_a and of its derivative at the Gauss
// points (6K values) are formed once in LDS; nothing of the geometry is read.
template <typename T, int K, bool OTF = false>
__global__ void __launch_bounds__(256) k_apply_general3(const T* __restrict__ x, T* y,
                                                        const T* __restrict__ G, const T* __restrict__ PHI,
                                                        const T* __restrict__ DPHI, const T* __restrict__ PHIT,
                                                        const T* __restrict__ DPHIT, int n, int64_t n_cells,
                                                        int dirichlet, T alpha, T beta, const T* bsrc,
                                                        const double* __restrict__ geo = nullptr, double amp = 0.0) {
  constexpr int TPC = K * K;
  constexpr int CPB = 256 / TPC;
  constexpr int RS = K + 1, PS = K * RS, CS = K * PS;
  constexpr int K3 = K * K * K;
  constexpr int k = K - 1;
  __shared__ T s0[CPB * CS];
  __shared__ T s1[CPB * CS];
  __shared__ T s2[CPB * CS];
  __shared__ double sg[OTF ? CPB * 9 * K : 1];   // per cell: s_a at the nodes (3K), interpolants (3K), derivatives (3K)
  const int tid = threadIdx.x;
  const int c = tid / TPC;
  const int p = tid - c * TPC;
  const int p0 = p % K, p1 = p / K;
  const int64_t cell = (int64_t)blockIdx.x * CPB + c;
  const bool active = cell < n_cells;
  int cx = 0, cy = 0, cz = 0;
  if (active) cell_coords3<TPC % 64 == 0>(cell, n, cx, cy, cz);
  T* l0 = s0 + c * CS;
  T* l1 = s1 + c * CS;
  T* l2 = s2 + c * CS;
  if (OTF) {
    // 1D tables of the shift field: s_a(node i), then its interpolant and
    // derivative at Gauss point q (geo: FP64 PHI, DPHI, WQ, XQ, XN tables)
    double* g = sg + c * 9 * K;
    const int cc[3] = {cx, cy, cz};
    for (int t = p; t < 3 * K; t += TPC) {
      const int a = t / K, i = t - a * K;
      g[t] = sin(2.0 * M_PI * ((cc[a] + geo[2 * K * K + 2 * K + i]) / n));
    }
    __syncthreads();
    for (int t = p; t < 6 * K; t += TPC) {
      const int which = t / (3 * K), r = t - which * 3 * K, a = r / K, q = r - a * K;
      const double* M = geo + which * K * K + q * K;
      double s = 0.0;
      for (int i = 0; i < K; ++i) s = fma(M[i], g[a * K + i], s);
      g[3 * K + t] = s;   // [3K + a K + q]: interpolant; [6K + a K + q]: derivative
    }
    __syncthreads();
  }
  uint32_t zmask = 0;
  if (dirichlet && active) {
    const bool mxy = on_boundary(cx, p0, n, k) || on_boundary(cy, p1, n, k);
#pragma unroll
    for (int iz = 0; iz < K; ++iz)
      if (mxy || on_boundary(cz, iz, n, k)) zmask |= 1u << iz;
  }
  T v[K], a[K], b[K], w[K];
  // (A) z-pencils (ix = p0, iy = p1): a = PHI_z u, b = DPHI_z u
  if (active) {
    const T* xc = x + cell * K3 + p0 + K * p1;
#pragma unroll
    for (int iz = 0; iz < K; ++iz) v[iz] = (zmask & (1u << iz)) ? T(0) : xc[iz * K * K];
  } else {
#pragma unroll
    for (int iz = 0; iz < K; ++iz) v[iz] = T(0);
  }
  pencil_mv<T, K>(PHI, v, a);
  pencil_mv<T, K>(DPHI, v, b);
#pragma unroll
  for (int q = 0; q < K; ++q) { l0[q * PS + p1 * RS + p0] = a[q]; l1[q * PS + p1 * RS + p0] = b[q]; }
  __syncthreads();
  // (B) y-pencils (ix = p0, qz = p1): aa = PHI a, ab = DPHI a, ba = PHI b
#pragma unroll
  for (int j = 0; j < K; ++j) { v[j] = l0[p1 * PS + j * RS + p0]; w[j] = l1[p1 * PS + j * RS + p0]; }
  pencil_mv<T, K>(PHI, v, a);
  pencil_mv<T, K>(DPHI, v, b);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < K; ++q) { l0[p1 * PS + q * RS + p0] = a[q]; l1[p1 * PS + q * RS + p0] = b[q]; }
  pencil_mv<T, K>(PHI, w, a);
#pragma unroll
  for (int q = 0; q < K; ++q) l2[p1 * PS + q * RS + p0] = a[q];
  __syncthreads();
  // (C) x-pencils (qy = p0, qz = p1): reference gradients, metric, first backward contraction
  T gx[K], gy[K], gz[K];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    v[j] = l0[p1 * PS + p0 * RS + j];
    w[j] = l1[p1 * PS + p0 * RS + j];
    b[j] = l2[p1 * PS + p0 * RS + j];
  }
  pencil_mv<T, K>(DPHI, v, gx);   // d/dxi   = DPHI_x PHI_y PHI_z u
  pencil_mv<T, K>(PHI, w, gy);    // d/deta  = PHI_x DPHI_y PHI_z u
  pencil_mv<T, K>(PHI, b, gz);    // d/dzeta = PHI_x PHI_y DPHI_z u
  if (active && OTF) {
    const T* kc = G + cell * K3 + K * (p0 + K * p1);
    const double* g = sg + c * 9 * K;
    const double* WQ = geo + 2 * K * K;
    const T Ay = (T)(amp * g[3 * K + K + p0]), By = (T)(amp * g[6 * K + K + p0]);
    const T Az = (T)g[3 * K + 2 * K + p1], Bz = (T)g[6 * K + 2 * K + p1];
    const T wyz = (T)(WQ[p0] * WQ[p1]);
    const T nn = (T)n;
#pragma unroll
    for (int q = 0; q < K; ++q) {
      const T Ax = (T)g[3 * K + q], Bx = (T)g[6 * K + q];
      const T v0 = Bx * Ay * Az, v1 = Ax * By * Az, v2 = Ax * Ay * Bz;
      const T sigma = T(1) + nn * (v0 + v1 + v2);
      const T cq = nn / sigma;
      const T vv = cq * cq * (v0 * v0 + v1 * v1 + v2 * v2);
      const T f = kc[q] * (T)WQ[q] * wyz * sigma / nn;
      const T gxx = f * (T(1) - 2 * cq * v0 + vv), gyy = f * (T(1) - 2 * cq * v1 + vv);
      const T gzz = f * (T(1) - 2 * cq * v2 + vv);
      const T gxy = f * (vv - cq * (v0 + v1)), gxz = f * (vv - cq * (v0 + v2)), gyz = f * (vv - cq * (v1 + v2));
      const T fx = gxx * gx[q] + gxy * gy[q] + gxz * gz[q];
      const T fy = gxy * gx[q] + gyy * gy[q] + gyz * gz[q];
      const T fz = gxz * gx[q] + gyz * gy[q] + gzz * gz[q];
      gx[q] = fx; gy[q] = fy; gz[q] = fz;
    }
  } else if (active) {
    const T* Gc = G + cell * 6 * K3 + K * (p0 + K * p1);
#pragma unroll
    for (int q = 0; q < K; ++q) {
      const T gxx = Gc[q], gyy = Gc[K3 + q], gzz = Gc[2 * K3 + q];
      const T gxy = Gc[3 * K3 + q], gxz = Gc[4 * K3 + q], gyz = Gc[5 * K3 + q];
      const T fx = gxx * gx[q] + gxy * gy[q] + gxz * gz[q];
      const T fy = gxy * gx[q] + gyy * gy[q] + gyz * gz[q];
      const T fz = gxz * gx[q] + gyz * gy[q] + gzz * gz[q];
      gx[q] = fx; gy[q] = fy; gz[q] = fz;
    }
  } else {
#pragma unroll
    for (int q = 0; q < K; ++q) gx[q] = gy[q] = gz[q] = T(0);
  }
  pencil_mv<T, K>(DPHIT, gx, a);   // s1 = DPHI_x^T fx
  pencil_mv<T, K>(PHIT, gy, b);    // s_eta = PHI_x^T fy
  pencil_mv<T, K>(PHIT, gz, w);    // s_zeta = PHI_x^T fz
  __syncthreads();
#pragma unroll
  for (int i = 0; i < K; ++i) {
    l0[p1 * PS + p0 * RS + i] = a[i];
    l1[p1 * PS + p0 * RS + i] = b[i];
    l2[p1 * PS + p0 * RS + i] = w[i];
  }
  __syncthreads();
  // (D) y-pencils (ix = p0, qz = p1): u1 = PHI^T s1 + DPHI^T s_eta, u2 = PHI^T s_zeta
#pragma unroll
  for (int j = 0; j < K; ++j) {
    v[j] = l0[p1 * PS + j * RS + p0];
    w[j] = l1[p1 * PS + j * RS + p0];
    b[j] = l2[p1 * PS + j * RS + p0];
  }
  {
    T t1[K], t2[K];
    pencil_mv<T, K>(PHIT, v, t1);
    pencil_mv<T, K>(DPHIT, w, t2);
#pragma unroll
    for (int i = 0; i < K; ++i) a[i] = t1[i] + t2[i];
    pencil_mv<T, K>(PHIT, b, t1);
#pragma unroll
    for (int i = 0; i < K; ++i) b[i] = t1[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < K; ++i) { l0[p1 * PS + i * RS + p0] = a[i]; l1[p1 * PS + i * RS + p0] = b[i]; }
  __syncthreads();
  // (E) z-pencils (ix = p0, iy = p1): y = PHI^T u1 + DPHI^T u2
#pragma unroll
  for (int j = 0; j < K; ++j) { v[j] = l0[j * PS + p1 * RS + p0]; w[j] = l1[j * PS + p1 * RS + p0]; }
  {
    T t1[K], t2[K];
    pencil_mv<T, K>(PHIT, v, t1);
    pencil_mv<T, K>(DPHIT, w, t2);
    if (active) {
      // epilogue y = alpha A x + beta bsrc (read before y is written: bsrc may alias y)
      const int64_t off = cell * K3 + p0 + K * p1;
      T* yc = y + off;
#pragma unroll
      for (int iz = 0; iz < K; ++iz) {
        T val = (zmask & (1u << iz)) ? T(0) : t1[iz] + t2[iz];
        val *= alpha;
        if (bsrc) val += beta * bsrc[off + iz * K * K];
        if constexpr (sizeof(T) == 8) __builtin_nontemporal_store(val, yc + iz * K * K);
        else yc[iz * K * K] = val;
      }
    }
  }
}

// Local diagonal of the general element matrix: thread per entry, loop over points.
template <int K>
__global__ void __launch_bounds__(256) k_diag_general(const double* __restrict__ G, const double* __restrict__ tab,
                                                      double* __restrict__ d, int64_t len) {
  constexpr int K3 = K * K * K;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  const int64_t cell = e / K3;
  const int i = (int)(e - cell * K3);
  const int ix = i % K, iy = (i / K) % K, iz = i / (K * K);
  const GeoTables T = geo_layout(K);
  const double* PHI = tab + T.off_phi;
  const double* DPHI = tab + T.off_dphi;
  const double* Gc = G + cell * 6 * K3;
  double s = 0.0;
  for (int q = 0; q < K3; ++q) {
    const int qx = q % K, qy = (q / K) % K, qz = q / (K * K);
    const double vx = PHI[qx * K + ix], vy = PHI[qy * K + iy], vz = PHI[qz * K + iz];
    const double a = DPHI[qx * K + ix] * vy * vz, b = vx * DPHI[qy * K + iy] * vz, c = vx * vy * DPHI[qz * K + iz];
    s += Gc[q] * a * a + Gc[K3 + q] * b * b + Gc[2 * K3 + q] * c * c +
         2.0 * (Gc[3 * K3 + q] * a * b + Gc[4 * K3 + q] * a * c + Gc[5 * K3 + q] * b * c);
  }
  d[e] = s;
}

// Load vector b_K,i = sum_q w_q det(J_q) f(x_q) phi_i(xi_q), Gauss rule with QN points
// per axis, f = 3 pi^2 prod sin(pi x_a).  One block per cell.
template <int K, int QN>
__global__ void __launch_bounds__(1024) k_rhs_general(const double* __restrict__ tabq, const double* __restrict__ xn,
                                                      int n, double amp, double* __restrict__ b) {
  constexpr int K3 = K * K * K;
  constexpr int Q3 = QN * QN * QN;
  __shared__ double X[3 * K3];
  __shared__ double F[Q3];
  const int64_t cell = blockIdx.x;
  const int cx = (int)(cell % n), cy = (int)((cell / n) % n), cz = (int)(cell / ((int64_t)n * n));
  load_cell_nodes<K>(X, xn, cx, cy, cz, n, amp);
  __syncthreads();
  const double* PHI = tabq;            // QN x K
  const double* DPHI = tabq + QN * K;
  const double* WQ = tabq + 2 * QN * K;
  for (int q = threadIdx.x; q < Q3; q += blockDim.x) {
    const int qx = q % QN, qy = (q / QN) % QN, qz = q / (QN * QN);
    double x[3], J[3][3];
    eval_map<K>(X, PHI + qx * K, DPHI + qx * K, PHI + qy * K, DPHI + qy * K, PHI + qz * K, DPHI + qz * K, x, J);
    const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                       J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                       J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    const double f = 3.0 * M_PI * M_PI * sin(M_PI * x[0]) * sin(M_PI * x[1]) * sin(M_PI * x[2]);
    F[q] = WQ[qx] * WQ[qy] * WQ[qz] * det * f;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < K3; i += blockDim.x) {
    const int ix = i % K, iy = (i / K) % K, iz = i / (K * K);
    double s = 0.0;
    for (int q = 0; q < Q3; ++q) {
      const int qx = q % QN, qy = (q / QN) % QN, qz = q / (QN * QN);
      s += F[q] * PHI[qx * K + ix] * PHI[qy * K + iy] * PHI[qz * K + iz];
    }
    b[cell * K3 + i] = s;
  }
}

// ---------------------------------------------------------------- host side

static std::vector<double> make_tables(int k, int nq) {
  const int K = k + 1;
  std::vector<double> nodes = gll_nodes(k), xq, wq;
  gauss_rule(nq, xq, wq);
  std::vector<double> t(2 * nq * K + 2 * nq + K, 0.0);
  for (int q = 0; q < nq; ++q)
    for (int i = 0; i < K; ++i) {
      t[q * K + i] = lagrange_value(nodes, i, xq[q]);
      t[nq * K + q * K + i] = lagrange_deriv(nodes, i, xq[q]);
    }
  for (int q = 0; q < nq; ++q) {
    t[2 * nq * K + q] = wq[q];
    t[2 * nq * K + nq + q] = xq[q];
  }
  for (int i = 0; i < K; ++i) t[2 * nq * K + 2 * nq + i] = nodes[i];
  return t;
}

template <int K>
static fe_status geometry_typed(fe_problem* p, hipStream_t s) {
  const int k = K - 1;
  std::vector<double> tab = make_tables(k, K);
  DeviceBuf dtab, dmodes, dscr;
  FE_CHECK(dtab.alloc(tab.size() * sizeof(double)));
  FE_HIP_CHECK(hipMemcpyAsync(dtab.p, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice, s));
  const int nm = (int)p->amp.size();
  std::vector<double> md(2 * nm + 1, 0.0);
  for (int j = 0; j < nm; ++j) { md[j] = p->amp[j]; md[nm + j] = p->phase[j]; }
  FE_CHECK(dmodes.alloc(md.size() * sizeof(double) + 3 * nm * sizeof(int32_t) + 64));
  double* damp = dmodes.as<double>();
  int* dm = reinterpret_cast<int*>(damp + md.size());
  FE_HIP_CHECK(hipMemcpyAsync(damp, md.data(), md.size() * sizeof(double), hipMemcpyHostToDevice, s));
  if (nm > 0) FE_HIP_CHECK(hipMemcpyAsync(dm, p->modes.data(), 3 * nm * sizeof(int32_t), hipMemcpyHostToDevice, s));
  const double amp = p->desc.deform_amp;
  constexpr int K3 = K * K * K;
  // scale from the finest level's Gauss points
  double scale = 1.0;
  Level& F = p->levels.back();
  if (nm > 0) {
    FE_CHECK(dscr.alloc(F.n_cells * K3 * sizeof(double)));
    hipLaunchKernelGGL((k_geometry<K>), dim3((unsigned)F.n_cells), dim3(K3), 0, s, dtab.as<double>(), F.n, amp, dm,
                       damp, damp + nm, nm, 1.0, 0, dscr.as<double>());
    FE_HIP_CHECK(hipGetLastError());
    const int64_t n = F.n_cells * K3;
    const int nparts = (int)std::min<int64_t>(1024, (n + 255) / 256);
    hipLaunchKernelGGL(k_absmax_partial, dim3(nparts), dim3(256), 0, s, dscr.as<double>(), n,
                       p->red_scratch.as<double>());
    std::vector<double> parts(nparts);
    FE_HIP_CHECK(hipMemcpyAsync(parts.data(), p->red_scratch.p, nparts * sizeof(double), hipMemcpyDeviceToHost, s));
    FE_HIP_CHECK(hipStreamSynchronize(s));
    double mx = 0.0;
    for (double v : parts) mx = std::max(mx, v);
    if (!(mx > 0.0)) return fail(FE_EINVAL, "coefficient field is identically zero");
    scale = 1.0 / mx;
  }
  p->coef_scale = scale;
  for (Level& L : p->levels) {
    const int64_t nm6 = L.n_cells * 6 * K3;
    FE_CHECK(L.metric64.alloc(nm6 * sizeof(double)));
    FE_CHECK(L.metric32.alloc(nm6 * sizeof(float)));
    hipLaunchKernelGGL((k_geometry<K>), dim3((unsigned)L.n_cells), dim3(K3), 0, s, dtab.as<double>(), L.n, amp, dm,
                       damp, damp + nm, nm, scale, 1, L.metric64.as<double>());
    FE_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL((k_convert_metric<float>), dim3((unsigned)((nm6 + 255) / 256)), dim3(256), 0, s,
                       L.metric64.as<double>(), L.metric32.as<float>(), nm6);
    FE_HIP_CHECK(hipGetLastError());
  }
  // apply tables (PHI, DPHI) per dtype, and their transposes: the backward
  // contractions (PHI^T v) read rows of PHI^T, fetched as whole rows by the
  // scalar unit, instead of columns of PHI one value per scalar load (at K = 8
  // FP64 that was 517 single loads and 300 scalar registers parked in vector
  // lanes per cell pass)
  std::vector<double> ap(2 * K * K), apt(2 * K * K);
  std::copy(tab.begin(), tab.begin() + 2 * K * K, ap.begin());
  for (int m = 0; m < 2; ++m)
    for (int q = 0; q < K; ++q)
      for (int i = 0; i < K; ++i) apt[m * K * K + i * K + q] = ap[m * K * K + q * K + i];
  std::vector<float> ap32(ap.begin(), ap.end()), apt32(apt.begin(), apt.end());
  FE_CHECK(p->geo_tab64.alloc(tab.size() * sizeof(double)));
  FE_CHECK(p->geo_tab32.alloc(ap32.size() * sizeof(float)));
  FE_CHECK(p->geo_tabT64.alloc(apt.size() * sizeof(double)));
  FE_CHECK(p->geo_tabT32.alloc(apt32.size() * sizeof(float)));
  FE_HIP_CHECK(hipMemcpyAsync(p->geo_tab64.p, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice, s));
  FE_HIP_CHECK(hipMemcpyAsync(p->geo_tab32.p, ap32.data(), ap32.size() * sizeof(float), hipMemcpyHostToDevice, s));
  FE_HIP_CHECK(hipMemcpyAsync(p->geo_tabT64.p, apt.data(), apt.size() * sizeof(double), hipMemcpyHostToDevice, s));
  FE_HIP_CHECK(hipMemcpyAsync(p->geo_tabT32.p, apt32.data(), apt32.size() * sizeof(float), hipMemcpyHostToDevice, s));
  FE_HIP_CHECK(hipStreamSynchronize(s));
  return FE_OK;
}

fe_status setup_geometry(fe_problem* p, hipStream_t s) {
  if (p->dim != 3) return fail(FE_EUNSUPPORTED, "deformed geometry is implemented for d = 3");
  FE_DISPATCH_K(p->K, return geometry_typed<KK>(p, s));
}

template <typename T, int K>
static fe_status apply_general_typed(const fe_problem* p, const Level& L, const T* x, T* y, const T* G,
                                     const T* tab, const T* tabT, T alpha, T beta, const T* b, hipStream_t s) {
  constexpr int CPB = 256 / (K * K);
  const unsigned nb = (unsigned)((L.n_cells + CPB - 1) / CPB);
  if (p->metric_otf) {
    ProfScope ps("apply_general_otf", s);
    const T* kap = sizeof(T) == 8 ? (const T*)L.kappa64.p : (const T*)L.kappa32.p;
    hipLaunchKernelGGL((k_apply_general3<T, K, true>), dim3(nb), dim3(CPB * K * K), 0, s, x, y, kap, tab,
                       tab + K * K, tabT, tabT + K * K, L.n, L.n_cells, p->bc, alpha, beta, b, p->geo_tab64.as<double>(),
                       p->desc.deform_amp);
  } else {
    ProfScope ps("apply_general", s);
    hipLaunchKernelGGL((k_apply_general3<T, K, false>), dim3(nb), dim3(CPB * K * K), 0, s, x, y, G, tab,
                       tab + K * K, tabT, tabT + K * K, L.n, L.n_cells, p->bc, alpha, beta, b, nullptr, 0.0);
  }
  FE_HIP_CHECK(hipGetLastError());
  return FE_OK;
}

fe_status launch_apply_general(const fe_problem* p, int level, const void* x, void* y, double alpha, double beta,
                               const void* b, fe_dtype dt, hipStream_t s) {
  const Level& L = level_of(p, level);
  if (dt == FE_F64) {
    FE_DISPATCH_K(p->K, return (apply_general_typed<double, KK>(p, L, (const double*)x, (double*)y,
                                                                L.metric64.as<double>(), p->geo_tab64.as<double>(),
                                                                p->geo_tabT64.as<double>(), alpha, beta,
                                                                (const double*)b, s)));
  }
  FE_DISPATCH_K(p->K, return (apply_general_typed<float, KK>(p, L, (const float*)x, (float*)y,
                                                             L.metric32.as<float>(), p->geo_tab32.as<float>(),
                                                             p->geo_tabT32.as<float>(),
                                                             (float)alpha, (float)beta, (const float*)b, s)));
}

// Coefficient kappa at the Gauss points of every level (both dtypes), for the
// apply that forms the metric itself.
template <int K>
static fe_status kappa_typed(fe_problem* p, hipStream_t s) {
  constexpr int K3 = K * K * K;
  const int nm = (int)p->amp.size();
  std::vector<double> md(2 * nm + 1, 0.0);
  for (int j = 0; j < nm; ++j) { md[j] = p->amp[j]; md[nm + j] = p->phase[j]; }
  DeviceBuf dmodes;
  FE_CHECK(dmodes.alloc(md.size() * sizeof(double) + 3 * nm * sizeof(int32_t) + 64));
  double* damp = dmodes.as<double>();
  int* dm = reinterpret_cast<int*>(damp + md.size());
  FE_HIP_CHECK(hipMemcpyAsync(damp, md.data(), md.size() * sizeof(double), hipMemcpyHostToDevice, s));
  if (nm > 0) FE_HIP_CHECK(hipMemcpyAsync(dm, p->modes.data(), 3 * nm * sizeof(int32_t), hipMemcpyHostToDevice, s));
  for (Level& L : p->levels) {
    const int64_t n = L.n_cells * K3;
    FE_CHECK(L.kappa64.alloc(n * sizeof(double)));
    FE_CHECK(L.kappa32.alloc(n * sizeof(float)));
    hipLaunchKernelGGL((k_geometry<K>), dim3((unsigned)L.n_cells), dim3(K3), 0, s, p->geo_tab64.as<double>(), L.n,
                       p->desc.deform_amp, dm, damp, damp + nm, nm, p->coef_scale, 2, L.kappa64.as<double>());
    FE_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL((k_convert_metric<float>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       L.kappa64.as<double>(), L.kappa32.as<float>(), n);
    FE_HIP_CHECK(hipGetLastError());
  }
  FE_HIP_CHECK(hipStreamSynchronize(s));
  return FE_OK;
}

}  // namespace fe

extern "C" fe_status fe_set_metric_mode(fe_problem* p, int mode, void* stream) {
  using namespace fe;
  if (!p) return fail(FE_EINVAL, "null problem");
  if (mode != 0 && mode != 1) return fail(FE_EINVAL, "metric mode must be 0 or 1");
  if (mode == 1 && p->desc.geometry != FE_GEOM_DEFORMED)
    return fail(FE_EINVAL, "the metric is formed in the kernel for the deformed geometry only");
  if (mode == 1 && !p->levels.back().kappa64.p) FE_DISPATCH_K(p->K, FE_CHECK(kappa_typed<KK>(p, (hipStream_t)stream)); break);
  p->metric_otf = mode;
  return FE_OK;
}

namespace fe {

template <int K>
static fe_status diag_general_typed(const fe_problem* p, const Level& L, double* d, hipStream_t s) {
  hipLaunchKernelGGL((k_diag_general<K>), dim3((unsigned)((L.len + 255) / 256)), dim3(256), 0, s,
                     L.metric64.as<double>(), p->geo_tab64.as<double>(), d, L.len);
  FE_HIP_CHECK(hipGetLastError());
  return FE_OK;
}

fe_status launch_diag_general(const fe_problem* p, int level, void* d, fe_dtype dt, hipStream_t s) {
  if (dt != FE_F64) return fail(FE_EINVAL, "the diagonal is formed in FP64");
  const Level& L = level_of(p, level);
  FE_DISPATCH_K(p->K, return diag_general_typed<KK>(p, L, (double*)d, s));
}

template <int K>
static fe_status rhs_general_typed(const fe_problem* p, double* b, hipStream_t s) {
  constexpr int QN = K + 1;   // k + 2 Gauss points per axis
  const Level& L = level_of(p, -1);
  std::vector<double> t = make_tables(K - 1, QN);
  std::vector<double> nodes = gll_nodes(K - 1);
  t.insert(t.end(), nodes.begin(), nodes.end());
  DeviceBuf d;
  FE_CHECK(d.alloc(t.size() * sizeof(double)));
  FE_HIP_CHECK(hipMemcpyAsync(d.p, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice, s));
  const double* xn = d.as<double>() + (2 * QN * K + 2 * QN + K);
  hipLaunchKernelGGL((k_rhs_general<K, QN>), dim3((unsigned)L.n_cells), dim3(std::min(1024, QN * QN * QN)), 0, s,
                     d.as<double>(), xn, L.n, p->desc.deform_amp, b);
  FE_HIP_CHECK(hipGetLastError());
  FE_HIP_CHECK(hipStreamSynchronize(s));
  return FE_OK;
}

fe_status launch_rhs_general(const fe_problem* p, void* b, hipStream_t s) {
  FE_DISPATCH_K(p->K, return rhs_general_typed<KK>(p, (double*)b, s));
}

}  // namespace fe

// ---------------------------------------------------------------- per-patch separable factors
//
// A patch operator on the deformed mesh is replaced by the separable
// surrogate
//   A_sep = Kx (x) My (x) Mz + Mx (x) Ky (x) Mz + Mx (x) My (x) Kz,
// K_d = sum_{c=0,1} alpha_{d,c} Dhat on interval c of the patch, M_d likewise
// with beta_{d,c} Bhat (interior nodes only).  The 12 weights of a patch
// come either from its averaged geometry (mode 1: least-squares fit in log
// space of the cell-averaged diagonal metric entries, 24 equations) or from
// the learned model (mode 2).  Each direction's pair (K_d, M_d) is then
// diagonalized, K_d S_d = M_d S_d L_d, S_d^T M_d S_d = I, one thread per
// (patch, direction).

namespace fe {

namespace fe_detail {}

template <int K>
__global__ void __launch_bounds__(256) k_cell_avg_metric(const double* __restrict__ G, double* __restrict__ out,
                                                         int64_t n_cells) {
  constexpr int K3 = K * K * K;
  const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= n_cells) return;
  for (int d = 0; d < 3; ++d) {
    const double* g = G + cell * 6 * K3 + d * K3;
    double s = 0.0;
    for (int q = 0; q < K3; ++q) s += g[q];
    out[cell * 3 + d] = s;
  }
}

// weights[pid*12 + d*2 + c] = alpha_{d,c}, weights[pid*12 + 6 + d*2 + c] = beta_{d,c}
__global__ void __launch_bounds__(256) k_patch_fit_avg(const double* __restrict__ gbar, const double* __restrict__ Pinv,
                                                       double* __restrict__ weights, int n) {
  const int nv = n - 1;
  const int64_t np = (int64_t)nv * nv * nv;
  const int64_t pid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pid >= np) return;
  const int vx = 1 + (int)(pid % nv), vy = 1 + (int)((pid / nv) % nv), vz = 1 + (int)(pid / ((int64_t)nv * nv));
  double lg[24];
  for (int s = 0; s < 8; ++s) {
    const int cx = vx - 1 + (s & 1), cy = vy - 1 + ((s >> 1) & 1), cz = vz - 1 + (s >> 2);
    const int64_t cell = cx + (int64_t)n * (cy + (int64_t)n * cz);
    for (int d = 0; d < 3; ++d) lg[d * 8 + s] = log(gbar[cell * 3 + d]);
  }
  for (int j = 0; j < 12; ++j) {
    double t = 0.0;
    for (int r = 0; r < 24; ++r) t = fma(Pinv[j * 24 + r], lg[r], t);
    weights[pid * 12 + j] = exp(t);
  }
}

// Generalized eigenproblem of one (patch, direction): Cholesky of M, cyclic
// Jacobi on L^{-1} K L^{-T}, eigenvalues ascending.
template <int M>
__device__ void small_geig(double (&A)[M][M], double (&B)[M][M], double (&S)[M][M], double (&lam)[M]) {
  // Cholesky B = L L^T (in place, lower)
  for (int j = 0; j < M; ++j) {
    double d = B[j][j];
    for (int q = 0; q < j; ++q) d -= B[j][q] * B[j][q];
    d = sqrt(fmax(d, 1e-300));
    B[j][j] = d;
    for (int i = j + 1; i < M; ++i) {
      double v = B[i][j];
      for (int q = 0; q < j; ++q) v -= B[i][q] * B[j][q];
      B[i][j] = v / d;
    }
  }
  // C = L^{-1} A L^{-T}: solve L X = A (columns), then L C^T = X^T
  for (int c = 0; c < M; ++c)
    for (int i = 0; i < M; ++i) {
      double v = A[i][c];
      for (int q = 0; q < i; ++q) v -= B[i][q] * A[q][c];
      A[i][c] = v / B[i][i];
    }
  for (int r = 0; r < M; ++r)
    for (int i = 0; i < M; ++i) {
      double v = A[r][i];
      for (int q = 0; q < i; ++q) v -= B[i][q] * A[r][q];
      A[r][i] = v / B[i][i];
    }
  for (int i = 0; i < M; ++i)
    for (int j = i + 1; j < M; ++j) A[i][j] = A[j][i] = 0.5 * (A[i][j] + A[j][i]);
  for (int i = 0; i < M; ++i)
    for (int j = 0; j < M; ++j) S[i][j] = i == j ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 30; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < M; ++i)
      for (int j = 0; j < M; ++j) {
        tot += A[i][j] * A[i][j];
        if (i != j) off += A[i][j] * A[i][j];
      }
    if (off <= 1e-30 * tot) break;
    for (int p = 0; p < M; ++p)
      for (int q = p + 1; q < M; ++q) {
        const double apq = A[p][q];
        if (fabs(apq) < 1e-300) continue;
        const double theta = (A[q][q] - A[p][p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int r = 0; r < M; ++r) {
          const double arp = A[r][p], arq = A[r][q];
          A[r][p] = c * arp - s * arq;
          A[r][q] = s * arp + c * arq;
        }
        for (int r = 0; r < M; ++r) {
          const double apr = A[p][r], aqr = A[q][r];
          A[p][r] = c * apr - s * aqr;
          A[q][r] = s * apr + c * aqr;
        }
        for (int r = 0; r < M; ++r) {
          const double srp = S[r][p], srq = S[r][q];
          S[r][p] = c * srp - s * srq;
          S[r][q] = s * srp + c * srq;
        }
      }
  }
  // eigenvectors of the pencil: L^{-T} S; eigenvalues on the diagonal (sorted ascending)
  for (int c = 0; c < M; ++c)
    for (int i = M - 1; i >= 0; --i) {
      double v = S[i][c];
      for (int q = i + 1; q < M; ++q) v -= B[q][i] * S[q][c];
      S[i][c] = v / B[i][i];
    }
  for (int i = 0; i < M; ++i) lam[i] = A[i][i];
  for (int i = 0; i < M; ++i) {   // selection sort of columns
    int m = i;
    for (int j = i + 1; j < M; ++j)
      if (lam[j] < lam[m]) m = j;
    if (m != i) {
      const double t = lam[i]; lam[i] = lam[m]; lam[m] = t;
      for (int r = 0; r < M; ++r) { const double u = S[r][i]; S[r][i] = S[r][m]; S[r][m] = u; }
    }
  }
}

template <int K>
__global__ void __launch_bounds__(64) k_patch_eig(const double* __restrict__ weights, const double* __restrict__ Bh,
                                                  const double* __restrict__ Dh, double* __restrict__ eig,
                                                  int64_t n_patches) {
  constexpr int k = K - 1;
  constexpr int M = 2 * k - 1;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= 3 * n_patches) return;
  const int64_t pid = gid / 3;
  const int d = (int)(gid - 3 * pid);
  const double a0 = weights[pid * 12 + 2 * d], a1 = weights[pid * 12 + 2 * d + 1];
  const double b0 = weights[pid * 12 + 6 + 2 * d], b1 = weights[pid * 12 + 6 + 2 * d + 1];
  double A[M][M], B[M][M], S[M][M], lam[M];
  for (int i = 0; i < M; ++i)
    for (int j = 0; j < M; ++j) {
      // interior node i of the patch is node i+1 of the two-interval line
      const int gi = i + 1, gj = j + 1;
      double kv = 0.0, mv = 0.0;
      for (int e = 0; e < 2; ++e) {
        const int li = gi - k * e, lj = gj - k * e;
        if (li < 0 || li > k || lj < 0 || lj > k) continue;
        kv += (e ? a1 : a0) * Dh[li * K + lj];
        mv += (e ? b1 : b0) * Bh[li * K + lj];
      }
      A[i][j] = kv;
      B[i][j] = mv;
    }
  small_geig<M>(A, B, S, lam);
  double* base = eig + pid * (3 * M * M + 3 * M);
  double* Sd = base + d * M * M;
  double* ld = base + 3 * M * M + d * M;
  for (int i = 0; i < M; ++i)
    for (int j = 0; j < M; ++j) Sd[i * M + j] = S[i][j];
  for (int i = 0; i < M; ++i) ld[i] = lam[i];
}

// Pseudo-inverse of the 24 x 12 design matrix of the log-space fit.
static std::vector<double> log_fit_pinv() {
  std::vector<double> A(24 * 12, 0.0);
  for (int d = 0; d < 3; ++d)
    for (int s = 0; s < 8; ++s) {
      const int sl[3] = {s & 1, (s >> 1) & 1, s >> 2};
      const int r = d * 8 + s;
      A[r * 12 + 2 * d + sl[d]] = 1.0;
      for (int e = 0; e < 3; ++e)
        if (e != d) A[r * 12 + 6 + 2 * e + sl[e]] = 1.0;
    }
  std::vector<double> AtA(144, 0.0), I(144, 0.0), V, lam;
  for (int i = 0; i < 12; ++i) {
    I[i * 12 + i] = 1.0;
    for (int j = 0; j < 12; ++j)
      for (int r = 0; r < 24; ++r) AtA[i * 12 + j] += A[r * 12 + i] * A[r * 12 + j];
  }
  sym_generalized_eig(12, AtA, I, V, lam);
  const double tol = 1e-10 * lam[11];
  std::vector<double> P(12 * 24, 0.0);
  for (int i = 0; i < 12; ++i)
    for (int r = 0; r < 24; ++r) {
      double s = 0.0;
      for (int m = 0; m < 12; ++m) {
        if (lam[m] <= tol) continue;
        double vAt = 0.0;   // (V^T A^T)[m, r]
        for (int j = 0; j < 12; ++j) vAt += V[j * 12 + m] * A[r * 12 + j];
        s += V[i * 12 + m] * vAt / lam[m];
      }
      P[i * 24 + r] = s;
    }
  return P;
}

template <int K>
static fe_status eig_from_weights(fe_problem* p, int level, int mode, const double* weights, hipStream_t s) {
  constexpr int M = 2 * (K - 1) - 1;
  Level& L = p->levels[level];
  const int64_t nv = L.n - 1;
  const int64_t np = nv * nv * nv;
  const int64_t ne = np * (3 * M * M + 3 * M);
  FE_CHECK(L.patch_eig64[mode].alloc(std::max<int64_t>(ne, 1) * sizeof(double)));
  FE_CHECK(L.patch_eig32[mode].alloc(std::max<int64_t>(ne, 1) * sizeof(float)));
  if (np > 0) {
    hipLaunchKernelGGL((k_patch_eig<K>), dim3((unsigned)((3 * np + 63) / 64)), dim3(64), 0, s, weights,
                       p->coef64.as<double>() + p->co.off_B, p->coef64.as<double>() + p->co.off_D,
                       L.patch_eig64[mode].as<double>(), np);
    FE_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL((k_convert_metric<float>), dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, s,
                       L.patch_eig64[mode].as<double>(), L.patch_eig32[mode].as<float>(), ne);
    FE_HIP_CHECK(hipGetLastError());
  }
  FE_HIP_CHECK(hipStreamSynchronize(s));
  L.patch_eig_ready[mode] = true;
  return FE_OK;
}

template <int K>
static fe_status averaged_factors_typed(fe_problem* p, int level, DeviceBuf& weights, hipStream_t s) {
  Level& L = p->levels[level];
  const int64_t nv = L.n - 1;
  const int64_t np = nv * nv * nv;
  DeviceBuf gbar, dP;
  FE_CHECK(gbar.alloc(L.n_cells * 3 * sizeof(double)));
  FE_CHECK(weights.alloc(std::max<int64_t>(np, 1) * 12 * sizeof(double)));
  std::vector<double> P = log_fit_pinv();
  FE_CHECK(dP.alloc(P.size() * sizeof(double)));
  FE_HIP_CHECK(hipMemcpyAsync(dP.p, P.data(), P.size() * sizeof(double), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL((k_cell_avg_metric<K>), dim3((unsigned)((L.n_cells + 255) / 256)), dim3(256), 0, s,
                     L.metric64.as<double>(), gbar.as<double>(), L.n_cells);
  FE_HIP_CHECK(hipGetLastError());
  if (np > 0) {
    hipLaunchKernelGGL(k_patch_fit_avg, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, gbar.as<double>(),
                       dP.as<double>(), weights.as<double>(), L.n);
    FE_HIP_CHECK(hipGetLastError());
  }
  FE_HIP_CHECK(hipStreamSynchronize(s));
  return FE_OK;
}

fe_status patch_weights(fe_problem* p, int level, int mode, DeviceBuf& weights, hipStream_t s);

fe_status setup_patch_factors(fe_problem* p, int level, int mode, hipStream_t s) {
  if (p->desc.geometry != FE_GEOM_DEFORMED) return fail(FE_EINVAL, "per-patch factors need the deformed geometry");
  if (mode < 1 || mode > 3) return fail(FE_EINVAL, "factor mode must be 1, 2 or 3");
  DeviceBuf weights;
  FE_CHECK(patch_weights(p, level, mode, weights, s));
  FE_DISPATCH_K(p->K, return eig_from_weights<KK>(p, level, mode, weights.as<double>(), s));
}

fe_status averaged_patch_weights(fe_problem* p, int level, DeviceBuf& weights, hipStream_t s) {
  FE_DISPATCH_K(p->K, return averaged_factors_typed<KK>(p, level, weights, s));
}

}  // namespace fe
