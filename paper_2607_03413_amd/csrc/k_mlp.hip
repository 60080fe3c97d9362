// Learned per-patch 1D factors on the deformed mesh.
//
//  * features: per cell, n kappa det(J) J^{-1} J^{-T} at the cell centre (6
//    entries), log kappa and log(n^3 det J) there; 8 cells per patch -> 64;
//  * training targets: the best Kronecker-sum fit of the patch operator,
//    min ||A_p - A_sep(w)||_F, by alternating least squares.  A_p is never
//    formed: every inner product the fit needs is a contraction of the 4x4x4
//    tensor C[i,j,l] = <A_p, E_l (x) E_j (x) E_i>, E in {D on interval 0, D on
//    interval 1, B on 0, B on 1}, which is integrated directly from the
//    quadrature metric (one wavefront per patch, one lane per entry of C);
//    the 1D Gram matrix of the E's supplies the norms of separable terms;
//  * model: 64 -> 64 -> 64 -> 12 MLP (tanh), FP32, trained with hand-written
//    forward, backward and Adam kernels; its output (12 log-weights) feeds the
//    batched 1D eigensolver that builds the per-patch FDM data (mode 2).
#include <cmath>
#include <numeric>

#include "fe_internal.h"
#include "kernel_common.h"

namespace fe {

constexpr int kIn = 64, kHid = 64, kOut = 12;
static_assert(kIn <= 256 && kHid <= 256, "k_layer_bwd_w splits the batch over 256 / nin thread groups");
constexpr int kW1 = kHid * kIn, kW2 = kHid * kHid, kW3 = kOut * kHid;
constexpr int kParams = kW1 + kHid + kW2 + kHid + kW3 + kOut;   // 9100
// Rows whose loss partials (ceil(rows * kOut / 256), one per block) fit the
// 1024 partial slots of the reduction scratch, below its result slot (2040).
constexpr int kMaxLossRows = 1024 * 256 / kOut;   // 21845

fe_status averaged_patch_weights(fe_problem* p, int level, DeviceBuf& weights, hipStream_t s);

// ---------------------------------------------------------------- features

__device__ __forceinline__ double deform_shift_m(double x, double y, double z, double amp) {
  return amp * sin(2.0 * M_PI * x) * sin(2.0 * M_PI * y) * sin(2.0 * M_PI * z);
}

// tab: [v(0.5) (K), d(0.5) (K), GLL nodes (K)]
template <int K>
__global__ void __launch_bounds__(256) k_cell_features(const double* __restrict__ tab, int n, double amp,
                                                       const int* __restrict__ modes, const double* __restrict__ mamp,
                                                       const double* __restrict__ mph, int n_modes, double scale,
                                                       double* __restrict__ out, int64_t n_cells) {
  const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= n_cells) return;
  const int cx = (int)(cell % n), cy = (int)((cell / n) % n), cz = (int)(cell / ((int64_t)n * n));
  const double* v = tab;
  const double* d = tab + K;
  const double* xn = tab + 2 * K;
  double x[3] = {0, 0, 0}, J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int iz = 0; iz < K; ++iz)
    for (int iy = 0; iy < K; ++iy)
      for (int ix = 0; ix < K; ++ix) {
        const double rx = (cx + xn[ix]) / n, ry = (cy + xn[iy]) / n, rz = (cz + xn[iz]) / n;
        const double sh = deform_shift_m(rx, ry, rz, amp);
        const double X[3] = {rx + sh, ry + sh, rz + sh};
        const double w = v[ix] * v[iy] * v[iz];
        const double wx = d[ix] * v[iy] * v[iz], wy = v[ix] * d[iy] * v[iz], wz = v[ix] * v[iy] * d[iz];
        for (int a = 0; a < 3; ++a) {
          x[a] += X[a] * w;
          J[a][0] += X[a] * wx;
          J[a][1] += X[a] * wy;
          J[a][2] += X[a] * wz;
        }
      }
  double g = 0.0;
  for (int j = 0; j < n_modes; ++j)
    g += mamp[j] * cos(M_PI * (modes[3 * j] * x[0] + modes[3 * j + 1] * x[1] + modes[3 * j + 2] * x[2]) + mph[j]);
  const double kap = exp(scale * g);
  const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
  double Ji[3][3];
  Ji[0][0] = c00 / det; Ji[1][0] = c01 / det; Ji[2][0] = c02 / det;
  Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
  Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
  Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
  Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
  Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
  Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
  auto C = [&](int a, int b) { return n * kap * det * (Ji[a][0] * Ji[b][0] + Ji[a][1] * Ji[b][1] + Ji[a][2] * Ji[b][2]); };
  double* o = out + cell * 8;
  o[0] = C(0, 0); o[1] = C(1, 1); o[2] = C(2, 2); o[3] = C(0, 1); o[4] = C(0, 2); o[5] = C(1, 2);
  o[6] = scale * g;
  o[7] = log(det * (double)n * n * n);
}

__global__ void __launch_bounds__(256) k_patch_gather_features(const double* __restrict__ cf, double* __restrict__ f,
                                                               int n) {
  const int nv = n - 1;
  const int64_t np = (int64_t)nv * nv * nv;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= np * 64) return;
  const int64_t pid = gid / 64;
  const int j = (int)(gid - pid * 64), s = j / 8, q = j % 8;
  const int vx = 1 + (int)(pid % nv), vy = 1 + (int)((pid / nv) % nv), vz = 1 + (int)(pid / ((int64_t)nv * nv));
  const int64_t cell = (vx - 1 + (s & 1)) + (int64_t)n * ((vy - 1 + ((s >> 1) & 1)) + (int64_t)n * (vz - 1 + (s >> 2)));
  f[gid] = cf[cell * 8 + q];
}

// ---------------------------------------------------------------- inner-product tensor C

// T1[((piece*2 + slot)*4 + variant)*K + q]: 1D quadratic form of the piece with the
// cell's basis values (variant bit 1: derivative on the left, bit 0: on the right).
template <int K>
__global__ void __launch_bounds__(64) k_patch_inner(const double* __restrict__ G, const double* __restrict__ T1,
                                                    double* __restrict__ C, int n) {
  constexpr int K3 = K * K * K;
  const int nv = n - 1;
  const int64_t pid = blockIdx.x;
  const int t = threadIdx.x;
  const int px = t & 3, py = (t >> 2) & 3, pz = t >> 4;
  const int vx = 1 + (int)(pid % nv), vy = 1 + (int)((pid / nv) % nv), vz = 1 + (int)(pid / ((int64_t)nv * nv));
  double acc = 0.0;
  for (int s = 0; s < 8; ++s) {
    const int sx = s & 1, sy = (s >> 1) & 1, sz = s >> 2;
    const int64_t cell = (vx - 1 + sx) + (int64_t)n * ((vy - 1 + sy) + (int64_t)n * (vz - 1 + sz));
    const double* Gc = G + cell * 6 * K3;
    const double* Tx = T1 + (px * 2 + sx) * 4 * K;
    const double* Ty = T1 + (py * 2 + sy) * 4 * K;
    const double* Tz = T1 + (pz * 2 + sz) * 4 * K;
    for (int q = 0; q < K3; ++q) {
      const int qx = q % K, qy = (q / K) % K, qz = q / (K * K);
      // pair (a, b) -> variants per axis: x uses bit (a==0, b==0), etc.
      double sum = 0.0;
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          const int comp = a == b ? a : (a + b == 1 ? 3 : (a + b == 2 ? 4 : 5));
          const double g = Gc[comp * K3 + q];
          const int vxv = 2 * (a == 0) + (b == 0), vyv = 2 * (a == 1) + (b == 1), vzv = 2 * (a == 2) + (b == 2);
          sum += g * Tx[vxv * K + qx] * Ty[vyv * K + qy] * Tz[vzv * K + qz];
        }
      acc += sum;
    }
  }
  C[pid * 64 + t] = acc;
}

// ---------------------------------------------------------------- alternating least squares

struct R1 {   // rank-one tensor a (x) b (x) c in the 4-piece basis per axis
  double v[3][4];
};

__device__ __forceinline__ double quad4(const double* G1, const double* a, const double* b) {
  double s = 0.0;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) s += a[i] * G1[i * 4 + j] * b[j];
  return s;
}
__device__ __forceinline__ double gdot(const double* G1, const R1& u, const R1& w) {
  return quad4(G1, u.v[0], w.v[0]) * quad4(G1, u.v[1], w.v[1]) * quad4(G1, u.v[2], w.v[2]);
}
__device__ __forceinline__ double cdot(const double* C, const R1& u) {
  double s = 0.0;
  for (int l = 0; l < 4; ++l)
    for (int j = 0; j < 4; ++j)
      for (int i = 0; i < 4; ++i) s += C[l * 16 + j * 4 + i] * u.v[0][i] * u.v[1][j] * u.v[2][l];
  return s;
}

template <int N>
__device__ void spd_solve(double (&A)[N][N], double (&b)[N]) {
  for (int j = 0; j < N; ++j) {   // Gaussian elimination with partial pivoting
    int piv = j;
    for (int i = j + 1; i < N; ++i)
      if (fabs(A[i][j]) > fabs(A[piv][j])) piv = i;
    if (piv != j) {
      for (int c = 0; c < N; ++c) { const double t = A[j][c]; A[j][c] = A[piv][c]; A[piv][c] = t; }
      const double t = b[j]; b[j] = b[piv]; b[piv] = t;
    }
    for (int i = j + 1; i < N; ++i) {
      const double f = A[i][j] / A[j][j];
      for (int c = j; c < N; ++c) A[i][c] -= f * A[j][c];
      b[i] -= f * b[j];
    }
  }
  for (int i = N - 1; i >= 0; --i) {
    double s = b[i];
    for (int c = i + 1; c < N; ++c) s -= A[i][c] * b[c];
    b[i] = s / A[i][i];
  }
}

// w: [alpha_x0, alpha_x1, alpha_y0, ..., beta_z1]; stiffness vector of axis d is
// (a0, a1, 0, 0), mass vector (0, 0, b0, b1) in the piece basis (D0, D1, B0, B1).
__device__ __forceinline__ void kvec(const double* w, int d, double* o) { o[0] = w[2 * d]; o[1] = w[2 * d + 1]; o[2] = o[3] = 0.0; }
__device__ __forceinline__ void mvec(const double* w, int d, double* o) { o[0] = o[1] = 0.0; o[2] = w[6 + 2 * d]; o[3] = w[7 + 2 * d]; }
__device__ __forceinline__ void unit(int i, double* o) { o[0] = o[1] = o[2] = o[3] = 0.0; o[i] = 1.0; }

// term e of A_sep (stiffness along e, masses elsewhere)
__device__ __forceinline__ R1 term(const double* w, int e) {
  R1 r;
  for (int d = 0; d < 3; ++d) {
    if (d == e) kvec(w, d, r.v[d]);
    else mvec(w, d, r.v[d]);
  }
  return r;
}

__global__ void __launch_bounds__(64) k_patch_als(const double* __restrict__ Call, const double* __restrict__ G1g,
                                                  const double* __restrict__ w0, const double* __restrict__ proj,
                                                  double log_h3, int sweeps, double* __restrict__ targets,
                                                  int64_t n_patches) {
  const int64_t pid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pid >= n_patches) return;
  double G1[16];
  for (int i = 0; i < 16; ++i) G1[i] = G1g[i];
  const double* C = Call + pid * 64;
  double w[12];
  for (int i = 0; i < 12; ++i) w[i] = w0[pid * 12 + i];
  for (int it = 0; it < sweeps; ++it) {
    // stiffness weights: u_{d,c} = unit(c) along d, masses elsewhere
    {
      R1 U[6];
      for (int d = 0; d < 3; ++d)
        for (int c = 0; c < 2; ++c) {
          R1& u = U[2 * d + c];
          for (int e = 0; e < 3; ++e) {
            if (e == d) unit(c, u.v[e]);
            else mvec(w, e, u.v[e]);
          }
        }
      double H[6][6], r[6];
      for (int i = 0; i < 6; ++i) {
        r[i] = cdot(C, U[i]);
        for (int j = 0; j < 6; ++j) H[i][j] = gdot(G1, U[i], U[j]);
      }
      spd_solve<6>(H, r);
      double mx = 0.0;
      for (int i = 0; i < 6; ++i) mx = fmax(mx, fabs(r[i]));
      for (int i = 0; i < 6; ++i) w[i] = fmax(r[i], 1e-12 * mx);
    }
    // mass weights of each axis d: V_c = sum_{e != d} term e with unit(2 + c) along d
    for (int d = 0; d < 3; ++d) {
      const R1 T0 = term(w, d);
      R1 V[2][2];   // [c][which of the two e != d]
      for (int c = 0; c < 2; ++c) {
        int q = 0;
        for (int e = 0; e < 3; ++e) {
          if (e == d) continue;
          R1 t = term(w, e);
          unit(2 + c, t.v[d]);
          V[c][q++] = t;
        }
      }
      double H[2][2], r[2];
      for (int i = 0; i < 2; ++i) {
        r[i] = cdot(C, V[i][0]) + cdot(C, V[i][1]) - gdot(G1, V[i][0], T0) - gdot(G1, V[i][1], T0);
        for (int j = 0; j < 2; ++j)
          H[i][j] = gdot(G1, V[i][0], V[j][0]) + gdot(G1, V[i][0], V[j][1]) + gdot(G1, V[i][1], V[j][0]) +
                    gdot(G1, V[i][1], V[j][1]);
      }
      spd_solve<2>(H, r);
      const double mx = fmax(fabs(r[0]), fabs(r[1]));
      w[6 + 2 * d] = fmax(r[0], 1e-12 * mx);
      w[7 + 2 * d] = fmax(r[1], 1e-12 * mx);
    }
  }
  // normalized, gauge-fixed log-weights
  double t[12];
  for (int i = 0; i < 12; ++i) t[i] = log(w[i]) - log_h3;
  for (int i = 0; i < 12; ++i) {
    double s = 0.0;
    for (int j = 0; j < 12; ++j) s += proj[i * 12 + j] * t[j];
    targets[pid * 12 + i] = s;
  }
}

// ---------------------------------------------------------------- MLP (FP32)

__global__ void __launch_bounds__(256) k_to_f32(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) b[e] = (float)a[e];
}
__global__ void __launch_bounds__(256) k_to_f64(const float* __restrict__ a, double* __restrict__ b, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) b[e] = (double)a[e];
}

// Y[b, o] = act(sum_i W[o, i] X[b, i] + bias[o]); one thread per (b, o)
__global__ void __launch_bounds__(256) k_layer_fwd(const float* __restrict__ X, const float* __restrict__ W,
                                                   const float* __restrict__ bias, float* __restrict__ Y, int nb,
                                                   int nin, int nout, int act) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= nb * nout) return;
  const int b = gid / nout, o = gid - b * nout;
  float s = bias[o];
  for (int i = 0; i < nin; ++i) s = fmaf(W[o * nin + i], X[b * nin + i], s);
  Y[gid] = act ? tanhf(s) : s;
}

// output delta d = 2 (Y - T) / (nb * nout); partial loss sums per block
__global__ void __launch_bounds__(256) k_out_delta(const float* __restrict__ Y, const float* __restrict__ T,
                                                   float* __restrict__ d, int n, float scale,
                                                   double* __restrict__ part) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  double sq = 0.0;
  if (gid < n) {
    const float diff = Y[gid] - T[gid];
    d[gid] = scale * diff;
    sq = (double)diff * diff;
  }
  __shared__ double red[256];
  red[threadIdx.x] = sq;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// dprev[b, i] = (sum_o d[b, o] W[o, i]) * (1 - a[b, i]^2)
__global__ void __launch_bounds__(256) k_layer_bwd_delta(const float* __restrict__ d, const float* __restrict__ W,
                                                         const float* __restrict__ a, float* __restrict__ dprev,
                                                         int nb, int nin, int nout) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= nb * nin) return;
  const int b = gid / nin, i = gid - b * nin;
  float s = 0.0f;
  for (int o = 0; o < nout; ++o) s = fmaf(d[b * nout + o], W[o * nin + i], s);
  const float ai = a[gid];
  dprev[gid] = s * (1.0f - ai * ai);
}

// Weight and bias gradients of one layer: gW[o][i] = sum_b d[b][o] X[b][i],
// gb[o] = sum_b d[b][o].  One block per output o; the batch is split over
// Q = 256 / nin groups of nin threads (thread (q, i) sums rows b = q, q+Q, ...
// for input i), and the Q partial sums are added in order through LDS.
// (One thread per weight walking the whole batch left the GPU nearly empty.)
__global__ void __launch_bounds__(256) k_layer_bwd_w(const float* __restrict__ d, const float* __restrict__ X,
                                                     float* __restrict__ gW, float* __restrict__ gb, int nb, int nin,
                                                     int nout) {
  __shared__ float part[256];
  __shared__ float bpart[256];
  const int o = blockIdx.x, t = threadIdx.x;
  const int Q = 256 / nin, q = t / nin, i = t - q * nin;
  float s = 0.0f, sb = 0.0f;
  if (q < Q) {
    for (int b = q; b < nb; b += Q) {
      const float db = d[b * nout + o];
      s = fmaf(db, X[b * nin + i], s);
      sb += db;
    }
  }
  part[t] = s;
  bpart[t] = sb;
  __syncthreads();
  if (t < nin) {
    float w = part[t];
    for (int r = 1; r < Q; ++r) w += part[r * nin + t];
    gW[o * nin + t] = w;
  }
  if (t == 0) {
    float b = bpart[0];
    for (int r = 1; r < Q; ++r) b += bpart[r * nin];
    gb[o] = b;
  }
}

__global__ void __launch_bounds__(256) k_adam(float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, int n, float lr,
                                              float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = 0.9f * m[i] + 0.1f * gi;
  const float vi = 0.999f * v[i] + 0.001f * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

__global__ void __launch_bounds__(256) k_gather_rows(const float* __restrict__ src, const int* __restrict__ idx,
                                                     float* __restrict__ dst, int nrows, int ncols) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= nrows * ncols) return;
  const int r = gid / ncols, c = gid - r * ncols;
  dst[gid] = src[(int64_t)idx[r] * ncols + c];
}

// ---------------------------------------------------------------- host side

struct MlpWork {
  DeviceBuf a1, a2, y, d3, d2, d1, g, xb, tb, idx;
  int cap = 0;
  fe_status ensure(int nb) {
    if (nb <= cap) return FE_OK;
    FE_CHECK(a1.alloc((size_t)nb * kHid * 4));
    FE_CHECK(a2.alloc((size_t)nb * kHid * 4));
    FE_CHECK(y.alloc((size_t)nb * kOut * 4));
    FE_CHECK(d3.alloc((size_t)nb * kOut * 4));
    FE_CHECK(d2.alloc((size_t)nb * kHid * 4));
    FE_CHECK(d1.alloc((size_t)nb * kHid * 4));
    FE_CHECK(g.alloc((size_t)kParams * 4));
    FE_CHECK(xb.alloc((size_t)nb * kIn * 4));
    FE_CHECK(tb.alloc((size_t)nb * kOut * 4));
    FE_CHECK(idx.alloc((size_t)nb * 4));
    cap = nb;
    return FE_OK;
  }
};

static unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

// The model changed: the learned patch factors of every level, and the
// Chebyshev eigenvalue estimates taken with them, are out of date.
static void invalidate_learned_factors(fe_problem* p) {
  for (Level& L : p->levels) {
    L.patch_eig_ready[2] = false;
    if (L.lmax_key >= 0 && L.lmax_key / 1000 == 2) L.lmax_key = -1;
  }
}

static fe_status mlp_forward(const float* P, const float* X, int nb, MlpWork& w, hipStream_t s) {
  const float *W1 = P, *b1 = W1 + kW1, *W2 = b1 + kHid, *b2 = W2 + kW2, *W3 = b2 + kHid, *b3 = W3 + kW3;
  hipLaunchKernelGGL(k_layer_fwd, dim3(nblk(nb * kHid)), dim3(256), 0, s, X, W1, b1, w.a1.as<float>(), nb, kIn, kHid, 1);
  hipLaunchKernelGGL(k_layer_fwd, dim3(nblk(nb * kHid)), dim3(256), 0, s, w.a1.as<float>(), W2, b2, w.a2.as<float>(),
                     nb, kHid, kHid, 1);
  hipLaunchKernelGGL(k_layer_fwd, dim3(nblk(nb * kOut)), dim3(256), 0, s, w.a2.as<float>(), W3, b3, w.y.as<float>(),
                     nb, kHid, kOut, 0);
  FE_HIP_CHECK(hipGetLastError());
  return FE_OK;
}

// gradient of the mean squared error into w.g; loss partials into red (device)
static fe_status mlp_backward(const float* P, const float* X, const float* T, int nb, MlpWork& w, double* part,
                              int* nparts, hipStream_t s) {
  const float *W1 = P, *W2 = W1 + kW1 + kHid, *W3 = W2 + kW2 + kHid;
  float* g = w.g.as<float>();
  float *gW1 = g, *gb1 = gW1 + kW1, *gW2 = gb1 + kHid, *gb2 = gW2 + kW2, *gW3 = gb2 + kHid, *gb3 = gW3 + kW3;
  const int n = nb * kOut;
  *nparts = (int)nblk(n);
  hipLaunchKernelGGL(k_out_delta, dim3(nblk(n)), dim3(256), 0, s, w.y.as<float>(), T, w.d3.as<float>(), n,
                     2.0f / (float)n, part);
  hipLaunchKernelGGL(k_layer_bwd_w, dim3(kOut), dim3(256), 0, s, w.d3.as<float>(), w.a2.as<float>(), gW3,
                     gb3, nb, kHid, kOut);
  hipLaunchKernelGGL(k_layer_bwd_delta, dim3(nblk(nb * kHid)), dim3(256), 0, s, w.d3.as<float>(), W3,
                     w.a2.as<float>(), w.d2.as<float>(), nb, kHid, kOut);
  hipLaunchKernelGGL(k_layer_bwd_w, dim3(kHid), dim3(256), 0, s, w.d2.as<float>(), w.a1.as<float>(), gW2,
                     gb2, nb, kHid, kHid);
  hipLaunchKernelGGL(k_layer_bwd_delta, dim3(nblk(nb * kHid)), dim3(256), 0, s, w.d2.as<float>(), W2,
                     w.a1.as<float>(), w.d1.as<float>(), nb, kHid, kHid);
  hipLaunchKernelGGL(k_layer_bwd_w, dim3(kHid), dim3(256), 0, s, w.d1.as<float>(), X, gW1, gb1, nb, kIn,
                     kHid);
  FE_HIP_CHECK(hipGetLastError());
  return FE_OK;
}

static fe_status ensure_model(fe_problem* p) {
  if (p->mlp_params.p) return FE_OK;
  FE_CHECK(p->mlp_params.alloc(kParams * 4));
  FE_CHECK(p->mlp_adam_m.alloc(kParams * 4));
  FE_CHECK(p->mlp_adam_v.alloc(kParams * 4));
  return FE_OK;
}

template <int K>
static fe_status features_typed(fe_problem* p, int level, double* feats, hipStream_t s) {
  Level& L = p->levels[level];
  std::vector<double> nodes = gll_nodes(K - 1), tab(3 * K);
  for (int i = 0; i < K; ++i) {
    tab[i] = lagrange_value(nodes, i, 0.5);
    tab[K + i] = lagrange_deriv(nodes, i, 0.5);
    tab[2 * K + i] = nodes[i];
  }
  const int nm = (int)p->amp.size();
  std::vector<double> md(tab);
  md.insert(md.end(), p->amp.begin(), p->amp.end());
  md.insert(md.end(), p->phase.begin(), p->phase.end());
  DeviceBuf d, cf;
  FE_CHECK(d.alloc(md.size() * sizeof(double) + 3 * nm * sizeof(int) + 64));
  FE_CHECK(cf.alloc(L.n_cells * 8 * sizeof(double)));
  double* dd = d.as<double>();
  int* dm = reinterpret_cast<int*>(dd + md.size());
  FE_HIP_CHECK(hipMemcpyAsync(dd, md.data(), md.size() * sizeof(double), hipMemcpyHostToDevice, s));
  if (nm) FE_HIP_CHECK(hipMemcpyAsync(dm, p->modes.data(), 3 * nm * sizeof(int), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL((k_cell_features<K>), dim3(nblk(L.n_cells)), dim3(256), 0, s, dd, L.n, p->desc.deform_amp, dm,
                     dd + 3 * K, dd + 3 * K + nm, nm, p->coef_scale, cf.as<double>(), L.n_cells);
  const int64_t nv = L.n - 1, np = nv * nv * nv;
  if (np > 0)
    hipLaunchKernelGGL(k_patch_gather_features, dim3(nblk(np * 64)), dim3(256), 0, s, cf.as<double>(), feats, L.n);
  FE_HIP_CHECK(hipGetLastError());
  FE_HIP_CHECK(hipStreamSynchronize(s));
  return FE_OK;
}

// 1D quadratic forms of the pieces with the cell basis at the metric's Gauss points.
static std::vector<double> inner_table(int k) {
  const int K = k + 1, M = 2 * k - 1;
  std::vector<double> nodes = gll_nodes(k), xq, wq;
  gauss_rule(K, xq, wq);
  std::vector<double> B = mass_1d(k), D = stiffness_1d(k);
  // pieces on the interior of the two-interval line (M x M)
  std::vector<std::vector<double>> E(4, std::vector<double>(M * M, 0.0));
  for (int pc = 0; pc < 4; ++pc) {
    const int e = pc & 1;
    const std::vector<double>& mat = pc < 2 ? D : B;
    for (int i = 0; i < K; ++i)
      for (int j = 0; j < K; ++j) {
        const int gi = k * e + i - 1, gj = k * e + j - 1;
        if (gi < 0 || gi >= M || gj < 0 || gj >= M) continue;
        E[pc][gi * M + gj] = mat[i * K + j];
      }
  }
  std::vector<double> T(4 * 2 * 4 * K, 0.0);
  for (int pc = 0; pc < 4; ++pc)
    for (int slot = 0; slot < 2; ++slot)
      for (int var = 0; var < 4; ++var)
        for (int q = 0; q < K; ++q) {
          double s = 0.0;
          for (int i = 0; i < K; ++i)
            for (int j = 0; j < K; ++j) {
              const int gi = slot * k + i - 1, gj = slot * k + j - 1;
              if (gi < 0 || gi >= M || gj < 0 || gj >= M) continue;
              const double fl = (var & 2) ? lagrange_deriv(nodes, i, xq[q]) : lagrange_value(nodes, i, xq[q]);
              const double fr = (var & 1) ? lagrange_deriv(nodes, j, xq[q]) : lagrange_value(nodes, j, xq[q]);
              s += fl * E[pc][gi * M + gj] * fr;
            }
          T[((pc * 2 + slot) * 4 + var) * K + q] = s;
        }
  return T;
}

static std::vector<double> piece_gram(int k) {
  const int K = k + 1, M = 2 * k - 1;
  std::vector<double> B = mass_1d(k), D = stiffness_1d(k);
  std::vector<std::vector<double>> E(4, std::vector<double>(M * M, 0.0));
  for (int pc = 0; pc < 4; ++pc) {
    const int e = pc & 1;
    const std::vector<double>& mat = pc < 2 ? D : B;
    for (int i = 0; i < K; ++i)
      for (int j = 0; j < K; ++j) {
        const int gi = k * e + i - 1, gj = k * e + j - 1;
        if (gi < 0 || gi >= M || gj < 0 || gj >= M) continue;
        E[pc][gi * M + gj] = mat[i * K + j];
      }
  }
  std::vector<double> G(16, 0.0);
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b)
      for (int i = 0; i < M * M; ++i) G[a * 4 + b] += E[a][i] * E[b][i];
  return G;
}

// projection that removes the three scaling gauges of the log-weights
static std::vector<double> gauge_projection() {
  double N[12][3] = {};
  for (int d = 0; d < 3; ++d) {
    N[6 + 2 * d][d] = N[7 + 2 * d][d] = 1.0;
    for (int e = 0; e < 3; ++e)
      if (e != d) N[2 * e][d] = N[2 * e + 1][d] = -1.0;
  }
  double NtN[3][3] = {};
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      for (int i = 0; i < 12; ++i) NtN[a][b] += N[i][a] * N[i][b];
  // inverse of the 3x3 Gram by cofactors
  const double det = NtN[0][0] * (NtN[1][1] * NtN[2][2] - NtN[1][2] * NtN[2][1]) -
                     NtN[0][1] * (NtN[1][0] * NtN[2][2] - NtN[1][2] * NtN[2][0]) +
                     NtN[0][2] * (NtN[1][0] * NtN[2][1] - NtN[1][1] * NtN[2][0]);
  double I[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      const int r0 = (b + 1) % 3, r1 = (b + 2) % 3, c0 = (a + 1) % 3, c1 = (a + 2) % 3;
      I[a][b] = (NtN[r0][c0] * NtN[r1][c1] - NtN[r0][c1] * NtN[r1][c0]) / det;
    }
  std::vector<double> P(144, 0.0);
  for (int i = 0; i < 12; ++i)
    for (int j = 0; j < 12; ++j) {
      double s = 0.0;
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) s += N[i][a] * I[a][b] * N[j][b];
      P[i * 12 + j] = (i == j ? 1.0 : 0.0) - s;
    }
  return P;
}

template <int K>
static fe_status inner_typed(fe_problem* p, int level, double* C, hipStream_t s) {
  Level& L = p->levels[level];
  const int64_t nv = L.n - 1, np = nv * nv * nv;
  std::vector<double> T = inner_table(K - 1);
  DeviceBuf d;
  FE_CHECK(d.alloc(T.size() * sizeof(double)));
  FE_HIP_CHECK(hipMemcpyAsync(d.p, T.data(), T.size() * sizeof(double), hipMemcpyHostToDevice, s));
  if (np > 0)
    hipLaunchKernelGGL((k_patch_inner<K>), dim3((unsigned)np), dim3(64), 0, s, L.metric64.as<double>(),
                       d.as<double>(), C, L.n);
  FE_HIP_CHECK(hipGetLastError());
  FE_HIP_CHECK(hipStreamSynchronize(s));
  return FE_OK;
}

static fe_status fit_targets(fe_problem* p, int level, int sweeps, double* targets, hipStream_t s) {
  Level& L = p->levels[level];
  const int64_t nv = L.n - 1, np = nv * nv * nv;
  if (np == 0) return FE_OK;
  DeviceBuf C, w0, consts;
  FE_CHECK(C.alloc(np * 64 * sizeof(double)));
  FE_DISPATCH_K(p->K, FE_CHECK(inner_typed<KK>(p, level, C.as<double>(), s)); break);
  FE_CHECK(averaged_patch_weights(p, level, w0, s));
  std::vector<double> G1 = piece_gram(p->k), P = gauge_projection();
  std::vector<double> cst(G1);
  cst.insert(cst.end(), P.begin(), P.end());
  FE_CHECK(consts.alloc(cst.size() * sizeof(double)));
  FE_HIP_CHECK(hipMemcpyAsync(consts.p, cst.data(), cst.size() * sizeof(double), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_patch_als, dim3((unsigned)((np + 63) / 64)), dim3(64), 0, s, C.as<double>(),
                     consts.as<double>(), w0.as<double>(), consts.as<double>() + 16, std::log(L.h) / 3.0, sweeps,
                     targets, np);
  FE_HIP_CHECK(hipGetLastError());
  FE_HIP_CHECK(hipStreamSynchronize(s));
  return FE_OK;
}

__global__ void __launch_bounds__(256) k_weights_from_log(const float* __restrict__ y, double log_h3,
                                                          double* __restrict__ w, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) w[e] = exp((double)y[e] + log_h3);
}

__global__ void __launch_bounds__(256) k_weights_from_log64(const double* __restrict__ y, double log_h3,
                                                            double* __restrict__ w, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) w[e] = exp(y[e] + log_h3);
}

// mode 1: averaged-geometry weights; mode 2: MLP prediction; mode 3: the
// per-patch best Kronecker-sum fit itself (the MLP's training target).
fe_status patch_weights(fe_problem* p, int level, int mode, DeviceBuf& weights, hipStream_t s) {
  if (mode == 1) return averaged_patch_weights(p, level, weights, s);
  if (mode == 3) {
    Level& L = p->levels[level];
    const int64_t nv = L.n - 1, np = nv * nv * nv;
    FE_CHECK(weights.alloc(std::max<int64_t>(np, 1) * 12 * sizeof(double)));
    if (np == 0) return FE_OK;
    DeviceBuf tg;
    FE_CHECK(tg.alloc(np * 12 * sizeof(double)));
    FE_CHECK(fit_targets(p, level, 20, tg.as<double>(), s));
    hipLaunchKernelGGL(k_weights_from_log64, dim3(nblk(np * 12)), dim3(256), 0, s, tg.as<double>(),
                       std::log(L.h) / 3.0, weights.as<double>(), np * 12);
    FE_HIP_CHECK(hipGetLastError());
    FE_HIP_CHECK(hipStreamSynchronize(s));
    return FE_OK;
  }
  if (!p->mlp_ready) return fail(FE_EINVAL, "learned factors need a trained model (fe_mlp_train or fe_mlp_set_params)");
  Level& L = p->levels[level];
  const int64_t nv = L.n - 1, np = nv * nv * nv;
  FE_CHECK(weights.alloc(std::max<int64_t>(np, 1) * 12 * sizeof(double)));
  if (np == 0) return FE_OK;
  DeviceBuf f64, f32;
  FE_CHECK(f64.alloc(np * 64 * sizeof(double)));
  FE_CHECK(f32.alloc(np * 64 * sizeof(float)));
  FE_DISPATCH_K(p->K, FE_CHECK(features_typed<KK>(p, level, f64.as<double>(), s)); break);
  hipLaunchKernelGGL(k_to_f32, dim3(nblk(np * 64)), dim3(256), 0, s, f64.as<double>(), f32.as<float>(), np * 64);
  MlpWork w;
  const int chunk = 65536;
  FE_CHECK(w.ensure((int)std::min<int64_t>(np, chunk)));
  for (int64_t b0 = 0; b0 < np; b0 += chunk) {
    const int nb = (int)std::min<int64_t>(chunk, np - b0);
    FE_CHECK(mlp_forward(p->mlp_params.as<float>(), f32.as<float>() + b0 * 64, nb, w, s));
    hipLaunchKernelGGL(k_weights_from_log, dim3(nblk(nb * 12)), dim3(256), 0, s, w.y.as<float>(), std::log(L.h) / 3.0,
                       weights.as<double>() + b0 * 12, (int64_t)nb * 12);
  }
  FE_HIP_CHECK(hipGetLastError());
  FE_HIP_CHECK(hipStreamSynchronize(s));
  return FE_OK;
}

}  // namespace fe

using namespace fe;

static fe_status check_learned(fe_problem* p, int level) {
  if (!p) return fail(FE_EINVAL, "null problem");
  if (p->desc.geometry != FE_GEOM_DEFORMED) return fail(FE_EINVAL, "learned factors need the deformed geometry");
  return check_level(p, level);
}

extern "C" {

int fe_mlp_num_params(void) { return kParams; }

int64_t fe_num_patches(const fe_problem* p, int level) {
  if (!p || level < -1 || level >= (int)p->levels.size()) return -1;
  const int64_t nv = level_of(p, level).n - 1;
  return p->dim == 3 ? nv * nv * nv : nv * nv;
}

fe_status fe_patch_features(fe_problem* p, int level, double* feats, void* stream) {
  FE_CHECK(check_learned(p, level));
  FE_CHECK(check_ptr(feats, "feats"));
  const int li = level < 0 ? (int)p->levels.size() - 1 : level;
  FE_DISPATCH_K(p->K, return features_typed<KK>(p, li, feats, (hipStream_t)stream));
}

fe_status fe_patch_inner_tensor(fe_problem* p, int level, double* C, void* stream) {
  FE_CHECK(check_learned(p, level));
  FE_CHECK(check_ptr(C, "C"));
  const int li = level < 0 ? (int)p->levels.size() - 1 : level;
  FE_DISPATCH_K(p->K, return inner_typed<KK>(p, li, C, (hipStream_t)stream));
}

fe_status fe_patch_fit_targets(fe_problem* p, int level, int sweeps, double* targets, void* stream) {
  FE_CHECK(check_learned(p, level));
  FE_CHECK(check_ptr(targets, "targets"));
  if (sweeps < 0 || sweeps > 1000) return fail(FE_EINVAL, "sweeps out of range");
  const int li = level < 0 ? (int)p->levels.size() - 1 : level;
  return fit_targets(p, li, sweeps, targets, (hipStream_t)stream);
}

fe_status fe_mlp_set_params(fe_problem* p, const float* params, void* stream) {
  if (!p) return fail(FE_EINVAL, "null problem");
  FE_CHECK(check_ptr(params, "params"));
  FE_CHECK(ensure_model(p));
  hipStream_t s = (hipStream_t)stream;
  FE_HIP_CHECK(hipMemcpyAsync(p->mlp_params.p, params, kParams * 4, hipMemcpyDeviceToDevice, s));
  FE_HIP_CHECK(hipMemsetAsync(p->mlp_adam_m.p, 0, kParams * 4, s));
  FE_HIP_CHECK(hipMemsetAsync(p->mlp_adam_v.p, 0, kParams * 4, s));
  FE_HIP_CHECK(hipStreamSynchronize(s));
  p->mlp_ready = 1;
  p->mlp_step = 0;
  invalidate_learned_factors(p);
  return FE_OK;
}

fe_status fe_mlp_get_params(const fe_problem* p, float* params, void* stream) {
  if (!p || !p->mlp_ready) return fail(FE_EINVAL, "no model");
  FE_CHECK(check_ptr(params, "params"));
  hipStream_t s = (hipStream_t)stream;
  FE_HIP_CHECK(hipMemcpyAsync(params, p->mlp_params.p, kParams * 4, hipMemcpyDeviceToDevice, s));
  FE_HIP_CHECK(hipStreamSynchronize(s));
  return FE_OK;
}

fe_status fe_mlp_forward(fe_problem* p, const float* X, float* Y, int n, void* stream) {
  if (!p || !p->mlp_ready) return fail(FE_EINVAL, "no model");
  FE_CHECK(check_ptr(X, "X"));
  FE_CHECK(check_ptr(Y, "Y"));
  if (n < 1) return fail(FE_EINVAL, "n must be positive");
  hipStream_t s = (hipStream_t)stream;
  MlpWork w;
  FE_CHECK(w.ensure(n));
  FE_CHECK(mlp_forward(p->mlp_params.as<float>(), X, n, w, s));
  FE_HIP_CHECK(hipMemcpyAsync(Y, w.y.p, (size_t)n * kOut * 4, hipMemcpyDeviceToDevice, s));
  FE_HIP_CHECK(hipStreamSynchronize(s));
  return FE_OK;
}

fe_status fe_mlp_loss_grad(fe_problem* p, const float* X, const float* T, int n, float* grad, double* loss,
                           void* stream) {
  if (!p || !p->mlp_ready) return fail(FE_EINVAL, "no model");
  FE_CHECK(check_ptr(X, "X"));
  FE_CHECK(check_ptr(T, "T"));
  FE_CHECK(check_ptr(grad, "grad"));
  if (n < 1 || !loss) return fail(FE_EINVAL, "bad arguments");
  // the loss partials (one per 256 outputs) must stay below the result slot of
  // the reduction scratch: checked before anything is launched
  if (n > kMaxLossRows) return fail(FE_EINVAL, "batch too large for the loss reduction (n > 21845)");
  hipStream_t s = (hipStream_t)stream;
  MlpWork w;
  FE_CHECK(w.ensure(n));
  int nparts = 0;
  FE_CHECK(mlp_forward(p->mlp_params.as<float>(), X, n, w, s));
  FE_CHECK(mlp_backward(p->mlp_params.as<float>(), X, T, n, w, p->red_scratch.as<double>(), &nparts, s));
  FE_CHECK(finish_reduction(p, nparts, p->red_scratch.as<double>() + 2040, s));
  FE_HIP_CHECK(hipMemcpyAsync(grad, w.g.p, kParams * 4, hipMemcpyDeviceToDevice, s));
  double tot = 0.0;
  FE_HIP_CHECK(hipMemcpyAsync(&tot, p->red_scratch.as<double>() + 2040, sizeof(double), hipMemcpyDeviceToHost, s));
  FE_HIP_CHECK(hipStreamSynchronize(s));
  *loss = tot / ((double)n * kOut);
  return FE_OK;
}

fe_status fe_mlp_adam_step(fe_problem* p, const float* grad, double lr, void* stream) {
  if (!p || !p->mlp_ready) return fail(FE_EINVAL, "no model");
  FE_CHECK(check_ptr(grad, "grad"));
  hipStream_t s = (hipStream_t)stream;
  p->mlp_step += 1;
  const double t = p->mlp_step;
  hipLaunchKernelGGL(k_adam, dim3(nblk(kParams)), dim3(256), 0, s, p->mlp_params.as<float>(), grad,
                     p->mlp_adam_m.as<float>(), p->mlp_adam_v.as<float>(), kParams, (float)lr,
                     (float)(1.0 - std::pow(0.9, t)), (float)(1.0 - std::pow(0.999, t)));
  FE_HIP_CHECK(hipGetLastError());
  invalidate_learned_factors(p);
  return FE_OK;
}

fe_status fe_mlp_train(fe_problem* p, const float* X, const float* T, int n, int epochs, int batch, double lr,
                       uint64_t seed, double* final_loss, void* stream) {
  if (!p || !p->mlp_ready) return fail(FE_EINVAL, "initialize the model with fe_mlp_set_params first");
  FE_CHECK(check_ptr(X, "X"));
  FE_CHECK(check_ptr(T, "T"));
  if (n < 1 || epochs < 0 || batch < 1 || batch > 4096 || !(lr > 0)) return fail(FE_EINVAL, "bad arguments");
  static_assert(4096 <= kMaxLossRows, "training batches must fit the loss reduction");
  hipStream_t s = (hipStream_t)stream;
  MlpWork w;
  FE_CHECK(w.ensure(batch));
  std::vector<int> perm(n);
  std::iota(perm.begin(), perm.end(), 0);
  uint64_t st = seed;
  auto next = [&]() {   // splitmix64
    st += 0x9E3779B97F4A7C15ull;
    uint64_t z = st;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  double last = 0.0;
  for (int ep = 0; ep < epochs; ++ep) {
    for (int i = n - 1; i > 0; --i) std::swap(perm[i], perm[next() % (uint64_t)(i + 1)]);
    double ep_loss = 0.0;
    int nbt = 0;
    for (int b0 = 0; b0 + batch <= n; b0 += batch) {
      FE_HIP_CHECK(hipMemcpyAsync(w.idx.p, perm.data() + b0, batch * sizeof(int), hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL(k_gather_rows, dim3(nblk(batch * kIn)), dim3(256), 0, s, X, w.idx.as<int>(), w.xb.as<float>(),
                         batch, kIn);
      hipLaunchKernelGGL(k_gather_rows, dim3(nblk(batch * kOut)), dim3(256), 0, s, T, w.idx.as<int>(),
                         w.tb.as<float>(), batch, kOut);
      int nparts = 0;
      FE_CHECK(mlp_forward(p->mlp_params.as<float>(), w.xb.as<float>(), batch, w, s));
      FE_CHECK(mlp_backward(p->mlp_params.as<float>(), w.xb.as<float>(), w.tb.as<float>(), batch, w,
                            p->red_scratch.as<double>(), &nparts, s));
      FE_CHECK(finish_reduction(p, nparts, p->red_scratch.as<double>() + 2040, s));
      p->mlp_step += 1;
      const double t = p->mlp_step;
      hipLaunchKernelGGL(k_adam, dim3(nblk(kParams)), dim3(256), 0, s, p->mlp_params.as<float>(), w.g.as<float>(),
                         p->mlp_adam_m.as<float>(), p->mlp_adam_v.as<float>(), kParams, (float)lr,
                         (float)(1.0 - std::pow(0.9, t)), (float)(1.0 - std::pow(0.999, t)));
      double bl = 0.0;
      FE_HIP_CHECK(hipMemcpyAsync(&bl, p->red_scratch.as<double>() + 2040, sizeof(double), hipMemcpyDeviceToHost, s));
      FE_HIP_CHECK(hipStreamSynchronize(s));
      ep_loss += bl / ((double)batch * kOut);
      ++nbt;
    }
    last = nbt ? ep_loss / nbt : 0.0;
  }
  FE_HIP_CHECK(hipGetLastError());
  invalidate_learned_factors(p);
  if (final_loss) *final_loss = last;
  return FE_OK;
}

}  // extern "C"
