// Multigrid building blocks: cell-wise transfers (Algorithms 2 and 3 with the
// fused residual of Sec. 5), the fused Jacobi update of Algorithm 9, the
// coarse solve, BLAS-1 kernels with deterministic FP64 reductions, and the
// manufactured load vector.
//
// Transfers: one group of K^2 threads per parent cell produces (or consumes)
// all 2^3 children in a single launch; the z-, y- and x-contractions with
// P_0 / P_1 are shared between children with equal bits (sum factorization
// over the child tree), and each child's values are streamed once.  The
// paper instead launches one kernel per child slot and stores each level in
// child-major order to make those launches coalesce; with all children of a
// parent in one group, the lexicographic order is already coalesced.
#include <cmath>

#include "fe_internal.h"
#include "kernel_common.h"

namespace fe {

template <typename T, int K>
__global__ void __launch_bounds__(256) k_prolong3(const T* __restrict__ ec, T* __restrict__ ef,
                                                  const T* __restrict__ P0, const T* __restrict__ P1, int nc,
                                                  int64_t n_parents) {
  constexpr int TPC = K * K;
  constexpr int CPB = 256 / TPC;
  constexpr int RS = K + 1, PS = K * RS, CS = K * PS;
  constexpr int K3 = K * K * K;
  __shared__ T sa[CPB * CS];
  __shared__ T sb[2 * CPB * CS];
  const int tid = threadIdx.x;
  const int c = tid / TPC;
  const int p = tid - c * TPC;
  const int p0 = p % K, p1 = p / K;
  const int64_t par = (int64_t)blockIdx.x * CPB + c;
  const bool active = par < n_parents;
  int px = 0, py = 0, pz = 0;
  if (active) { px = (int)(par % nc); const int64_t t = par / nc; py = (int)(t % nc); pz = (int)(t / nc); }
  const int nf = 2 * nc;
  T* la = sa + c * CS;
  T* lb0 = sb + c * CS;
  T* lb1 = sb + (CPB + c) * CS;
  T v[K], u[K], w[K];
  // Every lane loads (a lane past the last parent reads parent 0, in bounds,
  // and discards it): a load behind a lane-dependent branch waits for its data
  // before the next one is issued.
  {
    const T* src = ec + (active ? par : 0) * K3 + p0 + K * p1;
#pragma unroll
    for (int iz = 0; iz < K; ++iz) {
      const T x = src[iz * K * K];
      v[iz] = active ? x : T(0);
    }
  }
  for (int bz = 0; bz < 2; ++bz) {
    pencil_mv<T, K>(bz ? P1 : P0, v, u);
#pragma unroll
    for (int iz = 0; iz < K; ++iz) la[iz * PS + p1 * RS + p0] = u[iz];
    __syncthreads();
    // y-pencil (ix = p0, iz = p1)
#pragma unroll
    for (int j = 0; j < K; ++j) u[j] = la[p1 * PS + j * RS + p0];
    pencil_mv<T, K>(P0, u, w);
#pragma unroll
    for (int iy = 0; iy < K; ++iy) lb0[p1 * PS + iy * RS + p0] = w[iy];
    pencil_mv<T, K>(P1, u, w);
#pragma unroll
    for (int iy = 0; iy < K; ++iy) lb1[p1 * PS + iy * RS + p0] = w[iy];
    __syncthreads();
    // x-pencil (iy = p0, iz = p1): four children (bx, by) of this bz
    for (int by = 0; by < 2; ++by) {
      const T* lb = by ? lb1 : lb0;
#pragma unroll
      for (int j = 0; j < K; ++j) u[j] = lb[p1 * PS + p0 * RS + j];
      for (int bx = 0; bx < 2; ++bx) {
        pencil_mv<T, K>(bx ? P1 : P0, u, w);
        // loaded in every lane (px = py = pz = 0 past the last parent: in
        // bounds), stored by the active ones only
        const int64_t child = (2 * px + bx) + (int64_t)nf * ((2 * py + by) + (int64_t)nf * (2 * pz + bz));
        T* dst = ef + child * K3 + K * p0 + K * K * p1;
        T old[K];
#pragma unroll
        for (int ix = 0; ix < K; ++ix) old[ix] = dst[ix];
        if (active) {
#pragma unroll
          for (int ix = 0; ix < K; ++ix) dst[ix] = old[ix] + w[ix];
        }
      }
    }
    __syncthreads();
  }
}

template <typename T, int K>
__global__ void __launch_bounds__(256) k_restrict3(const T* __restrict__ bf, const T* __restrict__ vf,
                                                   T* __restrict__ bc, const T* __restrict__ P0T,
                                                   const T* __restrict__ P1T, int nc, int64_t n_parents) {
  constexpr int TPC = K * K;
  constexpr int CPB = 256 / TPC;
  constexpr int RS = K + 1, PS = K * RS, CS = K * PS;
  constexpr int K3 = K * K * K;
  __shared__ T sx[2 * CPB * CS];
  __shared__ T su[2 * CPB * CS];
  const int tid = threadIdx.x;
  const int c = tid / TPC;
  const int p = tid - c * TPC;
  const int p0 = p % K, p1 = p / K;
  const int64_t par = (int64_t)blockIdx.x * CPB + c;
  const bool active = par < n_parents;
  int px = 0, py = 0, pz = 0;
  if (active) { px = (int)(par % nc); const int64_t t = par / nc; py = (int)(t % nc); pz = (int)(t / nc); }
  const int nf = 2 * nc;
  T r[K], s[K], acc[K], u[K];
  for (int bz = 0; bz < 2; ++bz) {
    // x-pencils (iy = p0, iz = p1) of the four children (bx, by) of this bz
    for (int by = 0; by < 2; ++by) {
#pragma unroll
      for (int i = 0; i < K; ++i) acc[i] = T(0);
      for (int bx = 0; bx < 2; ++bx) {
        // every lane loads (px = py = pz = 0 past the last parent: in bounds,
        // discarded), and the branch on vf is uniform and comes before any load
        const int64_t child = (2 * px + bx) + (int64_t)nf * ((2 * py + by) + (int64_t)nf * (2 * pz + bz));
        const int64_t off = child * K3 + K * p0 + K * K * p1;
        T bv[K], vv[K];
        if (vf) {
#pragma unroll
          for (int ix = 0; ix < K; ++ix) { bv[ix] = bf[off + ix]; vv[ix] = vf[off + ix]; }
#pragma unroll
          for (int ix = 0; ix < K; ++ix) r[ix] = active ? bv[ix] - vv[ix] : T(0);
        } else {
#pragma unroll
          for (int ix = 0; ix < K; ++ix) bv[ix] = bf[off + ix];
#pragma unroll
          for (int ix = 0; ix < K; ++ix) r[ix] = active ? bv[ix] : T(0);
        }
        pencil_mv<T, K>(bx ? P1T : P0T, r, s);
#pragma unroll
        for (int i = 0; i < K; ++i) acc[i] += s[i];
      }
      T* dst = sx + (by * CPB + c) * CS;
#pragma unroll
      for (int ix = 0; ix < K; ++ix) dst[p1 * PS + p0 * RS + ix] = acc[ix];
    }
    __syncthreads();
    // y-pencils (ix = p0, iz = p1)
    {
      const T* s0 = sx + c * CS;
      const T* s1 = sx + (CPB + c) * CS;
#pragma unroll
      for (int j = 0; j < K; ++j) r[j] = s0[p1 * PS + j * RS + p0];
      pencil_mv<T, K>(P0T, r, acc);
#pragma unroll
      for (int j = 0; j < K; ++j) r[j] = s1[p1 * PS + j * RS + p0];
      pencil_mv<T, K>(P1T, r, s);
      T* dst = su + (bz * CPB + c) * CS;
#pragma unroll
      for (int iy = 0; iy < K; ++iy) dst[p1 * PS + iy * RS + p0] = acc[iy] + s[iy];
    }
    __syncthreads();
  }
  // z-pencils (ix = p0, iy = p1)
  const T* u0 = su + c * CS;
  const T* u1 = su + (CPB + c) * CS;
#pragma unroll
  for (int j = 0; j < K; ++j) r[j] = u0[j * PS + p1 * RS + p0];
  pencil_mv<T, K>(P0T, r, acc);
#pragma unroll
  for (int j = 0; j < K; ++j) r[j] = u1[j * PS + p1 * RS + p0];
  pencil_mv<T, K>(P1T, r, u);
  if (active) {
    T* dst = bc + par * K3 + p0 + K * p1;
#pragma unroll
    for (int iz = 0; iz < K; ++iz) dst[iz * K * K] = acc[iz] + u[iz];
  }
}

// u += omega * dinv * (b - v); with u_is_zero: u = omega * dinv * b.
template <typename T>
__global__ void __launch_bounds__(256) k_jacobi_update(const T* __restrict__ b, const T* __restrict__ v,
                                                       T* __restrict__ u, const T* __restrict__ dinv, T omega,
                                                       int u_is_zero, int64_t len) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  if (u_is_zero) u[e] = omega * dinv[e] * b[e];
  else u[e] = fma(omega * dinv[e], b[e] - v[e], u[e]);
}

// Coarse solve on level 0: b_int = (G^T b) on interior nodes, e_int = A0^{-1} b_int
// (dense FP64 inverse), e = G e_int (zero on the boundary).  One block.
template <typename T, int K>
__global__ void __launch_bounds__(1024) k_coarse3(const T* __restrict__ b, T* __restrict__ e,
                                                  const double* __restrict__ Ainv, int n0, int ni) {
  extern __shared__ double sh[];
  double* bi = sh;
  double* ei = sh + ni;
  constexpr int k = K - 1;
  const int N = k * n0 + 1, Ni = N - 2;
  for (int j = threadIdx.x; j < ni; j += blockDim.x) {
    const int gx = 1 + j % Ni, gy = 1 + (j / Ni) % Ni, gz = 1 + j / (Ni * Ni);
    const AxisCopies ax = axis_copies<K>(gx, n0), ay = axis_copies<K>(gy, n0), az = axis_copies<K>(gz, n0);
    bi[j] = (double)cascade_sum<T, K, 3>(b, ax, ay, az, n0);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < ni; i += blockDim.x) {
    double s = 0.0;
    const double* row = Ainv + (int64_t)i * ni;
    for (int j = 0; j < ni; ++j) s = fma(row[j], bi[j], s);
    ei[i] = s;
  }
  __syncthreads();
  const int64_t len = (int64_t)n0 * n0 * n0 * K * K * K;
  for (int64_t q = threadIdx.x; q < len; q += blockDim.x) {
    const int64_t cell = q / (K * K * K);
    const int loc = (int)(q - cell * (K * K * K));
    const int ix = loc % K, iy = (loc / K) % K, iz = loc / (K * K);
    const int cx = (int)(cell % n0), cy = (int)((cell / n0) % n0), cz = (int)(cell / (n0 * n0));
    const int gx = k * cx + ix, gy = k * cy + iy, gz = k * cz + iz;
    T val = T(0);
    if (gx > 0 && gx < N - 1 && gy > 0 && gy < N - 1 && gz > 0 && gz < N - 1)
      val = (T)ei[(gx - 1) + Ni * ((gy - 1) + Ni * (gz - 1))];
    e[q] = val;
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_axpby(int64_t n, T a, const T* __restrict__ x, T b, T* __restrict__ y) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) y[e] = b == T(0) ? a * x[e] : fma(a, x[e], b * y[e]);
}

// CG update with the step length formed on the device: alpha = rho / <p, A p>
// read from device memory (no host round trip), x += alpha p, r -= alpha q.
// A non-positive or non-finite <p, A p> leaves x and r as they are (the host
// reports the breakdown after its next read).
__global__ void __launch_bounds__(256) k_cg_update(int64_t n, double rho, const double* __restrict__ pq,
                                                   const double* __restrict__ p, const double* __restrict__ q,
                                                   double* __restrict__ x, double* __restrict__ r) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const double d = *pq;
  if (e >= n || !(d > 0.0) || !(d < INFINITY)) return;
  const double alpha = rho / d;
  x[e] = fma(alpha, p[e], x[e]);
  r[e] = fma(-alpha, q[e], r[e]);
}

fe_status launch_cg_update(int64_t n, double rho, const double* pq, const double* p, const double* q, double* x,
                           double* r, hipStream_t s) {
  const unsigned nb = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_cg_update, dim3(nb), dim3(256), 0, s, n, rho, pq, p, q, x, r);
  FE_HIP_CHECK(hipGetLastError());
  return FE_OK;
}

// y = a x + b y with an FP32 x (converted exactly) and FP64 y
__global__ void __launch_bounds__(256) k_axpby_f32x(int64_t n, double a, const float* __restrict__ x, double b,
                                                    double* __restrict__ y) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) y[e] = b == 0.0 ? a * (double)x[e] : fma(a, (double)x[e], b * y[e]);
}

// Chebyshev step: w = a v + c w (v may alias w), then e = w or e += w.
template <typename T>
__global__ void __launch_bounds__(256) k_cheb_update(int64_t n, T a, const T* v, T c, T* w, T* __restrict__ e,
                                                     int e_zero) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const T wn = c == T(0) ? a * v[i] : fma(a, v[i], c * w[i]);
  w[i] = wn;
  e[i] = e_zero ? wn : e[i] + wn;
}

template <typename S, typename D>
__global__ void __launch_bounds__(256) k_cast(int64_t n, const S* __restrict__ x, D* __restrict__ y) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) y[e] = (D)x[e];
}

template <typename T>
__global__ void __launch_bounds__(256) k_fill(int64_t n, T* __restrict__ x, T v) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) x[e] = v;
}

template <typename T, typename TB = T>
__global__ void __launch_bounds__(256) k_dot_partial(int64_t n, const T* __restrict__ a, const TB* __restrict__ b,
                                                     double* __restrict__ part) {
  double acc = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    acc = fma((double)a[e], (double)b[e], acc);
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) k_finish(int nparts, const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) acc += part[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// Manufactured load vector on the Cartesian mesh: f = d pi^2 prod sin(pi x_a) is
// separable, so b_K,i = d pi^2 prod_a F(c_a, i_a) with
// F(c, i) = sum_q w_q h sin(pi h (c + xq_q)) phi_i(xq_q).
__global__ void __launch_bounds__(256) k_rhs_cart(double* __restrict__ b, const double* __restrict__ phi,
                                                  const double* __restrict__ xq, const double* __restrict__ wq,
                                                  int nq, int K, int dim, int n, double h, int64_t len) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  const int NL = dim == 3 ? K * K * K : K * K;
  const int64_t cell = e / NL;
  const int loc = (int)(e - cell * NL);
  int ci[3] = {(int)(cell % n), (int)((cell / n) % n), dim == 3 ? (int)(cell / ((int64_t)n * n)) : 0};
  int li[3] = {loc % K, (loc / K) % K, loc / (K * K)};
  double val = dim * M_PI * M_PI;
  for (int a = 0; a < dim; ++a) {
    double F = 0.0;
    for (int q = 0; q < nq; ++q) F += wq[q] * h * sin(M_PI * h * (ci[a] + xq[q])) * phi[q * K + li[a]];
    val *= F;
  }
  b[e] = val;
}

// Inverse diagonal with valence and Dirichlet mask baked in (Sec. 5,
// eq. valence_baking, with the constraints folded into the diagonal):
// dinv = kappa / d on interior copies, 0 on boundary copies.  d is the
// assembled diagonal already gathered to every copy.
template <typename T, int K, int DIM>
__global__ void __launch_bounds__(256) k_make_dinv(const double* __restrict__ d, T* __restrict__ dinv, int n, int bc,
                                                   int64_t len) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  constexpr int k = K - 1;
  constexpr int NL = DIM == 3 ? K * K * K : K * K;
  const int64_t cell = e / NL;
  const int loc = (int)(e - cell * NL);
  const int li[3] = {loc % K, (loc / K) % K, loc / (K * K)};
  const int ci[3] = {(int)(cell % n), (int)((cell / n) % n), DIM == 3 ? (int)(cell / ((int64_t)n * n)) : 0};
  int kappa = 1;
  bool bnd = false;
  for (int a = 0; a < DIM; ++a) {
    const int g = k * ci[a] + li[a];
    if (g == 0 || g == k * n) bnd = true;
    else if (li[a] == 0 || li[a] == k) kappa *= 2;
  }
  dinv[e] = (bc && bnd) ? T(0) : (T)(kappa / d[e]);
}

template <int K>
static fe_status make_dinv_typed(const fe_problem* p, int level, const double* d, void* dinv, fe_dtype dt,
                                 hipStream_t s) {
  const Level& L = level_of(p, level);
  const unsigned nb = (unsigned)((L.len + 255) / 256);
  if (dt == FE_F64) {
    if (p->dim == 3) hipLaunchKernelGGL((k_make_dinv<double, K, 3>), dim3(nb), dim3(256), 0, s, d, (double*)dinv, L.n, p->bc, L.len);
    else hipLaunchKernelGGL((k_make_dinv<double, K, 2>), dim3(nb), dim3(256), 0, s, d, (double*)dinv, L.n, p->bc, L.len);
  } else {
    if (p->dim == 3) hipLaunchKernelGGL((k_make_dinv<float, K, 3>), dim3(nb), dim3(256), 0, s, d, (float*)dinv, L.n, p->bc, L.len);
    else hipLaunchKernelGGL((k_make_dinv<float, K, 2>), dim3(nb), dim3(256), 0, s, d, (float*)dinv, L.n, p->bc, L.len);
  }
  FE_HIP_CHECK(hipGetLastError());
  return FE_OK;
}

fe_status launch_make_dinv(const fe_problem* p, int level, const double* d, void* dinv, fe_dtype dt, hipStream_t s) {
  FE_DISPATCH_K(p->K, return make_dinv_typed<KK>(p, level, d, dinv, dt, s));
}

// Dual Dirichlet mask: zero every copy of a boundary node (restriction of a
// dual vector to the test space of the homogeneous Dirichlet problem).
template <typename T, int K>
__global__ void __launch_bounds__(256) k_mask_boundary(T* __restrict__ v, int n, int dim, int64_t len) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  constexpr int k = K - 1;
  const int NL = dim == 3 ? K * K * K : K * K;
  const int64_t cell = e / NL;
  const int loc = (int)(e - cell * NL);
  const int li[3] = {loc % K, (loc / K) % K, loc / (K * K)};
  const int ci[3] = {(int)(cell % n), (int)((cell / n) % n), dim == 3 ? (int)(cell / ((int64_t)n * n)) : 0};
  bool bnd = false;
  for (int a = 0; a < dim; ++a) bnd = bnd || on_boundary(ci[a], li[a], n, k);
  if (bnd) v[e] = T(0);
}

template <int K>
static fe_status mask_typed(const fe_problem* p, int level, void* v, fe_dtype dt, hipStream_t s) {
  const Level& L = level_of(p, level);
  const unsigned nb = (unsigned)((L.len + 255) / 256);
  if (dt == FE_F64) hipLaunchKernelGGL((k_mask_boundary<double, K>), dim3(nb), dim3(256), 0, s, (double*)v, L.n, p->dim, L.len);
  else hipLaunchKernelGGL((k_mask_boundary<float, K>), dim3(nb), dim3(256), 0, s, (float*)v, L.n, p->dim, L.len);
  FE_HIP_CHECK(hipGetLastError());
  return FE_OK;
}

fe_status launch_mask_boundary(const fe_problem* p, int level, void* v, fe_dtype dt, hipStream_t s) {
  FE_DISPATCH_K(p->K, return mask_typed<KK>(p, level, v, dt, s));
}

// ------------------------------------------------------------------ host side

template <typename T, int K>
static fe_status prolong_typed(const fe_problem* p, int fl, const T* ec, T* ef, const T* coef, hipStream_t s) {
  const Level& C = p->levels[fl - 1];
  constexpr int CPB = 256 / (K * K);
  const unsigned nb = (unsigned)((C.n_cells + CPB - 1) / CPB);
  ProfScope ps("prolongate", s);
  hipLaunchKernelGGL((k_prolong3<T, K>), dim3(nb), dim3(CPB * K * K), 0, s, ec, ef, coef + p->co.off_P0,
                     coef + p->co.off_P1, C.n, C.n_cells);
  FE_HIP_CHECK(hipGetLastError());
  return FE_OK;
}

template <typename T, int K>
static fe_status restrict_typed(const fe_problem* p, int fl, const T* bf, const T* vf, T* bc, const T* coef,
                                hipStream_t s) {
  const Level& C = p->levels[fl - 1];
  constexpr int CPB = 256 / (K * K);
  const unsigned nb = (unsigned)((C.n_cells + CPB - 1) / CPB);
  ProfScope ps("restrict", s);
  hipLaunchKernelGGL((k_restrict3<T, K>), dim3(nb), dim3(CPB * K * K), 0, s, bf, vf, bc, coef + p->co.off_P0T,
                     coef + p->co.off_P1T, C.n, C.n_cells);
  FE_HIP_CHECK(hipGetLastError());
  return FE_OK;
}

fe_status launch_prolongate_add(const fe_problem* p, int fl, const void* ec, void* ef, fe_dtype dt, hipStream_t s) {
  if (p->dim != 3) return fail(FE_EUNSUPPORTED, "transfers are implemented for d = 3");
  if (dt == FE_F64) {
    FE_DISPATCH_K(p->K, return (prolong_typed<double, KK>(p, fl, (const double*)ec, (double*)ef,
                                                          p->coef64.as<double>(), s)));
  }
  FE_DISPATCH_K(p->K, return (prolong_typed<float, KK>(p, fl, (const float*)ec, (float*)ef,
                                                       p->coef32.as<float>(), s)));
}

fe_status launch_restrict(const fe_problem* p, int fl, const void* bf, const void* vf, void* bc, fe_dtype dt,
                          hipStream_t s) {
  if (p->dim != 3) return fail(FE_EUNSUPPORTED, "transfers are implemented for d = 3");
  if (dt == FE_F64) {
    FE_DISPATCH_K(p->K, return (restrict_typed<double, KK>(p, fl, (const double*)bf, (const double*)vf,
                                                           (double*)bc, p->coef64.as<double>(), s)));
  }
  FE_DISPATCH_K(p->K, return (restrict_typed<float, KK>(p, fl, (const float*)bf, (const float*)vf, (float*)bc,
                                                        p->coef32.as<float>(), s)));
}

fe_status launch_jacobi_update(const fe_problem* p, int level, const void* b, const void* v, void* u,
                               const void* dinv, double omega, int u_is_zero, fe_dtype dt, hipStream_t s) {
  const Level& L = level_of(p, level);
  const unsigned nb = (unsigned)((L.len + 255) / 256);
  ProfScope ps("jacobi_update", s);
  if (dt == FE_F64)
    hipLaunchKernelGGL(k_jacobi_update<double>, dim3(nb), dim3(256), 0, s, (const double*)b, (const double*)v,
                       (double*)u, (const double*)dinv, omega, u_is_zero, L.len);
  else
    hipLaunchKernelGGL(k_jacobi_update<float>, dim3(nb), dim3(256), 0, s, (const float*)b, (const float*)v,
                       (float*)u, (const float*)dinv, (float)omega, u_is_zero, L.len);
  FE_HIP_CHECK(hipGetLastError());
  return FE_OK;
}

template <typename T, int K>
static fe_status coarse_typed(const fe_problem* p, const T* b, T* e, hipStream_t s) {
  const Level& L0 = p->levels[0];
  const size_t sh = 2 * (size_t)p->coarse_n * sizeof(double);
  ProfScope ps("coarse", s);
  hipLaunchKernelGGL((k_coarse3<T, K>), dim3(1), dim3(1024), sh, s, b, e, p->coarse_inv.as<double>(), L0.n,
                     p->coarse_n);
  FE_HIP_CHECK(hipGetLastError());
  return FE_OK;
}

fe_status launch_coarse_solve(const fe_problem* p, const void* b0, void* e0, fe_dtype dt, hipStream_t s) {
  if (dt == FE_F64) { FE_DISPATCH_K(p->K, return (coarse_typed<double, KK>(p, (const double*)b0, (double*)e0, s))); }
  FE_DISPATCH_K(p->K, return (coarse_typed<float, KK>(p, (const float*)b0, (float*)e0, s)));
}

fe_status launch_axpby(int64_t n, double a, const void* x, double b, void* y, fe_dtype dt, hipStream_t s) {
  const unsigned nb = (unsigned)((n + 255) / 256);
  if (dt == FE_F64)
    hipLaunchKernelGGL(k_axpby<double>, dim3(nb), dim3(256), 0, s, n, a, (const double*)x, b, (double*)y);
  else
    hipLaunchKernelGGL(k_axpby<float>, dim3(nb), dim3(256), 0, s, n, (float)a, (const float*)x, (float)b, (float*)y);
  FE_HIP_CHECK(hipGetLastError());
  return FE_OK;
}

fe_status launch_axpby_x(int64_t n, double a, const void* x, fe_dtype xdt, double b, double* y, hipStream_t s) {
  if (xdt == FE_F64) return launch_axpby(n, a, x, b, y, FE_F64, s);
  const unsigned nb = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_axpby_f32x, dim3(nb), dim3(256), 0, s, n, a, (const float*)x, b, y);
  FE_HIP_CHECK(hipGetLastError());
  return FE_OK;
}

fe_status launch_cheb_update(int64_t n, double a, const void* v, double c, void* w, void* e, int e_zero,
                             fe_dtype dt, hipStream_t s) {
  const unsigned nb = (unsigned)((n + 255) / 256);
  if (dt == FE_F64)
    hipLaunchKernelGGL(k_cheb_update<double>, dim3(nb), dim3(256), 0, s, n, a, (const double*)v, c, (double*)w,
                       (double*)e, e_zero);
  else
    hipLaunchKernelGGL(k_cheb_update<float>, dim3(nb), dim3(256), 0, s, n, (float)a, (const float*)v, (float)c,
                       (float*)w, (float*)e, e_zero);
  FE_HIP_CHECK(hipGetLastError());
  return FE_OK;
}

fe_status launch_cast(int64_t n, const void* src, fe_dtype st, void* dst, fe_dtype dtt, hipStream_t s) {
  const unsigned nb = (unsigned)((n + 255) / 256);
  ProfScope ps("cast", s);
  if (st == FE_F64 && dtt == FE_F32)
    hipLaunchKernelGGL((k_cast<double, float>), dim3(nb), dim3(256), 0, s, n, (const double*)src, (float*)dst);
  else if (st == FE_F32 && dtt == FE_F64)
    hipLaunchKernelGGL((k_cast<float, double>), dim3(nb), dim3(256), 0, s, n, (const float*)src, (double*)dst);
  else if (st == FE_F64)
    hipLaunchKernelGGL((k_cast<double, double>), dim3(nb), dim3(256), 0, s, n, (const double*)src, (double*)dst);
  else
    hipLaunchKernelGGL((k_cast<float, float>), dim3(nb), dim3(256), 0, s, n, (const float*)src, (float*)dst);
  FE_HIP_CHECK(hipGetLastError());
  return FE_OK;
}

fe_status launch_fill(int64_t n, void* x, double v, fe_dtype dt, hipStream_t s) {
  const unsigned nb = (unsigned)((n + 255) / 256);
  if (dt == FE_F64) hipLaunchKernelGGL(k_fill<double>, dim3(nb), dim3(256), 0, s, n, (double*)x, v);
  else hipLaunchKernelGGL(k_fill<float>, dim3(nb), dim3(256), 0, s, n, (float*)x, (float)v);
  FE_HIP_CHECK(hipGetLastError());
  return FE_OK;
}

fe_status finish_reduction(const fe_problem* p, int nparts, double* dev_out, hipStream_t s) {
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, s, nparts, p->red_scratch.as<double>(), dev_out);
  FE_HIP_CHECK(hipGetLastError());
  return FE_OK;
}

fe_status dot_async(const fe_problem* p, int64_t n, const void* a, const void* b, fe_dtype dt, double* dev_out,
                    hipStream_t s) {
  const int nparts = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (n + 255) / 256));
  ProfScope ps("dot", s);
  if (dt == FE_F64)
    hipLaunchKernelGGL(k_dot_partial<double>, dim3(nparts), dim3(256), 0, s, n, (const double*)a, (const double*)b,
                       p->red_scratch.as<double>());
  else
    hipLaunchKernelGGL(k_dot_partial<float>, dim3(nparts), dim3(256), 0, s, n, (const float*)a, (const float*)b,
                       p->red_scratch.as<double>());
  FE_HIP_CHECK(hipGetLastError());
  return finish_reduction(p, nparts, dev_out, s);
}

fe_status dot_async_x(const fe_problem* p, int64_t n, const double* a, const void* b, fe_dtype bdt, double* dev_out,
                      hipStream_t s) {
  if (bdt == FE_F64) return dot_async(p, n, a, b, FE_F64, dev_out, s);
  const int nparts = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (n + 255) / 256));
  ProfScope ps("dot", s);
  hipLaunchKernelGGL((k_dot_partial<double, float>), dim3(nparts), dim3(256), 0, s, n, a, (const float*)b,
                     p->red_scratch.as<double>());
  FE_HIP_CHECK(hipGetLastError());
  return finish_reduction(p, nparts, dev_out, s);
}

fe_status launch_rhs_cartesian(const fe_problem* p, void* b, hipStream_t s) {
  const Level& L = level_of(p, -1);
  const int K = p->K, nq = p->k + 2;
  std::vector<double> xq, wq;
  gauss_rule(nq, xq, wq);
  std::vector<double> nodes = gll_nodes(p->k), phi(nq * K);
  for (int q = 0; q < nq; ++q)
    for (int i = 0; i < K; ++i) phi[q * K + i] = lagrange_value(nodes, i, xq[q]);
  std::vector<double> host(phi);
  host.insert(host.end(), xq.begin(), xq.end());
  host.insert(host.end(), wq.begin(), wq.end());
  DeviceBuf tmp;
  FE_CHECK(tmp.alloc(host.size() * sizeof(double)));
  FE_HIP_CHECK(hipMemcpyAsync(tmp.p, host.data(), host.size() * sizeof(double), hipMemcpyHostToDevice, s));
  const double* d = tmp.as<double>();
  hipLaunchKernelGGL(k_rhs_cart, dim3((unsigned)((L.len + 255) / 256)), dim3(256), 0, s, (double*)b, d,
                     d + nq * K, d + nq * K + nq, nq, K, p->dim, L.n, L.h, L.len);
  FE_HIP_CHECK(hipGetLastError());
  FE_HIP_CHECK(hipStreamSynchronize(s));
  return FE_OK;
}

}  // namespace fe
