// Cell-wise Cartesian Laplace operator by sum factorization (paper, Sec. 6:
// the cube operator (D x B x B + B x D x B + B x B x D) det(J) J^-2 with one
// reference pair for all levels; Sec. 2.1: A maps a continuous primal vector
// to an unassembled dual vector, cell by cell).
//
// Work decomposition for a wave64 machine: a cell of K^3 values is handled by
// K^2 threads, each owning one pencil of K values in registers.  The first
// contraction runs along the pencil in registers; the pencils are then
// re-oriented through LDS twice (y, then x).  Loads and stores use the
// z-pencil orientation, in which the K^2 threads of a cell touch K^2
// consecutive values per instruction (coalesced).  LDS rows are padded to
// K+1 to break bank conflicts of the x-pencil reads.
#include "fe_internal.h"
#include "kernel_common.h"

namespace fe {

template <typename T, int K>
__global__ void __launch_bounds__(256) k_apply_cart3(const T* __restrict__ x, T* y,
                                                     const T* __restrict__ Bm, const T* __restrict__ Dm,
                                                     T scale, int n, int64_t n_cells, int dirichlet, T alpha,
                                                     T beta, const T* bsrc) {
  constexpr int TPC = K * K;
  constexpr int CPB = 256 / TPC;
  constexpr int RS = K + 1;
  constexpr int PS = K * RS;
  constexpr int CS = K * PS;
  constexpr int k = K - 1;
  __shared__ T sa[CPB * CS];
  __shared__ T sb[CPB * CS];

  const int tid = threadIdx.x;
  const int c = tid / TPC;
  const int p = tid - c * TPC;
  const int p0 = p % K, p1 = p / K;
  const int64_t cell = (int64_t)blockIdx.x * CPB + c;
  const bool active = cell < n_cells;
  int cx = 0, cy = 0, cz = 0;
  if (active) cell_coords3<TPC % 64 == 0>(cell, n, cx, cy, cz);   // K = 8: one cell per wavefront
  T* la = sa + c * CS;
  T* lb = sb + c * CS;

  // Dirichlet mask of z-pencil (ix = p0, iy = p1): bit iz set if masked
  uint32_t zmask = 0;
  if (dirichlet && active) {
    const bool mxy = on_boundary(cx, p0, n, k) || on_boundary(cy, p1, n, k);
#pragma unroll
    for (int iz = 0; iz < K; ++iz)
      if (mxy || on_boundary(cz, iz, n, k)) zmask |= 1u << iz;
  }

  T v[K], w[K], a[K], b[K];
  // phase A: z-pencils, contraction along z
  if (active) {
    const T* xc = x + cell * (K * K * K) + p0 + K * p1;
#pragma unroll
    for (int iz = 0; iz < K; ++iz) v[iz] = xc[iz * K * K];
#pragma unroll
    for (int iz = 0; iz < K; ++iz)
      if (zmask & (1u << iz)) v[iz] = T(0);
  } else {
#pragma unroll
    for (int iz = 0; iz < K; ++iz) v[iz] = T(0);
  }
  pencil_mv<T, K>(Bm, v, a);
  pencil_mv<T, K>(Dm, v, b);
#pragma unroll
  for (int iz = 0; iz < K; ++iz) {
    la[iz * PS + p1 * RS + p0] = a[iz];
    lb[iz * PS + p1 * RS + p0] = b[iz];
  }
  __syncthreads();

  // phase B: y-pencils (ix = p0, iz = p1)
#pragma unroll
  for (int j = 0; j < K; ++j) {
    v[j] = la[p1 * PS + j * RS + p0];
    w[j] = lb[p1 * PS + j * RS + p0];
  }
  pencil_mv<T, K>(Bm, v, a);            // c = B_y B_z x
  pencil_mv2<T, K>(Dm, v, Bm, w, b);    // g = D_y B_z x + B_y D_z x
  __syncthreads();
#pragma unroll
  for (int iy = 0; iy < K; ++iy) {
    la[p1 * PS + iy * RS + p0] = a[iy];
    lb[p1 * PS + iy * RS + p0] = b[iy];
  }
  __syncthreads();

  // phase C: x-pencils (iy = p0, iz = p1)
#pragma unroll
  for (int j = 0; j < K; ++j) {
    v[j] = la[p1 * PS + p0 * RS + j];
    w[j] = lb[p1 * PS + p0 * RS + j];
  }
  pencil_mv2<T, K>(Dm, v, Bm, w, a);    // D_x c + B_x g
  __syncthreads();
#pragma unroll
  for (int ix = 0; ix < K; ++ix) la[p1 * PS + p0 * RS + ix] = a[ix] * scale;
  __syncthreads();

  // store through the z-pencil orientation (ix = p0, iy = p1), with the
  // epilogue y = alpha A x + beta bsrc (read before y is written: bsrc may alias y)
  if (active) {
    const int64_t off = cell * (K * K * K) + p0 + K * p1;
    T* yc = y + off;
#pragma unroll
    for (int iz = 0; iz < K; ++iz) {
      T val = la[iz * PS + p1 * RS + p0];
      if (zmask & (1u << iz)) val = T(0);
      val *= alpha;
      if (bsrc) val += beta * bsrc[off + iz * K * K];
      yc[iz * K * K] = val;
    }
  }
}

template <typename T, int K>
__global__ void __launch_bounds__(256) k_apply_cart2(const T* __restrict__ x, T* y,
                                                     const T* __restrict__ Bm, const T* __restrict__ Dm,
                                                     T scale, int n, int64_t n_cells, int dirichlet, T alpha,
                                                     T beta, const T* bsrc) {
  constexpr int TPC = K;
  constexpr int CPB = 256 / TPC;
  constexpr int RS = K + 1;
  constexpr int CS = K * RS;
  constexpr int k = K - 1;
  __shared__ T sa[CPB * CS];
  __shared__ T sb[CPB * CS];
  const int tid = threadIdx.x;
  const int c = tid / TPC;
  const int p = tid - c * TPC;
  const int64_t cell = (int64_t)blockIdx.x * CPB + c;
  const bool active = cell < n_cells;
  int cx = 0, cy = 0;
  if (active) { cx = (int)(cell % n); cy = (int)(cell / n); }
  T* la = sa + c * CS;
  T* lb = sb + c * CS;
  uint32_t ymask = 0;  // y-pencil at ix = p
  if (dirichlet && active) {
    const bool mx = on_boundary(cx, p, n, k);
#pragma unroll
    for (int iy = 0; iy < K; ++iy)
      if (mx || on_boundary(cy, iy, n, k)) ymask |= 1u << iy;
  }
  T v[K], w[K], a[K], b[K];
  if (active) {
    const T* xc = x + cell * (K * K) + p;
#pragma unroll
    for (int iy = 0; iy < K; ++iy) v[iy] = (ymask & (1u << iy)) ? T(0) : xc[iy * K];
  } else {
#pragma unroll
    for (int iy = 0; iy < K; ++iy) v[iy] = T(0);
  }
  pencil_mv<T, K>(Bm, v, a);
  pencil_mv<T, K>(Dm, v, b);
#pragma unroll
  for (int iy = 0; iy < K; ++iy) {
    la[iy * RS + p] = a[iy];
    lb[iy * RS + p] = b[iy];
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < K; ++j) {
    v[j] = la[p * RS + j];
    w[j] = lb[p * RS + j];
  }
  pencil_mv2<T, K>(Dm, v, Bm, w, a);   // D_x B_y x + B_x D_y x
  __syncthreads();
#pragma unroll
  for (int ix = 0; ix < K; ++ix) la[p * RS + ix] = a[ix] * scale;
  __syncthreads();
  if (active) {
    const int64_t off = cell * (K * K) + p;
    T* yc = y + off;
#pragma unroll
    for (int iy = 0; iy < K; ++iy) {
      T val = (ymask & (1u << iy)) ? T(0) : la[iy * RS + p];
      val *= alpha;
      if (bsrc) val += beta * bsrc[off + iy * K];
      yc[iy * K] = val;
    }
  }
}

// Local diagonal of the Cartesian element matrix, cell by cell:
// scale * (D_ii B_jj B_ll + B_ii D_jj B_ll + B_ii B_jj D_ll).
template <typename T, int K>
__global__ void k_diag_cart(T* __restrict__ d, const T* __restrict__ Bm, const T* __restrict__ Dm, T scale,
                            int dim, int64_t len) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  const int loc = dim == 3 ? (int)(e % (K * K * K)) : (int)(e % (K * K));
  const int ix = loc % K, iy = (loc / K) % K, iz = loc / (K * K);
  const T bx = Bm[ix * K + ix], by = Bm[iy * K + iy], dx = Dm[ix * K + ix], dy = Dm[iy * K + iy];
  T val;
  if (dim == 3) {
    const T bz = Bm[iz * K + iz], dz = Dm[iz * K + iz];
    val = dx * by * bz + bx * dy * bz + bx * by * dz;
  } else {
    val = dx * by + bx * dy;
  }
  d[e] = scale * val;
}

template <typename T, int K>
static fe_status apply_typed(const fe_problem* p, const Level& L, const T* x, T* y, const T* coef, T alpha,
                             T beta, const T* b, hipStream_t s) {
  const T* Bm = coef + p->co.off_B;
  const T* Dm = coef + p->co.off_D;
  const T scale = (T)(p->dim == 3 ? L.h : 1.0);
  if (p->dim == 3) {
    constexpr int CPB = 256 / (K * K);
    const int64_t nb = (L.n_cells + CPB - 1) / CPB;
    ProfScope ps("apply", s);
    hipLaunchKernelGGL((k_apply_cart3<T, K>), dim3((unsigned)nb), dim3(CPB * K * K), 0, s, x, y, Bm, Dm,
                       scale, L.n, L.n_cells, p->bc, alpha, beta, b);
  } else {
    constexpr int CPB = 256 / K;
    const int64_t nb = (L.n_cells + CPB - 1) / CPB;
    ProfScope ps("apply", s);
    hipLaunchKernelGGL((k_apply_cart2<T, K>), dim3((unsigned)nb), dim3(CPB * K), 0, s, x, y, Bm, Dm,
                       scale, L.n, L.n_cells, p->bc, alpha, beta, b);
  }
  FE_HIP_CHECK(hipGetLastError());
  return FE_OK;
}

template <typename T, int K>
static fe_status diag_typed(const fe_problem* p, const Level& L, T* d, const T* coef, hipStream_t s) {
  const T scale = (T)(p->dim == 3 ? L.h : 1.0);
  const int64_t nb = (L.len + 255) / 256;
  hipLaunchKernelGGL((k_diag_cart<T, K>), dim3((unsigned)nb), dim3(256), 0, s, d, coef + p->co.off_B,
                     coef + p->co.off_D, scale, p->dim, L.len);
  FE_HIP_CHECK(hipGetLastError());
  return FE_OK;
}

fe_status launch_apply(const fe_problem* p, int level, const void* x, void* y, fe_dtype dt, hipStream_t s) {
  return launch_apply_ep(p, level, x, y, 1.0, 0.0, nullptr, dt, s);
}

fe_status launch_apply_ep(const fe_problem* p, int level, const void* x, void* y, double alpha, double beta,
                          const void* b, fe_dtype dt, hipStream_t s) {
  if (p->desc.geometry == FE_GEOM_DEFORMED) return launch_apply_general(p, level, x, y, alpha, beta, b, dt, s);
  const Level& L = level_of(p, level);
  if (dt == FE_F64) {
    FE_DISPATCH_K(p->K, return (apply_typed<double, KK>(p, L, (const double*)x, (double*)y,
                                                        p->coef64.as<double>(), alpha, beta, (const double*)b,
                                                        s)));
  } else {
    FE_DISPATCH_K(p->K, return (apply_typed<float, KK>(p, L, (const float*)x, (float*)y,
                                                       p->coef32.as<float>(), (float)alpha, (float)beta,
                                                       (const float*)b, s)));
  }
}

fe_status launch_diag_cartesian(const fe_problem* p, int level, void* d, fe_dtype dt, hipStream_t s) {
  const Level& L = level_of(p, level);
  if (dt == FE_F64) {
    FE_DISPATCH_K(p->K, return (diag_typed<double, KK>(p, L, (double*)d, p->coef64.as<double>(), s)));
  } else {
    FE_DISPATCH_K(p->K, return (diag_typed<float, KK>(p, L, (float*)d, p->coef32.as<float>(), s)));
  }
}

// The cube operator on a plain list of n_cells cells of side h (3D, FP64, no
// boundary treatment: inputs are zero on Dirichlet copies by construction):
// the cells of one level of a locally refined hierarchy.
template <int K>
static fe_status apply_cells_typed(const fe_problem* p, int64_t n_cells, double h, const double* x, double* y,
                                   double alpha, double beta, const double* b, hipStream_t s) {
  if (n_cells == 0) return FE_OK;
  const double* coef = p->coef64.as<double>();
  constexpr int CPB = 256 / (K * K);
  const int64_t nb = (n_cells + CPB - 1) / CPB;
  ProfScope ps("apply", s);
  hipLaunchKernelGGL((k_apply_cart3<double, K>), dim3((unsigned)nb), dim3(CPB * K * K), 0, s, x, y,
                     coef + p->co.off_B, coef + p->co.off_D, h, 1, n_cells, 0, alpha, beta, b);
  FE_HIP_CHECK(hipGetLastError());
  return FE_OK;
}

fe_status launch_apply_cells(const fe_problem* p, int64_t n_cells, double h, const double* x, double* y, double alpha,
                             double beta, const double* b, hipStream_t s) {
  if (p->dim != 3) return fail(FE_EINVAL, "cell-list apply is 3D");
  FE_DISPATCH_K(p->K, return (apply_cells_typed<KK>(p, n_cells, h, x, y, alpha, beta, b, s)));
}

// Diagonal of the cube operator on every copy of n_cells cells of side h (3D, FP64).
fe_status launch_diag_cells(const fe_problem* p, int64_t n_cells, double h, double* d, hipStream_t s) {
  const int64_t len = n_cells * p->K * p->K * p->K;
  if (len == 0) return FE_OK;
  const double* coef = p->coef64.as<double>();
  const int64_t nb = (len + 255) / 256;
  FE_DISPATCH_K(p->K, {
    hipLaunchKernelGGL((k_diag_cart<double, KK>), dim3((unsigned)nb), dim3(256), 0, s, d, coef + p->co.off_B,
                       coef + p->co.off_D, h, 3, len);
    FE_HIP_CHECK(hipGetLastError());
    return FE_OK;
  });
}

}  // namespace fe
