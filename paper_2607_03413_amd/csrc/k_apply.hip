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

// FP64: the output is written once, each store instruction covering whole
// 128-byte lines (a cell's z-plane), and is not read again by the kernel, so
// its stores are non-temporal (no L2 allocation), and so are the input loads.
// Measured (four rotating vector pairs): Q3 48^3 / 64^3 / 96^3 23.8 / 48.9 /
// 151.9 -> 21.5 / 45.5 / 145.0 us, Q7 32^3 65.7 -> 63.5 us.  In FP32 a cell's
// z-plane at K = 4 is half a line: non-temporal stores wrote 1.12x the bytes
// and, between patch inverses, gained nothing.
template <typename T>
__device__ __forceinline__ T load_in(const T* p) {
  if constexpr (sizeof(T) == 8) return __builtin_nontemporal_load(p);
  else return *p;
}
template <typename T>
__device__ __forceinline__ void store_out(T v, T* p) {
  if constexpr (sizeof(T) == 8) __builtin_nontemporal_store(v, p);
  else *p = v;
}

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
  if (TPC % 64 == 0) {   // K = 8: one cell per wavefront, divisions on the scalar unit
    if (active) cell_coords3<true>(cell, n, cx, cy, cz);
  } else if (n >= CPB) {
    // the block's first cell on the scalar unit, then at most one row wrap per cell
    int bx, by, bz;
    cell_coords3<true>((int64_t)blockIdx.x * CPB, n, bx, by, bz);
    cx = bx + c;
    cy = by;
    cz = bz;
    if (cx >= n) {
      cx -= n;
      if (++cy >= n) {
        cy = 0;
        ++cz;
      }
    }
  } else if (active) {
    cell_coords3<false>(cell, n, cx, cy, cz);
  }
  T* la = sa + c * CS;
  T* lb = sb + c * CS;

  // Dirichlet mask of z-pencil (ix = p0, iy = p1): bit iz set if masked (only
  // cells on the boundary of the cube have any)
  uint32_t zmask = 0;
  if (dirichlet && active && (cx == 0 || cy == 0 || cz == 0 || cx == n - 1 || cy == n - 1 || cz == n - 1)) {
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
    for (int iz = 0; iz < K; ++iz) v[iz] = load_in(xc + iz * K * K);
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
      store_out(val, yc + iz * K * K);
    }
  }
}

// The same operator with CPT cells per thread (cells c, c + CPB, ...): the same
// per-cell work with CPT times the bytes in flight per wavefront, which the
// FP32 Q3 apply needs to reach the memory rate (its cells are half the bytes
// of FP64 ones for the same wavefront count).  A separate kernel: compiled with
// one cell per thread it needs more scalar registers than the kernel above
// (K = 6..9 FP64 spilled them to vector lanes).
template <typename T, int K, int CPT>
__global__ void __launch_bounds__(256) k_apply_cart3_multi(const T* __restrict__ x, T* y,
                                                     const T* __restrict__ Bm, const T* __restrict__ Dm,
                                                     T scale, int n, int64_t n_cells, int dirichlet, T alpha,
                                                     T beta, const T* bsrc) {
  constexpr int TPC = K * K;
  constexpr int CPB = 256 / TPC;   // cells per block and pass
  constexpr int RS = K + 1;
  constexpr int PS = K * RS;
  constexpr int CS = K * PS;
  constexpr int k = K - 1;
  __shared__ T sa[CPT * CPB * CS];
  __shared__ T sb[CPT * CPB * CS];

  const int tid = threadIdx.x;
  const int c = tid / TPC;
  const int p = tid - c * TPC;
  const int p0 = p % K, p1 = p / K;
  int64_t cell[CPT];
  bool active[CPT];
  uint32_t zmask[CPT];
  T* la[CPT];
  T* lb[CPT];
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    const int64_t first = ((int64_t)blockIdx.x * CPT + j) * CPB;   // the pass's first cell
    cell[j] = first + c;
    active[j] = cell[j] < n_cells;
    int cx = 0, cy = 0, cz = 0;
    if (TPC % 64 == 0) {   // K = 8: one cell per wavefront, divisions on the scalar unit
      if (active[j]) cell_coords3<true>(cell[j], n, cx, cy, cz);
    } else if (n >= CPB) {
      // the pass's first cell on the scalar unit, then at most one row wrap per cell
      int bx, by, bz;
      cell_coords3<true>(first, n, bx, by, bz);
      cx = bx + c;
      cy = by;
      cz = bz;
      if (cx >= n) {
        cx -= n;
        if (++cy >= n) {
          cy = 0;
          ++cz;
        }
      }
    } else if (active[j]) {
      cell_coords3<false>(cell[j], n, cx, cy, cz);
    }
    la[j] = sa + (j * CPB + c) * CS;
    lb[j] = sb + (j * CPB + c) * CS;
    // Dirichlet mask of z-pencil (ix = p0, iy = p1): bit iz set if masked (only
    // cells on the boundary of the cube have any)
    zmask[j] = 0;
    if (dirichlet && active[j] && (cx == 0 || cy == 0 || cz == 0 || cx == n - 1 || cy == n - 1 || cz == n - 1)) {
      const bool mxy = on_boundary(cx, p0, n, k) || on_boundary(cy, p1, n, k);
#pragma unroll
      for (int iz = 0; iz < K; ++iz)
        if (mxy || on_boundary(cz, iz, n, k)) zmask[j] |= 1u << iz;
    }
  }

  T v[CPT][K];
  // phase A: z-pencils, contraction along z (every cell's loads issued first)
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    if (active[j]) {
      const T* xc = x + cell[j] * (K * K * K) + p0 + K * p1;
#pragma unroll
      for (int iz = 0; iz < K; ++iz) v[j][iz] = load_in(xc + iz * K * K);
    } else {
#pragma unroll
      for (int iz = 0; iz < K; ++iz) v[j][iz] = T(0);
    }
  }
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    T a[K], b[K];
#pragma unroll
    for (int iz = 0; iz < K; ++iz)
      if (zmask[j] & (1u << iz)) v[j][iz] = T(0);
    pencil_mv<T, K>(Bm, v[j], a);
    pencil_mv<T, K>(Dm, v[j], b);
#pragma unroll
    for (int iz = 0; iz < K; ++iz) {
      la[j][iz * PS + p1 * RS + p0] = a[iz];
      lb[j][iz * PS + p1 * RS + p0] = b[iz];
    }
  }
  __syncthreads();

  // phase B: y-pencils (ix = p0, iz = p1)
  T ra[CPT][K], rb[CPT][K];
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    T w[K];
#pragma unroll
    for (int q = 0; q < K; ++q) {
      v[j][q] = la[j][p1 * PS + q * RS + p0];
      w[q] = lb[j][p1 * PS + q * RS + p0];
    }
    pencil_mv<T, K>(Bm, v[j], ra[j]);            // c = B_y B_z x
    pencil_mv2<T, K>(Dm, v[j], Bm, w, rb[j]);    // g = D_y B_z x + B_y D_z x
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < CPT; ++j)
#pragma unroll
    for (int iy = 0; iy < K; ++iy) {
      la[j][p1 * PS + iy * RS + p0] = ra[j][iy];
      lb[j][p1 * PS + iy * RS + p0] = rb[j][iy];
    }
  __syncthreads();

  // phase C: x-pencils (iy = p0, iz = p1)
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    T w[K];
#pragma unroll
    for (int q = 0; q < K; ++q) {
      v[j][q] = la[j][p1 * PS + p0 * RS + q];
      w[q] = lb[j][p1 * PS + p0 * RS + q];
    }
    pencil_mv2<T, K>(Dm, v[j], Bm, w, ra[j]);    // D_x c + B_x g
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < CPT; ++j)
#pragma unroll
    for (int ix = 0; ix < K; ++ix) la[j][p1 * PS + p0 * RS + ix] = ra[j][ix] * scale;
  __syncthreads();

  // store through the z-pencil orientation (ix = p0, iy = p1), with the
  // epilogue y = alpha A x + beta bsrc (read before y is written: bsrc may alias y)
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    if (active[j]) {
      const int64_t off = cell[j] * (K * K * K) + p0 + K * p1;
      T* yc = y + off;
#pragma unroll
      for (int iz = 0; iz < K; ++iz) {
        T val = la[j][iz * PS + p1 * RS + p0];
        if (zmask[j] & (1u << iz)) val = T(0);
        val *= alpha;
        if (bsrc) val += beta * bsrc[off + iz * K * K];
        store_out(val, yc + iz * K * K);
      }
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

// Degree 7 (K = 8) on the matrix cores.  One wavefront per cell; each of the
// three contractions is a chain of 16x16x4 MFMAs whose 16 output rows carry
// two results at once, so that no operand is padded along the contraction:
//   z:  [B; D] (16 x 8) times the cell (8 z-rows x 64 (x, y) columns) gives
//       a = B_z x and b = D_z x;
//   y:  [[B, 0], [D, B]] (16 x 16) times [a; b] (16 y-rows x 64 (x, z)
//       columns) gives c = B_y a and g = D_y a + B_y b;
//   x:  [[D, B], [0, 0]] times [c; g] (16 x-rows x 64 (y, z) columns) gives
//       D_x c + B_x g in the upper 8 rows (the lower 8 are the only padding).
// Between the contractions the 16 x 64 results are re-laid out through the
// wavefront's own LDS area (rows padded against bank conflicts); a wavefront
// never waits for another, so there is no block barrier.  Lane layouts
// (16x16x4 FP32): A[i][k] in lane i + 16k, B[k][j] in lane j + 16k; the
// result D[i][j] in lane j + 16 (i / 4), register i % 4.
// FP32 only: the FP64 matrix rate of this chip equals its FP64 vector rate,
// and with the padded last contraction (40 MFMAs for 28 of useful work) the
// FP64 variant measured 73 us against 64 us for the vector kernel at Q7 32^3;
// in FP32 the matrix cores are twice the vector rate (44 us against 51 us).
template <typename T>
struct Mfma16;
template <>
struct Mfma16<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int r) { return 4 * (l >> 4) + r; }
  static constexpr int LP = 10, PZ = 80, PA = 640;
};

template <typename T>
__global__ void __launch_bounds__(256) k_apply_cart3_mfma(const T* __restrict__ x, T* y, const T* __restrict__ Bm,
                                                          const T* __restrict__ Dm, T scale, int n, int64_t n_cells,
                                                          int dirichlet, T alpha, T beta, const T* bsrc) {
  using M = Mfma16<T>;
  using v4 = typename M::v4;
  constexpr int CPB = 4, LP = M::LP, PZ = M::PZ, PA = M::PA;
  __shared__ T sm[CPB * 2 * PA];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  T* L = sm + w * 2 * PA;
  const int lr = l & 15, lq = l >> 4;

  // A operands: element (row lr, column 4s + lq) of the three stacked matrices
  T a1[2], a2[4], a3[4];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int kk = 4 * s + lq;
    a1[s] = lr < 8 ? Bm[lr * 8 + kk] : Dm[(lr - 8) * 8 + kk];
  }
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int kk = 4 * s + lq;
    if (lr < 8) {
      a2[s] = kk < 8 ? Bm[lr * 8 + kk] : T(0);
      a3[s] = kk < 8 ? Dm[lr * 8 + kk] : Bm[lr * 8 + kk - 8];
    } else {
      a2[s] = kk < 8 ? Dm[(lr - 8) * 8 + kk] : Bm[(lr - 8) * 8 + kk - 8];
      a3[s] = T(0);
    }
  }

  // Cells are taken in a grid-stride loop, one per wavefront at a time; the
  // next cell's operand is loaded while the current one is contracted.
  // z operand (z-row 4s + lq, column 16t + lr): x[ix + 8 iy + 64 iz]
  const int64_t stride = (int64_t)gridDim.x * CPB;
  int64_t cell = (int64_t)blockIdx.x * CPB + w;
  T xv[2][4];
  auto load_cell = [&](int64_t cl) {
    const T* xc = x + cl * 512 + 64 * lq + lr;
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int t = 0; t < 4; ++t) xv[s][t] = xc[256 * s + 16 * t];
  };
  if (cell < n_cells) load_cell(cell);
  for (; cell < n_cells; cell += stride) {
    T cur[2][4];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int t = 0; t < 4; ++t) cur[s][t] = xv[s][t];
    if (cell + stride < n_cells) load_cell(cell + stride);
    int cx, cy, cz;
    cell_coords3<true>(cell, n, cx, cy, cz);
    // Dirichlet copies: only cells on the domain boundary (uniform branch)
    const bool bnd = dirichlet && (cx == 0 || cy == 0 || cz == 0 || cx == n - 1 || cy == n - 1 || cz == n - 1);
    auto masked = [&](int ix, int iy, int iz) {
      return on_boundary(cx, ix, n, 7) || on_boundary(cy, iy, n, 7) || on_boundary(cz, iz, n, 7);
    };
    if (bnd) {
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int p = 16 * t + lr;
          if (masked(p & 7, p >> 3, 4 * s + lq)) cur[s][t] = T(0);
        }
    }

    // z
    v4 c[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) c[t] = v4{T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int t = 0; t < 4; ++t) c[t] = M::mma(a1[s], cur[s][t], c[t]);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = M::row(l, r);   // (a | b, z)
        L[(i >> 3) * PA + (i & 7) * PZ + (2 * t + (lr >> 3)) * LP + (lr & 7)] = c[t][r];
      }

    // y: operand (row 4s + lq = (a | b, y), column 16t + lr = (x, z))
#pragma unroll
    for (int t = 0; t < 4; ++t) c[t] = v4{T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int kr = 4 * s + lq, col = 16 * t + lr;
        c[t] = M::mma(a2[s], L[(kr >> 3) * PA + (col >> 3) * PZ + (kr & 7) * LP + (col & 7)], c[t]);
      }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = M::row(l, r);   // (c | g, y)
        L[(i >> 3) * PA + (2 * t + (lr >> 3)) * PZ + (i & 7) * LP + (lr & 7)] = c[t][r];
      }

    // x: operand (row 4s + lq = (c | g, x), column 16t + lr = (y, z))
#pragma unroll
    for (int t = 0; t < 4; ++t) c[t] = v4{T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int kr = 4 * s + lq, col = 16 * t + lr;
        c[t] = M::mma(a3[s], L[(kr >> 3) * PA + (col >> 3) * PZ + (col & 7) * LP + (kr & 7)], c[t]);
      }
    // rows 0..7 are x: through LDS into the cell's natural order (rows of 8
    // padded to 9), then stored 4 consecutive values per lane
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = M::row(l, r);
        if (i < 8) L[(2 * t + (lr >> 3)) * 72 + (lr & 7) * 9 + i] = c[t][r];
      }
    // the epilogue y = alpha A x + beta bsrc reads bsrc before y is written
    T* yc = y + cell * 512;
    const T* bc = bsrc ? bsrc + cell * 512 : nullptr;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int o = 4 * (l + 64 * q), iz = o >> 6, iy = (o >> 3) & 7, ix0 = o & 7;
      T v[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        v[e] = L[iz * 72 + iy * 9 + ix0 + e] * scale;
        if (bnd && masked(ix0 + e, iy, iz)) v[e] = T(0);
        v[e] *= alpha;
      }
      if (bc) {
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] += beta * bc[o + e];
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) __builtin_nontemporal_store(v[e], yc + o + e);   // 1 KB per instruction: 37.2 -> 35.2 us at 32^3
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
  if (p->dim == 3 && K == 8 && sizeof(T) == 4) {
    // grid-stride over cells: about eight cells per wavefront at the largest sizes
    static int resident = 0;
    if (resident == 0) {
      int dev = 0, cus = 0, per_cu = 0;
      FE_HIP_CHECK(hipGetDevice(&dev));
      FE_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
      FE_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_apply_cart3_mfma<float>, 256, 0));
      resident = cus * (per_cu > 0 ? per_cu : 1);
    }
    const int64_t nb = std::max<int64_t>(1, std::min<int64_t>((L.n_cells + 3) / 4, resident));
    ProfScope ps("apply", s);
    hipLaunchKernelGGL((k_apply_cart3_mfma<float>), dim3((unsigned)nb), dim3(256), 0, s, (const float*)x, (float*)y,
                       (const float*)Bm, (const float*)Dm, (float)scale, L.n, L.n_cells, p->bc, (float)alpha,
                       (float)beta, (const float*)b);
  } else if (p->dim == 3 && K == 4 && sizeof(T) == 4) {
    if constexpr (K == 4 && sizeof(T) == 4) {   // (instantiated only here)
      // FP32 Q3: two cells per thread (twice the bytes in flight)
      constexpr int CPB = 256 / (K * K), CPT = 2;
      const int64_t nb = (L.n_cells + CPB * CPT - 1) / (CPB * CPT);
      ProfScope ps("apply", s);
      hipLaunchKernelGGL((k_apply_cart3_multi<T, K, CPT>), dim3((unsigned)nb), dim3(CPB * K * K), 0, s, x, y, Bm,
                         Dm, scale, L.n, L.n_cells, p->bc, alpha, beta, b);
    }
  } else if (p->dim == 3) {
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
