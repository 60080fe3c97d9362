// Device helpers shared by the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fe {

// A K x K matrix of T that does not fit in the scalar registers next to
// everything else (more than 24 of them): its rows are fetched where they are
// used.  Without this the compiler loads the whole matrix up front and parks
// the entries in vector-register lanes (one readlane per use).
template <typename T, int K>
struct RowFetch {
  static constexpr bool value = K * K * (int)sizeof(T) > 4 * 24;
};
template <typename T, int K>
__device__ __forceinline__ void row_fence() {
  if (RowFetch<T, K>::value) asm volatile("" ::: "memory");
}

// Pencil matrix-vector product out = M in, M row-major K x K at a uniform
// (wave-invariant) address, so the entries are fetched with scalar loads.
template <typename T, int K>
__device__ __forceinline__ void pencil_mv(const T* __restrict__ M, const T (&in)[K], T (&out)[K]) {
#pragma unroll
  for (int i = 0; i < K; ++i) {
    row_fence<T, K>();
    T s = M[i * K] * in[0];
#pragma unroll
    for (int j = 1; j < K; ++j) s = fma(M[i * K + j], in[j], s);
    out[i] = s;
  }
}

// out = M^T in
template <typename T, int K>
__device__ __forceinline__ void pencil_mtv(const T* __restrict__ M, const T (&in)[K], T (&out)[K]) {
#pragma unroll
  for (int i = 0; i < K; ++i) {
    row_fence<T, K>();
    T s = M[i] * in[0];
#pragma unroll
    for (int j = 1; j < K; ++j) s = fma(M[j * K + i], in[j], s);
    out[i] = s;
  }
}

// out = A in_a + B in_b
template <typename T, int K>
__device__ __forceinline__ void pencil_mv2(const T* __restrict__ A, const T (&ia)[K],
                                           const T* __restrict__ B, const T (&ib)[K], T (&out)[K]) {
#pragma unroll
  for (int i = 0; i < K; ++i) {
    row_fence<T, K>();
    T s = A[i * K] * ia[0];
#pragma unroll
    for (int j = 1; j < K; ++j) s = fma(A[i * K + j], ia[j], s);
#pragma unroll
    for (int j = 0; j < K; ++j) s = fma(B[i * K + j], ib[j], s);
    out[i] = s;
  }
}

// Copies of one global node coordinate g along one axis: the cells c and
// local indices i with k*c + i = g (one copy inside a cell, two on an
// interior cell face, one on the domain boundary).  Order: lower cell first.
struct AxisCopies {
  int cnt;
  int c[2];
  int i[2];
};

template <int K>
__device__ __forceinline__ AxisCopies axis_copies(int g, int n) {
  constexpr int k = K - 1;
  AxisCopies a;
  const int q = g / k, r = g - q * k;
  if (r != 0) {
    a.cnt = 1; a.c[0] = q; a.i[0] = r; a.c[1] = q; a.i[1] = r;
  } else {
    a.cnt = 0;
    if (q > 0) { a.c[a.cnt] = q - 1; a.i[a.cnt] = k; ++a.cnt; }
    if (q < n) { a.c[a.cnt] = q; a.i[a.cnt] = 0; ++a.cnt; }
    if (a.cnt == 1) { a.c[1] = a.c[0]; a.i[1] = a.i[0]; }
  }
  return a;
}

// Coordinates of cell `cell` of an n^3 mesh.  Cell indices fit in 32 bits
// (problem creation bounds the cell-wise length by 2^33 values, so n^3 <=
// 2^30); with a wavefront-uniform cell (UNIFORM) the divisions run on the
// scalar unit.
template <bool UNIFORM>
__device__ __forceinline__ void cell_coords3(int64_t cell, int n, int& cx, int& cy, int& cz) {
  int c = (int)cell;
  if (UNIFORM) c = __builtin_amdgcn_readfirstlane(c);
  const int t = c / n;
  cx = c - t * n;
  cy = t % n;
  cz = t / n;
}

__device__ __forceinline__ bool on_boundary(int c, int i, int n, int k) {
  return (c == 0 && i == 0) || (c == n - 1 && i == k);
}

// Index of copy (sx, sy, sz) of a node with per-axis copies ax, ay, az.
template <int K, int DIM>
__device__ __forceinline__ int64_t copy_addr(const AxisCopies& ax, const AxisCopies& ay,
                                             const AxisCopies& az, int sx, int sy, int sz, int n) {
  if (DIM == 3) {
    const int64_t cell = ax.c[sx] + (int64_t)n * (ay.c[sy] + (int64_t)n * az.c[sz]);
    return cell * (K * K * K) + ax.i[sx] + K * (ay.i[sy] + K * az.i[sz]);
  } else {
    const int64_t cell = ax.c[sx] + (int64_t)n * ay.c[sy];
    return cell * (K * K) + ax.i[sx] + K * ay.i[sy];
  }
}

// Sum of all copies in cascade order.
template <typename T, int K, int DIM>
__device__ __forceinline__ T cascade_sum(const T* __restrict__ v, const AxisCopies& ax, const AxisCopies& ay,
                                         const AxisCopies& az, int n) {
  const int nz = DIM == 3 ? az.cnt : 1;
  T zs[2];
  for (int sz = 0; sz < nz; ++sz) {
    T ys[2];
    for (int sy = 0; sy < ay.cnt; ++sy) {
      T xs = v[copy_addr<K, DIM>(ax, ay, az, 0, sy, sz, n)];
      if (ax.cnt == 2) xs += v[copy_addr<K, DIM>(ax, ay, az, 1, sy, sz, n)];
      ys[sy] = xs;
    }
    zs[sz] = ay.cnt == 2 ? ys[0] + ys[1] : ys[0];
  }
  return nz == 2 ? zs[0] + zs[1] : zs[0];
}

}  // namespace fe

// Dispatch a runtime K = k+1 to a compile-time constant KK.
#define FE_DISPATCH_K(KVAL, CALL)          \
  switch (KVAL) {                          \
    case 2: { constexpr int KK = 2; CALL; } \
    case 3: { constexpr int KK = 3; CALL; } \
    case 4: { constexpr int KK = 4; CALL; } \
    case 5: { constexpr int KK = 5; CALL; } \
    case 6: { constexpr int KK = 6; CALL; } \
    case 7: { constexpr int KK = 7; CALL; } \
    case 8: { constexpr int KK = 8; CALL; } \
    case 9: { constexpr int KK = 9; CALL; } \
    default: return fail(FE_EINVAL, "unsupported degree"); \
  }
