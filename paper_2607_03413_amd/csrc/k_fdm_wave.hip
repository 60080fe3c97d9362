// Vertex-patch fast-diagonalization inverse with one block per patch and one
// lane per pencil (3D, k >= 4: m = 2k-1 = 7..15, m^2 pencils of m values,
// m^3 patch values in LDS; Q7: 169 pencils on three wavefronts).
//
// z = G sum_p R_p^T (S_x x S_y x S_z) (L_x + L_y + L_z)^{-1} (S_x x S_y x S_z)^T R_p G^T r
// (vertex-patch smoother admissible by eq. precond_consistency, Sec. 2.1;
// fast diagonalization of the separable patch operator).  The 1D factors
// are uniform over a wavefront: the Cartesian S (even/odd halves) and the
// eigenvalues are read through the scalar cache and every FMA takes one
// operand from a scalar register; per-patch factors (three dense m x m
// matrices) are staged in LDS and read as broadcasts, a row at a time:
//   * lane l owns pencil l (a line of m values) of every pass, so a patch is
//     spread over several wavefronts and each pass is one round; the LDS
//     array of a patch limits how many patches a CU holds, not the lanes;
//   * the residual is assembled per z-pencil straight from the cell-wise
//     input (copies summed in cascade order: x pairs, then y, then z) and
//     contracted with S_z^T in registers before it reaches LDS;
//   * y: S_y^T; x: S_x^T, scaling by the inverse eigenvalue sums, S_x; y: S_y,
//     each an in-place pass over LDS lines (no two lanes share a line; a
//     workgroup barrier separates the passes);
//   * z: S_z in registers, and the patch solution is written patch-major
//     (m^3 values per patch) for the summing pass.
// With the exact Cartesian factors the mirror symmetry of the two-cell patch
// is used: every eigenvector is even or odd about the middle node, so a
// line costs (c+1)^2 + c^2 instead of m^2 FMAs (c = k-1).
#include <type_traits>

#include "fe_internal.h"
#include "kernel_common.h"

namespace fe {

template <int K>
struct WavePatch {
  static constexpr int k = K - 1;
  static constexpr int M = 2 * k - 1;
  static constexpr int M2 = M * M;
  static constexpr int M3 = M2 * M;
  static constexpr int THREADS = (M2 + 63) / 64 * 64;   // one lane per pencil, whole wavefronts
  static constexpr int C = k - 1;         // middle node
  static constexpr int NE = C + 1, NO = C;
};
// LDS row stride of a per-patch factor matrix: M rounded up to 16 bytes
template <typename T, int M>
struct FactorRows {
  static constexpr int VPC = 16 / (int)sizeof(T);
  static constexpr int MS = (M + VPC - 1) / VPC * VPC;
};

// 1 / x: hardware reciprocal refined by Newton steps r <- r (2 - x r).
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = r * fma(-x, r, 2.0);
  r = r * fma(-x, r, 2.0);
  return r;
}
__device__ __forceinline__ float recip(float x) {
  float r = __builtin_amdgcn_rcpf(x);
  return r * fmaf(-x, r, 2.0f);
}

// y = S^T x (FWD) or y = S x for one line.  EO: S given by its even/odd
// halves (modes ordered evens first); otherwise S is M x M row-major, S[a*M + j].
template <typename T, int M, bool EO, bool FWD>
__device__ __forceinline__ void line_apply(const T* __restrict__ S, const T (&x)[M], T (&y)[M]) {
  if (EO) {
    constexpr int c = (M - 1) / 2, ne = c + 1, no = c;
    const T* __restrict__ SE = S;
    const T* __restrict__ SO = S + ne * (c + 1);
    if (FWD) {
      T sum[c + 1], dif[c > 0 ? c : 1];
#pragma unroll
      for (int a = 0; a < c; ++a) {
        sum[a] = x[a] + x[M - 1 - a];
        dif[a] = x[a] - x[M - 1 - a];
      }
      sum[c] = x[c];
#pragma unroll
      for (int j = 0; j < ne; ++j) {
        T s = SE[j * (c + 1)] * sum[0];
#pragma unroll
        for (int a = 1; a <= c; ++a) s = fma(SE[j * (c + 1) + a], sum[a], s);
        y[j] = s;
      }
#pragma unroll
      for (int j = 0; j < no; ++j) {
        T s = SO[j * c] * dif[0];
#pragma unroll
        for (int a = 1; a < c; ++a) s = fma(SO[j * c + a], dif[a], s);
        y[ne + j] = s;
      }
    } else {
#pragma unroll
      for (int a = 0; a <= c; ++a) {
        T e = SE[a] * x[0];
#pragma unroll
        for (int j = 1; j < ne; ++j) e = fma(SE[j * (c + 1) + a], x[j], e);
        if (a == c) {
          y[c] = e;
        } else {
          T o = SO[a] * x[ne];
#pragma unroll
          for (int j = 1; j < no; ++j) o = fma(SO[j * c + a], x[ne + j], o);
          y[a] = e + o;
          y[M - 1 - a] = e - o;
        }
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < M; ++i) {
      T s = (FWD ? S[i] : S[i * M]) * x[0];
#pragma unroll
      for (int a = 1; a < M; ++a) s = fma(FWD ? S[a * M + i] : S[i * M + a], x[a], s);
      y[i] = s;
    }
  }
}

// The same for per-patch factors staged in LDS (rows of MS >= M values, a
// multiple of 16 bytes, so that a row is read 16 bytes at a time; every lane
// reads the same address, a broadcast).  The products are accumulated in the
// order of line_apply (a ascending), so the results are the same.
template <typename T>
using lds_cptr = const __attribute__((address_space(3))) T*;
template <typename T, int M, int MS, bool FWD>
__device__ __forceinline__ void line_apply_lds(lds_cptr<T> S, const T (&x)[M], T (&y)[M]) {
  // one row of S in flight at a time (otherwise the whole matrix is loaded
  // into vector registers up front)
  if (FWD) {
#pragma unroll
    for (int i = 0; i < M; ++i) y[i] = S[i] * x[0];
#pragma unroll
    for (int a = 1; a < M; ++a) {
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int i = 0; i < M; ++i) y[i] = fma(S[a * MS + i], x[a], y[i]);
    }
  } else {
#pragma unroll
    for (int i = 0; i < M; ++i) {
      __builtin_amdgcn_sched_barrier(0);
      T s = S[i * MS] * x[0];
#pragma unroll
      for (int a = 1; a < M; ++a) s = fma(S[i * MS + a], x[a], s);
      y[i] = s;
    }
  }
}

// Copies of patch-local node a (0 <= a <= 2k-2) along one axis: cell slot
// (0 = lower cell, 1 = upper cell) and local index, lower slot first.
template <int K>
__device__ __forceinline__ AxisCopies wave_axis_copies(int a) {
  constexpr int k = K - 1;
  AxisCopies c;
  const int o = a + 1;
  if (o < k) { c.cnt = 1; c.c[0] = 0; c.i[0] = o; }
  else if (o > k) { c.cnt = 1; c.c[0] = 1; c.i[0] = o - k; }
  else { c.cnt = 2; c.c[0] = 0; c.i[0] = k; c.c[1] = 1; c.i[1] = 0; }
  if (c.cnt == 1) { c.c[1] = c.c[0]; c.i[1] = c.i[0]; }
  return c;
}

// eig (PER_PATCH): per patch S_x, S_y, S_z (M x M), l_x, l_y, l_z (M);
// otherwise (EO) the even/odd halves of the Cartesian S and the eigenvalues,
// and il the level's table of scale / (l_x + l_y + l_z) in the same mode order.
template <typename T, int K, bool PER_PATCH>
// (FP32: at least 5 wavefronts per SIMD with per-patch factors, measured
// faster than the 128 VGPRs the compiler takes by itself for the residual
// loads; at least 4 with the Cartesian factors, which would otherwise take 134)
__global__ void __launch_bounds__(WavePatch<K>::THREADS)
    __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? (PER_PATCH ? 5 : 4) : 1))) k_fdm_patch3_wave(const T* __restrict__ r, T* __restrict__ W,
                                                        const T* __restrict__ eig, const T* __restrict__ il,
                                                        T scale, int n) {
  using P = WavePatch<K>;
  constexpr int M = P::M, M2 = P::M2, M3 = P::M3;
  constexpr int K3 = K * K * K;
  constexpr bool EO = !PER_PATCH;
  __shared__ T t[M3];
  const int lane = threadIdx.x;
  const int nv = n - 1;
  // XCD-aware order: blocks are dealt to the 8 XCDs round-robin; give each XCD
  // a contiguous range of patches so that neighbouring patches, which read the
  // same cells, share an L2
  const int64_t nb = gridDim.x, q8 = nb >> 3, rem = nb & 7;
  const int64_t xcd = blockIdx.x & 7;
  const int64_t pid = xcd * q8 + (xcd < rem ? xcd : rem) + (blockIdx.x >> 3);
  const int vx = 1 + (int)(pid % nv), vy = 1 + (int)((pid / nv) % nv), vz = 1 + (int)(pid / ((int64_t)nv * nv));
  const T* const Sx = eig;   // Cartesian: one even/odd S for all axes
  const T* const Sy = eig;
  const T* const Sz = eig;
  // Per-patch factors: S_x, S_y, S_z and the eigenvalues of this patch go to
  // LDS (scalar registers cannot hold three m x m matrices: they were spilled
  // to vector lanes and read back one value at a time).
  constexpr int MS = FactorRows<T, M>::MS;
  __shared__ __attribute__((aligned(16))) T sF[PER_PATCH ? 3 * M * MS : 1];
  __shared__ T sL[PER_PATCH ? 3 * M : 1];
  if (PER_PATCH) {
    const T* base = eig + pid * (3 * M2 + 3 * M);
    for (int e = lane; e < 3 * M2; e += P::THREADS) {
      const int q = e / M2, rr = e - q * M2, a = rr / M, i = rr - a * M;
      sF[(q * M + a) * MS + i] = base[e];
    }
    for (int e = lane; e < 3 * M; e += P::THREADS) sL[e] = base[3 * M2 + e];
    __syncthreads();
  }
  const lds_cptr<T> fx = (lds_cptr<T>)sF, fy = fx + M * MS, fz = fy + M * MS;
  const int64_t c0 = (vx - 1) + (int64_t)n * ((vy - 1) + (int64_t)n * (vz - 1));
  const T* __restrict__ rc = r + c0 * K3;
  const int64_t sy_cells = (int64_t)n * K3, sz_cells = (int64_t)n * n * K3;

  // (1) z-pencils (x, y): assemble, S_z^T, store
  {
    const int l = lane;
    if (l < M2) {
      // Only pencils on the patch's middle cross (x = k-1 or y = k-1, a cell
      // face) have second copies along x or y.  They take the first lanes
      // (the column x = k-1, then the rest of the row y = k-1), the other
      // pencils follow in row order, so that the wavefronts without any such
      // pencil load one copy per node (a uniform branch around the whole
      // assembly, taken before any load).
      constexpr int C = P::C;
      int x, y;
      if (l < M) {
        x = C; y = l;
      } else if (l < 2 * M - 1) {
        const int q = l - M;
        x = q < C ? q : q + 1; y = C;
      } else {
        const int q = l - (2 * M - 1), yy = q / (M - 1), xx = q - yy * (M - 1);
        x = xx < C ? xx : xx + 1; y = yy < C ? yy : yy + 1;
      }
      const AxisCopies cx = wave_axis_copies<K>(x), cy = wave_axis_copies<K>(y);
      T v[M], w[M];
      // On the cross both copies along x and y are loaded in every lane (a
      // node with one copy reads it twice and weights the second by 0): a load
      // behind a lane-dependent branch waits for its data before the next is
      // issued.  fma(b, 1, a) rounds as a + b, so the sums are those of the copies.
      const T wx = cx.cnt == 2 ? T(1) : T(0), wy = cy.cnt == 2 ? T(1) : T(0);
      auto assemble = [&](auto cross) {
        constexpr int NC = decltype(cross)::value ? 2 : 1;
#pragma unroll
        for (int z = 0; z < M; ++z) {
          const AxisCopies cz = wave_axis_copies<K>(z);   // compile-time after unrolling
          T zs = T(0);
#pragma unroll
          for (int sz = 0; sz < 2; ++sz) {
            if (sz >= cz.cnt) break;
            T ys = T(0);
#pragma unroll
            for (int sy = 0; sy < NC; ++sy) {
              const T* cb = rc + cz.c[sz] * sz_cells + cy.c[sy] * sy_cells + K * (cy.i[sy] + K * cz.i[sz]);
              const T xs = NC == 2 ? fma(cb[cx.c[1] * K3 + cx.i[1]], wx, cb[cx.c[0] * K3 + cx.i[0]])
                                   : cb[cx.c[0] * K3 + cx.i[0]];
              ys = sy == 0 ? xs : fma(xs, wy, ys);
            }
            zs = sz == 0 ? ys : zs + ys;
          }
          v[z] = zs;
        }
      };
      if (__ballot(cx.cnt == 2 || cy.cnt == 2) != 0) assemble(std::true_type{});
      else assemble(std::false_type{});
      if (PER_PATCH) line_apply_lds<T, M, MS, true>(fz, v, w);
      else line_apply<T, M, EO, true>(Sz, v, w);
#pragma unroll
      for (int z = 0; z < M; ++z) t[z * M2 + y * M + x] = w[z];
    }
  }
  __syncthreads();
  // (2) y-pencils (x, z): S_y^T
  {
    const int l = lane;
    if (l < M2) {
      const int x = l % M, z = l / M;
      T v[M], w[M];
#pragma unroll
      for (int a = 0; a < M; ++a) v[a] = t[z * M2 + a * M + x];
      if (PER_PATCH) line_apply_lds<T, M, MS, true>(fy, v, w);
      else line_apply<T, M, EO, true>(Sy, v, w);
#pragma unroll
      for (int a = 0; a < M; ++a) t[z * M2 + a * M + x] = w[a];
    }
  }
  __syncthreads();
  // (3) x-pencils (y, z): S_x^T, scale by (l_x + l_y + l_z)^{-1}, S_x
  {
    const int l = lane;
    if (l < M2) {
      const int y = l % M, z = l / M;
      T v[M], w[M];
#pragma unroll
      for (int a = 0; a < M; ++a) v[a] = t[z * M2 + y * M + a];
      if (PER_PATCH) line_apply_lds<T, M, MS, true>(fx, v, w);
      else line_apply<T, M, EO, true>(Sx, v, w);
      if (PER_PATCH) {
        const T lyz = sL[M + y] + sL[2 * M + z];
#pragma unroll
        for (int a = 0; a < M; ++a) w[a] *= scale * recip(sL[a] + lyz);
      } else {
#pragma unroll
        for (int a = 0; a < M; ++a) w[a] *= il[l * M + a];
      }
      if (PER_PATCH) line_apply_lds<T, M, MS, false>(fx, w, v);
      else line_apply<T, M, EO, false>(Sx, w, v);
#pragma unroll
      for (int a = 0; a < M; ++a) t[z * M2 + y * M + a] = v[a];
    }
  }
  __syncthreads();
  // (4) y-pencils: S_y
  {
    const int l = lane;
    if (l < M2) {
      const int x = l % M, z = l / M;
      T v[M], w[M];
#pragma unroll
      for (int a = 0; a < M; ++a) v[a] = t[z * M2 + a * M + x];
      if (PER_PATCH) line_apply_lds<T, M, MS, false>(fy, v, w);
      else line_apply<T, M, EO, false>(Sy, v, w);
#pragma unroll
      for (int a = 0; a < M; ++a) t[z * M2 + a * M + x] = w[a];
    }
  }
  __syncthreads();
  // (5) z-pencils: S_z, then the patch solution, patch-major (m^3 values, x
  // fastest): consecutive lanes store consecutive values
  T* wp = W + pid * M3;
  {
    const int l = lane;
    if (l < M2) {
      T v[M], w[M];
#pragma unroll
      for (int z = 0; z < M; ++z) v[z] = t[z * M2 + l];
      if (PER_PATCH) line_apply_lds<T, M, MS, false>(fz, v, w);
      else line_apply<T, M, EO, false>(Sz, v, w);
#pragma unroll
      for (int z = 0; z < M; ++z) wp[z * M2 + l] = w[z];
    }
  }
}

bool patch_wave_supported(const fe_problem* p, bool per_patch) {
  return p->dim == 3 && p->k >= 4 && p->k <= 8 && (per_patch || p->co.off_Seo >= 0);
}

template <typename T, int K>
static fe_status patch_wave_typed(const Level& L, const T* r, T* W, const T* eig, const T* il, bool per_patch,
                                  T scale, hipStream_t s) {
  const int64_t nv = L.n - 1, np = nv * nv * nv;
  if (np == 0) return FE_OK;
  ProfScope ps("fdm_patch", s);
  if (per_patch)
    hipLaunchKernelGGL((k_fdm_patch3_wave<T, K, true>), dim3((unsigned)np), dim3(WavePatch<K>::THREADS), 0, s, r, W,
                       eig, il, scale, L.n);
  else
    hipLaunchKernelGGL((k_fdm_patch3_wave<T, K, false>), dim3((unsigned)np), dim3(WavePatch<K>::THREADS), 0, s, r, W,
                       eig, il, scale, L.n);
  FE_HIP_CHECK(hipGetLastError());
  return FE_OK;
}

// eig: per-patch eigen-data (per_patch) or null (the Cartesian even/odd table is used)
fe_status launch_patch_wave(const fe_problem* p, const Level& L, const void* r, void* W, const void* eig,
                            bool per_patch, double scale, fe_dtype dt, hipStream_t s) {
  if (!per_patch && p->co.off_il < 0) return fail(FE_EUNSUPPORTED, "wave patch inverse: no eigenvalue table");
  const int64_t M = 2 * p->k - 1;
  const int64_t il_off = per_patch ? 0 : p->co.off_il + (int64_t)(&L - p->levels.data()) * M * M * M;
  switch (p->K) {
#define FE_WAVE_CASE(KV)                                                                                   \
  case KV:                                                                                                 \
    if (dt == FE_F64)                                                                                      \
      return patch_wave_typed<double, KV>(L, (const double*)r, (double*)W,                                 \
                                          per_patch ? (const double*)eig                                   \
                                                    : p->coef64.as<double>() + p->co.off_Seo,              \
                                          p->coef64.as<double>() + il_off, per_patch, scale, s);           \
    return patch_wave_typed<float, KV>(L, (const float*)r, (float*)W,                                      \
                                       per_patch ? (const float*)eig : p->coef32.as<float>() + p->co.off_Seo, \
                                       p->coef32.as<float>() + il_off, per_patch, (float)scale, s);
    FE_WAVE_CASE(5)
    FE_WAVE_CASE(6)
    FE_WAVE_CASE(7)
    FE_WAVE_CASE(8)
    FE_WAVE_CASE(9)
#undef FE_WAVE_CASE
    default:
      return fail(FE_EUNSUPPORTED, "wave patch inverse: unsupported degree");
  }
}

}  // namespace fe
