// Fused masked Jacobi sweep of Algorithm 9 (its update and averaging steps in one pass):
//   out = S_bar (u + omega Dhat^{-1} (b - v)),
// Dhat^{-1} the valence-baked masked inverse diagonal (Sec. 5, eqs.
// valence_baking and deferred_assembly).  One thread per cell-wise entry
// gathers the raw per-copy updates of every copy of its node (index
// arithmetic, at most 2^d copies), sums them in the x-, y-, z-pair order of
// the structured cascade, divides by the valence (a power of two, exact)
// and writes its own entry.  Out of place: consecutive threads write
// consecutive addresses (whole cache lines), and no copy is read after it
// was overwritten.  Every copy of a node forms the same sum in the same
// order, so the output is continuous bit for bit.
#include "fe_internal.h"
#include "kernel_common.h"

namespace fe {

template <typename T, int K>
__global__ void __launch_bounds__(256) k_jacobi_avg3(const T* __restrict__ u, const T* __restrict__ b,
                                                     const T* __restrict__ v, const T* __restrict__ dinv,
                                                     T* __restrict__ out, T omega, int u_is_zero, int n,
                                                     int64_t len) {
  constexpr int k = K - 1;
  constexpr int K3 = K * K * K;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  const int64_t cell = e / K3;
  const int loc = (int)(e - cell * K3);
  const int ix = loc % K, iy = (loc / K) % K, iz = loc / (K * K);
  const int cx = (int)(cell % n);
  const int64_t t = cell / n;
  const int cy = (int)(t % n), cz = (int)(t / n);
  const AxisCopies ax = axis_copies<K>(k * cx + ix, n);
  const AxisCopies ay = axis_copies<K>(k * cy + iy, n);
  const AxisCopies az = axis_copies<K>(k * cz + iz, n);
  auto val = [&](int64_t a) -> T {
    return u_is_zero ? omega * dinv[a] * b[a] : fma(omega * dinv[a], b[a] - v[a], u[a]);
  };
  T zs[2];
  for (int sz = 0; sz < az.cnt; ++sz) {
    T ys[2];
    for (int sy = 0; sy < ay.cnt; ++sy) {
      T xs = val(copy_addr<K, 3>(ax, ay, az, 0, sy, sz, n));
      if (ax.cnt == 2) xs += val(copy_addr<K, 3>(ax, ay, az, 1, sy, sz, n));
      ys[sy] = xs;
    }
    zs[sz] = ay.cnt == 2 ? ys[0] + ys[1] : ys[0];
  }
  T s = az.cnt == 2 ? zs[0] + zs[1] : zs[0];
  const int kappa = ax.cnt * ay.cnt * az.cnt;
  out[e] = kappa == 1 ? s : s * (T(1) / T(kappa));
}

template <typename T, int K>
static fe_status jacobi_avg_typed(const fe_problem* p, int level, const T* u, const T* b, const T* v, const T* dinv,
                                  T* out, double omega, int u_is_zero, hipStream_t s) {
  const Level& L = level_of(p, level);
  ProfScope ps("jacobi_avg", s);
  hipLaunchKernelGGL((k_jacobi_avg3<T, K>), dim3((unsigned)((L.len + 255) / 256)), dim3(256), 0, s, u, b, v, dinv,
                     out, (T)omega, u_is_zero, L.n, L.len);
  FE_HIP_CHECK(hipGetLastError());
  return FE_OK;
}

fe_status launch_jacobi_avg(const fe_problem* p, int level, const void* u, const void* b, const void* v,
                            const void* dinv, void* out, double omega, int u_is_zero, fe_dtype dt, hipStream_t s) {
  if (p->dim != 3) return fail(FE_EUNSUPPORTED, "the fused sweep is implemented for d = 3");
  if (dt == FE_F64) {
    FE_DISPATCH_K(p->K, return (jacobi_avg_typed<double, KK>(p, level, (const double*)u, (const double*)b,
                                                             (const double*)v, (const double*)dinv, (double*)out,
                                                             omega, u_is_zero, s)));
  }
  FE_DISPATCH_K(p->K, return (jacobi_avg_typed<float, KK>(p, level, (const float*)u, (const float*)b,
                                                          (const float*)v, (const float*)dinv, (float*)out, omega,
                                                          u_is_zero, s)));
}

}  // namespace fe
