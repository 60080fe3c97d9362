// Inter-block passes of the multi-block DSS (paper, Sec. 4.3, Algorithm 8):
// macro-face pairs, and gather-scatter over macro-lines and macro-vertices.
// Every entity owns a disjoint set of entries, so no atomics are needed.
#include "fe_internal.h"

namespace fe {

// Macro-face DoFs: a fixed pairwise exchange between the two blocks' copies.
template <typename T>
__global__ void __launch_bounds__(256) k_mb_pairs(T* __restrict__ v, const int32_t* __restrict__ pairs, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t a = pairs[2 * i], b = pairs[2 * i + 1];
  const T s = v[a] + v[b];
  v[a] = s;
  v[b] = s;
}

// Macro-line / macro-vertex DoFs: sum one representative copy per sharing
// block (in block order), write the total to every copy.
template <typename T>
__global__ void __launch_bounds__(256) k_mb_gather_scatter(T* __restrict__ v, const int32_t* __restrict__ rep_ptr,
                                                           const int32_t* __restrict__ rep,
                                                           const int32_t* __restrict__ all_ptr,
                                                           const int32_t* __restrict__ all, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  T s = T(0);
  for (int32_t j = rep_ptr[i]; j < rep_ptr[i + 1]; ++j) s += v[rep[j]];
  for (int32_t j = all_ptr[i]; j < all_ptr[i + 1]; ++j) v[all[j]] = s;
}

template <typename T>
__global__ void __launch_bounds__(256) k_mb_scale(T* __restrict__ v, const double* __restrict__ w, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = (T)((double)v[i] * w[i]);
}

static unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

fe_status launch_mb_pairs(void* v, const int32_t* pairs, int64_t n, fe_dtype dt, hipStream_t s) {
  if (n == 0) return FE_OK;
  if (dt == FE_F64) hipLaunchKernelGGL(k_mb_pairs<double>, dim3(nblk(n)), dim3(256), 0, s, (double*)v, pairs, n);
  else hipLaunchKernelGGL(k_mb_pairs<float>, dim3(nblk(n)), dim3(256), 0, s, (float*)v, pairs, n);
  FE_HIP_CHECK(hipGetLastError());
  return FE_OK;
}

fe_status launch_mb_gather_scatter(void* v, const int32_t* rep_ptr, const int32_t* rep, const int32_t* all_ptr,
                                   const int32_t* all, int64_t n, fe_dtype dt, hipStream_t s) {
  if (n == 0) return FE_OK;
  if (dt == FE_F64)
    hipLaunchKernelGGL(k_mb_gather_scatter<double>, dim3(nblk(n)), dim3(256), 0, s, (double*)v, rep_ptr, rep, all_ptr,
                       all, n);
  else
    hipLaunchKernelGGL(k_mb_gather_scatter<float>, dim3(nblk(n)), dim3(256), 0, s, (float*)v, rep_ptr, rep, all_ptr,
                       all, n);
  FE_HIP_CHECK(hipGetLastError());
  return FE_OK;
}

fe_status launch_mb_scale(void* v, const double* w, int64_t n, fe_dtype dt, hipStream_t s) {
  if (n == 0) return FE_OK;
  if (dt == FE_F64) hipLaunchKernelGGL(k_mb_scale<double>, dim3(nblk(n)), dim3(256), 0, s, (double*)v, w, n);
  else hipLaunchKernelGGL(k_mb_scale<float>, dim3(nblk(n)), dim3(256), 0, s, (float*)v, w, n);
  FE_HIP_CHECK(hipGetLastError());
  return FE_OK;
}

}  // namespace fe
