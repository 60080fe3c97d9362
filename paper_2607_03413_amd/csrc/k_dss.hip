// Gather G, assembly G^T, direct stiffness summation S and averaging S_bar,
// and the assembled residual norm.
//
// Paper: G replicates, G^T sums the cell copies (Sec. 2.1); S = G G^T
// (Sec. 4.1, eq. dss_operator); S_bar = G (G^T G)^{-1} G^T (Sec. 5,
// eq. averaging_dss).  The paper evaluates S as d sequential axis passes over
// interface pairs (Algorithm 7).  Here one thread owns one global node: it
// reads every copy (at most 2^d, located by index arithmetic, no tables),
// forms the sum in the cascade's order -- x pairs, then y pairs, then z
// pairs -- and writes it to every copy.  Each copy belongs to exactly one
// node, so the pass runs in place without atomics and without a second or
// third launch, and the bits equal those of the cascade.  Interior nodes of a
// cell (valence 1) are left untouched, which S and S_bar do anyway.
#include "fe_internal.h"
#include "kernel_common.h"

namespace fe {

template <int DIM>
__device__ __forceinline__ void node_coords(int64_t g, int N, int& gx, int& gy, int& gz) {
  gx = (int)(g % N);
  const int64_t t = g / N;
  if (DIM == 3) { gy = (int)(t % N); gz = (int)(t / N); }
  else { gy = (int)t; gz = 0; }
}

template <typename T, int K, int DIM>
__global__ void __launch_bounds__(256) k_dss(T* __restrict__ v, int n, int64_t n_nodes, int averaging) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_nodes) return;
  const int N = (K - 1) * n + 1;
  int gx, gy, gz;
  node_coords<DIM>(g, N, gx, gy, gz);
  const AxisCopies ax = axis_copies<K>(gx, n), ay = axis_copies<K>(gy, n);
  const AxisCopies az = DIM == 3 ? axis_copies<K>(gz, n) : axis_copies<K>(1, n);
  const int nz = DIM == 3 ? az.cnt : 1;
  const int kappa = ax.cnt * ay.cnt * nz;
  if (kappa == 1) return;
  T s = cascade_sum<T, K, DIM>(v, ax, ay, az, n);
  if (averaging) s *= T(1) / T(kappa);   // kappa is a power of two: exact
  for (int sz = 0; sz < nz; ++sz)
    for (int sy = 0; sy < ay.cnt; ++sy)
      for (int sx = 0; sx < ax.cnt; ++sx) v[copy_addr<K, DIM>(ax, ay, az, sx, sy, sz, n)] = s;
}

template <typename T, int K, int DIM>
__global__ void __launch_bounds__(256) k_assemble(const T* __restrict__ v, T* __restrict__ out, int n,
                                                  int64_t n_nodes) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_nodes) return;
  const int N = (K - 1) * n + 1;
  int gx, gy, gz;
  node_coords<DIM>(g, N, gx, gy, gz);
  const AxisCopies ax = axis_copies<K>(gx, n), ay = axis_copies<K>(gy, n);
  const AxisCopies az = DIM == 3 ? axis_copies<K>(gz, n) : axis_copies<K>(1, n);
  out[g] = cascade_sum<T, K, DIM>(v, ax, ay, az, n);
}

template <typename T, int K, int DIM>
__global__ void __launch_bounds__(256) k_gather(const T* __restrict__ xg, T* __restrict__ xc, int n,
                                                int64_t len) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  constexpr int NL = DIM == 3 ? K * K * K : K * K;
  constexpr int k = K - 1;
  const int64_t cell = e / NL;
  const int loc = (int)(e - cell * NL);
  const int N = k * n + 1;
  const int ix = loc % K, iy = (loc / K) % K, iz = loc / (K * K);
  const int cx = (int)(cell % n);
  const int64_t t = cell / n;
  int64_t gidx;
  if (DIM == 3) {
    const int cy = (int)(t % n), cz = (int)(t / n);
    gidx = (k * cx + ix) + (int64_t)N * ((k * cy + iy) + (int64_t)N * (k * cz + iz));
  } else {
    gidx = (k * cx + ix) + (int64_t)N * (k * (int)t + iy);
  }
  xc[e] = xg[gidx];
}

// 3D, cell-wise: the thread of a cell-wise entry (cell c, local index i) finds
// the node's other copies by index arithmetic.  Along one axis, the other copy
// is (c-1, k) for i = 0 and (c+1, 0) for i = k when that cell exists (w = 1);
// otherwise it is the entry itself, with w = 0.
template <int K>
__device__ __forceinline__ void other_copy(int c, int i, int n, int& co, int& io, int& w) {
  constexpr int k = K - 1;
  const bool lo = i == 0 && c > 0, hi = i == k && c < n - 1;
  co = lo ? c - 1 : (hi ? c + 1 : c);
  io = lo ? k : (hi ? 0 : i);
  w = (lo || hi) ? 1 : 0;
}

// Sum of all copies of the node of entry (cx, cy, cz; ix, iy, iz), whose own
// copy is at *p, grouped as in the cascade: x pairs, then the y pair of x
// sums, then the z pair (each pair sum is the same whichever copy forms it).
// The other copies are 32-bit offsets from p.  The loads are not branched
// around per lane: an absent partner re-reads the entry's own copy and is
// added times 0, an exact 0, so that no load waits behind a divergent branch.
// kappa = number of copies.
template <typename T, int K>
__device__ __forceinline__ T node_sum3(const T* __restrict__ p, int cx, int cy, int cz, int ix, int iy, int iz, int n,
                                       int& kappa) {
  constexpr int K3 = K * K * K;
  int xo, jx, wx, yo, jy, wy, zo, jz, wz;
  other_copy<K>(cx, ix, n, xo, jx, wx);
  other_copy<K>(cy, iy, n, yo, jy, wy);
  other_copy<K>(cz, iz, n, zo, jz, wz);
  const int dx = (xo - cx) * K3 + (jx - ix);
  const int dy = (yo - cy) * (n * K3) + (jy - iy) * K;
  const int dz = (zo - cz) * (n * n * K3) + (jz - iz) * (K * K);
  // the z partners are loaded only where a lane of the wavefront has one (a
  // uniform branch taken before any load: at Q7 a wavefront is one z-plane of
  // a cell, and two planes in eight have z partners)
  T v000, v100, v010, v110, v001, v101, v011, v111;
  if (__ballot(wz) != 0) {
    v000 = p[0]; v100 = p[dx]; v010 = p[dy]; v110 = p[dx + dy];
    v001 = p[dz]; v101 = p[dx + dz]; v011 = p[dy + dz]; v111 = p[dx + dy + dz];
  } else {
    v000 = p[0]; v100 = p[dx]; v010 = p[dy]; v110 = p[dx + dy];
    v001 = v000; v101 = v100; v011 = v010; v111 = v110;
  }
  const T tx = T(wx), ty = T(wy), tz = T(wz);
  const T x00 = fma(v100, tx, v000), x10 = fma(v110, tx, v010);
  const T x01 = fma(v101, tx, v001), x11 = fma(v111, tx, v011);
  const T y0 = fma(x10, ty, x00), y1 = fma(x11, ty, x01);
  kappa = (1 + wx) * (1 + wy) * (1 + wz);
  return fma(y1, tz, y0);
}

// Whole cells per block for the cell-wise passes (at least one wavefront).
template <int K>
struct CellBlock {
  static constexpr int K3 = K * K * K;
  static constexpr int CPB = K3 >= 64 ? 1 : 64 / K3;
  static constexpr int THREADS = CPB * K3;
};

// Partial sums of (G^T r)_g^2, 3D: every node is counted once, by its copy of
// highest cell (local index < k, or the last cell along that axis).  A block
// takes whole x-rows of cells (contiguous n K^3 values; cy, cz uniform).
template <typename T, int K>
__global__ void __launch_bounds__(256) k_assembled_norm2_cells(const T* __restrict__ v, int n,
                                                               double* __restrict__ part) {
  constexpr int k = K - 1;
  constexpr int K3 = K * K * K;
  const int nrow = n * n, rowlen = n * K3;
  double acc = 0.0;
  for (int row = blockIdx.x; row < nrow; row += gridDim.x) {
    const int cz = row / n, cy = row - cz * n;
    const T* vr = v + (int64_t)row * rowlen;
    for (int j = threadIdx.x; j < rowlen; j += blockDim.x) {
      const int cx = j / K3, loc = j - cx * K3;
      const int ix = loc % K, iy = (loc / K) % K, iz = loc / (K * K);
      const bool owned = (ix < k || cx == n - 1) && (iy < k || cy == n - 1) && (iz < k || cz == n - 1);
      int kappa;
      const double s = (double)node_sum3<T, K>(vr + j, cx, cy, cz, ix, iy, iz, n, kappa);
      acc += owned ? s * s : 0.0;
    }
  }
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Partial sums of (G^T r)_g^2 over the nodes, one value per block (FP64).
template <typename T, int K, int DIM>
__global__ void __launch_bounds__(256) k_assembled_norm2_partial(const T* __restrict__ v, int n,
                                                                 int64_t n_nodes, double* __restrict__ part) {
  const int N = (K - 1) * n + 1;
  double acc = 0.0;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n_nodes;
       g += (int64_t)gridDim.x * blockDim.x) {
    int gx, gy, gz;
    node_coords<DIM>(g, N, gx, gy, gz);
    const AxisCopies ax = axis_copies<K>(gx, n), ay = axis_copies<K>(gy, n);
    const AxisCopies az = DIM == 3 ? axis_copies<K>(gz, n) : axis_copies<K>(1, n);
    const double s = (double)cascade_sum<T, K, DIM>(v, ax, ay, az, n);
    acc += s * s;
  }
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// out = S_bar r written to every copy (including valence-1 nodes), converted to
// the output precision after the FP64 sum.  G^T out = G^T r, and the entries
// are as small as the assembled residual, so a lower-precision copy keeps
// G^T r accurate even when the raw copies of r are much larger than their sum.
template <typename T, int K, int DIM>
__global__ void __launch_bounds__(256) k_average_convert(const double* __restrict__ r, T* __restrict__ out, int n,
                                                         int64_t n_nodes) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_nodes) return;
  const int N = (K - 1) * n + 1;
  int gx, gy, gz;
  node_coords<DIM>(g, N, gx, gy, gz);
  const AxisCopies ax = axis_copies<K>(gx, n), ay = axis_copies<K>(gy, n);
  const AxisCopies az = DIM == 3 ? axis_copies<K>(gz, n) : axis_copies<K>(1, n);
  const int nz = DIM == 3 ? az.cnt : 1;
  const int kappa = ax.cnt * ay.cnt * nz;
  const T s = (T)(cascade_sum<double, K, DIM>(r, ax, ay, az, n) * (1.0 / kappa));
  for (int sz = 0; sz < nz; ++sz)
    for (int sy = 0; sy < ay.cnt; ++sy)
      for (int sx = 0; sx < ax.cnt; ++sx) out[copy_addr<K, DIM>(ax, ay, az, sx, sy, sz, n)] = s;
}

// k_average_convert, 3D and cell-wise: a thread per cell-wise entry forms its
// node's average and writes its own entry, so the writes are whole cache lines
// (grid: x-groups of whole cells, n, n).
template <typename T, int K>
__global__ void __launch_bounds__(CellBlock<K>::THREADS) k_average_convert3(const double* __restrict__ r,
                                                                           T* __restrict__ out, int n) {
  constexpr int K3 = K * K * K;
  const int cl = threadIdx.x / K3, loc = threadIdx.x - cl * K3;
  const int cx = blockIdx.x * CellBlock<K>::CPB + cl, cy = blockIdx.y, cz = blockIdx.z;
  if (cx >= n) return;
  const int ix = loc % K, iy = (loc / K) % K, iz = loc / (K * K);
  const int64_t own = ((int64_t)cx + (int64_t)n * (cy + (int64_t)n * cz)) * K3 + loc;
  int kappa;
  const double s = node_sum3<double, K>(r + own, cx, cy, cz, ix, iy, iz, n, kappa);
  out[own] = (T)(s * (1.0 / kappa));
}

template <int K>
static fe_status average_convert_typed(const fe_problem* p, int level, const double* r, void* out, fe_dtype dt,
                                       hipStream_t s) {
  const Level& L = level_of(p, level);
  const int64_t N = (int64_t)p->k * L.n + 1;
  const int64_t nn = p->dim == 3 ? N * N * N : N * N;
  const unsigned nb = (unsigned)((nn + 255) / 256);
  ProfScope ps("average_convert", s);
  if (p->dim == 3) {
    const dim3 grid((unsigned)((L.n + CellBlock<K>::CPB - 1) / CellBlock<K>::CPB), (unsigned)L.n, (unsigned)L.n);
    if (dt == FE_F32)
      hipLaunchKernelGGL((k_average_convert3<float, K>), grid, dim3(CellBlock<K>::THREADS), 0, s, r, (float*)out, L.n);
    else
      hipLaunchKernelGGL((k_average_convert3<double, K>), grid, dim3(CellBlock<K>::THREADS), 0, s, r, (double*)out, L.n);
  } else if (dt == FE_F32) {
    hipLaunchKernelGGL((k_average_convert<float, K, 2>), dim3(nb), dim3(256), 0, s, r, (float*)out, L.n, nn);
  } else {
    hipLaunchKernelGGL((k_average_convert<double, K, 2>), dim3(nb), dim3(256), 0, s, r, (double*)out, L.n, nn);
  }
  FE_HIP_CHECK(hipGetLastError());
  return FE_OK;
}

fe_status launch_average_convert(const fe_problem* p, int level, const double* r, void* out, fe_dtype dt,
                                 hipStream_t s) {
  FE_DISPATCH_K(p->K, return average_convert_typed<KK>(p, level, r, out, dt, s));
}

fe_status finish_reduction(const fe_problem* p, int nparts, double* dev_out, hipStream_t s);

static int64_t n_nodes_of(const fe_problem* p, const Level& L) {
  const int64_t N = (int64_t)p->k * L.n + 1;
  return p->dim == 3 ? N * N * N : N * N;
}

template <typename T, int K>
static fe_status dss_typed(const fe_problem* p, const Level& L, T* v, int averaging, hipStream_t s) {
  const int64_t nn = n_nodes_of(p, L);
  const unsigned nb = (unsigned)((nn + 255) / 256);
  ProfScope ps(averaging ? "dss_avg" : "dss_sum", s);
  if (p->dim == 3)
    hipLaunchKernelGGL((k_dss<T, K, 3>), dim3(nb), dim3(256), 0, s, v, L.n, nn, averaging);
  else
    hipLaunchKernelGGL((k_dss<T, K, 2>), dim3(nb), dim3(256), 0, s, v, L.n, nn, averaging);
  FE_HIP_CHECK(hipGetLastError());
  return FE_OK;
}

template <typename T, int K>
static fe_status assemble_typed(const fe_problem* p, const Level& L, const T* v, T* out, hipStream_t s) {
  const int64_t nn = n_nodes_of(p, L);
  const unsigned nb = (unsigned)((nn + 255) / 256);
  if (p->dim == 3)
    hipLaunchKernelGGL((k_assemble<T, K, 3>), dim3(nb), dim3(256), 0, s, v, out, L.n, nn);
  else
    hipLaunchKernelGGL((k_assemble<T, K, 2>), dim3(nb), dim3(256), 0, s, v, out, L.n, nn);
  FE_HIP_CHECK(hipGetLastError());
  return FE_OK;
}

template <typename T, int K>
static fe_status gather_typed(const fe_problem* p, const Level& L, const T* xg, T* xc, hipStream_t s) {
  const unsigned nb = (unsigned)((L.len + 255) / 256);
  if (p->dim == 3)
    hipLaunchKernelGGL((k_gather<T, K, 3>), dim3(nb), dim3(256), 0, s, xg, xc, L.n, L.len);
  else
    hipLaunchKernelGGL((k_gather<T, K, 2>), dim3(nb), dim3(256), 0, s, xg, xc, L.n, L.len);
  FE_HIP_CHECK(hipGetLastError());
  return FE_OK;
}

template <typename T, int K>
static fe_status norm2_typed(const fe_problem* p, const Level& L, const T* v, double* dev_out, hipStream_t s) {
  const int64_t nn = n_nodes_of(p, L);
  double* part = p->red_scratch.as<double>();
  ProfScope ps("assembled_norm2", s);
  int nparts;
  if (p->dim == 3) {
    nparts = (int)std::min<int64_t>(1024, (int64_t)L.n * L.n);
    hipLaunchKernelGGL((k_assembled_norm2_cells<T, K>), dim3(nparts), dim3(256), 0, s, v, L.n, part);
  } else {
    nparts = (int)std::min<int64_t>(1024, (nn + 255) / 256);
    hipLaunchKernelGGL((k_assembled_norm2_partial<T, K, 2>), dim3(nparts), dim3(256), 0, s, v, L.n, nn, part);
  }
  FE_HIP_CHECK(hipGetLastError());
  return finish_reduction(p, nparts, dev_out, s);
}

fe_status launch_dss(const fe_problem* p, int level, void* v, int averaging, fe_dtype dt, hipStream_t s) {
  const Level& L = level_of(p, level);
  if (dt == FE_F64) { FE_DISPATCH_K(p->K, return (dss_typed<double, KK>(p, L, (double*)v, averaging, s))); }
  FE_DISPATCH_K(p->K, return (dss_typed<float, KK>(p, L, (float*)v, averaging, s)));
}

fe_status launch_assemble(const fe_problem* p, const void* yc, void* yg, fe_dtype dt, hipStream_t s) {
  const Level& L = level_of(p, -1);
  if (dt == FE_F64) {
    FE_DISPATCH_K(p->K, return (assemble_typed<double, KK>(p, L, (const double*)yc, (double*)yg, s)));
  }
  FE_DISPATCH_K(p->K, return (assemble_typed<float, KK>(p, L, (const float*)yc, (float*)yg, s)));
}

fe_status launch_gather(const fe_problem* p, const void* xg, void* xc, fe_dtype dt, hipStream_t s) {
  const Level& L = level_of(p, -1);
  if (dt == FE_F64) {
    FE_DISPATCH_K(p->K, return (gather_typed<double, KK>(p, L, (const double*)xg, (double*)xc, s)));
  }
  FE_DISPATCH_K(p->K, return (gather_typed<float, KK>(p, L, (const float*)xg, (float*)xc, s)));
}

fe_status assembled_norm2_async(const fe_problem* p, int level, const void* r, fe_dtype dt, double* dev_out,
                                hipStream_t s) {
  const Level& L = level_of(p, level);
  if (dt == FE_F64) {
    FE_DISPATCH_K(p->K, return (norm2_typed<double, KK>(p, L, (const double*)r, dev_out, s)));
  }
  FE_DISPATCH_K(p->K, return (norm2_typed<float, KK>(p, L, (const float*)r, dev_out, s)));
}

}  // namespace fe
