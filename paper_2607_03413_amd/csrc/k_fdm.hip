// Vertex-patch additive Schwarz inverse by fast diagonalization.
//
// The smoother is admissible in the sense of eq. precond_consistency
// (P = G P_CG G^T, Sec. 2.1): it reads the residual only through its
// assembly and returns a continuous correction.  For each interior vertex v
// the patch unknowns are the m^d nodes (m = 2k-1) strictly inside the 2^d
// cells around v.  With separable patch factors K_a S_a = M_a S_a L_a,
// S_a^T M_a S_a = I (one pair per axis), A_p^{-1} = (S x S x S) (L + L + L)^{-1}
// (S x S x S)^T.
//
// Dispatch (launch_patch_inverse): the 3D Cartesian k = 2, 3 case runs the
// fused single-pass kernel (k_fdm_fused.hip); otherwise two passes:
//  (1) patch solutions: for k >= 4 one wavefront per patch (k_fdm_patch3_wave,
//      k_fdm_wave.hip); for k <= 3 with per-patch factors, k_fdm_patch3 below:
//      one group of m^2 threads per patch sums the copies of one z-pencil of
//      patch nodes (cascade order, straight from the cell-wise residual, so
//      G^T r is never formed), applies S^T along z, y, x (pencils re-oriented
//      through LDS), divides by the eigenvalue sums, applies S along x, y, z;
//      its 3D solutions are written split by cell slot (8 blocks of k^3 per
//      patch), all others patch-major;
//  (2) one thread per cell-wise entry sums the solutions of the (at most 2^d)
//      patches containing its node, in a fixed order that depends only on the
//      node, so every copy receives bit-identical values (continuity).
#include <type_traits>

#include "fe_internal.h"
#include "kernel_common.h"

namespace fe {

template <int K>
struct PatchDims {
  static constexpr int k = K - 1;
  static constexpr int M = 2 * k - 1;
};

// eig layout per patch (or shared): Sx, Sy, Sz (M*M each, row-major S[i*M+j]),
// lx, ly, lz (M each).
template <typename T, int M>
struct EigPtrs {
  const T *Sx, *Sy, *Sz, *lx, *ly, *lz;
};

template <typename T, int M, bool PER_PATCH>
__device__ __forceinline__ EigPtrs<T, M> eig_ptrs(const T* __restrict__ eig, int64_t pid) {
  EigPtrs<T, M> e;
  if (PER_PATCH) {
    const T* base = eig + pid * (3 * M * M + 3 * M);
    e.Sx = base; e.Sy = base + M * M; e.Sz = base + 2 * M * M;
    e.lx = base + 3 * M * M; e.ly = e.lx + M; e.lz = e.ly + M;
  } else {
    e.Sx = e.Sy = e.Sz = eig;
    e.lx = e.ly = e.lz = eig + M * M;
  }
  return e;
}

// Copies of patch-local node offset o (1 <= o <= 2k-1) along one axis: cell
// slot 0 or 1 of the patch and the local index in that cell, lower slot first.
template <int K>
__device__ __forceinline__ AxisCopies patch_axis_copies(int o) {
  constexpr int k = K - 1;
  AxisCopies a;
  if (o < k) { a.cnt = 1; a.c[0] = 0; a.i[0] = o; }
  else if (o > k) { a.cnt = 1; a.c[0] = 1; a.i[0] = o - k; }
  else { a.cnt = 2; a.c[0] = 0; a.i[0] = k; a.c[1] = 1; a.i[1] = 0; }
  if (a.cnt == 1) { a.c[1] = a.c[0]; a.i[1] = a.i[0]; }
  return a;
}

// Thread layout of kernel (1) in 3D.  A patch is handled by M^2 threads, one
// z-pencil each.  When a patch fits in one wavefront (M^2 <= 64), PPW
// patches share a wavefront and never straddle two, so the pencil
// re-orientations through LDS only need wavefront-level ordering; otherwise
// a patch spans several wavefronts and the block synchronizes.
template <int K>
struct PatchLayout {
  static constexpr int k = K - 1;
  static constexpr int M = 2 * k - 1;
  static constexpr int TPP = M * M;
  static constexpr bool WAVE = TPP <= 64;
  static constexpr int PPW = WAVE ? 64 / TPP : 0;
  static constexpr int PPB = WAVE ? 4 * PPW : (256 / TPP > 0 ? 256 / TPP : 1);
  static constexpr int THREADS = WAVE ? 256 : PPB * TPP;
};

template <bool WAVE>
__device__ __forceinline__ void patch_sync() {
  if (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// Kernel (1), 3D.  A block owns PPB consecutive patches of one x-row
// (fixed vy, vz).  Their 2^3 cells form four contiguous runs of PPB+1 cells
// (cy in {vy-1, vy}, cz in {vz-1, vz}), which are first copied to LDS with
// coalesced loads; the patch residuals are then assembled from LDS.
template <typename T, int K, bool PER_PATCH>
__global__ void __launch_bounds__(256) k_fdm_patch3(const T* __restrict__ r, T* __restrict__ W,
                                                    const T* __restrict__ eig, T scale, int n, int segs) {
  using PL = PatchLayout<K>;
  constexpr int k = PL::k, M = PL::M, TPP = PL::TPP, PPB = PL::PPB;
  constexpr bool WAVE = PL::WAVE;
  constexpr int RS = M + 1;
  constexpr int PS = M * RS;
  constexpr int CS = M * PS;
  constexpr int K3 = K * K * K;
  constexpr int NCX = PPB + 1;
  __shared__ T sc[4 * NCX * K3];
  __shared__ T sl[PPB * CS];
  const int tid = threadIdx.x;
  int c, p;
  bool lane_ok = true;
  if (WAVE) {
    const int w = tid >> 6, lane = tid & 63;
    lane_ok = lane < PL::PPW * TPP;
    // surplus lanes shadow pencil 0 of the wave's first patch: identical values, no global store
    c = w * PL::PPW + (lane_ok ? lane / TPP : 0);
    p = lane_ok ? lane % TPP : 0;
  } else {
    c = tid / TPP;
    p = tid - c * TPP;
  }
  const int p0 = p % M, p1 = p / M;
  const int nv = n - 1;
  const int seg = blockIdx.x % segs;
  const int row = blockIdx.x / segs;
  const int vy = 1 + row % nv, vz = 1 + row / nv;
  const int vx0 = 1 + seg * PPB;
  const int npatch = min(PPB, nv - (vx0 - 1));
  const int ncells = npatch + 1;
  // stage the four runs of cells
  for (int q = 0; q < 4; ++q) {
    const int cy = vy - 1 + (q & 1), cz = vz - 1 + (q >> 1);
    const T* src = r + ((int64_t)(vx0 - 1) + (int64_t)n * (cy + (int64_t)n * cz)) * K3;
    T* dst = sc + q * NCX * K3;
    for (int i = tid; i < ncells * K3; i += blockDim.x) dst[i] = src[i];
  }
  // per-patch eigen-data of the block's patches (contiguous in pid) is staged too
  constexpr int EP = 3 * M * M + 3 * M;
  __shared__ T se[PER_PATCH ? PPB * EP : 1];
  const int64_t pid0 = (int64_t)(vx0 - 1) + (int64_t)nv * ((vy - 1) + (int64_t)nv * (vz - 1));
  if (PER_PATCH) {
    const T* src = eig + pid0 * EP;
    for (int i = tid; i < npatch * EP; i += blockDim.x) se[i] = src[i];
  }
  __syncthreads();
  const bool active = c < npatch;
  const int64_t pid = active ? pid0 + c : 0;
  const EigPtrs<T, M> E = PER_PATCH ? eig_ptrs<T, M, true>(se, active ? c : 0) : eig_ptrs<T, M, false>(eig, 0);
  T* ls = sl + c * CS;
  T v[M], t[M];

  // (a) assemble the residual on the z-pencil (a = p0, b = p1) from LDS, cascade order
  if (active) {
    const AxisCopies ax = patch_axis_copies<K>(p0 + 1);
    const AxisCopies ay = patch_axis_copies<K>(p1 + 1);
#pragma unroll
    for (int cz = 0; cz < M; ++cz) {
      const AxisCopies az = patch_axis_copies<K>(cz + 1);
      T zs[2];
      for (int sz = 0; sz < az.cnt; ++sz) {
        T ys[2];
        for (int sy = 0; sy < ay.cnt; ++sy) {
          const T* base = sc + ((az.c[sz] * 2 + ay.c[sy]) * NCX + c) * K3 + K * (ay.i[sy] + K * az.i[sz]);
          T xs = base[ax.c[0] * K3 + ax.i[0]];
          if (ax.cnt == 2) xs += base[ax.c[1] * K3 + ax.i[1]];
          ys[sy] = xs;
        }
        zs[sz] = ay.cnt == 2 ? ys[0] + ys[1] : ys[0];
      }
      v[cz] = az.cnt == 2 ? zs[0] + zs[1] : zs[0];
    }
  } else {
#pragma unroll
    for (int cz = 0; cz < M; ++cz) v[cz] = T(0);
  }
  // (b) S_z^T along z
  pencil_mtv<T, M>(E.Sz, v, t);
#pragma unroll
  for (int cz = 0; cz < M; ++cz) ls[cz * PS + p1 * RS + p0] = t[cz];
  patch_sync<WAVE>();
  // (c) S_y^T along y: thread (a = p0, cz = p1)
#pragma unroll
  for (int j = 0; j < M; ++j) v[j] = ls[p1 * PS + j * RS + p0];
  pencil_mtv<T, M>(E.Sy, v, t);
  patch_sync<WAVE>();
#pragma unroll
  for (int b = 0; b < M; ++b) ls[p1 * PS + b * RS + p0] = t[b];
  patch_sync<WAVE>();
  // (d) x-pencil (b = p0, cz = p1): S_x^T, divide, S_x
#pragma unroll
  for (int j = 0; j < M; ++j) v[j] = ls[p1 * PS + p0 * RS + j];
  pencil_mtv<T, M>(E.Sx, v, t);
  {
    const T lyz = E.ly[p0] + E.lz[p1];
#pragma unroll
    for (int a = 0; a < M; ++a) t[a] = t[a] * scale / (E.lx[a] + lyz);
  }
  pencil_mv<T, M>(E.Sx, t, v);
  patch_sync<WAVE>();
#pragma unroll
  for (int a = 0; a < M; ++a) ls[p1 * PS + p0 * RS + a] = v[a];
  patch_sync<WAVE>();
  // (e) S_y along y: thread (a = p0, cz = p1)
#pragma unroll
  for (int j = 0; j < M; ++j) v[j] = ls[p1 * PS + j * RS + p0];
  pencil_mv<T, M>(E.Sy, v, t);
  patch_sync<WAVE>();
#pragma unroll
  for (int b = 0; b < M; ++b) ls[p1 * PS + b * RS + p0] = t[b];
  patch_sync<WAVE>();
  // (f) S_z along z: thread (a = p0, b = p1); write the patch solution
#pragma unroll
  for (int j = 0; j < M; ++j) v[j] = ls[j * PS + p1 * RS + p0];
  pencil_mv<T, M>(E.Sz, v, t);
  // Write the solution split by cell slot: slot s = sx + 2 sy + 4 sz of the
  // patch holds the k^3 patch nodes inside that cell (offset o <= k in slot 0
  // at j = o - 1, o >= k in slot 1 at j = o - k; the node o = k is in both).
  // Each patch fills 8 k^3 contiguous values; each cell later reads one
  // contiguous k^3 block per corner.
  if (active && lane_ok) {
    constexpr int k3 = k * k * k;
    T* wp = W + pid * (8 * k3);
    const int ox = p0 + 1, oy = p1 + 1;
    for (int sy = 0; sy < 2; ++sy) {
      const int jy = sy ? oy - k : oy - 1;
      if (jy < 0 || jy >= k) continue;
      for (int sx = 0; sx < 2; ++sx) {
        const int jx = sx ? ox - k : ox - 1;
        if (jx < 0 || jx >= k) continue;
#pragma unroll
        for (int cz = 0; cz < M; ++cz) {
          const int oz = cz + 1;
          if (oz <= k) wp[(sx + 2 * sy) * k3 + jx + k * (jy + k * (oz - 1))] = t[cz];
          if (oz >= k) wp[(sx + 2 * sy + 4) * k3 + jx + k * (jy + k * (oz - k))] = t[cz];
        }
      }
    }
  }
}

// Kernel (2), 3D: one thread per cell-wise entry sums the contributions of the
// patches at the cell's (up to 8) corners from the slot-split buffer, in the
// order bz, by, bx ascending (= patch vertices ascending, the same for every
// copy of a node, so copies come out bit-identical), and writes its own entry:
// consecutive threads write consecutive addresses, whole cache lines.  A block
// holds SumSlots<K>::CPB consecutive cells of an x-row (grid: x-groups, n, n),
// so no thread divides by n.  No load is branched around (a branch per load
// made each one wait for its data before the next was issued): an absent
// patch is read at W[0] and added times 0, an exact 0.
// Optional Chebyshev step fused into the summing pass (CH != 0), in place of
// storing v = P r: w = a v (CH 1, 2) or w = a v + c w (CH 3), then e = w (CH 1)
// or e += w (CH 2, 3), the same arithmetic as the separate update kernel.  It
// saves writing v and reading it back, two full vectors per smoothing step.
template <typename T>
struct ChebArgs {
  T a, c;
  T* w;
  T* e;
};

template <int K>
struct SumSlots {
  static constexpr int K3 = K * K * K;
  static constexpr int CPB = K3 >= 64 ? 1 : 64 / K3;   // cells per block
  static constexpr int THREADS = CPB * K3;
};

template <typename T, int CH>
__device__ __forceinline__ void cheb_store(const ChebArgs<T>& ch, T* z, int64_t i, T v, T wo, T eo) {
  if (CH == 0) {
    z[i] = v;
  } else {
    const T wn = CH == 3 ? fma(ch.a, v, ch.c * wo) : ch.a * v;
    ch.w[i] = wn;
    ch.e[i] = CH == 1 ? wn : eo + wn;
  }
}

template <typename T, int K, int CH>
__global__ void __launch_bounds__(SumSlots<K>::THREADS) k_fdm_sum_slots3(const T* __restrict__ W, T* __restrict__ z, int n,
                                                                         ChebArgs<T> ch) {
  constexpr int k = K - 1;
  constexpr int k3 = k * k * k;
  constexpr int K3 = K * K * K;
  const int cl = threadIdx.x / K3, loc = threadIdx.x - cl * K3;
  const int cx = blockIdx.x * SumSlots<K>::CPB + cl, cy = blockIdx.y, cz = blockIdx.z;
  if (cx >= n) return;
  const int ix = loc % K, iy = (loc / K) % K, iz = loc / (K * K);
  const int nv = n - 1;
  const int64_t oi = ((int64_t)cx + (int64_t)n * (cy + (int64_t)n * cz)) * K3 + loc;
  if (nv < 1) {   // no patch at all (and possibly no scratch)
    cheb_store<T, CH>(ch, z, oi, T(0), CH == 3 ? ch.w[oi] : T(0), CH >= 2 ? ch.e[oi] : T(0));
    return;
  }
  // the Chebyshev operands are fetched ahead of the patch values (after the
  // branch above: used there, they were waited for before the patch loads)
  const T wo = CH == 3 ? ch.w[oi] : T(0);
  const T eo = CH >= 2 ? ch.e[oi] : T(0);
  T s = T(0);
#pragma unroll
  for (int bz = 0; bz < 2; ++bz) {
    const int vz = cz + bz, jz = iz - bz;
    const bool okz = vz >= 1 && vz <= nv && jz >= 0 && jz < k;
#pragma unroll
    for (int by = 0; by < 2; ++by) {
      const int vy = cy + by, jy = iy - by;
      const bool oky = vy >= 1 && vy <= nv && jy >= 0 && jy < k;
#pragma unroll
      for (int bx = 0; bx < 2; ++bx) {
        const int vx = cx + bx, jx = ix - bx;
        const bool use = okz && oky && vx >= 1 && vx <= nv && jx >= 0 && jx < k;
        const int64_t pid = (vx - 1) + (int64_t)nv * ((vy - 1) + (int64_t)nv * (vz - 1));
        const int slot = (1 - bx) + 2 * (1 - by) + 4 * (1 - bz);
        const int64_t idx = (pid * (8 * k3) + slot * k3 + jx + k * (jy + k * jz)) & -(int64_t)use;
        s = fma(W[idx], use ? T(1) : T(0), s);
      }
    }
  }
  cheb_store<T, CH>(ch, z, oi, s, wo, eo);
}

template <typename T, int K, bool PER_PATCH>
__global__ void __launch_bounds__(256) k_fdm_patch2(const T* __restrict__ r, T* __restrict__ W,
                                                    const T* __restrict__ eig, T scale, int n,
                                                    int64_t n_patches) {
  constexpr int k = K - 1;
  constexpr int M = 2 * k - 1;
  constexpr int TPP = M;
  constexpr int PPB = 256 / TPP;
  constexpr int RS = M + 1;
  constexpr int CS = M * RS;
  __shared__ T sl[PPB * CS];
  const int tid = threadIdx.x;
  const int c = tid / TPP;
  const int p = tid - c * TPP;
  const int64_t pid = (int64_t)blockIdx.x * PPB + c;
  const bool active = pid < n_patches;
  const int nv = n - 1;
  int vx = 1, vy = 1;
  if (active) { vx = 1 + (int)(pid % nv); vy = 1 + (int)(pid / nv); }
  const EigPtrs<T, M> E = eig_ptrs<T, M, PER_PATCH>(eig, active ? pid : 0);
  T* ls = sl + c * CS;
  T v[M], t[M];
  // y-pencil at a = p
  if (active) {
    const AxisCopies ax = axis_copies<K>(k * (vx - 1) + p + 1, n);
    const AxisCopies az = ax;
#pragma unroll
    for (int b = 0; b < M; ++b) {
      const AxisCopies ay = axis_copies<K>(k * (vy - 1) + b + 1, n);
      v[b] = cascade_sum<T, K, 2>(r, ax, ay, az, n);
    }
  } else {
#pragma unroll
    for (int b = 0; b < M; ++b) v[b] = T(0);
  }
  pencil_mtv<T, M>(E.Sy, v, t);
#pragma unroll
  for (int b = 0; b < M; ++b) ls[b * RS + p] = t[b];
  __syncthreads();
  // x-pencil at b = p
#pragma unroll
  for (int j = 0; j < M; ++j) v[j] = ls[p * RS + j];
  pencil_mtv<T, M>(E.Sx, v, t);
  {
    const T ly = E.ly[p];
#pragma unroll
    for (int a = 0; a < M; ++a) t[a] = t[a] * scale / (E.lx[a] + ly);
  }
  pencil_mv<T, M>(E.Sx, t, v);
  __syncthreads();
#pragma unroll
  for (int a = 0; a < M; ++a) ls[p * RS + a] = v[a];
  __syncthreads();
#pragma unroll
  for (int j = 0; j < M; ++j) v[j] = ls[j * RS + p];
  pencil_mv<T, M>(E.Sy, v, t);
  if (active) {
    T* w = W + pid * (M * M) + p;
#pragma unroll
    for (int b = 0; b < M; ++b) w[b * M] = t[b];
  }
}

// Patches containing node coordinate g along one axis: vertex v with
// k(v-1) < g < k(v+1) and 1 <= v <= n-1; offset o = g - k(v-1) - 1.
struct AxisPatches {
  int cnt;
  int v[2];
  int o[2];
};

template <int K>
__device__ __forceinline__ AxisPatches axis_patches(int g, int n) {
  constexpr int k = K - 1;
  AxisPatches a;
  a.cnt = 0;
  const int q = g / k, r = g - q * k;
  if (r == 0) {
    if (q >= 1 && q <= n - 1) { a.v[0] = q; a.o[0] = k - 1; a.cnt = 1; }
  } else {
    if (q >= 1) { a.v[a.cnt] = q; a.o[a.cnt] = k + r - 1; ++a.cnt; }
    if (q + 1 <= n - 1) { a.v[a.cnt] = q + 1; a.o[a.cnt] = r - 1; ++a.cnt; }
  }
  return a;
}

// Kernel (2), 2D: one thread per cell-wise entry sums the patch-major
// solutions of the (at most 4) patches containing its node, in ascending
// vertex order (y, then x), so all copies receive identical values.
template <typename T, int K>
__global__ void __launch_bounds__(256) k_fdm_sum2(const T* __restrict__ W, T* __restrict__ z, int n,
                                                  int64_t len) {
  constexpr int k = K - 1;
  constexpr int M = 2 * k - 1;
  constexpr int NL = K * K;
  constexpr int MP = M * M;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  const int64_t cell = e / NL;
  const int loc = (int)(e - cell * NL);
  const int ix = loc % K, iy = loc / K;
  const int cx = (int)(cell % n), cy = (int)(cell / n);
  const int nv = n - 1;
  const AxisPatches px = axis_patches<K>(k * cx + ix, n);
  const AxisPatches py = axis_patches<K>(k * cy + iy, n);
  T s = T(0);
  for (int b = 0; b < py.cnt; ++b)
    for (int c = 0; c < px.cnt; ++c) {
      const int64_t pid = (px.v[c] - 1) + (int64_t)nv * (py.v[b] - 1);
      s += W[pid * MP + px.o[c] + M * py.o[b]];
    }
  z[e] = s;
}

// Kernel (2), 3D, patch-major solutions (k >= 4): one block per cell, one
// thread per cell-wise entry, a fixed 2 x 2 x 2 set of candidate patches per
// entry so that lanes do not diverge.  Along each axis the node g = k c + i lies strictly inside
// patch c (offset k-1+i) when i < k and inside patch c+1 (offset i-1) when
// i > 0; candidates outside 1..n-1 or not containing the node contribute 0.
// The sum runs over (z, y, x) patch candidates in ascending vertex order,
// which depends only on the node: all copies receive identical values.
// (FP32: at most 4 wavefronts per SIMD asked for, so that the scheduler keeps
// every load in flight; aiming at more, it waited for each z node's loads
// before issuing the next once the Chebyshev operands were live as well)
template <typename T, int K, int CH>
__global__ void __launch_bounds__((K * K + 63) / 64 * 64)
    __attribute__((amdgpu_waves_per_eu(1, sizeof(T) == 4 ? 4 : 8))) k_fdm_sum_pm3(const T* __restrict__ W, T* __restrict__ z, int n,
                                                                       ChebArgs<T> ch) {
  constexpr int k = K - 1;
  constexpr int M = 2 * k - 1;
  constexpr int MP = M * M * M;
  constexpr int NL = K * K * K;
  // one block per cell, grid (n, n, n); a lane owns the z-line (ix, iy) of
  // the cell.  The cell and its candidate patches are block-uniform, and so
  // is, per z node, which of the two patch layers along z covers it.
  const int cx = blockIdx.x, cy = blockIdx.y, cz = blockIdx.z;
  const int loc = threadIdx.x;
  const bool act = loc < K * K;
  const int ix = loc % K, iy = loc / K;
  const int nv = n - 1;
  // candidate c = 0: vertex = cell (offset k-1+i), c = 1: vertex = cell+1 (offset i-1)
  const int c2[2] = {cx, cy}, i2[2] = {ix, iy};
  int off[2][2];
  bool ok[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    off[a][0] = k - 1 + i2[a];
    ok[a][0] = act && i2[a] < k && c2[a] >= 1;
    off[a][1] = i2[a] - 1;
    ok[a][1] = act && i2[a] > 0 && c2[a] + 1 <= nv;
  }
  // patch (cx-1, cy-1, cz-1) and the strides to its neighbours along y and z
  const int64_t p000 = (int64_t)(cx - 1) + (int64_t)nv * ((cy - 1) + (int64_t)nv * (cz - 1));
  const int64_t sy = nv, sz = (int64_t)nv * nv;
  // entry (ix, iy, iz) of the cell sits at oc + iz K^2 (lanes past K^2 use entry 0)
  const int64_t oc = ((int64_t)cx + (int64_t)n * (cy + (int64_t)n * cz)) * NL + (act ? loc : 0);
  // the Chebyshev operands are fetched ahead of the patch values
  T wo[K], eo[K];
#pragma unroll
  for (int iz = 0; iz < K; ++iz) {
    wo[iz] = CH == 3 ? ch.w[oc + iz * K * K] : T(0);
    eo[iz] = CH >= 2 ? ch.e[oc + iz * K * K] : T(0);
  }
  if (nv < 1) {   // no patch at all (and possibly no scratch)
#pragma unroll
    for (int iz = 0; iz < K; ++iz)
      if (act) cheb_store<T, CH>(ch, z, oc + iz * K * K, T(0), wo[iz], eo[iz]);
    return;
  }
  // Patches in ascending vertex order (z, then y, then x), as every copy of a
  // node sums them.  No load is branched around (a branch per load made each
  // one wait for its data before the next was issued): a lane without that
  // patch reads W[0] and adds it times 0, an exact 0 that leaves the sum
  // unchanged, and the stores come after all loads, so that all of them can
  // be in flight.
  // (the z-layer tests are uniform; computed from a vector copy of cz they
  // become selects rather than branches that would split the loads into groups)
  int czv = cz;
  asm volatile("" : "+v"(czv));
  const bool zlo = czv >= 1, zhi = czv + 1 <= nv;
  T acc[K];
#pragma unroll
  for (int iz = 0; iz < K; ++iz) {
    T s = T(0);
#pragma unroll
    for (int bz = 0; bz < 2; ++bz) {
      const bool okz = bz == 0 ? (iz < k && zlo) : (iz > 0 && zhi);
      const int oz = bz == 0 ? k - 1 + iz : iz - 1;
#pragma unroll
      for (int by = 0; by < 2; ++by)
#pragma unroll
        for (int bx = 0; bx < 2; ++bx) {
          const bool use = okz && ok[1][by] && ok[0][bx];
          const int o = off[0][bx] + M * (off[1][by] + M * oz);
          const int64_t idx = ((p000 + bx + by * sy + bz * sz) * MP + o) & -(int64_t)use;
          s = fma(W[idx], use ? T(1) : T(0), s);
        }
    }
    acc[iz] = s;
  }
  if (act) {
#pragma unroll
    for (int iz = 0; iz < K; ++iz) cheb_store<T, CH>(ch, z, oc + iz * K * K, acc[iz], wo[iz], eo[iz]);
  }
}

bool fused_patch_supported(const fe_problem* p, bool per_patch);
bool patch_wave_supported(const fe_problem* p, bool per_patch);
fe_status launch_patch_wave(const fe_problem* p, const Level& L, const void* r, void* W, const void* eig,
                            bool per_patch, double scale, fe_dtype dt, hipStream_t s);
fe_status launch_patch_fused(const fe_problem* p, int level, const void* r, void* z, fe_dtype dt, hipStream_t s);

size_t patch_scratch_bytes(const fe_problem* p, int level, fe_dtype dt) {
  const Level& L = level_of(p, level);
  const int64_t nv = L.n - 1;
  const int64_t M = 2 * p->k - 1;
  const int64_t k = p->k;
  const int64_t np = p->dim == 3 ? nv * nv * nv : nv * nv;
  // 3D: slot-split layout, 8 k^3 per patch (k >= 4: patch-major M^3 <= 8 k^3); 2D: patch-major, M^2 per patch
  const int64_t mp = p->dim == 3 ? 8 * k * k * k : M * M;
  return (size_t)(np * mp) * (dt == FE_F64 ? 8 : 4);
}

template <typename T, int K, int CH>
static fe_status launch_sum3(const fe_problem* p, const Level& L, const T* W, T* z, bool per_patch, const ChebArgs<T>& ch,
                             hipStream_t s) {
  ProfScope ps2("fdm_sum", s);
  if (patch_wave_supported(p, per_patch))   // patch-major solutions
    hipLaunchKernelGGL((k_fdm_sum_pm3<T, K, CH>), dim3((unsigned)L.n, (unsigned)L.n, (unsigned)L.n), dim3((K * K + 63) / 64 * 64), 0,
                       s, W, z, L.n, ch);
  else                                      // slot-split solutions
    hipLaunchKernelGGL((k_fdm_sum_slots3<T, K, CH>),
                       dim3((unsigned)((L.n + SumSlots<K>::CPB - 1) / SumSlots<K>::CPB), (unsigned)L.n, (unsigned)L.n),
                       dim3(SumSlots<K>::THREADS), 0, s, W, z, L.n, ch);
  FE_HIP_CHECK(hipGetLastError());
  return FE_OK;
}

// ch_mode 0: z = P r; 1..3: the fused Chebyshev step of ChebArgs (3D only)
template <typename T, int K>
static fe_status patch_typed(const fe_problem* p, const Level& L, const T* r, T* z, T* W, const T* eig,
                             bool per_patch, T scale, int ch_mode, const ChebArgs<T>& ch, hipStream_t s) {
  constexpr int M = 2 * (K - 1) - 1;
  const int64_t nv = L.n - 1;
  if (p->dim == 3) {
    const int64_t np = nv * nv * nv;
    if (np > 0 && patch_wave_supported(p, per_patch)) {
      FE_CHECK(launch_patch_wave(p, L, r, W, eig, per_patch, (double)scale, std::is_same<T, double>::value ? FE_F64 : FE_F32, s));
    } else if (np > 0) {
      constexpr int PPB = PatchLayout<K>::PPB;
      constexpr int THREADS = PatchLayout<K>::THREADS;
      const int segs = (int)((nv + PPB - 1) / PPB);
      const unsigned nb = (unsigned)(segs * nv * nv);
      ProfScope ps("fdm_patch", s);
      if (per_patch)
        hipLaunchKernelGGL((k_fdm_patch3<T, K, true>), dim3(nb), dim3(THREADS), 0, s, r, W, eig, scale, L.n, segs);
      else
        hipLaunchKernelGGL((k_fdm_patch3<T, K, false>), dim3(nb), dim3(THREADS), 0, s, r, W, eig, scale, L.n, segs);
      FE_HIP_CHECK(hipGetLastError());
    }
    switch (ch_mode) {
      case 1: return launch_sum3<T, K, 1>(p, L, W, z, per_patch, ch, s);
      case 2: return launch_sum3<T, K, 2>(p, L, W, z, per_patch, ch, s);
      case 3: return launch_sum3<T, K, 3>(p, L, W, z, per_patch, ch, s);
      default: return launch_sum3<T, K, 0>(p, L, W, z, per_patch, ch, s);
    }
  } else {
    const int64_t np = nv * nv;
    if (np > 0) {
      constexpr int PPB = 256 / M;
      const unsigned nb = (unsigned)((np + PPB - 1) / PPB);
      ProfScope ps("fdm_patch", s);
      if (per_patch)
        hipLaunchKernelGGL((k_fdm_patch2<T, K, true>), dim3(nb), dim3(PPB * M), 0, s, r, W, eig, scale, L.n, np);
      else
        hipLaunchKernelGGL((k_fdm_patch2<T, K, false>), dim3(nb), dim3(PPB * M), 0, s, r, W, eig, scale, L.n, np);
      FE_HIP_CHECK(hipGetLastError());
    }
    ProfScope ps2("fdm_sum", s);
    hipLaunchKernelGGL((k_fdm_sum2<T, K>), dim3((unsigned)((L.len + 255) / 256)), dim3(256), 0, s, W, z, L.n,
                       L.len);
  }
  FE_HIP_CHECK(hipGetLastError());
  return FE_OK;
}

// Chebyshev mode of the summing pass for w = a v + c w with e = w (e_zero) or
// e += w; 0 where it runs as a separate update (c != 0 with e = w does not occur
// in a smoothing sweep).
template <typename T>
static int cheb_mode(T c, int e_zero) {
  if (c == T(0)) return e_zero ? 1 : 2;
  return e_zero ? 0 : 3;
}

static fe_status patch_dispatch(const fe_problem* p, int level, const void* r, void* z, void* scratch, fe_dtype dt,
                                int factors, bool cheb, double a, double c, void* w, void* e, int e_zero,
                                hipStream_t s) {
  const Level& L = level_of(p, level);
  const bool per_patch = factors != 0;
  const double scale = per_patch ? 1.0 : std::pow(L.h, 2 - p->dim);
  const int li = level < 0 ? (int)p->levels.size() - 1 : level;
  const void* eig;
  if (per_patch) {
    const Level& LL = p->levels[li];
    if (!LL.patch_eig_ready[factors]) return fail(FE_EINVAL, "patch factors not available for this mode");
    eig = dt == FE_F64 ? LL.patch_eig64[factors].p : LL.patch_eig32[factors].p;
  } else {
    eig = dt == FE_F64 ? (const void*)(p->coef64.as<double>() + p->co.off_S)
                       : (const void*)(p->coef32.as<float>() + p->co.off_S);
  }
  if (dt == FE_F64) {
    const ChebArgs<double> ch{a, c, (double*)w, (double*)e};
    const int mode = cheb ? cheb_mode(ch.c, e_zero) : 0;
    FE_DISPATCH_K(p->K, return (patch_typed<double, KK>(p, L, (const double*)r, (double*)z, (double*)scratch,
                                                        (const double*)eig, per_patch, scale, mode, ch, s)));
  }
  const ChebArgs<float> ch{(float)a, (float)c, (float*)w, (float*)e};
  const int mode = cheb ? cheb_mode(ch.c, e_zero) : 0;
  FE_DISPATCH_K(p->K, return (patch_typed<float, KK>(p, L, (const float*)r, (float*)z, (float*)scratch,
                                                     (const float*)eig, per_patch, (float)scale, mode, ch, s)));
}

fe_status launch_patch_inverse(const fe_problem* p, int level, const void* r, void* z, void* scratch,
                               fe_dtype dt, int factors, hipStream_t s) {
  if (fused_patch_supported(p, factors != 0)) return launch_patch_fused(p, level, r, z, dt, s);
  return patch_dispatch(p, level, r, z, scratch, dt, factors, false, 0.0, 0.0, nullptr, nullptr, 0, s);
}

fe_status launch_patch_cheb(const fe_problem* p, int level, const void* r, void* v, void* scratch, fe_dtype dt,
                            int factors, double a, double c, void* w, void* e, int e_zero, hipStream_t s) {
  const bool c_zero = dt == FE_F64 ? c == 0.0 : (float)c == 0.0f;
  const bool fusable = p->dim == 3 && !fused_patch_supported(p, factors != 0) && (c_zero || !e_zero);
  if (!fusable) {
    FE_CHECK(launch_patch_inverse(p, level, r, v, scratch, dt, factors, s));
    return launch_cheb_update(level_of(p, level).len, a, v, c, w, e, e_zero, dt, s);
  }
  return patch_dispatch(p, level, r, nullptr, scratch, dt, factors, true, a, c, w, e, e_zero, s);
}

}  // namespace fe
