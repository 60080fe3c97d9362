// Vertex-patch fast-diagonalization inverse on the matrix cores (k >= 5).
//
// For high degree the six 1D contractions of a patch, (S^T x S^T x S^T), the
// eigenvalue division and (S x S x S), are dense m x m products with
// m = 2k-1 (13 for k = 7) applied to all m^2 pencils of the patch: exactly
// the batched small GEMMs the MFMA units execute.  Each contraction is
// written as OUT[16 x R] = A[16 x 16] * IN[16 x R] (m padded to 16, R = m^2
// padded to a multiple of 16) and issued as 16x16x4 MFMAs: A holds four
// 16 x 4 chunks of S or S^T in registers (the same for every tile), the
// B operand is read from the patch tensor in LDS, and each output tile is
// written straight into the layout the next contraction reads.  A block of
// four wavefronts owns one patch; the wavefronts split the R/16 tiles.
//
// Layouts of the patch tensor in LDS (row = contraction axis, rest = the
// other two axes, lower axis fastest, row stride RP):
//   LZ: row z, rest x + m y;  LY: row y, rest x + m z;  LX: row x, rest y + m z.
// Sequence: gather (LZ) -> S_z^T -> LY -> S_y^T -> LX -> S_x^T, divide -> LX
//           -> S_x -> LY -> S_y -> LZ -> S_z -> LZ -> slot-split output.
#include "fe_internal.h"
#include "kernel_common.h"

namespace fe {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
template <> struct Mfma<float> {
  typedef f32x4 acc;
  static __device__ __forceinline__ acc step(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // output row i of register r in lane l
  static __device__ __forceinline__ int row(int l, int r) { return 4 * (l >> 4) + r; }
};
template <> struct Mfma<double> {
  typedef f64x4 acc;
  static __device__ __forceinline__ acc step(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int r) { return (l >> 4) + 4 * r; }
};

template <int K>
struct MfmaPatch {
  static constexpr int k = K - 1;
  static constexpr int M = 2 * k - 1;       // <= 15
  static constexpr int R = M * M;
  static constexpr int TILES = (R + 15) / 16;
  static constexpr int RP = TILES * 16 + 1;  // odd row stride
  static constexpr int TS = 16 * RP;         // one tensor buffer (16 rows)
  static constexpr int K3 = K * K * K;
};

// where an output element (row a2 of the contraction, rest index q) goes next
enum { TO_LY_FROM_LZ = 0, TO_LX_FROM_LY = 1, TO_LX_SAME = 2, TO_LY_FROM_LX = 3, TO_LZ_FROM_LY = 4, TO_LZ_SAME = 5 };

template <int M, int RP, int MODE>
__device__ __forceinline__ int dest_index(int a2, int q) {
  // q decodes as (u + M v) of the input layout's rest
  const int u = q % M, v = q / M;
  switch (MODE) {
    case TO_LY_FROM_LZ:  // in LZ: rest = x + M y, out row z'  -> LY: row y, rest x + M z'
      return v * RP + u + M * a2;
    case TO_LX_FROM_LY:  // in LY: rest = x + M z, out row y'  -> LX: row x, rest y' + M z
      return u * RP + a2 + M * v;
    case TO_LX_SAME:     // in LX: rest = y + M z, out row x'  -> LX: row x', rest y + M z
      return a2 * RP + q;
    case TO_LY_FROM_LX:  // in LX: rest = y + M z, out row x   -> LY: row y, rest x + M z
      return u * RP + a2 + M * v;
    case TO_LZ_FROM_LY:  // in LY: rest = x + M z, out row y   -> LZ: row z, rest x + M y
      return v * RP + u + M * a2;
    default:             // TO_LZ_SAME: in LZ: rest = x + M y, out row z -> LZ
      return a2 * RP + q;
  }
}

// One contraction: out = Amat * in, Amat given as 4 register chunks (lane l holds
// Amat[l % 16][4 c + l / 16] in a[c]).  The wavefront's tiles (t = wave, wave + 4,
// ...) are issued back to back so that their MFMA chains overlap.  Optional
// eigenvalue scaling (MODE TO_LX_SAME): out[x'][y + M z] *= inv[x' + M (y + M z)].
template <typename T, int M, int RP, int TILES, int MODE>
__device__ __forceinline__ void contract(const T* __restrict__ in, T* __restrict__ out, const T (&a)[4], int wave,
                                         int lane, const T* __restrict__ inv) {
  typedef typename Mfma<T>::acc acc;
  constexpr int R = M * M;
  constexpr int TPW = (TILES + 3) / 4;   // tiles per wavefront (at most)
  const int j = lane & 15, kk = lane >> 4;
  acc d[TPW];
#pragma unroll
  for (int i = 0; i < TPW; ++i) d[i] = acc{0, 0, 0, 0};
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int t = wave + 4 * i;
      if (t < TILES) d[i] = Mfma<T>::step(a[c], in[(4 * c + kk) * RP + 16 * t + j], d[i]);
    }
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    const int col = 16 * (wave + 4 * i) + j;
    if (wave + 4 * i < TILES && col < R) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a2 = Mfma<T>::row(lane, r);
        if (a2 < M) {
          T v = d[i][r];
          if (MODE == TO_LX_SAME) v *= inv[a2 + M * col];
          out[dest_index<M, RP, MODE>(a2, col)] = v;
        }
      }
    }
  }
}

// Copies of patch-local node a (0 <= a <= 2k-2) along one axis: cell slot
// (0 = lower cell, 1 = upper cell) and local index, lower slot first.
template <int K>
__device__ __forceinline__ AxisCopies mfma_axis_copies(int a) {
  constexpr int k = K - 1;
  AxisCopies c;
  const int o = a + 1;
  if (o < k) { c.cnt = 1; c.c[0] = 0; c.i[0] = o; }
  else if (o > k) { c.cnt = 1; c.c[0] = 1; c.i[0] = o - k; }
  else { c.cnt = 2; c.c[0] = 0; c.i[0] = k; c.c[1] = 1; c.i[1] = 0; }
  if (c.cnt == 1) { c.c[1] = c.c[0]; c.i[1] = c.i[0]; }
  return c;
}

template <typename T, int K, bool PER_PATCH>
__global__ void __launch_bounds__(256) k_fdm_patch3_mfma(const T* __restrict__ r, T* __restrict__ W,
                                                         const T* __restrict__ eig, T scale, int n) {
  using P = MfmaPatch<K>;
  constexpr int k = P::k, M = P::M, RP = P::RP, TS = P::TS, TILES = P::TILES, K3 = P::K3;
  constexpr int CELLS = 8 * K3;
  constexpr int BUF0 = CELLS > TS ? CELLS : TS;
  constexpr int M3 = M * M * M;
  __shared__ T lds[BUF0 + TS + M3];
  T* b0 = lds;              // staged cells, then tensor buffer 0
  T* b1 = lds + BUF0;       // tensor buffer 1
  T* inv = b1 + TS;         // scale / (lx + ly + lz), index x + M (y + M z)
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int nv = n - 1;
  const int64_t pid = blockIdx.x;
  const int vx = 1 + (int)(pid % nv), vy = 1 + (int)((pid / nv) % nv), vz = 1 + (int)(pid / ((int64_t)nv * nv));
  // eigen-data: S_d (M x M, S[i*M + j]) and lambda_d
  const T* Sx;
  const T* Sy;
  const T* Sz;
  const T* lsrc[3];
  if (PER_PATCH) {
    const T* base = eig + pid * (3 * M * M + 3 * M);
    Sx = base; Sy = base + M * M; Sz = base + 2 * M * M;
    lsrc[0] = base + 3 * M * M; lsrc[1] = lsrc[0] + M; lsrc[2] = lsrc[1] + M;
  } else {
    Sx = Sy = Sz = eig;
    lsrc[0] = lsrc[1] = lsrc[2] = eig + M * M;
  }
  // stage the 8 cells of the patch: slot s = sx + 2 sy + 4 sz, contiguous K^3 each
  {
    const int64_t c0 = (vx - 1) + (int64_t)n * ((vy - 1) + (int64_t)n * (vz - 1));
    const int64_t sy = n, sz = (int64_t)n * n;
#pragma unroll 4
    for (int e = tid; e < CELLS; e += 256) {
      const int s = e / K3, loc = e - s * K3;
      const int64_t cell = c0 + (s & 1) + sy * ((s >> 1) & 1) + sz * (s >> 2);
      b0[e] = r[cell * K3 + loc];
    }
  }
  // inverse eigenvalue sums
  for (int e = tid; e < M3; e += 256) {
    const int x = e % M, y = (e / M) % M, z = e / (M * M);
    inv[e] = scale / (lsrc[0][x] + lsrc[1][y] + lsrc[2][z]);
  }
  // zero the padding rows M..15 of buffer 1 (buffer 0's are zeroed after the gather)
  for (int e = tid; e < (16 - M) * RP; e += 256) b1[M * RP + e] = T(0);
  __syncthreads();
  // assemble the patch residual into LZ of buffer 1: thread = (x, y) pencil,
  // copies summed in cascade order (x pairs, then y, then z)
  if (tid < M * M) {
    const int x = tid % M, y = tid / M;
    const AxisCopies cx = mfma_axis_copies<K>(x), cy = mfma_axis_copies<K>(y);
#pragma unroll
    for (int z = 0; z < M; ++z) {
      const AxisCopies cz = mfma_axis_copies<K>(z);
      T zs = T(0);
#pragma unroll
      for (int sz = 0; sz < 2; ++sz) {
        if (sz >= cz.cnt) break;
        T ys = T(0);
#pragma unroll
        for (int sy = 0; sy < 2; ++sy) {
          if (sy >= cy.cnt) break;
          const T* cb = b0 + (4 * cz.c[sz] + 2 * cy.c[sy]) * K3 + K * (cy.i[sy] + K * cz.i[sz]);
          T xs = cb[cx.c[0] * K3 + cx.i[0]];
          if (cx.cnt == 2) xs += cb[cx.c[1] * K3 + cx.i[1]];
          ys = sy == 0 ? xs : ys + xs;
        }
        zs = sz == 0 ? ys : zs + ys;
      }
      b1[z * RP + x + M * y] = zs;
    }
  }
  __syncthreads();
  for (int e = tid; e < (16 - M) * RP; e += 256) b0[M * RP + e] = T(0);
  // A operands: forward uses S^T (Amat[i][a] = S[a][i]), backward S (Amat[i][a] = S[i][a])
  T fx[4], fy[4], fz[4], gx[4], gy[4], gz[4];
  {
    const int i = lane & 15, kk = lane >> 4;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int a = 4 * c + kk;
      const bool ok = i < M && a < M;
      fx[c] = ok ? Sx[a * M + i] : T(0);
      fy[c] = ok ? Sy[a * M + i] : T(0);
      fz[c] = ok ? Sz[a * M + i] : T(0);
      gx[c] = ok ? Sx[i * M + a] : T(0);
      gy[c] = ok ? Sy[i * M + a] : T(0);
      gz[c] = ok ? Sz[i * M + a] : T(0);
    }
  }
  __syncthreads();
  contract<T, M, RP, TILES, TO_LY_FROM_LZ>(b1, b0, fz, wave, lane, inv);
  __syncthreads();
  contract<T, M, RP, TILES, TO_LX_FROM_LY>(b0, b1, fy, wave, lane, inv);
  __syncthreads();
  contract<T, M, RP, TILES, TO_LX_SAME>(b1, b0, fx, wave, lane, inv);
  __syncthreads();
  contract<T, M, RP, TILES, TO_LY_FROM_LX>(b0, b1, gx, wave, lane, inv);
  __syncthreads();
  contract<T, M, RP, TILES, TO_LZ_FROM_LY>(b1, b0, gy, wave, lane, inv);
  __syncthreads();
  contract<T, M, RP, TILES, TO_LZ_SAME>(b0, b1, gz, wave, lane, inv);
  __syncthreads();
  // slot-split output (8 k^3 contiguous values per patch) from LZ of buffer 1:
  // thread = (x, y) pencil; node a of an axis lies in slot 0 at a (a <= k-1) and
  // in slot 1 at a - (k-1) (a >= k-1)
  constexpr int k3 = k * k * k;
  T* wp = W + pid * (8 * k3);
  if (tid < M * M) {
    const int x = tid % M, y = tid / M;
#pragma unroll
    for (int z = 0; z < M; ++z) {
      const T v = b1[z * RP + x + M * y];
#pragma unroll
      for (int szs = 0; szs < 2; ++szs) {
        const int jz = szs ? z - (k - 1) : z;
        if (jz < 0 || jz >= k) continue;
#pragma unroll
        for (int sys = 0; sys < 2; ++sys) {
          const int jy = sys ? y - (k - 1) : y;
          if (jy < 0 || jy >= k) continue;
#pragma unroll
          for (int sxs = 0; sxs < 2; ++sxs) {
            const int jx = sxs ? x - (k - 1) : x;
            if (jx < 0 || jx >= k) continue;
            wp[(sxs + 2 * sys + 4 * szs) * k3 + jx + k * (jy + k * jz)] = v;
          }
        }
      }
    }
  }
}

template <typename T, int K>
static fe_status patch_mfma_typed(const fe_problem* p, const Level& L, const T* r, T* W, const T* eig,
                                  bool per_patch, T scale, hipStream_t s) {
  const int64_t nv = L.n - 1, np = nv * nv * nv;
  if (np == 0) return FE_OK;
  ProfScope ps("fdm_patch", s);
  if (per_patch)
    hipLaunchKernelGGL((k_fdm_patch3_mfma<T, K, true>), dim3((unsigned)np), dim3(256), 0, s, r, W, eig, scale, L.n);
  else
    hipLaunchKernelGGL((k_fdm_patch3_mfma<T, K, false>), dim3((unsigned)np), dim3(256), 0, s, r, W, eig, scale, L.n);
  FE_HIP_CHECK(hipGetLastError());
  return FE_OK;
}

bool patch_mfma_supported(const fe_problem* p) { return p->dim == 3 && p->k >= 5 && p->k <= 8; }

fe_status launch_patch_mfma(const fe_problem* p, const Level& L, const void* r, void* W, const void* eig,
                            bool per_patch, double scale, fe_dtype dt, hipStream_t s) {
  switch (p->K) {
#define FE_MFMA_CASE(KV)                                                                                      \
  case KV:                                                                                                    \
    if (dt == FE_F64)                                                                                         \
      return patch_mfma_typed<double, KV>(p, L, (const double*)r, (double*)W, (const double*)eig, per_patch, \
                                          scale, s);                                                          \
    return patch_mfma_typed<float, KV>(p, L, (const float*)r, (float*)W, (const float*)eig, per_patch,       \
                                       (float)scale, s);
    FE_MFMA_CASE(6)
    FE_MFMA_CASE(7)
    FE_MFMA_CASE(8)
    FE_MFMA_CASE(9)
#undef FE_MFMA_CASE
    default:
      return fail(FE_EUNSUPPORTED, "matrix-core patch kernel needs 5 <= k <= 8");
  }
}

}  // namespace fe
