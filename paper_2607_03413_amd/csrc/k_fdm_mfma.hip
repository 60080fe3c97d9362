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
// Amat[l % 16][4 c + l / 16] in a[c]).  Optional eigenvalue division (MODE
// TO_LX_SAME): out[x'][y + M z] *= scale / (lx[x'] + ly[y] + lz[z]).
template <typename T, int M, int RP, int TILES, int MODE>
__device__ __forceinline__ void contract(const T* __restrict__ in, T* __restrict__ out, const T (&a)[4], int wave,
                                         int lane, const T* lx, const T* ly, const T* lz, T scale) {
  typedef typename Mfma<T>::acc acc;
  constexpr int R = M * M;
  const int j = lane & 15, kk = lane >> 4;
  for (int t = wave; t < TILES; t += 4) {
    acc d = {0, 0, 0, 0};
    const int col = 16 * t + j;
#pragma unroll
    for (int c = 0; c < 4; ++c) d = Mfma<T>::step(a[c], in[(4 * c + kk) * RP + col], d);
    if (col < R) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a2 = Mfma<T>::row(lane, r);
        if (a2 < M) {
          T v = d[r];
          if (MODE == TO_LX_SAME) v = v * scale / (lx[a2] + ly[col % M] + lz[col / M]);
          out[dest_index<M, RP, MODE>(a2, col)] = v;
        }
      }
    }
  }
}

template <typename T, int K, bool PER_PATCH>
__global__ void __launch_bounds__(256) k_fdm_patch3_mfma(const T* __restrict__ r, T* __restrict__ W,
                                                         const T* __restrict__ eig, T scale, int n) {
  using P = MfmaPatch<K>;
  constexpr int k = P::k, M = P::M, RP = P::RP, TS = P::TS, TILES = P::TILES, K3 = P::K3;
  constexpr int CELLS = 8 * K3;
  constexpr int BUF0 = CELLS > TS ? CELLS : TS;
  __shared__ T lds[BUF0 + TS];
  __shared__ T lam[3 * 16];
  T* b0 = lds;          // staged cells, then tensor buffer 0
  T* b1 = lds + BUF0;   // tensor buffer 1
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
  if (tid < 48) {
    const int d = tid / 16, i = tid % 16;
    lam[tid] = i < M ? lsrc[d][i] : T(1);
  }
  // stage the 8 cells of the patch: slot s = sx + 2 sy + 4 sz, contiguous K^3 each
  for (int e = tid; e < CELLS; e += 256) {
    const int s = e / K3, loc = e - s * K3;
    const int64_t cell = (vx - 1 + (s & 1)) + (int64_t)n * ((vy - 1 + ((s >> 1) & 1)) + (int64_t)n * (vz - 1 + (s >> 2)));
    b0[e] = r[cell * K3 + loc];
  }
  // zero the padding rows M..15 of buffer 1 (buffer 0's are zeroed after the gather)
  for (int e = tid; e < (16 - M) * RP; e += 256) b1[M * RP + e] = T(0);
  __syncthreads();
  // assemble the patch residual (cascade order) into LZ of buffer 1
  for (int node = tid; node < M * M * M; node += 256) {
    const int x = node % M, y = (node / M) % M, z = node / (M * M);
    const int o[3] = {x + 1, y + 1, z + 1};
    int cnt[3], sl[3][2], il[3][2];
    for (int a = 0; a < 3; ++a) {
      if (o[a] < k) { cnt[a] = 1; sl[a][0] = 0; il[a][0] = o[a]; }
      else if (o[a] > k) { cnt[a] = 1; sl[a][0] = 1; il[a][0] = o[a] - k; }
      else { cnt[a] = 2; sl[a][0] = 0; il[a][0] = k; sl[a][1] = 1; il[a][1] = 0; }
    }
    T zs[2];
    for (int sz = 0; sz < cnt[2]; ++sz) {
      T ys[2];
      for (int sy = 0; sy < cnt[1]; ++sy) {
        T xs = T(0);
        for (int sx = 0; sx < cnt[0]; ++sx) {
          const int s = sl[0][sx] + 2 * sl[1][sy] + 4 * sl[2][sz];
          const T v = b0[s * K3 + il[0][sx] + K * (il[1][sy] + K * il[2][sz])];
          xs = sx ? xs + v : v;
        }
        ys[sy] = xs;
      }
      zs[sz] = cnt[1] == 2 ? ys[0] + ys[1] : ys[0];
    }
    b1[z * RP + x + M * y] = cnt[2] == 2 ? zs[0] + zs[1] : zs[0];
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
  const T* lx = lam;
  const T* ly = lam + 16;
  const T* lz = lam + 32;
  contract<T, M, RP, TILES, TO_LY_FROM_LZ>(b1, b0, fz, wave, lane, lx, ly, lz, scale);
  __syncthreads();
  contract<T, M, RP, TILES, TO_LX_FROM_LY>(b0, b1, fy, wave, lane, lx, ly, lz, scale);
  __syncthreads();
  contract<T, M, RP, TILES, TO_LX_SAME>(b1, b0, fx, wave, lane, lx, ly, lz, scale);
  __syncthreads();
  contract<T, M, RP, TILES, TO_LY_FROM_LX>(b0, b1, gx, wave, lane, lx, ly, lz, scale);
  __syncthreads();
  contract<T, M, RP, TILES, TO_LZ_FROM_LY>(b1, b0, gy, wave, lane, lx, ly, lz, scale);
  __syncthreads();
  contract<T, M, RP, TILES, TO_LZ_SAME>(b0, b1, gz, wave, lane, lx, ly, lz, scale);
  __syncthreads();
  // slot-split output (8 k^3 contiguous values per patch), read from LZ of buffer 1
  constexpr int k3 = k * k * k;
  T* wp = W + pid * (8 * k3);
  for (int e = tid; e < 8 * k3; e += 256) {
    const int s = e / k3, q = e - s * k3;
    const int jx = q % k, jy = (q / k) % k, jz = q / (k * k);
    const int x = (s & 1) ? jx + k - 1 : jx;
    const int y = ((s >> 1) & 1) ? jy + k - 1 : jy;
    const int z = (s >> 2) ? jz + k - 1 : jz;
    wp[e] = b1[z * RP + x + M * y];
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
