// Fused vertex-patch inverse for the 3D Cartesian mesh at low degree
// (k = 2, 3), where one patch (m^3 = 27 or 125 values, m = 2k-1) fits in the
// registers of one thread.
//
// The operation is the additive Schwarz inverse of the vertex patches with
// fast diagonalization (Sec. 3.3 / Sec. 4.1 vertex-patch smoothers; the
// admissible form P = G P_CG G^T of eq. precond_consistency):
//   z = G sum_p R_p^T (S x S x S) (L + L + L)^{-1} (S x S x S)^T R_p G^T r.
// Instead of writing each patch solution to a scratch buffer and summing the
// overlaps in a second pass, the overlaps are summed on chip:
//
//   * thread = one patch; lanes 0..62 of a wavefront hold the patches of one
//     x-row (vertex vx = X0 + lane; lane 63 only owns a cell at the upper
//     boundary), a block holds WY = 4 consecutive x-rows (vy = Y0 + wave) and
//     marches upwards through a chunk of vertex levels vz;
//   * per level, the 2k cell slices (fixed z-local index) that hold patch
//     nodes are staged in LDS for the block's 64 x 5 cells; where a slice is a
//     whole number of 16-byte chunks (k = 3) the copy runs asynchronously
//     (global -> LDS), and the first slices of the next level are fetched
//     while the current level computes;
//   * each thread sums the copies of its patch nodes (x pairs, then y, then
//     z) and applies the six 1D contractions in registers, using that the
//     patch eigenvectors are even or odd about the middle node (sums and
//     differences of mirrored nodes); S and the inverse eigenvalue sums come
//     through the scalar cache;
//   * plane by plane, overlaps in x are summed across lanes (lane - 1 holds
//     patch vx-1) and overlaps in y through LDS (the wave below holds patch
//     vy-1); the thread that owns cell (vx-1, vy-1, .) holds the merged plane;
//   * the merged upper planes (inside cell layer vz) are stored as partial sums
//     in the owner's cell and completed by the same thread with the next
//     level's merged lower planes: after level vz, cell layer vz-1 is final.
// Every node value is summed in a fixed order (x, then y, then the lower
// level first along z), so all copies of a node are written with identical
// values.
// Patch rows at the lower edge of a tile (lane 0, wave 0, the first level of a
// z chunk) are recomputed by the neighbouring tile, which owns their cells.
#include "fe_internal.h"
#include "kernel_common.h"

namespace fe {

typedef __attribute__((address_space(3))) void lds_void_t;
template <typename T>
using lds_ptr = __attribute__((address_space(3))) const T*;

template <typename T, int K>
struct FusedPatch {
  static constexpr int k = K - 1;
  static constexpr int M = 2 * k - 1;
  static constexpr int K2 = K * K;
  static constexpr int WY = 4;            // x-rows of patches per block
  static constexpr int OWN_X = 62;        // owned cells per row (tiles after the first)
  static constexpr int OWN_Y = WY - 1;
  static constexpr int NXC = 64;          // cells per staged row: X0-1 .. X0+62
  static constexpr int NYC = WY + 1;      // staged rows: Y0-1 .. Y0+3
  // asynchronous staging when a cell slice is a whole number of 16-byte chunks
  static constexpr bool DMA = (K2 * sizeof(T)) % 16 == 0;
  static constexpr int VPC = 16 / sizeof(T);                  // values per chunk
  static constexpr int NCH = DMA ? K2 * (int)sizeof(T) / 16 : 1;
  static constexpr int NBUF = DMA ? 3 : 2;                    // slice buffers
  // DMA layout of one slice buffer: [row][chunk][cell][VPC]; otherwise [row][cell][K2 | 1]
  static constexpr int SLICE = DMA ? NYC * NCH * NXC * VPC : NYC * NXC * (K2 | 1);
  static constexpr int XPLANE = k * K;    // values handed to the wave above, per plane
};

// Copies of patch-local node a (0 <= a <= 2k-2) along one axis: cell slot
// (0 = lower cell, 1 = upper cell) and local index, lower slot first.
template <int K>
__device__ __forceinline__ AxisCopies fused_axis_copies(int a) {
  constexpr int k = K - 1;
  AxisCopies c;
  const int o = a + 1;
  if (o < k) { c.cnt = 1; c.c[0] = 0; c.i[0] = o; }
  else if (o > k) { c.cnt = 1; c.c[0] = 1; c.i[0] = o - k; }
  else { c.cnt = 2; c.c[0] = 0; c.i[0] = k; c.c[1] = 1; c.i[1] = 0; }
  if (c.cnt == 1) { c.c[1] = c.c[0]; c.i[1] = c.i[0]; }
  return c;
}

// Element (p, q, a) of the patch block w[az][ay][ax] for a line along axis AX
// (Q = M planes; a block of Q < M planes only takes lines along x and y).
template <int AX, typename T, int Q, int M>
__device__ __forceinline__ T& line_at(T (&w)[Q][M][M], int p, int q, int a) {
  static_assert(AX < 2 || Q == M, "lines along z need every plane");
  if (AX == 0) return w[q][p][a];
  if (AX == 1) return w[q][a][p];
  return w[a][q][p];
}

// In-register 1D contraction along axis AX with the mirror-symmetric patch
// eigenvectors (c = (M-1)/2 is the middle node; modes ordered evens first).
// Forward (S^T): t_e[j] = sum_{a<c} SE[j][a] (x_a + x_{M-1-a}) + SE[j][c] x_c,
//                t_o[j] = sum_{a<c} SO[j][a] (x_a - x_{M-1-a}).
// Backward (S):  E_a = sum_j SE[j][a] t_e[j], O_a = sum_j SO[j][a] t_o[j],
//                x_a = E_a + O_a, x_{M-1-a} = E_a - O_a, x_c = E_c.
template <int AX, bool FWD, typename T, int Q, int M>
__device__ __forceinline__ void contract_axis(T (&w)[Q][M][M], const T* __restrict__ Seo) {
  constexpr int c = (M - 1) / 2, ne = c + 1, no = c;
  const T* __restrict__ SE = Seo;
  const T* __restrict__ SO = Seo + ne * (c + 1);
#pragma unroll
  for (int q = 0; q < Q; ++q)
#pragma unroll
    for (int p = 0; p < M; ++p) {
      T x[M], y[M];
#pragma unroll
      for (int a = 0; a < M; ++a) x[a] = line_at<AX>(w, p, q, a);
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
#pragma unroll
      for (int a = 0; a < M; ++a) line_at<AX>(w, p, q, a) = y[a];
    }
}

// Workgroup barrier without a memory fence.  A fence here would also wait for
// every copy still in flight into LDS (vmcnt(0)) and serialize the staging
// pipeline; instead each wavefront waits for the copies it needs explicitly
// (wait_vmcnt_le), its LDS operations complete before the barrier
// (lgkmcnt(0)), and the "memory" clobber keeps the compiler from moving
// memory accesses across it.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Value of lane - 1 (0 in lane 0): a DPP wavefront shift, no LDS traffic.
__device__ __forceinline__ float lane_shift_up(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, false));
}
__device__ __forceinline__ double lane_shift_up(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), 0x138, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x138, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Wait until at most `n` vector memory operations of this wavefront are
// outstanding (s_waitcnt vmcnt(n), n a compile-time constant after unrolling;
// expcnt and lgkmcnt left at their maxima).
__device__ __forceinline__ void wait_vmcnt_le(int n) {
  switch (n) {
#define FE_VMCNT_CASE(N) \
    case N: __builtin_amdgcn_s_waitcnt(((N) & 0xF) | (((N) >> 4) << 14) | (0x7 << 4) | (0xF << 8)); break;
    FE_VMCNT_CASE(0) FE_VMCNT_CASE(1) FE_VMCNT_CASE(2) FE_VMCNT_CASE(3) FE_VMCNT_CASE(4) FE_VMCNT_CASE(5)
    FE_VMCNT_CASE(6) FE_VMCNT_CASE(7) FE_VMCNT_CASE(8) FE_VMCNT_CASE(9) FE_VMCNT_CASE(10) FE_VMCNT_CASE(12)
    FE_VMCNT_CASE(14) FE_VMCNT_CASE(15) FE_VMCNT_CASE(16) FE_VMCNT_CASE(18) FE_VMCNT_CASE(20) FE_VMCNT_CASE(24)
    FE_VMCNT_CASE(25) FE_VMCNT_CASE(30) FE_VMCNT_CASE(40)
#undef FE_VMCNT_CASE
    default: __builtin_amdgcn_s_waitcnt(0x0F70); break;   // vmcnt(0)
  }
}

// Slice s of patch level vz: cell layer and z-local index (see the header).
template <int K>
__device__ __forceinline__ void slice_of(int s, int vz, int& layer, int& iz) {
  constexpr int k = K - 1;
  layer = s < k ? vz - 1 : vz;
  iz = s < k ? s + 1 : s - k;
}

// Stage slice s of level vz into buffer `buf` for the block's 64 x 5 cells.
// Cells outside the mesh are clamped to a valid address; they are never read.
template <typename T, int K>
__device__ __forceinline__ void stage_slice(T* buf, const T* __restrict__ r, int s, int vz, int X0, int Y0, int n,
                                            int tid) {
  using FP = FusedPatch<T, K>;
  constexpr int K2 = FP::K2, K3 = K2 * K, NXC = FP::NXC, NYC = FP::NYC;
  int layer, iz;
  slice_of<K>(s, vz, layer, iz);
  if (FP::DMA) {
    // one 16-byte chunk per lane, one (row, chunk) pair per wavefront instruction
    const int lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int gx = min(X0 - 1 + lane, n - 1);
    for (int q = w; q < NYC * FP::NCH; q += FP::WY) {
      const int cyl = q / FP::NCH, ch = q % FP::NCH;
      const int gy = min(Y0 - 1 + cyl, n - 1);
      const T* src = r + ((int64_t)gx + (int64_t)n * (gy + (int64_t)n * layer)) * K3 + iz * K2 + ch * FP::VPC;
      T* dst = buf + (q * NXC) * FP::VPC;
      __builtin_amdgcn_global_load_lds((const void*)src, (lds_void_t*)dst, 16, 0, 0);
    }
  } else {
    constexpr int CS = K2 | 1;
#pragma unroll 4
    for (int e = tid; e < NYC * NXC * K2; e += 64 * FP::WY) {
      const int ent = e % K2, cell = e / K2;
      const int cxl = cell % NXC, cyl = cell / NXC;
      const int gx = min(X0 - 1 + cxl, n - 1), gy = min(Y0 - 1 + cyl, n - 1);
      buf[(cyl * NXC + cxl) * CS + ent] =
          r[((int64_t)gx + (int64_t)n * (gy + (int64_t)n * layer)) * K3 + iz * K2 + ent];
    }
  }
}

// Offset (in values) of staged cell (cxl, cyl), slice-local entry e = iy*K + ix.
template <typename T, int K>
__device__ __forceinline__ constexpr int staged_offset(int cyl, int cxl, int e) {
  using FP = FusedPatch<T, K>;
  return FP::DMA ? ((cyl * FP::NCH + e / FP::VPC) * FP::NXC + cxl) * FP::VPC + e % FP::VPC
                 : (cyl * FP::NXC + cxl) * (FP::K2 | 1) + e;
}

// Row iy (K values) of staged cell (cxl, cyl) relative to the thread's own
// cell; in the chunked layout a row is K / VPC whole 16-byte vectors, read at
// compile-time offsets from one base.
template <typename T, int K>
__device__ __forceinline__ void staged_row(lds_ptr<T> lb, int cyl, int cxl, int iy, T (&row)[K]) {
  using FP = FusedPatch<T, K>;
  if constexpr (FP::DMA) {
    typedef T vec_t __attribute__((ext_vector_type(FP::VPC)));
#pragma unroll
    for (int c = 0; c < K / FP::VPC; ++c) {
      const vec_t v = *reinterpret_cast<__attribute__((address_space(3))) const vec_t*>(
          lb + staged_offset<T, K>(cyl, cxl, iy * K + c * FP::VPC));
#pragma unroll
      for (int j = 0; j < FP::VPC; ++j) row[c * FP::VPC + j] = v[j];
    }
  } else {
#pragma unroll
    for (int i = 0; i < K; ++i) row[i] = lb[staged_offset<T, K>(cyl, cxl, iy * K + i)];
  }
}

// Sum the copies that slice s holds for every node of patch plane az(s).
// `lb` points at the thread's own cell (row wy, cell lane) of the staged
// slice; every other read is at a compile-time offset from it.
template <typename T, int K, int M>
__device__ __forceinline__ void pull_slice(T (&w)[M][M][M], lds_ptr<T> lb, int s) {
  constexpr int k = K - 1;
  const int az = s < k ? s : s - 1;
  const bool accumulate = s == k;   // second slice of the vertex plane
#pragma unroll
  for (int ay = 0; ay < M; ++ay) {
    const AxisCopies cyc = fused_axis_copies<K>(ay);
    T rows[2][2][K];   // [y copy][x cell][ix]
#pragma unroll
    for (int sy = 0; sy < 2; ++sy) {
      if (sy >= cyc.cnt) break;
      staged_row<T, K>(lb, cyc.c[sy], 0, cyc.i[sy], rows[sy][0]);
      staged_row<T, K>(lb, cyc.c[sy], 1, cyc.i[sy], rows[sy][1]);
    }
#pragma unroll
    for (int ax = 0; ax < M; ++ax) {
      const AxisCopies cxc = fused_axis_copies<K>(ax);
      T ys = T(0);
#pragma unroll
      for (int sy = 0; sy < 2; ++sy) {
        if (sy >= cyc.cnt) break;
        T xs = rows[sy][cxc.c[0]][cxc.i[0]];
        if (cxc.cnt == 2) xs += rows[sy][cxc.c[1]][cxc.i[1]];
        ys = sy == 0 ? xs : ys + xs;
      }
      if (accumulate) w[az][ay][ax] += ys;
      else w[az][ay][ax] = ys;
    }
  }
}

template <typename T, int K>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 2 : 1)))
k_fdm_fused3(const T* __restrict__ r, T* __restrict__ z, const T* __restrict__ Seo, const T* __restrict__ il, int n,
                                                    int nxt, int nyt, int zlen) {
  using FP = FusedPatch<T, K>;
  constexpr int k = FP::k, M = FP::M, WY = FP::WY, K2 = FP::K2, K3 = K2 * K;
  constexpr int NBUF = FP::NBUF, SLICE = FP::SLICE, XPLANE = FP::XPLANE;
  constexpr int NS = 2 * k;   // slices per level
  // three distinct LDS arrays (rather than one) let the compiler see that a
  // read of one buffer does not depend on the copies still landing in another
  __shared__ __attribute__((aligned(16))) T sbuf0[SLICE];
  __shared__ __attribute__((aligned(16))) T sbuf1[SLICE];
  __shared__ __attribute__((aligned(16))) T sbuf2[NBUF > 2 ? SLICE : 1];
  auto buf = [&](int j) -> T* { return j == 0 ? sbuf0 : (j == 1 ? sbuf1 : sbuf2); };
  __shared__ T xch[XPLANE * 64 * WY];
  static_assert(XPLANE * 64 * WY <= SLICE, "the overlap exchange also uses a slice buffer");

  // XCD-aware block order: consecutive logical tiles land on the same XCD
  // (blocks are dealt to the 8 XCDs round-robin), so that the halo rows and
  // levels shared by neighbouring tiles are re-read from the same L2.
  const int nb = gridDim.x;
  const int xcd = blockIdx.x & 7, q8 = nb >> 3, rem = nb & 7;
  const int logical = xcd * q8 + min(xcd, rem) + (int)(blockIdx.x >> 3);
  const int nzc = nb / (nxt * nyt);
  const int tz = logical % nzc;
  const int t2 = logical / nzc;
  const int ty = t2 % nyt, tx = t2 / nyt;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wy = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int X0 = 1 + FP::OWN_X * tx, Y0 = 1 + FP::OWN_Y * ty;
  const int vx = X0 + lane, vy = Y0 + wy;
  const bool pxy = lane <= 62 && vx <= n - 1 && vy <= n - 1;
  const int cx = vx - 1, cy = vy - 1;
  const bool own_xy = cx <= n - 1 && cy <= n - 1 && (lane >= 1 || tx == 0) && (lane <= 62 || vx == n) &&
                      (wy >= 1 || ty == 0);
  const int C0 = tz * zlen, C1 = min(n, C0 + zlen);
  const int lane_off = staged_offset<T, K>(wy, lane, 0);

  // slices 0 .. NBUF-1 of the first level are in flight before the loop
  if (C0 >= 1 && C0 <= n - 1) {
#pragma unroll
    for (int s = 0; s < NBUF; ++s) stage_slice<T, K>(buf(s), r, s, C0, X0, Y0, n, tid);
  }

  for (int vz = C0; vz <= C1; ++vz) {
    T w[M][M][M];
    const bool level_ok = vz >= 1 && vz <= n - 1;   // uniform over the block
    const bool next_ok = vz + 1 <= C1 && vz + 1 <= n - 1;
    if (level_ok) {
      // (1) patch residual R_p G^T r, slice by slice: slice s is read from
      // buffer s % NBUF, which then receives slice s + NBUF, so that NBUF - 1
      // copies stay in flight while a slice is summed
#pragma unroll
      for (int sl = 0; sl < NS; ++sl) {
        // wait until slice sl has landed.  Loads (copies included) complete in
        // issue order, so while slice sl is outstanding every copy issued after
        // it is too: allowing that many outstanding operations is safe even with
        // stores of the previous level, which may complete out of order, still
        // in flight (they only make the wait longer).
        constexpr int DPW = FP::DMA ? (FP::NYC * FP::NCH) / WY : 0;
        const int later = (sl + NBUF - 1 < NS - 1 ? sl + NBUF - 1 : NS - 1) - sl;
        if (FP::DMA) wait_vmcnt_le(later * DPW);
        lds_barrier();
        if (pxy) {
          // the lane offset is made opaque so that it is recomputed here
          // instead of three buffer bases being kept live across the level loop
          int off = lane_off;
          asm volatile("" : "+v"(off));
          lds_ptr<T> lb = (lds_ptr<T>)(buf(sl % NBUF)) + off;
          pull_slice<T, K, M>(w, lb, sl);
        }
        if (sl + NBUF < NS) {
          lds_barrier();   // readers of this buffer are done
          stage_slice<T, K>(buf(sl % NBUF), r, sl + NBUF, vz, X0, Y0, n, tid);
        }
      }
      if (!pxy) {
#pragma unroll
        for (int az = 0; az < M; ++az)
#pragma unroll
          for (int ay = 0; ay < M; ++ay)
#pragma unroll
            for (int ax = 0; ax < M; ++ax) w[az][ay][ax] = T(0);
      }
      // the next level's first slices are fetched while this level computes;
      // the last buffer serves the overlap exchange first and is refilled after it
      lds_barrier();
      if (next_ok) {
#pragma unroll
        for (int s = 0; s < NBUF - 1; ++s) stage_slice<T, K>(buf(s), r, s, vz + 1, X0, Y0, n, tid);
      }
      // (2) fast diagonalization in registers
      contract_axis<2, true>(w, Seo);
      contract_axis<1, true>(w, Seo);
      contract_axis<0, true>(w, Seo);
#pragma unroll
      for (int az = 0; az < M; ++az)
#pragma unroll
        for (int ay = 0; ay < M; ++ay)
#pragma unroll
          for (int ax = 0; ax < M; ++ax) w[az][ay][ax] *= il[(az * M + ay) * M + ax];
      contract_axis<0, false>(w, Seo);
      contract_axis<1, false>(w, Seo);
      contract_axis<2, false>(w, Seo);
    } else {
#pragma unroll
      for (int az = 0; az < M; ++az)
#pragma unroll
        for (int ay = 0; ay < M; ++ay)
#pragma unroll
          for (int ax = 0; ax < M; ++ax) w[az][ay][ax] = T(0);
      if (next_ok) {
        lds_barrier();
#pragma unroll
        for (int s = 0; s < NBUF - 1; ++s) stage_slice<T, K>(buf(s), r, s, vz + 1, X0, Y0, n, tid);
      }
    }

    // (3) merge the overlaps plane by plane.  Patch plane az holds nodes of
    // cell layer vz-1 (plane iz = az + 1) for az <= k-1 and of layer vz
    // (iz = az - k + 1) for az >= k-1.  Per plane: x overlap across lanes
    // (lane - 1 holds patch vx-1), then y overlap through LDS (the wave below
    // holds patch vy-1).  The merged upper planes of this level are stored in
    // the owner's cell as partial sums, which the same thread completes with
    // the next level's merged lower planes.
    const int64_t cell_xy = (int64_t)cx + (int64_t)n * cy;
    T* out_lo = z + (cell_xy + (int64_t)n * n * (vz - 1)) * K3;   // cell layer vz-1
    T* out_hi = z + (cell_xy + (int64_t)n * n * vz) * K3;         // cell layer vz
    const bool write_lo = own_xy && vz - 1 >= C0;
    const bool write_hi = own_xy && vz < C1;
#pragma unroll
    for (int az = 0; az < M; ++az) {
      T X[M][K];
#pragma unroll
      for (int b = 0; b < M; ++b) {
#pragma unroll
        for (int i = 0; i < K; ++i) {
          T lo = T(0);
          if (i < k) lo = lane_shift_up(w[az][b][k - 1 + i]);   // lane 0: patch vx-1 is not in this wavefront
          if (i == 0) X[b][i] = lo;
          else if (i < k) X[b][i] = lo + w[az][b][i - 1];
          else X[b][i] = w[az][b][k - 1];
        }
      }
      // planes alternate between two exchange buffers, so one barrier per plane
      // suffices within a level: a buffer is rewritten two planes later, after
      // every reader has passed the barrier of the plane in between (across
      // levels, see the barrier at the end of the level)
      T* xb = (az & 1) ? buf(NBUF - 1) : xch;
#pragma unroll
      for (int j = 0; j < k; ++j)
#pragma unroll
        for (int i = 0; i < K; ++i) xb[(j * K + i) * (64 * WY) + tid] = X[k - 1 + j][i];
      lds_barrier();
      T Y[K][K];
#pragma unroll
      for (int j = 0; j < K; ++j)
#pragma unroll
        for (int i = 0; i < K; ++i) {
          T lo = T(0);
          if (j < k && wy >= 1) lo = xb[(j * K + i) * (64 * WY) + tid - 64];
          if (j == 0) Y[j][i] = lo;
          else if (j < k) Y[j][i] = lo + X[j - 1][i];
          else Y[j][i] = X[k - 1][i];
        }
      if (az < k - 1) {
        // layer vz-1, plane az+1: add to what the level below left there
        if (write_lo) {
#pragma unroll
          for (int j = 0; j < K; ++j)
#pragma unroll
            for (int i = 0; i < K; ++i) out_lo[(az + 1) * K2 + j * K + i] += Y[j][i];
        }
      } else if (az == k - 1) {
        // vertex plane: layer vz-1 plane k and layer vz plane 0
        if (write_lo) {
#pragma unroll
          for (int j = 0; j < K; ++j)
#pragma unroll
            for (int i = 0; i < K; ++i) out_lo[k * K2 + j * K + i] = Y[j][i];
        }
        if (write_hi) {
#pragma unroll
          for (int j = 0; j < K; ++j)
#pragma unroll
            for (int i = 0; i < K; ++i) out_hi[j * K + i] = Y[j][i];
        }
      } else if (write_hi) {
        // layer vz, plane az-k+1: partial sum, completed by the next level
#pragma unroll
        for (int j = 0; j < K; ++j)
#pragma unroll
          for (int i = 0; i < K; ++i) out_hi[(az - k + 1) * K2 + j * K + i] = Y[j][i];
      }
    }
    // Every wavefront has read the exchange data of this level's last plane
    // before the next level writes it: the last plane (M-1, even) and the next
    // level's first plane (0, even) use the same buffer, and a level without a
    // patch (vz = n) stages nothing, so no other barrier separates them.  Then
    // the last slice buffer is refilled for the next level.
    lds_barrier();
    if (next_ok) stage_slice<T, K>(buf(NBUF - 1), r, NBUF - 1, vz + 1, X0, Y0, n, tid);
  }
  __builtin_amdgcn_s_waitcnt(0);
}

// ---------------------------------------------------------------------------
// Two lanes per patch (3D, k = 3, FP64 and FP32).
//
// One thread per patch needs the M^3 = 125 patch values in registers, which
// in FP64 is the whole register file of a lane: one wavefront per SIMD and
// values parked in accumulation registers.  The patch eigenvectors are even
// or odd about the middle node along z, so the z sums s_a = x_a + x_{M-1-a}
// (a <= c, s_c = x_c) feed only the even z-modes and the differences
// d_a = x_a - x_{M-1-a} (a < c) only the odd ones.  Lane pi of the lower
// half-wavefront keeps the c+1 planes s_a of patch X0+pi, lane pi+32 the c
// planes d_a (plus one plane of zeros), and both run the same instructions:
// the z contraction with their own 1D block (even or odd eigenvectors), the
// y and x contractions and the inverse eigenvalue sums plane by plane, and
// the z back-transform, which leaves E_a in the lower and O_a in the upper
// lane.  The patch planes a and M-1-a are E_a + O_a and E_a - O_a; a swap
// between the half-wavefronts gives the lower lane plane a and the upper lane
// plane M-1-a, and the overlaps are then merged as in the one-lane kernel
// (x across lanes, y through LDS, z through partial sums in the output).
// A lane's merged plane is one cell's 128 contiguous bytes, 512 bytes from
// the next lane's: written directly, every store instruction would touch 64
// cache lines.  Instead each half-wavefront deposits its 32 planes in a
// wavefront-private staging area (the last slice buffer, whose copy for the
// next level is issued after the merge) and the wavefront stores them as
// 16-byte chunks, 8 consecutive lanes per plane; the partial sums of the
// level below are read back in the same orientation (FP32: kept in LDS from
// one level to the next instead, in the same orientation).
//
// A row of 32 patches touches 33 cells; the upper boundary cell of the mesh
// (x = n-1) has no patch of its own and is assembled by the lane of patch
// n-1, then stored with the row's other cells.  Blocks are 8 rows (one
// wavefront each) of which the first recomputes the last row of the tile
// below.
template <typename T, int K, int WY_ = 8, int NBUF_ = 3>
struct SplitPatch {
  using value_type = T;
  static constexpr int K_ = K;
  static constexpr int k = K - 1;
  static constexpr int M = 2 * k - 1;
  static constexpr int K2 = K * K, K3 = K2 * K;
  static constexpr int C = k - 1;              // middle node of a patch line
  static constexpr int NE = C + 1, NO = C;     // even / odd z-planes
  static constexpr int WY = WY_;               // rows of patches per block (one wavefront each)
  static constexpr int NPX = 32;               // patches per row (one per half-wavefront lane)
  static constexpr int OWN_X = NPX - 1;        // cells owned per row by tiles after the first
  static constexpr int OWN_Y = WY - 1;
  static constexpr int NXC = NPX + 1;          // staged cells per row: X0-1 .. X0+31
  static constexpr int NYC = WY + 1;           // staged rows: Y0-1 .. Y0+7
  static constexpr int VPC = 16 / (int)sizeof(T);
  static constexpr int NCH = K2 * (int)sizeof(T) / 16;
  static constexpr int SLOTS = NYC * NCH * NXC;       // 16-byte chunks per slice
  static constexpr int NCOPY = (SLOTS + 63) / 64;     // copy instructions per slice
  static constexpr int SLICE = NCOPY * 64 * VPC;      // values per slice buffer
  static constexpr int CPW = (NCOPY + WY - 1) / WY;   // copies per wavefront and slice
  static constexpr int NBUF = NBUF_;                  // slice buffers
  static constexpr int XPLANE = k * K;                // values handed to the row above, per plane
  static constexpr int XCH = XPLANE * 64 * (WY - 1);
  static constexpr int XEB = M * k * WY * 2;          // boundary-cell rows, per wavefront and half
  static constexpr int ILS = 2 * NE * M * M;          // inverse eigenvalue sums per lane half
  static_assert((K2 * sizeof(T)) % 16 == 0, "a cell slice must be whole 16-byte chunks");
};

// Number of x-tiles: tiles before the last own 32 (first) or 31 cells; the
// last one ends at patch n-1 and owns the cells up to n-1.
static int split_x_tiles(int n) { return n - 1 <= 32 ? 1 : (n - 33 + 30) / 31 + 1; }

// Offset (in values) of staged cell (cxl, cyl), slice-local entry e, in the
// [row][chunk][cell][VPC] layout with NXC cells per row.
template <typename T, int NXC, int NCH>
__device__ __forceinline__ constexpr int split_offset(int cyl, int cxl, int e) {
  constexpr int VPC = 16 / (int)sizeof(T);
  return ((cyl * NCH + e / VPC) * NXC + cxl) * VPC + e % VPC;
}

// Stage slice s of level vz: the block's 33 x 9 cells, one 16-byte chunk per
// lane, chunks in [row][chunk][cell] order (whole wavefront instructions of
// 64 consecutive chunks; the tail of the last one repeats the final chunk).
template <typename SP>
__device__ __forceinline__ void stage_slice_split(typename SP::value_type* buf, const typename SP::value_type* __restrict__ r,
                                                  int s, int vz, int X0, int Y0, int n, int tid) {
  using T = typename SP::value_type;
  constexpr int K = SP::K_;
  int layer, iz;
  slice_of<K>(s, vz, layer, iz);
  const int lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
  // every wavefront issues the same number of copies (a compile-time count, so
  // that the outstanding-copy accounting is exact); a wavefront with one copy
  // less repeats its last one, which rewrites the same bytes
#pragma unroll
  for (int t = 0; t < SP::CPW; ++t) {
    const int q = w + SP::WY * t < SP::NCOPY ? w + SP::WY * t : w + SP::WY * (t - 1);
    const int L = min(q * 64 + lane, SP::SLOTS - 1);
    const int pair = L / SP::NXC, cell = L - pair * SP::NXC;
    const int cyl = pair / SP::NCH, ch = pair - cyl * SP::NCH;
    const int gx = min(X0 - 1 + cell, n - 1), gy = min(Y0 - 1 + cyl, n - 1);
    const T* src = r + ((int64_t)gx + (int64_t)n * (gy + (int64_t)n * layer)) * SP::K3 + iz * SP::K2 + ch * SP::VPC;
    T* dst = buf + q * 64 * SP::VPC;
    __builtin_amdgcn_global_load_lds((const void*)src, (lds_void_t*)dst, 16, 0, 0);
  }
}

// Sum the copies that slice s holds for every node of patch plane az(s) and
// fold the plane into the lane's z sums (lower half: +) or differences (upper
// half: + below the middle, - above, 0 for the middle plane): ca, cm and cn
// are the lane's factors for the planes below the middle, the middle plane
// and the planes above it (all 0 in lanes without a patch).
template <typename T, int K, int M, int NE, int NXC, int NCH>
__device__ __forceinline__ void pull_slice_fold(T (&w)[NE][M][M], lds_ptr<T> lb, int s, T ca, T cm, T cn) {
  constexpr int k = K - 1, C = k - 1, VPC = 16 / (int)sizeof(T);
  typedef T vec_t __attribute__((ext_vector_type(VPC)));
  const int az = s < k ? s : s - 1;
  const int j = az <= C ? az : M - 1 - az;
#pragma unroll
  for (int ay = 0; ay < M; ++ay) {
    // one patch row at a time (no instruction moves across): bounds the values
    // in flight to one row's copies
    __builtin_amdgcn_sched_barrier(0);
    const AxisCopies cyc = fused_axis_copies<K>(ay);
    T rows[2][2][K];   // [y copy][x cell][ix]
#pragma unroll
    for (int sy = 0; sy < 2; ++sy) {
      if (sy >= cyc.cnt) break;
#pragma unroll
      for (int cx = 0; cx < 2; ++cx)
#pragma unroll
        for (int c = 0; c < K / VPC; ++c) {
          const vec_t v = *reinterpret_cast<__attribute__((address_space(3))) const vec_t*>(
              lb + split_offset<T, NXC, NCH>(cyc.c[sy], cx, cyc.i[sy] * K + c * VPC));
#pragma unroll
          for (int e = 0; e < VPC; ++e) rows[sy][cx][c * VPC + e] = v[e];
        }
    }
#pragma unroll
    for (int ax = 0; ax < M; ++ax) {
      const AxisCopies cxc = fused_axis_copies<K>(ax);
      T ys = T(0);
#pragma unroll
      for (int sy = 0; sy < 2; ++sy) {
        if (sy >= cyc.cnt) break;
        T xs = rows[sy][cxc.c[0]][cxc.i[0]];
        if (cxc.cnt == 2) xs += rows[sy][cxc.c[1]][cxc.i[1]];
        ys = sy == 0 ? xs : ys + xs;
      }
      if (s < k) w[j][ay][ax] = (az < C ? ca : cm) * ys;
      else w[j][ay][ax] = fma(az == C ? cm : cn, ys, w[j][ay][ax]);
      asm volatile("" : "+v"(w[j][ay][ax]));   // fold here, not at the next use
    }
  }
}

// z contraction of the lane's planes with its own (NE x NE) block Z:
// forward t_j = sum_a Z[j][a] w_a, backward u_a = sum_j Z[j][a] w_j.
template <bool FWD, typename T, int NE, int M>
__device__ __forceinline__ void zmix(T (&w)[NE][M][M], const T (&Z)[NE][NE]) {
#pragma unroll
  for (int y = 0; y < M; ++y)
#pragma unroll
    for (int x = 0; x < M; ++x) {
      T t[NE];
#pragma unroll
      for (int j = 0; j < NE; ++j) {
        T acc = (FWD ? Z[j][0] : Z[0][j]) * w[0][y][x];
#pragma unroll
        for (int a = 1; a < NE; ++a) acc = fma(FWD ? Z[j][a] : Z[a][j], w[a][y][x], acc);
        t[j] = acc;
      }
#pragma unroll
      for (int j = 0; j < NE; ++j) w[j][y][x] = t[j];
    }
}

// Exchange between the half-wavefronts: lane l < 32 gets v_l + v_{l+32},
// lane l >= 32 gets v_{l-32} - v_l (sg = +1 below, -1 above).
__device__ __forceinline__ float half_combine(float v, float sg) {
  const unsigned b = __float_as_uint(v);
  const auto p = __builtin_amdgcn_permlane32_swap(b, b, false, false);
  return fmaf(sg, __uint_as_float(p[1]), __uint_as_float(p[0]));
}
__device__ __forceinline__ double half_combine(double v, double sg) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)(b & 0xffffffffULL), (unsigned)(b & 0xffffffffULL),
                                                   false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
  const double r0 = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0]));
  const double r1 = __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
  return fma(sg, r1, r0);
}

template <typename T, int K, int WYB, int NB>
__global__ void __launch_bounds__(64 * WYB) __attribute__((amdgpu_waves_per_eu(2)))
k_fdm_fused3_split(const T* __restrict__ r, T* __restrict__ z, const T* __restrict__ Seo, const T* __restrict__ il,
                   int n, int nxt, int nyt, int zlen) {
  using SP = SplitPatch<T, K, WYB, NB>;
  constexpr int k = SP::k, M = SP::M, C = SP::C, NE = SP::NE, NO = SP::NO, WY = SP::WY;
  constexpr int K2 = SP::K2, K3 = SP::K3, NS = 2 * k, NBUF = SP::NBUF, SLICE = SP::SLICE;
  constexpr int NXC = SP::NXC, NCH = SP::NCH;
  __shared__ __attribute__((aligned(16))) T sbuf0[SLICE];
  __shared__ __attribute__((aligned(16))) T sbuf1[SLICE];
  __shared__ __attribute__((aligned(16))) T sbuf2[NBUF > 2 ? SLICE : 1];
  auto buf = [&](int j) -> T* { return j == 0 ? sbuf0 : (j == 1 ? sbuf1 : sbuf2); };
  __shared__ T xch[SP::XCH];
  __shared__ T xeb[SP::XEB];
  __shared__ T ils[SP::ILS];

  const int nb = gridDim.x;
  const int xcd = blockIdx.x & 7, q8 = nb >> 3, rem = nb & 7;
  const int logical = xcd * q8 + min(xcd, rem) + (int)(blockIdx.x >> 3);
  const int nzc = nb / (nxt * nyt);
  const int tz = logical % nzc;
  const int t2 = logical / nzc;
  const int ty = t2 % nyt, tx = t2 / nyt;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wy = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int half = lane >> 5, pi = lane & 31;
  const bool last_tx = tx == nxt - 1;
  const int X0 = last_tx ? max(1, n - SP::NPX) : 1 + SP::OWN_X * tx;
  const int own_lo = tx == 0 ? 0 : 1 + SP::OWN_X * tx;
  const int own_hi = last_tx ? n - 1 : SP::OWN_X * (tx + 1);
  const int Y0 = 1 + SP::OWN_Y * ty;
  const int vx = X0 + pi, vy = Y0 + wy;
  const bool pxy = vx <= n - 1 && vy <= n - 1;
  const int cx = vx - 1, cy = vy - 1;
  const bool own_y = cy <= n - 1 && (wy >= 1 || ty == 0);
  // The boundary cell x = n-1 is the cell of the lane on vertex n (no patch,
  // completed by the x merge) when the tile reaches that far; otherwise
  // (X0 + 32 = n) the lane of patch n-1 assembles it as an extra cell.
  const bool ext = last_tx && vx == n - 1 && X0 + SP::NPX == n;
  const int C0 = tz * zlen, C1 = min(n, C0 + zlen);
  const int lane_off = split_offset<T, NXC, NCH>(wy, pi, 0);

  // lane constants: fold factors (zero without a patch), exchange sign
  const T ca = pxy ? T(1) : T(0);
  const T cm = pxy && !half ? T(1) : T(0), cn = pxy ? (half ? T(-1) : T(1)) : T(0);
  const T sg = half ? T(-1) : T(1);
  const T xm = pi == 0 ? T(0) : T(1);   // lane 32 must not take the shifted value of lane 31

  // merge stores: lane (tq, tc) writes chunk tc of the plane of cell X0-1+q,
  // q = t*PPI + tq, t < NST; step t = NST, lanes tq = 0, writes the extra
  // boundary cell X0+31 = n-1.  Bit t of ownm: this block owns it.
  // staging rows padded by one chunk in FP64 (conflict-free deposits); FP32 rows stay unpadded so
  // that the staging area fits one slice buffer
  constexpr int VPC = SP::VPC, PPI = 64 / NCH, NST = SP::NPX / PPI, TSTR = K2 + (sizeof(T) == 8 ? VPC : 0);
  static_assert(SP::NPX % PPI == 0 && (SP::NPX + 1) * TSTR * WY <= SLICE, "store staging must fit one slice buffer");
  typedef T vec_t __attribute__((ext_vector_type(VPC)));
  typedef __attribute__((address_space(3))) vec_t lds_vec_t;
  const int tq = lane / NCH, tc = lane - tq * NCH;
  int ownm = 0;
#pragma unroll
  for (int t = 0; t < NST; ++t) {
    const int q = t * PPI + tq, cq = X0 - 1 + q;
    if (own_y && X0 + q <= n && cq >= own_lo && cq <= own_hi) ownm |= 1 << t;
  }
  if (own_y && last_tx && tq == 0 && X0 + SP::NPX == n) ownm |= 1 << NST;
  // wavefront-private staging area (padded rows: conflict-free deposits)
  __attribute__((address_space(3))) T* const stg =
      (__attribute__((address_space(3))) T*)buf(NBUF - 1) + wy * ((SP::NPX + 1) * TSTR);
  // FP32: the partial sums of the upper planes wait for the next level in LDS
  // (in the store orientation, wavefront-private) instead of a global write
  // and read back; FP64 has no LDS left for them
  constexpr bool PL = sizeof(T) == 4;
  constexpr int PLN = PL ? WY * C * (NST + 1) * 64 * VPC : VPC;
  __shared__ __attribute__((aligned(16))) T psum[PLN];
  auto pslot = [&](int plane, int t) -> lds_vec_t* {   // partial plane 1..C, step t <= NST
    return reinterpret_cast<lds_vec_t*>((__attribute__((address_space(3))) T*)psum +
                                        (((wy * C + plane - 1) * (NST + 1) + t) * 64 + lane) * VPC);
  };

  for (int e = tid; e < SP::ILS; e += 64 * WY) {
    const int h = e / (NE * M * M), rest = e - h * (NE * M * M), j = rest / (M * M), yx = rest - j * (M * M);
    ils[e] = h == 0 ? il[j * M * M + yx] : (j < NO ? il[(NE + j) * M * M + yx] : T(0));
  }

  if (C0 >= 1 && C0 <= n - 1) {
#pragma unroll
    for (int s = 0; s < NBUF; ++s) stage_slice_split<SP>(buf(s), r, s, C0, X0, Y0, n, tid);
  }

  for (int vz = C0; vz <= C1; ++vz) {
    T w[NE][M][M];
    const bool level_ok = vz >= 1 && vz <= n - 1;
    const bool next_ok = vz + 1 <= C1 && vz + 1 <= n - 1;
    if (level_ok) {
#pragma unroll
      for (int sl = 0; sl < NS; ++sl) {
        const int later = (sl + NBUF - 1 < NS - 1 ? sl + NBUF - 1 : NS - 1) - sl;
        wait_vmcnt_le(later * SP::CPW);
        lds_barrier();
        {
          // every lane reads inside the staged block; lanes without a patch fold with 0
          int off = lane_off;
          asm volatile("" : "+v"(off));
          lds_ptr<T> lb = (lds_ptr<T>)(buf(sl % NBUF)) + off;
          pull_slice_fold<T, K, M, NE, NXC, NCH>(w, lb, sl, ca, cm, cn);
        }
        if (sl + NBUF < NS) {
          lds_barrier();
          stage_slice_split<SP>(buf(sl % NBUF), r, sl + NBUF, vz, X0, Y0, n, tid);
        }
      }
      // every buffer has been read: fetch the next level's first slices (the
      // last buffer is the merge's store staging area and is filled after it)
      lds_barrier();
      if (next_ok) {
#pragma unroll
        for (int s = 0; s < NBUF - 1; ++s) stage_slice_split<SP>(buf(s), r, s, vz + 1, X0, Y0, n, tid);
      }
      {
        const T* __restrict__ SE = Seo;
        const T* __restrict__ SO = Seo + NE * (C + 1);
        // built here from an opaque copy of the lane half, so that the block
        // is not kept live (or spilled) across the level loop
        int hz = half;
        asm volatile("" : "+v"(hz));
        T Z[NE][NE];
#pragma unroll
        for (int j = 0; j < NE; ++j)
#pragma unroll
          for (int a = 0; a < NE; ++a) {
            const T se = SE[j * (C + 1) + a];
            const T so = (j < NO && a < NO) ? SO[j * C + a] : T(0);
            Z[j][a] = hz ? so : se;
          }
        zmix<true>(w, Z);
      }
      contract_axis<1, true>(w, Seo);
      contract_axis<0, true>(w, Seo);
      {
        lds_ptr<T> ib = (lds_ptr<T>)ils + half * (NE * M * M);
#pragma unroll
        for (int j = 0; j < NE; ++j)
#pragma unroll
          for (int y = 0; y < M; ++y) {
            __builtin_amdgcn_sched_barrier(0);   // one row of factors in flight at a time
#pragma unroll
            for (int x = 0; x < M; ++x) w[j][y][x] *= ib[(j * M + y) * M + x];
          }
      }
      contract_axis<0, false>(w, Seo);
      contract_axis<1, false>(w, Seo);
      {
        const T* __restrict__ SE = Seo;
        const T* __restrict__ SO = Seo + NE * (C + 1);
        // built here from an opaque copy of the lane half, so that the block
        // is not kept live (or spilled) across the level loop
        int hz = half;
        asm volatile("" : "+v"(hz));
        T Z[NE][NE];
#pragma unroll
        for (int j = 0; j < NE; ++j)
#pragma unroll
          for (int a = 0; a < NE; ++a) {
            const T se = SE[j * (C + 1) + a];
            const T so = (j < NO && a < NO) ? SO[j * C + a] : T(0);
            Z[j][a] = hz ? so : se;
          }
        zmix<false>(w, Z);
      }
    } else {
#pragma unroll
      for (int j = 0; j < NE; ++j)
#pragma unroll
        for (int y = 0; y < M; ++y)
#pragma unroll
          for (int x = 0; x < M; ++x) w[j][y][x] = T(0);
      if (next_ok) {
        lds_barrier();
#pragma unroll
        for (int s = 0; s < NBUF - 1; ++s) stage_slice_split<SP>(buf(s), r, s, vz + 1, X0, Y0, n, tid);
      }
    }

    // Merge plane by plane: step a gives the lower lane patch plane a and the
    // upper lane plane M-1-a (the middle plane only in the lower lane).
    // Plane az holds nodes of cell layer vz-1 (iz = az + 1) for az <= k-1 and
    // of layer vz (iz = az - k + 1) for az >= k-1.
    const int64_t cell_xy = (int64_t)cx + (int64_t)n * cy;
    const bool lo_ok = vz - 1 >= C0, hi_ok = vz < C1;
    // store orientation: chunk tc of the plane of cell X0-1+q, q = t*PPI + tq,
    // at st_lo + t*PPI*K3 (layer vz-1) and st_hi + t*PPI*K3 (layer vz)
    T* const st_lo = z + (cell_xy - pi + tq + (int64_t)n * n * (vz - 1)) * K3 + tc * VPC;
    T* const st_hi = st_lo + (int64_t)n * n * K3;
    // FP32: the partial sums this level completes, read before step 0 rewrites
    // plane C with this level's own partial sums (one LDS slot per plane)
    vec_t pold[PL ? C : 1][NST + 1];
#pragma unroll
    for (int pl = 0; pl < (PL ? C : 1); ++pl)
#pragma unroll
      for (int t = 0; t <= NST; ++t) {
        pold[pl][t] = vec_t{};
        if (PL && lo_ok && ((ownm >> t) & 1)) pold[pl][t] = *pslot(pl + 1, t);
      }
#pragma unroll
    for (int a = 0; a <= C; ++a) {
      if (a > 0) lds_barrier();   // the row above has read the previous plane
      // x merge row by row; rows k-1.. go to the row above, rows ..k-1 stay
      T Xk[k][K];
#pragma unroll
      for (int b = 0; b < M; ++b) {
        __builtin_amdgcn_sched_barrier(0);
        T v[M];
#pragma unroll
        for (int x = 0; x < M; ++x) v[x] = a < C ? half_combine(w[a][b][x], sg) : w[C][b][x];
        T X[K];
#pragma unroll
        for (int i = 0; i < K; ++i) {
          if (i == 0) X[i] = lane_shift_up(v[k - 1]) * xm;
          else if (i < k) X[i] = fma(lane_shift_up(v[k - 1 + i]), xm, v[i - 1]);
          else X[i] = v[k - 1];
        }
        if (b < k) {
#pragma unroll
          for (int i = 0; i < K; ++i) Xk[b][i] = X[i];
        }
        if (b >= k - 1 && wy < WY - 1) {
#pragma unroll
          for (int i = 0; i < K; ++i) xch[((b - k + 1) * K + i) * (64 * (WY - 1)) + tid] = X[i];
        }
        if (last_tx && ext) {
          // boundary cell x = n-1: only patch n-1 covers it along x
#pragma unroll
          for (int i = 0; i < k; ++i) xeb[((b * k + i) * WY + wy) * 2 + half] = v[k - 1 + i];
        }
      }
      // partial sums of the level below, read in the store orientation
      vec_t old[NST + 1];
#pragma unroll
      for (int t = 0; t <= NST; ++t) {
        old[t] = vec_t{};   // defined on every path: no value is carried across levels
        if (PL) {
          if (a < C) old[t] = pold[a < C ? a : 0][t];
        } else if (t < NST) {
          if (a < C && lo_ok && ((ownm >> t) & 1)) old[t] = *reinterpret_cast<const vec_t*>(st_lo + t * PPI * K3 + (a + 1) * K2);
        }
      }
      lds_barrier();
      // the extra boundary cell, one value per lane (pi < K2, both halves):
      // rows of patch n-1 from this wavefront and the one below, x node k on
      // the boundary; read here so that the latency overlaps the merge below
      T ye = T(0);
      if (last_tx && X0 + SP::NPX == n && pi < K2) {
        const int j = pi / K, i = pi - j * K;
        if (i < k) {
          const T lo = (j < k && wy >= 1) ? xeb[(((k - 1 + j) * k + i) * WY + wy - 1) * 2 + half] : T(0);
          if (j == 0) ye = lo;
          else if (j < k) ye = lo + xeb[(((j - 1) * k + i) * WY + wy) * 2 + half];
          else ye = xeb[(((k - 1) * k + i) * WY + wy) * 2 + half];
        }
      }
      T Y[K][K];
#pragma unroll
      for (int j = 0; j < K; ++j)
#pragma unroll
        for (int i = 0; i < K; ++i) {
          T lo = T(0);
          if (j < k && wy >= 1) lo = xch[(j * K + i) * (64 * (WY - 1)) + tid - 64];
          if (j == 0) Y[j][i] = lo;
          else if (j < k) Y[j][i] = lo + Xk[j - 1][i];
          else Y[j][i] = Xk[k - 1][i];
        }
      // lower half: planes 0..k-2 complete layer vz-1, the middle plane is the
      // vertex plane of both layers; upper half: the planes above the middle
      // start layer vz as partial sums
      // Stores: a half-wavefront deposits its 32 cell planes in the staging
      // area and the whole wavefront writes them out as 16-byte chunks, NCH
      // consecutive lanes per contiguous plane.
      auto deposit = [&](int h) {
        if (half == h) {
#pragma unroll
          for (int c = 0; c < NCH; ++c) {
            vec_t v;
#pragma unroll
            for (int e = 0; e < VPC; ++e) v[e] = Y[(c * VPC + e) / K][(c * VPC + e) % K];
            *reinterpret_cast<lds_vec_t*>(stg + pi * TSTR + c * VPC) = v;
          }
        }
        if (last_tx && X0 + SP::NPX == n && half == h && pi < K2) stg[SP::NPX * TSTR + pi] = ye;
        __builtin_amdgcn_wave_barrier();
      };
      auto fetch = [&](int t) -> vec_t {
        return *reinterpret_cast<const lds_vec_t*>(stg + (t * PPI + tq) * TSTR + tc * VPC);
      };
      if (a < C) {
        // lower half: planes a+1 of layer vz-1 complete the partial sums
        deposit(0);
#pragma unroll
        for (int t = 0; t < NST; ++t)
          if (lo_ok && ((ownm >> t) & 1)) *reinterpret_cast<vec_t*>(st_lo + t * PPI * K3 + (a + 1) * K2) = fetch(t) + old[t];
        if (lo_ok && ((ownm >> NST) & 1)) {
          const vec_t v = fetch(NST);
          T* const e = st_lo + NST * PPI * K3 + (a + 1) * K2;
          if (PL) {
            *reinterpret_cast<vec_t*>(e) = v + old[NST];
          } else {
            // boundary cell: added in memory (no load, so no wait behind the stores above)
#pragma unroll
            for (int i = 0; i < VPC; ++i) unsafeAtomicAdd(e + i, v[i]);
          }
        }
        __builtin_amdgcn_wave_barrier();
        // upper half: planes k-1-a of layer vz start as partial sums
        deposit(1);
#pragma unroll
        for (int t = 0; t <= NST; ++t) {
          if (!(hi_ok && ((ownm >> t) & 1))) continue;
          if (PL) *pslot(k - 1 - a, t) = fetch(t);
          else *reinterpret_cast<vec_t*>(st_hi + t * PPI * K3 + (k - 1 - a) * K2) = fetch(t);
        }
      } else {
        // the middle plane: the vertex plane of both layers
        deposit(0);
#pragma unroll
        for (int t = 0; t <= NST; ++t) {
          if (!((ownm >> t) & 1)) continue;
          const vec_t v = fetch(t);
          if (lo_ok) *reinterpret_cast<vec_t*>(st_lo + t * PPI * K3 + k * K2) = v;
          if (hi_ok) *reinterpret_cast<vec_t*>(st_hi + t * PPI * K3) = v;
        }
      }
      __builtin_amdgcn_wave_barrier();
    }
    // the exchange area and the store staging area are rewritten by the next level
    lds_barrier();
    if (next_ok) stage_slice_split<SP>(buf(NBUF - 1), r, NBUF - 1, vz + 1, X0, Y0, n, tid);
  }
  __builtin_amdgcn_s_waitcnt(0);
}

bool fused_patch_supported(const fe_problem* p, bool per_patch) {
  return p->dim == 3 && !per_patch && p->k >= 2 && p->k <= 3 && p->co.off_il >= 0 && p->co.off_Seo >= 0;
}

// Number of x-tiles: tile t owns cells up to X0 + 61 = 62 (t + 1), or up to
// X0 + 62 = n - 1 when its lane 63 sits on the boundary vertex n.
static int fused_x_tiles(int n) {
  int t = 0;
  while (!(62 * (t + 1) >= n - 1 || 1 + 62 * t + 63 == n)) ++t;
  return t + 1;
}

template <typename T, int K>
static fe_status fused_typed(const fe_problem* p, int li, const T* r, T* z, const T* coef, hipStream_t s) {
  using FP = FusedPatch<T, K>;
  constexpr int M = FP::M;
  const Level& L = p->levels[li];
  const int n = L.n;
  const int nxt = fused_x_tiles(n);
  const int nyt = n - 1 > 0 ? (n - 1 + FP::OWN_Y - 1) / FP::OWN_Y : 1;
  // Resident blocks per device, then the z-chunk length that minimizes
  // (rounds of blocks) x (levels per block).
  static int resident = 0;
  if (resident == 0) {
    int dev = 0, cus = 0, per_cu = 0;
    FE_HIP_CHECK(hipGetDevice(&dev));
    FE_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    FE_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_fdm_fused3<T, K>, 256, 0));
    resident = cus * (per_cu > 0 ? per_cu : 1);
  }
  int best_len = n;
  double best = 1e300;
  for (int len = 1; len <= n; ++len) {
    const int nzc = (n + len - 1) / len;
    const int64_t blocks = (int64_t)nxt * nyt * nzc;
    const double cost = (double)((blocks + resident - 1) / resident) * (len + 1);
    if (cost < best) { best = cost; best_len = len; }
  }
  const int nzc = (n + best_len - 1) / best_len;
  const int64_t blocks = (int64_t)nxt * nyt * nzc;
  const T* Seo = coef + p->co.off_Seo;
  const T* il = coef + p->co.off_il + (int64_t)li * M * M * M;
  ProfScope ps("fdm_fused", s);
  hipLaunchKernelGGL((k_fdm_fused3<T, K>), dim3((unsigned)blocks), dim3(256), 0, s, r, z, Seo, il, n, nxt, nyt,
                     best_len);
  FE_HIP_CHECK(hipGetLastError());
  return FE_OK;
}

#ifndef FE_SPLIT_WY
#define FE_SPLIT_WY 8
#define FE_SPLIT_NB 3
#endif

// Z-chunk length that minimizes (rounds of blocks) x (levels per block).
static int split_chunk_len(int n, int64_t columns, int resident) {
  int best_len = n;
  double best = 1e300;
  for (int len = 1; len <= n; ++len) {
    const int64_t blocks = columns * ((n + len - 1) / len);
    const double cost = (double)((blocks + resident - 1) / resident) * (len + 1);
    if (cost < best) { best = cost; best_len = len; }
  }
  return best_len;
}

template <typename T, int K, int WYB, int NB>
static fe_status split_typed(const fe_problem* p, int li, const T* r, T* z, const T* coef, hipStream_t s) {
  using SP = SplitPatch<T, K, WYB, NB>;
  constexpr int M = SP::M;
  const Level& L = p->levels[li];
  const int n = L.n;
  const int nxt = split_x_tiles(n);
  const int nyt = (n - 1 + SP::OWN_Y - 1) / SP::OWN_Y;
  static int resident = 0;
  if (resident == 0) {
    int dev = 0, cus = 0, per_cu = 0;
    FE_HIP_CHECK(hipGetDevice(&dev));
    FE_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    FE_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_fdm_fused3_split<T, K, WYB, NB>, 64 * SP::WY, 0));
    resident = cus * (per_cu > 0 ? per_cu : 1);
  }
  const int len = split_chunk_len(n, (int64_t)nxt * nyt, resident);
  const int64_t blocks = (int64_t)nxt * nyt * ((n + len - 1) / len);
  const T* Seo = coef + p->co.off_Seo;
  const T* il = coef + p->co.off_il + (int64_t)li * M * M * M;
  ProfScope ps("fdm_fused", s);
  hipLaunchKernelGGL((k_fdm_fused3_split<T, K, WYB, NB>), dim3((unsigned)blocks), dim3(64 * SP::WY), 0, s, r, z, Seo, il, n,
                     nxt, nyt, len);
  FE_HIP_CHECK(hipGetLastError());
  return FE_OK;
}

fe_status launch_patch_lattice(const fe_problem* p, int level, const void* r, void* z, fe_dtype dt, hipStream_t s);

fe_status launch_patch_fused(const fe_problem* p, int level, const void* r, void* z, fe_dtype dt, hipStream_t s) {
  const int li = level < 0 ? (int)p->levels.size() - 1 : level;
  if (p->K == 4 && p->levels[li].n >= 2) return launch_patch_lattice(p, li, r, z, dt, s);
  if (dt == FE_F64) {
    if (p->K == 3) return fused_typed<double, 3>(p, li, (const double*)r, (double*)z, p->coef64.as<double>(), s);
    if (p->K == 4 && p->levels[li].n >= 2)
      return split_typed<double, 4, FE_SPLIT_WY, FE_SPLIT_NB>(p, li, (const double*)r, (double*)z, p->coef64.as<double>(), s);
    if (p->K == 4) return fused_typed<double, 4>(p, li, (const double*)r, (double*)z, p->coef64.as<double>(), s);
  } else {
    if (p->K == 3) return fused_typed<float, 3>(p, li, (const float*)r, (float*)z, p->coef32.as<float>(), s);
    if (p->K == 4 && p->levels[li].n >= 2)
      return split_typed<float, 4, FE_SPLIT_WY, FE_SPLIT_NB>(p, li, (const float*)r, (float*)z, p->coef32.as<float>(), s);
    if (p->K == 4) return fused_typed<float, 4>(p, li, (const float*)r, (float*)z, p->coef32.as<float>(), s);
  }
  return fail(FE_EUNSUPPORTED, "fused patch inverse: unsupported degree");
}

}  // namespace fe
