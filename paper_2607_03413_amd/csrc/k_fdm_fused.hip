// Fused vertex-patch inverse for the 3D Cartesian mesh at low degree
// (k = 2, 3), where one patch (m^3 = 27 or 125 values, m = 2k-1) fits in the
// registers of one thread.  At k = 3 it serves only meshes of one cell (no
// patch); larger k = 3 meshes take the lattice kernel (k_fdm_lattice.hip).
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

fe_status launch_patch_lattice(const fe_problem* p, int level, const void* r, void* z, fe_dtype dt, hipStream_t s);

fe_status launch_patch_fused(const fe_problem* p, int level, const void* r, void* z, fe_dtype dt, hipStream_t s) {
  const int li = level < 0 ? (int)p->levels.size() - 1 : level;
  if (p->K == 4 && p->levels[li].n >= 2) return launch_patch_lattice(p, li, r, z, dt, s);
  if (dt == FE_F64) {
    if (p->K == 3) return fused_typed<double, 3>(p, li, (const double*)r, (double*)z, p->coef64.as<double>(), s);
    if (p->K == 4) return fused_typed<double, 4>(p, li, (const double*)r, (double*)z, p->coef64.as<double>(), s);
  } else {
    if (p->K == 3) return fused_typed<float, 3>(p, li, (const float*)r, (float*)z, p->coef32.as<float>(), s);
    if (p->K == 4) return fused_typed<float, 4>(p, li, (const float*)r, (float*)z, p->coef32.as<float>(), s);
  }
  return fail(FE_EUNSUPPORTED, "fused patch inverse: unsupported degree");
}

}  // namespace fe
