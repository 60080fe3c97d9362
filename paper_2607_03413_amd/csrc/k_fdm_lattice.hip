// Vertex-patch inverse on the 3D Cartesian mesh at degree 3 by sum
// factorization over the node lattice of a tile of patches.
//
// The operation is the additive Schwarz inverse of the vertex patches with
// fast diagonalization (Sec. 3.3 / Sec. 4.1 vertex-patch smoothers; the
// admissible form G P_CG G^T of eq. precond_consistency):
//   z = G sum_p R_p^T (S x S x S) L^{-1} (S x S x S)^T R_p G^T r,
// with L the sums of the 1D eigenvalues.  Along one axis the patch of vertex
// v covers the 5 nodes 3v-2 .. 3v+2; neighbouring windows share 2 nodes.
//
// Instead of one thread per patch (all 125 patch values in registers, each
// patch transformed on its own), the transforms are applied to the lattice
// of a tile of 7 x 10 patches, one patch level vz at a time, marching up in
// z:
//   * z: each lattice column (x, y node) forms its 5 z-values once (the
//     vertex plane sums its two copies) and takes them to the 5 z-modes; the
//     column is shared by every patch whose x-y window holds it, so this is
//     done once per node instead of once per patch node;
//   * x: per z-mode and lattice row, window px takes its 5 nodes (2 from the
//     lane below, by a DPP row shift) to 5 x-modes; the row is shared by the
//     patches of the tile's patch rows that hold it;
//   * y: per (z-mode, patch column, x-mode), the 32 lattice rows of the tile
//     go through the 10 windows; forward, scaling by the inverse eigenvalue
//     sums and backward are one symmetric 5 x 5 operator per task, applied as
//     a 3 x 3 block to the window's mirror sums and a 2 x 2 block to its
//     mirror differences (13 instead of 26 multiply-adds per window); the
//     overlapping rows of consecutive windows are summed in registers;
//   * back along x (the window's 2 lower nodes go to the lane below) and z
//     (the 2 upper planes are kept as partial sums for the next level).
// The x-modes sit in LDS between the x and y passes (one array for the whole
// level; the lanes of cell X0-1, which have no window, read a zero window and
// write a discarded one, so that the x pass has no lane-dependent branch); all
// other values stay in registers.  A thread owns the nodes 0..2
// of one cell along x in one lattice row: 8 lanes are the cells X0-1 ..
// X0+6 of a row, the 32 lattice rows make a 256-thread block.  Narrow tiles
// keep the x-modes of a block at 45 KB (FP64), so that two blocks share a
// compute unit and one's memory phase overlaps the other's compute (15
// patches per row, one block per CU, measured 124 against 113 us FP64 at
// 64^3 when the two shapes were compared).
//
// Every node is summed in a fixed order (lower window first along each axis;
// in z the partial sums of the level below first), and every copy of a node
// is written from the one value, so the copies are bit-identical; nodes that
// two tiles both compute (the tiles overlap by one patch) are computed by the
// same arithmetic in both.
//
// Tiles: tile t along x has patches X0 .. X0+6 and owns the cells X0 ..
// X0+5 (the first also cell 0, the last everything up to n-1; the last tile
// is shifted down so that it ends at patch n-1).  Along y, 10 patches and 9
// cells.  Along z the mesh is cut into chunks of levels C0 .. C1; a chunk owns
// the cell layers C0 .. C1-1 and computes the levels C0 .. C1 (level C1 for
// the upper planes of layer C1-1; level C0's lower planes are the chunk
// below's).  Even chunks march up, odd chunks down, so that two neighbouring
// chunks read the layers they share at the same time (from L2 for the second).
//
// In FP64 the next level's input rows are loaded into registers while the
// current level computes, and waited for at the end of the level, before its
// stores are issued (with one counter for loads and stores, a later wait for
// loads would wait for the stores too); the stores are not waited for.  Rows
// are loaded and stored through raw buffer resources over one plane of a cell
// layer, so that lanes with nothing to load or store point past the range
// (loads return zeros, stores are dropped) instead of branching: 3-7% at 64^3.
#include "fe_internal.h"
#include "kernel_common.h"

namespace fe {

namespace {

constexpr int kLPX = 7;                   // patches per tile along x (lanes 1..7)
constexpr int kLX = kLPX + 1;             // lanes per lattice row (cells X0-1 .. X0+6)
constexpr int kLPY = 10;                  // patches per tile along y
constexpr int kLRows = 3 * (kLPY + 1) - 1;  // lattice rows per tile (32)
constexpr int kLThreads = kLX * kLRows;     // 256
constexpr int kLCols = kLPX * 5;            // (patch column, x-mode) pairs per row (35)
constexpr int kLYTasks = 5 * kLCols;        // y passes per level (175)
constexpr int kLX1 = 5 * kLRows * kLCols;   // x-modes of one level (5600 values)

// DPP row shifts (16-lane rows).  Lanes without a source get 0.  A 16-lane row
// holds two lattice rows of 8 lanes; a shift that crosses from one to the
// other only reaches lane 0 of a lattice row (shift up: its node 0 and its
// window inputs, which lane 0 does not use) or takes lane 0's values into
// lane 7 (shift down: lane 0 has no window, so its backward x-modes and its
// node 0 are exact zeros, as a lane past the row would give).
constexpr int kRowShr1 = 0x111;   // lane i takes lane i-1
constexpr int kRowShl1 = 0x101;   // lane i takes lane i+1

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// 1D transforms of one 5-node window with the mirror-symmetric patch
// eigenvectors (modes ordered evens first; SE = 3 x 3 even block, SO = 2 x 2
// odd block, both row = mode).
template <typename T>
__device__ __forceinline__ void fwd5(const T (&x)[5], T (&y)[5], const T* __restrict__ SE, const T* __restrict__ SO) {
  const T s0 = x[0] + x[4], s1 = x[1] + x[3], d0 = x[0] - x[4], d1 = x[1] - x[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) y[j] = fma(SE[3 * j + 2], x[2], fma(SE[3 * j + 1], s1, SE[3 * j] * s0));
#pragma unroll
  for (int j = 0; j < 2; ++j) y[3 + j] = fma(SO[2 * j + 1], d1, SO[2 * j] * d0);
}
template <typename T>
__device__ __forceinline__ void bwd5(const T (&y)[5], T (&x)[5], const T* __restrict__ SE, const T* __restrict__ SO) {
  T e[3], o[2];
#pragma unroll
  for (int a = 0; a < 3; ++a) e[a] = fma(SE[6 + a], y[2], fma(SE[3 + a], y[1], SE[a] * y[0]));
#pragma unroll
  for (int a = 0; a < 2; ++a) o[a] = fma(SO[2 + a], y[4], SO[a] * y[3]);
  x[0] = e[0] + o[0];
  x[4] = e[0] - o[0];
  x[1] = e[1] + o[1];
  x[3] = e[1] - o[1];
  x[2] = e[2];
}

// One row (4 values along x) of one z-plane of a cell.
template <typename T>
struct Row4 {
  T v[4];
};
template <typename T>
__device__ __forceinline__ Row4<T> load_row_buf(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
  typedef int v4i __attribute__((ext_vector_type(4)));
  Row4<T> r;
  if constexpr (sizeof(T) == 8) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2 a = __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
    const d2 b = __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(rs, off + 16, 0, 0));
    r.v[0] = a[0]; r.v[1] = a[1]; r.v[2] = b[0]; r.v[3] = b[1];
  } else {
    typedef float f4 __attribute__((ext_vector_type(4)));
    const f4 a = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
    r.v[0] = a[0]; r.v[1] = a[1]; r.v[2] = a[2]; r.v[3] = a[3];
  }
  return r;
}
template <typename T>
__device__ __forceinline__ void store_row_buf(__amdgpu_buffer_rsrc_t rs, uint32_t off, T a, T b, T c, T d) {
  typedef int v4i __attribute__((ext_vector_type(4)));
  if constexpr (sizeof(T) == 8) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(v4i, d2{a, b}), rs, off, 0, 0);
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(v4i, d2{c, d}), rs, off + 16, 0, 0);
  } else {
    typedef float f4 __attribute__((ext_vector_type(4)));
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(v4i, f4{a, b, c, d}), rs, off, 0, 0);
  }
}
template <typename T>
__device__ __forceinline__ void store_row(T* __restrict__ p, T a, T b, T c, T d) {
  if constexpr (sizeof(T) == 8) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    *reinterpret_cast<d2*>(p) = d2{a, b};
    *reinterpret_cast<d2*>(p + 2) = d2{c, d};
  } else {
    typedef float f4 __attribute__((ext_vector_type(4)));
    *reinterpret_cast<f4*>(p) = f4{a, b, c, d};
  }
}

}  // namespace

template <typename T, bool YFULL>
__global__ void __launch_bounds__(kLThreads) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 2)))
k_fdm_lattice3(const T* __restrict__ r, T* __restrict__ z,
                                                            const T* __restrict__ Seo, const T* __restrict__ il,
                                                            int n, int nxt, int nyt, int zlen) {
  // [z-mode][lattice row][patch column][x-mode], then a zero window (read by the
  // lanes of cell X0-1, which have no window of their own) and a window that the
  // same lanes write and nobody reads: no lane-dependent branch around the LDS
  // accesses of the x pass
  __shared__ T X1[kLX1 + 16];
  if (threadIdx.x < 16) X1[kLX1 + threadIdx.x] = T(0);   // ordered before its first read by the level's barriers
  const T* __restrict__ SE = Seo;
  const T* __restrict__ SO = Seo + 9;

  // XCD-aware block order: consecutive logical tiles land on the same XCD
  // (blocks are dealt to the 8 XCDs round-robin), so that the halo cells
  // shared by neighbouring tiles are read from the same L2.
  const int nb = gridDim.x;
  const int xcd = blockIdx.x & 7, q8 = nb >> 3, rem = nb & 7;
  const int logical = xcd * q8 + min(xcd, rem) + (int)(blockIdx.x >> 3);
  const int nzc = nb / (nxt * nyt);
  const int tz = logical % nzc, t2 = logical / nzc;
  const int ty = t2 % nyt, tx = t2 / nyt;
  const int X0 = tx == nxt - 1 ? max(1, n - kLPX) : 1 + (kLPX - 1) * tx;
  const int Y0 = ty == nyt - 1 ? max(1, n - kLPY) : 1 + (kLPY - 1) * ty;
  const int oxl = tx == 0 ? 0 : (kLPX - 1) * tx + 1, oxh = tx == nxt - 1 ? n - 1 : (kLPX - 1) * (tx + 1);
  const int oyl = ty == 0 ? 0 : (kLPY - 1) * ty + 1, oyh = ty == nyt - 1 ? n - 1 : (kLPY - 1) * (ty + 1);
  const int C0 = tz * zlen, C1 = min(n, C0 + zlen);

  const int tid = threadIdx.x;
  const int lam = tid % kLX, m = tid / kLX;            // lane in the row, lattice row
  const int mu = (m + 1) / 3, iy = (m + 1) - 3 * ((m + 1) / 3);   // cell row in the tile, local y index
  const int cx = X0 - 1 + lam, cy = Y0 - 1 + mu;
  const bool in_x = cx <= n - 1;                       // cx >= 0 always
  const bool own_x = in_x && cx >= oxl && cx <= oxh;
  const bool own_y = cy <= n - 1 && cy >= oyl && cy <= oyh;
  const bool copy_y = iy == 0;                         // the row is also row 3 of cell row cy-1
  const bool own_yc = copy_y && cy - 1 >= oyl && cy - 1 <= oyh;
  const int px = lam - 1;                              // this lane's x-window (none in lane 0)
  const int64_t K3 = 64, plane = (int64_t)n * n * K3;
  const int64_t row_off = ((int64_t)min(cx, n - 1) + (int64_t)n * min(cy, n - 1)) * K3 + iy * 4;
  const int64_t copy_off = ((int64_t)min(cx, n - 1) + (int64_t)n * max(cy - 1, 0)) * K3 + 3 * 4;
  const bool ld_row = in_x && cy <= n - 1;
  const bool ld_copy = in_x && copy_y && cy >= 1 && cy - 1 <= n - 1;

  // The y pass's operator for its (z-mode, x-mode): forward along y, scaling
  // by the inverse eigenvalue sums, backward along y is one symmetric 5 x 5
  // matrix S diag(il) S^T per task.  The eigenvectors are even or odd about
  // the middle node, so it maps the sums (x0+x4, x1+x3, x2) through a 3 x 3
  // block and the differences (x0-x4, x1-x3) through a 2 x 2 block:
  //   Me = SE^T diag(il_even) SE,  Mo = SO^T diag(il_odd) SO
  // (zero for windows of patches beyond the mesh, x > n-1).
  const int yj = tid / kLCols, ycol = tid - yj * kLCols, ypx = ycol / 5, yix = ycol - 5 * (ycol / 5);
  const bool ypx_ok = tid < kLYTasks && X0 + ypx <= n - 1;
  T Me[3][3], Mo[2][2];
  {
    T ily[5];
#pragma unroll
    for (int a = 0; a < 5; ++a) ily[a] = ypx_ok ? il[(yj * 5 + a) * 5 + yix] : T(0);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = a; b < 3; ++b) {
        T v = (SE[a] * ily[0]) * SE[b];
        v = fma(SE[3 + a] * ily[1], SE[3 + b], v);
        v = fma(SE[6 + a] * ily[2], SE[6 + b], v);
        Me[a][b] = Me[b][a] = v;
      }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = a; b < 2; ++b) {
        T v = (SO[a] * ily[3]) * SO[b];
        v = fma(SO[2 + a] * ily[4], SO[2 + b], v);
        Mo[a][b] = Mo[b][a] = v;
      }
  }

  // Input rows of one z-plane (own row and, in copy rows, row 3 of the cell row
  // below), read through a raw buffer resource covering the plane (iz) of cell
  // layer lz: a lane whose row lies outside the mesh points past the range
  // (offset 2^31, above any plane of n <= 2000) and a layer outside the mesh
  // gets an empty range, so that the buffer's range check returns the zeros,
  // with no branch and no zero fill; stores drop out-of-range writes alike.
  const uint32_t plane_bytes = (uint32_t)(plane * (int64_t)sizeof(T));
  const uint32_t boff_row = ld_row ? (uint32_t)(row_off * (int64_t)sizeof(T)) : 0x80000000u;
  const uint32_t boff_copy = ld_copy ? (uint32_t)(copy_off * (int64_t)sizeof(T)) : 0x80000000u;
  const uint32_t soff_row = own_x && own_y ? (uint32_t)(row_off * (int64_t)sizeof(T)) : 0x80000000u;
  const uint32_t soff_copy = own_x && own_yc ? (uint32_t)(copy_off * (int64_t)sizeof(T)) : 0x80000000u;
  auto load_plane = [&](int lz, int iz, Row4<T>& a, Row4<T>& b) {
    const bool lz_ok = lz >= 0 && lz <= n - 1;   // uniform
    const T* base = r + (int64_t)(lz_ok ? lz : 0) * plane + iz * 16;
    const int nrec = lz_ok ? (int)(plane_bytes - (uint32_t)(iz * 16 * (int)sizeof(T))) : 0;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(base), (short)0, nrec, 0x00020000);
    a = load_row_buf<T>(rs, boff_row);
    b = load_row_buf<T>(rs, boff_copy);
  };
  // the three own nodes of a loaded plane (x copies: local 3 of the lane below)
  auto gather = [&](const Row4<T>& a, const Row4<T>& b, T (&nd)[3]) {
    T v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = a.v[i] + b.v[i];
    nd[0] = v[0] + dpp<kRowShr1>(v[3]);
    nd[1] = v[1];
    nd[2] = v[2];
  };

  // Chunks march alternately up (even tz) and down (odd tz): two neighbouring
  // chunks reach the layers they both read at the same time (both at their
  // first level, or both at their last), so that one of them finds them in
  // L2.  Downward, the z window is taken in reverse (planes 3vz+2 .. 3vz-2):
  // the even modes of a reversed window are the same and the odd modes
  // exactly negated, so every plane comes out of the same additions as
  // upward, bit for bit.
  const bool down = (tz & 1) != 0;
  const int lvl0 = down ? C1 : C0;
  // p[0], p[1]: the first two planes of the window (upward 3vz-2, 3vz-1; downward
  // 3vz+2, 3vz+1), carried from the level before
  T p0[3], p1[3];
  {
    Row4<T> a0, b0, a1, b1;
    load_plane(down ? C1 : C0 - 1, down ? 2 : 1, a0, b0);
    load_plane(down ? C1 : C0 - 1, down ? 1 : 2, a1, b1);
    gather(a0, b0, p0);
    gather(a1, b1, p1);
  }
  // input of the level: (vz-1, iz 3) and (vz, 0) (the vertex plane's copies),
  // then upward (vz, 1), (vz, 2), downward (vz-1, 2), (vz-1, 1)
  Row4<T> ia[4], ib[4];
  auto load_level = [&](int vz) {
    load_plane(vz - 1, 3, ia[0], ib[0]);
    load_plane(vz, 0, ia[1], ib[1]);
    load_plane(down ? vz - 1 : vz, down ? 2 : 1, ia[2], ib[2]);
    load_plane(down ? vz - 1 : vz, down ? 1 : 2, ia[3], ib[3]);
  };
  // FP64 loads the next level's rows during the current level (two blocks per
  // compute unit, 201 VGPRs); FP32 loads a level's rows at its start and hides
  // the wait behind more blocks instead (88 VGPRs, five blocks per compute
  // unit; prefetching, at 111 VGPRs and four blocks, measured 59.1 against
  // 58.1 us at 64^3, and six blocks at 80 VGPRs spill: 68.0 us).
  constexpr bool PREFETCH = sizeof(T) == 8;
  if (PREFETCH) load_level(lvl0);
  T co0[3] = {T(0), T(0), T(0)}, co1[3] = {T(0), T(0), T(0)};   // partial sums of the window's first two planes

  for (int step = 0; step <= C1 - C0; ++step) {
    const int vz = down ? C1 - step : C0 + step;
    T p2[3], p3[3], p4[3];
    {
      if (!PREFETCH) load_level(vz);
      T s0[3], s1[3];
      gather(ia[0], ib[0], s0);
      gather(ia[1], ib[1], s1);
#pragma unroll
      for (int i = 0; i < 3; ++i) p2[i] = s0[i] + s1[i];
      gather(ia[2], ib[2], p3);
      gather(ia[3], ib[3], p4);
    }
    // The level's loads and stores are issued at a raised wavefront priority,
    // so that the other block's waves on the SIMD, in their compute phase, do
    // not hold them back (FP64 at 64^3: 102 -> 100 us).
    __builtin_amdgcn_s_setprio(3);
    if (PREFETCH && step + 1 <= C1 - C0) load_level(down ? vz - 1 : vz + 1);
    __builtin_amdgcn_s_setprio(0);
    T E[3][3], O[3][2];
    const bool level_ok = vz >= 1 && vz <= n - 1;   // uniform over the block
    if (!level_ok) {
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        E[i][0] = E[i][1] = E[i][2] = T(0);
        O[i][0] = O[i][1] = T(0);
      }
    } else {
      // z: the columns' 5 planes to the 5 z-modes
      T md[5][3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const T x[5] = {p0[i], p1[i], p2[i], p3[i], p4[i]};
        T y[5];
        fwd5(x, y, SE, SO);
#pragma unroll
        for (int j = 0; j < 5; ++j) md[j][i] = y[j];
      }
      // x: window px of each row, per z-mode, to the x-modes in LDS
#pragma unroll
      for (int j = 0; j < 5; ++j) {
        const T x[5] = {dpp<kRowShr1>(md[j][1]), dpp<kRowShr1>(md[j][2]), md[j][0], md[j][1], md[j][2]};
        T y[5];
        fwd5(x, y, SE, SO);
        T* dst = lam >= 1 ? X1 + ((j * kLRows + m) * kLPX + px) * 5 : X1 + kLX1 + 8;
#pragma unroll
        for (int a = 0; a < 5; ++a) dst[a] = y[a];
      }
      __syncthreads();
      // y: one (z-mode, patch column, x-mode) per thread, all windows
      if (tid < kLYTasks) {
        T* col = X1 + yj * kLRows * kLCols + ycol;
        T c0 = T(0), c1 = T(0);
#pragma unroll
        for (int py = 0; py < kLPY; ++py) {
          const int m0 = 3 * py;
          const T x[5] = {col[(m0 + 0) * kLCols], col[(m0 + 1) * kLCols], col[(m0 + 2) * kLCols],
                          col[(m0 + 3) * kLCols], col[(m0 + 4) * kLCols]};
          // (rows of patches beyond the mesh, y > n-1, exist only when the tile
          // is larger than the mesh)
          const bool ok = YFULL || Y0 + py <= n - 1;
          const T s0 = ok ? x[0] + x[4] : T(0), s1 = ok ? x[1] + x[3] : T(0), s2 = ok ? x[2] : T(0);
          const T d0 = ok ? x[0] - x[4] : T(0), d1 = ok ? x[1] - x[3] : T(0);
          T e[3], o[2];
#pragma unroll
          for (int a = 0; a < 3; ++a) e[a] = fma(Me[a][2], s2, fma(Me[a][1], s1, Me[a][0] * s0));
#pragma unroll
          for (int a = 0; a < 2; ++a) o[a] = fma(Mo[a][1], d1, Mo[a][0] * d0);
          col[(m0 + 0) * kLCols] = c0 + (e[0] + o[0]);
          col[(m0 + 1) * kLCols] = c1 + (e[1] + o[1]);
          col[(m0 + 2) * kLCols] = e[2];
          c0 = e[1] - o[1];
          c1 = e[0] - o[0];
        }
        col[(3 * kLPY) * kLCols] = c0;
        col[(3 * kLPY + 1) * kLCols] = c1;
      }
      __syncthreads();
      // back along x, then accumulate the z back-transform of each mode
#pragma unroll
      for (int j = 0; j < 5; ++j) {
        T y[5], w[5];
        const T* src = lam >= 1 ? X1 + ((j * kLRows + m) * kLPX + px) * 5 : X1 + kLX1;
#pragma unroll
        for (int a = 0; a < 5; ++a) y[a] = src[a];
        bwd5(y, w, SE, SO);
        const T v[3] = {w[2], w[3] + dpp<kRowShl1>(w[0]), w[4] + dpp<kRowShl1>(w[1])};
        // (the first even and the first odd mode start the accumulators)
        if (j == 0) {
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int a = 0; a < 3; ++a) E[i][a] = SE[a] * v[i];
        } else if (j < 3) {
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int a = 0; a < 3; ++a) E[i][a] = fma(SE[3 * j + a], v[i], E[i][a]);
        } else if (j == 3) {
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int a = 0; a < 2; ++a) O[i][a] = SO[a] * v[i];
        } else {
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int a = 0; a < 2; ++a) O[i][a] = fma(SO[2 * (j - 3) + a], v[i], O[i][a]);
        }
      }
      __syncthreads();   // every row has read its x-modes before the next level writes them
    }
    // the level's planes (upward; downward mirrored): 3vz-2 and 3vz-1 complete the
    // partial sums of the level before, 3vz is the vertex plane (two copies),
    // 3vz+1 and 3vz+2 start the next
    T w1[3], w2[3], w3[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      w1[i] = co0[i] + (E[i][0] + O[i][0]);
      w2[i] = co1[i] + (E[i][1] + O[i][1]);
      w3[i] = E[i][2];
      co0[i] = E[i][1] - O[i][1];
      co1[i] = E[i][0] - O[i][0];
    }
    auto store_plane = [&](int lz, int iz, const T (&w)[3]) {
      const T w3x = dpp<kRowShl1>(w[0]);   // local 3: node 0 of the next cell
      const int64_t zoff = (int64_t)lz * plane + iz * 16;
      // the owned row and copy row through a raw buffer resource over the plane:
      // lanes that own neither point past its range and their writes are dropped
      const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
          z + zoff, (short)0, (int)(plane_bytes - (uint32_t)(iz * 16 * (int)sizeof(T))), 0x00020000);
      store_row_buf<T>(rs, soff_row, w[0], w[1], w[2], w3x);
      store_row_buf<T>(rs, soff_copy, w[0], w[1], w[2], w3x);
      // domain boundary rows without a lattice row of their own: node rows 0 and 3n
      if (m == 0 && own_x && own_y && cy == 0) store_row(z + zoff + (row_off - 4), T(0), T(0), T(0), T(0));
      if (m == kLRows - 1 && own_x && own_y && cy == n - 1)
        store_row(z + zoff + (row_off + 4), T(0), T(0), T(0), T(0));
    };
    // The next level's rows have had the whole level to arrive: wait for them
    // here, before the stores, so that the wait at the next level's gather is
    // not also a wait for these stores.
    if (PREFETCH) __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
    __builtin_amdgcn_s_setprio(3);
    if (down ? vz < C1 : vz - 1 >= C0) {   // the window's first two planes are in an owned layer
      store_plane(down ? vz : vz - 1, down ? 2 : 1, w1);
      store_plane(down ? vz : vz - 1, down ? 1 : 2, w2);
    }
    if (vz - 1 >= C0) store_plane(vz - 1, 3, w3);
    if (vz < C1) store_plane(vz, 0, w3);
    __builtin_amdgcn_s_setprio(0);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      p0[i] = p3[i];
      p1[i] = p4[i];
    }
  }
}

bool lattice_patch_supported(const fe_problem* p) {
  return p->dim == 3 && p->k == 3 && p->co.off_il >= 0 && p->co.off_Seo >= 0;
}

template <typename T>
static fe_status lattice_typed(const fe_problem* p, int li, const T* r, T* z, const T* coef, hipStream_t s) {
  const Level& L = p->levels[li];
  const int n = L.n;
  // plane byte offsets fit the buffer resources' 31-bit ranges (n^2 64 8 < 2^31)
  if (n > 2000) return fail(FE_EUNSUPPORTED, "lattice patch inverse: more than 2000 cells per axis");
  const int nxt = n <= kLPX + 1 ? 1 : (n - kLPX - 1 + kLPX - 2) / (kLPX - 1) + 1;
  const int nyt = n <= kLPY + 1 ? 1 : (n - kLPY - 1 + kLPY - 2) / (kLPY - 1) + 1;
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    FE_HIP_CHECK(hipGetDevice(&dev));
    FE_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    if (cus < 1) cus = 1;
  }
  // z-chunk length that minimizes (blocks per compute unit) x (levels per
  // block): the blocks on a compute unit share its throughput, so this is the
  // time of the most loaded unit; a unit with fewer than two blocks is counted
  // as two, since one block alone cannot overlap its memory and compute
  // phases (at 64^3 this picks 5 levels, the measured best in FP64 and FP32)
  const int64_t columns = (int64_t)nxt * nyt;
  int len = n;
  double best = 1e300;
  for (int l = 1; l <= n; ++l) {
    const int64_t blocks = columns * ((n + l - 1) / l);
    const double cost = (double)std::max<int64_t>((blocks + cus - 1) / cus, 2) * (l + 1);
    if (cost < best) { best = cost; len = l; }
  }
  const int64_t blocks = columns * ((n + len - 1) / len);
  const T* Seo = coef + p->co.off_Seo;
  const T* il = coef + p->co.off_il + (int64_t)li * 125;
  ProfScope ps("fdm_lattice", s);
  if (n > kLPY)   // every tile's patch rows are in the mesh
    hipLaunchKernelGGL((k_fdm_lattice3<T, true>), dim3((unsigned)blocks), dim3(kLThreads), 0, s, r, z, Seo, il, n, nxt,
                       nyt, len);
  else
    hipLaunchKernelGGL((k_fdm_lattice3<T, false>), dim3((unsigned)blocks), dim3(kLThreads), 0, s, r, z, Seo, il, n, nxt,
                       nyt, len);
  FE_HIP_CHECK(hipGetLastError());
  return FE_OK;
}

fe_status launch_patch_lattice(const fe_problem* p, int level, const void* r, void* z, fe_dtype dt, hipStream_t s) {
  const int li = level < 0 ? (int)p->levels.size() - 1 : level;
  if (dt == FE_F64) return lattice_typed<double>(p, li, (const double*)r, (double*)z, p->coef64.as<double>(), s);
  return lattice_typed<float>(p, li, (const float*)r, (float*)z, p->coef32.as<float>(), s);
}

}  // namespace fe
