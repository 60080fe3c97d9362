/* Plain C FP64 reference of the two Cartesian hot-path operators, written out
 * from their definitions (test infrastructure: only the tests and the
 * benchmark's CPU baseline load it; it shares nothing with the HIP library).
 *
 * Layouts are the oracle's (oracle/mesh.py): cells lexicographic (x fastest),
 * K^3 cell-wise entries per cell with the local node (ix, iy, iz) at
 * ix + K (iy + K iz); global nodes (gx, gy, gz) = k c + i at
 * gx + N (gy + N gz), N = k n + 1; patch interiors of vertex v hold the nodes
 * k (v-1) + o, o = 1 .. 2k-1, x fastest.
 *
 * Every output is computed by one thread from its inputs (OpenMP over cells,
 * nodes or patches; no accumulation across threads), so the results do not
 * depend on the thread count.
 */
#include <stdint.h>
#include <string.h>

/* y_K = A_K x_K for every cell, the copies of boundary nodes (Dirichlet) set to
 * zero in the input and in the output (the Dirichlet operator of Sec. 2.1 in
 * cell-wise form). A: K^3 x K^3 row-major element matrix, the same for every
 * cell of the uniform mesh. */
void oracle_apply_dirichlet(int k, int n, const double* A, const double* x, double* y) {
  const int K = k + 1, NL = K * K * K, N = k * n + 1;
  const int64_t cells = (int64_t)n * n * n;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < cells; ++e) {
    const int cx = (int)(e % n), cy = (int)((e / n) % n), cz = (int)(e / ((int64_t)n * n));
    double xm[4096];
    unsigned char bnd[4096];
    for (int i = 0; i < NL; ++i) {
      const int ix = i % K, iy = (i / K) % K, iz = i / (K * K);
      const int gx = k * cx + ix, gy = k * cy + iy, gz = k * cz + iz;
      bnd[i] = gx == 0 || gy == 0 || gz == 0 || gx == N - 1 || gy == N - 1 || gz == N - 1;
      xm[i] = bnd[i] ? 0.0 : x[e * NL + i];
    }
    for (int i = 0; i < NL; ++i) {
      double s = 0.0;
      for (int j = 0; j < NL; ++j) s += A[(int64_t)i * NL + j] * xm[j];
      y[e * NL + i] = bnd[i] ? 0.0 : s;
    }
  }
}

/* The cells c and local indices i with k c + i = g along one axis (one or two). */
static int axis_copies(int k, int n, int g, int* c, int* i) {
  int cnt = 0;
  const int c0 = g / k;
  if (c0 < n) { c[cnt] = c0; i[cnt] = g - k * c0; ++cnt; }
  if (g % k == 0 && c0 >= 1) { c[cnt] = c0 - 1; i[cnt] = k; ++cnt; }
  return cnt;
}

/* z = G sum_p R_p^T A_p^{-1} R_p G^T r on the uniform Cartesian mesh (the
 * additive vertex-patch inverse, eq. precond_consistency with the patch
 * smoother of Sec. 3.3), every interior patch with the same inverse Ainv
 * (M^3 x M^3 row-major, M = 2k - 1):
 *   g   = G^T r            (each global node sums its cell-wise copies),
 *   W_p = Ainv (R_p g)     (one dense product per patch),
 *   zg  = sum_p R_p^T W_p  (each node sums the patches whose interior holds it),
 *   z   = G zg.
 * g and zg: N^3 work arrays; W: (n-1)^3 M^3. */
void oracle_patch_inverse(int k, int n, const double* Ainv, const double* r, double* z, double* g, double* zg,
                          double* W) {
  const int K = k + 1, NL = K * K * K, N = k * n + 1, M = 2 * k - 1, MP = M * M * M, nv = n - 1;
  const int64_t nodes = (int64_t)N * N * N;
#pragma omp parallel for schedule(static)
  for (int64_t q = 0; q < nodes; ++q) {
    const int g3[3] = {(int)(q % N), (int)((q / N) % N), (int)(q / ((int64_t)N * N))};
    int c[3][2], li[3][2], cnt[3];
    for (int a = 0; a < 3; ++a) cnt[a] = axis_copies(k, n, g3[a], c[a], li[a]);
    double s = 0.0;
    for (int a = 0; a < cnt[2]; ++a)
      for (int b = 0; b < cnt[1]; ++b)
        for (int d = 0; d < cnt[0]; ++d) {
          const int64_t e = c[0][d] + (int64_t)n * (c[1][b] + (int64_t)n * c[2][a]);
          s += r[e * NL + li[0][d] + K * (li[1][b] + K * li[2][a])];
        }
    g[q] = s;
  }
  const int64_t patches = (int64_t)nv * nv * nv;
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < patches; ++p) {
    const int vx = 1 + (int)(p % nv), vy = 1 + (int)((p / nv) % nv), vz = 1 + (int)(p / ((int64_t)nv * nv));
    double v[3375];
    for (int o = 0; o < MP; ++o) {
      const int ox = 1 + o % M, oy = 1 + (o / M) % M, oz = 1 + o / (M * M);
      v[o] = g[(k * (vx - 1) + ox) + (int64_t)N * ((k * (vy - 1) + oy) + (int64_t)N * (k * (vz - 1) + oz))];
    }
    for (int i = 0; i < MP; ++i) {
      double s = 0.0;
      for (int j = 0; j < MP; ++j) s += Ainv[(int64_t)i * MP + j] * v[j];
      W[p * MP + i] = s;
    }
  }
#pragma omp parallel for schedule(static)
  for (int64_t q = 0; q < nodes; ++q) {
    const int g3[3] = {(int)(q % N), (int)((q / N) % N), (int)(q / ((int64_t)N * N))};
    /* patches v with k (v-1) < g < k (v+1), 1 <= v <= n-1, and the interior offset g - k (v-1) */
    int pv[3][2], po[3][2], cnt[3];
    for (int a = 0; a < 3; ++a) {
      cnt[a] = 0;
      for (int v = g3[a] / k; v <= g3[a] / k + 1; ++v)
        if (v >= 1 && v <= nv && k * (v - 1) < g3[a] && g3[a] < k * (v + 1)) {
          pv[a][cnt[a]] = v;
          po[a][cnt[a]] = g3[a] - k * (v - 1);
          ++cnt[a];
        }
    }
    double s = 0.0;
    for (int a = 0; a < cnt[2]; ++a)
      for (int b = 0; b < cnt[1]; ++b)
        for (int d = 0; d < cnt[0]; ++d) {
          const int64_t p = (pv[0][d] - 1) + (int64_t)nv * ((pv[1][b] - 1) + (int64_t)nv * (pv[2][a] - 1));
          s += W[p * MP + (po[0][d] - 1) + M * ((po[1][b] - 1) + M * (po[2][a] - 1))];
        }
    zg[q] = s;
  }
  const int64_t cells = (int64_t)n * n * n;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < cells; ++e) {
    const int cx = (int)(e % n), cy = (int)((e / n) % n), cz = (int)(e / ((int64_t)n * n));
    for (int i = 0; i < NL; ++i) {
      const int ix = i % K, iy = (i / K) % K, iz = i / (K * K);
      z[e * NL + i] = zg[(k * cx + ix) + (int64_t)N * ((k * cy + iy) + (int64_t)N * (k * cz + iz))];
    }
  }
}

int oracle_max_threads(void) {
#ifdef _OPENMP
  extern int omp_get_max_threads(void);
  return omp_get_max_threads();
#else
  return 1;
#endif
}
