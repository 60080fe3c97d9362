/*
 * fe.h - C ABI of the MI355X cell-wise matrix-free Q_k finite element library.
 *
 * Method: W. Wichrowski, "Coalesced Matrix-Free Geometric Multigrid on
 * Persistent Cell-Wise Storage".  Every vector lives in redundant cell-wise
 * storage (Sec. 2.1): each cell keeps its own copy of all (k+1)^d nodal DoFs
 * it touches.  Primal vectors (iterates, corrections) are continuous: all
 * copies of a DoF agree.  Dual vectors (residuals, operator outputs) hold
 * unassembled partial integrals: only the sum of the copies is meaningful.
 *
 * Layout of a cell-wise vector (host or device, dtype given per call):
 *   n_cells blocks of (k+1)^d contiguous values, cell index
 *   e = cx + n*cy (+ n^2*cz), local index i = ix + K*iy (+ K^2*iz), K = k+1,
 *   x fastest.  The mesh is the unit square/cube split into n^d equal cells.
 * Global (assembled) vectors are indexed by node (gx, gy, gz), g = k*c + i,
 *   on the (k n + 1)^d grid, x fastest.
 *
 * Ownership: every pointer argument to a compute call is a DEVICE pointer
 * owned by the caller (e.g. a torch tensor); the library never frees it.
 * Buffers must be 16-byte aligned.  The library owns the setup data behind
 * the fe_problem handle and releases it in fe_problem_destroy.
 *
 * Streams: `stream` is a hipStream_t (NULL = the default stream).  Compute
 * calls are asynchronous on that stream unless stated otherwise.  Calls on one
 * problem handle must not overlap on different streams.
 *
 * Errors: every call returns an fe_status and never throws.  On a non-OK
 * status, fe_last_error() returns a thread-local description.  Output buffers
 * are left unspecified after an error.
 */
#ifndef FE_H
#define FE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fe_problem fe_problem;

typedef enum {
  FE_OK = 0,
  FE_EINVAL = -1,       /* bad argument: null pointer, misaligned buffer, unsupported (d,k), ... */
  FE_ENOMEM = -2,       /* a device or host allocation failed */
  FE_EHIP = -3,         /* a HIP runtime call failed */
  FE_ENOTCONV = -4,     /* iteration limit reached; x holds the last iterate */
  FE_EBREAKDOWN = -5,   /* CG breakdown: <p, A p> <= 0 or <r, z> <= 0, or a non-finite value */
  FE_EUNSUPPORTED = -6  /* valid request that the library does not implement */
} fe_status;

typedef enum { FE_F64 = 0, FE_F32 = 1 } fe_dtype;

typedef enum { FE_GEOM_CARTESIAN = 0, FE_GEOM_DEFORMED = 1 } fe_geometry;

/* Smooth coefficient field kappa(x) = exp(g(x)),
 *   g(x) = s * sum_j amp[j] * cos(pi * (m_j . x) + phase[j]),
 * with s chosen so that max |g| over the quadrature points equals 1
 * (host arrays, read during fe_problem_create only).  n_modes = 0 means kappa = 1. */
typedef struct {
  int n_modes;
  const int32_t* modes;    /* n_modes x 3, (mx, my, mz) */
  const double* amp;       /* n_modes */
  const double* phase;     /* n_modes */
} fe_coefficient;

typedef struct {
  int dim;                 /* 2 or 3 */
  int degree;              /* k, 1..8 */
  int n;                   /* cells per direction on the finest level */
  int geometry;            /* fe_geometry */
  double deform_amp;       /* deformed geometry: x_a += amp * prod_b sin(2 pi x_b), each a */
  fe_coefficient coef;     /* deformed geometry only; ignored for Cartesian */
  int bc;                  /* 0: no boundary condition (A 1 = 0); 1: homogeneous Dirichlet */
  int n_coarse;            /* cells per direction on the coarsest level (0: smallest possible) */
} fe_problem_desc;

/* Sec. 2 (model problem) and Sec. 3 (hierarchy T_0 < ... < T_L by uniform
 * bisection).  Builds the level hierarchy and the per-problem constant data
 * (1D reference matrices, patch eigen-data, geometry for the deformed case)
 * on the device of `stream`.  Synchronous. */
fe_status fe_problem_create(const fe_problem_desc* desc, void* stream, fe_problem** out);
void fe_problem_destroy(fe_problem* prob);

int64_t fe_num_cells(const fe_problem* prob);      /* n^d on the finest level */
int64_t fe_cellvec_len(const fe_problem* prob);    /* n^d (k+1)^d */
int64_t fe_num_dofs(const fe_problem* prob);       /* (k n + 1)^d unique DoFs */
int fe_num_levels(const fe_problem* prob);         /* L + 1 */
int fe_level_cells_1d(const fe_problem* prob, int level);   /* n_l, level 0 = coarsest */

/* Sec. 2.1: gather G (replicate global coefficients into every cell copy).
 * x_glob: (k n+1)^d values; x_cell: cell-wise, finest level.  Bit-exact copy. */
fe_status fe_gather(const fe_problem* prob, const void* x_glob, void* x_cell, fe_dtype dt, void* stream);

/* Sec. 2.1: assembly G^T (sum all cell copies of each global DoF). */
fe_status fe_assemble(const fe_problem* prob, const void* y_cell, void* y_glob, fe_dtype dt, void* stream);

/* Sec. 4.1 eq. dss_operator (averaging = 0): S v = G G^T v, in place, every
 * copy receives the sum of all copies.  Sec. 5 eq. averaging_dss
 * (averaging = 1): S_bar v = G (G^T G)^{-1} G^T v.  Copies are summed in the
 * order of the axis-split cascade of Algorithm 7 (x pairs, then y, then z),
 * so the result equals that cascade bit for bit.  `level` selects the mesh
 * level (-1 = finest). */
fe_status fe_dss(const fe_problem* prob, int level, void* v_cell, int averaging, fe_dtype dt, void* stream);

/* Sec. 2.1 (cell-wise operator A: V_cell -> V_cell^*) and Sec. 6 (cube:
 * (D x B x B + B x D x B + B x B x D) det(J) J^-2; deformed: general
 * cell-wise Laplacian with coefficient).  y = A x cell by cell (dual output,
 * unassembled).  x should be continuous.  With bc = 1 the boundary copies of
 * x are treated as zero and the boundary copies of y are set to zero.
 * x and y must not alias. */
fe_status fe_apply(const fe_problem* prob, const void* x_cell, void* y_cell, fe_dtype dt, void* stream);
fe_status fe_apply_level(const fe_problem* prob, int level, const void* x_cell, void* y_cell,
                         fe_dtype dt, void* stream);

/* Geometry traffic of the deformed operator (Sec. 6.4: on curved meshes the
 * per-point metric terms, not the DoF data, fill the memory bandwidth).
 * mode 0 (default): the general apply streams the 6 metric entries stored per
 * Gauss point.  mode 1: it forms the metric in the kernel from the map (the
 * shift of this geometry is the same separable field in every coordinate, so
 * J = I / n + 1 (grad S)^T has a closed-form inverse and determinant built
 * from 1D tables per cell) and streams only the coefficient per point: 1
 * value instead of 6.  The first switch to mode 1 computes the coefficient
 * arrays (setup, allocates).  Same operator to rounding; the setup kernels
 * (diagonal, per-patch factors) keep using the stored metric.  Deformed
 * geometry only. */
fe_status fe_set_metric_mode(fe_problem* prob, int mode, void* stream);

/* Vertex-patch additive Schwarz inverse, an admissible smoother of the form
 * P = G P_CG G^T (Sec. 2.1 eq. precond_consistency; Sec. 3.3 and Sec. 4.1
 * name overlapping vertex-patch smoothers as substitutes):
 *   z = G sum_p R_p^T A_p^{-1} R_p G^T r,
 * p over the interior mesh vertices, R_p the (2k-1)^d DoFs strictly inside
 * the 2^d cells around the vertex.  A_p^{-1} is applied by fast
 * diagonalization with 1D generalized eigenpairs (K S = M S Lambda).
 *   factors = 0: exact separable factors (Cartesian mesh only),
 *   factors = 1: per-patch averaged-geometry factors (deformed mesh),
 *   factors = 2: per-patch learned factors (after fe_mlp_train),
 *   factors = 3: per-patch best Kronecker-sum fit of A_p (the learned model's
 *                training target, computed per patch at setup; the reference
 *                the learned factors approximate).
 * r: dual cell-wise; z: primal cell-wise (continuous, copies bit-identical).
 * The result depends only on G^T r.  r and z must not alias. */
fe_status patch_fdm_inverse(const fe_problem* prob, const void* r_cell, void* z_cell, fe_dtype dt,
                            int factors, void* stream);
fe_status patch_fdm_inverse_level(const fe_problem* prob, int level, const void* r_cell, void* z_cell,
                                  fe_dtype dt, int factors, void* stream);

/* Set-up of patch_fdm_inverse on (level, dt, factors): the per-patch factors
 * of `factors` (deformed mesh: quadrature inner products, eigensolves, model
 * inference) and, where the two-pass kernels serve the problem (k >= 4, k = 1,
 * d = 2, per-patch factors), the patch-solution scratch in dtype dt, owned by
 * the problem until fe_problem_destroy.  Synchronous.  patch_fdm_inverse on a
 * prepared (level, dt, factors) allocates nothing; on an unprepared one it
 * runs this set-up first.  pcg_solve prepares every level it smooths on. */
fe_status fe_patch_prepare(fe_problem* prob, int level, fe_dtype dt, int factors, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation as patch_fdm_inverse_level, bit for bit, with the two-pass
 * kernels' patch-solution scratch taken from a fixed device array of
 * fe_noalloc_scratch_bytes() = 64 MiB that the library holds on every GPU it
 * runs on until the process ends.  No hipMalloc, hipFree or other allocating
 * call is made.  Errors: FE_EINVAL when the scratch this (level, dt) needs
 * (patch_fdm_inverse's two-pass kernels: (n_l - 1)^d patches x 8 k^3 values in
 * 3D, x (2k-1)^2 in 2D) exceeds 64 MiB, or when factors >= 1 and the per-patch
 * factors of that level were not set up (call fe_patch_prepare first, which
 * does allocate); the scratch-free one-pass kernels (3D Cartesian, k = 2, 3)
 * have no size limit.  All calls on one GPU share the one array: calls that
 * overlap in time on one GPU (different streams or threads) race and give
 * wrong results.  The array keeps the last call's contents; every entry a
 * call reads is written by that call first. */
size_t fe_noalloc_scratch_bytes(void);
fe_status patch_fdm_inverse_noalloc(const fe_problem* prob, int level, const void* r_cell, void* z_cell,
                                    fe_dtype dt, int factors, void* stream);

/* Sec. 3.1 Algorithm 2: e_fine += (P_b1 x P_b2 x P_b3) e_coarse on every
 * child, level `fine_level` >= 1.  Continuous in, continuous out (lemma on
 * commutativity of prolongation). */
fe_status fe_prolongate_add(const fe_problem* prob, int fine_level, const void* e_coarse, void* e_fine,
                            fe_dtype dt, void* stream);

/* Sec. 3.1 Algorithm 3 with the fused residual of Sec. 5:
 * b_coarse = sum_c (P_b1^T x ...) (b_fine - v_fine)|child c (overwrites b_coarse).
 * v_fine may be NULL (treated as zero).  Unassembled in, unassembled out. */
fe_status fe_restrict_residual(const fe_problem* prob, int fine_level, const void* b_fine,
                               const void* v_fine, void* b_coarse, fe_dtype dt, void* stream);

/* Sec. 5 Algorithm 9, one fused masked Jacobi sweep on `level`:
 *   v = A u;  u += omega * Dhat^{-1} (b - v);  u = S_bar u,
 * Dhat^{-1} = valence / assembled diagonal, zero on Dirichlet DoFs.
 * v is caller scratch (cell-wise, same dtype).  If u_is_zero, v = A u is skipped. */
fe_status fe_jacobi_sweep(const fe_problem* prob, int level, const void* b, void* u, void* v,
                          double omega, int u_is_zero, fe_dtype dt, void* stream);

/* Manufactured load vector of the model problem (Sec. 2, eq. poisson):
 * b_K,i = int_K f phi_i with f = d pi^2 prod_a sin(pi x_a) (mapped through
 * the geometry, times the coefficient if any), Gauss rule with k+2 points per
 * direction.  FP64 output, dual cell-wise. */
fe_status fe_rhs_manufactured(const fe_problem* prob, void* b_cell, void* stream);

/* Energy pairing of Sec. 3.4 eq. energy_measure and friends: local
 * Euclidean pairing sum_i a_i b_i over the cell-wise vectors (FP64 result,
 * FP64 accumulation, deterministic).  Synchronous. */
fe_status fe_dot(const fe_problem* prob, const void* a, const void* b, fe_dtype dt, double* out, void* stream);

/* ||G^T r||_2^2 for a dual cell-wise vector (assembled residual norm), FP64
 * accumulation.  Synchronous. */
fe_status fe_assembled_norm2(const fe_problem* prob, const void* r_cell, fe_dtype dt, double* out,
                             void* stream);

typedef enum { FE_SMOOTH_JACOBI = 0, FE_SMOOTH_CHEB_FDM = 1 } fe_smoother;

typedef struct {
  double tol;              /* stop when ||G^T r||_2 <= tol * ||G^T b||_2 */
  int maxit;
  int nu_pre, nu_post;     /* smoothing sweeps per level */
  int smoother;            /* fe_smoother */
  int cheb_degree;         /* Chebyshev degree (smoother = 1) */
  double cheb_ratio;       /* interval [lmax/ratio, lmax] */
  double cheb_lmax;        /* > 0: lmax, the top of the interval, on every level, taken as given;
                              0: per level 1.2 x a 15-step Lanczos estimate of lambda_max(P A) */
  double omega;            /* Jacobi relaxation (smoother = 0); 0: per level 4/(3 lambda_max(D^-1 A)) */
  int inner;               /* fe_dtype of the V-cycle (FE_F32: FP32 preconditioner) */
  int factors;             /* patch factors for smoother = 1 (see patch_fdm_inverse) */
  int flexible;            /* 1: Polak-Ribiere beta (recommended with inner = FE_F32) */
  int precond;             /* 1: V-cycle preconditioner, 0: none (plain CG) */
  int stop;                /* 0: stop when ||G^T r||_2 <= tol ||G^T b||_2;
                              1: stop when the energy pairing of the residual with its
                                 preconditioned form, gamma = <r, M r> (Sec. 3.4 eq. energy_measure,
                                 the square of a preconditioner-induced norm), has fallen to
                                 tol * gamma_0 (Sec. 6 uses a 1e-14 reduction) */
} fe_pcg_opts;

typedef struct {
  int iters;
  int converged;
  double relres;           /* ||G^T r||_2 / ||G^T b||_2 at exit */
  double energy0, energy;  /* <r, z> at start and exit */
  double t_setup, t_solve; /* seconds (host wall clock, synchronized) */
} fe_pcg_report;

/* Fill opts with defaults: tol 1e-10, maxit 200, nu 2/2, Jacobi omega 0.7,
 * Chebyshev degree 3, ratio 20, FP64 inner, standard beta. */
void fe_pcg_default_opts(fe_pcg_opts* opts);

/* Sec. 4.4: conjugate gradients in primal-dual form, preconditioned by the
 * cell-wise V-cycle of Algorithm 1 (zero initial guess, Sec. 5), coarse
 * solve by a dense FP64 inverse.  b: dual FP64 (its boundary copies carry no
 * equation and are ignored); x: primal FP64, initial guess on input (boundary
 * copies set to zero), solution on output.  Setup (levels, diagonals, lambda_max
 * estimates) happens on the first call with a given opts and is kept in the
 * handle.  Synchronous; fills `report` if non-NULL.  Returns FE_ENOTCONV if
 * maxit was reached. */
fe_status pcg_solve(fe_problem* prob, const void* b_cell, void* x_cell, const fe_pcg_opts* opts,
                    fe_pcg_report* report, void* stream);

/* Sec. 6.1: the V-cycle as a stationary iteration, x <- x + MG(b - A x),
 * `cycles` times (Algorithm 1 with opts' smoother, sweeps and precision),
 * recording after each cycle c the energy measure eta[c] = <b - A x, x> (Sec.
 * 3.4 eq. energy_measure: a dual paired with a primal vector, no assembly)
 * and res[c] = ||G^T (b - A x)||_2.  b: dual FP64 (boundary copies ignored);
 * x: primal FP64, initial guess in (boundary copies set to zero), last
 * iterate out.  eta, res: HOST arrays of `cycles` doubles, either may be NULL.
 * Synchronous. */
fe_status fe_mg_iterate(fe_problem* prob, const void* b_cell, void* x_cell, const fe_pcg_opts* opts, int cycles,
                        double* eta, double* res, void* stream);

/* One application of the V-cycle preconditioner e = MG(b) (Algorithm 1 with
 * a zero initial guess) on the finest level, in opts->inner precision.
 * b: dual, e: primal, both in dtype `dt` == opts->inner. */
fe_status fe_vcycle(fe_problem* prob, const void* b_cell, void* e_cell, const fe_pcg_opts* opts,
                    fe_dtype dt, void* stream);

/* lambda_max estimate of P A on `level` by `steps` Lanczos steps (CG
 * coefficients) from a fixed start vector; P = patch inverse (smoother =
 * FE_SMOOTH_CHEB_FDM) or Jacobi D^{-1} (smoother = FE_SMOOTH_JACOBI).  Synchronous. */
fe_status fe_estimate_lmax(fe_problem* prob, int level, int smoother, int factors, int steps,
                           double* out, void* stream);

/* ---- Learned per-patch factors (deformed geometry; factors = 2 above) ----
 * The paper's admissible smoother class (eq. precond_consistency) admits any
 * patch solver; on the deformed mesh the separable surrogate
 *   A_sep = Kx (x) My (x) Mz + Mx (x) Ky (x) Mz + Mx (x) My (x) Kz
 * has 12 weights per patch (alpha_{d,c} scale D on interval c of axis d in
 * K_d, beta_{d,c} scale B in M_d), stored as
 *   [alpha_x0, alpha_x1, alpha_y0, alpha_y1, alpha_z0, alpha_z1, beta_x0, ..., beta_z1].
 * A 64 -> 64 -> 64 -> 12 MLP (tanh, FP32) predicts their normalized logs
 * t = P(log w - log(h)/3) (P removes the 3 scaling gauges) from 64 patch
 * features.  All arrays are DEVICE pointers, row-major, one row per patch
 * (patch index (vx-1) + (n-1)((vy-1) + (n-1)(vz-1)), interior vertices). */

int fe_mlp_num_params(void);                                  /* 9100 */
int64_t fe_num_patches(const fe_problem* prob, int level);    /* (n_l - 1)^d */

/* Features (FP64, n_patches x 64): per cell slot s = sx + 2 sy + 4 sz, the
 * entries (xx, yy, zz, xy, xz, yz) of n kappa det(J) J^-1 J^-T at the cell
 * centre, log kappa and log(n^3 det J) there. */
fe_status fe_patch_features(fe_problem* prob, int level, double* feats, void* stream);

/* C[p][i + 4 j + 16 l] = <A_p, E_l (x) E_j (x) E_i>_F, E in {D on interval 0,
 * D on interval 1, B on 0, B on 1} (FP64, n_patches x 64), from the metric. */
fe_status fe_patch_inner_tensor(fe_problem* prob, int level, double* C, void* stream);

/* Training targets (FP64, n_patches x 12): normalized log-weights of the best
 * Kronecker-sum fit min ||A_p - A_sep(w)||_F by `sweeps` sweeps of alternating
 * least squares (stiffness weights, then masses of x, y, z) from the
 * averaged-geometry weights. */
fe_status fe_patch_fit_targets(fe_problem* prob, int level, int sweeps, double* targets, void* stream);

/* Model parameters (FP32, fe_mlp_num_params() values: W1 64x64, b1, W2 64x64,
 * b2, W3 12x64, b3; W row-major [out][in]).  set_params also resets Adam. */
fe_status fe_mlp_set_params(fe_problem* prob, const float* params, void* stream);
fe_status fe_mlp_get_params(const fe_problem* prob, float* params, void* stream);
/* Y (n x 12) = model(X (n x 64)), FP32. */
fe_status fe_mlp_forward(fe_problem* prob, const float* X, float* Y, int n, void* stream);
/* Mean squared error over the n x 12 outputs and its gradient (FP32, same layout as the parameters). */
fe_status fe_mlp_loss_grad(fe_problem* prob, const float* X, const float* T, int n, float* grad, double* loss,
                           void* stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with the given gradient. */
fe_status fe_mlp_adam_step(fe_problem* prob, const float* grad, double lr, void* stream);
/* Minibatch Adam training: `epochs` passes over a permutation of the n rows
 * (splitmix64 shuffle from `seed`), batches of `batch` rows (the last partial
 * batch is dropped).  final_loss: mean loss of the last epoch.  Synchronous. */
fe_status fe_mlp_train(fe_problem* prob, const float* X, const float* T, int n, int epochs, int batch, double lr,
                       uint64_t seed, double* final_loss, void* stream);

/* Per-kernel timing with HIP events on the launch stream (tracing aid).
 * enable = 1 starts recording, 0 stops; reset clears.  fe_prof_query
 * synchronizes and returns, for kernel family `name`, the number of launches
 * and the summed duration in milliseconds. */
void fe_prof_enable(int enable);
void fe_prof_reset(void);
fe_status fe_prof_query(const char* name, int* count, double* total_ms);

/* pcg_solve replays the preconditioner application z = M r (one V-cycle and
 * its conversions, a fixed sequence of kernel launches per setup) as a HIP
 * graph from its third application on: the first runs eagerly (it performs any
 * first-use allocation), the second is captured.  pcg_solve runs on a stream
 * of its own (capture needs a non-null stream), after the caller's stream has
 * drained; the result is complete when it returns, as before.  enable = 0
 * keeps every application eager (default 1).  Not used while per-kernel
 * timing is on, or for the Jacobi smoother with an odd number of sweeps
 * (whose sweeps alternate buffers between applications).  Process-wide. */
void fe_set_graphs(int enable);

/* ---- Locally refined meshes: local multigrid (Sec. 3.2, Algorithms 4-5) ----
 * The unit cube refined as an octree: levels 0..g uniform (level l has 2^l
 * cells per direction), then up to `adaptive_refinements` levels on which only
 * the cells near a feature are refined, 2:1 balanced across faces, edges and
 * vertices.  The level mesh T_l holds ALL level-l cells (active leaves and
 * cells refined further); level 0 is the single cell of the cube.  Storage:
 * level l >= 1 lists its cells in bricks of 8, the children (c = bx + 2 by +
 * 4 bz) of the refined level-(l-1) cells taken in their order; each cell keeps
 * (k+1)^3 values (local index x fastest).  A vector of the active mesh is kept
 * in LEVEL LAYOUT: the level blocks concatenated (offsets from
 * fe_adaptive_level_offset), zeros on refined cells.  Primal vectors are
 * continuous on the active mesh (hanging copies interpolate the coarse side);
 * dual vectors are unassembled.  Homogeneous Dirichlet conditions on the cube.
 * FP64 only; all vector pointers are device pointers owned by the caller.
 * No hanging-node constraint is stored or applied: the smoother masks the
 * refinement edge E_l (found at setup by one DSS of a face marker, Sec. 5) on
 * both sides of the structured DSS cascade (Sec. 4.3), and the transfers act
 * on unassembled residuals (lemma on the residual transfer). */
typedef struct fe_adaptive fe_adaptive;
typedef enum { FE_FEATURE_SPHERE = 0, FE_FEATURE_POINT = 1 } fe_feature;
typedef struct {
  int degree;                /* k, 1..5 */
  int global_refinements;    /* g: uniform levels 0..g */
  int adaptive_refinements;  /* levels beyond g refined toward the feature (g + this <= 12) */
  int feature;               /* fe_feature */
  double center[3];          /* sphere centre / the point */
  double radius;             /* sphere radius */
  double band;               /* refine a level-l cell whose centre is within band * 2^-l of the feature
                                (dyadic centre, radius and band make the test exact) */
} fe_adaptive_desc;

/* Builds the tree, the per-level brick tables, the masked valence-baked
 * inverse diagonals (Algorithm 9) and the coarse solve.  Synchronous. */
fe_status fe_adaptive_create(const fe_adaptive_desc* desc, void* stream, fe_adaptive** out);
void fe_adaptive_destroy(fe_adaptive* a);
int fe_adaptive_num_levels(const fe_adaptive* a);                 /* L + 1 */
int64_t fe_adaptive_level_cells(const fe_adaptive* a, int level);  /* cells of T_l */
int64_t fe_adaptive_level_offset(const fe_adaptive* a, int level); /* level = L+1: total length */
int64_t fe_adaptive_active_cells(const fe_adaptive* a);            /* leaves */
/* Host copies: coords (n_cells x 3 int32, level-l integer cell coordinates),
 * refined (n_cells bytes); either may be NULL. */
fe_status fe_adaptive_level_info(const fe_adaptive* a, int level, int32_t* coords, uint8_t* refined);
/* Host copies for level >= 1: nbr (n_bricks x 6: brick of the -x, +x, -y, +y,
 * -z, +z neighbour, -1 if absent), parent (n_bricks: parent cell on level-1). */
fe_status fe_adaptive_brick_neighbors(const fe_adaptive* a, int level, int32_t* nbr, int32_t* parent);
/* Sec. 5, detection of the refinement edge: mask (device, level length) >= 1 on
 * the copies of E_l, 0 elsewhere -- the summed face marker. */
fe_status fe_adaptive_edge_mask(fe_adaptive* a, int level, double* mask, void* stream);
/* Algorithm 7 on level l (in place; averaging = 1: S_bar): the structured
 * cascade of brick and neighbour-brick pairs, pairs without a partner skipped. */
fe_status fe_adaptive_dss(fe_adaptive* a, int level, double* v, int averaging, void* stream);
/* Copy of the masked, valence-baked inverse diagonal of level >= 1 (Algorithm 9). */
fe_status fe_adaptive_dinv(const fe_adaptive* a, int level, double* dinv, void* stream);
/* y = A_act x over the level layout (cell by cell; refined cells give 0). */
fe_status fe_adaptive_apply(fe_adaptive* a, const double* x, double* y, void* stream);
/* Algorithm 2 / Algorithm 3 between level fine_level - 1 and fine_level
 * (level blocks, not the level layout): e_fine += P e_coarse on the children
 * of every refined coarse cell; b_coarse += R (b_fine - v_fine) on every
 * refined coarse cell. */
fe_status fe_adaptive_prolongate_add(fe_adaptive* a, int fine_level, const double* e_coarse, double* e_fine,
                                     void* stream);
fe_status fe_adaptive_restrict_add(fe_adaptive* a, int fine_level, const double* b_fine, const double* v_fine,
                                   double* b_coarse, void* stream);
/* Manufactured load vector on the active cells (f = 3 pi^2 prod sin(pi x_a)). */
fe_status fe_adaptive_rhs_manufactured(fe_adaptive* a, double* b, void* stream);
/* Algorithm 4 from a zero iterate: z = MG_local(r), level distribution of the
 * unassembled residual r, the local V-cycle of Algorithm 5 with opts' Jacobi
 * omega and sweeps (smoother = FE_SMOOTH_JACOBI, inner = FE_F64), reassembly
 * of the active components.  r, z: level layout. */
fe_status fe_adaptive_precondition(fe_adaptive* a, const double* r, double* z, const fe_pcg_opts* opts,
                                   void* stream);
/* CG in primal-dual form on the active mesh preconditioned by Algorithm 4;
 * opts->stop must be 1 (gamma = <r, z> reduced to tol * gamma_0; relres in the
 * report is sqrt(gamma / gamma_0)).  b: dual, x: primal initial guess in,
 * solution out (level layout; refined and Dirichlet copies are zeroed).
 * Synchronous. */
fe_status fe_adaptive_pcg(fe_adaptive* a, const double* b, double* x, const fe_pcg_opts* opts,
                          fe_pcg_report* report, void* stream);

/* ---- Multi-block meshes: inter-block DSS (Sec. 4.3, Algorithm 8) ----
 * A 7-block atlas: a centre cube and six caps between its faces and the faces
 * of the cube of twice its size, each block an n^3 grid of Q_k cells with its
 * own orientation (block b's lattice axes are permuted and flipped against its
 * neighbours'; the table is fixed in the library).  Macro-faces join 2 blocks,
 * macro-lines 2 or 3, macro-vertices 3 or 4.  Layout of a multi-block
 * cell-wise vector: the 7 blocks in order, each n^3 cells lexicographic,
 * (k+1)^3 values per cell (x fastest).  Degree 1..8; the vector length must
 * stay below 2^31 entries. */
typedef struct fe_multiblock fe_multiblock;
fe_status fe_multiblock_create(int degree, int n, void* stream, fe_multiblock** out);
void fe_multiblock_destroy(fe_multiblock* mb);
int64_t fe_multiblock_len(const fe_multiblock* mb);         /* 7 n^3 (k+1)^3 entries */
int64_t fe_multiblock_num_nodes(const fe_multiblock* mb);   /* unique DoFs of the glued mesh */
/* counts[0] macro-face copy pairs, counts[1] macro-line DoFs, counts[2] macro-vertex DoFs. */
fe_status fe_multiblock_counts(const fe_multiblock* mb, int64_t* counts);
/* S v = G G^T v in place (averaging = 1: S_bar v, the sum divided by the node's
 * copy count): the structured cascade inside every block, then the macro-face
 * pairs, macro-line and macro-vertex passes (one representative copy per
 * sharing block gathered, the total scattered to every copy). */
fe_status fe_multiblock_dss(fe_multiblock* mb, void* v, int averaging, fe_dtype dt, void* stream);

/* Thread-local description of the last non-OK status. */
const char* fe_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FE_H */
