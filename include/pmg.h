/*
 * pmg.h -- C ABI of the MI355X (gfx950) vertex-patch smoother with nested
 * matrix-free p-multigrid local solvers, and of the geometric-multigrid CG
 * built on it.
 *
 * Method (arXiv 2510.17785):
 *   problem      a(u,v) = int mu grad u . grad v on a structured quad/hex mesh,
 *                continuous Q_p elements, homogeneous Dirichlet conditions
 *                (Section 2, bilinear form and discrete problem)
 *   smoother     multiplicative vertex-patch smoother: gather, evaluate the
 *                local residual, solve locally, scatter-add (Section 2.1,
 *                Algorithm 1; equations gather, main:4, main:5, scatter)
 *   local solver p-multigrid V-cycle on the patch (Section 3.1, Algorithm 2):
 *                embedding/transpose transfers, rediscretised level operators,
 *                exact coarse solve at the lowest degree, Chebyshev-accelerated
 *                Jacobi smoothing (damped Jacobi is its degree-1 case)
 *   outer solver geometric multigrid V-cycle with one patch sweep per side
 *                (Section 2, Section 4), used as CG preconditioner
 *
 * Conventions shared by every entry point:
 *   - Global vectors are FP64, length (N p + 1)^dim, lexicographic with x
 *     fastest, and hold 0 on Dirichlet nodes.  Vertices are
 *     ((N+1)^dim x dim) FP64, x fastest; coefficients one FP64 per cell.
 *   - "host" pointers are read during the call and never kept; "device"
 *     pointers are device memory owned by the caller (for instance the
 *     data_ptr() of a torch tensor) and are not kept after the call returns.
 *   - Work is enqueued on opts.stream (a hipStream_t; NULL = the null stream)
 *     and runs asynchronously unless stated otherwise.
 *   - Every function returns a status: PMG_OK (0), a negative error code, or
 *     PMG_WARN_NOT_CONVERGED (+1).  Nothing throws across the ABI.
 *     pmg_last_error() returns the message of the last non-zero status of the
 *     calling thread.
 *   - Patches are numbered in sweep order: colours ascending, and within a
 *     colour vertices in lexicographic order (x fastest).  The colour of
 *     interior vertex v is sum_i 2^i (v_i mod 2).
 */
#ifndef PMG_H
#define PMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define PMG_OK 0
#define PMG_ERR_INVALID_ARG (-1)  /* null pointer, bad size, bad level list */
#define PMG_ERR_UNSUPPORTED (-2)  /* valid request the library has no kernel for */
#define PMG_ERR_DEGENERATE (-3)   /* a cell with det J <= 0 at a quadrature point */
#define PMG_ERR_HIP (-4)          /* a HIP runtime call failed */
#define PMG_ERR_OOM (-5)          /* device allocation failed */
#define PMG_ERR_BREAKDOWN (-6)    /* CG breakdown: p^T A p <= 0 or NaN */
#define PMG_WARN_NOT_CONVERGED 1  /* CG hit maxit; outputs are valid */

/* precision of the local p-multigrid (global vectors stay FP64) */
#define PMG_FP64 0
#define PMG_FP32 1
/* FP32 local p-multigrid whose top-level interpolation contractions take
 * BF16-rounded inputs on the matrix cores and accumulate in FP32; the
 * collocation derivatives, the metric, Chebyshev updates, diagonals and all
 * lower levels stay FP32.  3D top-level degrees 6 and 7 only (others return
 * PMG_ERR_UNSUPPORTED). */
#define PMG_BF16_FP32ACC 2
/* As PMG_BF16_FP32ACC with every operand split into two BF16 numbers
 * (x = hi + lo, hi = bf16(x), lo = bf16(x - hi)) and three products per
 * tile (hi hi + hi lo + lo hi), accumulated in FP32: about 16 significant
 * bits per operand instead of 8. */
#define PMG_BF16X3_FP32ACC 3

/* source of the Chebyshev eigenvalue bounds */
#define PMG_BOUNDS_LANCZOS 0  /* per-patch Lanczos at setup */
#define PMG_BOUNDS_FIXED 1    /* caller sets them with pmg_set_bounds */

/* which vertices get a patch (Section 2.1: the patch of a vertex is the
 * set of cells sharing it).  PMG_PATCH_WITH_BOUNDARY adds the patches of
 * boundary vertices, cut to the cells inside the mesh (4, 2 or 1 cells in
 * 3D); their interior excludes the Dirichlet boundary, their coarsest p-level
 * is the lowest one with an interior node, solved exactly (FP64 Cholesky
 * inverse formed at setup), and learned Chebyshev bounds fall back to
 * Lanczos for them. */
#define PMG_PATCH_INTERIOR 0
#define PMG_PATCH_WITH_BOUNDARY 1

/* coarse-cell coefficients of the geometric multigrid hierarchy */
#define PMG_COARSE_ARITHMETIC 0
#define PMG_COARSE_GEOMETRIC 1
#define PMG_COARSE_HARMONIC 2

/* pmg_query keys */
#define PMG_Q_N_PATCHES 0
#define PMG_Q_N_COLORS 1
#define PMG_Q_N_LEVELS 2
#define PMG_Q_N_DOFS 3           /* (N p + 1)^dim */
#define PMG_Q_N_INTERIOR_DOFS 4  /* (N p - 1)^dim */
#define PMG_Q_DEVICE_BYTES 5
#define PMG_Q_N_BOUNDARY_PATCHES 6  /* patches of boundary vertices */
#define PMG_Q_LOCAL_DOFS 7          /* sum over patches of local interior nodes (top level) */
#define PMG_Q_TUNED_GRID 8          /* smoothing launch: workgroups (0 = one per patch) */
#define PMG_Q_TUNED_MAP 9           /* smoothing launch: 0 linear, 1 XCD-aware mapping */
#define PMG_Q_COLOR_OFFSET 16    /* + c: first patch of colour c, c <= n_colors */
#define PMG_Q_LEVEL_DEGREE 32    /* + l: degree of local level l */
#define PMG_Q_LEVEL_SIZE 48      /* + l: interior nodes per patch at level l */

typedef struct pmg_handle pmg_handle; /* opaque; owns the device memory it allocates */
typedef struct gmg_handle gmg_handle;
typedef struct pmg_batch pmg_batch;   /* opaque; owns its instance handles */

/* Structured mesh of [0,1]^dim with n_cells cells per direction. */
typedef struct pmg_mesh {
  int32_t dim;            /* 2 or 3 */
  int32_t n_cells;        /* N >= 2 */
  const double* vertices; /* host, ((N+1)^dim x dim), x fastest */
} pmg_mesh;

typedef struct pmg_opts {
  int32_t precision;     /* PMG_FP64, PMG_FP32, PMG_BF16_FP32ACC or PMG_BF16X3_FP32ACC */
  int32_t n_levels;      /* number of local p-levels, 2..4 */
  int32_t levels[8];     /* degrees, strictly descending, levels[0] = p, last = 1 */
  int32_t cheb_degree;   /* Chebyshev steps per smoothing pass, 1..8 (default 3) */
  int32_t n_vcycles;     /* local V-cycles per patch solve, N_MG >= 1 (default 1) */
  int32_t bounds;        /* PMG_BOUNDS_LANCZOS or PMG_BOUNDS_FIXED */
  int32_t lanczos_steps; /* Lanczos steps, 2..64 (default 12) */
  double cheb_safety;    /* s: b = s lambda_max (default 1.1) */
  double cheb_range;     /* rho: a = max(lambda_min, b / rho) (default 15) */
  uint64_t seed;         /* seed of the Lanczos start vectors (default 0) */
  void* stream;          /* hipStream_t, NULL = null stream */
  int32_t patch_set;     /* PMG_PATCH_INTERIOR (default) or PMG_PATCH_WITH_BOUNDARY */
  int32_t coarse_mean;   /* gmg_setup: coefficient of a coarse cell from its 2^d children,
                            PMG_COARSE_ARITHMETIC (default), _GEOMETRIC or _HARMONIC mean */
} pmg_opts;

/* Fill *o with the defaults listed above (levels: p, floor halvings, 1 is
 * not known without p, so n_levels = 0 means "p, p/2, ..., 1" at setup). */
int pmg_default_opts(pmg_opts* o);

/* Build the smoother for all interior vertex patches of a mesh at degree p
 * (Section 2.1).  Uploads geometry and coefficients, computes the inverse
 * diagonals of every level operator and, for PMG_BOUNDS_LANCZOS, the
 * Chebyshev bounds.  mesh, coeff: host.  Synchronises opts->stream.
 * Errors: INVALID_ARG (null, dim, N < 2, p outside 1..15, levels), DEGENERATE,
 * UNSUPPORTED (a level list without a compiled kernel), OOM, HIP. */
int pmg_patch_setup(const pmg_mesh* mesh, const double* coeff, int32_t p,
                    const pmg_opts* opts, pmg_handle** out);

/* One multiplicative sweep (Algorithm 1) over all patches: u += corrections.
 * direction +1 visits colours ascending, -1 descending.  u: device in/out,
 * b: device right-hand side (load vector), both FP64 global vectors; they
 * must not overlap.  Asynchronous on the handle's stream. */
int pmg_patch_smooth(pmg_handle* h, double* u, const double* b, int32_t direction);

/* Same as pmg_patch_smooth restricted to colours [c_begin, c_end). */
int pmg_patch_smooth_colors(pmg_handle* h, double* u, const double* b, int32_t c_begin,
                            int32_t c_end);

/* Evaluate step for all patches (equation main:4):
 * r[j] = Pi_j b - Pi_j A-bar_j Pi-bar_j u, in the local precision.
 * u, b: device global vectors; r: device, n_patches x (2p-1)^dim FP64, the
 * patch interior in x-fastest order. */
int pmg_patch_residual(pmg_handle* h, const double* u, const double* b, double* r);

/* Batched level operators A_{j,q} (Section 3.1, level operators):
 * y[j] = A_{j,q} x[j] for every patch, q = degree of level `level`.
 * x, y: device, n_patches x (2q-1)^dim FP64, interior x-fastest. */
int pmg_patch_apply(pmg_handle* h, int32_t level, const double* x, double* y);

/* Batched local solves (equation main:5): d[j] = N_MG V-cycles (Algorithm 2)
 * from zero on A_{j,p} d = r[j].  r, d: device, n_patches x (2p-1)^dim. */
int pmg_patch_local_solve(pmg_handle* h, const double* r, double* d);

/* Largest maxit that pmg_patch_pcg accepts (bounds the kernel's run time). */
#define PMG_PCG_MAXIT_LIMIT 10000

/* Batched patch CG, the measure of the local solver in Section 3.2: for every
 * patch j, conjugate gradients on A_{j,p} x = b[j] from x = 0, preconditioned
 * by N_MG V-cycles (Algorithm 2) with the handle's levels, Chebyshev degree
 * and intervals (degree 1 on an interval with a + b = 4 is the paper's damped
 * Jacobi, omega = 1/2).  A patch stops after the first iteration k with
 * ||r_k|| <= rtol ||b[j]||, or after maxit; each patch runs its own count.
 * b, x: device, n_patches x (2p-1)^dim FP64, interior x-fastest.
 * iters: device, n_patches int32 (k; 0 if b[j] = 0 or maxit = 0);
 * relres: device, n_patches FP64 (||r_k|| / ||b[j]||, 0 if b[j] = 0).
 * Residuals are the updated ones of the recurrence, as in the method.
 * FP64 handles only (PMG_ERR_UNSUPPORTED otherwise), and not for handles
 * with boundary-vertex patches (PMG_ERR_UNSUPPORTED).  PMG_ERR_INVALID_ARG:
 * null pointer, bounds not set, rtol negative or not finite, maxit outside
 * 0..PMG_PCG_MAXIT_LIMIT.  The first call allocates the handle's work
 * vectors (2 x n_patches x (2p-1)^dim FP64), kept until pmg_patch_destroy.
 * Asynchronous on the handle's stream. */
int pmg_patch_pcg(pmg_handle* h, const double* b, double* x, double rtol, int32_t maxit,
                  int32_t* iters, double* relres);

/* Largest work memory of pmg_patch_pcg_noalloc: 64 MiB per GPU. */
#define PMG_PCG_SCRATCH_BYTES ((size_t)64 << 20)

/* pmg_patch_pcg for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and results, with the per-patch residual and search
 * direction (2 x top-level size x n_patches doubles) in a library-owned
 * device array of PMG_PCG_SCRATCH_BYTES per GPU instead of a buffer the
 * handle allocates on its first pmg_patch_pcg call.  The call allocates and
 * frees nothing.  Arguments, layout and errors as pmg_patch_pcg; in addition
 * PMG_ERR_INVALID_ARG when the work exceeds PMG_PCG_SCRATCH_BYTES (the
 * message gives both sizes), before any device work.  Every call on a GPU
 * shares that GPU's array: calls that overlap on one GPU (other streams or
 * threads) race, and the caller must order them.  The array keeps the last
 * call's contents; the kernel writes every entry it reads. */
int pmg_patch_pcg_noalloc(pmg_handle* h, const double* b, double* x, double rtol, int32_t maxit,
                          int32_t* iters, double* relres);

/* The additive variant of the patch smoother: every local residual from the
 * same u (equation main:4), every local solve (equation main:5), then
 * u += theta sum_j Pi_j^T d_j (equation scatter with damping theta), the
 * corrections added colour by colour so that the sums are deterministic.
 * u, b: device global vectors as for pmg_patch_smooth.  Work buffers of
 * 2 x n_patches x (2p-1)^dim FP64 are allocated at the first call and kept
 * until pmg_patch_destroy.  Mesh handles (PMG_ERR_UNSUPPORTED for
 * independent patches); with PMG_PATCH_WITH_BOUNDARY the masked nodes of the
 * boundary-vertex patches are not scattered.  PMG_ERR_INVALID_ARG: null
 * pointer, theta not finite and > 0, bounds not set.  Asynchronous on the
 * handle's stream. */
int pmg_patch_smooth_additive(pmg_handle* h, double* u, const double* b, double theta);

/* Local smoothers of the V-cycle (Section 3.1, smoothers). */
#define PMG_SMOOTHER_CHEBYSHEV 0  /* Chebyshev-accelerated Jacobi (the default) */
#define PMG_SMOOTHER_CARTESIAN 1  /* Cartesian-reinforced */

/* Choose the local smoother.  PMG_SMOOTHER_CARTESIAN: one Richardson step
 * d += omega P (r - A d) before and one after the coarse correction on every
 * level above the coarsest, P = D diag(A_b) A_b^{-1} (Section 3.1), with D
 * the inverse diagonal of the patch's level operator and A_b the operator of
 * the Cartesian reference patch with unit cells, coefficient 1 and the
 * patch's own cell count per direction (one where the domain boundary cuts
 * the patch) at the level's degree, inverted by fast diagonalisation of the
 * 1D mass and stiffness matrices (tables formed in FP64 on the host at the
 * first call, stored in the handle's precision, kept until
 * pmg_patch_destroy).  Used by the sweeps (pmg_patch_smooth(_colors), the
 * GMG smoothers, batch sweeps) and by pmg_patch_pcg; pmg_patch_local_solve
 * and the additive sweep return PMG_ERR_UNSUPPORTED with it set.  Chebyshev
 * bounds are not needed for it.  PMG_ERR_INVALID_ARG: null handle, unknown
 * kind, omega not finite and > 0 (ignored for Chebyshev).  Synchronous
 * (uploads the tables). */
int pmg_set_smoother(pmg_handle* h, int32_t kind, double omega);

/* Inverse diagonal of A_{j,q} at level `level`: out device, n_patches x (2q-1)^dim. */
int pmg_get_inv_diag(const pmg_handle* h, int32_t level, double* out);

/* Eigenvalue estimates of D^{-1} A_{j,q}: lam host, n_patches x (n_levels-1) x 2
 * (lambda_min, lambda_max) per smoothed level.  Synchronises the stream. */
int pmg_get_bounds(const pmg_handle* h, double* lam);

/* Replace the bounds (same layout as pmg_get_bounds, host) and recompute the
 * Chebyshev intervals.  Requires 0 < lambda_min <= lambda_max. */
int pmg_set_bounds(pmg_handle* h, const double* lam);

/* A batch of n independent vertex patches (no mesh): every patch has its own
 * 3^dim vertices (offsets t in {0,1,2}^dim, x fastest; the patch vertex is
 * t = (1,...,1)) and 2^dim cell coefficients (cell c = sum c_i 2^i).
 * verts: host, n x 3^dim x dim; coeff: host, n x 2^dim; both copied.  The
 * handle supports the batched entry points (apply, local solve, inverse
 * diagonals, bounds, features) but not pmg_patch_smooth / pmg_patch_residual
 * (there is no global vector).  Lanczos start vectors use the patch number in
 * place of the vertex index.  Same errors as pmg_patch_setup. */
int pmg_patches_setup(int32_t dim, int64_t n, const double* verts, const double* coeff, int32_t p,
                      const pmg_opts* opts, pmg_handle** out);

/* Features of every patch for the bound-predicting network: for each cell c
 * and each point g of the 2-point Gauss rule, det J / h^d, ||J||_F^2 / h^2 and
 * ||cof J||_F^2 / h^(2(d-1)) at index (c 2^d + g) 3 + {0,1,2}, then
 * log10 mu_c minus the patch mean at 3 4^d + c; h = (mean cell volume)^(1/d).
 * out: device, n_patches x (3 4^d + 2^d) floats (200 in 3D, 52 in 2D). */
int pmg_patch_features(pmg_handle* h, float* out);

/* Linear vertex index sum_i v_i (N+1)^i of every patch, in patch order.
 * out: host, n_patches int32. */
int pmg_get_patch_vertices(const pmg_handle* h, int32_t* out);

/* Sizes and counters; see the PMG_Q_* keys. */
int pmg_query(const pmg_handle* h, int32_t what, int64_t* value);

int pmg_patch_destroy(pmg_handle* h);

/* Launch shape of the smoothing kernel (no change to the arithmetic: every
 * patch update is the same).  grid = 0: one workgroup per patch of a colour;
 * grid > 0: at most `grid` workgroups, each updating several patches in
 * turn.  map_mode 0: patch i of a colour goes to workgroup i mod grid;
 * map_mode 1: the colour's patches are split into 8 contiguous ranges, one
 * per XCD (workgroups are dealt to the XCDs round-robin), so neighbouring
 * patches share an L2. */
int pmg_set_launch(pmg_handle* h, int32_t grid, int32_t map_mode);

/* Autotuner: times the largest colour of a sweep (on a device copy of u,
 * which is left unchanged) for the launch shapes (one workgroup per patch,
 * linear or XCD-aware; 1, 2 or 4 workgroups per compute unit, XCD-aware; 2
 * per compute unit, linear), after a warm-up, in two rounds, and keeps the
 * fastest.  u, b: device, as for pmg_patch_smooth.  best_ms (host, may be
 * NULL): its time per colour launch.  Synchronises the handle's stream. */
int pmg_autotune(pmg_handle* h, const double* u, const double* b, float* best_ms);

/* Batches of independent problems (meshes of their own, degrees may differ),
 * smoothed together: a sweep takes the colours in order and, per colour,
 * launches every instance's patches concurrently on a stream of its own,
 * joined before the next colour.  meshes[i], coeffs[i] (host), p[i]: instance
 * i, set up as by pmg_patch_setup with opts (opts->n_levels must be 0:
 * default level lists p, p/2, ..., 1).  Synchronises opts->stream. */
int pmg_batch_setup(const pmg_mesh* meshes, const double* const* coeffs, const int32_t* p,
                    int32_t n, const pmg_opts* opts, pmg_batch** out);
/* The handle of instance i (owned by the batch: do not destroy it). */
int pmg_batch_instance(pmg_batch* b, int32_t i, pmg_handle** h);
/* One sweep of every instance captured into a HIP graph and replayed.
 * Switched off: returns PMG_ERR_UNSUPPORTED without device work (capturing
 * and replaying the batch sweep ended in a host crash whose cause is not
 * known); pmg_batch_smooth_eager runs the sweep. */
int pmg_batch_smooth(pmg_batch* b, double* const* u, const double* const* rhs, int32_t direction);
/* One sweep of every instance (direction +1 or -1), enqueued directly on
 * opts->stream (asynchronous); u[i], rhs[i]: device vectors of instance i.
 * Every instance's launch shape (pmg_set_launch) is honoured. */
int pmg_batch_smooth_eager(pmg_batch* b, double* const* u, const double* const* rhs,
                           int32_t direction);
/* Launch shapes for every instance, chosen with the instances running
 * together: whole-batch graph sweeps (captured per candidate) on copies of u
 * (left unchanged), one instance's shape at a time, highest degree first,
 * over the candidates of pmg_autotune.  Switched off: returns
 * PMG_ERR_UNSUPPORTED without device work (timing graph replays of tuned
 * shapes ended in a host crash whose cause is not known); set shapes per
 * instance with pmg_set_launch on pmg_batch_instance handles and sweep with
 * pmg_batch_smooth_eager. */
int pmg_batch_autotune(pmg_batch* b, double* const* u, const double* const* rhs);
/* Batch queries: the number of instances; graph captures and replays
 * (always 0 while graph sweeps are switched off). */
#define PMG_BQ_N_INSTANCES 0
#define PMG_BQ_CAPTURES 1
#define PMG_BQ_REPLAYS 2
int pmg_batch_query(const pmg_batch* b, int32_t what, int64_t* value);
int pmg_batch_destroy(pmg_batch* b);

/* Geometric multigrid over meshes with N, N/2, ... cells (halving while N
 * stays even and the halved mesh has an interior vertex), degree p on every
 * level.  Coarse vertices are the shared fine vertices; a coarse cell's
 * coefficient is the arithmetic, geometric or harmonic mean of its children
 * (opts->coarse_mean).  Smoothers on every level but the
 * coarsest use opts; the coarsest level is solved exactly (dense Cholesky,
 * FP64).  mesh, coeff: host.  Synchronises opts->stream. */
int gmg_setup(const pmg_mesh* mesh, const double* coeff, int32_t p, const pmg_opts* opts,
              gmg_handle** out);

/* y = A x on the finest level (Dirichlet rows/columns removed).  Device FP64. */
int gmg_apply(gmg_handle* g, const double* x, double* y);

/* z = V-cycle(r) (Section 2 and Section 4: forward sweep, residual,
 * restriction, recursion, prolongation, post-sweep).  The post-sweep runs the
 * colours in reverse (default, a symmetric V-cycle) or in the pre-sweep's
 * order after gmg_set_post_direction(+1) (the paper's order, non-symmetric);
 * with gmg_set_additive both sweeps are additive.  Device FP64. */
int gmg_vcycle(gmg_handle* g, const double* r, double* z);

/* Preconditioned CG from x = 0 until ||r|| <= rtol ||b|| or maxit iterations.
 * x, b: device FP64.  iters, relres: host (may be NULL).  Synchronous.
 * Returns PMG_WARN_NOT_CONVERGED when maxit is hit, PMG_ERR_BREAKDOWN on
 * breakdown, PMG_ERR_UNSUPPORTED when the V-cycle is not symmetric
 * (multiplicative sweeps with gmg_set_post_direction(+1): use
 * gmg_gmres_solve). */
int gmg_cg_solve(gmg_handle* g, double* x, const double* b, double rtol, int32_t maxit,
                 int32_t* iters, double* relres);

/* Largest maxit that gmg_gmres_solve accepts. */
#define PMG_GMRES_MAXIT_LIMIT 500

/* Colour order of the post-smoothing sweep of the V-cycle: -1 (the default)
 * reverses the pre-smoothing order, which keeps the preconditioner
 * symmetric; +1 repeats it, as the paper does (Section 4), for GMRES.
 * PMG_ERR_INVALID_ARG for other values. */
int gmg_set_post_direction(gmg_handle* g, int32_t direction);

/* theta > 0: both smoothing steps of the V-cycle are additive sweeps
 * (pmg_patch_smooth_additive) with damping theta, which keeps the
 * preconditioner symmetric; theta = 0 (the default): multiplicative sweeps.
 * Interior-vertex patch sets only (the sweeps return PMG_ERR_UNSUPPORTED
 * otherwise).  PMG_ERR_INVALID_ARG: theta negative or not finite. */
int gmg_set_additive(gmg_handle* g, double theta);

/* GMRES from x = 0 with one V-cycle as right preconditioner (the outer
 * solver of Section 4; flexible form, no restart: 2 maxit + 1 device vectors
 * of the fine size, allocated at the first call that needs them and kept
 * until gmg_destroy), until ||b - A x|| <= rtol ||b|| or maxit iterations.
 * x, b: device FP64; iters, relres: host (may be NULL); iters = maxit + 1
 * and PMG_WARN_NOT_CONVERGED when maxit is hit.  Synchronous.
 * PMG_ERR_INVALID_ARG: null pointer, rtol not finite and > 0, maxit outside
 * 1..PMG_GMRES_MAXIT_LIMIT; PMG_ERR_BREAKDOWN on a zero or non-finite
 * rotation. */
int gmg_gmres_solve(gmg_handle* g, double* x, const double* b, double rtol, int32_t maxit,
                    int32_t* iters, double* relres);

/* Number of mesh levels, or the smoother handle of level l (1 = coarsest
 * smoothed level, n_levels-1 = finest); the handle stays owned by g. */
int gmg_query(const gmg_handle* g, int32_t what, int64_t* value);
int gmg_level_smoother(gmg_handle* g, int32_t level, pmg_handle** h);

int gmg_destroy(gmg_handle* g);

/* Bound-predicting network: n_in -> 64 -> 64 -> 64 -> n_out, tanh hidden
 * layers, linear output, inputs standardised by a stored mean and 1/std.
 * Parameters (FP32) in the layout W1 (n_in x 64, row-major), b1, W2, b2, W3,
 * b3, W4 (64 x n_out), b4.  Trained by mean squared error with Adam on the
 * GPU.  All work on the given stream; max_batch bounds the rows processed at
 * once (training batches, gradients). */
typedef struct pmg_mlp pmg_mlp;
int pmg_mlp_param_count(int32_t n_in, int32_t n_out, int64_t* count);
/* params: host, param_count floats (the initial weights). */
int pmg_mlp_create(int32_t n_in, int32_t n_out, const float* params, int64_t max_batch, void* stream,
                   pmg_mlp** out);
int pmg_mlp_get_params(const pmg_mlp* m, float* params);   /* host */
int pmg_mlp_set_params(pmg_mlp* m, const float* params);   /* host; resets Adam */
/* mean and 1/std of every input over the rows of X (device, n x n_in). */
int pmg_mlp_fit_standardizer(pmg_mlp* m, const float* X, int64_t n);
int pmg_mlp_get_standardizer(const pmg_mlp* m, float* mean, float* inv_std); /* host, n_in each */
int pmg_mlp_set_standardizer(pmg_mlp* m, const float* mean, const float* inv_std);
/* Y = net(X): X device n x n_in, Y device n x n_out. */
int pmg_mlp_predict(pmg_mlp* m, const float* X, int64_t n, float* Y);
/* gradient of the mean squared error over all rows (n <= max_batch):
 * X, T device; grad host (param_count); loss host. */
int pmg_mlp_gradient(pmg_mlp* m, const float* X, const float* T, int64_t n, float* grad, double* loss);
/* Adam (beta 0.9, 0.999, eps 1e-8) over `epochs` passes; order (device,
 * epochs x n int32) lists the sample of every position of every epoch;
 * batches of `batch` consecutive positions.  epoch_loss: host, mean batch loss
 * of every epoch (may be NULL).  Synchronous. */
int pmg_mlp_train(pmg_mlp* m, const float* X, const float* T, int64_t n, const int32_t* order,
                  int32_t epochs, int32_t batch, float lr, double* epoch_loss);
int pmg_mlp_destroy(pmg_mlp* m);
/* Save a network to a file: the 8 bytes "PMGMLP1" and a zero, int32 n_in,
 * int32 n_out, double margin (the caller's lambda_max margin, stored for
 * pmg_set_bounds_mlp), the parameters (param_count floats), the input mean
 * and 1/std (n_in floats each); little-endian.  Synchronises the network's
 * stream. */
int pmg_mlp_save(const pmg_mlp* m, double margin, const char* path);
/* Load a saved network (checked: magic, sizes, file length) on `stream`;
 * margin (host, may be NULL) receives the stored margin.  A malformed file
 * returns PMG_ERR_INVALID_ARG before any device work. */
int pmg_mlp_load(const char* path, int64_t max_batch, void* stream, pmg_mlp** out, double* margin);

/* Chebyshev bounds from the network: features of every patch, prediction of
 * (ln lambda_min, ln lambda_max) per smoothed level, lambda_max raised by the
 * factor exp(margin).  Patches with a standardised feature beyond ood_z in
 * magnitude (outside the training distribution) or a non-finite prediction
 * fall back to per-patch Lanczos; n_fallback (host, may be NULL) returns their
 * number.  The network must have 3 4^d + 2^d inputs and 2 (n_levels - 1)
 * outputs.  Synchronous. */
int pmg_set_bounds_mlp(pmg_handle* h, pmg_mlp* m, double margin, double ood_z, int64_t* n_fallback);

/* Train the network on the Chebyshev bounds of a handle (learned bounds, the
 * project's extension of the smoother's interval; the labels are the Lanczos
 * bounds the method computes for the patches of `labels`, usually a
 * pmg_patches_setup handle of random patches).  Steps, all in the library:
 * the features of every patch of `labels` (as pmg_patch_features) and its
 * targets ln lambda_min, ln lambda_max per smoothed level (from its bounds, as
 * pmg_get_bounds); the standardiser fitted on the training rows (the first
 * epoch's row list); `epochs` epochs of pmg_mlp_train over those rows; then,
 * over the validation rows, the root mean squared error of every output and
 * the lambda_max margin = 3 x the largest error of an ln lambda_max output
 * (the margin pmg_set_bounds_mlp takes).
 * train_order: device int32, epochs x n_train patch numbers of `labels` (one
 * permutation of the training rows per epoch); val_rows: device int32, n_val
 * patch numbers.  epoch_loss (host, epochs), val_rmse (host, n_out floats)
 * and margin (host) may be NULL.  Synchronous.  PMG_ERR_INVALID_ARG: null
 * network, handle or row lists, n_train or n_val < 1, a row number outside
 * the handle's patches (checked on the host copy), a network whose sizes do
 * not match the handle (3 4^d + 2^d inputs, 2 (n_levels - 1) outputs), bounds
 * not set or not positive, batch above max_batch. */
int pmg_mlp_fit_bounds(pmg_mlp* m, const pmg_handle* labels, const int32_t* train_order, int64_t n_train,
                       const int32_t* val_rows, int64_t n_val, int32_t epochs, int32_t batch, float lr,
                       double* epoch_loss, float* val_rmse, double* margin);

/* Simplicial vertex patches (Section 3.2: patches of 3 quadrilaterals in 2D
 * and 4 hexahedra in 3D around one vertex, the cells of a triangle or a
 * tetrahedron cut around its centroid).  A patch is nv vertices (7 in 2D: 3
 * corners, 3 edge midpoints, the centroid; 15 in 3D: 4 corners, 6 edge
 * midpoints, 4 face centroids, the centroid) and dim + 1 multilinear cells
 * given by their corner lists (x fastest, corner 0 a corner of the simplex,
 * the last corner the centroid; every cell positively oriented).  The
 * unknowns are the nodes of the conforming degree-q space off the patch
 * boundary (a node is on the boundary when a local index is 0); they are
 * numbered in order of first appearance over the cells in order, the nodes
 * of a cell x fastest: 3(q-1)^2 + 3(q-1) + 1 in 2D and 4(q-1)^3 + 6(q-1)^2 +
 * 4(q-1) + 1 in 3D.  The local solver is the p-multigrid V-cycle of
 * Algorithm 2 with rediscretised level operators, the embedding of the
 * degree-q space into the degree-p one as prolongation and its transpose as
 * restriction, Chebyshev-Jacobi smoothing and the exact solve at degree 1
 * (the centroid alone).  FP64. */
typedef struct pmg_simplex pmg_simplex;
/* The numbering of the unknowns at degree q for a cell list (host, no
 * device work): codes (host, (dim+1) x (q+1)^dim) receives 2 g + f for the
 * cell node holding unknown g (f = 1 in the first cell holding it), -1 on the
 * boundary; count the number of unknowns.  PMG_ERR_INVALID_ARG: null
 * pointer, dim, q outside 1..15, a corner outside the vertex list. */
int pmg_simplex_numbering(int32_t dim, const int32_t* cells, int32_t q, int32_t* codes, int32_t* count);
/* n patches: verts (host, n x nv x dim), cells (host, (dim+1) x 2^dim, one
 * list for all patches), coeff (host, n x (dim+1) cell coefficients), degree
 * p.  opts: precision PMG_FP64 and bounds PMG_BOUNDS_FIXED (intervals from
 * pmg_simplex_set_bounds) only, else PMG_ERR_UNSUPPORTED; n_levels = 0 takes
 * p followed by the members of 1, 3, 7, 15 below it (the paper's nested
 * degrees); kernels exist for 2D levels (3,1), (7,3,1), (15,7,3,1) and 3D
 * (3,1), (7,3,1) (PMG_ERR_UNSUPPORTED otherwise).  Computes the inverse
 * diagonal of every level on the device.  PMG_ERR_INVALID_ARG: null pointer,
 * dim, n, bad level list, non-positive coefficient, cells that do not form a
 * simplicial patch; PMG_ERR_DEGENERATE: a cell with det J <= 0 at a corner or
 * a Gauss point.  Synchronises opts->stream. */
int pmg_simplex_setup(int32_t dim, int64_t n, const double* verts, const int32_t* cells, const double* coeff,
                      int32_t p, const pmg_opts* opts, pmg_simplex** out);
/* PMG_Q_N_PATCHES, PMG_Q_N_LEVELS, PMG_Q_DEVICE_BYTES, PMG_Q_LEVEL_DEGREE + l,
 * PMG_Q_LEVEL_SIZE + l (unknowns per patch at level l). */
int pmg_simplex_query(const pmg_simplex* s, int32_t what, int64_t* value);
/* lam: host, n x (n_levels - 1) x 2 bounds of D^{-1} A per smoothed level;
 * intervals as for pmg_set_bounds. */
int pmg_simplex_set_bounds(pmg_simplex* s, const double* lam);
/* out: device, n x size_level (FP64 inverse diagonal of level `level`). */
int pmg_simplex_get_inv_diag(const pmg_simplex* s, int32_t level, double* out);
/* y = A_level x per patch; x, y device n x size_level.  Asynchronous. */
int pmg_simplex_apply(pmg_simplex* s, int32_t level, const double* x, double* y);
/* d = N_MG V-cycles from zero on r per patch; device n x size_0.  Asynchronous. */
int pmg_simplex_local_solve(pmg_simplex* s, const double* r, double* d);
/* CG on every A_p x = b preconditioned by the V-cycle, as pmg_patch_pcg:
 * b, x device n x size_0; iters (int32) and relres device, n each.
 * PMG_ERR_INVALID_ARG: null pointer, bounds not set, rtol not finite and
 * >= 0, maxit outside 0..PMG_PCG_MAXIT_LIMIT.  Asynchronous. */
int pmg_simplex_pcg(pmg_simplex* s, const double* b, double* x, double rtol, int32_t maxit, int32_t* iters,
                    double* relres);
int pmg_simplex_destroy(pmg_simplex* s);

const char* pmg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PMG_H */
