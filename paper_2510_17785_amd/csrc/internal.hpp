// Internal declarations shared by the host API and the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/pmg.h"

namespace pmgi {

constexpr int kThreads = 256;        // threads per patch workgroup
constexpr int kMaxLevels = 4;        // local p-levels per patch
constexpr int kTabLevelStride = 3 * 256 + 2 * 16;  // B, Dc, D (n x n) + xg, wg (n), n <= 16
constexpr int kTabTransferStride = 29 * 29;        // (2p-1) x (2q-1), p <= 15
constexpr int kTabSize = kMaxLevels * kTabLevelStride + (kMaxLevels - 1) * kTabTransferStride;

// Kernel modes of the patch kernel.
enum PatchMode : int {
  kModeSmooth = 0,    // gather, evaluate, local solve, scatter-add
  kModeResidual = 1,  // gather, evaluate, write the local residual
  kModeSolve = 2,     // read local residuals, local solve, write corrections
  kModeApply = 3,     // read interior vectors, apply one level operator
  kModeMetric = 4,    // setup: compute the cached levels' metric, write it to metric_out
  kModePcg = 5,       // FP64 only: CG on each patch problem, preconditioned by the V-cycle
  kModePcgCart = 6,   // the same with the Cartesian-reinforced smoother in the V-cycle
  kModeSmoothCart = 7,  // kModeSmooth with the Cartesian-reinforced smoother in the V-cycle
};

// Per level of fdm tables, three direction types (a direction with two
// cells; one cell whose interior nodes are the low ones 1 .. q-1; one cell
// with the high ones q+1 .. 2q-1, both embedded in the two-cell numbering),
// each: S (29 x 29 at most), lam, dM, dK (29 each).
constexpr int kFdmTypeStride = 29 * 29 + 3 * 29;
constexpr int kFdmStride = 3 * kFdmTypeStride;

// Arguments of every per-patch kernel.  Pointers to T-valued arrays are
// void* here and cast inside the kernel.
struct PatchArgs {
  const double* verts;       // (N+1)^dim x dim
  const double* mu;          // N^dim
  const int32_t* patch_vertex;  // per patch (sweep order): linear vertex index
  int32_t N, p;
  int32_t patch_begin;       // first patch of this launch (sweep order)
  int32_t n_patch;           // patches in this launch (= grid size)
  const void* tab;           // T tables, kTabSize
  const double* tab64;       // FP64 tables, kTabSize
  const void* invdiag[kMaxLevels];      // T, n_patches_total x size_l
  const double* invdiag64[kMaxLevels];  // FP64, same layout
  const void* cheb;          // T, n_patches_total x (L-1) x 2: theta, delta
  int32_t cheb_degree, n_vcycles;
  double* u;                 // global vector (smooth)
  const double* b;           // global right-hand side (smooth, residual)
  const double* in;          // batched local input (solve, apply)
  double* out;               // batched local output (residual, solve, apply, diag)
  int32_t level;             // level index (apply, diag)
  void* vec_scratch;         // per-block vector storage when it does not fit in LDS
  int64_t vec_stride;        // elements per block in vec_scratch
  // Lanczos
  int32_t lanczos_steps;
  uint64_t seed;
  double* lanczos_basis;     // per block: m x size_l doubles
  double* bounds_out;        // n_patches_total x (L-1) x 2
  // independent patches (no mesh): 3^d vertices and 2^d coefficients each
  const double* patch_geo;   // n_patches_total x 3^d x d, or null for a mesh
  const double* patch_mu;    // n_patches_total x 2^d
  // optional list of patch numbers: block b handles patch_list[patch_begin + b]
  const int32_t* patch_list;
  // small levels held as dense matrices (see PatchVariant::dense_level)
  const void* dense[kMaxLevels];   // T, n_patches_total x size_l^2, row-major
  double* dense64[kMaxLevels];     // FP64 copies, written by the setup kernel
  // patches of boundary vertices (mesh handles only): cells outside the mesh
  // are ghosts with mu = 0, nodes on or beyond the boundary are masked
  int32_t with_boundary;
  // per patch: row of trunc_inv holding the FP64 inverse of its lowest
  // non-empty level (level count - 2, masked rows and columns zero), or -1
  const int32_t* trunc_index;
  const double* trunc_inv;   // rows x size_{L-2}^2
  // patch kernel launch shape: grid (0 = one workgroup per patch, else at
  // most this many workgroups, each taking several patches) and the
  // patch-to-workgroup mapping (0 linear, 1 XCD-aware ranges)
  int32_t grid, map_mode;
  // metric G of the levels whose metric is kept in LDS, per patch (T,
  // n_patches_total x metric elements, the LDS layout), computed once at
  // setup by kModeMetric; null: computed in every patch update
  const void* metric;
  void* metric_out;
  // kModePcg: in = b, out = x (n_patches_total x size_0 each); work holds the
  // residual and search direction (2 x size_0 per patch); per patch the
  // iterations taken and ||r_k|| / ||b||
  double pcg_rtol;
  int32_t pcg_maxit;
  double* pcg_work;
  int32_t* pcg_iters;
  double* pcg_relres;
  // Cartesian-reinforced smoother (kModePcgCart, kModeSmoothCart):
  // fast-diagonalisation tables per smoothed level, kFdmStride elements of T
  // each (per direction type: S row-major with column k the k-th
  // eigenvector, then lam, dM, dK), and the damping omega
  const void* fdm_tab;
  double fdm_omega;
};

// One compiled (precision, dim, levels) variant of the patch kernels.
struct PatchVariant {
  int precision, dim, n_levels;
  int levels[kMaxLevels];
  // launch one patch kernel in `mode` over args.n_patch patches
  hipError_t (*launch)(int mode, const PatchArgs& a, hipStream_t s);
  // set the launch attributes (dynamic LDS) of every patch kernel of this
  // variant on the current device; called at setup, before any capture
  hipError_t (*prime)();
  // dynamic LDS bytes of `mode`, and per-block vector-scratch elements needed
  // when vectors do not fit in LDS (0 if they do)
  size_t (*lds_bytes)(int mode);
  int64_t (*vec_scratch_elems)();
  int64_t (*vec_scratch_elems64)();  // same for the FP64 layout of the setup kernels
  // FP64 matrix of level args.level for the patches args.patch_list[patch_begin + b],
  // written to args.out + (patch_begin + b) * size^2 (row-major)
  hipError_t (*launch_level_matrix)(const PatchArgs& a, hipStream_t s);
  // FP64 setup kernels (inverse diagonals of every level; Lanczos bounds)
  hipError_t (*launch_diag)(const PatchArgs& a, hipStream_t s);
  hipError_t (*launch_lanczos)(const PatchArgs& a, int level, hipStream_t s);
  // levels applied as a stored dense matrix (1) instead of by sum factorisation,
  // and the FP64 setup kernel that forms them from the matrix-free operator
  int dense_level[kMaxLevels];
  hipError_t (*launch_dense)(const PatchArgs& a, hipStream_t s);
  // elements per patch of the metric kept in LDS (0: none), see
  // PatchArgs::metric; kModeMetric writes them
  int64_t (*metric_elems)();
};

const PatchVariant* find_variant(int precision, int dim, int n_levels, const int* levels);

// Simplicial vertex patches (simplex_kernels.hip): a triangle cut into 3
// quadrilaterals (2D) or a tetrahedron cut into 4 hexahedra (3D) around its
// centroid.  Unknowns per patch at degree q: the cells' interiors, the
// faces and edges they share, and the centroid.
constexpr __host__ __device__ int simplex_unknowns(int dim, int q) {
  return dim == 2 ? 3 * (q - 1) * (q - 1) + 3 * (q - 1) + 1
                  : 4 * (q - 1) * (q - 1) * (q - 1) + 6 * (q - 1) * (q - 1) + 4 * (q - 1) + 1;
}
constexpr int kSimplexThreads = 256;
enum SimplexMode : int {
  kSimplexDiag = 0,   // setup: inverse diagonal of level `level`
  kSimplexApply = 1,  // y = A_level x per patch
  kSimplexSolve = 2,  // N_MG V-cycles from zero
  kSimplexPcg = 3,    // CG preconditioned by the V-cycle
};
struct SimplexArgs {
  int32_t n_patch, patch_begin;
  const double* geo;        // per patch: (dim+1) cells x 2^dim corners x dim, then (dim+1) mu
  int32_t geo_stride;
  const int32_t* gat[kMaxLevels];  // per level: (dim+1) x (q+1)^dim codes 2 g + owner, -1 boundary
  const double* tab;        // per level B, E (n x n), xg, wg (n); per transfer P1 (nf x nc)
  const double* dinv[kMaxLevels];  // per level: n_patch_total x size
  const double* cheb;       // n_patch_total x (L-1) x 2: theta, delta
  int32_t cheb_degree, n_vcycles;
  const double* in;
  double* out;
  int32_t level;
  double rtol;
  int32_t maxit;
  double* work;             // CG: 2 x size_0 per patch
  int32_t* iters;
  double* relres;
};
struct SimplexVariant {
  int dim, n_levels;
  int levels[kMaxLevels];
  hipError_t (*launch)(int mode, const SimplexArgs& a, hipStream_t s);
  hipError_t (*prime)();
  size_t lds_bytes;
  int cell_nodes;
};
const SimplexVariant* find_simplex_variant(int dim, int n_levels, const int* levels);
// Set the message pmg_last_error returns; returns code.
int set_error(int code, const char* msg);
// Features of every patch for the bound-predicting network (n x nf floats).
hipError_t launch_features(int dim, const PatchArgs& a, int n_patch, float* out, hipStream_t s);
// Fill the per-degree 1D tables in constant memory of the current device.
hipError_t init_constant_tables();
// Device address and size of the current device's work array of
// pmg_patch_pcg_noalloc (looked up once per device, never allocated).
hipError_t pcg_scratch(double** ptr, size_t* bytes);
std::string list_variants();

// Global (h-level) FP64 kernels.
struct CellArgs {
  const double* verts;
  const double* mu;
  int32_t N, p, dim;
  const double* tab64;  // tables of degree p at level slot 0
};
hipError_t launch_cell_apply(const CellArgs& a, const double* x, double* cellbuf, hipStream_t s);
hipError_t launch_cell_gather(int dim, int N, int p, const double* cellbuf, double* y, hipStream_t s);
hipError_t launch_element_matrices(const CellArgs& a, double* Ke, hipStream_t s);
hipError_t launch_h_prolong_axis(int dim, int axis, const int* sizes_in, const int* sizes_out,
                                 const int* first, const double* w, int p, const double* in,
                                 double* out, int transpose, hipStream_t s);
hipError_t launch_mask_dirichlet(int dim, int M, double* x, hipStream_t s);
hipError_t launch_patch_scatter(int dim, int N, int p, const int32_t* vertex, int begin, int count,
                                const double* d, double theta, double* u, hipStream_t s);
hipError_t launch_axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t s);
hipError_t launch_xpay_to(int64_t n, const double* x, double a, const double* y, double* z,
                          hipStream_t s);
hipError_t launch_dot_partial(int64_t n, const double* x, const double* y, double* partial,
                              int nblocks, hipStream_t s);
hipError_t launch_dot_final(const double* partial, int nblocks, double* out, hipStream_t s);
hipError_t launch_gemv(int n, const double* A, const double* x, double* y, hipStream_t s);
hipError_t launch_gather_interior(int dim, int M, const double* full, double* packed,
                                  hipStream_t s);
hipError_t launch_scatter_interior(int dim, int M, const double* packed, double* full,
                                   hipStream_t s);
hipError_t launch_convert_to_float(int64_t n, const double* in, float* out, hipStream_t s);
constexpr int kDotBlocks = 512;

// The bound-predicting MLP (mlp_kernels.hip).
int64_t mlp_param_count(int n_in, int n_out);
struct MlpNet {
  int n_in = 0, n_out = 0;
  int64_t cap = 0;  // largest batch the work buffers hold
  int t = 0;        // Adam step counter
  hipStream_t stream = nullptr;
  float *theta = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
  float *mean = nullptr, *inv_std = nullptr;
  float *xb = nullptr, *tb = nullptr, *xs = nullptr, *h1 = nullptr, *h2 = nullptr, *h3 = nullptr;
  float *y = nullptr, *d3 = nullptr, *d2 = nullptr, *d1 = nullptr, *dy = nullptr;
  double *partial = nullptr, *loss = nullptr;
  int32_t* idx = nullptr;
  ~MlpNet();
  int64_t offset(int layer) const;
  hipError_t alloc(int64_t max_batch);
  hipError_t forward(const float* in_std, int B);
  hipError_t backward(const float* in_std, const float* targets, int B);
  hipError_t standardize(const float* X, int64_t B, float* out);
  hipError_t fit_standardizer(const float* X, int64_t n);
  hipError_t adam_step(float lr, float b1, float b2, float eps);
  hipError_t gather(const float* X, const float* T, const int32_t* order, int B);
  // out (B x K) = rows idx[0..B) of X (rows of K floats)
  hipError_t gather_rows(const float* X, const int32_t* idx, int B, int K, float* out);
  hipError_t max_abs_z(const float* X, int64_t n, float* zmax);
};

}  // namespace pmgi
