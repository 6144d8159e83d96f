// Per-patch kernels of the vertex-patch smoother with a nested p-multigrid
// local solver (arXiv 2510.17785, Section 2.1 and Section 3.1), for CDNA4.
//
// Templates only: every translation unit that includes this header gets its
// own copy of the kernels it instantiates and of the constant-memory tables
// they read (upload_tables fills that copy).  The kernels of each level list
// are instantiated in one patch_variants_*.hip file; patch_kernels.hip holds
// the registry over them.
//
// One workgroup (512 threads in FP32, 256 in FP64) owns one patch at a time.  Everything the
// local solver touches lives in LDS: the 1D tables, the patch geometry (3^d
// vertices relative to the patch centre and 2^d coefficients), the closure
// input of the operator, its interior output, the sum-factorisation slab
// buffers and, when they fit, the level vectors.  Global memory is touched
// only to gather u and b, to read the per-patch inverse diagonals and
// Chebyshev intervals, and to scatter-add the FP64 correction.
//
// Level operator (Section 3.1, level operators; Section 2, bilinear form):
//   A_{j,q} x = sum over the 2^d cells of B^T G B x in sum-factorised form.
// The patch is treated as one tensor-product object with 2 cells per
// direction: a closure line of 2q+1 nodes maps to 2(q+1) Gauss points (q+1
// per cell) through a block-structured 1D matrix, so the node shared by the
// two cells of a line is handled once and the transposed contraction sums the
// contributions of both cells without any atomics.  Gradients at the Gauss
// points use the collocation derivative on the Gauss points.  The metric
// G = mu w det J J^{-1} J^{-T} is recomputed at every quadrature point from
// the multilinear cell map (the paper's matrix-free local solver keeps only
// O(p^d) data per patch, Section 1 and Section 3.1), except on the levels
// whose layout keeps it: there it is computed once at setup and read back.  In 3D the work is split
// into two slabs (the two cell layers in z) to bound the LDS footprint.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <mutex>
#include <set>
#include <string>
#include <tuple>
#include <type_traits>
#include <vector>
#include <algorithm>

#include "fe_tables.hpp"
#include "internal.hpp"

namespace pmgi {
namespace {

constexpr __host__ __device__ int ipow(int b, int e) {
  int r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}
constexpr __host__ __device__ int round_up(int x, int a) { return (x + a - 1) / a * a; }

// Address-space-qualified pointers: out-of-line device functions only get
// ds_read/ds_write (not flat accesses) for LDS when the pointer type says so.
#define LDSP __attribute__((address_space(3)))
template <typename T>
__device__ __forceinline__ LDSP T* lds_cast(T* p) {
  return (LDSP T*)p;
}
template <typename T>
__device__ __forceinline__ const LDSP T* lds_cast(const T* p) {
  return (const LDSP T*)p;
}
// the same for global memory: global (not flat) loads, which count against
// the vector-memory counter only, so waits for LDS reads do not wait for them
#define GLBP __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ const GLBP T* glb_cast(const T* p) {
  return (const GLBP T*)p;
}

// Wavefront-level sync: the LDS writes of this wavefront's lanes are visible
// to its other lanes afterwards (no workgroup barrier).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The value v holds in lane j of the wavefront (j uniform).
__device__ __forceinline__ float lane_value(float v, int j) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), j));
}
__device__ __forceinline__ double lane_value(double v, int j) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), j);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), j);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// 1D tables of every degree 1..kMaxDegree, B (n x n), Dc (n x n), D (n x n),
// Gauss points and weights, in constant memory: they depend on the degree
// only, and reads at compile-time offsets become scalar loads.
constexpr __host__ __device__ int ctab_size(int q) { return 3 * (q + 1) * (q + 1) + 2 * (q + 1); }
constexpr __host__ __device__ int ctab_off(int q) {
  int o = 0;
  for (int r = 1; r < q; ++r) o += ctab_size(r);
  return o;
}
constexpr int kConstTab = ctab_off(kMaxDegree + 1);
__constant__ float c_tab32[kConstTab];
__constant__ double c_tab64[kConstTab];
template <typename T>
__device__ __forceinline__ const T* ctab() {
  if constexpr (std::is_same<T, double>::value)
    return c_tab64;
  else
    return c_tab32;
}

// Threads per patch workgroup: 8 waves for FP32 (segment-form tops held to
// 128 VGPRs so that two workgroups share a CU; the slab-form tops take up to
// 256 and one CU each), 4 waves for FP64 (up to 256 VGPRs).
template <typename T>
constexpr int NT = sizeof(T) == 4 ? 512 : 256;

template <int... Qs>
struct Levels {
  static constexpr int count = sizeof...(Qs);
  static constexpr int q[kMaxLevels] = {Qs...};
  static constexpr bool bf16 = false;
  static constexpr bool split = false;
};
// The same level list with the BF16-input / FP32-accumulate top-level
// operator (interpolation contractions on the matrix cores); SPLIT: every
// operand as a sum of two BF16 numbers, three products per tile.
template <bool SPLIT, int... Qs>
struct LevelsBF16 : Levels<Qs...> {
  static constexpr bool bf16 = true;
  static constexpr bool split = SPLIT;
};

template <int DIM, int Q>
struct Sh {
  static constexpr int n = Q + 1;       // nodes / Gauss points per cell per direction
  static constexpr int m = 2 * Q + 1;   // closure nodes per direction
  static constexpr int mi = 2 * Q - 1;  // interior nodes per direction
  static constexpr int NQ = 2 * n;      // Gauss points per direction over the patch
  static constexpr int closure = ipow(m, DIM);
  static constexpr int interior = ipow(mi, DIM);
  static constexpr int S = DIM == 3 ? n * NQ * NQ : n * NQ;  // one slab buffer
};

constexpr __host__ __device__ int tab_size(int q) { return 3 * (q + 1) * (q + 1) + 2 * (q + 1); }

// LDS layout (in elements of T) of one patch workgroup.
template <typename T, int DIM, class LV>
struct Layout {
  static constexpr int L = LV::count;
  using S0 = Sh<DIM, LV::q[0]>;
  static constexpr int tab_level_off(int l) {
    int o = 0;
    for (int i = 0; i < l; ++i) o += tab_size(LV::q[i]);
    return o;
  }
  static constexpr int tab_transfer_off(int t) {
    int o = tab_level_off(L);
    for (int i = 0; i < t; ++i) o += (2 * LV::q[i] - 1) * (2 * LV::q[i + 1] - 1);
    return o;
  }
  static constexpr int tab_total = tab_transfer_off(L - 1);
  static constexpr int geo_off = round_up(tab_total, 4);
  static constexpr int nvert = ipow(3, DIM);
  // per cell: DIM Jacobian columns x DIM components x 2^(DIM-1) multilinear coefficients
  static constexpr int njc = ipow(2, DIM) * DIM * DIM * ipow(2, DIM - 1);
  static constexpr int jc_rel = nvert * DIM + ipow(2, DIM) + 2 * kMaxLevels;
  static constexpr int geo_size = jc_rel + njc;
  static constexpr int X_off = round_up(geo_off + geo_size, 4);
  static constexpr int Out_off = round_up(X_off + S0::closure, 4);
  static constexpr int abuf_off = round_up(Out_off + S0::interior, 4);
  // 3D levels use the segment-form operator when its four Gauss-point
  // buffers fit 40 KB at the top degree (else the two-slab form)
  static constexpr int P0 = ipow(2 * (LV::q[0] + 1), DIM);
  static constexpr bool seg_top = DIM == 3 && 4 * P0 * (int)sizeof(T) <= 40 * 1024;
  // FP64 degree-7 tops keep the level vectors in LDS: the top level then
  // works in quarter-slabs and its inverse diagonal is read from global memory
  static constexpr bool f64_vec = sizeof(T) == 8 && DIM == 3 && LV::q[0] == 7;
  static constexpr bool dinv0_global = f64_vec;
  // where four full slabs would take more than 64 KB, the top level works in
  // quarter-slabs (n x n x NQ buffers)
  static constexpr bool quarter_top =
      DIM == 3 && !seg_top && (4 * S0::S * (int)sizeof(T) > 64 * 1024 || f64_vec);
  static constexpr int abuf_elems =
      seg_top ? 4 * P0 : (quarter_top ? 4 * S0::n * S0::n * S0::NQ : 4 * S0::S);
  static constexpr bool use_seg(int l) {
    return DIM == 3 && 4 * ipow(2 * (LV::q[l] + 1), DIM) <= abuf_elems;
  }
  static constexpr bool use_quarter(int l) {
    return DIM == 3 && !use_seg(l) && 4 * ipow(2 * (LV::q[l] + 1), 3) / 2 > abuf_elems;
  }
  static constexpr int base_total = round_up(abuf_off + abuf_elems, 4);
  static constexpr int level_size(int l) { return ipow(2 * LV::q[l] - 1, DIM); }
  // vectors: r_l, d_l, dinv_l per level, then res and z at the top size
  static constexpr int vec_r(int l) {
    int o = 0;
    for (int i = 0; i < l; ++i) o += (dinv0_global && i == 0 ? 2 : 3) * level_size(i);
    return o;
  }
  static constexpr int vec_d(int l) { return vec_r(l) + level_size(l); }
  static constexpr int vec_dinv(int l) { return vec_r(l) + 2 * level_size(l); }
  static constexpr int vec_res = vec_r(L);
  static constexpr int vec_z = vec_res + level_size(0);
  static constexpr int vec_total = vec_z + level_size(0);
  // Levels below the top with at most 32 interior nodes (degree 2 in 3D) and
  // not the coarsest are applied as a stored dense matrix: their sum
  // factorisation is all fixed per-phase cost.
  static constexpr bool dense_level(int l) {
    return l > 0 && l < L - 1 && level_size(l) <= 32;
  }
  static constexpr int dense_rel(int l) {
    int o = 0;
    for (int i = 0; i < l; ++i) o += dense_level(i) ? level_size(i) * level_size(i) : 0;
    return o;
  }
  static constexpr int dense_total = dense_rel(L);
  // Intermediate levels of up to 125 interior nodes (degree 3 in 3D) that do
  // not fit LDS as dense matrices are applied as dense matrices read from
  // global memory: one matrix-vector phase instead of seven latency-bound
  // sum-factorisation phases on a tiny tensor.
  static constexpr bool dense_global(int l) {
    return l > 0 && l < L - 1 && !dense_level(l) && level_size(l) <= 125;
  }
  // metric G at every Gauss point of every level, structure of arrays
  static constexpr int NG = DIM == 3 ? 6 : 3;
  // Gauss points of level l that need the metric (none for the stored dense
  // levels and the coarsest level, which the V-cycle never applies)
  static constexpr int npts(int l) {
    return (l > 0 && (l == L - 1 || dense_level(l) || dense_global(l))) ? 0
                                                                        : ipow(2 * (LV::q[l] + 1), DIM);
  }
  static constexpr int G_all = [] {
    int o = 0;
    for (int i = 0; i < L; ++i) o += NG * npts(i);
    return o;
  }();
  // LDS budgets: 80 KB keeps two workgroups per CU; the slab-form degrees
  // (6 and up in 3D) hold one workgroup per CU by their registers anyway, so
  // they may use nearly all of the 160 KB for the top level's metric
  static constexpr int kBudget = 80 * 1024, kBudgetOne = 159 * 1024;
  static constexpr int sz = (int)sizeof(T);
  static constexpr bool all_fit = (base_total + G_all + vec_total) * sz <= kBudget;
  static constexpr bool one_wg = DIM == 3 && !seg_top;
  static constexpr int G_top = NG * ipow(2 * (LV::q[0] + 1), DIM);
  static constexpr bool top_vec_fit = !all_fit && one_wg && (base_total + G_top + vec_total) * sz <= kBudgetOne;
  // FP32 slab-form tops where the level vectors and the top metric do not
  // fit together keep the vectors in LDS (the metric is then read from its
  // setup copy in global memory, or recomputed at every Gauss point where
  // there is none): vectors in global memory make every Chebyshev update a
  // chain of memory round trips, which cost more than either
  static constexpr bool vec_over_G = !all_fit && one_wg && !top_vec_fit && sz == 4 &&
                                     (base_total + vec_total) * sz <= kBudgetOne;
  static constexpr bool top_fit = !all_fit && one_wg && !vec_over_G && (base_total + G_top) * sz <= kBudgetOne;
  // the metric of level l is kept in LDS (else recomputed at every Gauss point)
  static constexpr bool cache_level(int l) {
    return npts(l) > 0 && (all_fit || ((top_vec_fit || top_fit) && l == 0));
  }
  static constexpr int G_rel(int l) {
    int o = 0;
    for (int i = 0; i < l; ++i) o += cache_level(i) ? NG * npts(i) : 0;
    return o;
  }
  static constexpr int G_total = G_rel(L);
  static constexpr bool cache_G = G_total > 0;
  // levels l .. L-1 all have at most 64 nodes and are stored dense (or are
  // the coarsest), with the vectors in LDS: one wavefront can run their
  // V-cycle alone (vcycle_small)
  static constexpr bool small_from(int l) {
    if (l >= L || !vec_in_lds) return false;
    for (int i = l; i < L; ++i)
      if (level_size(i) > 64 || !(i == L - 1 || dense_level(i))) return false;
    return true;
  }
  // some level that the V-cycle applies recomputes its metric at the Gauss
  // points (from the per-cell Jacobian coefficients)
  static constexpr bool needs_jc = [] {
    for (int l = 0; l < L; ++l)
      if (npts(l) > 0 && !cache_level(l)) return true;
    return false;
  }();
  // level vectors in LDS when they fit next to the cached metric, in place of
  // it (above), or, with no metric cached, within the two-workgroup budget;
  // else global scratch
  static constexpr bool vec_in_lds =
      all_fit || top_vec_fit || vec_over_G || (!cache_G && (base_total + vec_total) * sz <= kBudget) ||
      (f64_vec && !cache_G && (base_total + vec_total) * sz <= kBudgetOne);
  // FP32 slab-form tops on the matrix cores (degree 7 at most) that keep the
  // level vectors in LDS instead of the metric read the top level's metric
  // from the setup's copy in global memory (per patch NG x npts(0) values,
  // the LDS layout) when the handle has one, instead of recomputing it at
  // every Gauss point
  static constexpr bool G_global = vec_over_G && npts(0) > 0 && LV::q[0] <= 7 && !use_quarter(0);
  static constexpr int G_glob_elems = G_global ? NG * npts(0) : 0;
  static constexpr int G_off = base_total;
  static constexpr int vec_off = base_total + G_total;
  static constexpr int dense_off = round_up(vec_off + (vec_in_lds ? vec_total : 0), 4);
  static constexpr int lds_elems = dense_off + dense_total;
  static_assert(!f64_vec || vec_in_lds, "FP64 degree-7 level vectors must fit in LDS");
};

// ---------------------------------------------------------------------------
// geometry: G = scale * det J J^{-1} J^{-T} = scale * adj(J) adj(J)^T / det J
// ---------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ void metric3(const T* __restrict__ V, int cx, int cy, int cz, T x,
                                        T y, T z, T scale, T* G) {
  // V: 27 patch vertices x 3, vertex (i,j,k) at ((k*3 + j)*3 + i)*3
  const T* c = V + ((cz * 3 + cy) * 3 + cx) * 3;
  auto P = [&](int i, int j, int k, int r) { return c[((k * 3 + j) * 3 + i) * 3 + r]; };
  const T x0 = T(1) - x, y0 = T(1) - y, z0 = T(1) - z;
  T J[3][3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    J[r][0] = y0 * z0 * (P(1, 0, 0, r) - P(0, 0, 0, r)) + y * z0 * (P(1, 1, 0, r) - P(0, 1, 0, r)) +
              y0 * z * (P(1, 0, 1, r) - P(0, 0, 1, r)) + y * z * (P(1, 1, 1, r) - P(0, 1, 1, r));
    J[r][1] = x0 * z0 * (P(0, 1, 0, r) - P(0, 0, 0, r)) + x * z0 * (P(1, 1, 0, r) - P(1, 0, 0, r)) +
              x0 * z * (P(0, 1, 1, r) - P(0, 0, 1, r)) + x * z * (P(1, 1, 1, r) - P(1, 0, 1, r));
    J[r][2] = x0 * y0 * (P(0, 0, 1, r) - P(0, 0, 0, r)) + x * y0 * (P(1, 0, 1, r) - P(1, 0, 0, r)) +
              x0 * y * (P(0, 1, 1, r) - P(0, 1, 0, r)) + x * y * (P(1, 1, 1, r) - P(1, 1, 0, r));
  }
  T a[3][3];  // adjugate
  a[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  a[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
  a[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
  a[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  a[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
  a[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
  a[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  a[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
  a[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  const T det = J[0][0] * a[0][0] + J[0][1] * a[1][0] + J[0][2] * a[2][0];
  const T s = scale / det;
  G[0] = s * (a[0][0] * a[0][0] + a[0][1] * a[0][1] + a[0][2] * a[0][2]);
  G[1] = s * (a[0][0] * a[1][0] + a[0][1] * a[1][1] + a[0][2] * a[1][2]);
  G[2] = s * (a[0][0] * a[2][0] + a[0][1] * a[2][1] + a[0][2] * a[2][2]);
  G[3] = s * (a[1][0] * a[1][0] + a[1][1] * a[1][1] + a[1][2] * a[1][2]);
  G[4] = s * (a[1][0] * a[2][0] + a[1][1] * a[2][1] + a[1][2] * a[2][2]);
  G[5] = s * (a[2][0] * a[2][0] + a[2][1] * a[2][1] + a[2][2] * a[2][2]);
}

template <typename T>
__device__ __forceinline__ void metric2(const T* __restrict__ V, int cx, int cy, T x, T y,
                                        T scale, T* G) {
  // V: 9 patch vertices x 2, vertex (i,j) at (j*3 + i)*2
  const T* c = V + (cy * 3 + cx) * 2;
  auto P = [&](int i, int j, int r) { return c[(j * 3 + i) * 2 + r]; };
  const T x0 = T(1) - x, y0 = T(1) - y;
  T J[2][2];
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    J[r][0] = y0 * (P(1, 0, r) - P(0, 0, r)) + y * (P(1, 1, r) - P(0, 1, r));
    J[r][1] = x0 * (P(0, 1, r) - P(0, 0, r)) + x * (P(1, 1, r) - P(1, 0, r));
  }
  const T det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  // adj = [[J11, -J01], [-J10, J00]]
  const T s = scale / det;
  G[0] = s * (J[1][1] * J[1][1] + J[0][1] * J[0][1]);
  G[1] = -s * (J[1][1] * J[1][0] + J[0][1] * J[0][0]);
  G[2] = s * (J[1][0] * J[1][0] + J[0][0] * J[0][0]);
}

// The Jacobian columns of a multilinear cell are multilinear in the other
// reference coordinates: column 0 of a hex is a + b y + c z + d y z (per
// component).  These coefficients are formed once per patch (jc, per cell:
// [column][component][4] in 3D, [column][component][2] in 2D), so the metric
// costs about 60 instructions per Gauss point.
template <typename T, typename PJ>
__device__ __forceinline__ void metric3c(PJ jc, T x, T y, T z, T scale, T* G) {
  T J[3][3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const auto c0 = jc + (0 * 3 + r) * 4;
    const auto c1 = jc + (1 * 3 + r) * 4;
    const auto c2 = jc + (2 * 3 + r) * 4;
    J[r][0] = c0[0] + c0[1] * y + z * (c0[2] + c0[3] * y);
    J[r][1] = c1[0] + c1[1] * x + z * (c1[2] + c1[3] * x);
    J[r][2] = c2[0] + c2[1] * x + y * (c2[2] + c2[3] * x);
  }
  T a[3][3];
  a[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  a[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
  a[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
  a[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  a[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
  a[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
  a[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  a[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
  a[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  const T det = J[0][0] * a[0][0] + J[0][1] * a[1][0] + J[0][2] * a[2][0];
  const T s = scale / det;
  G[0] = s * (a[0][0] * a[0][0] + a[0][1] * a[0][1] + a[0][2] * a[0][2]);
  G[1] = s * (a[0][0] * a[1][0] + a[0][1] * a[1][1] + a[0][2] * a[1][2]);
  G[2] = s * (a[0][0] * a[2][0] + a[0][1] * a[2][1] + a[0][2] * a[2][2]);
  G[3] = s * (a[1][0] * a[1][0] + a[1][1] * a[1][1] + a[1][2] * a[1][2]);
  G[4] = s * (a[1][0] * a[2][0] + a[1][1] * a[2][1] + a[1][2] * a[2][2]);
  G[5] = s * (a[2][0] * a[2][0] + a[2][1] * a[2][1] + a[2][2] * a[2][2]);
}

template <typename T, typename PJ>
__device__ __forceinline__ void metric2c(PJ jc, T x, T y, T scale, T* G) {
  T J[2][2];
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const auto c0 = jc + (0 * 2 + r) * 2;
    const auto c1 = jc + (1 * 2 + r) * 2;
    J[r][0] = c0[0] + c0[1] * y;
    J[r][1] = c1[0] + c1[1] * x;
  }
  const T det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  const T s = scale / det;
  G[0] = s * (J[1][1] * J[1][1] + J[0][1] * J[0][1]);
  G[1] = -s * (J[1][1] * J[1][0] + J[0][1] * J[0][0]);
  G[2] = s * (J[1][0] * J[1][0] + J[0][0] * J[0][0]);
}

// multilinear coefficients of the Jacobian columns of every cell of the patch
template <typename T, int DIM>
__device__ void jacobian_coefficients(const T* __restrict__ V, T* __restrict__ jc) {
  constexpr int ncell = ipow(2, DIM);
  constexpr int per = DIM * DIM * ipow(2, DIM - 1);
  for (int i = threadIdx.x; i < ncell * DIM * DIM; i += NT<T>) {
    const int r = i % DIM, col = (i / DIM) % DIM, cell = i / (DIM * DIM);
    const int cx = cell & 1, cy = (cell >> 1) & 1, cz = (cell >> 2) & 1;
    T* out = jc + cell * per + (col * DIM + r) * ipow(2, DIM - 1);
    if constexpr (DIM == 3) {
      auto P = [&](int i0, int j0, int k0) {
        return V[(((cz + k0) * 3 + (cy + j0)) * 3 + (cx + i0)) * 3 + r];
      };
      // e[b][c]: difference along the column direction at the corners (b, c)
      // of the other two directions, in increasing axis order
      T e[2][2];
      for (int b = 0; b < 2; ++b)
        for (int cc = 0; cc < 2; ++cc) {
          if (col == 0) e[b][cc] = P(1, b, cc) - P(0, b, cc);
          else if (col == 1) e[b][cc] = P(b, 1, cc) - P(b, 0, cc);
          else e[b][cc] = P(b, cc, 1) - P(b, cc, 0);
        }
      out[0] = e[0][0];
      out[1] = e[1][0] - e[0][0];
      out[2] = e[0][1] - e[0][0];
      out[3] = e[1][1] - e[1][0] - e[0][1] + e[0][0];
    } else {
      auto P = [&](int i0, int j0) { return V[((cy + j0) * 3 + (cx + i0)) * 2 + r]; };
      T e0, e1;
      if (col == 0) {
        e0 = P(1, 0) - P(0, 0);
        e1 = P(1, 1) - P(0, 1);
      } else {
        e0 = P(0, 1) - P(0, 0);
        e1 = P(1, 1) - P(1, 0);
      }
      out[0] = e0;
      out[1] = e1 - e0;
    }
  }
}

// ---------------------------------------------------------------------------
// per-workgroup context
// ---------------------------------------------------------------------------

template <typename T, int DIM, class LV>
struct Ctx {
  using Lay = Layout<T, DIM, LV>;
  T* lds;
  T* vec;          // vector storage (LDS or global scratch)
  const T* gtab;   // the same 1D tables in global memory (read with scalar loads)
  // patch of a boundary vertex: FP64 inverse of its lowest non-empty level
  // (level count - 2), which the V-cycle solves exactly; null otherwise
  const double* trunc = nullptr;
  int pf = 0;  // boundary flags of the patch (see patch_flags)
  const T* dglob[kMaxLevels] = {nullptr};  // this patch's dense matrices in global memory
  const T* Gg = nullptr;  // this patch's top-level metric in global memory (Layout::G_global)
  __device__ const T* gB(int l) const { return gtab + l * kTabLevelStride; }
  __device__ const T* gDc(int l) const {
    const int n = LV::q[l] + 1;
    return gtab + l * kTabLevelStride + n * n;
  }
  __device__ const T* tabB(int l) const { return lds + Lay::tab_level_off(l); }
  __device__ const T* tabDc(int l) const {
    const int n = LV::q[l] + 1;
    return lds + Lay::tab_level_off(l) + n * n;
  }
  __device__ const T* tabD(int l) const {
    const int n = LV::q[l] + 1;
    return lds + Lay::tab_level_off(l) + 2 * n * n;
  }
  __device__ const T* tabXg(int l) const {
    const int n = LV::q[l] + 1;
    return lds + Lay::tab_level_off(l) + 3 * n * n;
  }
  __device__ const T* tabWg(int l) const {
    const int n = LV::q[l] + 1;
    return lds + Lay::tab_level_off(l) + 3 * n * n + n;
  }
  __device__ const T* tabP(int t) const { return lds + Lay::tab_transfer_off(t); }
  __device__ T* geo() const { return lds + Lay::geo_off; }
  __device__ T* mu() const { return lds + Lay::geo_off + Lay::nvert * DIM; }
  __device__ T* cheb() const { return lds + Lay::geo_off + Lay::nvert * DIM + ipow(2, DIM); }
  __device__ T* jc() const { return lds + Lay::geo_off + Lay::jc_rel; }
  __device__ T* Gc(int l) const { return lds + Lay::G_off + Lay::G_rel(l); }
  __device__ T* dense(int l) const { return lds + Lay::dense_off + Lay::dense_rel(l); }
  bool dense_ok = false;  // dense level matrices loaded (not in the setup kernels)
  bool metric_loaded = false;  // the cached metric was read from the setup's copy
  bool geo_needed = true;      // the patch geometry is used (Jacobian or metric)
  const T* fdm = nullptr;  // Cartesian-reinforced smoother tables (kModePcgCart, kModeSmoothCart)
  double omega = 0;
  // FP64 inverse of the coarsest level's 1 x 1 matrix (interior patches of
  // FP32 handles): the coarse solve runs in FP64 in every precision
  double coarse_inv = 0;
  // d = A^{-1} r on the coarsest level of an interior patch
  __device__ T coarse_solve(T r, T dinv) const {
    if constexpr (sizeof(T) == 8) return dinv * r;
    else return T(coarse_inv * double(r));
  }
  __device__ T* X() const { return lds + Lay::X_off; }
  __device__ T* Out() const { return lds + Lay::Out_off; }
  __device__ T* abuf() const { return lds + Lay::abuf_off; }
  __device__ T* r(int l) const { return vec + Lay::vec_r(l); }
  __device__ T* d(int l) const { return vec + Lay::vec_d(l); }
  // top level's inverse diagonal in global memory (Layout::dinv0_global)
  T* dinv0 = nullptr;
  __device__ T* dinv(int l) const { return (Lay::dinv0_global && l == 0) ? dinv0 : vec + Lay::vec_dinv(l); }
  __device__ T* res() const { return vec + Lay::vec_res; }
  __device__ T* z() const { return vec + Lay::vec_z; }
};

// ---------------------------------------------------------------------------
// sum-factorised level operator
//   X  : closure values (2Q+1)^DIM, x fastest (boundary entries included)
//   Out: interior rows (2Q-1)^DIM of A-bar X
// ---------------------------------------------------------------------------

template <typename T, int Q, bool CACHE>
__device__ __noinline__ void apply3(const LDSP T* __restrict__ X, LDSP T* __restrict__ Out,
                                    LDSP T* __restrict__ ab, const LDSP T* __restrict__ Bt,
                                    const LDSP T* __restrict__ Dc, const LDSP T* __restrict__ xg,
                                    const LDSP T* __restrict__ wg, const LDSP T* __restrict__ jc,
                                    const LDSP T* __restrict__ mu, const LDSP T* __restrict__ Gc) {
  using SH = Sh<3, Q>;
  constexpr int n = SH::n, m = SH::m, mi = SH::mi, NQ = SH::NQ, S = SH::S;
  LDSP T* A = ab;
  LDSP T* Bf = ab + S;
  LDSP T* C = ab + 2 * S;
  LDSP T* Dd = ab + 3 * S;
  const int tid = threadIdx.x;
#pragma unroll 1
  for (int cz = 0; cz < 2; ++cz) {
    // x: A[zl][y][QX] = sum_a B[kx][a] X[cz Q + zl][y][cx Q + a]
#pragma unroll 1
    for (int idx = tid; idx < n * m * NQ; idx += NT<T>) {
      const int QX = idx % NQ, t = idx / NQ, y = t % m, zl = t / m;
      const int cx = QX >= n, kx = QX - cx * n;
      const LDSP T* xr = X + ((cz * Q + zl) * m + y) * m + cx * Q;
      const LDSP T* br = Bt + kx * n;
      T acc = 0;
#pragma unroll
      for (int a = 0; a < n; ++a) acc += br[a] * xr[a];
      A[idx] = acc;
    }
    __syncthreads();
    // y: Bf[zl][QY][QX] = sum_a B[ky][a] A[zl][cy Q + a][QX]
#pragma unroll 1
    for (int idx = tid; idx < S; idx += NT<T>) {
      const int QX = idx % NQ, t = idx / NQ, QY = t % NQ, zl = t / NQ;
      const int cy = QY >= n, ky = QY - cy * n;
      const LDSP T* ar = A + (zl * m + cy * Q) * NQ + QX;
      const LDSP T* br = Bt + ky * n;
      T acc = 0;
#pragma unroll
      for (int a = 0; a < n; ++a) acc += br[a] * ar[a * NQ];
      Bf[idx] = acc;
    }
    __syncthreads();
    // z: C[kz][QY][QX] = sum_zl B[kz][zl] Bf[zl][QY][QX]   (values at Gauss points)
#pragma unroll 1
    for (int idx = tid; idx < S; idx += NT<T>) {
      const int kz = idx / (NQ * NQ), rem = idx % (NQ * NQ);
      const LDSP T* br = Bt + kz * n;
      T acc = 0;
#pragma unroll
      for (int a = 0; a < n; ++a) acc += br[a] * Bf[a * NQ * NQ + rem];
      C[idx] = acc;
    }
    __syncthreads();
    // reference gradients by collocation, then the flux G grad
#pragma unroll 1
    for (int idx = tid; idx < S; idx += NT<T>) {
      const int QX = idx % NQ, t = idx / NQ, QY = t % NQ, kz = t / NQ;
      const int cx = QX >= n, kx = QX - cx * n, cy = QY >= n, ky = QY - cy * n;
      const LDSP T* dx = Dc + kx * n;
      const LDSP T* dy = Dc + ky * n;
      const LDSP T* dz = Dc + kz * n;
      const LDSP T* cxr = C + (kz * NQ + QY) * NQ + cx * n;
      const LDSP T* cyr = C + (kz * NQ + cy * n) * NQ + QX;
      const LDSP T* czr = C + QY * NQ + QX;
      T gx = 0, gy = 0, gz = 0;
#pragma unroll
      for (int a = 0; a < n; ++a) {
        gx += dx[a] * cxr[a];
        gy += dy[a] * cyr[a * NQ];
        gz += dz[a] * czr[a * NQ * NQ];
      }
      T G[6];
      if constexpr (CACHE) {
        const int gp = cz * S + idx;  // (QZ NQ + QY) NQ + QX with QZ = cz n + kz
#pragma unroll
        for (int c = 0; c < 6; ++c) G[c] = Gc[c * 2 * S + gp];
      } else {
        const int cell = cz * 4 + cy * 2 + cx;
        metric3c<T>(jc + cell * 36, xg[kx], xg[ky], xg[kz], mu[cell] * wg[kx] * wg[ky] * wg[kz], G);
      }
      A[idx] = G[0] * gx + G[1] * gy + G[2] * gz;
      Bf[idx] = G[1] * gx + G[3] * gy + G[4] * gz;
      Dd[idx] = G[2] * gx + G[4] * gy + G[5] * gz;
    }
    __syncthreads();
    // transposed collocation: C = Dc^T F
#pragma unroll 1
    for (int idx = tid; idx < S; idx += NT<T>) {
      const int QX = idx % NQ, t = idx / NQ, QY = t % NQ, kz = t / NQ;
      const int cx = QX >= n, kx = QX - cx * n, cy = QY >= n, ky = QY - cy * n;
      const LDSP T* fx = A + (kz * NQ + QY) * NQ + cx * n;
      const LDSP T* fy = Bf + (kz * NQ + cy * n) * NQ + QX;
      const LDSP T* fz = Dd + QY * NQ + QX;
      T acc = 0;
#pragma unroll
      for (int a = 0; a < n; ++a) {
        acc += Dc[a * n + kx] * fx[a];
        acc += Dc[a * n + ky] * fy[a * NQ];
        acc += Dc[a * n + kz] * fz[a * NQ * NQ];
      }
      C[idx] = acc;
    }
    __syncthreads();
    // z^T: A[zl][QY][QX] = sum_kz B[kz][zl] C[kz][QY][QX]
#pragma unroll 1
    for (int idx = tid; idx < S; idx += NT<T>) {
      const int zl = idx / (NQ * NQ), rem = idx % (NQ * NQ);
      T acc = 0;
#pragma unroll
      for (int k = 0; k < n; ++k) acc += Bt[k * n + zl] * C[k * NQ * NQ + rem];
      A[idx] = acc;
    }
    __syncthreads();
    // y^T onto interior rows: Bf[zl][yi][QX], y = yi + 1
#pragma unroll 1
    for (int idx = tid; idx < n * mi * NQ; idx += NT<T>) {
      const int QX = idx % NQ, t = idx / NQ, yi = t % mi, zl = t / mi;
      const int y = yi + 1;
      T acc = 0;
      if (y <= Q) {
        const LDSP T* ar = A + (zl * NQ) * NQ + QX;
#pragma unroll
        for (int k = 0; k < n; ++k) acc += Bt[k * n + y] * ar[k * NQ];
      }
      if (y >= Q) {
        const LDSP T* ar = A + (zl * NQ + n) * NQ + QX;
#pragma unroll
        for (int k = 0; k < n; ++k) acc += Bt[k * n + (y - Q)] * ar[k * NQ];
      }
      Bf[idx] = acc;
    }
    __syncthreads();
    // x^T onto interior columns and the interior z-planes of this slab
    const int zl0 = cz == 0 ? 1 : 0;
    constexpr int nz = Q;  // interior planes per slab: z = 1..Q or Q..2Q-1
#pragma unroll 1
    for (int idx = tid; idx < nz * mi * mi; idx += NT<T>) {
      const int xi = idx % mi, t = idx / mi, yi = t % mi, zl = zl0 + t / mi;
      const int x = xi + 1;
      const LDSP T* br = Bf + (zl * mi + yi) * NQ;
      T acc = 0;
      if (x <= Q) {
#pragma unroll
        for (int k = 0; k < n; ++k) acc += Bt[k * n + x] * br[k];
      }
      if (x >= Q) {
#pragma unroll
        for (int k = 0; k < n; ++k) acc += Bt[k * n + (x - Q)] * br[n + k];
      }
      const int zz = cz * Q + zl - 1;
      LDSP T* o = Out + (zz * mi + yi) * mi + xi;
      if (cz == 1 && zl == 0)
        *o += acc;
      else
        *o = acc;
    }
    __syncthreads();
  }
}


// The same operator in quarter-slabs: cell layer cz and cell row cy at a
// time, so the four work buffers hold n x n x NQ values instead of
// n x NQ x NQ (for degrees whose full slabs do not fit LDS next to the rest
// of the patch).  Out is cleared first and every quarter adds its part.
template <typename T, int Q, bool CACHE>
__device__ __forceinline__ void apply3q(const LDSP T* __restrict__ X, LDSP T* __restrict__ Out,
                                     LDSP T* __restrict__ ab, const LDSP T* __restrict__ Bt,
                                     const LDSP T* __restrict__ Dc, const LDSP T* __restrict__ xg,
                                     const LDSP T* __restrict__ wg, const LDSP T* __restrict__ jc,
                                     const LDSP T* __restrict__ mu, const LDSP T* __restrict__ Gc) {
  using SH = Sh<3, Q>;
  constexpr int n = SH::n, m = SH::m, mi = SH::mi, NQ = SH::NQ;
  constexpr int H = n * n * NQ;  // one quarter-slab buffer: [z or kz][y or ky][QX]
  LDSP T* A = ab;
  LDSP T* Bf = ab + H;
  LDSP T* C = ab + 2 * H;
  LDSP T* Dd = ab + 3 * H;
  const int tid = threadIdx.x;
#pragma unroll 1
  for (int i = tid; i < SH::interior; i += NT<T>) Out[i] = T(0);
#pragma unroll 1
  for (int qs = 0; qs < 4; ++qs) {
    const int cz = qs >> 1, cy = qs & 1;
    // x: A[zl][ya][QX] = sum_a B[kx][a] X[cz Q + zl][cy Q + ya][cx Q + a]
#pragma unroll 1
    for (int idx = tid; idx < H; idx += NT<T>) {
      const int QX = idx % NQ, t = idx / NQ, ya = t % n, zl = t / n;
      const int cx = QX >= n, kx = QX - cx * n;
      const LDSP T* xr = X + ((cz * Q + zl) * m + cy * Q + ya) * m + cx * Q;
      const LDSP T* br = Bt + kx * n;
      T acc = 0;
#pragma unroll
      for (int a = 0; a < n; ++a) acc += br[a] * xr[a];
      A[idx] = acc;
    }
    __syncthreads();
    // y: Bf[zl][ky][QX] = sum_a B[ky][a] A[zl][a][QX]
#pragma unroll 1
    for (int idx = tid; idx < H; idx += NT<T>) {
      const int QX = idx % NQ, t = idx / NQ, ky = t % n, zl = t / n;
      const LDSP T* ar = A + zl * n * NQ + QX;
      const LDSP T* br = Bt + ky * n;
      T acc = 0;
#pragma unroll
      for (int a = 0; a < n; ++a) acc += br[a] * ar[a * NQ];
      Bf[idx] = acc;
    }
    __syncthreads();
    // z: C[kz][ky][QX] = sum_zl B[kz][zl] Bf[zl][ky][QX]   (values at Gauss points)
#pragma unroll 1
    for (int idx = tid; idx < H; idx += NT<T>) {
      const int kz = idx / (n * NQ), rem = idx % (n * NQ);
      const LDSP T* br = Bt + kz * n;
      T acc = 0;
#pragma unroll
      for (int a = 0; a < n; ++a) acc += br[a] * Bf[a * n * NQ + rem];
      C[idx] = acc;
    }
    __syncthreads();
    // reference gradients by collocation, then the flux G grad
#pragma unroll 1
    for (int idx = tid; idx < H; idx += NT<T>) {
      const int QX = idx % NQ, t = idx / NQ, ky = t % n, kz = t / n;
      const int cx = QX >= n, kx = QX - cx * n;
      const LDSP T* dx = Dc + kx * n;
      const LDSP T* dy = Dc + ky * n;
      const LDSP T* dz = Dc + kz * n;
      const LDSP T* cxr = C + (kz * n + ky) * NQ + cx * n;
      const LDSP T* cyr = C + kz * n * NQ + QX;
      const LDSP T* czr = C + ky * NQ + QX;
      T gx = 0, gy = 0, gz = 0;
#pragma unroll
      for (int a = 0; a < n; ++a) {
        gx += dx[a] * cxr[a];
        gy += dy[a] * cyr[a * NQ];
        gz += dz[a] * czr[a * n * NQ];
      }
      T G[6];
      if constexpr (CACHE) {
        const int gp = ((cz * n + kz) * NQ + cy * n + ky) * NQ + QX;
#pragma unroll
        for (int c = 0; c < 6; ++c) G[c] = Gc[c * NQ * NQ * NQ + gp];
      } else {
        const int cell = cz * 4 + cy * 2 + cx;
        metric3c<T>(jc + cell * 36, xg[kx], xg[ky], xg[kz], mu[cell] * wg[kx] * wg[ky] * wg[kz], G);
      }
      A[idx] = G[0] * gx + G[1] * gy + G[2] * gz;
      Bf[idx] = G[1] * gx + G[3] * gy + G[4] * gz;
      Dd[idx] = G[2] * gx + G[4] * gy + G[5] * gz;
    }
    __syncthreads();
    // transposed collocation: C = Dc^T F
#pragma unroll 1
    for (int idx = tid; idx < H; idx += NT<T>) {
      const int QX = idx % NQ, t = idx / NQ, ky = t % n, kz = t / n;
      const int cx = QX >= n, kx = QX - cx * n;
      const LDSP T* fx = A + (kz * n + ky) * NQ + cx * n;
      const LDSP T* fy = Bf + kz * n * NQ + QX;
      const LDSP T* fz = Dd + ky * NQ + QX;
      T acc = 0;
#pragma unroll
      for (int a = 0; a < n; ++a) {
        acc += Dc[a * n + kx] * fx[a];
        acc += Dc[a * n + ky] * fy[a * NQ];
        acc += Dc[a * n + kz] * fz[a * n * NQ];
      }
      C[idx] = acc;
    }
    __syncthreads();
    // z^T: A[zl][ky][QX] = sum_kz B[kz][zl] C[kz][ky][QX]
#pragma unroll 1
    for (int idx = tid; idx < H; idx += NT<T>) {
      const int zl = idx / (n * NQ), rem = idx % (n * NQ);
      T acc = 0;
#pragma unroll
      for (int k = 0; k < n; ++k) acc += Bt[k * n + zl] * C[k * n * NQ + rem];
      A[idx] = acc;
    }
    __syncthreads();
    // y^T: Bf[zl][ya][QX] = sum_ky B[ky][ya] A[zl][ky][QX]
#pragma unroll 1
    for (int idx = tid; idx < H; idx += NT<T>) {
      const int QX = idx % NQ, t = idx / NQ, ya = t % n, zl = t / n;
      const LDSP T* ar = A + zl * n * NQ + QX;
      T acc = 0;
#pragma unroll
      for (int k = 0; k < n; ++k) acc += Bt[k * n + ya] * ar[k * NQ];
      Bf[idx] = acc;
    }
    __syncthreads();
    // x^T onto the interior nodes of this quarter: z = cz Q + zl and
    // y = cy Q + ya in 1 .. 2Q-1, Q planes and Q rows per quarter
    const int zl0 = cz == 0 ? 1 : 0, ya0 = cy == 0 ? 1 : 0;
#pragma unroll 1
    for (int idx = tid; idx < Q * Q * mi; idx += NT<T>) {
      const int xi = idx % mi, t = idx / mi, ya = ya0 + t % Q, zl = zl0 + t / Q;
      const int x = xi + 1;
      const LDSP T* br = Bf + (zl * n + ya) * NQ;
      T acc = 0;
      if (x <= Q) {
#pragma unroll
        for (int k = 0; k < n; ++k) acc += Bt[k * n + x] * br[k];
      }
      if (x >= Q) {
#pragma unroll
        for (int k = 0; k < n; ++k) acc += Bt[k * n + (x - Q)] * br[n + k];
      }
      const int zz = cz * Q + zl - 1, yy = cy * Q + ya - 1;
      Out[(zz * mi + yy) * mi + xi] += acc;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Contractions on the matrix cores (FP32 accumulation)
//
// One contraction phase is a product D = M In with a 1D (patch-level) matrix
// M of at most 16 x 16 and an input of at most 16 rows and ncols columns.
// Every wavefront takes 16-column tiles.  Lane l supplies M[l % 16][4 (l / 16)
// + s] and In[4 (l / 16) + s][j] for its column j = 16 tile + l % 16
// (s = 0..3), and receives D[4 (l / 16) + r][j] (r = 0..3).  With BF16
// operands the inputs are rounded (nearest even) when they are packed, the
// products are exact in FP32 and accumulated in FP32; with FP32 operands the
// four values of a lane go to four 16x16x4 products.  Results are stored in
// FP32.
// ---------------------------------------------------------------------------

typedef short mm_s4 __attribute__((ext_vector_type(4)));
typedef float mm_f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short to_bf16(float x) { return __builtin_bit_cast(short, (__bf16)x); }

__device__ __forceinline__ float from_bf16(short h) {
  return (float)__builtin_bit_cast(__bf16, h);
}

// Operand modes: kMmBf16 rounds both operands to BF16 (one product per
// tile); kMmBf16x3 splits x = hi + lo with hi = bf16(x), lo = bf16(x - hi)
// and takes M In as Mhi Inhi + Mhi Inlo + Mlo Inhi (the dropped lo lo term is
// below 2^-16 relative); kMmF32 keeps FP32 operands (v_mfma_f32_16x16x4_f32,
// four products over K = 16: step s takes k = 4 (l / 16) + s from lane l).
// All accumulate in FP32.
constexpr int kMmBf16 = 0, kMmBf16x3 = 1, kMmF32 = 2;
template <int MODE, class MatF, class InF, class OutF>
__device__ __forceinline__ void mm_phase(int ncols, MatF mat, InF in, OutF out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int NW = NT<float> / 64;
  const int i = lane & 15, g = lane >> 4;
  mm_s4 av, al;
  float af[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const float x = mat(i, 4 * g + s);
    af[s] = x;
    if constexpr (MODE != kMmF32) av[s] = to_bf16(x);
    if constexpr (MODE == kMmBf16x3) al[s] = to_bf16(x - from_bf16(av[s]));
  }
#pragma unroll 1
  for (int tile = wave; tile * 16 < ncols; tile += NW) {
    const int j = tile * 16 + i;
    const bool live = j < ncols;
    mm_s4 bv, bl;
    float bf[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const float x = live ? in(4 * g + s, j) : 0.0f;
      bf[s] = x;
      if constexpr (MODE != kMmF32) bv[s] = to_bf16(x);
      if constexpr (MODE == kMmBf16x3) bl[s] = to_bf16(x - from_bf16(bv[s]));
    }
    mm_f4 c = {0.0f, 0.0f, 0.0f, 0.0f};
    if constexpr (MODE == kMmF32) {
#pragma unroll
      for (int s = 0; s < 4; ++s) c = __builtin_amdgcn_mfma_f32_16x16x4f32(af[s], bf[s], c, 0, 0, 0);
    } else {
      if constexpr (MODE == kMmBf16x3) {
        c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bv, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bl, c, 0, 0, 0);
      }
      c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, c, 0, 0, 0);
    }
    if (live) {
#pragma unroll
      for (int r = 0; r < 4; ++r) out(4 * g + r, j, c[r]);
    }
  }
}

// The slab-form operator (apply3) with its six interpolation contractions
// (x, y, z and their transposes) on the matrix cores; the collocation
// derivatives and the flux G grad stay in FP32 on the vector ALUs.
// GM: where the metric comes from (0 recomputed at every Gauss point from
// the Jacobian coefficients, 1 the LDS cache Gc, 2 the global copy Gg).
// VIN: the input is an interior vector with a zero patch boundary (read in
// place), else the closure values X.  epi(i, (A x)_i) is called once per
// interior row, in the last phase: rows of the z-plane that both cell layers
// share are summed in Out first (at their own rows).  An epilogue may
// change the input vector at row i: the second layer reads only its own
// planes, none of which the first layer's epilogue calls touch.
template <int Q, int GM, int MODE, bool VIN, class Epi>
__device__ __noinline__ void apply3mm(const LDSP float* __restrict__ X, Epi epi, LDSP float* __restrict__ Out,
                                      LDSP float* __restrict__ ab, const LDSP float* __restrict__ Bt,
                                      const LDSP float* __restrict__ Dc,
                                      const LDSP float* __restrict__ xg,
                                      const LDSP float* __restrict__ wg,
                                      const LDSP float* __restrict__ jc,
                                      const LDSP float* __restrict__ mu,
                                      const LDSP float* __restrict__ Gc,
                                      const GLBP float* __restrict__ Gg) {
  using T = float;
  using SH = Sh<3, Q>;
  constexpr int n = SH::n, m = SH::m, mi = SH::mi, NQ = SH::NQ, S = SH::S, NQ2 = NQ * NQ;
  static_assert(NQ <= 16 && m <= 16, "one matrix-core tile per contraction");
  LDSP T* A = ab;
  LDSP T* Bf = ab + S;
  LDSP T* C = ab + 2 * S;
  LDSP T* Dd = ab + 3 * S;
  const int tid = threadIdx.x;
  // patch-level 1D interpolation matrix: row = Gauss point QA = c n + k of
  // cell c, column = closure node x; B[k][x - c q] inside cell c, else 0
  auto Bp = [&](int QA, int x) -> T {
    const int c = QA >= n ? 1 : 0, k = QA - c * n, a = x - c * Q;
    return (QA < NQ && x < m && a >= 0 && a <= Q) ? Bt[k * n + a] : T(0);
  };
  auto Bc = [&](int k, int a) -> T { return (k < n && a < n) ? Bt[k * n + a] : T(0); };
#pragma unroll 1
  for (int cz = 0; cz < 2; ++cz) {
    // the slab's metric from global memory, loaded before the contractions
    // so that its latency hides behind them
    constexpr int kGIt = GM == 2 ? (S + NT<T> - 1) / NT<T> : 1;
    T Gp[kGIt][6];
    if constexpr (GM == 2) {
#pragma unroll
      for (int it = 0; it < kGIt; ++it) {
        const int idx = tid + it * NT<T>;
        const int gp = cz * S + (idx < S ? idx : 0);
#pragma unroll
        for (int c = 0; c < 6; ++c) Gp[it][c] = Gg[c * 2 * S + gp];
      }
    }
    // x: A[zl][y][QX] = sum_x Bp[QX][x] X[cz Q + zl][y][x]
    mm_phase<MODE>(
        n * m, Bp,
        [&](int x, int j) -> T {
          const int zc = cz * Q + j / m, y = j % m;
          if constexpr (VIN) {
            const bool in = x >= 1 && x < m - 1 && y >= 1 && y < m - 1 && zc >= 1 && zc < m - 1;
            return in ? X[((zc - 1) * mi + (y - 1)) * mi + (x - 1)] : T(0);
          } else {
            return x < m ? X[zc * m * m + y * m + x] : T(0);
          }
        },
        [&](int QX, int j, T v) {
          if (QX < NQ) A[j * NQ + QX] = v;
        });
    __syncthreads();
    // y: Bf[zl][QY][QX] = sum_y Bp[QY][y] A[zl][y][QX]
    mm_phase<MODE>(
        n * NQ, Bp,
        [&](int y, int j) -> T { return y < m ? A[((j / NQ) * m + y) * NQ + j % NQ] : T(0); },
        [&](int QY, int j, T v) {
          if (QY < NQ) Bf[((j / NQ) * NQ + QY) * NQ + j % NQ] = v;
        });
    __syncthreads();
    // z: C[kz][QY][QX] = sum_zl B[kz][zl] Bf[zl][QY][QX]
    mm_phase<MODE>(
        NQ2, Bc, [&](int zl, int j) -> T { return zl < n ? Bf[zl * NQ2 + j] : T(0); },
        [&](int kz, int j, T v) {
          if (kz < n) C[kz * NQ2 + j] = v;
        });
    __syncthreads();
    // reference gradients by collocation, then the flux G grad (FP32)
    auto flux = [&](int idx, auto metric) {
      const int QX = idx % NQ, t = idx / NQ, QY = t % NQ, kz = t / NQ;
      const int cx = QX >= n, kx = QX - cx * n, cy = QY >= n, ky = QY - cy * n;
      const LDSP T* dx = Dc + kx * n;
      const LDSP T* dy = Dc + ky * n;
      const LDSP T* dz = Dc + kz * n;
      const LDSP T* cxr = C + (kz * NQ + QY) * NQ + cx * n;
      const LDSP T* cyr = C + (kz * NQ + cy * n) * NQ + QX;
      const LDSP T* czr = C + QY * NQ + QX;
      T gx = 0, gy = 0, gz = 0;
#pragma unroll
      for (int a = 0; a < n; ++a) {
        gx += dx[a] * cxr[a];
        gy += dy[a] * cyr[a * NQ];
        gz += dz[a] * czr[a * NQ2];
      }
      T G[6];
      metric(G, cx, cy, kx, ky, kz);
      A[idx] = G[0] * gx + G[1] * gy + G[2] * gz;
      Bf[idx] = G[1] * gx + G[3] * gy + G[4] * gz;
      Dd[idx] = G[2] * gx + G[4] * gy + G[5] * gz;
    };
    if constexpr (GM == 2) {
#pragma unroll
      for (int it = 0; it < kGIt; ++it) {
        const int idx = tid + it * NT<T>;
        if (idx < S)
          flux(idx, [&](T* G, int, int, int, int, int) {
#pragma unroll
            for (int c = 0; c < 6; ++c) G[c] = Gp[it][c];
          });
      }
    } else {
#pragma unroll 1
      for (int idx = tid; idx < S; idx += NT<T>)
        flux(idx, [&](T* G, int cx, int cy, int kx, int ky, int kz) {
          if constexpr (GM == 1) {
            const int gp = cz * S + idx;
#pragma unroll
            for (int c = 0; c < 6; ++c) G[c] = Gc[c * 2 * S + gp];
          } else {
            const int cell = cz * 4 + cy * 2 + cx;
            metric3c<T>(jc + cell * 36, xg[kx], xg[ky], xg[kz], mu[cell] * wg[kx] * wg[ky] * wg[kz], G);
          }
        });
    }
    __syncthreads();
    // transposed collocation: C = Dc^T F (FP32)
#pragma unroll 1
    for (int idx = tid; idx < S; idx += NT<T>) {
      const int QX = idx % NQ, t = idx / NQ, QY = t % NQ, kz = t / NQ;
      const int cx = QX >= n, kx = QX - cx * n, cy = QY >= n, ky = QY - cy * n;
      const LDSP T* fx = A + (kz * NQ + QY) * NQ + cx * n;
      const LDSP T* fy = Bf + (kz * NQ + cy * n) * NQ + QX;
      const LDSP T* fz = Dd + QY * NQ + QX;
      T acc = 0;
#pragma unroll
      for (int a = 0; a < n; ++a) {
        acc += Dc[a * n + kx] * fx[a];
        acc += Dc[a * n + ky] * fy[a * NQ];
        acc += Dc[a * n + kz] * fz[a * NQ2];
      }
      C[idx] = acc;
    }
    __syncthreads();
    // z^T: A[zl][QY][QX] = sum_kz B[kz][zl] C[kz][QY][QX]
    mm_phase<MODE>(
        NQ2, [&](int zl, int kz) -> T { return Bc(kz, zl); },
        [&](int kz, int j) -> T { return kz < n ? C[kz * NQ2 + j] : T(0); },
        [&](int zl, int j, T v) {
          if (zl < n) A[zl * NQ2 + j] = v;
        });
    __syncthreads();
    // y^T onto interior rows: Bf[zl][yi][QX] = sum_QY Bp[QY][yi + 1] A[zl][QY][QX]
    mm_phase<MODE>(
        n * NQ, [&](int yi, int QY) -> T { return yi < mi ? Bp(QY, yi + 1) : T(0); },
        [&](int QY, int j) -> T { return QY < NQ ? A[((j / NQ) * NQ + QY) * NQ + j % NQ] : T(0); },
        [&](int yi, int j, T v) {
          if (yi < mi) Bf[((j / NQ) * mi + yi) * NQ + j % NQ] = v;
        });
    __syncthreads();
    // x^T onto interior columns and the interior z-planes of this slab
    const int zl0 = cz == 0 ? 1 : 0;
    mm_phase<MODE>(
        Q * mi, [&](int xi, int QX) -> T { return xi < mi ? Bp(QX, xi + 1) : T(0); },
        [&](int QX, int j) -> T {
          return QX < NQ ? Bf[((zl0 + j / mi) * mi + j % mi) * NQ + QX] : T(0);
        },
        [&](int xi, int j, T v) {
          if (xi < mi) {
            const int zl = zl0 + j / mi, yi = j % mi;
            const int zz = cz * Q + zl - 1, row = (zz * mi + yi) * mi + xi;
            LDSP T* o = Out + row;  // rows of the shared plane zz = Q - 1
            if (zz != Q - 1)
              epi(row, v);
            else if (cz == 0)
              *o = v;
            else
              epi(row, *o + v);
          }
        });
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// 3D level operator in segment form
//
// Every contraction phase works on line segments: a work item reads the n =
// q+1 values of one cell segment of a line, multiplies them by the n x n 1D
// matrix (uniform across the wavefront, so it sits in scalar registers) and
// writes n values.  Intermediate results use a cell-local layout per
// direction (index c n + a for local node a of cell c), in which the node
// shared by the two cells of a line appears twice; the transposed
// contractions therefore never add into a shared node, and the duplicates
// are summed once in the final assembly of the interior rows.  An input with
// a zero patch boundary (a level vector) is read in interior layout directly.
// ---------------------------------------------------------------------------

template <typename T, int Q>
struct Seg3 {
  static constexpr int n = Q + 1, m = 2 * Q + 1, mi = 2 * Q - 1, NQ = 2 * n;
  static constexpr int P = NQ * NQ * NQ;  // one buffer
  static constexpr int NB = 2 * n - 2;    // cell-local indices of interior nodes
};

// Epilogues: what to do with row i of A x (fused into the last phase).
// PT is the pointer type of the vectors: LDS-qualified when they live in LDS.
template <typename T, class PT>
struct EpiStore {  // out = A x
  PT out;
  __device__ __forceinline__ void operator()(int i, T v) const { out[i] = v; }
};
template <typename T, class PT>
struct EpiResidual {  // res = f - A x
  PT f, res;
  __device__ __forceinline__ void operator()(int i, T v) const { res[i] = f[i] - v; }
};
template <typename T, class PT, class DT = PT>
struct EpiChebStart {  // res = f - A x, z = D^{-1} res / theta
  PT f, res, z;
  DT dinv;
  T inv_theta;
  __device__ __forceinline__ void operator()(int i, T v) const {
    const T r = f[i] - v;
    res[i] = r;
    z[i] = dinv[i] * r * inv_theta;
  }
};
template <typename T, class PT, class DT = PT>
struct EpiChebStep {  // x += z, res -= A z, z = c1 z + c2 D^{-1} res
  PT x, res, z;
  DT dinv;
  T c1, c2;
  __device__ __forceinline__ void operator()(int i, T v) const {
    const T zi = z[i];
    x[i] += zi;
    const T r = res[i] - v;
    res[i] = r;
    z[i] = c1 * zi + c2 * dinv[i] * r;
  }
};

template <typename T, int Q, bool CLOSURE_IN, bool CACHE, class Epi>
__device__ __forceinline__ void apply3seg_body(const LDSP T* __restrict__ in, Epi epi,
                                       LDSP T* __restrict__ ab, const LDSP T* __restrict__ Bl,
                                       const LDSP T* __restrict__ Dcl,
                                       const LDSP T* __restrict__ jc, const LDSP T* __restrict__ mu,
                                       const LDSP T* __restrict__ Gc) {
  using SG = Seg3<T, Q>;
  constexpr int n = SG::n, m = SG::m, mi = SG::mi, NQ = SG::NQ, P = SG::P;
  const T* gB = ctab<T>() + ctab_off(Q);
  const T* gDc = gB + n * n;
  const T* xg = gB + 3 * n * n;
  const T* wg = xg + n;
  constexpr int R0 = CLOSURE_IN ? 0 : 1;   // first node row held by the input
  constexpr int NR = CLOSURE_IN ? m : mi;  // node rows held per direction
  constexpr int NQ2 = NQ * NQ;
  LDSP T* A = ab;
  LDSP T* Bb = ab + P;
  LDSP T* C = ab + 2 * P;
  LDSP T* D = ab + 3 * P;
  const int tid = threadIdx.x;

  // 1. x: A[zr][yr][QX] = sum_a B[k][a] in[zr][yr][cx q + a]
#pragma unroll 1
  for (int it = tid; it < 2 * NR * NR; it += NT<T>) {
    const int line = it % (NR * NR), cx = it / (NR * NR);
    const LDSP T* src = in + line * NR;
    T v[n];
#pragma unroll
    for (int a = 0; a < n; ++a) {
      const int x = cx * Q + a;
      v[a] = (CLOSURE_IN || (x >= 1 && x <= m - 2)) ? src[x - R0] : T(0);
    }
    LDSP T* dst = A + line * NQ + cx * n;
#pragma unroll
    for (int k = 0; k < n; ++k) {
      T acc = 0;
#pragma unroll
      for (int a = 0; a < n; ++a) acc += gB[k * n + a] * v[a];
      dst[k] = acc;
    }
  }
  __syncthreads();
  // 2. y: Bb[zr][QY][QX] = sum_a B[k][a] A[zr][cy q + a][QX]
#pragma unroll 1
  for (int it = tid; it < 2 * NR * NQ; it += NT<T>) {
    const int QX = it % NQ, r = it / NQ, zr = r % NR, cy = r / NR;
    T v[n];
#pragma unroll
    for (int a = 0; a < n; ++a) {
      const int y = cy * Q + a;
      v[a] = (CLOSURE_IN || (y >= 1 && y <= m - 2)) ? A[(zr * NR + (y - R0)) * NQ + QX] : T(0);
    }
    LDSP T* dst = Bb + (zr * NQ + cy * n) * NQ + QX;
#pragma unroll
    for (int k = 0; k < n; ++k) {
      T acc = 0;
#pragma unroll
      for (int a = 0; a < n; ++a) acc += gB[k * n + a] * v[a];
      dst[k * NQ] = acc;
    }
  }
  __syncthreads();
  // 3. z: C[QZ][QY][QX] = sum_a B[k][a] Bb[cz q + a][QY][QX]   (values at Gauss points)
#pragma unroll 1
  for (int it = tid; it < 2 * NQ2; it += NT<T>) {
    const int col = it % NQ2, cz = it / NQ2;
    T v[n];
#pragma unroll
    for (int a = 0; a < n; ++a) {
      const int z = cz * Q + a;
      v[a] = (CLOSURE_IN || (z >= 1 && z <= m - 2)) ? Bb[(z - R0) * NQ2 + col] : T(0);
    }
    LDSP T* dst = C + cz * n * NQ2 + col;
#pragma unroll
    for (int k = 0; k < n; ++k) {
      T acc = 0;
#pragma unroll
      for (int a = 0; a < n; ++a) acc += gB[k * n + a] * v[a];
      dst[k * NQ2] = acc;
    }
  }
  __syncthreads();
  // 4. reference gradients by collocation and the flux G grad; a thread owns
  //    one local Gauss point (kx, ky, kz) of the four cells of layer cz
  constexpr int n3 = n * n * n;
#pragma unroll 1
  for (int t = tid; t < 2 * n3; t += NT<T>) {
    const int k3 = t % n3, cz = t / n3;
    const int kx = k3 % n, ky = (k3 / n) % n, kz = k3 / (n * n);
    T dx[n], dy[n], dz[n];
#pragma unroll
    for (int a = 0; a < n; ++a) {
      dx[a] = Dcl[kx * n + a];
      dy[a] = Dcl[ky * n + a];
      dz[a] = Dcl[kz * n + a];
    }
    const int QZ = cz * n + kz;
#pragma unroll 2
    for (int cc = 0; cc < 4; ++cc) {
      const int cx = cc & 1, cy = cc >> 1;
      const int QY = cy * n + ky, QX = cx * n + kx;
      const int pt = (QZ * NQ + QY) * NQ + QX;
      const LDSP T* rx = C + (QZ * NQ + QY) * NQ + cx * n;
      const LDSP T* ry = C + (QZ * NQ + cy * n) * NQ + QX;
      const LDSP T* rz = C + (cz * n * NQ + QY) * NQ + QX;
      T gx = 0, gy = 0, gz = 0;
#pragma unroll
      for (int a = 0; a < n; ++a) {
        gx += dx[a] * rx[a];
        gy += dy[a] * ry[a * NQ];
        gz += dz[a] * rz[a * NQ2];
      }
      T G[6];
      if constexpr (CACHE) {
#pragma unroll
        for (int g = 0; g < 6; ++g) G[g] = Gc[g * P + pt];
      } else {
        const int cell = cz * 4 + cy * 2 + cx;
        metric3c<T>(jc + cell * 36, xg[kx], xg[ky], xg[kz], mu[cell] * wg[kx] * wg[ky] * wg[kz], G);
      }
      A[pt] = G[0] * gx + G[1] * gy + G[2] * gz;
      Bb[pt] = G[1] * gx + G[3] * gy + G[4] * gz;
      D[pt] = G[2] * gx + G[4] * gy + G[5] * gz;
    }
  }
  __syncthreads();
  // 5. transposed collocation W = Dc^T F along the z segment of one cell of
  //    a Gauss-point column, then z^T of that cell: C[zc][QY][QX] in the
  //    cell-local z layout (zc = cz n + a; the shared node appears twice)
#pragma unroll 1
  for (int it = tid; it < 2 * NQ2; it += NT<T>) {
    const int col = it % NQ2, cz = it / NQ2;
    const int QX = col % NQ, QY = col / NQ;
    const int cx = QX >= n, kx = QX - cx * n, cy = QY >= n, ky = QY - cy * n;
    T ex[n], ey[n], f2[n];
#pragma unroll
    for (int a = 0; a < n; ++a) {
      ex[a] = Dcl[a * n + kx];
      ey[a] = Dcl[a * n + ky];
      f2[a] = D[(cz * n + a) * NQ2 + col];
    }
    T w[n];
    // plane k of this cell layer is a constant offset k NQ^2 from these
    const LDSP T* fx0 = A + (cz * n * NQ + QY) * NQ + cx * n;
    const LDSP T* fy0 = Bb + (cz * n * NQ + cy * n) * NQ + QX;
#pragma unroll
    for (int k = 0; k < n; ++k) {
      const LDSP T* fx = fx0 + k * NQ2;
      const LDSP T* fy = fy0 + k * NQ2;
      // one multiply-add per term (a single fused chain, no zero start)
      T acc = gDc[k] * f2[0];
#pragma unroll
      for (int a = 0; a < n; ++a) {
        if (a > 0) acc = fma(gDc[a * n + k], f2[a], acc);
        acc = fma(ex[a], fx[a], acc);
        acc = fma(ey[a], fy[a * NQ], acc);
      }
      w[k] = acc;
    }
    LDSP T* dst = C + cz * n * NQ2 + col;
#pragma unroll
    for (int a = 0; a < n; ++a) {
      T acc = 0;
#pragma unroll
      for (int k = 0; k < n; ++k) acc += gB[k * n + a] * w[k];
      dst[a * NQ2] = acc;
    }
  }
  __syncthreads();
  // 6. y^T, one interior (z, y) pair and one QX per item; the two cell-local
  //    copies of the shared z node are summed on read: A[zi][yi][QX].
  //    Branch-free: both copies and both y cells are read for every item
  //    (the second copy with weight 0 off the shared node, a cell the node
  //    is not in with a clamped row, its sum discarded), so all loads are
  //    issued together.
#pragma unroll 1
  for (int it = tid; it < mi * mi * NQ; it += NT<T>) {
    const int QX = it % NQ, r = it / NQ, yi = r % mi, zi = r / mi;
    const int z = zi + 1, y = yi + 1;
    const int zc0 = z <= Q ? z : n + z - Q;          // cell-local z of node z
    const int zc1 = z == Q ? n : zc0;                 // its second copy (z = q)
    const T t1 = z == Q ? T(1) : T(0);
    const int a0 = y <= Q ? y : Q, a1 = y >= Q ? y - Q : 0;
    const LDSP T* s0 = C + zc0 * NQ2 + QX;
    const LDSP T* s1 = C + zc1 * NQ2 + QX;
    T v0[n], v1[n];
#pragma unroll
    for (int k = 0; k < n; ++k) {
      v0[k] = fma(t1, s1[k * NQ], s0[k * NQ]);
      v1[k] = fma(t1, s1[(n + k) * NQ], s0[(n + k) * NQ]);
    }
    T acc0 = Bl[a0] * v0[0], acc1 = Bl[a1] * v1[0];
#pragma unroll
    for (int k = 1; k < n; ++k) {
      acc0 = fma(Bl[k * n + a0], v0[k], acc0);
      acc1 = fma(Bl[k * n + a1], v1[k], acc1);
    }
    A[r * NQ + QX] = y < Q ? acc0 : (y > Q ? acc1 : acc0 + acc1);
  }
  __syncthreads();
  // 7. x^T, one interior row per item, handed to the epilogue with its
  //    interior index (the caller's vector update is fused here); both x
  //    cells computed, as in step 6
#pragma unroll 1
  for (int i = tid; i < mi * mi * mi; i += NT<T>) {
    const int xi = i % mi, line = i / mi;
    const int x = xi + 1;
    const int a0 = x <= Q ? x : Q, a1 = x >= Q ? x - Q : 0;
    const LDSP T* src = A + line * NQ;
    T acc0 = Bl[a0] * src[0], acc1 = Bl[a1] * src[n];
#pragma unroll
    for (int k = 1; k < n; ++k) {
      acc0 = fma(Bl[k * n + a0], src[k], acc0);
      acc1 = fma(Bl[k * n + a1], src[n + k], acc1);
    }
    epi(i, x < Q ? acc0 : (x > Q ? acc1 : acc0 + acc1));
  }
  __syncthreads();
}

// FP32 patches take the segment operator inline (their kernels are held to
// 128 registers so that two patches share a CU); FP64 patches call it out of
// line, which measured faster for them.
template <typename T, int Q, bool CLOSURE_IN, bool CACHE, class Epi>
__device__ __noinline__ void apply3seg_call(const LDSP T* __restrict__ in, Epi epi, LDSP T* __restrict__ ab,
                                            const LDSP T* __restrict__ Bl, const LDSP T* __restrict__ Dcl,
                                            const LDSP T* __restrict__ jc, const LDSP T* __restrict__ mu,
                                            const LDSP T* __restrict__ Gc) {
  apply3seg_body<T, Q, CLOSURE_IN, CACHE>(in, epi, ab, Bl, Dcl, jc, mu, Gc);
}
template <typename T, int Q, bool CLOSURE_IN, bool CACHE, class Epi>
__device__ __forceinline__ void apply3seg(const LDSP T* __restrict__ in, Epi epi, LDSP T* __restrict__ ab,
                                          const LDSP T* __restrict__ Bl, const LDSP T* __restrict__ Dcl,
                                          const LDSP T* __restrict__ jc, const LDSP T* __restrict__ mu,
                                          const LDSP T* __restrict__ Gc) {
  if constexpr (sizeof(T) == 4)
    apply3seg_body<T, Q, CLOSURE_IN, CACHE>(in, epi, ab, Bl, Dcl, jc, mu, Gc);
  else
    apply3seg_call<T, Q, CLOSURE_IN, CACHE>(in, epi, ab, Bl, Dcl, jc, mu, Gc);
}

template <typename T, int Q, bool CACHE>
__device__ __forceinline__ void apply2(const T* __restrict__ X, T* __restrict__ Out, T* __restrict__ ab,
                       const T* __restrict__ Bt, const T* __restrict__ Dc, const T* __restrict__ xg,
                       const T* __restrict__ wg, const T* __restrict__ jc, const T* __restrict__ mu,
                       const T* __restrict__ Gc) {
  using SH = Sh<2, Q>;
  constexpr int n = SH::n, m = SH::m, mi = SH::mi, NQ = SH::NQ;
  T* A = ab;
  T* Bf = ab + SH::S;
  T* C = ab + 2 * SH::S;
  const int tid = threadIdx.x;
#pragma unroll 1
  for (int cy = 0; cy < 2; ++cy) {
    // x: A[yl][QX] = sum_a B[kx][a] X[cy Q + yl][cx Q + a]
#pragma unroll 1
    for (int idx = tid; idx < n * NQ; idx += NT<T>) {
      const int QX = idx % NQ, yl = idx / NQ;
      const int cx = QX >= n, kx = QX - cx * n;
      const T* xr = X + (cy * Q + yl) * m + cx * Q;
      T acc = 0;
#pragma unroll
      for (int a = 0; a < n; ++a) acc += Bt[kx * n + a] * xr[a];
      A[idx] = acc;
    }
    __syncthreads();
    // y: C[ky][QX] = sum_yl B[ky][yl] A[yl][QX]
#pragma unroll 1
    for (int idx = tid; idx < n * NQ; idx += NT<T>) {
      const int QX = idx % NQ, ky = idx / NQ;
      T acc = 0;
#pragma unroll
      for (int a = 0; a < n; ++a) acc += Bt[ky * n + a] * A[a * NQ + QX];
      C[idx] = acc;
    }
    __syncthreads();
#pragma unroll 1
    for (int idx = tid; idx < n * NQ; idx += NT<T>) {
      const int QX = idx % NQ, ky = idx / NQ;
      const int cx = QX >= n, kx = QX - cx * n;
      T gx = 0, gy = 0;
#pragma unroll
      for (int a = 0; a < n; ++a) {
        gx += Dc[kx * n + a] * C[ky * NQ + cx * n + a];
        gy += Dc[ky * n + a] * C[a * NQ + QX];
      }
      T G[3];
      if constexpr (CACHE) {
        const int gp = cy * SH::S + idx;
#pragma unroll
        for (int c = 0; c < 3; ++c) G[c] = Gc[c * 2 * SH::S + gp];
      } else {
        const int cell = cy * 2 + cx;
        metric2c<T>(jc + cell * 8, xg[kx], xg[ky], mu[cell] * wg[kx] * wg[ky], G);
      }
      A[idx] = G[0] * gx + G[1] * gy;
      Bf[idx] = G[1] * gx + G[2] * gy;
    }
    __syncthreads();
#pragma unroll 1
    for (int idx = tid; idx < n * NQ; idx += NT<T>) {
      const int QX = idx % NQ, ky = idx / NQ;
      const int cx = QX >= n, kx = QX - cx * n;
      T acc = 0;
#pragma unroll
      for (int a = 0; a < n; ++a) {
        acc += Dc[a * n + kx] * A[ky * NQ + cx * n + a];
        acc += Dc[a * n + ky] * Bf[a * NQ + QX];
      }
      C[idx] = acc;
    }
    __syncthreads();
    // y^T: A[yl][QX] = sum_ky B[ky][yl] C[ky][QX]
#pragma unroll 1
    for (int idx = tid; idx < n * NQ; idx += NT<T>) {
      const int QX = idx % NQ, yl = idx / NQ;
      T acc = 0;
#pragma unroll
      for (int k = 0; k < n; ++k) acc += Bt[k * n + yl] * C[k * NQ + QX];
      A[idx] = acc;
    }
    __syncthreads();
    const int yl0 = cy == 0 ? 1 : 0;
#pragma unroll 1
    for (int idx = tid; idx < Q * mi; idx += NT<T>) {
      const int xi = idx % mi, yl = yl0 + idx / mi;
      const int x = xi + 1;
      const T* ar = A + yl * NQ;
      T acc = 0;
      if (x <= Q) {
#pragma unroll
        for (int k = 0; k < n; ++k) acc += Bt[k * n + x] * ar[k];
      }
      if (x >= Q) {
#pragma unroll
        for (int k = 0; k < n; ++k) acc += Bt[k * n + (x - Q)] * ar[n + k];
      }
      const int yy = cy * Q + yl - 1;
      T* o = Out + yy * mi + xi;
      if (cy == 1 && yl == 0)
        *o += acc;
      else
        *o = acc;
    }
    __syncthreads();
  }
}

// FP32 slab-form level on the matrix cores (apply3mm): input x (closure
// values, or with VIN an interior vector with zero boundary), epi(i, (A x)_i)
template <typename T, int DIM, class LV, int L>
constexpr bool slab_mm() {
  return DIM == 3 && std::is_same<T, float>::value && L == 0 && LV::q[L] <= 7 &&
         !Layout<T, DIM, LV>::use_seg(L) && !Layout<T, DIM, LV>::use_quarter(L);
}
template <typename T, int DIM, class LV, int L, bool VIN, class Epi>
__device__ __forceinline__ void apply_slab_mm(const Ctx<T, DIM, LV>& c, const T* x, Epi epi) {
  if constexpr (slab_mm<T, DIM, LV, L>()) {
    constexpr int Q = LV::q[L];
    static_assert(4 * Sh<3, Q>::S <= Layout<T, DIM, LV>::abuf_elems, "slab buffers exceed the work area");
    constexpr int MODE = !LV::bf16 ? kMmF32 : (LV::split ? kMmBf16x3 : kMmBf16);
    constexpr int GM0 = Layout<T, DIM, LV>::cache_level(L) ? 1 : 0;
    if (Layout<T, DIM, LV>::G_global && c.Gg)
      apply3mm<Q, 2, MODE, VIN>(lds_cast(x), epi, lds_cast(c.Out()), lds_cast(c.abuf()), lds_cast(c.tabB(L)),
                                lds_cast(c.tabDc(L)), lds_cast(c.tabXg(L)), lds_cast(c.tabWg(L)),
                                lds_cast(c.jc()), lds_cast(c.mu()), lds_cast(c.Gc(L)), glb_cast(c.Gg));
    else
      apply3mm<Q, GM0, MODE, VIN>(lds_cast(x), epi, lds_cast(c.Out()), lds_cast(c.abuf()),
                                  lds_cast(c.tabB(L)), lds_cast(c.tabDc(L)), lds_cast(c.tabXg(L)),
                                  lds_cast(c.tabWg(L)), lds_cast(c.jc()), lds_cast(c.mu()), lds_cast(c.Gc(L)),
                                  nullptr);
  }
}

template <typename T, int DIM, class LV, int L>
__device__ __forceinline__ void apply_level(const Ctx<T, DIM, LV>& c) {
  constexpr int Q = LV::q[L];
  constexpr bool CACHE = Layout<T, DIM, LV>::cache_level(L);
  if constexpr (Layout<T, DIM, LV>::use_seg(L))
    apply3seg<T, Q, true, CACHE>(lds_cast(c.X()), EpiStore<T, LDSP T*>{lds_cast(c.Out())},
                                 lds_cast(c.abuf()), lds_cast(c.tabB(L)), lds_cast(c.tabDc(L)),
                                 lds_cast(c.jc()),
                                 lds_cast(c.mu()), lds_cast(c.Gc(L)));
  else if constexpr (Layout<T, DIM, LV>::use_quarter(L)) {
    static_assert(4 * (Q + 1) * (Q + 1) * 2 * (Q + 1) <= Layout<T, DIM, LV>::abuf_elems,
                  "quarter-slab buffers exceed the work area");
    apply3q<T, Q, CACHE>(lds_cast(c.X()), lds_cast(c.Out()), lds_cast(c.abuf()),
                         lds_cast(c.tabB(L)), lds_cast(c.tabDc(L)), lds_cast(c.tabXg(L)),
                         lds_cast(c.tabWg(L)), lds_cast(c.jc()), lds_cast(c.mu()),
                         lds_cast(c.Gc(L)));
  } else if constexpr (DIM == 3 && std::is_same<T, float>::value && L == 0 && Q <= 7) {
    // slab-form top level in FP32 storage: contractions on the matrix cores
    // (BF16 or split-BF16 operands for those variants, FP32 operands else)
    static_assert(4 * Sh<3, Q>::S <= Layout<T, DIM, LV>::abuf_elems,
                  "slab buffers exceed the work area");
    apply_slab_mm<T, DIM, LV, L, false>(c, c.X(), EpiStore<T, LDSP T*>{lds_cast(c.Out())});
  } else if constexpr (DIM == 3) {
    static_assert(4 * Sh<3, Q>::S <= Layout<T, DIM, LV>::abuf_elems,
                  "slab buffers exceed the work area");
    apply3<T, Q, CACHE>(lds_cast(c.X()), lds_cast(c.Out()), lds_cast(c.abuf()), lds_cast(c.tabB(L)),
                        lds_cast(c.tabDc(L)), lds_cast(c.tabXg(L)), lds_cast(c.tabWg(L)),
                        lds_cast(c.jc()), lds_cast(c.mu()), lds_cast(c.Gc(L)));
  }
  else
    apply2<T, Q, CACHE>(c.X(), c.Out(), c.abuf(), c.tabB(L), c.tabDc(L), c.tabXg(L), c.tabWg(L),
                        c.jc(), c.mu(), c.Gc(L));
}

// Metric at every Gauss point of every level (when cached in LDS) and the
// per-cell Jacobian coefficients; requires the geometry to be loaded.
template <typename T, int DIM, class LV>
__device__ void prepare_geometry(const Ctx<T, DIM, LV>& c, bool any_level = true) {
  using Lay = Layout<T, DIM, LV>;
  if (c.metric_loaded) {
    // the cached metric came from the setup; the Jacobian coefficients only
    // serve levels that recompute theirs: those the V-cycle applies without
    // a cached metric, or any level when any_level (a single level apply)
    if (Lay::needs_jc || any_level) {
      jacobian_coefficients<T, DIM>(c.geo(), c.jc());
      __syncthreads();
    }
    return;
  }
  jacobian_coefficients<T, DIM>(c.geo(), c.jc());
  __syncthreads();
  if constexpr (Lay::cache_G) {
    for (int l = 0; l < LV::count; ++l) {
      const int n = LV::q[l] + 1, NQ = 2 * n;
      const int NP = Lay::cache_level(l) ? Lay::npts(l) : 0;  // 0: not cached
      const T* xg = c.tabXg(l);
      const T* wg = c.tabWg(l);
      T* Gl = c.Gc(l);
      for (int pt = threadIdx.x; pt < NP; pt += NT<T>) {
        const int QX = pt % NQ, QY = (pt / NQ) % NQ, QZ = DIM == 3 ? pt / (NQ * NQ) : 0;
        const int cx = QX >= n, cy = QY >= n, cz = QZ >= n;
        const int kx = QX - cx * n, ky = QY - cy * n, kz = QZ - cz * n;
        if constexpr (DIM == 3) {
          const int cell = cz * 4 + cy * 2 + cx;
          T G[6];
          metric3c<T>(c.jc() + cell * 36, xg[kx], xg[ky], xg[kz],
                      c.mu()[cell] * wg[kx] * wg[ky] * wg[kz], G);
          for (int g = 0; g < 6; ++g) Gl[g * NP + pt] = G[g];
        } else {
          const int cell = cy * 2 + cx;
          T G[3];
          metric2c<T>(c.jc() + cell * 8, xg[kx], xg[ky], c.mu()[cell] * wg[kx] * wg[ky], G);
          for (int g = 0; g < 3; ++g) Gl[g * NP + pt] = G[g];
        }
      }
    }
    __syncthreads();
  }
}

// X <- closure layout of an interior vector (zero on the patch boundary)
template <typename T, int DIM, int Q>
__device__ __forceinline__ void load_closure(T* __restrict__ X, const T* __restrict__ v) {
  using SH = Sh<DIM, Q>;
  constexpr int m = SH::m, mi = SH::mi;
#pragma unroll 1
  for (int idx = threadIdx.x; idx < SH::closure; idx += NT<T>) {
    const int x = idx % m, t = idx / m, y = t % m;
    const int zc = DIM == 3 ? t / m : 0;
    bool in = x > 0 && x < m - 1 && y > 0 && y < m - 1;
    if (DIM == 3) in = in && zc > 0 && zc < m - 1;
    int ii = (y - 1) * mi + (x - 1);
    if (DIM == 3) ii += (zc - 1) * mi * mi;
    X[idx] = in ? v[ii] : T(0);
  }
  __syncthreads();
}

// Out = A_{j,q} v
// Vector pointer type of a layout: LDS-qualified when the vectors live in LDS.
template <typename T, int DIM, class LV>
using VecPtr = typename std::conditional<Layout<T, DIM, LV>::vec_in_lds, LDSP T*, T*>::type;
template <typename T, int DIM, class LV>
__device__ __forceinline__ VecPtr<T, DIM, LV> vp(T* p) {
  return (VecPtr<T, DIM, LV>)p;
}

// epi(i, (A_{j,q} v)_i) for every interior row i; v has a zero patch boundary
template <typename T, int DIM, class LV, int L, class Epi>
__device__ __forceinline__ void apply_vec_epi(const Ctx<T, DIM, LV>& c, const T* v, Epi epi) {
  constexpr int Q = LV::q[L];
  using Lay = Layout<T, DIM, LV>;
  if constexpr (Lay::dense_global(L)) {
    if (c.dense_ok) {
      // symmetric: column j is row j, so threads of consecutive rows read
      // consecutive addresses; four partial sums per row, added in LDS
      constexpr int N = Lay::level_size(L);
      constexpr int NP = NT<T> / N >= 4 ? 4 : NT<T> / N;
      constexpr int CH = (N + NP - 1) / NP;
      static_assert(NP >= 1 && NP * N <= Lay::abuf_elems, "dense global apply layout");
      const T* M = c.dglob[L];
      T* part = c.abuf();
      const int t = threadIdx.x;
      if (t < NP * N) {
        const int i = t % N, ch = t / N;
        // the chunk's loads issued in batches before their sums: all at once
        // in FP32 (these levels occur under slab-form tops, which hold one
        // workgroup per CU by their LDS, so registers are free), eight at a
        // time in FP64, where more in flight would cost workgroups per CU
        constexpr int BT = sizeof(T) == 4 ? CH : 8;
        T acc = 0;
#pragma unroll 1
        for (int j0 = 0; j0 < CH; j0 += BT) {
          T mv[BT];
#pragma unroll
          for (int jj = 0; jj < BT; ++jj) {
            const int j = ch * CH + j0 + jj;
            mv[jj] = (j0 + jj < CH && j < N) ? M[(int64_t)j * N + i] : T(0);
          }
#pragma unroll
          for (int jj = 0; jj < BT; ++jj) {
            const int j = ch * CH + j0 + jj;
            acc += (j0 + jj < CH && j < N) ? mv[jj] * v[j] : T(0);
          }
        }
        part[ch * N + i] = acc;
      }
      __syncthreads();
      for (int i = threadIdx.x; i < N; i += NT<T>) {
        T acc = 0;
#pragma unroll
        for (int ch = 0; ch < NP; ++ch) acc += part[ch * N + i];
        epi(i, acc);
      }
      __syncthreads();
      return;
    }
  }
  if constexpr (Lay::dense_level(L)) {
    if (c.dense_ok) {
      constexpr int N = Lay::level_size(L);
      const T* M = c.dense(L);
      for (int i = threadIdx.x; i < N; i += NT<T>) {
        T acc = 0;
#pragma unroll
        for (int j = 0; j < N; ++j) acc += M[i * N + j] * v[j];
        epi(i, acc);
      }
      __syncthreads();
      return;
    }
  }
  if constexpr (Lay::use_seg(L) && Lay::vec_in_lds) {
    apply3seg<T, Q, false, Lay::cache_level(L)>(lds_cast(v), epi, lds_cast(c.abuf()), lds_cast(c.tabB(L)),
                                         lds_cast(c.tabDc(L)), lds_cast(c.jc()), lds_cast(c.mu()),
                                         lds_cast(c.Gc(L)));
  } else if constexpr (slab_mm<T, DIM, LV, L>() && Lay::vec_in_lds) {
    // input read in place; the epilogue in a pass of its own (in the last
    // phase it would raise the operator's registers past the file)
    apply_slab_mm<T, DIM, LV, L, true>(c, v, EpiStore<T, LDSP T*>{lds_cast(c.Out())});
    constexpr int N = Lay::level_size(L);
#pragma unroll 1
    for (int i = threadIdx.x; i < N; i += NT<T>) epi(i, c.Out()[i]);
    __syncthreads();
  } else {
    load_closure<T, DIM, Q>(c.X(), v);
    apply_level<T, DIM, LV, L>(c);
    constexpr int N = Lay::level_size(L);
#pragma unroll 1
    for (int i = threadIdx.x; i < N; i += NT<T>) epi(i, c.Out()[i]);
    __syncthreads();
  }
}

// Out = A_{j,q} v
template <typename T, int DIM, class LV, int L>
__device__ __forceinline__ void apply_vec(const Ctx<T, DIM, LV>& c, const T* v) {
  apply_vec_epi<T, DIM, LV, L>(c, v, EpiStore<T, VecPtr<T, DIM, LV>>{vp<T, DIM, LV>(c.Out())});
}

// Chebyshev-accelerated Jacobi on A_{j,q} x = f over [theta - delta, theta + delta]
// (Saad, Iterative Methods for Sparse Linear Systems, Algorithm 12.1, with
// D^{-1} applied to the residuals).  Degree 1 on an interval with
// theta = 2 is the paper's damped Jacobi step with omega = 1/2.
template <typename T, int DIM, class LV, int L>
__device__ __forceinline__ void chebyshev(const Ctx<T, DIM, LV>& c, int k, bool x_zero) {
  constexpr int N = Layout<T, DIM, LV>::level_size(L);
  using PT = VecPtr<T, DIM, LV>;
  PT f = vp<T, DIM, LV>(c.r(L));
  PT x = vp<T, DIM, LV>(c.d(L));
  PT res = vp<T, DIM, LV>(c.res());
  PT z = vp<T, DIM, LV>(c.z());
  // the top level's inverse diagonal may live in global memory
  using DT = typename std::conditional<Layout<T, DIM, LV>::dinv0_global && L == 0, const T*, PT>::type;
  DT dinv = (DT)c.dinv(L);
  const T theta = c.cheb()[2 * L], delta = c.cheb()[2 * L + 1];
  const T sigma = theta / delta;
  T rho = T(1) / sigma;
  const int tid = threadIdx.x;
  if (x_zero) {
    // r_0 = f, z_0 = D^{-1} f / theta, x = 0
#pragma unroll 1
    for (int i = tid; i < N; i += NT<T>) {
      res[i] = f[i];
      z[i] = dinv[i] * f[i] / theta;
      x[i] = 0;
    }
    __syncthreads();
  } else {
    // r_0 = f - A x, z_0 = D^{-1} r_0 / theta
    apply_vec_epi<T, DIM, LV, L>(c, c.d(L), EpiChebStart<T, PT, DT>{f, res, z, dinv, T(1) / theta});
  }
  for (int it = 0; it + 1 < k; ++it) {
    // x += z_i, r_{i+1} = r_i - A z_i, z_{i+1} = c1 z_i + c2 D^{-1} r_{i+1}
    const T rho_new = T(1) / (T(2) * sigma - rho);
    apply_vec_epi<T, DIM, LV, L>(c, c.z(),
                                 EpiChebStep<T, PT, DT>{x, res, z, dinv, rho_new * rho, T(2) * rho_new / delta});
    rho = rho_new;
  }
#pragma unroll 1
  for (int i = tid; i < N; i += NT<T>) x[i] += z[i];
  __syncthreads();
}

// 1D contraction helpers for the Kronecker transfers.  P1: (mf x mc)
// row-major (fine rows, coarse columns).

// restriction: rc = (P1^T (x) ... (x) P1^T) rf
// STAGE: copy the fine vector into LDS first (it lives in global scratch);
// without, rf is an LDS vector and is read in place.
template <typename T, int DIM, int QF, int QC, bool STAGE = true>
__device__ __forceinline__ void restrict_vec(const T* __restrict__ rf, T* __restrict__ rc,
                                             const LDSP T* __restrict__ P1, LDSP T* __restrict__ ab) {
  constexpr int mf = 2 * QF - 1, mc = 2 * QC - 1;
  const int tid = threadIdx.x;
  if constexpr (DIM == 3) {
    LDSP T* t1 = ab;                  // [c][b][i]: mf*mf*mc
    LDSP T* t2 = t1 + mf * mf * mc;   // [c][j][i]: mf*mc*mc
    const LDSP T* sf = nullptr;
    if constexpr (!STAGE) sf = lds_cast(rf);
    if constexpr (STAGE) {
      LDSP T* st = t2 + mf * mc * mc;  // the fine vector, staged in LDS
#pragma unroll 1
      for (int idx = tid; idx < mf * mf * mf; idx += NT<T>) st[idx] = rf[idx];
      __syncthreads();
      sf = st;
    }
#pragma unroll 1
    for (int idx = tid; idx < mf * mf * mc; idx += NT<T>) {
      const int i = idx % mc, cb = idx / mc;
      T acc = 0;
#pragma unroll
      for (int a = 0; a < mf; ++a) acc += P1[a * mc + i] * sf[cb * mf + a];
      t1[idx] = acc;
    }
    __syncthreads();
#pragma unroll 1
    for (int idx = tid; idx < mf * mc * mc; idx += NT<T>) {
      const int i = idx % mc, t = idx / mc, j = t % mc, cc = t / mc;
      T acc = 0;
#pragma unroll
      for (int b = 0; b < mf; ++b) acc += P1[b * mc + j] * t1[(cc * mf + b) * mc + i];
      t2[idx] = acc;
    }
    __syncthreads();
#pragma unroll 1
    for (int idx = tid; idx < mc * mc * mc; idx += NT<T>) {
      const int ji = idx % (mc * mc), k = idx / (mc * mc);
      T acc = 0;
#pragma unroll
      for (int cc = 0; cc < mf; ++cc) acc += P1[cc * mc + k] * t2[cc * mc * mc + ji];
      rc[idx] = acc;
    }
  } else {
    LDSP T* t1 = ab;            // [b][i]: mf*mc
    const LDSP T* sf = nullptr;
    if constexpr (!STAGE) sf = lds_cast(rf);
    if constexpr (STAGE) {
      LDSP T* st = t1 + mf * mc;  // the fine vector, staged in LDS
#pragma unroll 1
      for (int idx = tid; idx < mf * mf; idx += NT<T>) st[idx] = rf[idx];
      __syncthreads();
      sf = st;
    }
#pragma unroll 1
    for (int idx = tid; idx < mf * mc; idx += NT<T>) {
      const int i = idx % mc, b = idx / mc;
      T acc = 0;
#pragma unroll
      for (int a = 0; a < mf; ++a) acc += P1[a * mc + i] * sf[b * mf + a];
      t1[idx] = acc;
    }
    __syncthreads();
#pragma unroll 1
    for (int idx = tid; idx < mc * mc; idx += NT<T>) {
      const int i = idx % mc, j = idx / mc;
      T acc = 0;
#pragma unroll
      for (int b = 0; b < mf; ++b) acc += P1[b * mc + j] * t1[b * mc + i];
      rc[idx] = acc;
    }
  }
  __syncthreads();
}

// prolongation and correction: df += (P1 (x) ... (x) P1) dc
template <typename T, int DIM, int QF, int QC, bool STAGE = true>
__device__ __forceinline__ void prolong_add(const T* __restrict__ dc, T* __restrict__ df,
                                            const LDSP T* __restrict__ P1, LDSP T* __restrict__ ab) {
  constexpr int mf = 2 * QF - 1, mc = 2 * QC - 1;
  const int tid = threadIdx.x;
  if constexpr (DIM == 3) {
    LDSP T* t1 = ab;                  // [k][j][a]: mc*mc*mf
    LDSP T* t2 = t1 + mc * mc * mf;   // [k][b][a]: mc*mf*mf
    const LDSP T* sc = nullptr;
    if constexpr (!STAGE) sc = lds_cast(dc);
    if constexpr (STAGE) {
      LDSP T* st = t2 + mc * mf * mf;  // the coarse vector, staged in LDS
#pragma unroll 1
      for (int idx = tid; idx < mc * mc * mc; idx += NT<T>) st[idx] = dc[idx];
      __syncthreads();
      sc = st;
    }
#pragma unroll 1
    for (int idx = tid; idx < mc * mc * mf; idx += NT<T>) {
      const int a = idx % mf, kj = idx / mf;
      T acc = 0;
#pragma unroll
      for (int i = 0; i < mc; ++i) acc += P1[a * mc + i] * sc[kj * mc + i];
      t1[idx] = acc;
    }
    __syncthreads();
#pragma unroll 1
    for (int idx = tid; idx < mc * mf * mf; idx += NT<T>) {
      const int a = idx % mf, t = idx / mf, b = t % mf, k = t / mf;
      T acc = 0;
#pragma unroll
      for (int j = 0; j < mc; ++j) acc += P1[b * mc + j] * t1[(k * mc + j) * mf + a];
      t2[idx] = acc;
    }
    __syncthreads();
#pragma unroll 1
    for (int idx = tid; idx < mf * mf * mf; idx += NT<T>) {
      const int ba = idx % (mf * mf), cc = idx / (mf * mf);
      T acc = 0;
#pragma unroll
      for (int k = 0; k < mc; ++k) acc += P1[cc * mc + k] * t2[k * mf * mf + ba];
      df[idx] += acc;
    }
  } else {
    LDSP T* t1 = ab;            // [j][a]: mc*mf
    const LDSP T* sc = nullptr;
    if constexpr (!STAGE) sc = lds_cast(dc);
    if constexpr (STAGE) {
      LDSP T* st = t1 + mc * mf;  // the coarse vector, staged in LDS
#pragma unroll 1
      for (int idx = tid; idx < mc * mc; idx += NT<T>) st[idx] = dc[idx];
      __syncthreads();
      sc = st;
    }
#pragma unroll 1
    for (int idx = tid; idx < mc * mf; idx += NT<T>) {
      const int a = idx % mf, j = idx / mf;
      T acc = 0;
#pragma unroll
      for (int i = 0; i < mc; ++i) acc += P1[a * mc + i] * sc[j * mc + i];
      t1[idx] = acc;
    }
    __syncthreads();
#pragma unroll 1
    for (int idx = tid; idx < mf * mf; idx += NT<T>) {
      const int a = idx % mf, b = idx / mf;
      T acc = 0;
#pragma unroll
      for (int j = 0; j < mc; ++j) acc += P1[b * mc + j] * t1[j * mf + a];
      df[idx] += acc;
    }
  }
  __syncthreads();
}

// LDS writes of this wavefront visible to all its lanes: the memory
// operations of one wavefront complete in order, so only the compiler must
// be kept from moving accesses across this point

// The V-cycle (Algorithm 2) from level L down, for levels of at most 64
// nodes stored as dense matrices: run by wavefront 0 alone, lane i owning
// row i, with the Chebyshev iterates in registers and wavefront-level syncs
// between the steps (a workgroup barrier per step would leave the other
// wavefronts idle at every one).  Same arithmetic, in the same order, as
// vcycle and chebyshev: the dense products sum over j ascending, the
// transfers contract x, then y, then z.  Leaves d_L in LDS.
template <typename T, int DIM, class LV, int L>
__device__ void vcycle_small(const Ctx<T, DIM, LV>& c, int k) {
  using Lay = Layout<T, DIM, LV>;
  constexpr int N = Lay::level_size(L);
  static_assert(N <= 64, "one row per lane");
  const int i = threadIdx.x;  // < 64
  LDSP T* d = lds_cast(c.d(L));
  const LDSP T* r = lds_cast(c.r(L));
  const LDSP T* dinv = lds_cast(c.dinv(L));
  if constexpr (L == LV::count - 1) {
    if (i == 0) d[0] = c.coarse_solve(r[0], dinv[0]);
    wave_sync();
    return;
  } else {
    if constexpr (L + 2 == LV::count) {
      if (c.trunc) {
        // exact solve of a boundary-vertex patch's lowest level (as in vcycle)
        constexpr int q = LV::q[L], mi = 2 * q - 1;
        int lo[3], nb[3];
        for (int a = 0; a < 3; ++a) {
          const int fl = a < DIM ? (c.pf >> (2 * a)) & 3 : 0;
          lo[a] = (fl & 1) ? q + 1 : 1;
          nb[a] = a < DIM ? (fl ? q - 1 : mi) : 1;
        }
        const int nu = nb[0] * nb[1] * nb[2];
        auto full = [&](int u) {
          const int ox = u % nb[0], oy = (u / nb[0]) % nb[1], oz = u / (nb[0] * nb[1]);
          return (lo[0] + ox - 1) + mi * ((lo[1] + oy - 1) + (DIM == 3 ? mi * (lo[2] + oz - 1) : 0));
        };
        if (i < N) d[i] = T(0);
        wave_sync();
        if (i < nu) {
          const double* row = c.trunc + (int64_t)i * nu;
          double acc = 0;
          for (int w = 0; w < nu; ++w) acc += row[w] * double(r[full(w)]);
          d[full(i)] = T(acc);
        }
        wave_sync();
        return;
      }
    }
    const bool own = i < N;
    LDSP T* rb = lds_cast(c.res());  // the residual, for the restriction
    const T f = own ? r[i] : T(0), di = own ? dinv[i] : T(0);
    const T theta = c.cheb()[2 * L], delta = c.cheb()[2 * L + 1];
    const T sigma = theta / delta;
    // row i of the stored level matrix, held in registers for the whole
    // visit; a product takes the vector's entries from their lanes
    // (readlane), so no LDS round trip or wavefront sync is needed
    T Mrow[N];
    {
      const LDSP T* M = lds_cast(c.dense(L));
#pragma unroll
      for (int j = 0; j < N; ++j) Mrow[j] = own ? M[i * N + j] : T(0);
    }
    auto Av = [&](T v) {  // row i times the vector whose entry j lane j holds
      T acc = 0;
#pragma unroll
      for (int j = 0; j < N; ++j) acc += Mrow[j] * lane_value(v, j);
      return own ? acc : T(0);
    };
    // Chebyshev-Jacobi with the iterates of row i in registers (as chebyshev)
    auto smooth = [&](T& x, bool x_zero) {
      T rho = T(1) / sigma, res, z;
      if (x_zero) {
        res = f;
        z = di * f / theta;
        x = 0;
      } else {
        res = f - Av(x);
        z = di * res * (T(1) / theta);
      }
      for (int it = 0; it + 1 < k; ++it) {
        const T rho_new = T(1) / (T(2) * sigma - rho);
        const T c1 = rho_new * rho, c2 = T(2) * rho_new / delta;
        const T az = Av(z);
        x = x + z;
        res = res - az;
        z = c1 * z + c2 * di * res;
        rho = rho_new;
      }
      x = x + z;
    };
    T x;
    smooth(x, true);
    // residual, restriction (x, then y, then z) to level L + 1
    const T res = f - Av(x);
    if (own) rb[i] = res;
    wave_sync();
    constexpr int QF = LV::q[L], QC = LV::q[L + 1];
    constexpr int mf = 2 * QF - 1, mc = 2 * QC - 1;
    constexpr int NC = Lay::level_size(L + 1);
    const LDSP T* P1 = lds_cast(c.tabP(L));
    if (i < NC) {
      const int ix = i % mc, iy = (i / mc) % mc, iz = DIM == 3 ? i / (mc * mc) : 0;
      T acc = 0;
      for (int cc = 0; cc < (DIM == 3 ? mf : 1); ++cc) {
        T ay = 0;
        for (int b = 0; b < mf; ++b) {
          T ax = 0;
          for (int a = 0; a < mf; ++a) ax += P1[a * mc + ix] * rb[(cc * mf + b) * mf + a];
          ay += P1[b * mc + iy] * ax;
        }
        if (DIM == 3)
          acc += P1[cc * mc + iz] * ay;
        else
          acc = ay;
      }
      lds_cast(c.r(L + 1))[i] = acc;
    }
    wave_sync();
    vcycle_small<T, DIM, LV, L + 1>(c, k);
    // prolongation and correction (x, then y, then z), post-smoothing
    const LDSP T* dc = lds_cast(c.d(L + 1));
    if (own) {
      const int ax_ = i % mf, by = (i / mf) % mf, cz = DIM == 3 ? i / (mf * mf) : 0;
      T acc = 0;
      for (int kk = 0; kk < (DIM == 3 ? mc : 1); ++kk) {
        T ay = 0;
        for (int j = 0; j < mc; ++j) {
          T ax = 0;
          for (int ii = 0; ii < mc; ++ii) ax += P1[ax_ * mc + ii] * dc[(kk * mc + j) * mc + ii];
          ay += P1[by * mc + j] * ax;
        }
        if (DIM == 3)
          acc += P1[cz * mc + kk] * ay;
        else
          acc = ay;
      }
      x = x + acc;
    }
    smooth(x, false);
    if (own) d[i] = x;
    wave_sync();
  }
}

// V-cycle at level L (Algorithm 2): pre-smooth, residual, restrict, recurse,
// prolongate and correct, post-smooth; the coarsest level is solved exactly.
// One pass of the fast diagonalisation along direction `dir` of an m^DIM
// vector (x fastest): out_k = sum_a S[a][k] in_a (FWD, S^T) or
// out_a = sum_k S[a][k] in_k (S).
// One pass of the fast diagonalisation along direction dir: out = S^T in
// (FWD) or S in along that direction, with the direction's own table (the
// type of the direction: two cells, or one cell at the low or high nodes).
template <typename T, int DIM, int m, bool FWD>
__device__ void fdm_pass(const T* in, T* out, const T* S, int dir) {
  constexpr int N = ipow(m, DIM);
  const int stride = dir == 0 ? 1 : (dir == 1 ? m : m * m);
  for (int idx = threadIdx.x; idx < N; idx += NT<T>) {
    const int i = (idx / stride) % m;
    const int base = idx - i * stride;
    T acc = 0;
    for (int a = 0; a < m; ++a) acc += (FWD ? S[a * m + i] : S[i * m + a]) * in[base + a * stride];
    out[idx] = acc;
  }
}

// One Richardson step of the Cartesian-reinforced smoother (Section 3.1) on
// level L: d += omega D diag(A_b) A_b^{-1} (r - A d), D the level's inverse
// diagonal and A_b the operator of the Cartesian reference patch with unit
// cells and coefficient 1 and the patch's own cell count per direction
// (one along a direction the boundary cuts), inverted by fast
// diagonalisation: A_b^{-1} = S^(x d) diag(1 / sum_i lam_{k_i}) (S^T)^(x d).
// A one-cell direction's tables are embedded in the two-cell numbering of
// the masked patch layout (identity and lam = 1 on the masked nodes, whose
// values stay zero).
template <typename T, int DIM, class LV, int L>
__device__ void cartesian_step(const Ctx<T, DIM, LV>& c, bool d_zero) {
  using PT = VecPtr<T, DIM, LV>;
  constexpr int N = Layout<T, DIM, LV>::level_size(L);
  constexpr int m = 2 * LV::q[L] - 1;
  // per direction: the table of its type (0: two cells; 1: one cell, low
  // nodes, the high side cut; 2: one cell, high nodes, the low side cut)
  const T* tab[3];
  for (int i = 0; i < 3; ++i) {
    const int fl = i < DIM ? (c.pf >> (2 * i)) & 3 : 0;
    const int type = (fl & 1) ? 2 : ((fl & 2) ? 1 : 0);
    tab[i] = c.fdm + L * kFdmStride + type * kFdmTypeStride;
  }
  T* d = c.d(L);
  const T* dinv = c.dinv(L);
  T* u = c.res();
  T* v = c.z();
  if (d_zero) {
    const T* r = c.r(L);
    for (int i = threadIdx.x; i < N; i += NT<T>) u[i] = r[i];
    __syncthreads();
  } else {
    apply_vec_epi<T, DIM, LV, L>(c, d, EpiResidual<T, PT>{vp<T, DIM, LV>(c.r(L)), vp<T, DIM, LV>(u)});
  }
  T* src = u;
  T* dst = v;
  for (int dir = 0; dir < DIM; ++dir) {
    fdm_pass<T, DIM, m, true>(src, dst, tab[dir], dir);
    __syncthreads();
    T* t = src; src = dst; dst = t;
  }
  for (int i = threadIdx.x; i < N; i += NT<T>) {
    const int k0 = i % m, k1 = (i / m) % m, k2 = DIM == 3 ? i / (m * m) : 0;
    src[i] /= tab[0][m * m + k0] + tab[1][m * m + k1] + (DIM == 3 ? tab[2][m * m + k2] : T(0));
  }
  __syncthreads();
  for (int dir = 0; dir < DIM; ++dir) {
    fdm_pass<T, DIM, m, false>(src, dst, tab[dir], dir);
    __syncthreads();
    T* t = src; src = dst; dst = t;
  }
  for (int i = threadIdx.x; i < N; i += NT<T>) {
    const int a0 = i % m, a1 = (i / m) % m, a2 = DIM == 3 ? i / (m * m) : 0;
    const T m0 = tab[0][m * m + m + a0], k0 = tab[0][m * m + 2 * m + a0];
    const T m1 = tab[1][m * m + m + a1], k1 = tab[1][m * m + 2 * m + a1];
    T diag;
    if constexpr (DIM == 3) {
      const T m2 = tab[2][m * m + m + a2], k2 = tab[2][m * m + 2 * m + a2];
      diag = k0 * m1 * m2 + m0 * k1 * m2 + m0 * m1 * k2;
    } else {
      diag = k0 * m1 + m0 * k1;
    }
    const T step = T(c.omega) * dinv[i] * diag * src[i];
    d[i] = d_zero ? step : d[i] + step;
  }
  __syncthreads();
}

template <typename T, int DIM, class LV, int L, bool CART = false>
__device__ void vcycle(const Ctx<T, DIM, LV>& c, int k, bool d_zero) {
  constexpr int N = Layout<T, DIM, LV>::level_size(L);
  const int tid = threadIdx.x;
  if constexpr (L == LV::count - 1) {
    // coarsest level of an interior patch: a 1x1 matrix, inverse = 1 / diagonal
    static_assert(N == 1, "coarsest interior level must have one node");
    T* d = c.d(L);
    const T* r = c.r(L);
    const T* dinv = c.dinv(L);
    if (tid == 0) d[0] = c.coarse_solve(r[0], dinv[0]);
    __syncthreads();
  } else {
    if constexpr (L + 2 == LV::count) {
      // a boundary-vertex patch has no node at degree 1: its lowest level
      // with nodes is solved exactly (FP64 Cholesky inverse from the setup)
      if (c.trunc) {
        // the inverse is stored over the unmasked nodes only, in the cut
        // patch's numbering (x fastest over the unmasked box)
        constexpr int q = LV::q[L], mi = 2 * q - 1;
        int lo[3], nb[3];
        for (int i = 0; i < 3; ++i) {
          const int fl = i < DIM ? (c.pf >> (2 * i)) & 3 : 0;
          lo[i] = (fl & 1) ? q + 1 : 1;
          nb[i] = i < DIM ? (fl ? q - 1 : mi) : 1;
        }
        const int nu = nb[0] * nb[1] * nb[2];
        auto full = [&](int u) {
          const int ox = u % nb[0], oy = (u / nb[0]) % nb[1], oz = u / (nb[0] * nb[1]);
          return (lo[0] + ox - 1) + mi * ((lo[1] + oy - 1) + (DIM == 3 ? mi * (lo[2] + oz - 1) : 0));
        };
        T* d = c.d(L);
        const T* r = c.r(L);
        for (int i = tid; i < N; i += NT<T>) d[i] = T(0);
        __syncthreads();
        for (int u = tid; u < nu; u += NT<T>) {
          const double* row = c.trunc + (int64_t)u * nu;
          double acc = 0;
          for (int w = 0; w < nu; ++w) acc += row[w] * double(r[full(w)]);
          d[full(u)] = T(acc);
        }
        __syncthreads();
        return;
      }
    }
    constexpr int QF = LV::q[L], QC = LV::q[L + 1];
    constexpr int mf = 2 * QF - 1, mc = 2 * QC - 1;
    static_assert((DIM == 3 ? mf * mf * mc + mf * mc * mc + mf * mf * mf
                            : mf * mc + mf * mf) <= Layout<T, DIM, LV>::abuf_elems,
                  "transfer temporaries exceed the work area");
    using PT = VecPtr<T, DIM, LV>;
    if constexpr (CART)                               // pre-smoothing
      cartesian_step<T, DIM, LV, L>(c, d_zero);
    else
      chebyshev<T, DIM, LV, L>(c, k, d_zero);
    T* res = c.res();
    apply_vec_epi<T, DIM, LV, L>(c, c.d(L),           // residual
                                 EpiResidual<T, PT>{vp<T, DIM, LV>(c.r(L)), vp<T, DIM, LV>(res)});
    constexpr bool STAGE = !Layout<T, DIM, LV>::vec_in_lds;
    restrict_vec<T, DIM, QF, QC, STAGE>(res, c.r(L + 1), lds_cast(c.tabP(L)), lds_cast(c.abuf()));  // restriction
    if constexpr (!CART && Layout<T, DIM, LV>::small_from(L + 1)) {     // recursion
      if (c.dense_ok) {
        if (tid < 64) vcycle_small<T, DIM, LV, L + 1>(c, k);
        __syncthreads();
      } else {
        vcycle<T, DIM, LV, L + 1>(c, k, true);
      }
    } else {
      vcycle<T, DIM, LV, L + 1, CART>(c, k, true);
    }
    prolong_add<T, DIM, QF, QC, STAGE>(c.d(L + 1), c.d(L), lds_cast(c.tabP(L)), lds_cast(c.abuf()));  // correction
    if constexpr (CART)                               // post-smoothing
      cartesian_step<T, DIM, LV, L>(c, false);
    else
      chebyshev<T, DIM, LV, L>(c, k, false);
  }
}

// ---------------------------------------------------------------------------
// the patch kernel
// ---------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ const T* tptr(const void* p) {
  return reinterpret_cast<const T*>(p);
}

// Global node of closure offset s of the patch at vertex v (top degree p).
template <int DIM>
__device__ __forceinline__ void patch_base(int vlin, int N, int p, int& base, int& M) {
  const int N1 = N + 1;
  M = N * p + 1;
  const int vx = vlin % N1, vy = (vlin / N1) % N1;
  base = (vx - 1) * p + (vy - 1) * p * M;
  if (DIM == 3) {
    const int vz = vlin / (N1 * N1);
    base += (vz - 1) * p * M * M;
  }
}

// Patches of boundary vertices keep the two-cell shape per direction: the
// cells outside the mesh are ghosts with coefficient zero, and the interior
// nodes on or beyond the boundary are masked (zero inverse diagonal, never
// gathered or scattered), so the unmasked rows and columns of every level
// operator are those of the cut patch.  Bit 2i of the flags: vertex on the
// low boundary of direction i (v_i = 0); bit 2i+1: on the high one (v_i = N).
template <int DIM>
__device__ __forceinline__ int patch_flags(const PatchArgs& a, int patch) {
  if (!a.with_boundary || a.patch_geo) return 0;
  const int N1 = a.N + 1, vlin = a.patch_vertex[patch];
  const int v[3] = {vlin % N1, (vlin / N1) % N1, DIM == 3 ? vlin / (N1 * N1) : 1};
  int f = 0;
  for (int i = 0; i < DIM; ++i) {
    if (v[i] == 0) f |= 1 << (2 * i);
    if (v[i] == a.N) f |= 2 << (2 * i);
  }
  return f;
}

// Interior node idx (x fastest over (2q-1)^DIM) at degree q lies inside the
// mesh; *ci gets its number among the unmasked nodes (x fastest), i.e. in
// the cut patch's own interior numbering.
template <int DIM>
__device__ __forceinline__ bool interior_node(int f, int q, int idx, int* ci) {
  const int mi = 2 * q - 1;
  const int s[3] = {idx % mi + 1, (idx / mi) % mi + 1, DIM == 3 ? idx / (mi * mi) + 1 : 1};
  int c = 0, stride = 1;
  for (int i = 0; i < DIM; ++i) {
    const int fl = (f >> (2 * i)) & 3;
    const int lo = (fl & 1) ? q + 1 : 1, n = fl ? q - 1 : 2 * q - 1;
    const int o = s[i] - lo;
    if (o < 0 || o >= n) return false;
    c += o * stride;
    stride *= n;
  }
  if (ci) *ci = c;
  return true;
}

// evaluate epilogue (equation main:4), fused into the segment operator's
// last phase: r = b - A u-bar on the unmasked rows, zero on the masked rows
// of a boundary-vertex patch
template <typename T, int DIM, class PT>
struct EpiEvaluate {
  PT r;
  int pf, p;
  __device__ __forceinline__ void operator()(int i, T v) const {
    r[i] = (pf == 0 || interior_node<DIM>(pf, p, i, nullptr)) ? r[i] - v : T(0);
  }
};

// Mesh vertex at indices ii (each in -1 .. N+1), continued linearly across
// the boundary for -1 and N+1 (ghost vertices: only a finite metric is
// needed there, the ghost coefficient is zero).
template <int DIM>
__device__ double mesh_vertex(const PatchArgs& a, const int* ii, int r) {
  const int N = a.N, N1 = N + 1;
  double acc = 0;
  for (int combo = 0; combo < (1 << DIM); ++combo) {
    double w = 1;
    int64_t g = 0, stride = 1;
    bool used = true;
    for (int d = 0; d < DIM; ++d) {
      const int v = ii[d], bit = (combo >> d) & 1;
      int idx;
      double cf;
      if (v < 0) {
        idx = bit ? 1 : 0;
        cf = bit ? -1.0 : 2.0;
      } else if (v > N) {
        idx = bit ? N - 1 : N;
        cf = bit ? -1.0 : 2.0;
      } else {
        if (bit) {
          used = false;
          break;
        }
        idx = v;
        cf = 1.0;
      }
      w *= cf;
      g += idx * stride;
      stride *= N1;
    }
    if (used) acc += w * a.verts[g * DIM + r];
  }
  return acc;
}

// Patch geometry: 3^d vertices relative to the patch centre and 2^d cell
// coefficients, from the mesh or from the arrays of independent patches.
// f(i) for the rows i = tid, tid + NTH, ... < n of this thread (n <= NMAX),
// unrolled over the compile-time bound
template <int NTH, int NMAX, class F>
__device__ __forceinline__ void rows(int n, F f) {
#pragma unroll
  for (int j = 0; j < (NMAX + NTH - 1) / NTH; ++j) {
    const int i = (int)threadIdx.x + j * NTH;
    if (i < n) f(i);
  }
}

// The same rows as st(i, ld(i)), with every load issued before any store.
// Nothing is guarded: a slot past the last row loads and stores row n - 1
// again (the value its owner stores too), so st must be a plain store of
// what ld returned.  Guarded, each load would be moved into its row's
// branch and wait for its data before the next one is issued; this way a
// thread pays one memory round trip, not one per row.  n >= 1.
template <int NTH, int NMAX, class LD, class ST>
__device__ __forceinline__ void rows_ld_st(int n, LD ld, ST st) {
  constexpr int IT = (NMAX + NTH - 1) / NTH;
  using V = decltype(ld(0));
  V v[IT];
#pragma unroll
  for (int j = 0; j < IT; ++j) {
    const int i = (int)threadIdx.x + j * NTH;
    v[j] = ld(i < n ? i : n - 1);
  }
#pragma unroll
  for (int j = 0; j < IT; ++j) {
    const int i = (int)threadIdx.x + j * NTH;
    st(i < n ? i : n - 1, v[j]);
  }
}

template <typename T, int DIM, int NTH = 0, class PG = T*>
__device__ void load_geometry(const PatchArgs& a, int patch, PG geo, PG mu) {
  constexpr int nvert = ipow(3, DIM), ncell = ipow(2, DIM);
  const int tid = threadIdx.x;
  // f(i) over the rows of this thread: with NTH > 0 (the block size, known
  // at compile time) unrolled, so the loads of all rows can issue together
  auto each = [&](auto nmax, int n, auto f) {
    if constexpr (NTH > 0) {
      rows<NTH, decltype(nmax)::value>(n, f);
    } else {
      for (int i = tid; i < n; i += blockDim.x) f(i);
    }
  };
  using NV = std::integral_constant<int, nvert * DIM>;
  using NC = std::integral_constant<int, ncell>;
  if (a.patch_geo) {
    const double* V = a.patch_geo + (int64_t)patch * nvert * DIM;
    constexpr int centre = (nvert - 1) / 2;
    each(NV{}, nvert * DIM, [&](int i) { geo[i] = T(V[i] - V[centre * DIM + i % DIM]); });
    each(NC{}, ncell, [&](int i) { mu[i] = T(a.patch_mu[(int64_t)patch * ncell + i]); });
    return;
  }
  const int vlin = a.patch_vertex[patch];
  const int N1 = a.N + 1;
  const int vx = vlin % N1, vy = (vlin / N1) % N1, vz = DIM == 3 ? vlin / (N1 * N1) : 0;
  each(NV{}, nvert * DIM, [&](int i) {
    const int r = i % DIM, t = i / DIM;
    const int ii[3] = {vx - 1 + t % 3, vy - 1 + (t / 3) % 3, DIM == 3 ? vz - 1 + t / 9 : 0};
    bool inside = true;
    for (int d = 0; d < DIM; ++d) inside = inside && ii[d] >= 0 && ii[d] <= a.N;
    int64_t g = ii[0] + (int64_t)ii[1] * N1;
    if (DIM == 3) g += (int64_t)ii[2] * N1 * N1;
    const double x = inside ? a.verts[g * DIM + r] : mesh_vertex<DIM>(a, ii, r);
    geo[i] = T(x - a.verts[(int64_t)vlin * DIM + r]);
  });
  each(NC{}, ncell, [&](int i) {
    const int ci[3] = {vx - 1 + (i & 1), vy - 1 + ((i >> 1) & 1), DIM == 3 ? vz - 1 + ((i >> 2) & 1) : 0};
    bool inside = true;
    for (int d = 0; d < DIM; ++d) inside = inside && ci[d] >= 0 && ci[d] < a.N;
    int64_t g = ci[0] + (int64_t)ci[1] * a.N;
    if (DIM == 3) g += (int64_t)ci[2] * a.N * a.N;
    mu[i] = inside ? T(a.mu[g]) : T(0);   // ghost cells of a boundary-vertex patch
  });
}

__device__ __forceinline__ int patch_of_block(const PatchArgs& a) {
  return a.patch_list ? a.patch_list[a.patch_begin + blockIdx.x] : a.patch_begin + blockIdx.x;
}

template <typename T, int DIM, class LV>
__device__ void load_patch(const Ctx<T, DIM, LV>& c, const PatchArgs& a, int patch) {
  using Lay = Layout<T, DIM, LV>;
  constexpr int L = LV::count;
  constexpr int NTH = NT<T>;
  LDSP T* lds = lds_cast(c.lds);
  // tables
  const T* tab = tptr<T>(a.tab);
#pragma unroll
  for (int l = 0; l < L; ++l) {
    const T* src = tab + l * kTabLevelStride;
    LDSP T* dst = lds + Lay::tab_level_off(l);
    rows_ld_st<NTH, tab_size(LV::q[0])>(
        tab_size(LV::q[l]), [&](int i) { return src[i]; }, [&](int i, T v) { dst[i] = v; });
  }
#pragma unroll
  for (int t = 0; t + 1 < L; ++t) {
    const T* src = tab + kMaxLevels * kTabLevelStride + t * kTabTransferStride;
    LDSP T* dst = lds + Lay::tab_transfer_off(t);
    rows_ld_st<NTH, (2 * LV::q[0] - 1) * (2 * LV::q[1] - 1)>(
        (2 * LV::q[t] - 1) * (2 * LV::q[t + 1] - 1), [&](int i) { return src[i]; },
        [&](int i, T v) { dst[i] = v; });
  }
  if (c.geo_needed) load_geometry<T, DIM, NTH>(a, patch, lds_cast(c.geo()), lds_cast(c.mu()));
  {
    const T* src = tptr<T>(a.cheb) + (int64_t)patch * 2 * (L - 1);
    LDSP T* dst = lds_cast(c.cheb());
    rows_ld_st<NTH, 2 * kMaxLevels>(2 * (L - 1), [&](int i) { return src[i]; },
                                    [&](int i, T v) { dst[i] = v; });
  }
#pragma unroll
  for (int l = 0; l < L; ++l) {
    if (Lay::dinv0_global && l == 0) continue;  // read in place (Ctx::dinv0)
    const int sz = Lay::level_size(l);
    const T* src = tptr<T>(a.invdiag[l]) + (int64_t)patch * sz;
    VecPtr<T, DIM, LV> dst = vp<T, DIM, LV>(c.dinv(l));
    rows_ld_st<NTH, Lay::level_size(0)>(sz, [&](int i) { return src[i]; }, [&](int i, T v) { dst[i] = v; });
  }
#pragma unroll
  for (int l = 0; l < L; ++l) {
    if (!Lay::dense_level(l)) continue;
    const int sz = Lay::level_size(l) * Lay::level_size(l);
    const T* src = tptr<T>(a.dense[l]) + (int64_t)patch * sz;
    LDSP T* dst = lds_cast(c.dense(l));
    rows_ld_st<NTH, 32 * 32>(sz, [&](int i) { return src[i]; }, [&](int i, T v) { dst[i] = v; });
  }
  if constexpr (Lay::cache_G) {
    if (c.metric_loaded) {
      const T* src = tptr<T>(a.metric) + (int64_t)patch * Lay::G_total;
      LDSP T* dst = lds_cast(c.lds) + Lay::G_off;
      rows_ld_st<NTH, Lay::G_total>(Lay::G_total, [&](int i) { return src[i]; },
                                    [&](int i, T v) { dst[i] = v; });
    }
  }
  __syncthreads();
}

// Sum of v over the FP64 workgroup; every thread gets the same value (the
// per-wave partials are added in one order).  red: NT<double> / 64 doubles.
__device__ double block_sum(double v, double* red) {
  using T = double;
  // wavefront shuffle reduction, then across the waves of the block
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0;
  for (int w = 0; w < NT<T> / 64; ++w) s += red[w];
  __syncthreads();
  return s;
}

// Conjugate gradients preconditioned by N_MG V-cycles from zero (Algorithm 2)
// on one patch problem A_{j,p} x = b_j, from x = 0 (Hestenes and Stiefel; Saad,
// Iterative Methods for Sparse Linear Systems, Algorithm 9.1).  Section 3.2
// judges the local solver by the iterations of this method.  Stops after the
// first iteration with ||r_k|| <= rtol ||b|| or after maxit iterations.
// FP64: x, the residual and the search direction live in global memory (this
// patch's rows; a row is touched by one thread only, so they need no
// barrier), the operator input and the V-cycle vectors in the patch context.
// Each exit test uses a workgroup sum that every thread holds, so all
// threads leave the loop together.
template <int DIM, class LV, bool CART>
__device__ void patch_pcg(const Ctx<double, DIM, LV>& c, const PatchArgs& a, int patch) {
  using T = double;
  constexpr int N = Layout<T, DIM, LV>::level_size(0);
  const int tid = threadIdx.x;
  double* red = c.abuf();  // unused between operator applications and V-cycles
  const double* b = a.in + (int64_t)patch * N;
  double* x = a.out + (int64_t)patch * N;
  double* r = a.pcg_work + (int64_t)patch * 2 * N;
  double* p = r + N;
  T* r0 = c.r(0);         // V-cycle right-hand side
  const T* d0 = c.d(0);   // V-cycle result
  T* v = c.z();           // operator input
  auto precondition = [&]() {
    for (int it = 0; it < a.n_vcycles; ++it) vcycle<T, DIM, LV, 0, CART>(c, a.cheb_degree, it == 0);
    __syncthreads();
  };
  double bb = 0;
  for (int i = tid; i < N; i += NT<T>) {
    const double bi = b[i];
    x[i] = 0.0;
    r[i] = bi;
    r0[i] = bi;
    bb += bi * bi;
  }
  bb = block_sum(bb, red);
  const double stop = a.pcg_rtol * a.pcg_rtol * bb;
  double rr = bb;
  int k = 0;
  if (bb > 0.0 && a.pcg_maxit > 0) {
    precondition();
    double rz = 0;
    for (int i = tid; i < N; i += NT<T>) {
      const double zi = d0[i];
      p[i] = zi;
      rz += r[i] * zi;
    }
    rz = block_sum(rz, red);
#pragma unroll 1
    for (;;) {
      for (int i = tid; i < N; i += NT<T>) v[i] = p[i];
      __syncthreads();
      apply_vec<T, DIM, LV, 0>(c, v);
      const T* Ap = c.Out();
      double pap = 0;
      for (int i = tid; i < N; i += NT<T>) pap += p[i] * Ap[i];
      pap = block_sum(pap, red);
      const double alpha = rz / pap;
      double rn = 0;
      for (int i = tid; i < N; i += NT<T>) {
        x[i] += alpha * p[i];
        const double ri = r[i] - alpha * Ap[i];
        r[i] = ri;
        r0[i] = ri;
        rn += ri * ri;
      }
      rr = block_sum(rn, red);
      ++k;
      if (rr <= stop || k >= a.pcg_maxit) break;
      precondition();
      double rzn = 0;
      for (int i = tid; i < N; i += NT<T>) rzn += r[i] * d0[i];
      rzn = block_sum(rzn, red);
      const double beta = rzn / rz;
      rz = rzn;
      for (int i = tid; i < N; i += NT<T>) p[i] = d0[i] + beta * p[i];
    }
  }
  if (tid == 0) {
    a.pcg_iters[patch] = k;
    a.pcg_relres[patch] = bb > 0.0 ? sqrt(rr / bb) : 0.0;
  }
}

// One patch update (mode: smooth, residual, local solve or level apply).
template <typename T, int DIM, class LV, int MODE>
__device__ __forceinline__ void patch_update(const PatchArgs& a, Ctx<T, DIM, LV>& c, int patch) {
  using Lay = Layout<T, DIM, LV>;
  using S0 = Sh<DIM, LV::q[0]>;
  const int tid = threadIdx.x;
  // the smoothing modes: local solves with Chebyshev or Cartesian-reinforced smoothing
  constexpr bool SMOOTH = MODE == kModeSmooth || MODE == kModeSmoothCart;
  constexpr bool CART = MODE == kModeSmoothCart;
  const int pf = patch_flags<DIM>(a, patch);
  c.pf = pf;
  c.trunc = nullptr;
  if constexpr (sizeof(T) == 4) c.coarse_inv = a.invdiag64[LV::count - 1][patch];
  if constexpr (Lay::dinv0_global)
    c.dinv0 = const_cast<T*>(tptr<T>(a.invdiag[0])) + (int64_t)patch * Lay::level_size(0);
  if (pf && a.trunc_index) {
    const int k = a.trunc_index[patch];
    // one slot holds the largest unmasked box, a face patch's
    constexpr int qc = LV::q[LV::count - 2];
    constexpr int nbox = ipow(2 * qc - 1, DIM - 1) * (qc - 1);
    if (k >= 0) c.trunc = a.trunc_inv + (int64_t)k * nbox * nbox;
  }
  constexpr int N0 = S0::interior;
  constexpr int m = S0::m, mi = S0::mi;
  T* r0 = c.r(0);
  int base = 0, M = 0;
  if constexpr (SMOOTH || MODE == kModeResidual) {
    // gather u-bar_j (closure) and b_j (interior), equation gather; issued
    // first so that its global loads overlap those of the patch data
    patch_base<DIM>(a.patch_vertex[patch], a.N, a.p, base, M);
    LDSP T* X = lds_cast(c.X());
    VecPtr<T, DIM, LV> rv = vp<T, DIM, LV>(r0);
    auto st_x = [&](int idx, double v) { X[idx] = T(v); };
    auto st_r = [&](int idx, double v) { rv[idx] = T(v); };
    if (pf == 0) {
      rows_ld_st<NT<T>, S0::closure>(
          S0::closure,
          [&](int idx) {
            const int x = idx % m, t = idx / m, y = t % m, z = DIM == 3 ? t / m : 0;
            return a.u[base + x + y * M + (int64_t)z * M * M];
          },
          st_x);
      rows_ld_st<NT<T>, N0>(
          N0,
          [&](int idx) {
            const int x = idx % mi + 1, t = idx / mi, y = t % mi + 1, z = DIM == 3 ? t / mi + 1 : 0;
            return a.b[base + x + y * M + (int64_t)z * M * M];
          },
          st_r);
    } else {
      // boundary-vertex patch: closure nodes outside the mesh read as zero
      // (their loads go to node 0, a valid address, and are discarded)
      const int N1 = a.N + 1, vlin = a.patch_vertex[patch];
      const int g0[3] = {(vlin % N1 - 1) * a.p, ((vlin / N1) % N1 - 1) * a.p,
                         DIM == 3 ? (vlin / (N1 * N1) - 1) * a.p : 0};
      rows_ld_st<NT<T>, S0::closure>(
          S0::closure,
          [&](int idx) {
            const int x = idx % m, t = idx / m, y = t % m, z = DIM == 3 ? t / m : 0;
            const bool in = g0[0] + x >= 0 && g0[0] + x < M && g0[1] + y >= 0 && g0[1] + y < M &&
                            (DIM == 2 || (g0[2] + z >= 0 && g0[2] + z < M));
            const double v = a.u[in ? base + x + y * M + (int64_t)z * M * M : 0];
            return in ? v : 0.0;
          },
          st_x);
      rows_ld_st<NT<T>, N0>(
          N0,
          [&](int idx) {
            const int x = idx % mi + 1, t = idx / mi, y = t % mi + 1, z = DIM == 3 ? t / mi + 1 : 0;
            const bool in = interior_node<DIM>(pf, a.p, idx, nullptr);
            const double v = a.b[in ? base + x + y * M + (int64_t)z * M * M : 0];
            return in ? v : 0.0;
          },
          st_r);
    }
  }
  c.metric_loaded = Lay::cache_G && MODE != kModeMetric && a.metric != nullptr;
  c.Gg = (Lay::G_global && MODE != kModeMetric && a.metric)
             ? tptr<T>(a.metric) + (int64_t)patch * Lay::G_glob_elems
             : nullptr;
  // with the metric loaded, the geometry only serves levels that recompute
  // theirs (prepare_geometry computes the Jacobian coefficients for those)
  c.geo_needed = !c.metric_loaded || Lay::needs_jc || MODE == kModeApply;
  load_patch<T, DIM, LV>(c, a, patch);  // ends with a barrier: the gather is in place too
  c.dense_ok = true;
#pragma unroll
  for (int l = 0; l < kMaxLevels; ++l)
    if (l < LV::count && Lay::dense_global(l))
      c.dglob[l] = tptr<T>(a.dense[l]) + (int64_t)patch * Lay::level_size(l) * Lay::level_size(l);
  prepare_geometry<T, DIM, LV>(c, MODE == kModeApply);

  if constexpr (MODE == kModeMetric) {
    // setup: keep this patch's metric for the patch updates
    if constexpr (Lay::cache_G) {
      T* dst = reinterpret_cast<T*>(a.metric_out) + (int64_t)patch * Lay::G_total;
      const T* src = c.lds + Lay::G_off;
      for (int i = tid; i < Lay::G_total; i += NT<T>) dst[i] = src[i];
    } else if constexpr (Lay::G_global && DIM == 3) {
      // the top level's metric at every Gauss point, in the LDS-cache layout
      constexpr int n = LV::q[0] + 1, NQ = 2 * n, NP = Lay::npts(0);
      T* dst = reinterpret_cast<T*>(a.metric_out) + (int64_t)patch * Lay::G_glob_elems;
      const T* xg = c.tabXg(0);
      const T* wg = c.tabWg(0);
      for (int pt = tid; pt < NP; pt += NT<T>) {
        const int QX = pt % NQ, QY = (pt / NQ) % NQ, QZ = pt / (NQ * NQ);
        const int cx = QX >= n, cy = QY >= n, cz = QZ >= n;
        const int kx = QX - cx * n, ky = QY - cy * n, kz = QZ - cz * n;
        const int cell = cz * 4 + cy * 2 + cx;
        T G[6];
        metric3c<T>(c.jc() + cell * 36, xg[kx], xg[ky], xg[kz], c.mu()[cell] * wg[kx] * wg[ky] * wg[kz], G);
        for (int g = 0; g < 6; ++g) dst[g * NP + pt] = G[g];
      }
    }
    return;
  } else if constexpr (MODE == kModePcg || MODE == kModePcgCart) {
    if constexpr (std::is_same<T, double>::value) {
      c.fdm = tptr<T>(a.fdm_tab);
      c.omega = a.fdm_omega;
      patch_pcg<DIM, LV, MODE == kModePcgCart>(c, a, patch);
    }
    return;
  } else if constexpr (MODE == kModeApply) {
    // y = A_{j,q} x for the requested level
    auto run = [&](auto Lc) {
      constexpr int L = decltype(Lc)::value;
      constexpr int NL = Lay::level_size(L);
      T* v = c.z();
      const double* in = a.in + (int64_t)patch * NL;
      for (int i = tid; i < NL; i += NT<T>) v[i] = T(in[i]);
      __syncthreads();
      apply_vec<T, DIM, LV, L>(c, v);
      double* out = a.out + (int64_t)patch * NL;
      for (int i = tid; i < NL; i += NT<T>) out[i] = double(c.Out()[i]);
    };
    if (a.level == 0) run(std::integral_constant<int, 0>{});
    if constexpr (LV::count > 1)
      if (a.level == 1) run(std::integral_constant<int, 1>{});
    if constexpr (LV::count > 2)
      if (a.level == 2) run(std::integral_constant<int, 2>{});
    if constexpr (LV::count > 3)
      if (a.level == 3) run(std::integral_constant<int, 3>{});
    return;
  } else {
    if constexpr (SMOOTH || MODE == kModeResidual) {
      // evaluate: r_j = b_j - Pi_j A-bar_j u-bar_j (equation main:4); masked
      // rows (boundary-vertex patches) are set to zero
      if constexpr (Lay::use_seg(0)) {
        using PT = VecPtr<T, DIM, LV>;
        apply3seg<T, LV::q[0], true, Lay::cache_level(0)>(
            lds_cast(c.X()), EpiEvaluate<T, DIM, PT>{vp<T, DIM, LV>(r0), pf, a.p}, lds_cast(c.abuf()),
            lds_cast(c.tabB(0)), lds_cast(c.tabDc(0)), lds_cast(c.jc()), lds_cast(c.mu()),
            lds_cast(c.Gc(0)));
      } else {
        apply_level<T, DIM, LV, 0>(c);
        for (int i = tid; i < N0; i += NT<T>)
          r0[i] = (pf == 0 || interior_node<DIM>(pf, a.p, i, nullptr)) ? r0[i] - c.Out()[i] : T(0);
        __syncthreads();
      }
      if constexpr (MODE == kModeResidual) {
        double* out = a.out + (int64_t)patch * N0;
        for (int i = tid; i < N0; i += NT<T>) out[i] = double(r0[i]);
        return;
      }
    } else {
      const double* in = a.in + (int64_t)patch * N0;
      for (int i = tid; i < N0; i += NT<T>) r0[i] = T(in[i]);
      __syncthreads();
    }
    // local solve: N_MG V-cycles from zero (equation main:5)
    if constexpr (CART) {
      c.fdm = tptr<T>(a.fdm_tab);
      c.omega = a.fdm_omega;
    }
    for (int it = 0; it < a.n_vcycles; ++it) vcycle<T, DIM, LV, 0, CART>(c, a.cheb_degree, it == 0);
    const T* d0 = c.d(0);
    if constexpr (SMOOTH) {
      // scatter-add in FP64 (equation scatter); interiors of one colour are disjoint
  #pragma unroll 1
    for (int idx = tid; idx < N0; idx += NT<T>) {
        const int x = idx % mi + 1, t = idx / mi, y = t % mi + 1, z = DIM == 3 ? t / mi + 1 : 0;
        if (pf == 0 || interior_node<DIM>(pf, a.p, idx, nullptr))
          a.u[base + x + y * M + (int64_t)z * M * M] += double(d0[idx]);
      }
    } else {
      double* out = a.out + (int64_t)patch * N0;
      for (int i = tid; i < N0; i += NT<T>) out[i] = double(d0[i]);
    }
  }
}

// Work item k of workgroup b in a grid of G workgroups over n patches, or -1
// when the workgroup is done.  map_mode 0: item b + k G.  map_mode 1
// (XCD-aware; workgroups are dealt to the 8 XCDs round-robin): the patches
// are split into 8 contiguous ranges, workgroup b works in range b mod 8, so
// neighbouring patches, which share closure nodes, meet in one L2.
__device__ __forceinline__ int work_item(const PatchArgs& a, int b, int k, int G) {
  const int n = a.n_patch;
  if (a.map_mode == 1 && (G & 7) == 0) {
    const int per = G >> 3, chunk = (n + 7) >> 3;
    const int o = (b >> 3) + k * per;
    const int i = (b & 7) * chunk + o;
    return (o < chunk && i < n) ? i : -1;
  }
  const int i = b + k * G;
  return i < n ? i : -1;
}

// Patch kernel: one workgroup per patch (PERSIST false), or fewer workgroups
// that each take several patches in turn (PERSIST true: a separate
// instantiation, since the loop raises register use); the mapping is a
// launch parameter.
// FP32 segment-form patches, one workgroup per patch: at least four waves
// per SIMD (128 registers), so that two patches share a CU as their LDS
// allows (the persistent form's loop would spill at that limit)
template <typename T, int DIM, class LV, bool PERSIST>
constexpr int seg_min_waves() {
  return DIM == 3 && sizeof(T) == 4 && !PERSIST && Layout<T, DIM, LV>::seg_top ? 4 : 1;
}
template <typename T, int DIM, class LV, int MODE, bool PERSIST>
__global__ __launch_bounds__(NT<T>, (seg_min_waves<T, DIM, LV, PERSIST>())) void patch_kernel(PatchArgs a) {
  using Lay = Layout<T, DIM, LV>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  Ctx<T, DIM, LV> c;
  c.lds = reinterpret_cast<T*>(smem_raw);
  c.vec = Lay::vec_in_lds ? c.lds + Lay::vec_off
                          : reinterpret_cast<T*>(a.vec_scratch) + (int64_t)blockIdx.x * a.vec_stride;
  c.gtab = tptr<T>(a.tab);
  if constexpr (!PERSIST) {
    const int i = work_item(a, blockIdx.x, 0, gridDim.x);
    if (i < 0) return;
    patch_update<T, DIM, LV, MODE>(a, c, a.patch_list ? a.patch_list[a.patch_begin + i] : a.patch_begin + i);
  } else {
#pragma unroll 1
    for (int k = 0;; ++k) {
      const int i = work_item(a, blockIdx.x, k, gridDim.x);
      if (i < 0) break;
      if (k > 0) __syncthreads();  // the previous patch is done with the LDS
      const int patch = a.patch_list ? a.patch_list[a.patch_begin + i] : a.patch_begin + i;
      patch_update<T, DIM, LV, MODE>(a, c, patch);
    }
  }
}

// ---------------------------------------------------------------------------
// setup: inverse diagonals of every level operator (FP64)
//   diag_a = sum over cells and Gauss points of grad phi_a^T G grad phi_a
// ---------------------------------------------------------------------------

template <int DIM, class LV>
__global__ __launch_bounds__(NT<double>) void diag_kernel(PatchArgs a) {
  using T = double;
  using Lay = Layout<T, DIM, LV>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  Ctx<T, DIM, LV> c;
  c.lds = reinterpret_cast<T*>(smem_raw);
  c.vec = Lay::vec_in_lds ? c.lds + Lay::vec_off
                          : reinterpret_cast<T*>(a.vec_scratch) + (int64_t)blockIdx.x * a.vec_stride;
  c.gtab = a.tab64;
  const int patch = patch_of_block(a);
  const int tid = threadIdx.x;
  // load tables and geometry only (the inverse diagonals are the output)
  {
    const T* tab = a.tab64;
    for (int l = 0; l < LV::count; ++l) {
      const int sz = tab_size(LV::q[l]);
      for (int i = tid; i < sz; i += NT<T>) c.lds[Lay::tab_level_off(l) + i] = tab[l * kTabLevelStride + i];
    }
    load_geometry<T, DIM>(a, patch, c.geo(), c.mu());
    __syncthreads();
  }
  auto run = [&](auto Lc) {
    constexpr int L = decltype(Lc)::value;
    constexpr int Q = LV::q[L];
    constexpr int n = Q + 1, m = 2 * Q + 1, mi = 2 * Q - 1;
    constexpr int ncell = ipow(2, DIM), npt = ipow(n, DIM);
    T* dg = c.X();      // closure diagonal
    T* G = c.abuf();    // metric at the Gauss points of one cell
    constexpr int NG = DIM == 3 ? 6 : 3;
    static_assert(NG * npt <= Lay::abuf_elems, "one cell's metric exceeds the work area");
    const T* B = c.tabB(L);
    const T* D = c.tabD(L);
    const T* xg = c.tabXg(L);
    const T* wg = c.tabWg(L);
    for (int i = tid; i < ipow(m, DIM); i += NT<T>) dg[i] = 0;
    __syncthreads();
    for (int cell = 0; cell < ncell; ++cell) {
      const int cx = cell & 1, cy = (cell >> 1) & 1, cz = (cell >> 2) & 1;
      for (int k = tid; k < npt; k += NT<T>) {
        const int kx = k % n, ky = (k / n) % n, kz = DIM == 3 ? k / (n * n) : 0;
        if constexpr (DIM == 3)
          metric3<T>(c.geo(), cx, cy, cz, xg[kx], xg[ky], xg[kz],
                     c.mu()[cell] * wg[kx] * wg[ky] * wg[kz], G + NG * k);
        else
          metric2<T>(c.geo(), cx, cy, xg[kx], xg[ky], c.mu()[cell] * wg[kx] * wg[ky], G + NG * k);
      }
      __syncthreads();
      for (int aidx = tid; aidx < npt; aidx += NT<T>) {
        const int ax = aidx % n, ay = (aidx / n) % n, az = DIM == 3 ? aidx / (n * n) : 0;
        T acc = 0;
        for (int k = 0; k < npt; ++k) {
          const int kx = k % n, ky = (k / n) % n, kz = DIM == 3 ? k / (n * n) : 0;
          const T* g = G + NG * k;
          if constexpr (DIM == 3) {
            const T bx = B[kx * n + ax], by = B[ky * n + ay], bz = B[kz * n + az];
            const T g0 = D[kx * n + ax] * by * bz, g1 = bx * D[ky * n + ay] * bz,
                    g2 = bx * by * D[kz * n + az];
            acc += g[0] * g0 * g0 + g[3] * g1 * g1 + g[5] * g2 * g2 +
                   T(2) * (g[1] * g0 * g1 + g[2] * g0 * g2 + g[4] * g1 * g2);
          } else {
            const T bx = B[kx * n + ax], by = B[ky * n + ay];
            const T g0 = D[kx * n + ax] * by, g1 = bx * D[ky * n + ay];
            acc += g[0] * g0 * g0 + g[2] * g1 * g1 + T(2) * g[1] * g0 * g1;
          }
        }
        int s = (cx * Q + ax) + (cy * Q + ay) * m;
        if (DIM == 3) s += (cz * Q + az) * m * m;
        dg[s] += acc;
      }
      __syncthreads();
    }
    constexpr int NL = Lay::level_size(L);
    double* out = const_cast<double*>(a.invdiag64[L]) + (int64_t)patch * NL;
    const int pf = patch_flags<DIM>(a, patch);
    for (int i = tid; i < NL; i += NT<T>) {
      const int x = i % mi + 1, t = i / mi, y = t % mi + 1, z = DIM == 3 ? t / mi + 1 : 0;
      // masked nodes of a boundary-vertex patch: zero, so no update reaches them
      out[i] = (pf && !interior_node<DIM>(pf, Q, i, nullptr)) ? 0.0 : 1.0 / dg[x + y * m + z * m * m];
    }
    __syncthreads();
  };
  run(std::integral_constant<int, 0>{});
  if constexpr (LV::count > 1) run(std::integral_constant<int, 1>{});
  if constexpr (LV::count > 2) run(std::integral_constant<int, 2>{});
  if constexpr (LV::count > 3) run(std::integral_constant<int, 3>{});
}

// ---------------------------------------------------------------------------
// setup: Lanczos on D^{-1/2} A_{j,q} D^{-1/2} (FP64), extreme Ritz values
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t n) {
  // n-th output of the SplitMix64 stream seeded with `seed` (Steele, Lea and
  // Flood, OOPSLA 2014): mix(seed + (n+1) * golden gamma)
  uint64_t z = seed + (n + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// number of eigenvalues of the symmetric tridiagonal (al, be) below x
__device__ int sturm_count(const double* al, const double* be, int n, double x) {
  int cnt = 0;
  double q = al[0] - x;
  if (q < 0) ++cnt;
  for (int i = 1; i < n; ++i) {
    if (q == 0) q = 1e-300;
    q = al[i] - x - be[i - 1] * be[i - 1] / q;
    if (q < 0) ++cnt;
  }
  return cnt;
}

__device__ double tridiag_eig(const double* al, const double* be, int n, int k) {
  // k-th smallest eigenvalue by bisection inside the Gershgorin interval
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < n; ++i) {
    double r = (i > 0 ? fabs(be[i - 1]) : 0.0) + (i < n - 1 ? fabs(be[i]) : 0.0);
    lo = fmin(lo, al[i] - r);
    hi = fmax(hi, al[i] + r);
  }
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (sturm_count(al, be, n, mid) > k)
      hi = mid;
    else
      lo = mid;
  }
  return 0.5 * (lo + hi);
}

template <int DIM, class LV, int L>
__device__ void lanczos_level(Ctx<double, DIM, LV>& c, const PatchArgs& a, int patch) {
  using T = double;
  using Lay = Layout<T, DIM, LV>;
  constexpr int NL = Lay::level_size(L);
  const int tid = threadIdx.x;
  const int m = min(a.lanczos_steps, NL);
  double* Vb = a.lanczos_basis + (int64_t)blockIdx.x * (int64_t)a.lanczos_steps * NL;
  T* w = c.res();
  T* s = c.z();   // s = sqrt(dinv) * v, the operator input
  __shared__ double red[NT<double> / 64];
  __shared__ double al[64], be[64], coef[64];
  const T* dinv = c.dinv(L);
  // start vector: entry i of patch vertex v at smoothed level L
  // independent patches are numbered by their position in the batch
  const uint64_t vlin = a.patch_geo ? (uint64_t)patch : (uint64_t)a.patch_vertex[patch];
  const uint64_t base = ((vlin * 16u + (uint64_t)L) << 24);
  // a boundary-vertex patch numbers its unmasked nodes as the cut patch does
  const int pf = patch_flags<DIM>(a, patch);
  double nrm = 0;
  for (int i = tid; i < NL; i += NT<T>) {
    int ci = i;
    const bool live = pf == 0 || interior_node<DIM>(pf, LV::q[L], i, &ci);
    const double x =
        live ? (double)(splitmix64(a.seed, base + (uint64_t)ci) >> 11) * 0x1.0p-52 - 1.0 : 0.0;
    Vb[i] = x;
    nrm += x * x;
  }
  nrm = sqrt(block_sum(nrm, red));
  for (int i = tid; i < NL; i += NT<T>) Vb[i] /= nrm;
  __syncthreads();
  double b_prev = 0;
  int steps = 0;
  for (int j = 0; j < m; ++j) {
    const double* v = Vb + (int64_t)j * NL;
    for (int i = tid; i < NL; i += NT<T>) s[i] = sqrt(dinv[i]) * v[i];
    __syncthreads();
    apply_vec<T, DIM, LV, L>(c, s);
    double dot = 0;
    for (int i = tid; i < NL; i += NT<T>) {
      double wi = sqrt(dinv[i]) * c.Out()[i];
      if (j > 0) wi -= b_prev * Vb[(int64_t)(j - 1) * NL + i];
      w[i] = wi;
      dot += wi * v[i];
    }
    const double alpha = block_sum(dot, red);
    for (int i = tid; i < NL; i += NT<T>) w[i] -= alpha * v[i];
    __syncthreads();
    // full reorthogonalisation (classical Gram-Schmidt, twice)
    for (int pass = 0; pass < 2; ++pass) {
      for (int q = 0; q <= j; ++q) {
        const double* vq = Vb + (int64_t)q * NL;
        double cq = 0;
        for (int i = tid; i < NL; i += NT<T>) cq += vq[i] * w[i];
        cq = block_sum(cq, red);
        if (tid == 0) coef[q] = cq;
      }
      __syncthreads();
      for (int i = tid; i < NL; i += NT<T>) {
        double wi = w[i];
        for (int q = 0; q <= j; ++q) wi -= coef[q] * Vb[(int64_t)q * NL + i];
        w[i] = wi;
      }
      __syncthreads();
    }
    if (tid == 0) al[j] = alpha;
    double bn = 0;
    for (int i = tid; i < NL; i += NT<T>) bn += w[i] * w[i];
    bn = sqrt(block_sum(bn, red));
    steps = j + 1;
    if (j == m - 1 || bn < 1e-12 * fabs(alpha)) break;
    if (tid == 0) be[j] = bn;
    double* vn = Vb + (int64_t)(j + 1) * NL;
    for (int i = tid; i < NL; i += NT<T>) vn[i] = w[i] / bn;
    b_prev = bn;
    __syncthreads();
  }
  __syncthreads();
  if (tid == 0) {
    double lo, hi;
    if (steps == 1) {
      lo = hi = al[0];
    } else {
      lo = tridiag_eig(al, be, steps, 0);
      hi = tridiag_eig(al, be, steps, steps - 1);
    }
    double* o = a.bounds_out + ((int64_t)patch * (LV::count - 1) + L) * 2;
    o[0] = lo;
    o[1] = hi;
  }
  __syncthreads();
}

template <int DIM, class LV>
__global__ __launch_bounds__(NT<double>) void lanczos_kernel(PatchArgs a) {
  using T = double;
  using Lay = Layout<T, DIM, LV>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  Ctx<T, DIM, LV> c;
  c.lds = reinterpret_cast<T*>(smem_raw);
  c.vec = Lay::vec_in_lds ? c.lds + Lay::vec_off
                          : reinterpret_cast<T*>(a.vec_scratch) + (int64_t)blockIdx.x * a.vec_stride;
  c.gtab = a.tab64;
  const int patch = patch_of_block(a);
  {
    // load_patch without the Chebyshev parameters
    const int tid = threadIdx.x;
    const T* tab = a.tab64;
    for (int l = 0; l < LV::count; ++l) {
      const int sz = tab_size(LV::q[l]);
      for (int i = tid; i < sz; i += NT<T>) c.lds[Lay::tab_level_off(l) + i] = tab[l * kTabLevelStride + i];
    }
    load_geometry<T, DIM>(a, patch, c.geo(), c.mu());
    if constexpr (Lay::dinv0_global) c.dinv0 = const_cast<double*>(a.invdiag64[0]) + (int64_t)patch * Lay::level_size(0);
    for (int l = 0; l < LV::count; ++l) {
      if (Lay::dinv0_global && l == 0) continue;
      const int sz = Lay::level_size(l);
      const double* src = a.invdiag64[l] + (int64_t)patch * sz;
      for (int i = tid; i < sz; i += NT<T>) c.dinv(l)[i] = src[i];
    }
    __syncthreads();
  }
  prepare_geometry<T, DIM, LV>(c);
  if (a.level == 0) lanczos_level<DIM, LV, 0>(c, a, patch);
  if constexpr (LV::count > 2)
    if (a.level == 1) lanczos_level<DIM, LV, 1>(c, a, patch);
  if constexpr (LV::count > 3)
    if (a.level == 2) lanczos_level<DIM, LV, 2>(c, a, patch);
}

// ---------------------------------------------------------------------------
// setup: dense matrices of the small levels, A_{j,q} e_j column by column
// with the matrix-free FP64 operator
// ---------------------------------------------------------------------------

template <int DIM, class LV>
__global__ __launch_bounds__(NT<double>) void dense_kernel(PatchArgs a) {
  using T = double;
  using Lay = Layout<T, DIM, LV>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  Ctx<T, DIM, LV> c;
  c.lds = reinterpret_cast<T*>(smem_raw);
  c.vec = Lay::vec_in_lds ? c.lds + Lay::vec_off
                          : reinterpret_cast<T*>(a.vec_scratch) + (int64_t)blockIdx.x * a.vec_stride;
  c.gtab = a.tab64;
  const int patch = patch_of_block(a);
  const int tid = threadIdx.x;
  {
    const T* tab = a.tab64;
    for (int l = 0; l < LV::count; ++l) {
      const int sz = tab_size(LV::q[l]);
      for (int i = tid; i < sz; i += NT<T>) c.lds[Lay::tab_level_off(l) + i] = tab[l * kTabLevelStride + i];
    }
    load_geometry<T, DIM>(a, patch, c.geo(), c.mu());
    __syncthreads();
  }
  prepare_geometry<T, DIM, LV>(c);
  auto run = [&](auto Lc) {
    constexpr int L = decltype(Lc)::value;
    if constexpr (Lay::dense_level(L) || Lay::dense_global(L)) {
      constexpr int N = Lay::level_size(L);
      double* M = a.dense64[L] + (int64_t)patch * N * N;
      T* e = c.z();
      for (int j = 0; j < N; ++j) {
        for (int i = tid; i < N; i += NT<T>) e[i] = i == j ? 1.0 : 0.0;
        __syncthreads();
        apply_vec<T, DIM, LV, L>(c, e);
        for (int i = tid; i < N; i += NT<T>) M[i * N + j] = c.Out()[i];
        __syncthreads();
      }
    }
  };
  run(std::integral_constant<int, 0>{});
  if constexpr (LV::count > 1) run(std::integral_constant<int, 1>{});
  if constexpr (LV::count > 2) run(std::integral_constant<int, 2>{});
  if constexpr (LV::count > 3) run(std::integral_constant<int, 3>{});
}

// setup: FP64 matrix of one level (args.level) for a list of patches, by the
// matrix-free operator applied to unit vectors; row-major, one matrix per
// list position
template <int DIM, class LV>
__global__ __launch_bounds__(NT<double>) void level_matrix_kernel(PatchArgs a) {
  using T = double;
  using Lay = Layout<T, DIM, LV>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  Ctx<T, DIM, LV> c;
  c.lds = reinterpret_cast<T*>(smem_raw);
  c.vec = Lay::vec_in_lds ? c.lds + Lay::vec_off
                          : reinterpret_cast<T*>(a.vec_scratch) + (int64_t)blockIdx.x * a.vec_stride;
  c.gtab = a.tab64;
  const int patch = patch_of_block(a);
  const int tid = threadIdx.x;
  {
    const T* tab = a.tab64;
    for (int l = 0; l < LV::count; ++l) {
      const int sz = tab_size(LV::q[l]);
      for (int i = tid; i < sz; i += NT<T>) c.lds[Lay::tab_level_off(l) + i] = tab[l * kTabLevelStride + i];
    }
    load_geometry<T, DIM>(a, patch, c.geo(), c.mu());
    __syncthreads();
  }
  prepare_geometry<T, DIM, LV>(c);
  auto run = [&](auto Lc) {
    constexpr int L = decltype(Lc)::value;
    constexpr int N = Lay::level_size(L);
    double* M = a.out + (int64_t)(a.patch_begin + blockIdx.x) * N * N;
    T* e = c.z();
    for (int j = 0; j < N; ++j) {
      for (int i = tid; i < N; i += NT<T>) e[i] = i == j ? 1.0 : 0.0;
      __syncthreads();
      apply_vec<T, DIM, LV, L>(c, e);
      for (int i = tid; i < N; i += NT<T>) M[(int64_t)i * N + j] = c.Out()[i];
      __syncthreads();
    }
  };
  if (a.level == 0) run(std::integral_constant<int, 0>{});
  if constexpr (LV::count > 1)
    if (a.level == 1) run(std::integral_constant<int, 1>{});
  if constexpr (LV::count > 2)
    if (a.level == 2) run(std::integral_constant<int, 2>{});
  if constexpr (LV::count > 3)
    if (a.level == 3) run(std::integral_constant<int, 3>{});
}

// ---------------------------------------------------------------------------
// features of the bound-predicting network, one 64-thread block per patch:
// for every cell c and every point g of the 2-point Gauss rule,
// det J / h^d, ||J||_F^2 / h^2 and ||cof J||_F^2 / h^(2(d-1)) at (c 2^d + g) 3,
// then log10 mu_c minus its patch mean; h = (mean cell volume)^(1/d)
// ---------------------------------------------------------------------------

template <int DIM>
__global__ __launch_bounds__(64) void feature_kernel(PatchArgs a, float* out) {
  constexpr int ncell = ipow(2, DIM), npt = ipow(2, DIM), nvert = ipow(3, DIM);
  constexpr int NF = 3 * ncell * npt + ncell;
  __shared__ double geo[nvert * DIM], mu[ncell], red[64];
  const int patch = a.patch_begin + blockIdx.x;
  const int t = threadIdx.x;
  load_geometry<double, DIM>(a, patch, geo, mu);
  __syncthreads();
  double det = 0, fro = 0, cfro = 0;
  if (t < ncell * npt) {
    const int c = t / npt, g = t % npt;
    const double lo = 0.5 - 0.5 / sqrt(3.0), hi = 0.5 + 0.5 / sqrt(3.0);
    const double xi[3] = {(g & 1) ? hi : lo, ((g >> 1) & 1) ? hi : lo, ((g >> 2) & 1) ? hi : lo};
    const int cc[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
    double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int k = 0; k < ncell; ++k) {
      int b[3] = {k & 1, (k >> 1) & 1, (k >> 2) & 1};
      int v = (cc[0] + b[0]) + 3 * (cc[1] + b[1]);
      if (DIM == 3) v += 9 * (cc[2] + b[2]);
      for (int s2 = 0; s2 < DIM; ++s2) {
        double dphi = 1.0;
        for (int i = 0; i < DIM; ++i)
          dphi *= (i == s2) ? (b[i] ? 1.0 : -1.0) : (b[i] ? xi[i] : 1.0 - xi[i]);
        for (int r = 0; r < DIM; ++r) J[r][s2] += geo[v * DIM + r] * dphi;
      }
    }
    if (DIM == 3) {
      double C[3][3];
      C[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
      C[0][1] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
      C[0][2] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
      C[1][0] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
      C[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
      C[1][2] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
      C[2][0] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
      C[2][1] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
      C[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
      det = J[0][0] * C[0][0] + J[0][1] * C[0][1] + J[0][2] * C[0][2];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          fro += J[i][j] * J[i][j];
          cfro += C[i][j] * C[i][j];
        }
    } else {
      det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
      fro = J[0][0] * J[0][0] + J[0][1] * J[0][1] + J[1][0] * J[1][0] + J[1][1] * J[1][1];
      cfro = fro;  // the 2D cofactor matrix is a signed permutation of J
    }
  }
  red[t] = det;
  __syncthreads();
  if (t == 0) {
    double sdet = 0;
    for (int i = 0; i < ncell * npt; ++i) sdet += red[i];
    red[0] = sdet / (ncell * npt);  // mean cell volume (Gauss weights 2^-d)
  }
  __syncthreads();
  const double h = pow(red[0], 1.0 / DIM);
  float* o = out + (int64_t)patch * NF;
  if (t < ncell * npt) {
    o[3 * t] = (float)(det / pow(h, (double)DIM));
    o[3 * t + 1] = (float)(fro / (h * h));
    o[3 * t + 2] = (float)(cfro / pow(h, 2.0 * (DIM - 1)));
  }
  if (t < ncell) {
    double m = 0;
    for (int i = 0; i < ncell; ++i) m += log10(mu[i]);
    o[3 * ncell * npt + t] = (float)(log10(mu[t]) - m / ncell);
  }
}

// ---------------------------------------------------------------------------
// launchers and registry
// ---------------------------------------------------------------------------

// Workgroups may use more than 64 KB of LDS on gfx950 (160 KB per CU); ask
// for it explicitly before the first launch of a kernel that needs it.
template <typename K>
hipError_t allow_lds(K kernel, size_t bytes) {
  if (bytes == 0) return hipSuccess;
  // set once per kernel and device: the attribute persists, and launches
  // recorded into a graph must not be preceded by other runtime calls
  static std::mutex mu;
  static std::set<std::tuple<const void*, int, size_t>> done;
  int dev = 0;
  (void)hipGetDevice(&dev);
  const auto key = std::make_tuple(reinterpret_cast<const void*>(kernel), dev, bytes);
  {
    std::lock_guard<std::mutex> lock(mu);
    if (done.count(key)) return hipSuccess;
  }
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess) {
    std::lock_guard<std::mutex> lock(mu);
    done.insert(key);
  } else {
    int dev = 0, lim = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    fprintf(stderr, "libpmg: cannot grant %zu bytes of LDS (device limit %d): %s\n", bytes, lim,
            hipGetErrorString(e));
  }
  return e;
}

// On a failed launch, print what the runtime knows about the kernel.
template <typename K>
hipError_t report_launch(K kernel, const char* what, dim3 grid, size_t lds, int threads = 256) {
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) return e;
  hipFuncAttributes fa{};
  hipError_t e2 = hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(kernel));
  fprintf(stderr,
          "libpmg: launch of %s failed: %s (grid %u, block %d, dynamic LDS %zu); attributes "
          "(%s): maxThreads %d, static LDS %zu, max dynamic LDS %d, regs %d, local %zu\n",
          what, hipGetErrorString(e), grid.x, threads, lds, hipGetErrorString(e2),
          fa.maxThreadsPerBlock, fa.sharedSizeBytes, fa.maxDynamicSharedSizeBytes, fa.numRegs,
          fa.localSizeBytes);
  return e;
}

template <typename T, int DIM, class LV>
struct Variant {
  using Lay = Layout<T, DIM, LV>;
  static size_t lds_bytes(int) { return (size_t)Lay::lds_elems * sizeof(T); }
  static int64_t vec_elems() { return Lay::vec_in_lds ? 0 : (int64_t)Lay::vec_total; }
  static int64_t metric_elems() {
    return Lay::cache_G ? (int64_t)Lay::G_total : (int64_t)Lay::G_glob_elems;
  }
  template <int MODE, bool PERSIST>
  static hipError_t go(const PatchArgs& a, int g, size_t lds, hipStream_t s) {
    hipError_t e = allow_lds(patch_kernel<T, DIM, LV, MODE, PERSIST>, lds);
    if (e) return e;
    (void)hipGetLastError();  // clear a stale error of an earlier call
    hipLaunchKernelGGL((patch_kernel<T, DIM, LV, MODE, PERSIST>), dim3(g), dim3(NT<T>), lds, s, a);
    return report_launch(patch_kernel<T, DIM, LV, MODE, PERSIST>, "patch", dim3(g), lds, NT<T>);
  }
  // Grant the LDS of every patch-kernel instantiation the handle may launch
  // (both launch forms of the smoothing kernel), so that no first launch,
  // which sets the kernel attribute, happens while a stream is captured.
  template <int MODE, bool PERSIST>
  static hipError_t prime_one() {
    return allow_lds(patch_kernel<T, DIM, LV, MODE, PERSIST>, lds_bytes(MODE));
  }
  static hipError_t prime() {
    hipError_t e = prime_one<kModeSmooth, false>();
    if (!e) e = prime_one<kModeSmooth, true>();
    if (!e) e = prime_one<kModeResidual, false>();
    if (!e) e = prime_one<kModeSolve, false>();
    if (!e) e = prime_one<kModeApply, false>();
    if (!e) e = prime_one<kModeMetric, false>();
    if (!e) e = prime_one<kModeSmoothCart, false>();
    if (!e) e = prime_one<kModeSmoothCart, true>();
    if constexpr (std::is_same<T, double>::value) {
      if (!e) e = prime_one<kModePcg, false>();
      if (!e) e = prime_one<kModePcgCart, false>();
    }
    return e;
  }
  static hipError_t launch(int mode, const PatchArgs& a, hipStream_t s) {
    if (a.n_patch <= 0) return hipSuccess;
    const size_t lds = lds_bytes(mode);
    // persistent grids for smoothing only; other modes: one workgroup per patch
    const bool persist = (mode == kModeSmooth || mode == kModeSmoothCart) && a.grid > 0 && a.grid < a.n_patch;
    int g = persist ? a.grid : a.n_patch;
    if (a.map_mode == 1) g = (g + 7) / 8 * 8;  // whole rounds over the 8 XCDs
    switch (mode) {
      case kModeSmooth:
        return persist ? go<kModeSmooth, true>(a, g, lds, s) : go<kModeSmooth, false>(a, g, lds, s);
      case kModeSmoothCart:
        return persist ? go<kModeSmoothCart, true>(a, g, lds, s) : go<kModeSmoothCart, false>(a, g, lds, s);
      case kModeResidual: return go<kModeResidual, false>(a, g, lds, s);
      case kModeSolve: return go<kModeSolve, false>(a, g, lds, s);
      case kModeApply: return go<kModeApply, false>(a, g, lds, s);
      case kModeMetric: return go<kModeMetric, false>(a, g, lds, s);
      case kModePcg:
        if constexpr (std::is_same<T, double>::value) return go<kModePcg, false>(a, g, lds, s);
        return hipErrorInvalidValue;
      case kModePcgCart:
        if constexpr (std::is_same<T, double>::value) return go<kModePcgCart, false>(a, g, lds, s);
        return hipErrorInvalidValue;
      default: return hipErrorInvalidValue;
    }
  }
  static hipError_t launch_diag(const PatchArgs& a, hipStream_t s) {
    using L64 = Layout<double, DIM, LV>;
    if (a.n_patch <= 0) return hipSuccess;
    const size_t lds = (size_t)L64::lds_elems * sizeof(double);
    hipError_t e = allow_lds(diag_kernel<DIM, LV>, lds);
    if (e != hipSuccess) return e;
    (void)hipGetLastError();
    hipLaunchKernelGGL((diag_kernel<DIM, LV>), dim3(a.n_patch), dim3(NT<double>), lds, s, a);
    return report_launch(diag_kernel<DIM, LV>, "diag", dim3(a.n_patch), lds);
  }
  static hipError_t launch_dense(const PatchArgs& a, hipStream_t s) {
    using L64 = Layout<double, DIM, LV>;
    if (a.n_patch <= 0) return hipSuccess;
    const size_t lds = (size_t)L64::lds_elems * sizeof(double);
    hipError_t e = allow_lds(dense_kernel<DIM, LV>, lds);
    if (e != hipSuccess) return e;
    (void)hipGetLastError();
    hipLaunchKernelGGL((dense_kernel<DIM, LV>), dim3(a.n_patch), dim3(NT<double>), lds, s, a);
    return report_launch(dense_kernel<DIM, LV>, "dense", dim3(a.n_patch), lds);
  }
  static hipError_t launch_level_matrix(const PatchArgs& a, hipStream_t s) {
    using L64 = Layout<double, DIM, LV>;
    if (a.n_patch <= 0) return hipSuccess;
    const size_t lds = (size_t)L64::lds_elems * sizeof(double);
    hipError_t e = allow_lds(level_matrix_kernel<DIM, LV>, lds);
    if (e != hipSuccess) return e;
    (void)hipGetLastError();
    hipLaunchKernelGGL((level_matrix_kernel<DIM, LV>), dim3(a.n_patch), dim3(NT<double>), lds, s, a);
    return report_launch(level_matrix_kernel<DIM, LV>, "level matrix", dim3(a.n_patch), lds);
  }
  static hipError_t launch_lanczos(const PatchArgs& a, int level, hipStream_t s) {
    using L64 = Layout<double, DIM, LV>;
    if (a.n_patch <= 0) return hipSuccess;
    PatchArgs b = a;
    b.level = level;
    const size_t lds = (size_t)L64::lds_elems * sizeof(double);
    hipError_t e = allow_lds(lanczos_kernel<DIM, LV>, lds);
    if (e != hipSuccess) return e;
    (void)hipGetLastError();
    hipLaunchKernelGGL((lanczos_kernel<DIM, LV>), dim3(a.n_patch), dim3(NT<double>), lds, s, b);
    return report_launch(lanczos_kernel<DIM, LV>, "lanczos", dim3(a.n_patch), lds);
  }
};

template <typename T, int DIM, int... Qs>
PatchVariant make_variant() {
  using LV = Levels<Qs...>;
  using V = Variant<T, DIM, LV>;
  PatchVariant v{};
  v.precision = std::is_same<T, double>::value ? PMG_FP64 : PMG_FP32;
  v.dim = DIM;
  v.n_levels = LV::count;
  const int q[] = {Qs...};
  for (int i = 0; i < kMaxLevels; ++i) v.levels[i] = i < LV::count ? q[i] : 0;
  v.launch = &V::launch;
  v.prime = &V::prime;
  v.lds_bytes = &V::lds_bytes;
  v.vec_scratch_elems = &V::vec_elems;
  v.metric_elems = &V::metric_elems;
  v.vec_scratch_elems64 = &Variant<double, DIM, LV>::vec_elems;
  // the FP64 setup kernels use the FP64 layout of the same level list
  v.launch_diag = &Variant<double, DIM, LV>::launch_diag;
  v.launch_lanczos = &Variant<double, DIM, LV>::launch_lanczos;
  v.launch_dense = &Variant<double, DIM, LV>::launch_dense;
  v.launch_level_matrix = &Variant<double, DIM, LV>::launch_level_matrix;
  for (int l = 0; l < kMaxLevels; ++l)
    v.dense_level[l] = l < LV::count && (Layout<T, DIM, LV>::dense_level(l) ||
                                         Layout<T, DIM, LV>::dense_global(l)) ? 1 : 0;
  return v;
}

// BF16-input / FP32-accumulate variants: FP32 layout and vectors, the top
// level's interpolation contractions on the matrix cores (slab-form tops of
// degree 6 and 7); setup kernels as for the plain level list.
template <bool SPLIT, int DIM, int... Qs>
PatchVariant make_variant_bf16() {
  using LV = LevelsBF16<SPLIT, Qs...>;
  using LP = Levels<Qs...>;
  using V = Variant<float, DIM, LV>;
  static_assert(!Layout<float, DIM, LV>::seg_top && !Layout<float, DIM, LV>::quarter_top,
                "the matrix-core operator is the slab form");
  PatchVariant v = make_variant<float, DIM, Qs...>();
  v.precision = SPLIT ? PMG_BF16X3_FP32ACC : PMG_BF16_FP32ACC;
  v.launch = &V::launch;
  v.prime = &V::prime;
  v.lds_bytes = &V::lds_bytes;
  v.vec_scratch_elems = &V::vec_elems;
  v.metric_elems = &V::metric_elems;
  v.vec_scratch_elems64 = &Variant<double, DIM, LP>::vec_elems;
  return v;
}

// Fill this translation unit's copy of the per-degree 1D tables on the
// current device.
inline hipError_t upload_tables() {
  std::vector<double> t64(kConstTab, 0.0);
  for (int q = 1; q <= kMaxDegree; ++q) {
    DegreeTables t = degree_tables(q);
    const int n = t.n;
    double* dst = t64.data() + ctab_off(q);
    std::copy(t.B.begin(), t.B.end(), dst);
    std::copy(t.Dc.begin(), t.Dc.end(), dst + n * n);
    std::copy(t.D.begin(), t.D.end(), dst + 2 * n * n);
    std::copy(t.xg.begin(), t.xg.end(), dst + 3 * n * n);
    std::copy(t.wg.begin(), t.wg.end(), dst + 3 * n * n + n);
  }
  std::vector<float> t32(t64.begin(), t64.end());
  hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_tab64), t64.data(), t64.size() * sizeof(double));
  if (e != hipSuccess) return e;
  return hipMemcpyToSymbol(HIP_SYMBOL(c_tab32), t32.data(), t32.size() * sizeof(float));
}

}  // namespace

// One table of variants per patch_variants_*.hip file (level lists grouped
// so that the files take similar compile times), and the upload of that
// file's constant tables.
struct VariantPart {
  const PatchVariant* (*table)(size_t* count);
  hipError_t (*upload)();
};
#define PMG_VARIANT_PART(name)                      \
  const PatchVariant* name##_table(size_t* count); \
  hipError_t name##_upload();
PMG_VARIANT_PART(variants_2d)
PMG_VARIANT_PART(variants_3d_low)
PMG_VARIANT_PART(variants_3d_q6)
PMG_VARIANT_PART(variants_3d_q7)
PMG_VARIANT_PART(variants_3d_q8)
#undef PMG_VARIANT_PART

}  // namespace pmgi
