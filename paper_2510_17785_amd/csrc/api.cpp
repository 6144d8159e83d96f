// C ABI of the patch smoother and the GMG-CG solver: validation, handle
// lifetime, setup orchestration and the host loops of the outer solver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "fe_tables.hpp"
#include "internal.hpp"

using namespace pmgi;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

}  // namespace

// the thread-local message of pmg_last_error, for the other translation units
int pmgi::set_error(int code, const char* msg) {
  g_last_error = msg;
  return code;
}

namespace {

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(e_ == hipErrorOutOfMemory ? PMG_ERR_OOM : PMG_ERR_HIP, "%s: %s (%s:%d)", \
                  #expr, hipGetErrorString(e_), __FILE__, __LINE__);                   \
  } while (0)

#define PMG_TRY(expr)         \
  do {                        \
    int s_ = (expr);          \
    if (s_ < 0) return s_;    \
  } while (0)

int ipow(int b, int e) {
  int r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

template <typename P>
int dev_alloc(P** ptr, size_t bytes, size_t* counter) {
  void* p = nullptr;
  if (bytes == 0) bytes = 8;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess)
    return fail(e == hipErrorOutOfMemory ? PMG_ERR_OOM : PMG_ERR_HIP, "hipMalloc(%zu): %s", bytes,
                hipGetErrorString(e));
  *ptr = reinterpret_cast<P*>(p);
  if (counter) *counter += bytes;
  return PMG_OK;
}

// det J > 0 at the corners and Gauss points of every cell (the paper excludes
// degenerate patches, Section 3.2)
int check_mesh(int dim, int N, const double* X, int p) {
  // det J at the cell corners and at the Gauss points of degree p, every
  // cell; shape-function derivatives tabulated once, cells split over threads
  std::vector<double> xg, wg;
  gauss_rule(p + 1, xg, wg);
  std::vector<double> pts = {0.0, 1.0};
  pts.insert(pts.end(), xg.begin(), xg.end());
  const int N1 = N + 1;
  const int ncell = ipow(N, dim);
  const int np = (int)pts.size(), nc = 1 << dim;
  const int npt = dim == 3 ? np * np * np : np * np;
  std::vector<double> dN((size_t)npt * nc * dim);
  for (int k = 0; k < npt; ++k) {
    const double xi[3] = {pts[k % np], pts[(k / np) % np], dim == 3 ? pts[k / (np * np)] : 0.0};
    for (int c = 0; c < nc; ++c)
      for (int s = 0; s < dim; ++s) {
        double d = 1.0;
        for (int i = 0; i < dim; ++i) {
          const int b = (c >> i) & 1;
          d *= (i == s) ? (b ? 1.0 : -1.0) : (b ? xi[i] : 1.0 - xi[i]);
        }
        dN[((size_t)k * nc + c) * dim + s] = d;
      }
  }
  auto bad_cell = [&](auto dim_tag, int e) {
    constexpr int D = decltype(dim_tag)::value, NC = 1 << D;
    const int ex = e % N, ey = (e / N) % N, ez = D == 3 ? e / (N * N) : 0;
    double C[NC][D];
    for (int c = 0; c < NC; ++c) {
      int g = (ex + (c & 1)) + (ey + ((c >> 1) & 1)) * N1;
      if (D == 3) g += (ez + ((c >> 2) & 1)) * N1 * N1;
      for (int r = 0; r < D; ++r) C[c][r] = X[g * D + r];
    }
    for (int k = 0; k < npt; ++k) {
      double J[D][D] = {};
      const double* d = dN.data() + (size_t)k * NC * D;
      for (int c = 0; c < NC; ++c)
        for (int s2 = 0; s2 < D; ++s2)
          for (int r = 0; r < D; ++r) J[r][s2] += C[c][r] * d[c * D + s2];
      double det;
      if constexpr (D == 2)
        det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
      else
        det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
              J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
              J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
      if (!(det > 0.0)) return true;
    }
    return false;
  };
  const int nthreads = std::max(1, std::min<int>(16, (int)std::thread::hardware_concurrency()));
  std::vector<int> first_bad(nthreads, ncell);
  std::vector<std::thread> pool;
  for (int t = 0; t < nthreads; ++t)
    pool.emplace_back([&, t]() {
      for (int e = t; e < ncell; e += nthreads)
        if (dim == 3 ? bad_cell(std::integral_constant<int, 3>{}, e)
                     : bad_cell(std::integral_constant<int, 2>{}, e)) {
          first_bad[t] = e;
          return;
        }
    });
  for (auto& th : pool) th.join();
  const int e = *std::min_element(first_bad.begin(), first_bad.end());
  if (e < ncell)
    return fail(PMG_ERR_DEGENERATE, "cell %d (%d,%d,%d) has det J <= 0 at a quadrature point", e,
                e % N, (e / N) % N, dim == 3 ? e / (N * N) : 0);
  return PMG_OK;
}

}  // namespace

struct pmg_handle {
  int dim = 0, N = 0, p = 0, precision = 0, L = 0;
  int levels[kMaxLevels] = {0};
  int cheb_degree = 3, n_vcycles = 1, bounds_kind = PMG_BOUNDS_LANCZOS, lanczos_steps = 12;
  double safety = 1.1, range = 15.0;
  uint64_t seed = 0;
  hipStream_t stream = nullptr;
  const PatchVariant* var = nullptr;
  int n_patches = 0, n_colors = 0;
  std::vector<int> color_off;
  int max_color = 0;
  size_t device_bytes = 0;
  bool bounds_valid = false;
  // device memory
  double* verts = nullptr;
  double* mu = nullptr;
  int32_t* patch_vertex = nullptr;
  double* patch_geo = nullptr;  // independent patches: n x 3^d x d
  double* patch_mu = nullptr;   // independent patches: n x 2^d
  double* tab64 = nullptr;
  void* tab = nullptr;
  double* invdiag64[kMaxLevels] = {nullptr};
  void* invdiag[kMaxLevels] = {nullptr};
  double* dense64[kMaxLevels] = {nullptr};
  void* dense[kMaxLevels] = {nullptr};
  void* cheb = nullptr;
  void* vec_scratch = nullptr;
  void* metric = nullptr;  // per patch: the metric the patch kernel keeps in LDS (see PatchArgs)
  double* pcg_work = nullptr;  // pmg_patch_pcg: residual and search direction per patch
  // local smoother: PMG_SMOOTHER_CHEBYSHEV, or PMG_SMOOTHER_CARTESIAN with its
  // damping and fast-diagonalisation tables (kFdmStride per level, in T)
  int smoother = PMG_SMOOTHER_CHEBYSHEV;
  double omega = 0.5;
  void* fdm_tab = nullptr;  // T, kMaxLevels x kFdmStride
  double* add_buf = nullptr;  // additive smoother: local residuals and corrections per patch
  int64_t vec_bytes = 0;  // bytes per block slot of vec_scratch
  int64_t vec_blocks = 0;
  std::vector<double> bounds;  // host copy, n_patches x (L-1) x 2
  // patches of boundary vertices (PMG_PATCH_WITH_BOUNDARY)
  bool with_boundary = false;
  std::vector<int32_t> vertex_host;  // patch vertex per patch (mesh handles)
  std::vector<int32_t> trunc_host;   // per patch: slot of its coarse inverse or -1
  int32_t* trunc_index = nullptr;
  double* trunc_inv = nullptr;
  int n_trunc = 0;
  // launch shape of the smoothing kernel (set by pmg_autotune)
  int tune_grid = 0, tune_map = 0;
  int64_t local_dofs = 0;  // sum over patches of unmasked interior nodes (top level)
  int level_size(int l) const { return ipow(2 * levels[l] - 1, dim); }
  size_t tsize() const { return precision == PMG_FP64 ? sizeof(double) : sizeof(float); }
  PatchArgs args() const {
    PatchArgs a{};
    a.verts = verts;
    a.mu = mu;
    a.patch_vertex = patch_vertex;
    a.patch_geo = patch_geo;
    a.patch_mu = patch_mu;
    a.N = N;
    a.p = p;
    a.tab = tab;
    a.tab64 = tab64;
    for (int l = 0; l < kMaxLevels; ++l) {
      a.invdiag[l] = invdiag[l];
      a.invdiag64[l] = invdiag64[l];
      a.dense[l] = dense[l];
      a.dense64[l] = dense64[l];
    }
    a.cheb = cheb;
    a.cheb_degree = cheb_degree;
    a.n_vcycles = n_vcycles;
    a.vec_scratch = vec_scratch;
    a.vec_stride = vec_bytes / (int64_t)tsize();
    a.lanczos_steps = lanczos_steps;
    a.seed = seed;
    a.with_boundary = with_boundary ? 1 : 0;
    a.trunc_index = trunc_index;
    a.trunc_inv = trunc_inv;
    a.grid = tune_grid;
    a.map_mode = tune_map;
    a.metric = metric;
    return a;
  }
};

namespace {

void free_handle(pmg_handle* h) {
  if (!h) return;
  void* ptrs[] = {h->verts, h->mu,          h->patch_vertex, h->patch_geo, h->patch_mu,
                  h->tab64, h->cheb,        h->vec_scratch,  h->trunc_index, h->trunc_inv,
                  h->metric,  h->pcg_work,     h->fdm_tab,      h->add_buf};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (h->tab && h->tab != h->tab64) (void)hipFree(h->tab);  // FP64 handles share the tables
  for (int l = 0; l < kMaxLevels; ++l) {
    if (h->invdiag64[l]) (void)hipFree(h->invdiag64[l]);
    if (h->invdiag[l] && h->invdiag[l] != h->invdiag64[l]) (void)hipFree(h->invdiag[l]);
    if (h->dense64[l]) (void)hipFree(h->dense64[l]);
    if (h->dense[l] && h->dense[l] != h->dense64[l]) (void)hipFree(h->dense[l]);
  }
  delete h;
}

// launch a per-patch kernel over patches [begin, end) in chunks that fit the
// vector scratch
int launch_chunks(pmg_handle* h, int mode, PatchArgs a, int begin, int end,
                  hipStream_t stream) {
  const int chunk = h->vec_blocks > 0 ? (int)h->vec_blocks : (end - begin);
  for (int s = begin; s < end; s += std::max(chunk, 1)) {
    a.patch_begin = s;
    a.n_patch = std::min(chunk, end - s);
    HIP_TRY(h->var->launch(mode, a, stream));
  }
  return PMG_OK;
}
int launch_chunks(pmg_handle* h, int mode, PatchArgs a, int begin, int end) {
  return launch_chunks(h, mode, a, begin, end, h->stream);
}

size_t n_dofs(const pmg_handle* h) {
  const int64_t M = (int64_t)h->N * h->p + 1;
  return (size_t)(h->dim == 3 ? M * M * M : M * M);
}

// launch shapes the autotuners try: (workgroups, mapping); 0 workgroups =
// one per patch
constexpr int kLaunchCandidates = 6;
int launch_candidates(int (*c)[2]) {
  int dev = 0, cus = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int t[kLaunchCandidates][2] = {{0, 0}, {0, 1}, {cus, 1}, {2 * cus, 1}, {4 * cus, 1}, {2 * cus, 0}};
  for (int k = 0; k < kLaunchCandidates; ++k) {
    c[k][0] = t[k][0];
    c[k][1] = t[k][1];
  }
  return PMG_OK;
}

// reps calls of fn on `stream`, timed with events (ms for all of them)
template <class F>
int time_launches(hipStream_t stream, int reps, F fn, float* ms) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (!e) e = hipEventCreate(&e1);
  if (!e) e = hipEventRecord(e0, stream);
  int st = PMG_OK;
  for (int r = 0; r < reps && !e && st == PMG_OK; ++r) st = fn();
  if (!e) e = hipEventRecord(e1, stream);
  if (!e) e = hipEventSynchronize(e1);
  if (!e && ms) e = hipEventElapsedTime(ms, e0, e1);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (st != PMG_OK) return st;
  if (e) return fail(PMG_ERR_HIP, "timing: %s", hipGetErrorString(e));
  return PMG_OK;
}

// colours [c_begin, c_end) of a sweep (reversed for direction -1) on `stream`
int smooth_on(pmg_handle* h, double* u, const double* b, int c_begin, int c_end, int direction,
              hipStream_t stream) {
  const bool cart = h->smoother == PMG_SMOOTHER_CARTESIAN;
  PatchArgs a = h->args();
  a.u = u;
  a.b = b;
  a.fdm_tab = h->fdm_tab;
  a.fdm_omega = h->omega;
  for (int k = c_begin; k < c_end; ++k) {
    const int c = direction > 0 ? k : c_end - 1 - (k - c_begin);
    PMG_TRY(launch_chunks(h, cart ? kModeSmoothCart : kModeSmooth, a, h->color_off[c], h->color_off[c + 1],
                          stream));
  }
  return PMG_OK;
}

int set_cheb(pmg_handle* h) {
  const int nl = h->L - 1;
  std::vector<double> c64((size_t)h->n_patches * nl * 2);
  for (int j = 0; j < h->n_patches; ++j)
    for (int l = 0; l < nl; ++l) {
      const double lo = h->bounds[((size_t)j * nl + l) * 2], hi = h->bounds[((size_t)j * nl + l) * 2 + 1];
      if (!(lo > 0.0) || !(hi >= lo) || !std::isfinite(hi))
        return fail(PMG_ERR_INVALID_ARG, "patch %d level %d: bad bounds (%g, %g)", j, l, lo, hi);
      // interval [a, b]: b = s lambda_max, a = max(lambda_min, b / rho)
      const double b = h->safety * hi;
      const double a = std::max(lo, b / h->range);
      c64[((size_t)j * nl + l) * 2] = 0.5 * (b + a);
      c64[((size_t)j * nl + l) * 2 + 1] = 0.5 * (b - a);
    }
  if (h->precision == PMG_FP64) {
    HIP_TRY(hipMemcpyAsync(h->cheb, c64.data(), c64.size() * sizeof(double), hipMemcpyHostToDevice,
                           h->stream));
  } else {
    std::vector<float> c32(c64.begin(), c64.end());
    HIP_TRY(hipMemcpyAsync(h->cheb, c32.data(), c32.size() * sizeof(float), hipMemcpyHostToDevice,
                           h->stream));
  }
  HIP_TRY(hipStreamSynchronize(h->stream));
  h->bounds_valid = true;
  return PMG_OK;
}

// option checks shared by every setup; fills the level list and the kernel variant
int check_opts(const pmg_opts* o, int dim, int p, int* levels, int& L, const PatchVariant*& var) {
  if (o->precision < PMG_FP64 || o->precision > PMG_BF16X3_FP32ACC)
    return fail(PMG_ERR_INVALID_ARG, "unknown precision %d", o->precision);
  if (o->cheb_degree < 1 || o->cheb_degree > 8)
    return fail(PMG_ERR_INVALID_ARG, "Chebyshev degree %d outside 1..8", o->cheb_degree);
  if (o->n_vcycles < 1) return fail(PMG_ERR_INVALID_ARG, "n_vcycles must be >= 1");
  if (o->bounds != PMG_BOUNDS_LANCZOS && o->bounds != PMG_BOUNDS_FIXED)
    return fail(PMG_ERR_INVALID_ARG, "unknown bounds source %d", o->bounds);
  if (o->patch_set != PMG_PATCH_INTERIOR && o->patch_set != PMG_PATCH_WITH_BOUNDARY)
    return fail(PMG_ERR_INVALID_ARG, "unknown patch set %d", o->patch_set);
  if (o->coarse_mean < PMG_COARSE_ARITHMETIC || o->coarse_mean > PMG_COARSE_HARMONIC)
    return fail(PMG_ERR_INVALID_ARG, "unknown coarse coefficient rule %d", o->coarse_mean);
  if (o->lanczos_steps < 2 || o->lanczos_steps > 64)
    return fail(PMG_ERR_INVALID_ARG, "lanczos_steps %d outside 2..64", o->lanczos_steps);
  if (!(o->cheb_safety >= 1.0) || !(o->cheb_range > 1.0))
    return fail(PMG_ERR_INVALID_ARG, "cheb_safety must be >= 1 and cheb_range > 1");
  L = o->n_levels;
  if (L == 0) {
    int q = p;
    while (true) {
      if (L >= kMaxLevels) return fail(PMG_ERR_UNSUPPORTED, "default halving needs > %d levels", kMaxLevels);
      levels[L++] = q;
      if (q == 1) break;
      q = q / 2;
    }
  } else {
    if (L < 2 || L > kMaxLevels) return fail(PMG_ERR_INVALID_ARG, "n_levels %d outside 2..%d", L, kMaxLevels);
    for (int l = 0; l < L; ++l) levels[l] = o->levels[l];
  }
  if (levels[0] != p) return fail(PMG_ERR_INVALID_ARG, "levels[0] = %d must equal p = %d", levels[0], p);
  if (levels[L - 1] != 1) return fail(PMG_ERR_INVALID_ARG, "last level must be degree 1");
  for (int l = 1; l < L; ++l)
    if (levels[l] >= levels[l - 1]) return fail(PMG_ERR_INVALID_ARG, "levels must strictly decrease");
  var = find_variant(o->precision, dim, L, levels);
  if (!var)
    return fail(PMG_ERR_UNSUPPORTED, "no kernel compiled for this level list (available: %s)",
                list_variants().c_str());
  return PMG_OK;
}

int init_tables_once() {
  {
    // the per-degree tables in constant memory, once per device
    static int initialised_device = -1;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (initialised_device != dev) {
      HIP_TRY(init_constant_tables());
      initialised_device = dev;
    }
  }

  return PMG_OK;
}

// Boundary-vertex patches: per direction the first unmasked interior offset
// and the number of unmasked offsets at degree q (flags as in the kernels:
// bit 2i low boundary, bit 2i+1 high boundary of direction i).
int vertex_flags(const pmg_handle* h, int vlin) {
  const int N1 = h->N + 1;
  const int v[3] = {vlin % N1, (vlin / N1) % N1, h->dim == 3 ? vlin / (N1 * N1) : 1};
  int f = 0;
  for (int i = 0; i < h->dim; ++i) {
    if (v[i] == 0) f |= 1 << (2 * i);
    if (v[i] == h->N) f |= 2 << (2 * i);
  }
  return f;
}
void unmasked_box(int f, int dim, int q, int* lo, int* n) {
  for (int i = 0; i < 3; ++i) {
    const int fl = i < dim ? (f >> (2 * i)) & 3 : 0;
    lo[i] = (fl & 1) ? q + 1 : 1;
    n[i] = i < dim ? (fl ? q - 1 : 2 * q - 1) : 1;
  }
}

// Exact coarse solves of the boundary-vertex patches: the matrix of level
// L-2 (the lowest with nodes) formed on the device in FP64, its unmasked
// block inverted on the host by Cholesky, stored per patch in the cut
// patch's own node numbering.
int setup_truncated(pmg_handle* h) {
  const int L = h->L, Lc = L - 2, q = h->levels[Lc], n = h->level_size(Lc);
  std::vector<int32_t> list;
  h->trunc_host.assign(h->n_patches, -1);
  for (int j = 0; j < h->n_patches; ++j)
    if (vertex_flags(h, h->vertex_host[j])) {
      h->trunc_host[j] = (int32_t)list.size();
      list.push_back(j);
    }
  h->n_trunc = (int)list.size();
  if (list.empty()) return PMG_OK;
  int lo[3], nn[3];
  unmasked_box(1, h->dim, q, lo, nn);  // a face patch has the largest unmasked box
  const int64_t slot = (int64_t)nn[0] * nn[1] * nn[2] * nn[0] * nn[1] * nn[2];
  int s;
  hipError_t e;
  int32_t* dlist = nullptr;
  double* dmat = nullptr;
  const int chunk_max = 1024;
  if ((s = dev_alloc(&dlist, list.size() * sizeof(int32_t), nullptr)) < 0) return s;
  if ((s = dev_alloc(&dmat, (size_t)chunk_max * n * n * sizeof(double), nullptr)) < 0) {
    (void)hipFree(dlist);
    return s;
  }
  std::vector<double> inv((size_t)list.size() * slot, 0.0), A((size_t)chunk_max * n * n);
  int st = PMG_OK;
  if ((e = hipMemcpy(dlist, list.data(), list.size() * sizeof(int32_t), hipMemcpyHostToDevice)))
    st = fail(PMG_ERR_HIP, "upload: %s", hipGetErrorString(e));
  PatchArgs a = h->args();
  a.vec_stride = h->vec_bytes / (int64_t)sizeof(double);  // FP64 setup kernels
  a.level = Lc;
  a.out = dmat;
  for (int b = 0; b < (int)list.size() && st == PMG_OK; b += chunk_max) {
    const int cnt = std::min(chunk_max, (int)list.size() - b);
    const int c2 = h->vec_blocks > 0 ? std::min<int>(cnt, (int)h->vec_blocks) : cnt;
    a.patch_list = dlist + b;  // the kernel writes list position patch_begin + block
    for (int b2 = b; b2 < b + cnt && st == PMG_OK; b2 += c2) {
      a.patch_begin = b2 - b;
      a.n_patch = std::min(c2, b + cnt - b2);
      if ((e = h->var->launch_level_matrix(a, h->stream)))
        st = fail(PMG_ERR_HIP, "level matrix kernel: %s", hipGetErrorString(e));
    }
    if (st == PMG_OK &&
        ((e = hipMemcpyAsync(A.data(), dmat, (size_t)cnt * n * n * sizeof(double), hipMemcpyDeviceToHost,
                             h->stream)) ||
         (e = hipStreamSynchronize(h->stream))))
      st = fail(PMG_ERR_HIP, "level matrices: %s", hipGetErrorString(e));
    for (int k = 0; k < cnt && st == PMG_OK; ++k) {
      const int j = list[b + k];
      unmasked_box(vertex_flags(h, h->vertex_host[j]), h->dim, q, lo, nn);
      const int nu = nn[0] * nn[1] * nn[2], mi = 2 * q - 1;
      std::vector<int> full(nu);
      for (int u = 0; u < nu; ++u) {
        const int ox = u % nn[0], oy = (u / nn[0]) % nn[1], oz = u / (nn[0] * nn[1]);
        full[u] = (lo[0] + ox - 1) + mi * ((lo[1] + oy - 1) + (h->dim == 3 ? mi * (lo[2] + oz - 1) : 0));
      }
      // Cholesky A = R^T R of the unmasked block, then the inverse column by column
      std::vector<double> R((size_t)nu * nu);
      const double* Ak = A.data() + (size_t)k * n * n;
      for (int r = 0; r < nu; ++r)
        for (int c = 0; c < nu; ++c) R[(size_t)r * nu + c] = Ak[(size_t)full[r] * n + full[c]];
      for (int c = 0; c < nu && st == PMG_OK; ++c) {
        double d = R[(size_t)c * nu + c];
        for (int t = 0; t < c; ++t) d -= R[(size_t)t * nu + c] * R[(size_t)t * nu + c];
        if (!(d > 0.0)) {
          st = fail(PMG_ERR_DEGENERATE, "patch %d: coarse level matrix not positive definite", j);
          break;
        }
        d = std::sqrt(d);
        R[(size_t)c * nu + c] = d;
        for (int r = c + 1; r < nu; ++r) {
          double v = R[(size_t)c * nu + r];
          for (int t = 0; t < c; ++t) v -= R[(size_t)t * nu + c] * R[(size_t)t * nu + r];
          R[(size_t)c * nu + r] = v / d;
        }
      }
      if (st != PMG_OK) break;
      double* out = inv.data() + (size_t)(b + k) * slot;
      std::vector<double> y(nu);
      for (int c = 0; c < nu; ++c) {
        // R^T y = e_c, then R x = y
        for (int r = 0; r < nu; ++r) {
          double v = r == c ? 1.0 : 0.0;
          for (int t = 0; t < r; ++t) v -= R[(size_t)t * nu + r] * y[t];
          y[r] = v / R[(size_t)r * nu + r];
        }
        for (int r = nu - 1; r >= 0; --r) {
          double v = y[r];
          for (int t = r + 1; t < nu; ++t) v -= R[(size_t)r * nu + t] * out[(size_t)t * nu + c];
          out[(size_t)r * nu + c] = v / R[(size_t)r * nu + r];
        }
      }
    }
  }
  (void)hipFree(dlist);
  (void)hipFree(dmat);
  if (st != PMG_OK) return st;
  if ((s = dev_alloc(&h->trunc_inv, inv.size() * sizeof(double), &h->device_bytes)) < 0) return s;
  if ((s = dev_alloc(&h->trunc_index, (size_t)h->n_patches * sizeof(int32_t), &h->device_bytes)) < 0)
    return s;
  if ((e = hipMemcpy(h->trunc_inv, inv.data(), inv.size() * sizeof(double), hipMemcpyHostToDevice)) ||
      (e = hipMemcpy(h->trunc_index, h->trunc_host.data(), h->trunc_host.size() * sizeof(int32_t),
                     hipMemcpyHostToDevice)))
    return fail(PMG_ERR_HIP, "upload: %s", hipGetErrorString(e));
  return PMG_OK;
}

// everything after the geometry is on the device: tables, scratch, inverse
// diagonals, dense small levels, Chebyshev bounds
int setup_common(pmg_handle* h) {
  const int L = h->L;
  const int* levels = h->levels;
  const PatchVariant* var = h->var;
  hipError_t e;
  int s;
  auto cleanup = [&](int st) { return st; };
  // launch attributes of every patch kernel of the variant, once per device,
  // before any launch can be recorded into a graph
  if ((e = var->prime())) return fail(PMG_ERR_HIP, "patch kernel attributes: %s", hipGetErrorString(e));
  // 1D tables: per level B, Dc, D, xg, wg; per transfer the patch prolongation
  std::vector<double> tab(kTabSize, 0.0);
  for (int l = 0; l < L; ++l) {
    DegreeTables t = degree_tables(levels[l]);
    const int n = t.n;
    double* dst = tab.data() + l * kTabLevelStride;
    std::copy(t.B.begin(), t.B.end(), dst);
    std::copy(t.Dc.begin(), t.Dc.end(), dst + n * n);
    std::copy(t.D.begin(), t.D.end(), dst + 2 * n * n);
    std::copy(t.xg.begin(), t.xg.end(), dst + 3 * n * n);
    std::copy(t.wg.begin(), t.wg.end(), dst + 3 * n * n + n);
  }
  for (int l = 0; l + 1 < L; ++l) {
    std::vector<double> P = patch_prolongation_1d(levels[l], levels[l + 1], 2);
    std::copy(P.begin(), P.end(), tab.data() + kMaxLevels * kTabLevelStride + l * kTabTransferStride);
  }
  if ((s = dev_alloc(&h->tab64, tab.size() * sizeof(double), &h->device_bytes)) < 0) return cleanup(s);
  if ((e = hipMemcpy(h->tab64, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice)))
    return cleanup(fail(PMG_ERR_HIP, "upload: %s", hipGetErrorString(e)));
  if (h->precision == PMG_FP64) {
    h->tab = h->tab64;
  } else {
    std::vector<float> t32(tab.begin(), tab.end());
    if ((s = dev_alloc(&h->tab, t32.size() * sizeof(float), &h->device_bytes)) < 0) return cleanup(s);
    if ((e = hipMemcpy(h->tab, t32.data(), t32.size() * sizeof(float), hipMemcpyHostToDevice)))
      return cleanup(fail(PMG_ERR_HIP, "upload: %s", hipGetErrorString(e)));
  }

  // vector scratch when the level vectors do not fit in LDS (sized for the
  // larger of the working-precision and FP64 layouts)
  {
    const int64_t e1 = var->vec_scratch_elems() * (int64_t)h->tsize();
    const int64_t e2 = var->vec_scratch_elems64() * (int64_t)sizeof(double);
    const int64_t bytes_per_block = std::max(e1, e2);
    if (bytes_per_block > 0) {
      // a multiple of 8 slots: the XCD-aware launch rounds its grid up to one
      h->vec_blocks = (h->max_color + 7) / 8 * 8;
      h->vec_bytes = bytes_per_block;
      if ((s = dev_alloc(&h->vec_scratch, (size_t)bytes_per_block * h->vec_blocks, &h->device_bytes)) < 0)
        return cleanup(s);
    }
  }

  // inverse diagonals of every level (FP64), then the working-precision copy
  for (int l = 0; l < L; ++l) {
    const size_t cnt = (size_t)h->n_patches * h->level_size(l);
    if ((s = dev_alloc(&h->invdiag64[l], cnt * sizeof(double), &h->device_bytes)) < 0) return cleanup(s);
    if (h->precision == PMG_FP64) {
      h->invdiag[l] = h->invdiag64[l];
    } else if ((s = dev_alloc(&h->invdiag[l], cnt * sizeof(float), &h->device_bytes)) < 0) {
      return cleanup(s);
    }
  }
  {
    PatchArgs a = h->args();
    a.vec_stride = h->vec_bytes / (int64_t)sizeof(double);  // FP64 setup kernels
    const int chunk = h->vec_blocks > 0 ? (int)h->vec_blocks : h->n_patches;
    for (int b = 0; b < h->n_patches; b += chunk) {
      a.patch_begin = b;
      a.n_patch = std::min(chunk, h->n_patches - b);
      if ((e = var->launch_diag(a, h->stream)))
        return cleanup(fail(PMG_ERR_HIP, "diagonal kernel (%d patches, LDS %zu bytes of FP64 layout): %s",
                            a.n_patch, var->lds_bytes(-1), hipGetErrorString(e)));
    }
    if (h->precision != PMG_FP64)
      for (int l = 0; l < L; ++l)
        if ((e = launch_convert_to_float((int64_t)h->n_patches * h->level_size(l), h->invdiag64[l],
                                         reinterpret_cast<float*>(h->invdiag[l]), h->stream)))
          return cleanup(fail(PMG_ERR_HIP, "convert: %s", hipGetErrorString(e)));
  }
  // dense matrices of the small levels (formed with the FP64 matrix-free operator)
  {
    bool any = false;
    for (int l = 0; l < L; ++l) {
      if (!var->dense_level[l]) continue;
      any = true;
      const size_t cnt = (size_t)h->n_patches * h->level_size(l) * h->level_size(l);
      if ((s = dev_alloc(&h->dense64[l], cnt * sizeof(double), &h->device_bytes)) < 0) return cleanup(s);
      if (h->precision == PMG_FP64) {
        h->dense[l] = h->dense64[l];
      } else if ((s = dev_alloc(&h->dense[l], cnt * sizeof(float), &h->device_bytes)) < 0) {
        return cleanup(s);
      }
    }
    if (any) {
      PatchArgs a = h->args();
      a.vec_stride = h->vec_bytes / (int64_t)sizeof(double);  // FP64 setup kernels
      const int chunk = h->vec_blocks > 0 ? (int)h->vec_blocks : h->n_patches;
      for (int b = 0; b < h->n_patches; b += chunk) {
        a.patch_begin = b;
        a.n_patch = std::min(chunk, h->n_patches - b);
        if ((e = var->launch_dense(a, h->stream)))
          return cleanup(fail(PMG_ERR_HIP, "dense level kernel: %s", hipGetErrorString(e)));
      }
      if (h->precision != PMG_FP64)
        for (int l = 0; l < L; ++l)
          if (var->dense_level[l] &&
              (e = launch_convert_to_float((int64_t)h->n_patches * h->level_size(l) * h->level_size(l),
                                           h->dense64[l], reinterpret_cast<float*>(h->dense[l]),
                                           h->stream)))
            return cleanup(fail(PMG_ERR_HIP, "convert: %s", hipGetErrorString(e)));
    }
  }
  if (h->with_boundary && !h->patch_geo && (s = setup_truncated(h)) < 0) return cleanup(s);
  const size_t ncheb = (size_t)h->n_patches * (L - 1) * 2;
  if ((s = dev_alloc(&h->cheb, ncheb * h->tsize(), &h->device_bytes)) < 0) return cleanup(s);
  h->bounds.assign(ncheb, 0.0);
  // the metric of the levels that keep it in LDS, once per patch of a mesh:
  // the patch updates read it instead of recomputing it at every sweep
  if (!h->patch_geo && var->metric_elems() > 0) {
    const size_t cnt = (size_t)h->n_patches * var->metric_elems();
    if ((s = dev_alloc(&h->metric, cnt * h->tsize(), &h->device_bytes)) < 0) return cleanup(s);
    PatchArgs a = h->args();
    a.metric = nullptr;  // computed by this launch
    a.metric_out = h->metric;
    a.grid = 0;
    a.map_mode = 0;
    if ((s = launch_chunks(h, kModeMetric, a, 0, h->n_patches)) < 0) return cleanup(s);
  }

  if (h->bounds_kind == PMG_BOUNDS_LANCZOS) {
    double* dbounds = nullptr;
    double* basis = nullptr;
    const int chunk = std::min(h->n_patches, 4096);
    const size_t basis_elems = (size_t)chunk * h->lanczos_steps * h->level_size(0);
    if ((s = dev_alloc(&dbounds, ncheb * sizeof(double), nullptr)) < 0) return cleanup(s);
    if ((s = dev_alloc(&basis, basis_elems * sizeof(double), nullptr)) < 0) {
      (void)hipFree(dbounds);
      return cleanup(s);
    }
    PatchArgs a = h->args();
    a.vec_stride = h->vec_bytes / (int64_t)sizeof(double);  // FP64 setup kernels
    a.lanczos_basis = basis;
    a.bounds_out = dbounds;
    int st = PMG_OK;
    for (int l = 0; l + 1 < L && st == PMG_OK; ++l) {
      for (int b = 0; b < h->n_patches; b += chunk) {
        // the vector scratch (if any) has vec_blocks slots
        const int c2 = h->vec_blocks > 0 ? std::min<int>(chunk, (int)h->vec_blocks) : chunk;
        for (int b2 = b; b2 < std::min(b + chunk, h->n_patches); b2 += c2) {
          a.patch_begin = b2;
          a.n_patch = std::min(c2, std::min(b + chunk, h->n_patches) - b2);
          if ((e = var->launch_lanczos(a, l, h->stream))) {
            st = fail(PMG_ERR_HIP, "lanczos kernel: %s", hipGetErrorString(e));
            break;
          }
        }
      }
    }
    if (st == PMG_OK) {
      if ((e = hipMemcpyAsync(h->bounds.data(), dbounds, ncheb * sizeof(double), hipMemcpyDeviceToHost,
                              h->stream)) ||
          (e = hipStreamSynchronize(h->stream)))
        st = fail(PMG_ERR_HIP, "bounds: %s", hipGetErrorString(e));
    }
    (void)hipFree(dbounds);
    (void)hipFree(basis);
    if (st != PMG_OK) return cleanup(st);
    if ((s = set_cheb(h)) < 0) return cleanup(s);
  } else {
    if ((e = hipStreamSynchronize(h->stream)))
      return cleanup(fail(PMG_ERR_HIP, "setup: %s", hipGetErrorString(e)));
  }
  return PMG_OK;
}

pmg_handle* new_handle(const pmg_opts* o, int dim, int N, int p, int L, const int* levels,
                       const PatchVariant* var) {
  pmg_handle* h = new pmg_handle();
  h->dim = dim;
  h->N = N;
  h->p = p;
  h->precision = o->precision;
  h->L = L;
  for (int l = 0; l < L; ++l) h->levels[l] = levels[l];
  h->cheb_degree = o->cheb_degree;
  h->n_vcycles = o->n_vcycles;
  h->bounds_kind = o->bounds;
  h->lanczos_steps = o->lanczos_steps;
  h->safety = o->cheb_safety;
  h->range = o->cheb_range;
  h->seed = o->seed;
  h->stream = reinterpret_cast<hipStream_t>(o->stream);
  h->var = var;
  h->with_boundary = o->patch_set == PMG_PATCH_WITH_BOUNDARY;

  return h;
}

int patch_setup_impl(const pmg_mesh* mesh, const double* coeff, int p, const pmg_opts* o,
                     pmg_handle** out) {
  if (!mesh || !coeff || !o || !out || !mesh->vertices)
    return fail(PMG_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  const int dim = mesh->dim, N = mesh->n_cells;
  if (dim != 2 && dim != 3) return fail(PMG_ERR_INVALID_ARG, "dim must be 2 or 3, got %d", dim);
  if (N < 2) return fail(PMG_ERR_INVALID_ARG, "need at least 2 cells per direction, got %d", N);
  if (p < 1 || p > kMaxDegree) return fail(PMG_ERR_INVALID_ARG, "degree %d outside 1..15", p);
  int levels[kMaxLevels] = {0};
  int L = 0;
  const PatchVariant* var = nullptr;
  PMG_TRY(check_opts(o, dim, p, levels, L, var));
  PMG_TRY(check_mesh(dim, N, mesh->vertices, p));
  for (size_t i = 0, nc = (size_t)ipow(N, dim); i < nc; ++i)
    if (!(coeff[i] > 0.0) || !std::isfinite(coeff[i]))
      return fail(PMG_ERR_INVALID_ARG, "coefficient of cell %zu is %g", i, coeff[i]);
  PMG_TRY(init_tables_once());
  pmg_handle* h = new_handle(o, dim, N, p, L, levels, var);
  auto cleanup = [&](int s) {
    free_handle(h);
    return s;
  };
  // patches in sweep order: colour sum_i 2^i (v_i mod 2), lexicographic within
  const int N1 = N + 1;
  std::vector<int32_t> order;
  h->n_colors = 1 << dim;
  h->color_off.assign(h->n_colors + 1, 0);
  const int v_lo = h->with_boundary ? 0 : 1, v_hi = h->with_boundary ? N : N - 1;
  for (int col = 0; col < h->n_colors; ++col) {
    h->color_off[col] = (int)order.size();
    for (int vz = (dim == 3 ? v_lo : 0); vz <= (dim == 3 ? v_hi : 0); ++vz)
      for (int vy = v_lo; vy <= v_hi; ++vy)
        for (int vx = v_lo; vx <= v_hi; ++vx) {
          int c = (vx & 1) | ((vy & 1) << 1) | (dim == 3 ? ((vz & 1) << 2) : 0);
          if (c != col) continue;
          order.push_back(vx + vy * N1 + (dim == 3 ? vz * N1 * N1 : 0));
        }
    h->max_color = std::max(h->max_color, (int)order.size() - h->color_off[col]);
  }
  h->color_off[h->n_colors] = (int)order.size();
  h->n_patches = (int)order.size();
  h->vertex_host = order;
  for (int32_t v : order) {  // local interior nodes: 2p-1 per direction, p-1 where cut
    int64_t cnt = 1;
    for (int i = 0; i < dim; ++i) {
      const int vi = i == 0 ? v % N1 : i == 1 ? (v / N1) % N1 : v / (N1 * N1);
      cnt *= (vi == 0 || vi == N) ? p - 1 : 2 * p - 1;
    }
    h->local_dofs += cnt;
  }

  const size_t nv = (size_t)ipow(N1, dim), nc = (size_t)ipow(N, dim);
  int s;
  if ((s = dev_alloc(&h->verts, nv * dim * sizeof(double), &h->device_bytes)) < 0) return cleanup(s);
  if ((s = dev_alloc(&h->mu, nc * sizeof(double), &h->device_bytes)) < 0) return cleanup(s);
  if ((s = dev_alloc(&h->patch_vertex, order.size() * sizeof(int32_t), &h->device_bytes)) < 0)
    return cleanup(s);
  hipError_t e;
  if ((e = hipMemcpy(h->verts, mesh->vertices, nv * dim * sizeof(double), hipMemcpyHostToDevice)) ||
      (e = hipMemcpy(h->mu, coeff, nc * sizeof(double), hipMemcpyHostToDevice)) ||
      (e = hipMemcpy(h->patch_vertex, order.data(), order.size() * sizeof(int32_t),
                     hipMemcpyHostToDevice)))
    return cleanup(fail(PMG_ERR_HIP, "upload: %s", hipGetErrorString(e)));

  if ((s = setup_common(h)) < 0) return cleanup(s);
  *out = h;
  return PMG_OK;
}

}  // namespace

int patches_setup_impl(int dim, int64_t n, const double* verts, const double* coeff, int p,
                       const pmg_opts* o, pmg_handle** out) {
  if (!verts || !coeff || !o || !out) return fail(PMG_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  if (dim != 2 && dim != 3) return fail(PMG_ERR_INVALID_ARG, "dim must be 2 or 3, got %d", dim);
  if (n < 1 || n > (1 << 26)) return fail(PMG_ERR_INVALID_ARG, "patch count %lld out of range", (long long)n);
  if (p < 1 || p > kMaxDegree) return fail(PMG_ERR_INVALID_ARG, "degree %d outside 1..15", p);
  int levels[kMaxLevels] = {0};
  int L = 0;
  const PatchVariant* var = nullptr;
  PMG_TRY(check_opts(o, dim, p, levels, L, var));
  const int nvert = ipow(3, dim), ncell = ipow(2, dim);
  // every patch is a 2-cell-per-direction mesh: reuse the cell check
  for (int64_t j = 0; j < n; ++j) {
    int st = check_mesh(dim, 2, verts + j * nvert * dim, p);
    if (st < 0) return fail(st, "patch %lld: %s", (long long)j, pmg_last_error());
    for (int c = 0; c < ncell; ++c)
      if (!(coeff[j * ncell + c] > 0.0) || !std::isfinite(coeff[j * ncell + c]))
        return fail(PMG_ERR_INVALID_ARG, "patch %lld cell %d: coefficient %g", (long long)j, c,
                    coeff[j * ncell + c]);
  }
  PMG_TRY(init_tables_once());
  pmg_handle* h = new_handle(o, dim, 2, p, L, levels, var);
  h->with_boundary = false;  // independent patches have no mesh boundary
  auto cleanup = [&](int st) {
    free_handle(h);
    return st;
  };
  h->n_patches = (int)n;
  h->n_colors = 1;
  h->color_off = {0, (int)n};
  h->max_color = (int)n;
  int s;
  hipError_t e;
  if ((s = dev_alloc(&h->patch_geo, (size_t)n * nvert * dim * sizeof(double), &h->device_bytes)) < 0)
    return cleanup(s);
  if ((s = dev_alloc(&h->patch_mu, (size_t)n * ncell * sizeof(double), &h->device_bytes)) < 0)
    return cleanup(s);
  if ((e = hipMemcpy(h->patch_geo, verts, (size_t)n * nvert * dim * sizeof(double), hipMemcpyHostToDevice)) ||
      (e = hipMemcpy(h->patch_mu, coeff, (size_t)n * ncell * sizeof(double), hipMemcpyHostToDevice)))
    return cleanup(fail(PMG_ERR_HIP, "upload: %s", hipGetErrorString(e)));
  if ((s = setup_common(h)) < 0) return cleanup(s);
  *out = h;
  return PMG_OK;
}

int n_features(int dim) { return 3 * ipow(4, dim) + ipow(2, dim); }

// Lanczos bounds for the listed patches (host indices) into h->bounds
int lanczos_for(pmg_handle* h, const std::vector<int32_t>& list) {
  if (list.empty()) return PMG_OK;
  const int L = h->L;
  const size_t nb = (size_t)h->n_patches * (L - 1) * 2;
  double* dbounds = nullptr;
  double* basis = nullptr;
  int32_t* dlist = nullptr;
  int st = PMG_OK;
  const int cnt = (int)list.size();
  int chunk = std::min(cnt, 4096);
  if (h->vec_blocks > 0) chunk = std::min<int>(chunk, (int)h->vec_blocks);
  if ((st = dev_alloc(&dbounds, nb * sizeof(double), nullptr)) < 0) return st;
  if ((st = dev_alloc(&basis, (size_t)chunk * h->lanczos_steps * h->level_size(0) * sizeof(double), nullptr)) < 0 ||
      (st = dev_alloc(&dlist, list.size() * sizeof(int32_t), nullptr)) < 0) {
    (void)hipFree(dbounds);
    if (basis) (void)hipFree(basis);
    return st;
  }
  hipError_t e = hipMemcpy(dlist, list.data(), list.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  PatchArgs a = h->args();
  a.vec_stride = h->vec_bytes / (int64_t)sizeof(double);
  a.lanczos_basis = basis;
  a.bounds_out = dbounds;
  a.patch_list = dlist;
  for (int l = 0; l + 1 < L && e == hipSuccess; ++l)
    for (int b = 0; b < cnt && e == hipSuccess; b += chunk) {
      a.patch_begin = b;
      a.n_patch = std::min(chunk, cnt - b);
      e = h->var->launch_lanczos(a, l, h->stream);
    }
  std::vector<double> hb(nb);
  if (e == hipSuccess)
    e = hipMemcpyAsync(hb.data(), dbounds, nb * sizeof(double), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) st = fail(PMG_ERR_HIP, "lanczos fallback: %s", hipGetErrorString(e));
  else
    for (int32_t j : list)
      for (int k = 0; k < (L - 1) * 2; ++k) h->bounds[(size_t)j * (L - 1) * 2 + k] = hb[(size_t)j * (L - 1) * 2 + k];
  (void)hipFree(dbounds);
  (void)hipFree(basis);
  (void)hipFree(dlist);
  return st;
}

// ---------------------------------------------------------------------------
// GMG
// ---------------------------------------------------------------------------

struct gmg_handle {
  int dim = 0, p = 0, nlev = 0;
  hipStream_t stream = nullptr;
  std::vector<int> sizes;             // cells per direction, coarsest first
  std::vector<pmg_handle*> smoother;  // [0] unused
  std::vector<double*> verts, mu;     // per level
  std::vector<double*> f, u, t, cellbuf;
  std::vector<int*> hfirst;           // per transfer (coarse level l -> l+1)
  std::vector<double*> hw;
  double* tab64 = nullptr;
  double* tbuf[2] = {nullptr, nullptr};  // transfer intermediates (finest size)
  double* coarse_inv = nullptr;
  double* cpack[2] = {nullptr, nullptr};
  int coarse_n = 0;
  double *x = nullptr, *r = nullptr, *z = nullptr, *d = nullptr, *Ad = nullptr;
  double* partial = nullptr;
  double* scal = nullptr;  // device scalars
  double* hscal = nullptr; // pinned host scalars
  int post_dir = -1;       // colour order of the post-smoothing sweep (-1: reversed)
  double add_theta = 0.0;  // > 0: additive sweeps with this damping instead of multiplicative ones
  std::vector<double*> kv; // GMRES: Krylov basis and preconditioned vectors (grown on demand)
  int64_t len(int l) const {
    int64_t M = (int64_t)sizes[l] * p + 1;
    return dim == 3 ? M * M * M : M * M;
  }
  int M(int l) const { return sizes[l] * p + 1; }
};

namespace {

void free_gmg(gmg_handle* g) {
  if (!g) return;
  for (pmg_handle* h : g->smoother)
    if (h) free_handle(h);
  auto fr = [](void* p) {
    if (p) (void)hipFree(p);
  };
  for (auto* p : g->verts) fr(p);
  for (auto* p : g->mu) fr(p);
  for (auto* p : g->f) fr(p);
  for (auto* p : g->u) fr(p);
  for (auto* p : g->t) fr(p);
  for (auto* p : g->cellbuf) fr(p);
  for (auto* p : g->hfirst) fr(p);
  for (auto* p : g->hw) fr(p);
  fr(g->tab64);
  fr(g->tbuf[0]);
  fr(g->tbuf[1]);
  fr(g->coarse_inv);
  fr(g->cpack[0]);
  fr(g->cpack[1]);
  fr(g->x);
  fr(g->r);
  fr(g->z);
  fr(g->d);
  fr(g->Ad);
  fr(g->partial);
  fr(g->scal);
  for (auto* p : g->kv) fr(p);
  if (g->hscal) (void)hipHostFree(g->hscal);
  delete g;
}

int global_apply(gmg_handle* g, int l, const double* x, double* y) {
  CellArgs a{g->verts[l], g->mu[l], g->sizes[l], g->p, g->dim, g->tab64};
  HIP_TRY(launch_cell_apply(a, x, g->cellbuf[l], g->stream));
  HIP_TRY(launch_cell_gather(g->dim, g->sizes[l], g->p, g->cellbuf[l], y, g->stream));
  return PMG_OK;
}

// out (fine level l+1) = P in (coarse level l), or its transpose
int h_transfer(gmg_handle* g, int l, const double* in, double* out, bool transpose) {
  const int Mc = g->M(l), Mf = g->M(l + 1), dim = g->dim;
  int cur[3] = {transpose ? Mf : Mc, transpose ? Mf : Mc, dim == 3 ? (transpose ? Mf : Mc) : 1};
  const double* src = in;
  for (int axis = 0; axis < dim; ++axis) {
    int nxt[3] = {cur[0], cur[1], cur[2]};
    nxt[axis] = transpose ? Mc : Mf;
    double* dst = axis == dim - 1 ? out : g->tbuf[axis & 1];
    HIP_TRY(launch_h_prolong_axis(dim, axis, cur, nxt, g->hfirst[l], g->hw[l], g->p, src, dst,
                                  transpose ? 1 : 0, g->stream));
    src = dst;
    for (int i = 0; i < 3; ++i) cur[i] = nxt[i];
  }
  HIP_TRY(launch_mask_dirichlet(dim, transpose ? Mc : Mf, out, g->stream));
  return PMG_OK;
}

int vcycle(gmg_handle* g, int l, const double* f, double* u) {
  const int dim = g->dim;
  if (l == 0) {
    HIP_TRY(launch_gather_interior(dim, g->M(0), f, g->cpack[0], g->stream));
    HIP_TRY(launch_gemv(g->coarse_n, g->coarse_inv, g->cpack[0], g->cpack[1], g->stream));
    HIP_TRY(hipMemsetAsync(u, 0, g->len(0) * sizeof(double), g->stream));
    HIP_TRY(launch_scatter_interior(dim, g->M(0), g->cpack[1], u, g->stream));
    return PMG_OK;
  }
  pmg_handle* S = g->smoother[l];
  HIP_TRY(hipMemsetAsync(u, 0, g->len(l) * sizeof(double), g->stream));
  if (g->add_theta > 0.0)
    PMG_TRY(pmg_patch_smooth_additive(S, u, f, g->add_theta));
  else
    PMG_TRY(pmg_patch_smooth(S, u, f, +1));
  // residual r = f - A u, restricted to level l-1
  double* t = g->t[l];
  PMG_TRY(global_apply(g, l, u, t));
  HIP_TRY(launch_axpby(g->len(l), 1.0, f, -1.0, t, g->stream));
  PMG_TRY(h_transfer(g, l - 1, t, g->f[l - 1], true));
  PMG_TRY(vcycle(g, l - 1, g->f[l - 1], g->u[l - 1]));
  PMG_TRY(h_transfer(g, l - 1, g->u[l - 1], t, false));
  HIP_TRY(launch_axpby(g->len(l), 1.0, t, 1.0, u, g->stream));
  if (g->add_theta > 0.0)
    PMG_TRY(pmg_patch_smooth_additive(S, u, f, g->add_theta));
  else
    PMG_TRY(pmg_patch_smooth(S, u, f, g->post_dir));
  return PMG_OK;
}

int dot(gmg_handle* g, const double* x, const double* y, int slot) {
  const int64_t n = g->len(g->nlev - 1);
  HIP_TRY(launch_dot_partial(n, x, y, g->partial, kDotBlocks, g->stream));
  HIP_TRY(launch_dot_final(g->partial, kDotBlocks, g->scal + slot, g->stream));
  return PMG_OK;
}

// Run f(i) for i in [lo, hi) on all host threads, rows dealt round-robin
// (the triangular loops below give row i work proportional to i).
template <class F>
void parallel_rows(int lo, int hi, F f) {
  const int nt = (int)std::max(1u, std::min(std::thread::hardware_concurrency(), 64u));
  if (hi - lo < 2 * nt) {
    for (int i = lo; i < hi; ++i) f(i);
    return;
  }
  std::vector<std::thread> pool;
  for (int t = 0; t < nt; ++t)
    pool.emplace_back([&, t]() {
      for (int i = lo + t; i < hi; i += nt) f(i);
    });
  for (auto& th : pool) th.join();
}

// Dense SPD inverse through the Cholesky factor (host, FP64, all host
// threads): A = L L^T by blocked right-looking elimination (row-major, lower
// triangle in place), W = L^{-1} column by column, A^{-1} = W^T W.  Every
// inner loop is a dot product over contiguous memory.
int spd_inverse(std::vector<double>& A, int n) {
  constexpr int kB = 64;
  auto a = [&](int i, int j) -> double& { return A[(size_t)i * n + j]; };
  int bad = -1;
  for (int k0 = 0; k0 < n && bad < 0; k0 += kB) {
    const int k1 = std::min(n, k0 + kB);
    // diagonal block (the columns before k0 are already eliminated)
    for (int j = k0; j < k1 && bad < 0; ++j) {
      double d = a(j, j);
      for (int k = k0; k < j; ++k) d -= a(j, k) * a(j, k);
      if (!(d > 0.0)) {
        bad = j;
        break;
      }
      d = std::sqrt(d);
      a(j, j) = d;
      for (int i = j + 1; i < k1; ++i) {
        double v = a(i, j);
        for (int k = k0; k < j; ++k) v -= a(i, k) * a(j, k);
        a(i, j) = v / d;
      }
    }
    if (bad >= 0) break;
    // the panel below it, then the trailing lower triangle
    parallel_rows(k1, n, [&](int i) {
      double* ai = &a(i, 0);
      for (int j = k0; j < k1; ++j) {
        const double* aj = &a(j, 0);
        double v = ai[j];
        for (int k = k0; k < j; ++k) v -= ai[k] * aj[k];
        ai[j] = v / aj[j];
      }
    });
    parallel_rows(k1, n, [&](int i) {
      double* ai = &a(i, 0);
      for (int j = k1; j <= i; ++j) {
        const double* aj = &a(j, 0);
        double v = 0;
        for (int k = k0; k < k1; ++k) v += ai[k] * aj[k];
        ai[j] -= v;
      }
    });
  }
  if (bad >= 0) return fail(PMG_ERR_BREAKDOWN, "coarse matrix not SPD at row %d", bad);
  // Wt[c][i] = (L^{-1})[i][c] for i >= c: forward substitution per column c
  std::vector<double> Wt((size_t)n * n, 0.0);
  parallel_rows(0, n, [&](int c) {
    double* w = &Wt[(size_t)c * n];
    w[c] = 1.0 / a(c, c);
    for (int i = c + 1; i < n; ++i) {
      const double* ai = &a(i, 0);
      double v = 0;
      for (int k = c; k < i; ++k) v -= ai[k] * w[k];
      w[i] = v / ai[i];
    }
  });
  // A^{-1}[i][j] = sum_{k >= max(i, j)} W[k][i] W[k][j], symmetric
  parallel_rows(0, n, [&](int i) {
    const double* wi = &Wt[(size_t)i * n];
    for (int j = 0; j <= i; ++j) {
      const double* wj = &Wt[(size_t)j * n];
      double v = 0;
      for (int k = i; k < n; ++k) v += wi[k] * wj[k];
      A[(size_t)i * n + j] = v;
    }
  });
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j) A[(size_t)j * n + i] = A[(size_t)i * n + j];
  return PMG_OK;
}

int gmg_setup_impl(const pmg_mesh* mesh, const double* coeff, int p, const pmg_opts* o,
                   gmg_handle** out) {
  if (!mesh || !coeff || !o || !out || !mesh->vertices) return fail(PMG_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  const int dim = mesh->dim;
  if (dim != 2 && dim != 3) return fail(PMG_ERR_INVALID_ARG, "dim must be 2 or 3");
  if (p < 1 || p > kMaxDegree) return fail(PMG_ERR_INVALID_ARG, "degree %d outside 1..15", p);
  // hierarchy: halve while even and the halved mesh keeps an interior vertex
  std::vector<int> sizes = {mesh->n_cells};
  while (sizes.back() % 2 == 0 && sizes.back() / 2 >= 2) sizes.push_back(sizes.back() / 2);
  if (sizes.size() < 2) return fail(PMG_ERR_INVALID_ARG, "mesh with %d cells cannot be coarsened", mesh->n_cells);
  std::reverse(sizes.begin(), sizes.end());
  gmg_handle* g = new gmg_handle();
  g->dim = dim;
  g->p = p;
  g->nlev = (int)sizes.size();
  g->sizes = sizes;
  g->stream = reinterpret_cast<hipStream_t>(o->stream);
  auto cleanup = [&](int s) {
    free_gmg(g);
    return s;
  };
  const int L = g->nlev;
  // level geometry: shared vertices, mean coefficients of the children
  std::vector<std::vector<double>> V(L), Mu(L);
  V[L - 1].assign(mesh->vertices, mesh->vertices + (size_t)ipow(mesh->n_cells + 1, dim) * dim);
  Mu[L - 1].assign(coeff, coeff + (size_t)ipow(mesh->n_cells, dim));
  for (int l = L - 2; l >= 0; --l) {
    const int Nc = sizes[l], Nf = sizes[l + 1];
    const int Nc1 = Nc + 1, Nf1 = Nf + 1;
    V[l].assign((size_t)ipow(Nc1, dim) * dim, 0.0);
    Mu[l].assign((size_t)ipow(Nc, dim), 0.0);
    for (int v = 0; v < ipow(Nc1, dim); ++v) {
      const int vx = v % Nc1, vy = (v / Nc1) % Nc1, vz = dim == 3 ? v / (Nc1 * Nc1) : 0;
      const int f = 2 * vx + 2 * vy * Nf1 + (dim == 3 ? 2 * vz * Nf1 * Nf1 : 0);
      for (int r = 0; r < dim; ++r) V[l][(size_t)v * dim + r] = V[l + 1][(size_t)f * dim + r];
    }
    for (int e = 0; e < ipow(Nc, dim); ++e) {
      const int ex = e % Nc, ey = (e / Nc) % Nc, ez = dim == 3 ? e / (Nc * Nc) : 0;
      double s = 0;
      for (int c = 0; c < (1 << dim); ++c) {
        int f = (2 * ex + (c & 1)) + (2 * ey + ((c >> 1) & 1)) * Nf;
        if (dim == 3) f += (2 * ez + ((c >> 2) & 1)) * Nf * Nf;
        const double mu = Mu[l + 1][f];
        s += o->coarse_mean == PMG_COARSE_GEOMETRIC ? std::log(mu)
             : o->coarse_mean == PMG_COARSE_HARMONIC ? 1.0 / mu
                                                     : mu;
      }
      s /= (1 << dim);
      Mu[l][e] = o->coarse_mean == PMG_COARSE_GEOMETRIC ? std::exp(s)
                 : o->coarse_mean == PMG_COARSE_HARMONIC ? 1.0 / s
                                                         : s;
    }
  }
  g->smoother.assign(L, nullptr);
  g->verts.assign(L, nullptr);
  g->mu.assign(L, nullptr);
  g->f.assign(L, nullptr);
  g->u.assign(L, nullptr);
  g->t.assign(L, nullptr);
  g->cellbuf.assign(L, nullptr);
  int s;
  hipError_t e;
  for (int l = 0; l < L; ++l) {
    const int N = sizes[l];
    const size_t nv = (size_t)ipow(N + 1, dim), nc = (size_t)ipow(N, dim);
    if ((s = dev_alloc(&g->verts[l], nv * dim * sizeof(double), nullptr)) < 0) return cleanup(s);
    if ((s = dev_alloc(&g->mu[l], nc * sizeof(double), nullptr)) < 0) return cleanup(s);
    if ((e = hipMemcpy(g->verts[l], V[l].data(), nv * dim * sizeof(double), hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(g->mu[l], Mu[l].data(), nc * sizeof(double), hipMemcpyHostToDevice)))
      return cleanup(fail(PMG_ERR_HIP, "upload: %s", hipGetErrorString(e)));
    const size_t len = (size_t)g->len(l);
    if ((s = dev_alloc(&g->f[l], len * sizeof(double), nullptr)) < 0) return cleanup(s);
    if ((s = dev_alloc(&g->u[l], len * sizeof(double), nullptr)) < 0) return cleanup(s);
    if ((s = dev_alloc(&g->t[l], len * sizeof(double), nullptr)) < 0) return cleanup(s);
    if ((s = dev_alloc(&g->cellbuf[l], nc * ipow(p + 1, dim) * sizeof(double), nullptr)) < 0)
      return cleanup(s);
    if (l > 0) {
      pmg_mesh m{dim, N, V[l].data()};
      pmg_handle* h = nullptr;
      if ((s = patch_setup_impl(&m, Mu[l].data(), p, o, &h)) < 0) return cleanup(s);
      g->smoother[l] = h;
    }
  }
  for (int l = 0; l + 1 < L; ++l) {
    std::vector<int> first;
    std::vector<double> w;
    h_prolongation_1d(sizes[l], p, first, w);
    int* df = nullptr;
    double* dw = nullptr;
    if ((s = dev_alloc(&df, first.size() * sizeof(int), nullptr)) < 0) return cleanup(s);
    g->hfirst.push_back(df);
    if ((s = dev_alloc(&dw, w.size() * sizeof(double), nullptr)) < 0) return cleanup(s);
    g->hw.push_back(dw);
    if ((e = hipMemcpy(df, first.data(), first.size() * sizeof(int), hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(dw, w.data(), w.size() * sizeof(double), hipMemcpyHostToDevice)))
      return cleanup(fail(PMG_ERR_HIP, "upload: %s", hipGetErrorString(e)));
  }
  {
    DegreeTables t = degree_tables(p);
    const int n = t.n;
    std::vector<double> tab(3 * n * n + 2 * n);
    std::copy(t.B.begin(), t.B.end(), tab.begin());
    std::copy(t.Dc.begin(), t.Dc.end(), tab.begin() + n * n);
    std::copy(t.D.begin(), t.D.end(), tab.begin() + 2 * n * n);
    std::copy(t.xg.begin(), t.xg.end(), tab.begin() + 3 * n * n);
    std::copy(t.wg.begin(), t.wg.end(), tab.begin() + 3 * n * n + n);
    if ((s = dev_alloc(&g->tab64, tab.size() * sizeof(double), nullptr)) < 0) return cleanup(s);
    if ((e = hipMemcpy(g->tab64, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice)))
      return cleanup(fail(PMG_ERR_HIP, "upload: %s", hipGetErrorString(e)));
  }
  const size_t lf = (size_t)g->len(L - 1);
  for (int i = 0; i < 2; ++i)
    if ((s = dev_alloc(&g->tbuf[i], lf * sizeof(double), nullptr)) < 0) return cleanup(s);
  for (double** v : {&g->x, &g->r, &g->z, &g->d, &g->Ad})
    if ((s = dev_alloc(v, lf * sizeof(double), nullptr)) < 0) return cleanup(s);
  if ((s = dev_alloc(&g->partial, kDotBlocks * sizeof(double), nullptr)) < 0) return cleanup(s);
  if ((s = dev_alloc(&g->scal, 8 * sizeof(double), nullptr)) < 0) return cleanup(s);
  if ((e = hipHostMalloc((void**)&g->hscal, 8 * sizeof(double), hipHostMallocDefault)))
    return cleanup(fail(PMG_ERR_HIP, "hipHostMalloc: %s", hipGetErrorString(e)));

  // coarsest level: element matrices on the GPU, dense assembly and Cholesky
  // inverse on the host (FP64), inverse kept on the device for a GEMV solve
  {
    const int Nc = sizes[0], n = p + 1, npt = ipow(n, dim), ncell = ipow(Nc, dim);
    const int Mc = Nc * p + 1, mi = Mc - 2;
    const int nint = ipow(mi, dim);
    g->coarse_n = nint;
    double* dKe = nullptr;
    if ((s = dev_alloc(&dKe, (size_t)ncell * npt * npt * sizeof(double), nullptr)) < 0) return cleanup(s);
    CellArgs a{g->verts[0], g->mu[0], Nc, p, dim, g->tab64};
    std::vector<double> Ke((size_t)ncell * npt * npt);
    if ((e = launch_element_matrices(a, dKe, g->stream)) ||
        (e = hipMemcpyAsync(Ke.data(), dKe, Ke.size() * sizeof(double), hipMemcpyDeviceToHost, g->stream)) ||
        (e = hipStreamSynchronize(g->stream))) {
      (void)hipFree(dKe);
      return cleanup(fail(PMG_ERR_HIP, "coarse element matrices: %s", hipGetErrorString(e)));
    }
    (void)hipFree(dKe);
    std::vector<double> A((size_t)nint * nint, 0.0);
    std::vector<int> loc(npt);
    for (int c = 0; c < ncell; ++c) {
      const int ex = c % Nc, ey = (c / Nc) % Nc, ez = dim == 3 ? c / (Nc * Nc) : 0;
      for (int k = 0; k < npt; ++k) {
        const int ax = k % n, ay = (k / n) % n, az = dim == 3 ? k / (n * n) : 0;
        const int gx = ex * p + ax, gy = ey * p + ay, gz = ez * p + az;
        bool bd = gx == 0 || gx == Mc - 1 || gy == 0 || gy == Mc - 1;
        if (dim == 3) bd = bd || gz == 0 || gz == Mc - 1;
        loc[k] = bd ? -1 : (gx - 1) + (gy - 1) * mi + (dim == 3 ? (gz - 1) * mi * mi : 0);
      }
      for (int i = 0; i < npt; ++i) {
        if (loc[i] < 0) continue;
        for (int j = 0; j < npt; ++j)
          if (loc[j] >= 0) A[(size_t)loc[i] * nint + loc[j]] += Ke[((size_t)c * npt + i) * npt + j];
      }
    }
    if ((s = spd_inverse(A, nint)) < 0) return cleanup(s);
    if ((s = dev_alloc(&g->coarse_inv, A.size() * sizeof(double), nullptr)) < 0) return cleanup(s);
    for (int i = 0; i < 2; ++i)
      if ((s = dev_alloc(&g->cpack[i], (size_t)nint * sizeof(double), nullptr)) < 0) return cleanup(s);
    if ((e = hipMemcpy(g->coarse_inv, A.data(), A.size() * sizeof(double), hipMemcpyHostToDevice)))
      return cleanup(fail(PMG_ERR_HIP, "upload: %s", hipGetErrorString(e)));
  }
  *out = g;
  return PMG_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// exported functions
// ---------------------------------------------------------------------------

extern "C" {

int pmg_default_opts(pmg_opts* o) {
  if (!o) return fail(PMG_ERR_INVALID_ARG, "null opts");
  std::memset(o, 0, sizeof(*o));
  o->precision = PMG_FP64;
  o->n_levels = 0;
  o->cheb_degree = 3;
  o->n_vcycles = 1;
  o->bounds = PMG_BOUNDS_LANCZOS;
  o->lanczos_steps = 12;
  o->cheb_safety = 1.1;
  o->cheb_range = 15.0;
  o->seed = 0;
  o->stream = nullptr;
  o->patch_set = PMG_PATCH_INTERIOR;
  o->coarse_mean = PMG_COARSE_ARITHMETIC;
  return PMG_OK;
}

int pmg_patch_setup(const pmg_mesh* mesh, const double* coeff, int32_t p, const pmg_opts* opts,
                    pmg_handle** out) {
  return patch_setup_impl(mesh, coeff, p, opts, out);
}

int pmg_patch_smooth_colors(pmg_handle* h, double* u, const double* b, int32_t c_begin,
                            int32_t c_end) {
  if (!h || !u || !b) return fail(PMG_ERR_INVALID_ARG, "null argument");
  if (h->patch_geo) return fail(PMG_ERR_UNSUPPORTED, "independent patches have no global vector to smooth");
  if (h->smoother == PMG_SMOOTHER_CHEBYSHEV && !h->bounds_valid)
    return fail(PMG_ERR_INVALID_ARG, "Chebyshev bounds not set");
  if (c_begin < 0 || c_end > h->n_colors || c_begin > c_end)
    return fail(PMG_ERR_INVALID_ARG, "colour range [%d, %d) outside [0, %d)", c_begin, c_end, h->n_colors);
  return smooth_on(h, u, b, c_begin, c_end, 1, h->stream);
}

int pmg_patch_smooth(pmg_handle* h, double* u, const double* b, int32_t direction) {
  if (!h || !u || !b) return fail(PMG_ERR_INVALID_ARG, "null argument");
  if (direction != 1 && direction != -1) return fail(PMG_ERR_INVALID_ARG, "direction must be +1 or -1");
  if (direction > 0) return pmg_patch_smooth_colors(h, u, b, 0, h->n_colors);
  for (int c = h->n_colors - 1; c >= 0; --c) PMG_TRY(pmg_patch_smooth_colors(h, u, b, c, c + 1));
  return PMG_OK;
}

int pmg_patch_residual(pmg_handle* h, const double* u, const double* b, double* r) {
  if (!h || !u || !b || !r) return fail(PMG_ERR_INVALID_ARG, "null argument");
  if (h->patch_geo) return fail(PMG_ERR_UNSUPPORTED, "independent patches have no global vector");
  PatchArgs a = h->args();
  a.u = const_cast<double*>(u);
  a.b = b;
  a.out = r;
  if (!h->bounds_valid) {
    // the evaluate step reads no Chebyshev data; keep the kernel's loads valid
  }
  return launch_chunks(h, kModeResidual, a, 0, h->n_patches);
}

int pmg_patch_apply(pmg_handle* h, int32_t level, const double* x, double* y) {
  if (!h || !x || !y) return fail(PMG_ERR_INVALID_ARG, "null argument");
  if (level < 0 || level >= h->L) return fail(PMG_ERR_INVALID_ARG, "level %d outside 0..%d", level, h->L - 1);
  PatchArgs a = h->args();
  a.in = x;
  a.out = y;
  a.level = level;
  return launch_chunks(h, kModeApply, a, 0, h->n_patches);
}

int pmg_patch_local_solve(pmg_handle* h, const double* r, double* d) {
  if (!h || !r || !d) return fail(PMG_ERR_INVALID_ARG, "null argument");
  if (h->smoother != PMG_SMOOTHER_CHEBYSHEV)
    return fail(PMG_ERR_UNSUPPORTED, "the batched local solve runs the Chebyshev smoother only");
  if (!h->bounds_valid) return fail(PMG_ERR_INVALID_ARG, "Chebyshev bounds not set");
  PatchArgs a = h->args();
  a.in = r;
  a.out = d;
  return launch_chunks(h, kModeSolve, a, 0, h->n_patches);
}

namespace {

int pcg_checks(const pmg_handle* h, const double* b, double* x, double rtol, int32_t maxit,
               int32_t* iters, double* relres) {
  if (!h || !b || !x || !iters || !relres) return fail(PMG_ERR_INVALID_ARG, "null argument");
  const bool cart = h->smoother == PMG_SMOOTHER_CARTESIAN;
  if (!cart && !h->bounds_valid) return fail(PMG_ERR_INVALID_ARG, "Chebyshev bounds not set");
  if (!(rtol >= 0.0) || !std::isfinite(rtol)) return fail(PMG_ERR_INVALID_ARG, "rtol must be finite and >= 0");
  if (maxit < 0 || maxit > PMG_PCG_MAXIT_LIMIT)
    return fail(PMG_ERR_INVALID_ARG, "maxit %d outside 0..%d", maxit, PMG_PCG_MAXIT_LIMIT);
  if (h->precision != PMG_FP64) return fail(PMG_ERR_UNSUPPORTED, "patch CG runs on FP64 handles only");
  if (h->with_boundary)
    return fail(PMG_ERR_UNSUPPORTED, "patch CG is not available with boundary-vertex patches");
  return PMG_OK;
}

// the patch CG kernel with the residual and search directions in `work`
// (2 x top-level size per patch)
int pcg_launch(pmg_handle* h, const double* b, double* x, double rtol, int32_t maxit, int32_t* iters,
               double* relres, double* work) {
  PatchArgs a = h->args();
  a.in = b;
  a.out = x;
  a.pcg_rtol = rtol;
  a.pcg_maxit = maxit;
  a.pcg_work = work;
  a.pcg_iters = iters;
  a.pcg_relres = relres;
  a.fdm_tab = h->fdm_tab;
  a.fdm_omega = h->omega;
  a.grid = 0;
  a.map_mode = 0;
  return launch_chunks(h, h->smoother == PMG_SMOOTHER_CARTESIAN ? kModePcgCart : kModePcg, a, 0,
                       h->n_patches);
}

}  // namespace

int pmg_patch_pcg_noalloc(pmg_handle* h, const double* b, double* x, double rtol, int32_t maxit,
                          int32_t* iters, double* relres) {
  PMG_TRY(pcg_checks(h, b, x, rtol, maxit, iters, relres));
  const size_t need = (size_t)h->n_patches * 2 * h->level_size(0) * sizeof(double);
  if (need > PMG_PCG_SCRATCH_BYTES)
    return fail(PMG_ERR_INVALID_ARG, "patch CG work of %zu bytes (%d patches of %d unknowns) exceeds the "
                                     "%zu bytes of pmg_patch_pcg_noalloc", need, h->n_patches,
                h->level_size(0), (size_t)PMG_PCG_SCRATCH_BYTES);
  double* work = nullptr;
  size_t have = 0;
  HIP_TRY(pcg_scratch(&work, &have));
  if (need > have) return fail(PMG_ERR_INVALID_ARG, "patch CG work of %zu bytes exceeds %zu", need, have);
  return pcg_launch(h, b, x, rtol, maxit, iters, relres, work);
}

int pmg_patch_pcg(pmg_handle* h, const double* b, double* x, double rtol, int32_t maxit,
                  int32_t* iters, double* relres) {
  PMG_TRY(pcg_checks(h, b, x, rtol, maxit, iters, relres));
  if (!h->pcg_work) {
    int s = dev_alloc(&h->pcg_work, (size_t)h->n_patches * 2 * h->level_size(0) * sizeof(double),
                      &h->device_bytes);
    if (s < 0) return s;
  }
  return pcg_launch(h, b, x, rtol, maxit, iters, relres, h->pcg_work);
}

int pmg_patch_smooth_additive(pmg_handle* h, double* u, const double* b, double theta) {
  if (!h || !u || !b) return fail(PMG_ERR_INVALID_ARG, "null argument");
  if (!(theta > 0.0) || !std::isfinite(theta)) return fail(PMG_ERR_INVALID_ARG, "theta must be finite and > 0");
  if (h->patch_geo) return fail(PMG_ERR_UNSUPPORTED, "independent patches have no global vector to smooth");
  const int64_t n0 = h->level_size(0);
  if (!h->add_buf) PMG_TRY(dev_alloc(&h->add_buf, (size_t)2 * h->n_patches * n0 * sizeof(double), &h->device_bytes));
  double* r = h->add_buf;
  double* d = r + (size_t)h->n_patches * n0;
  // every local residual from the same u, every local solve, then the damped
  // corrections colour by colour (disjoint interiors: no atomics, one order)
  PMG_TRY(pmg_patch_residual(h, u, b, r));
  PMG_TRY(pmg_patch_local_solve(h, r, d));
  for (int c = 0; c < h->n_colors; ++c)
    HIP_TRY(launch_patch_scatter(h->dim, h->N, h->p, h->patch_vertex, h->color_off[c],
                                 h->color_off[c + 1] - h->color_off[c], d, theta, u, h->stream));
  return PMG_OK;
}

int pmg_set_smoother(pmg_handle* h, int32_t kind, double omega) {
  if (!h) return fail(PMG_ERR_INVALID_ARG, "null argument");
  if (kind == PMG_SMOOTHER_CHEBYSHEV) {
    h->smoother = kind;
    return PMG_OK;
  }
  if (kind != PMG_SMOOTHER_CARTESIAN) return fail(PMG_ERR_INVALID_ARG, "unknown smoother %d", kind);
  if (!(omega > 0.0) || !std::isfinite(omega)) return fail(PMG_ERR_INVALID_ARG, "omega must be finite and > 0");
  if (!h->fdm_tab) {
    // per smoothed level: the tables of a two-cell direction, then those of a
    // one-cell direction embedded at the low and at the high interior nodes
    // of the two-cell numbering (identity, lam = 1 and zero diagonals on the
    // other nodes, which are masked in a cut patch)
    std::vector<double> tab((size_t)kMaxLevels * kFdmStride, 0.0);
    for (int l = 0; l + 1 < h->L; ++l) {
      const int q = h->levels[l], m = 2 * q - 1;
      for (int type = 0; type < 3; ++type) {
        const FdmTables f = fdm_tables(q, type == 0 ? 2 : 1);
        const int off = type == 2 ? q : 0;  // first embedded node
        double* S = tab.data() + (size_t)l * kFdmStride + type * kFdmTypeStride;
        double* lam = S + m * m;
        double* dM = lam + m;
        double* dK = dM + m;
        for (int i = 0; i < m; ++i) {
          S[i * m + i] = 1.0;
          lam[i] = 1.0;
        }
        for (int i = 0; i < f.m; ++i) {
          for (int j = 0; j < f.m; ++j) S[(off + i) * m + off + j] = f.S[i * f.m + j];
          lam[off + i] = f.lam[i];
          dM[off + i] = f.dM[i];
          dK[off + i] = f.dK[i];
        }
      }
    }
    const size_t ts = h->tsize();
    int st = dev_alloc(&h->fdm_tab, tab.size() * ts, &h->device_bytes);
    if (st < 0) return st;
    hipError_t e;
    if (h->precision == PMG_FP64) {
      e = hipMemcpy(h->fdm_tab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice);
    } else {
      std::vector<float> t32(tab.begin(), tab.end());
      e = hipMemcpy(h->fdm_tab, t32.data(), t32.size() * sizeof(float), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) return fail(PMG_ERR_HIP, "smoother tables: %s", hipGetErrorString(e));
  }
  h->smoother = kind;
  h->omega = omega;
  return PMG_OK;
}

int pmg_get_inv_diag(const pmg_handle* h, int32_t level, double* out) {
  if (!h || !out) return fail(PMG_ERR_INVALID_ARG, "null argument");
  if (level < 0 || level >= h->L) return fail(PMG_ERR_INVALID_ARG, "level %d outside 0..%d", level, h->L - 1);
  HIP_TRY(hipMemcpyAsync(out, h->invdiag64[level], (size_t)h->n_patches * h->level_size(level) * sizeof(double),
                         hipMemcpyDeviceToDevice, h->stream));
  return PMG_OK;
}

int pmg_get_bounds(const pmg_handle* h, double* lam) {
  if (!h || !lam) return fail(PMG_ERR_INVALID_ARG, "null argument");
  std::copy(h->bounds.begin(), h->bounds.end(), lam);
  return PMG_OK;
}

int pmg_set_bounds(pmg_handle* h, const double* lam) {
  if (!h || !lam) return fail(PMG_ERR_INVALID_ARG, "null argument");
  std::vector<double> old = h->bounds;
  std::copy(lam, lam + h->bounds.size(), h->bounds.begin());
  int s = set_cheb(h);
  if (s < 0) h->bounds = old;
  return s;
}

int pmg_get_patch_vertices(const pmg_handle* h, int32_t* out) {
  if (!h || !out) return fail(PMG_ERR_INVALID_ARG, "null argument");
  if (h->patch_geo) {
    for (int j = 0; j < h->n_patches; ++j) out[j] = j;
    return PMG_OK;
  }
  HIP_TRY(hipMemcpy(out, h->patch_vertex, (size_t)h->n_patches * sizeof(int32_t), hipMemcpyDeviceToHost));
  return PMG_OK;
}

int pmg_query(const pmg_handle* h, int32_t what, int64_t* value) {
  if (!h || !value) return fail(PMG_ERR_INVALID_ARG, "null argument");
  const int64_t M = (int64_t)h->N * h->p + 1;
  switch (what) {
    case PMG_Q_N_PATCHES: *value = h->n_patches; return PMG_OK;
    case PMG_Q_N_COLORS: *value = h->n_colors; return PMG_OK;
    case PMG_Q_N_LEVELS: *value = h->L; return PMG_OK;
    case PMG_Q_N_DOFS: *value = h->dim == 3 ? M * M * M : M * M; return PMG_OK;
    case PMG_Q_N_INTERIOR_DOFS: *value = h->dim == 3 ? (M - 2) * (M - 2) * (M - 2) : (M - 2) * (M - 2); return PMG_OK;
    case PMG_Q_DEVICE_BYTES: *value = (int64_t)h->device_bytes; return PMG_OK;
    case PMG_Q_N_BOUNDARY_PATCHES: *value = h->n_trunc; return PMG_OK;
    case PMG_Q_LOCAL_DOFS: *value = h->local_dofs; return PMG_OK;
    case PMG_Q_TUNED_GRID: *value = h->tune_grid; return PMG_OK;
    case PMG_Q_TUNED_MAP: *value = h->tune_map; return PMG_OK;
    default: break;
  }
  if (what >= PMG_Q_COLOR_OFFSET && what <= PMG_Q_COLOR_OFFSET + h->n_colors) {
    *value = h->color_off[what - PMG_Q_COLOR_OFFSET];
    return PMG_OK;
  }
  if (what >= PMG_Q_LEVEL_DEGREE && what < PMG_Q_LEVEL_DEGREE + h->L) {
    *value = h->levels[what - PMG_Q_LEVEL_DEGREE];
    return PMG_OK;
  }
  if (what >= PMG_Q_LEVEL_SIZE && what < PMG_Q_LEVEL_SIZE + h->L) {
    *value = h->level_size(what - PMG_Q_LEVEL_SIZE);
    return PMG_OK;
  }
  return fail(PMG_ERR_INVALID_ARG, "unknown query %d", what);
}

int pmg_patch_destroy(pmg_handle* h) {
  if (!h) return PMG_OK;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  else (void)hipDeviceSynchronize();
  free_handle(h);
  return PMG_OK;
}

int gmg_setup(const pmg_mesh* mesh, const double* coeff, int32_t p, const pmg_opts* opts,
              gmg_handle** out) {
  return gmg_setup_impl(mesh, coeff, p, opts, out);
}

int gmg_apply(gmg_handle* g, const double* x, double* y) {
  if (!g || !x || !y) return fail(PMG_ERR_INVALID_ARG, "null argument");
  return global_apply(g, g->nlev - 1, x, y);
}

int gmg_vcycle(gmg_handle* g, const double* r, double* z) {
  if (!g || !r || !z) return fail(PMG_ERR_INVALID_ARG, "null argument");
  return vcycle(g, g->nlev - 1, r, z);
}

int gmg_cg_solve(gmg_handle* g, double* x, const double* b, double rtol, int32_t maxit, int32_t* iters,
                 double* relres) {
  if (!g || !x || !b) return fail(PMG_ERR_INVALID_ARG, "null argument");
  if (!(rtol > 0.0) || maxit < 1) return fail(PMG_ERR_INVALID_ARG, "need rtol > 0 and maxit >= 1");
  if (g->post_dir == 1 && !(g->add_theta > 0.0))
    return fail(PMG_ERR_UNSUPPORTED, "the V-cycle with the same sweep order before and after the coarse "
                                     "correction is not symmetric: use gmg_gmres_solve");
  const int lf = g->nlev - 1;
  const int64_t n = g->len(lf);
  hipStream_t s = g->stream;
  auto fetch = [&](int k) -> int {
    HIP_TRY(hipMemcpyAsync(g->hscal, g->scal, 8 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    (void)k;
    return PMG_OK;
  };
  // x = 0, r = b (Dirichlet entries of b are ignored)
  HIP_TRY(hipMemsetAsync(x, 0, n * sizeof(double), s));
  HIP_TRY(hipMemcpyAsync(g->r, b, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIP_TRY(launch_mask_dirichlet(g->dim, g->M(lf), g->r, s));
  PMG_TRY(dot(g, g->r, g->r, 0));
  PMG_TRY(vcycle(g, lf, g->r, g->z));
  HIP_TRY(hipMemcpyAsync(g->d, g->z, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  PMG_TRY(dot(g, g->r, g->z, 1));
  PMG_TRY(fetch(0));
  const double nb = std::sqrt(g->hscal[0]);
  double rz = g->hscal[1];
  if (nb == 0.0) {
    if (iters) *iters = 0;
    if (relres) *relres = 0.0;
    return PMG_OK;
  }
  double rel = 1.0;
  for (int k = 1; k <= maxit; ++k) {
    PMG_TRY(global_apply(g, lf, g->d, g->Ad));
    PMG_TRY(dot(g, g->d, g->Ad, 2));
    PMG_TRY(fetch(k));
    const double dAd = g->hscal[2];
    if (!(dAd > 0.0) || !std::isfinite(dAd)) {
      if (iters) *iters = k;
      if (relres) *relres = rel;
      return fail(PMG_ERR_BREAKDOWN, "CG breakdown at iteration %d: d^T A d = %g", k, dAd);
    }
    const double alpha = rz / dAd;
    HIP_TRY(launch_axpby(n, alpha, g->d, 1.0, x, s));
    HIP_TRY(launch_axpby(n, -alpha, g->Ad, 1.0, g->r, s));
    PMG_TRY(dot(g, g->r, g->r, 3));
    PMG_TRY(fetch(k));
    rel = std::sqrt(g->hscal[3]) / nb;
    if (rel <= rtol) {
      if (iters) *iters = k;
      if (relres) *relres = rel;
      return PMG_OK;
    }
    PMG_TRY(vcycle(g, lf, g->r, g->z));
    PMG_TRY(dot(g, g->r, g->z, 4));
    PMG_TRY(fetch(k));
    const double rz_new = g->hscal[4];
    HIP_TRY(launch_xpay_to(n, g->z, rz_new / rz, g->d, g->d, s));
    rz = rz_new;
  }
  if (iters) *iters = maxit + 1;
  if (relres) *relres = rel;
  g_last_error = "CG did not converge within maxit iterations";
  return PMG_WARN_NOT_CONVERGED;
}

int gmg_set_post_direction(gmg_handle* g, int32_t direction) {
  if (!g) return fail(PMG_ERR_INVALID_ARG, "null argument");
  if (direction != 1 && direction != -1) return fail(PMG_ERR_INVALID_ARG, "direction must be +1 or -1");
  g->post_dir = direction;
  return PMG_OK;
}

int gmg_set_additive(gmg_handle* g, double theta) {
  if (!g) return fail(PMG_ERR_INVALID_ARG, "null argument");
  if (!(theta >= 0.0) || !std::isfinite(theta)) return fail(PMG_ERR_INVALID_ARG, "theta must be finite and >= 0");
  g->add_theta = theta;
  return PMG_OK;
}

int gmg_gmres_solve(gmg_handle* g, double* x, const double* b, double rtol, int32_t maxit, int32_t* iters,
                    double* relres) {
  if (!g || !x || !b) return fail(PMG_ERR_INVALID_ARG, "null argument");
  if (!(rtol > 0.0) || !std::isfinite(rtol)) return fail(PMG_ERR_INVALID_ARG, "need a finite rtol > 0");
  if (maxit < 1 || maxit > PMG_GMRES_MAXIT_LIMIT)
    return fail(PMG_ERR_INVALID_ARG, "maxit %d outside 1..%d", maxit, PMG_GMRES_MAXIT_LIMIT);
  const int lf = g->nlev - 1;
  const int64_t n = g->len(lf);
  hipStream_t s = g->stream;
  // V_0 .. V_maxit (Arnoldi basis), then Z_0 .. Z_{maxit-1} (preconditioned)
  const size_t need = 2 * (size_t)maxit + 1;
  while (g->kv.size() < need) {
    double* p = nullptr;
    PMG_TRY(dev_alloc(&p, (size_t)n * sizeof(double), nullptr));
    g->kv.push_back(p);
  }
  auto V = [&](int i) { return g->kv[i]; };
  auto Z = [&](int i) { return g->kv[maxit + 1 + i]; };
  auto scalar = [&](const double* a, const double* c, double* out) -> int {
    PMG_TRY(dot(g, a, c, 0));
    HIP_TRY(hipMemcpyAsync(g->hscal, g->scal, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *out = g->hscal[0];
    return PMG_OK;
  };
  // x = 0; v_0 = b / ||b|| (Dirichlet entries of b are ignored)
  HIP_TRY(hipMemsetAsync(x, 0, n * sizeof(double), s));
  HIP_TRY(hipMemcpyAsync(V(0), b, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIP_TRY(launch_mask_dirichlet(g->dim, g->M(lf), V(0), s));
  double beta2 = 0;
  PMG_TRY(scalar(V(0), V(0), &beta2));
  const double beta = std::sqrt(beta2);
  if (beta == 0.0) {
    if (iters) *iters = 0;
    if (relres) *relres = 0.0;
    return PMG_OK;
  }
  HIP_TRY(launch_axpby(n, 0.0, V(0), 1.0 / beta, V(0), s));
  // Arnoldi with modified Gram-Schmidt on A M^{-1}, Givens rotations on the
  // Hessenberg matrix (Saad, Iterative Methods for Sparse Linear Systems,
  // Algorithm 9.6, flexible GMRES, no restart)
  std::vector<double> H((size_t)(maxit + 1) * maxit, 0.0), cs(maxit), sn(maxit), gv(maxit + 1, 0.0);
  auto h = [&](int i, int j) -> double& { return H[(size_t)i * maxit + j]; };
  gv[0] = beta;
  int k_done = maxit + 1;
  for (int j = 0; j < maxit; ++j) {
    PMG_TRY(vcycle(g, lf, V(j), Z(j)));
    PMG_TRY(global_apply(g, lf, Z(j), V(j + 1)));
    for (int i = 0; i <= j; ++i) {
      double hij = 0;
      PMG_TRY(scalar(V(j + 1), V(i), &hij));
      h(i, j) = hij;
      HIP_TRY(launch_axpby(n, -hij, V(i), 1.0, V(j + 1), s));
    }
    double hn2 = 0;
    PMG_TRY(scalar(V(j + 1), V(j + 1), &hn2));
    const double hn = std::sqrt(hn2);
    h(j + 1, j) = hn;
    if (hn != 0.0) HIP_TRY(launch_axpby(n, 0.0, V(j + 1), 1.0 / hn, V(j + 1), s));
    for (int i = 0; i < j; ++i) {
      const double hi = cs[i] * h(i, j) + sn[i] * h(i + 1, j);
      h(i + 1, j) = -sn[i] * h(i, j) + cs[i] * h(i + 1, j);
      h(i, j) = hi;
    }
    const double den = std::hypot(h(j, j), h(j + 1, j));
    if (!(den > 0.0) || !std::isfinite(den)) {
      if (iters) *iters = j + 1;
      return fail(PMG_ERR_BREAKDOWN, "GMRES breakdown at iteration %d", j + 1);
    }
    cs[j] = h(j, j) / den;
    sn[j] = h(j + 1, j) / den;
    h(j, j) = den;
    h(j + 1, j) = 0.0;
    gv[j + 1] = -sn[j] * gv[j];
    gv[j] = cs[j] * gv[j];
    if (std::fabs(gv[j + 1]) <= rtol * beta) {
      k_done = j + 1;
      break;
    }
  }
  // x = Z y with H y = g (upper triangular, the first k rows)
  const int k = std::min(k_done, (int)maxit);
  std::vector<double> y(k);
  for (int i = k - 1; i >= 0; --i) {
    double v = gv[i];
    for (int t = i + 1; t < k; ++t) v -= h(i, t) * y[t];
    y[i] = v / h(i, i);
  }
  for (int i = 0; i < k; ++i) HIP_TRY(launch_axpby(n, y[i], Z(i), 1.0, x, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (iters) *iters = k_done;
  if (relres) *relres = std::fabs(gv[k]) / beta;
  if (k_done > maxit) {
    g_last_error = "GMRES did not converge within maxit iterations";
    return PMG_WARN_NOT_CONVERGED;
  }
  return PMG_OK;
}

int gmg_query(const gmg_handle* g, int32_t what, int64_t* value) {
  if (!g || !value) return fail(PMG_ERR_INVALID_ARG, "null argument");
  if (what == 0) {
    *value = g->nlev;
    return PMG_OK;
  }
  if (what >= 16 && what < 16 + g->nlev) {
    *value = g->sizes[what - 16];
    return PMG_OK;
  }
  return fail(PMG_ERR_INVALID_ARG, "unknown query %d", what);
}

int gmg_level_smoother(gmg_handle* g, int32_t level, pmg_handle** h) {
  if (!g || !h) return fail(PMG_ERR_INVALID_ARG, "null argument");
  if (level < 1 || level >= g->nlev) return fail(PMG_ERR_INVALID_ARG, "level %d outside 1..%d", level, g->nlev - 1);
  *h = g->smoother[level];
  return PMG_OK;
}

int gmg_destroy(gmg_handle* g) {
  if (!g) return PMG_OK;
  if (g->stream) (void)hipStreamSynchronize(g->stream);
  else (void)hipDeviceSynchronize();
  free_gmg(g);
  return PMG_OK;
}


int pmg_patches_setup(int32_t dim, int64_t n, const double* verts, const double* coeff, int32_t p,
                      const pmg_opts* opts, pmg_handle** out) {
  return patches_setup_impl(dim, n, verts, coeff, p, opts, out);
}

int pmg_patch_features(pmg_handle* h, float* out) {
  if (!h || !out) return fail(PMG_ERR_INVALID_ARG, "null argument");
  PatchArgs a = h->args();
  a.patch_begin = 0;
  HIP_TRY(launch_features(h->dim, a, h->n_patches, out, h->stream));
  return PMG_OK;
}

int pmg_mlp_param_count(int32_t n_in, int32_t n_out, int64_t* count) {
  if (!count || n_in < 1 || n_out < 1) return fail(PMG_ERR_INVALID_ARG, "bad network size");
  *count = mlp_param_count(n_in, n_out);
  return PMG_OK;
}

int pmg_mlp_create(int32_t n_in, int32_t n_out, const float* params, int64_t max_batch, void* stream,
                   pmg_mlp** out) {
  if (!params || !out || n_in < 1 || n_out < 1 || max_batch < 1)
    return fail(PMG_ERR_INVALID_ARG, "bad network arguments");
  *out = nullptr;
  MlpNet* m = new MlpNet();
  m->n_in = n_in;
  m->n_out = n_out;
  m->stream = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = m->alloc(max_batch);
  const size_t P = (size_t)mlp_param_count(n_in, n_out);
  if (e == hipSuccess) e = hipMemcpy(m->theta, params, P * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(m->m, 0, P * 4);
  if (e == hipSuccess) e = hipMemset(m->v, 0, P * 4);
  if (e == hipSuccess) {
    std::vector<float> zero(n_in, 0.0f), one(n_in, 1.0f);
    e = hipMemcpy(m->mean, zero.data(), n_in * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->inv_std, one.data(), n_in * 4, hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    delete m;
    return fail(e == hipErrorOutOfMemory ? PMG_ERR_OOM : PMG_ERR_HIP, "network allocation: %s",
                hipGetErrorString(e));
  }
  *out = reinterpret_cast<pmg_mlp*>(m);
  return PMG_OK;
}

int pmg_mlp_get_params(const pmg_mlp* mm, float* params) {
  const MlpNet* m = reinterpret_cast<const MlpNet*>(mm);
  if (!m || !params) return fail(PMG_ERR_INVALID_ARG, "null argument");
  HIP_TRY(hipStreamSynchronize(m->stream));
  HIP_TRY(hipMemcpy(params, m->theta, (size_t)mlp_param_count(m->n_in, m->n_out) * 4, hipMemcpyDeviceToHost));
  return PMG_OK;
}

int pmg_mlp_set_params(pmg_mlp* mm, const float* params) {
  MlpNet* m = reinterpret_cast<MlpNet*>(mm);
  if (!m || !params) return fail(PMG_ERR_INVALID_ARG, "null argument");
  const size_t P = (size_t)mlp_param_count(m->n_in, m->n_out);
  HIP_TRY(hipStreamSynchronize(m->stream));
  HIP_TRY(hipMemcpy(m->theta, params, P * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemset(m->m, 0, P * 4));
  HIP_TRY(hipMemset(m->v, 0, P * 4));
  m->t = 0;
  return PMG_OK;
}

int pmg_mlp_fit_standardizer(pmg_mlp* mm, const float* X, int64_t n) {
  MlpNet* m = reinterpret_cast<MlpNet*>(mm);
  if (!m || !X || n < 1) return fail(PMG_ERR_INVALID_ARG, "bad arguments");
  HIP_TRY(m->fit_standardizer(X, n));
  return PMG_OK;
}

int pmg_mlp_get_standardizer(const pmg_mlp* mm, float* mean, float* inv_std) {
  const MlpNet* m = reinterpret_cast<const MlpNet*>(mm);
  if (!m || !mean || !inv_std) return fail(PMG_ERR_INVALID_ARG, "null argument");
  HIP_TRY(hipStreamSynchronize(m->stream));
  HIP_TRY(hipMemcpy(mean, m->mean, m->n_in * 4, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(inv_std, m->inv_std, m->n_in * 4, hipMemcpyDeviceToHost));
  return PMG_OK;
}

int pmg_mlp_set_standardizer(pmg_mlp* mm, const float* mean, const float* inv_std) {
  MlpNet* m = reinterpret_cast<MlpNet*>(mm);
  if (!m || !mean || !inv_std) return fail(PMG_ERR_INVALID_ARG, "null argument");
  HIP_TRY(hipStreamSynchronize(m->stream));
  HIP_TRY(hipMemcpy(m->mean, mean, m->n_in * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(m->inv_std, inv_std, m->n_in * 4, hipMemcpyHostToDevice));
  return PMG_OK;
}

int pmg_mlp_predict(pmg_mlp* mm, const float* X, int64_t n, float* Y) {
  MlpNet* m = reinterpret_cast<MlpNet*>(mm);
  if (!m || !X || !Y || n < 0) return fail(PMG_ERR_INVALID_ARG, "bad arguments");
  for (int64_t s = 0; s < n; s += m->cap) {
    const int B = (int)std::min<int64_t>(m->cap, n - s);
    HIP_TRY(m->standardize(X + s * m->n_in, B, m->xs));
    HIP_TRY(m->forward(m->xs, B));
    HIP_TRY(hipMemcpyAsync(Y + s * m->n_out, m->y, (size_t)B * m->n_out * 4, hipMemcpyDeviceToDevice,
                           m->stream));
  }
  return PMG_OK;
}

int pmg_mlp_gradient(pmg_mlp* mm, const float* X, const float* T, int64_t n, float* grad, double* loss) {
  MlpNet* m = reinterpret_cast<MlpNet*>(mm);
  if (!m || !X || !T || !grad || n < 1) return fail(PMG_ERR_INVALID_ARG, "bad arguments");
  if (n > m->cap) return fail(PMG_ERR_INVALID_ARG, "%lld rows exceed max_batch %lld", (long long)n, (long long)m->cap);
  HIP_TRY(hipMemsetAsync(m->loss, 0, sizeof(double), m->stream));
  HIP_TRY(m->standardize(X, n, m->xs));
  HIP_TRY(m->forward(m->xs, (int)n));
  HIP_TRY(m->backward(m->xs, T, (int)n));
  HIP_TRY(hipStreamSynchronize(m->stream));
  HIP_TRY(hipMemcpy(grad, m->grad, (size_t)mlp_param_count(m->n_in, m->n_out) * 4, hipMemcpyDeviceToHost));
  if (loss) HIP_TRY(hipMemcpy(loss, m->loss, sizeof(double), hipMemcpyDeviceToHost));
  return PMG_OK;
}

int pmg_mlp_train(pmg_mlp* mm, const float* X, const float* T, int64_t n, const int32_t* order,
                  int32_t epochs, int32_t batch, float lr, double* epoch_loss) {
  MlpNet* m = reinterpret_cast<MlpNet*>(mm);
  if (!m || !X || !T || !order || n < 1 || epochs < 1 || batch < 1 || !(lr > 0.0f))
    return fail(PMG_ERR_INVALID_ARG, "bad training arguments");
  if (batch > m->cap) return fail(PMG_ERR_INVALID_ARG, "batch %d exceeds max_batch %lld", batch, (long long)m->cap);
  for (int ep = 0; ep < epochs; ++ep) {
    HIP_TRY(hipMemsetAsync(m->loss, 0, sizeof(double), m->stream));
    int nbatch = 0;
    for (int64_t s = 0; s < n; s += batch, ++nbatch) {
      const int B = (int)std::min<int64_t>(batch, n - s);
      HIP_TRY(m->gather(X, T, order + (int64_t)ep * n + s, B));
      HIP_TRY(m->standardize(m->xb, B, m->xs));
      HIP_TRY(m->forward(m->xs, B));
      HIP_TRY(m->backward(m->xs, m->tb, B));
      HIP_TRY(m->adam_step(lr, 0.9f, 0.999f, 1e-8f));
    }
    if (epoch_loss) {
      double l = 0;
      HIP_TRY(hipMemcpyAsync(&l, m->loss, sizeof(double), hipMemcpyDeviceToHost, m->stream));
      HIP_TRY(hipStreamSynchronize(m->stream));
      epoch_loss[ep] = l / nbatch;
    }
  }
  HIP_TRY(hipStreamSynchronize(m->stream));
  return PMG_OK;
}

int pmg_mlp_destroy(pmg_mlp* mm) {
  MlpNet* m = reinterpret_cast<MlpNet*>(mm);
  if (!m) return PMG_OK;
  (void)hipStreamSynchronize(m->stream);
  delete m;
  return PMG_OK;
}

int pmg_mlp_save(const pmg_mlp* mm, double margin, const char* path) {
  const MlpNet* m = reinterpret_cast<const MlpNet*>(mm);
  if (!m || !path) return fail(PMG_ERR_INVALID_ARG, "null argument");
  const size_t P = (size_t)mlp_param_count(m->n_in, m->n_out);
  std::vector<float> theta(P), mean(m->n_in), inv(m->n_in);
  PMG_TRY(pmg_mlp_get_params(mm, theta.data()));
  PMG_TRY(pmg_mlp_get_standardizer(mm, mean.data(), inv.data()));
  FILE* f = std::fopen(path, "wb");
  if (!f) return fail(PMG_ERR_INVALID_ARG, "cannot open %s for writing", path);
  const char magic[8] = {'P', 'M', 'G', 'M', 'L', 'P', '1', 0};
  const int32_t dims[2] = {m->n_in, m->n_out};
  bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(dims, 4, 2, f) == 2 &&
            std::fwrite(&margin, 8, 1, f) == 1 && std::fwrite(theta.data(), 4, P, f) == P &&
            std::fwrite(mean.data(), 4, m->n_in, f) == (size_t)m->n_in &&
            std::fwrite(inv.data(), 4, m->n_in, f) == (size_t)m->n_in;
  ok = (std::fclose(f) == 0) && ok;
  return ok ? PMG_OK : fail(PMG_ERR_INVALID_ARG, "write to %s failed", path);
}

int pmg_mlp_load(const char* path, int64_t max_batch, void* stream, pmg_mlp** out, double* margin) {
  if (!path || !out) return fail(PMG_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(PMG_ERR_INVALID_ARG, "cannot open %s", path);
  char magic[8] = {0};
  int32_t dims[2] = {0, 0};
  double mg = 0;
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "PMGMLP1", 8) == 0 &&
            std::fread(dims, 4, 2, f) == 2 && dims[0] >= 1 && dims[0] <= 4096 && dims[1] >= 1 &&
            dims[1] <= 64 && std::fread(&mg, 8, 1, f) == 1;
  std::vector<float> theta, mean, inv;
  if (ok) {
    const size_t P = (size_t)mlp_param_count(dims[0], dims[1]);
    theta.resize(P);
    mean.resize(dims[0]);
    inv.resize(dims[0]);
    char extra;
    ok = std::fread(theta.data(), 4, P, f) == P && std::fread(mean.data(), 4, dims[0], f) == (size_t)dims[0] &&
         std::fread(inv.data(), 4, dims[0], f) == (size_t)dims[0] && std::fread(&extra, 1, 1, f) == 0;
  }
  std::fclose(f);
  if (!ok) return fail(PMG_ERR_INVALID_ARG, "%s is not a saved network (magic, sizes or length)", path);
  pmg_mlp* m = nullptr;
  PMG_TRY(pmg_mlp_create(dims[0], dims[1], theta.data(), max_batch, stream, &m));
  const int st = pmg_mlp_set_standardizer(m, mean.data(), inv.data());
  if (st < 0) {
    pmg_mlp_destroy(m);
    return st;
  }
  if (margin) *margin = mg;
  *out = m;
  return PMG_OK;
}

int pmg_set_bounds_mlp(pmg_handle* h, pmg_mlp* mm, double margin, double ood_z, int64_t* n_fallback) {
  MlpNet* m = reinterpret_cast<MlpNet*>(mm);
  if (!h || !m) return fail(PMG_ERR_INVALID_ARG, "null argument");
  const int nl = h->L - 1;
  if (m->n_in != n_features(h->dim) || m->n_out != 2 * nl)
    return fail(PMG_ERR_INVALID_ARG, "network has %d inputs and %d outputs, need %d and %d", m->n_in,
                m->n_out, n_features(h->dim), 2 * nl);
  if (!(margin >= 0.0) || !(ood_z > 0.0)) return fail(PMG_ERR_INVALID_ARG, "need margin >= 0 and ood_z > 0");
  const int n = h->n_patches, nf = n_features(h->dim);
  float *F = nullptr, *Y = nullptr, *Z = nullptr;
  int st;
  if ((st = dev_alloc(&F, (size_t)n * nf * 4, nullptr)) < 0) return st;
  if ((st = dev_alloc(&Y, (size_t)n * 2 * nl * 4, nullptr)) < 0 || (st = dev_alloc(&Z, (size_t)n * 4, nullptr)) < 0) {
    (void)hipFree(F);
    if (Y) (void)hipFree(Y);
    return st;
  }
  std::vector<float> hy((size_t)n * 2 * nl), hz(n);
  PatchArgs a = h->args();
  a.patch_begin = 0;
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e == hipSuccess) e = launch_features(h->dim, a, n, F, m->stream);
  if (e == hipSuccess) st = pmg_mlp_predict(mm, F, n, Y);
  if (e == hipSuccess && st == PMG_OK) e = m->max_abs_z(F, n, Z);
  if (e == hipSuccess && st == PMG_OK) e = hipMemcpyAsync(hy.data(), Y, hy.size() * 4, hipMemcpyDeviceToHost, m->stream);
  if (e == hipSuccess && st == PMG_OK) e = hipMemcpyAsync(hz.data(), Z, hz.size() * 4, hipMemcpyDeviceToHost, m->stream);
  if (e == hipSuccess && st == PMG_OK) e = hipStreamSynchronize(m->stream);
  (void)hipFree(F);
  (void)hipFree(Y);
  (void)hipFree(Z);
  if (st != PMG_OK) return st;
  if (e != hipSuccess) return fail(PMG_ERR_HIP, "learned bounds: %s", hipGetErrorString(e));
  std::vector<double> old = h->bounds;
  std::vector<int32_t> fallback;
  for (int j = 0; j < n; ++j) {
    // boundary-vertex patches are outside the training distribution: Lanczos
    bool ok = hz[j] <= ood_z && (h->trunc_host.empty() || h->trunc_host[j] < 0);
    for (int l = 0; l < nl && ok; ++l) {
      const double lo = std::exp((double)hy[(size_t)j * 2 * nl + 2 * l]);
      double hi = std::exp((double)hy[(size_t)j * 2 * nl + 2 * l + 1] + margin);
      ok = std::isfinite(lo) && std::isfinite(hi) && lo > 0.0;
      if (!ok) break;
      h->bounds[((size_t)j * nl + l) * 2] = std::min(lo, hi);
      h->bounds[((size_t)j * nl + l) * 2 + 1] = hi;
    }
    if (!ok) fallback.push_back(j);
  }
  if ((st = lanczos_for(h, fallback)) < 0 || (st = set_cheb(h)) < 0) {
    h->bounds = old;
    return st;
  }
  if (n_fallback) *n_fallback = (int64_t)fallback.size();
  return PMG_OK;
}

int pmg_mlp_fit_bounds(pmg_mlp* mm, const pmg_handle* h, const int32_t* train_order, int64_t n_train,
                       const int32_t* val_rows, int64_t n_val, int32_t epochs, int32_t batch, float lr,
                       double* epoch_loss, float* val_rmse, double* margin) {
  MlpNet* m = reinterpret_cast<MlpNet*>(mm);
  if (!m || !h || !train_order || !val_rows) return fail(PMG_ERR_INVALID_ARG, "null argument");
  if (n_train < 1 || n_val < 1 || epochs < 1) return fail(PMG_ERR_INVALID_ARG, "need n_train, n_val, epochs >= 1");
  if (!h->bounds_valid) return fail(PMG_ERR_INVALID_ARG, "the label handle has no bounds");
  const int nl = h->L - 1, n = h->n_patches, nf = n_features(h->dim), no = 2 * nl;
  if (m->n_in != nf || m->n_out != no)
    return fail(PMG_ERR_INVALID_ARG, "network has %d inputs and %d outputs, need %d and %d", m->n_in, m->n_out,
                nf, no);
  if (n_train > INT32_MAX || n_val > INT32_MAX) return fail(PMG_ERR_INVALID_ARG, "too many rows");
  // row numbers are indices into the handle's patches: check the host copies
  std::vector<int32_t> ord((size_t)epochs * n_train), vr(n_val);
  HIP_TRY(hipMemcpy(ord.data(), train_order, ord.size() * 4, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(vr.data(), val_rows, vr.size() * 4, hipMemcpyDeviceToHost));
  for (int32_t r : ord)
    if (r < 0 || r >= n) return fail(PMG_ERR_INVALID_ARG, "training row %d outside 0..%d", r, n - 1);
  for (int32_t r : vr)
    if (r < 0 || r >= n) return fail(PMG_ERR_INVALID_ARG, "validation row %d outside 0..%d", r, n - 1);
  // targets: ln lambda per smoothed level, from the handle's bounds
  std::vector<float> th((size_t)n * no);
  for (size_t i = 0; i < th.size(); ++i) {
    const double lam = h->bounds[i];
    if (!(lam > 0.0) || !std::isfinite(lam))
      return fail(PMG_ERR_INVALID_ARG, "bound %zu of the label handle is %g, not positive", i, lam);
    th[i] = (float)std::log(lam);
  }
  float *F = nullptr, *T = nullptr, *W = nullptr;
  const int64_t nw = std::max<int64_t>(n_train, n_val);
  int st;
  if ((st = dev_alloc(&F, (size_t)n * nf * 4, nullptr)) < 0) return st;
  if ((st = dev_alloc(&T, (size_t)n * no * 4, nullptr)) < 0 ||
      (st = dev_alloc(&W, (size_t)nw * (nf + 2 * no) * 4, nullptr)) < 0) {
    (void)hipFree(F);
    if (T) (void)hipFree(T);
    return st;
  }
  auto release = [&]() {
    (void)hipStreamSynchronize(m->stream);
    (void)hipFree(F);
    (void)hipFree(T);
    (void)hipFree(W);
  };
  PatchArgs a = h->args();
  a.patch_begin = 0;
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e == hipSuccess) e = launch_features(h->dim, a, n, F, m->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(T, th.data(), th.size() * 4, hipMemcpyHostToDevice, m->stream);
  // standardiser over the training rows (the first epoch lists each once)
  if (e == hipSuccess) e = m->gather_rows(F, train_order, (int)n_train, nf, W);
  if (e == hipSuccess) e = m->fit_standardizer(W, n_train);
  if (e != hipSuccess) {
    release();
    return fail(PMG_ERR_HIP, "bound network features: %s", hipGetErrorString(e));
  }
  st = pmg_mlp_train(mm, F, T, n_train, train_order, epochs, batch, lr, epoch_loss);
  if (st < 0) {
    release();
    return st;
  }
  // validation: predictions of the validation rows against their targets
  float* Xv = W;
  float* Tv = W + (size_t)n_val * nf;
  float* Yv = Tv + (size_t)n_val * no;
  std::vector<float> yh((size_t)n_val * no), tv((size_t)n_val * no);
  e = m->gather_rows(F, val_rows, (int)n_val, nf, Xv);
  if (e == hipSuccess) e = m->gather_rows(T, val_rows, (int)n_val, no, Tv);
  if (e == hipSuccess) st = pmg_mlp_predict(mm, Xv, n_val, Yv);
  if (e == hipSuccess && st == PMG_OK)
    e = hipMemcpyAsync(yh.data(), Yv, yh.size() * 4, hipMemcpyDeviceToHost, m->stream);
  if (e == hipSuccess && st == PMG_OK)
    e = hipMemcpyAsync(tv.data(), Tv, tv.size() * 4, hipMemcpyDeviceToHost, m->stream);
  release();
  if (st < 0) return st;
  if (e != hipSuccess) return fail(PMG_ERR_HIP, "bound network validation: %s", hipGetErrorString(e));
  double worst_max = 0.0;
  for (int k = 0; k < no; ++k) {
    double s = 0.0;
    for (int64_t i = 0; i < n_val; ++i) {
      const double d = (double)yh[(size_t)i * no + k] - (double)tv[(size_t)i * no + k];
      s += d * d;
    }
    const double rmse = std::sqrt(s / (double)n_val);
    if (val_rmse) val_rmse[k] = (float)rmse;
    if (k % 2 == 1) worst_max = std::max(worst_max, rmse);  // ln lambda_max outputs
  }
  if (margin) *margin = 3.0 * worst_max;
  return PMG_OK;
}

int pmg_autotune(pmg_handle* h, const double* u, const double* b, float* best_ms) {
  if (!h || !u || !b) return fail(PMG_ERR_INVALID_ARG, "null argument");
  if (h->patch_geo) return fail(PMG_ERR_UNSUPPORTED, "independent patches have no sweep to tune");
  if (!h->bounds_valid) return fail(PMG_ERR_INVALID_ARG, "Chebyshev bounds not set");
  int cands[kLaunchCandidates][2];
  PMG_TRY(launch_candidates(cands));
  // the largest colour, smoothed on a copy of u
  int cbig = 0;
  for (int c = 1; c < h->n_colors; ++c)
    if (h->color_off[c + 1] - h->color_off[c] > h->color_off[cbig + 1] - h->color_off[cbig]) cbig = c;
  const size_t n = n_dofs(h);
  double* w = nullptr;
  int st;
  if ((st = dev_alloc(&w, n * sizeof(double), nullptr)) < 0) return st;
  hipError_t e = hipMemcpyAsync(w, u, n * sizeof(double), hipMemcpyDeviceToDevice, h->stream);
  if (e) {
    (void)hipFree(w);
    return fail(PMG_ERR_HIP, "autotune: %s", hipGetErrorString(e));
  }
  float best_t[kLaunchCandidates];
  for (float& t : best_t) t = 1e30f;
  auto run = [&]() { return smooth_on(h, w, b, cbig, cbig + 1, 1, h->stream); };
  // warm-up at the default shape (clocks and caches), then two rounds over
  // the candidates, keeping each one's best time
  h->tune_grid = h->tune_map = 0;
  st = time_launches(h->stream, 20, run, nullptr);
  for (int round = 0; round < 2 && st == PMG_OK; ++round)
    for (int k = 0; k < kLaunchCandidates && st == PMG_OK; ++k) {
      h->tune_grid = cands[k][0];
      h->tune_map = cands[k][1];
      float ms = 0;
      if ((st = time_launches(h->stream, 1, run, nullptr)) == PMG_OK &&
          (st = time_launches(h->stream, 10, run, &ms)) == PMG_OK)
        best_t[k] = std::min(best_t[k], ms / 10);
    }
  (void)hipFree(w);
  if (st != PMG_OK) return st;
  int kb = 0;
  for (int k = 1; k < kLaunchCandidates; ++k)
    if (best_t[k] < best_t[kb]) kb = k;
  h->tune_grid = cands[kb][0];
  h->tune_map = cands[kb][1];
  if (best_ms) *best_ms = best_t[kb];
  return PMG_OK;
}

int pmg_set_launch(pmg_handle* h, int32_t grid, int32_t map_mode) {
  if (!h) return fail(PMG_ERR_INVALID_ARG, "null argument");
  if (grid < 0 || (map_mode != 0 && map_mode != 1))
    return fail(PMG_ERR_INVALID_ARG, "grid must be >= 0 and map_mode 0 or 1");
  h->tune_grid = grid;
  h->tune_map = map_mode;
  return PMG_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batches of independent instances (meshes of their own, mixed degrees):
// a sweep runs colour by colour, the instances of one colour concurrently on
// one stream each, joined before the next colour
// ---------------------------------------------------------------------------

struct pmg_batch {
  std::vector<pmg_handle*> inst;
  hipStream_t stream = nullptr;  // the caller's stream (opts.stream)
  std::vector<hipStream_t> side;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
  int max_colors = 0;
};

namespace {

void free_batch(pmg_batch* b) {
  if (!b) return;
  for (hipStream_t s : b->side)
    if (s) (void)hipStreamDestroy(s);
  for (hipEvent_t e : b->join)
    if (e) (void)hipEventDestroy(e);
  if (b->fork) (void)hipEventDestroy(b->fork);
  for (pmg_handle* h : b->inst) free_handle(h);
  delete b;
}

// enqueue one sweep of every instance: colour by colour, instances forked
// onto their side streams and joined back before the next colour
int enqueue_sweep(pmg_batch* b, double* const* u, const double* const* rhs, int direction,
                  hipStream_t main) {
  hipError_t e;
  int st = PMG_OK;
  for (int k = 0; k < b->max_colors && st == PMG_OK; ++k) {
    if ((e = hipEventRecord(b->fork, main))) return fail(PMG_ERR_HIP, "batch fork: %s", hipGetErrorString(e));
    for (size_t i = 0; i < b->inst.size(); ++i) {
      pmg_handle* h = b->inst[i];
      const int c = direction > 0 ? k : h->n_colors - 1 - k;
      if (c < 0 || c >= h->n_colors) continue;
      if ((e = hipStreamWaitEvent(b->side[i], b->fork, 0)))
        return fail(PMG_ERR_HIP, "batch wait: %s", hipGetErrorString(e));
      if (st == PMG_OK) st = smooth_on(h, u[i], rhs[i], c, c + 1, 1, b->side[i]);
      if ((e = hipEventRecord(b->join[i], b->side[i])) || (e = hipStreamWaitEvent(main, b->join[i], 0)))
        return fail(PMG_ERR_HIP, "batch join: %s", hipGetErrorString(e));
    }
  }
  return st;
}

}  // namespace

extern "C" {

int pmg_batch_setup(const pmg_mesh* meshes, const double* const* coeffs, const int32_t* p, int32_t n,
                    const pmg_opts* o, pmg_batch** out) {
  if (!meshes || !coeffs || !p || !o || !out || n < 1) return fail(PMG_ERR_INVALID_ARG, "null argument or n < 1");
  if (o->n_levels != 0)
    return fail(PMG_ERR_INVALID_ARG, "a batch of mixed degrees uses the default level lists (n_levels = 0)");
  *out = nullptr;
  pmg_batch* b = new pmg_batch();
  b->stream = reinterpret_cast<hipStream_t>(o->stream);
  hipError_t e;
  auto bail = [&](int st) {
    free_batch(b);
    return st;
  };
  for (int i = 0; i < n; ++i) {
    pmg_handle* h = nullptr;
    int st = patch_setup_impl(&meshes[i], coeffs[i], p[i], o, &h);
    if (st < 0) return bail(st);
    b->inst.push_back(h);
    b->max_colors = std::max(b->max_colors, h->n_colors);
    hipStream_t s = nullptr;
    hipEvent_t ev = nullptr;
    if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) ||
        (e = hipEventCreateWithFlags(&ev, hipEventDisableTiming))) {
      if (s) (void)hipStreamDestroy(s);
      return bail(fail(PMG_ERR_HIP, "batch streams: %s", hipGetErrorString(e)));
    }
    b->side.push_back(s);
    b->join.push_back(ev);
  }
  if ((e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming)))
    return bail(fail(PMG_ERR_HIP, "batch events: %s", hipGetErrorString(e)));
  // set the launch attributes of every kernel before the first sweep: smooth
  // each instance's first colour once on zero vectors
  for (pmg_handle* h : b->inst) {
    const int64_t M = (int64_t)h->N * h->p + 1;
    const size_t nd = (size_t)(h->dim == 3 ? M * M * M : M * M);
    double* z = nullptr;
    int st = dev_alloc(&z, 2 * nd * sizeof(double), nullptr);
    if (st < 0) return bail(st);
    if (!(e = hipMemsetAsync(z, 0, 2 * nd * sizeof(double), h->stream)) && h->bounds_valid)
      st = smooth_on(h, z, z + nd, 0, 1, 1, h->stream);
    if (!e) e = hipStreamSynchronize(h->stream);
    (void)hipFree(z);
    if (st < 0) return bail(st);
    if (e) return bail(fail(PMG_ERR_HIP, "batch warm-up: %s", hipGetErrorString(e)));
  }
  *out = b;
  return PMG_OK;
}

int pmg_batch_instance(pmg_batch* b, int32_t i, pmg_handle** h) {
  if (!b || !h || i < 0 || i >= (int)b->inst.size()) return fail(PMG_ERR_INVALID_ARG, "no instance %d", i);
  *h = b->inst[i];
  return PMG_OK;
}

int pmg_batch_smooth_eager(pmg_batch* b, double* const* u, const double* const* rhs, int32_t direction) {
  if (!b || !u || !rhs) return fail(PMG_ERR_INVALID_ARG, "null argument");
  if (direction != 1 && direction != -1) return fail(PMG_ERR_INVALID_ARG, "direction must be +1 or -1");
  for (size_t i = 0; i < b->inst.size(); ++i)
    if (!u[i] || !rhs[i] || !b->inst[i]->bounds_valid)
      return fail(PMG_ERR_INVALID_ARG, "instance %zu: null vector or bounds not set", i);
  return enqueue_sweep(b, u, rhs, direction, b->stream);
}

int pmg_batch_smooth(pmg_batch* b, double* const* u, const double* const* rhs, int32_t direction) {
  if (!b || !u || !rhs) return fail(PMG_ERR_INVALID_ARG, "null argument");
  if (direction != 1 && direction != -1) return fail(PMG_ERR_INVALID_ARG, "direction must be +1 or -1");
  // Switched off: capturing the batch sweep into a HIP graph and replaying
  // it ended in a host crash of unknown cause, as did the batch tuner's
  // graph timing before it; the capture code is taken out until a cause is
  // shown.
  return fail(PMG_ERR_UNSUPPORTED,
              "batch graph sweeps are switched off (a host crash of unknown cause while capturing and "
              "replaying them); use pmg_batch_smooth_eager");
}

int pmg_batch_autotune(pmg_batch* b, double* const* u, const double* const* rhs) {
  if (!b || !u || !rhs) return fail(PMG_ERR_INVALID_ARG, "null argument");
  // Switched off: timing whole-batch graphs of every candidate shape ended in
  // a host crash twice, the second time after the kernel attributes were set
  // at setup and the capture error paths were fixed; its cause is not known.
  return fail(PMG_ERR_UNSUPPORTED,
              "batch autotuning is switched off (a host crash of unknown cause while timing graph "
              "replays of tuned shapes); set shapes per instance with pmg_set_launch and sweep with "
              "pmg_batch_smooth_eager");
}

int pmg_batch_query(const pmg_batch* b, int32_t what, int64_t* value) {
  if (!b || !value) return fail(PMG_ERR_INVALID_ARG, "null argument");
  switch (what) {
    case PMG_BQ_N_INSTANCES: *value = (int64_t)b->inst.size(); return PMG_OK;
    case PMG_BQ_CAPTURES: *value = 0; return PMG_OK;  // graph sweeps are switched off
    case PMG_BQ_REPLAYS: *value = 0; return PMG_OK;
    default: return fail(PMG_ERR_INVALID_ARG, "unknown batch query %d", what);
  }
}

int pmg_batch_destroy(pmg_batch* b) {
  if (!b) return PMG_OK;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  else (void)hipDeviceSynchronize();
  free_batch(b);
  return PMG_OK;
}

const char* pmg_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
