// Host side of the simplicial vertex patches (Section 3.2): numbering of the
// conforming unknowns, per-patch geometry, setup of the inverse diagonals and
// Chebyshev intervals, and the C ABI (pmg_simplex_*).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <map>
#include <vector>

#include "fe_tables.hpp"
#include "internal.hpp"

using namespace pmgi;

struct pmg_simplex {
  int dim = 0, p = 0, L = 0, n = 0;
  int levels[kMaxLevels] = {0};
  int sizes[kMaxLevels] = {0};
  int cheb_degree = 3, n_vcycles = 1;
  double safety = 1.1, range = 15.0;
  hipStream_t stream = nullptr;
  const SimplexVariant* var = nullptr;
  size_t device_bytes = 0;
  bool bounds_valid = false;
  int geo_stride = 0;
  double* geo = nullptr;
  int32_t* gat[kMaxLevels] = {nullptr};
  double* tab = nullptr;
  double* dinv[kMaxLevels] = {nullptr};
  double* cheb = nullptr;
  double* work = nullptr;
  std::vector<double> bounds;  // host, n x (L-1) x 2
  SimplexArgs args() const {
    SimplexArgs a{};
    a.n_patch = n;
    a.patch_begin = 0;
    a.geo = geo;
    a.geo_stride = geo_stride;
    for (int l = 0; l < kMaxLevels; ++l) {
      a.gat[l] = gat[l];
      a.dinv[l] = dinv[l];
    }
    a.tab = tab;
    a.cheb = cheb;
    a.cheb_degree = cheb_degree;
    a.n_vcycles = n_vcycles;
    return a;
  }
};

namespace {

int sfail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  return set_error(code, buf);
}

#define SHIP_TRY(expr)                                                                  \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return sfail(e_ == hipErrorOutOfMemory ? PMG_ERR_OOM : PMG_ERR_HIP, "%s: %s", #expr, \
                   hipGetErrorString(e_));                                              \
  } while (0)

template <typename P>
int salloc(pmg_simplex* s, P** ptr, size_t bytes) {
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, bytes ? bytes : 8);
  if (e != hipSuccess)
    return sfail(e == hipErrorOutOfMemory ? PMG_ERR_OOM : PMG_ERR_HIP, "hipMalloc(%zu): %s", bytes,
                 hipGetErrorString(e));
  *ptr = reinterpret_cast<P*>(q);
  s->device_bytes += bytes;
  return PMG_OK;
}

void free_simplex(pmg_simplex* s) {
  if (!s) return;
  void* ptrs[] = {s->geo, s->tab, s->cheb, s->work};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  for (int l = 0; l < kMaxLevels; ++l) {
    if (s->gat[l]) (void)hipFree(s->gat[l]);
    if (s->dinv[l]) (void)hipFree(s->dinv[l]);
  }
  delete s;
}

int ipow_(int b, int e) {
  int r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

// Numbering of the conforming unknowns at degree q from the cells' corner
// lists alone.  A cell node with local indices a lies on the sub-cell entity
// spanned by the directions where 0 < a_i < q, at the corners selected by
// a_i = q in the others; the entity is named by its vertices, and the node's
// position in it is measured from the entity's lowest-numbered vertex
// towards its neighbours in that entity in ascending vertex order, so two
// cells that share the entity name the node alike.  Nodes with a zero local
// index lie on the patch boundary (every cell's faces through its corner 0).
// Unknowns are numbered in order of first appearance (cells in order, nodes
// x fastest); the code of a cell node is 2 g + (this cell is the first
// holding g), -1 on the boundary.
std::vector<int32_t> numbering(int dim, const int32_t* cells, int q, int* count) {
  const int ncell = dim + 1, nb = ipow_(2, dim), nn = ipow_(q + 1, dim);
  std::vector<int32_t> code((size_t)ncell * nn, -1);
  std::map<std::vector<int64_t>, int> id;
  int next = 0;
  for (int c = 0; c < ncell; ++c) {
    const int32_t* cor = cells + (size_t)c * nb;
    for (int a = 0; a < nn; ++a) {
      int ai[3] = {0, 0, 0};
      for (int i = 0, t = a; i < dim; ++i, t /= (q + 1)) ai[i] = t % (q + 1);
      bool bdry = false;
      for (int i = 0; i < dim; ++i) bdry = bdry || ai[i] == 0;
      if (bdry) continue;
      std::vector<int> freed;
      int fixed_bits = 0;
      for (int i = 0; i < dim; ++i) {
        if (ai[i] == q) fixed_bits |= 1 << i;
        else freed.push_back(i);
      }
      std::vector<int64_t> key;
      if (freed.size() == (size_t)dim) {
        key = {-1, c, a};  // a cell interior node
      } else if (freed.empty()) {
        key = {0, cor[fixed_bits]};
      } else if (freed.size() == 1) {
        const int i = freed[0];
        const int v0 = cor[fixed_bits], v1 = cor[fixed_bits | (1 << i)];
        const int t = v0 < v1 ? ai[i] : q - ai[i];
        key = {1, std::min(v0, v1), std::max(v0, v1), t};
      } else {
        // a face (3D): the corners at the four bit patterns of directions i < j
        const int i = freed[0], j = freed[1];
        int best = -1, ob = 0;
        for (int bi = 0; bi < 2; ++bi)
          for (int bj = 0; bj < 2; ++bj) {
            const int v = cor[fixed_bits | (bi << i) | (bj << j)];
            if (best < 0 || v < best) {
              best = v;
              ob = (bi << i) | (bj << j);
            }
          }
        const int oi = (ob >> i) & 1, oj = (ob >> j) & 1;
        const int ni = cor[fixed_bits | ((1 - oi) << i) | (oj << j)];  // neighbour along i
        const int nj = cor[fixed_bits | (oi << i) | ((1 - oj) << j)];  // neighbour along j
        const int di = oi ? q - ai[i] : ai[i], dj = oj ? q - ai[j] : ai[j];
        std::vector<int64_t> vs = {cor[fixed_bits], cor[fixed_bits | (1 << i)], cor[fixed_bits | (1 << j)],
                                   cor[fixed_bits | (1 << i) | (1 << j)]};
        std::sort(vs.begin(), vs.end());
        key = {2, vs[0], vs[1], vs[2], vs[3]};
        if (ni < nj) {
          key.push_back(di);
          key.push_back(dj);
        } else {
          key.push_back(dj);
          key.push_back(di);
        }
      }
      auto it = id.find(key);
      if (it == id.end()) {
        id.emplace(key, next);
        code[(size_t)c * nn + a] = 2 * next + 1;
        ++next;
      } else {
        code[(size_t)c * nn + a] = 2 * it->second;
      }
    }
  }
  *count = next;
  return code;
}

// det J > 0 at the corners and the 2-point Gauss points of every cell
bool cells_untangled(int dim, const double* X, const int32_t* cells) {
  const int nb = ipow_(2, dim);
  const double g[2] = {0.5 - 0.5 / std::sqrt(3.0), 0.5 + 0.5 / std::sqrt(3.0)};
  for (int c = 0; c <= dim; ++c) {
    for (int pt = 0; pt < 2 * nb; ++pt) {
      double xi[3];
      for (int i = 0; i < dim; ++i) xi[i] = pt < nb ? (double)((pt >> i) & 1) : g[((pt - nb) >> i) & 1];
      double J[3][3] = {{0}};
      for (int b = 0; b < nb; ++b)
        for (int i = 0; i < dim; ++i) {
          double dN = ((b >> i) & 1) ? 1.0 : -1.0;
          for (int j = 0; j < dim; ++j)
            if (j != i) dN *= ((b >> j) & 1) ? xi[j] : 1.0 - xi[j];
          for (int r = 0; r < dim; ++r) J[r][i] += X[(size_t)cells[c * nb + b] * dim + r] * dN;
        }
      const double det = dim == 2 ? J[0][0] * J[1][1] - J[0][1] * J[1][0]
                                  : J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                                        J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                                        J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
      if (!(det > 0.0)) return false;
    }
  }
  return true;
}

int set_intervals(pmg_simplex* s) {
  const int nl = s->L - 1;
  std::vector<double> c64((size_t)s->n * nl * 2);
  for (int j = 0; j < s->n; ++j)
    for (int l = 0; l < nl; ++l) {
      const double lo = s->bounds[((size_t)j * nl + l) * 2], hi = s->bounds[((size_t)j * nl + l) * 2 + 1];
      if (!(lo > 0.0) || !(hi >= lo) || !std::isfinite(hi))
        return sfail(PMG_ERR_INVALID_ARG, "patch %d level %d: bad bounds (%g, %g)", j, l, lo, hi);
      // interval [a, b]: b = s lambda_max, a = max(lambda_min, b / rho)
      const double b = s->safety * hi;
      const double a = std::max(lo, b / s->range);
      c64[((size_t)j * nl + l) * 2] = 0.5 * (b + a);
      c64[((size_t)j * nl + l) * 2 + 1] = 0.5 * (b - a);
    }
  SHIP_TRY(hipMemcpy(s->cheb, c64.data(), c64.size() * sizeof(double), hipMemcpyHostToDevice));
  s->bounds_valid = true;
  return PMG_OK;
}

}  // namespace

extern "C" {

int pmg_simplex_numbering(int32_t dim, const int32_t* cells, int32_t q, int32_t* codes, int32_t* count) {
  if (!cells || !codes || !count) return sfail(PMG_ERR_INVALID_ARG, "null argument");
  if (dim != 2 && dim != 3) return sfail(PMG_ERR_INVALID_ARG, "dim must be 2 or 3");
  if (q < 1 || q > kMaxDegree) return sfail(PMG_ERR_INVALID_ARG, "degree %d outside 1..%d", q, kMaxDegree);
  const int nb = ipow_(2, dim), nv = dim == 2 ? 7 : 15;
  for (int i = 0; i < (dim + 1) * nb; ++i)
    if (cells[i] < 0 || cells[i] >= nv) return sfail(PMG_ERR_INVALID_ARG, "corner %d: vertex %d outside 0..%d", i, cells[i], nv - 1);
  int cnt = 0;
  std::vector<int32_t> code = numbering(dim, cells, q, &cnt);
  std::copy(code.begin(), code.end(), codes);
  *count = cnt;
  return PMG_OK;
}

int pmg_simplex_setup(int32_t dim, int64_t n, const double* verts, const int32_t* cells, const double* coeff,
                      int32_t p, const pmg_opts* o, pmg_simplex** out) {
  if (!verts || !cells || !coeff || !o || !out) return sfail(PMG_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  if (dim != 2 && dim != 3) return sfail(PMG_ERR_INVALID_ARG, "dim must be 2 or 3");
  if (n < 1 || n > (1 << 24)) return sfail(PMG_ERR_INVALID_ARG, "need 1 <= n <= 2^24 patches");
  if (o->precision != PMG_FP64)
    return sfail(PMG_ERR_UNSUPPORTED, "simplicial patches run in FP64 only");
  if (o->bounds != PMG_BOUNDS_FIXED)
    return sfail(PMG_ERR_UNSUPPORTED, "simplicial patches take their Chebyshev bounds from "
                                      "pmg_simplex_set_bounds (opts.bounds = PMG_BOUNDS_FIXED)");
  if (o->cheb_degree < 1 || o->cheb_degree > 16 || o->n_vcycles < 1 || o->n_vcycles > 100)
    return sfail(PMG_ERR_INVALID_ARG, "need 1 <= cheb_degree <= 16 and 1 <= n_vcycles <= 100");
  if (!(o->cheb_safety >= 1.0) || !(o->cheb_range > 1.0))
    return sfail(PMG_ERR_INVALID_ARG, "need cheb_safety >= 1 and cheb_range > 1");
  int levels[kMaxLevels] = {0}, L = 0;
  if (o->n_levels == 0) {
    // the paper's nested degrees: p, then the members of 1, 3, 7, 15 below it
    levels[L++] = p;
    for (int q : {15, 7, 3, 1})
      if (q < p && L < kMaxLevels) levels[L++] = q;
  } else {
    if (o->n_levels > kMaxLevels) return sfail(PMG_ERR_INVALID_ARG, "at most %d levels", kMaxLevels);
    L = o->n_levels;
    for (int l = 0; l < L; ++l) levels[l] = o->levels[l];
  }
  if (levels[0] != p || levels[L - 1] != 1)
    return sfail(PMG_ERR_INVALID_ARG, "the level list must start at p = %d and end at 1", p);
  const SimplexVariant* var = find_simplex_variant(dim, L, levels);
  if (!var)
    return sfail(PMG_ERR_UNSUPPORTED, "no simplicial kernel for dim %d, levels %d..1 (built: 2D 3,1 / "
                                      "7,3,1 / 15,7,3,1; 3D 3,1 / 7,3,1)", dim, p);
  const int nb = ipow_(2, dim), ncell = dim + 1, nv = dim == 2 ? 7 : 15;
  for (int c = 0; c < ncell; ++c)
    for (int b = 0; b < nb; ++b)
      if (cells[c * nb + b] < 0 || cells[c * nb + b] >= nv)
        return sfail(PMG_ERR_INVALID_ARG, "cell %d corner %d: vertex %d outside 0..%d", c, b, cells[c * nb + b],
                     nv - 1);
  for (int64_t j = 0; j < n; ++j) {
    for (int c = 0; c < ncell; ++c)
      if (!(coeff[j * ncell + c] > 0.0) || !std::isfinite(coeff[j * ncell + c]))
        return sfail(PMG_ERR_INVALID_ARG, "patch %lld cell %d: coefficient %g is not positive", (long long)j, c,
                     coeff[j * ncell + c]);
    if (!cells_untangled(dim, verts + j * nv * dim, cells))
      return sfail(PMG_ERR_DEGENERATE, "patch %lld: a cell with det J <= 0", (long long)j);
  }
  pmg_simplex* s = new pmg_simplex();
  auto bail = [&](int st) {
    free_simplex(s);
    return st;
  };
  s->dim = dim;
  s->p = p;
  s->L = L;
  s->n = (int)n;
  for (int l = 0; l < L; ++l) s->levels[l] = levels[l];
  s->cheb_degree = o->cheb_degree;
  s->n_vcycles = o->n_vcycles;
  s->safety = o->cheb_safety;
  s->range = o->cheb_range;
  s->stream = reinterpret_cast<hipStream_t>(o->stream);
  s->var = var;
  hipError_t e;
  if ((e = var->prime())) return bail(sfail(PMG_ERR_HIP, "simplex kernel attributes: %s", hipGetErrorString(e)));
  // numbering per level
  for (int l = 0; l < L; ++l) {
    int cnt = 0;
    std::vector<int32_t> code = numbering(dim, cells, levels[l], &cnt);
    if (cnt != simplex_unknowns(dim, levels[l]))
      return bail(sfail(PMG_ERR_INVALID_ARG, "the cells do not form a simplicial patch: %d unknowns at degree "
                                             "%d, expected %d", cnt, levels[l], simplex_unknowns(dim, levels[l])));
    s->sizes[l] = cnt;
    int st = salloc(s, &s->gat[l], code.size() * sizeof(int32_t));
    if (st < 0) return bail(st);
    if ((e = hipMemcpy(s->gat[l], code.data(), code.size() * sizeof(int32_t), hipMemcpyHostToDevice)))
      return bail(sfail(PMG_ERR_HIP, "upload: %s", hipGetErrorString(e)));
  }
  // geometry: per patch the cells' corners, then the coefficients
  s->geo_stride = ncell * nb * dim + ncell;
  {
    std::vector<double> g((size_t)n * s->geo_stride);
    for (int64_t j = 0; j < n; ++j) {
      double* dst = g.data() + j * s->geo_stride;
      for (int c = 0; c < ncell; ++c)
        for (int b = 0; b < nb; ++b)
          for (int r = 0; r < dim; ++r) dst[(c * nb + b) * dim + r] = verts[(j * nv + cells[c * nb + b]) * dim + r];
      for (int c = 0; c < ncell; ++c) dst[ncell * nb * dim + c] = coeff[j * ncell + c];
    }
    int st = salloc(s, &s->geo, g.size() * sizeof(double));
    if (st < 0) return bail(st);
    if ((e = hipMemcpy(s->geo, g.data(), g.size() * sizeof(double), hipMemcpyHostToDevice)))
      return bail(sfail(PMG_ERR_HIP, "upload: %s", hipGetErrorString(e)));
  }
  // 1D tables: per level B, E, Gauss points and weights; per transfer the
  // embedding P1[s][t] = l^{q'}_t(x^q_s) of the coarse degree's GLL basis at
  // the fine degree's GLL points
  {
    std::vector<double> tab((size_t)kTabSize, 0.0);
    for (int l = 0; l < L; ++l) {
      DegreeTables t = degree_tables(levels[l]);
      const int nq = t.n;
      double* dst = tab.data() + (size_t)l * kTabLevelStride;
      std::copy(t.B.begin(), t.B.end(), dst);
      std::copy(t.D.begin(), t.D.end(), dst + nq * nq);
      std::copy(t.xg.begin(), t.xg.end(), dst + 2 * nq * nq);
      std::copy(t.wg.begin(), t.wg.end(), dst + 2 * nq * nq + nq);
    }
    for (int l = 0; l + 1 < L; ++l) {
      std::vector<double> xf = gll_nodes(levels[l]), xc = gll_nodes(levels[l + 1]);
      const int nf = levels[l] + 1, nc = levels[l + 1] + 1;
      double* dst = tab.data() + (size_t)kMaxLevels * kTabLevelStride + (size_t)l * kTabTransferStride;
      for (int a = 0; a < nf; ++a)
        for (int b = 0; b < nc; ++b) dst[a * nc + b] = lagrange(xc, b, xf[a]);
    }
    int st = salloc(s, &s->tab, tab.size() * sizeof(double));
    if (st < 0) return bail(st);
    if ((e = hipMemcpy(s->tab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice)))
      return bail(sfail(PMG_ERR_HIP, "upload: %s", hipGetErrorString(e)));
  }
  // inverse diagonals of every level (FP64 setup kernel)
  for (int l = 0; l < L; ++l) {
    int st = salloc(s, &s->dinv[l], (size_t)n * s->sizes[l] * sizeof(double));
    if (st < 0) return bail(st);
  }
  for (int l = 0; l < L; ++l) {
    SimplexArgs a = s->args();
    a.level = l;
    a.out = s->dinv[l];
    if ((e = var->launch(kSimplexDiag, a, s->stream)))
      return bail(sfail(PMG_ERR_HIP, "simplex diagonal: %s", hipGetErrorString(e)));
  }
  int st = salloc(s, &s->cheb, (size_t)n * std::max(L - 1, 1) * 2 * sizeof(double));
  if (st < 0) return bail(st);
  st = salloc(s, &s->work, (size_t)n * 2 * s->sizes[0] * sizeof(double));
  if (st < 0) return bail(st);
  s->bounds.assign((size_t)n * (L - 1) * 2, 0.0);
  if ((e = hipStreamSynchronize(s->stream))) return bail(sfail(PMG_ERR_HIP, "simplex setup: %s", hipGetErrorString(e)));
  *out = s;
  return PMG_OK;
}

int pmg_simplex_query(const pmg_simplex* s, int32_t what, int64_t* value) {
  if (!s || !value) return sfail(PMG_ERR_INVALID_ARG, "null argument");
  switch (what) {
    case PMG_Q_N_PATCHES: *value = s->n; return PMG_OK;
    case PMG_Q_N_LEVELS: *value = s->L; return PMG_OK;
    case PMG_Q_DEVICE_BYTES: *value = (int64_t)s->device_bytes; return PMG_OK;
    default: break;
  }
  if (what >= PMG_Q_LEVEL_DEGREE && what < PMG_Q_LEVEL_DEGREE + s->L) {
    *value = s->levels[what - PMG_Q_LEVEL_DEGREE];
    return PMG_OK;
  }
  if (what >= PMG_Q_LEVEL_SIZE && what < PMG_Q_LEVEL_SIZE + s->L) {
    *value = s->sizes[what - PMG_Q_LEVEL_SIZE];
    return PMG_OK;
  }
  return sfail(PMG_ERR_INVALID_ARG, "unknown query %d", what);
}

int pmg_simplex_set_bounds(pmg_simplex* s, const double* lam) {
  if (!s || !lam) return sfail(PMG_ERR_INVALID_ARG, "null argument");
  std::vector<double> old = s->bounds;
  std::copy(lam, lam + s->bounds.size(), s->bounds.begin());
  const int st = set_intervals(s);
  if (st < 0) s->bounds = old;
  return st;
}

int pmg_simplex_get_inv_diag(const pmg_simplex* s, int32_t level, double* out) {
  if (!s || !out) return sfail(PMG_ERR_INVALID_ARG, "null argument");
  if (level < 0 || level >= s->L) return sfail(PMG_ERR_INVALID_ARG, "level %d outside 0..%d", level, s->L - 1);
  SHIP_TRY(hipMemcpyAsync(out, s->dinv[level], (size_t)s->n * s->sizes[level] * sizeof(double),
                          hipMemcpyDeviceToDevice, s->stream));
  return PMG_OK;
}

int pmg_simplex_apply(pmg_simplex* s, int32_t level, const double* x, double* y) {
  if (!s || !x || !y) return sfail(PMG_ERR_INVALID_ARG, "null argument");
  if (level < 0 || level >= s->L) return sfail(PMG_ERR_INVALID_ARG, "level %d outside 0..%d", level, s->L - 1);
  SimplexArgs a = s->args();
  a.level = level;
  a.in = x;
  a.out = y;
  SHIP_TRY(s->var->launch(kSimplexApply, a, s->stream));
  return PMG_OK;
}

int pmg_simplex_local_solve(pmg_simplex* s, const double* r, double* d) {
  if (!s || !r || !d) return sfail(PMG_ERR_INVALID_ARG, "null argument");
  if (!s->bounds_valid) return sfail(PMG_ERR_INVALID_ARG, "Chebyshev bounds not set");
  SimplexArgs a = s->args();
  a.in = r;
  a.out = d;
  SHIP_TRY(s->var->launch(kSimplexSolve, a, s->stream));
  return PMG_OK;
}

int pmg_simplex_pcg(pmg_simplex* s, const double* b, double* x, double rtol, int32_t maxit, int32_t* iters,
                    double* relres) {
  if (!s || !b || !x || !iters || !relres) return sfail(PMG_ERR_INVALID_ARG, "null argument");
  if (!s->bounds_valid) return sfail(PMG_ERR_INVALID_ARG, "Chebyshev bounds not set");
  if (!(rtol >= 0.0) || !std::isfinite(rtol)) return sfail(PMG_ERR_INVALID_ARG, "rtol must be finite and >= 0");
  if (maxit < 0 || maxit > PMG_PCG_MAXIT_LIMIT)
    return sfail(PMG_ERR_INVALID_ARG, "maxit %d outside 0..%d", maxit, PMG_PCG_MAXIT_LIMIT);
  SimplexArgs a = s->args();
  a.in = b;
  a.out = x;
  a.rtol = rtol;
  a.maxit = maxit;
  a.work = s->work;
  a.iters = iters;
  a.relres = relres;
  SHIP_TRY(s->var->launch(kSimplexPcg, a, s->stream));
  return PMG_OK;
}

int pmg_simplex_destroy(pmg_simplex* s) {
  if (!s) return PMG_OK;
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  else (void)hipDeviceSynchronize();
  free_simplex(s);
  return PMG_OK;
}

}  // extern "C"
