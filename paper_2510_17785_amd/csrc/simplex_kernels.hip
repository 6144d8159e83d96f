// Kernels of the simplicial (unstructured) vertex patches of Section 3.2: 3
// quadrilaterals around one vertex in 2D, 4 hexahedra in 3D.  The cells are
// multilinear and carry the tensor-product degree-q basis, but the patch is
// not a tensor product: each cell is applied by sum factorisation on its own
// (q+1)^d nodes, and the cells meet the patch's unknowns through explicit
// gather maps (one per level, shared by all patches of a batch), so the
// transfers between degrees are cell-wise Kronecker products glued by the
// same maps instead of one patch-wide Kronecker product.
//
// One workgroup (256 threads, FP64) owns one patch: its vertices, the level
// vectors, the V-cycle and the CG iteration live in LDS and registers; the
// cells are processed one after another, so every sum into a shared unknown
// happens in the same order on every run.
//
// Cell operator (Section 2, bilinear form; Section 3.1, level operators):
//   A_c u = B^T G B u in sum-factorised form, the reference gradient at the
// Gauss points taken through the nodal derivative table E[k][a] = l_a'(xg_k)
// inside the interpolation chains (d/dx = Ex (x) By (x) Bz, and so on), and
// G = mu w adj(J) adj(J)^T / det J computed at each Gauss point from the
// cell's corners.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>
#include <set>
#include <tuple>

#include "internal.hpp"

namespace pmgi {
namespace {

constexpr int NTS = kSimplexThreads;

constexpr __host__ __device__ int spow(int b, int e) {
  int r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

template <int... Qs>
struct SLevels {
  static constexpr int count = sizeof...(Qs);
  static constexpr int q[kMaxLevels] = {Qs...};
};

// LDS layout (doubles) of one patch workgroup.
template <int DIM, class LV>
struct SLayout {
  static constexpr int L = LV::count;
  static constexpr int ncell = DIM + 1;
  static constexpr int nb = spow(2, DIM);
  static constexpr int size(int l) { return simplex_unknowns(DIM, LV::q[l]); }
  static constexpr int n0 = LV::q[0] + 1;
  static constexpr int cellN = spow(n0, DIM);
  static constexpr int geo_off = 0;                                    // ncell x nb x DIM corners
  static constexpr int mu_off = ncell * nb * DIM;                      // ncell coefficients
  static constexpr int vec_off = (mu_off + ncell + 3) / 4 * 4;
  static constexpr int vr(int l) {
    int o = vec_off;
    for (int i = 0; i < l; ++i) o += 3 * size(i);
    return o;
  }
  static constexpr int vd(int l) { return vr(l) + size(l); }
  static constexpr int vdinv(int l) { return vr(l) + 2 * size(l); }
  static constexpr int res_off = vr(L);
  static constexpr int z_off = res_off + size(0);
  static constexpr int out_off = z_off + size(0);
  static constexpr int u_off = (out_off + size(0) + 3) / 4 * 4;        // cell-local input
  static constexpr int co_off = u_off + cellN;                         // cell-local output
  static constexpr int w1_off = co_off + cellN;                        // 3 cellN
  static constexpr int w2_off = w1_off + 3 * cellN;                    // 3 cellN
  static constexpr int red_off = w2_off + 3 * cellN;                   // 8
  static constexpr int total = red_off + 8;
};

struct SCtx {
  double* lds;
  const SimplexArgs* a;
  int patch;
};

// metric G = scale adj(J) adj(J)^T / det J at reference point xi of the
// multilinear cell with corners X (nb x DIM, x fastest); 2D: (G00, G01, G11),
// 3D: (G00, G01, G02, G11, G12, G22)
template <int DIM>
__device__ void cell_metric(const double* X, const double* xi, double scale, double* G) {
  double J[DIM][DIM];
  for (int r = 0; r < DIM; ++r)
    for (int i = 0; i < DIM; ++i) J[r][i] = 0.0;
  for (int b = 0; b < spow(2, DIM); ++b) {
    for (int i = 0; i < DIM; ++i) {
      double dN = ((b >> i) & 1) ? 1.0 : -1.0;
      for (int j = 0; j < DIM; ++j)
        if (j != i) dN *= ((b >> j) & 1) ? xi[j] : 1.0 - xi[j];
      for (int r = 0; r < DIM; ++r) J[r][i] += X[b * DIM + r] * dN;
    }
  }
  if constexpr (DIM == 2) {
    const double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    // adj(J) = det J J^{-1}: rows reference, columns physical
    const double a00 = J[1][1], a01 = -J[0][1], a10 = -J[1][0], a11 = J[0][0];
    const double s = scale / det;
    G[0] = s * (a00 * a00 + a01 * a01);
    G[1] = s * (a00 * a10 + a01 * a11);
    G[2] = s * (a10 * a10 + a11 * a11);
  } else {
    double A[3][3];  // adj(J)[i][k] = cofactor of J[k][i]
    A[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    A[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
    A[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
    A[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    A[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
    A[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
    A[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    A[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
    A[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    const double det = J[0][0] * A[0][0] + J[0][1] * A[1][0] + J[0][2] * A[2][0];
    const double s = scale / det;
    int g = 0;
    for (int i = 0; i < 3; ++i)
      for (int j = i; j < 3; ++j) G[g++] = s * (A[i][0] * A[j][0] + A[i][1] * A[j][1] + A[i][2] * A[j][2]);
  }
}

// co = A_c u on the nodes of cell c at level L (all in LDS); ends with a barrier
template <int DIM, class LV, int L>
__device__ void cell_apply(const SCtx& s, int c, const double* u, double* co) {
  using Lay = SLayout<DIM, LV>;
  constexpr int Q = LV::q[L], n = Q + 1, N = spow(n, DIM);
  const double* tab = s.a->tab + L * kTabLevelStride;
  const double* B = tab;
  const double* E = tab + n * n;
  const double* xg = tab + 2 * n * n;
  const double* wg = xg + n;
  const double* X = s.lds + Lay::geo_off + c * Lay::nb * DIM;
  const double mu = s.lds[Lay::mu_off + c];
  double* w1 = s.lds + Lay::w1_off;
  double* w2 = s.lds + Lay::w2_off;
  const int tid = threadIdx.x;
  if constexpr (DIM == 2) {
    // X: rows (y) of the cell along x: A0 = B u, A1 = E u
    for (int y = tid; y < n; y += NTS) {
      double v[n];
      for (int a = 0; a < n; ++a) v[a] = u[y * n + a];
      for (int k = 0; k < n; ++k) {
        double s0 = 0, s1 = 0;
        for (int a = 0; a < n; ++a) {
          s0 = fma(B[k * n + a], v[a], s0);
          s1 = fma(E[k * n + a], v[a], s1);
        }
        w1[y * n + k] = s0;
        w1[N + y * n + k] = s1;
      }
    }
    __syncthreads();
    // Y: columns (xq): gradient, flux, transposed y contractions
    for (int xq = tid; xq < n; xq += NTS) {
      double v0[n], v1[n], fx[n], fy[n];
      for (int a = 0; a < n; ++a) {
        v0[a] = w1[a * n + xq];
        v1[a] = w1[N + a * n + xq];
      }
      for (int k = 0; k < n; ++k) {
        double gx = 0, gy = 0;
        for (int a = 0; a < n; ++a) {
          gx = fma(B[k * n + a], v1[a], gx);
          gy = fma(E[k * n + a], v0[a], gy);
        }
        const double xi[2] = {xg[xq], xg[k]};
        double G[3];
        cell_metric<2>(X, xi, mu * wg[xq] * wg[k], G);
        fx[k] = G[0] * gx + G[1] * gy;
        fy[k] = G[1] * gx + G[2] * gy;
      }
      for (int a = 0; a < n; ++a) {
        double wx = 0, wy = 0;
        for (int k = 0; k < n; ++k) {
          wx = fma(B[k * n + a], fx[k], wx);
          wy = fma(E[k * n + a], fy[k], wy);
        }
        w2[a * n + xq] = wx;
        w2[N + a * n + xq] = wy;
      }
    }
    __syncthreads();
    // XT: rows (y) along x
    for (int y = tid; y < n; y += NTS) {
      double wx[n], wy[n];
      for (int k = 0; k < n; ++k) {
        wx[k] = w2[y * n + k];
        wy[k] = w2[N + y * n + k];
      }
      for (int a = 0; a < n; ++a) {
        double acc = 0;
        for (int k = 0; k < n; ++k) {
          acc = fma(E[k * n + a], wx[k], acc);
          acc = fma(B[k * n + a], wy[k], acc);
        }
        co[y * n + a] = acc;
      }
    }
    __syncthreads();
  } else {
    constexpr int n2 = n * n;
    // X: line (y, z) along x
    for (int it = tid; it < n2; it += NTS) {
      double v[n];
      for (int a = 0; a < n; ++a) v[a] = u[it * n + a];
      for (int k = 0; k < n; ++k) {
        double s0 = 0, s1 = 0;
        for (int a = 0; a < n; ++a) {
          s0 = fma(B[k * n + a], v[a], s0);
          s1 = fma(E[k * n + a], v[a], s1);
        }
        w1[it * n + k] = s0;
        w1[N + it * n + k] = s1;
      }
    }
    __syncthreads();
    // Y: line (xq, z) along y
    for (int it = tid; it < n2; it += NTS) {
      const int xq = it % n, z = it / n;
      double v0[n], v1[n];
      for (int a = 0; a < n; ++a) {
        v0[a] = w1[(z * n + a) * n + xq];
        v1[a] = w1[N + (z * n + a) * n + xq];
      }
      for (int k = 0; k < n; ++k) {
        double s00 = 0, s01 = 0, s10 = 0;
        for (int a = 0; a < n; ++a) {
          s00 = fma(B[k * n + a], v0[a], s00);
          s01 = fma(E[k * n + a], v0[a], s01);
          s10 = fma(B[k * n + a], v1[a], s10);
        }
        const int o = (z * n + k) * n + xq;
        w2[o] = s00;
        w2[N + o] = s01;
        w2[2 * N + o] = s10;
      }
    }
    __syncthreads();
    // Z: line (xq, yq) along z: gradient, flux, transposed z contractions
    for (int it = tid; it < n2; it += NTS) {
      const int xq = it % n, yq = it / n;
      double u00[n], u01[n], u10[n], fx[n], fy[n], fz[n];
      for (int a = 0; a < n; ++a) {
        const int o = (a * n + yq) * n + xq;
        u00[a] = w2[o];
        u01[a] = w2[N + o];
        u10[a] = w2[2 * N + o];
      }
      for (int k = 0; k < n; ++k) {
        double gx = 0, gy = 0, gz = 0;
        for (int a = 0; a < n; ++a) {
          gx = fma(B[k * n + a], u10[a], gx);
          gy = fma(B[k * n + a], u01[a], gy);
          gz = fma(E[k * n + a], u00[a], gz);
        }
        const double xi[3] = {xg[xq], xg[yq], xg[k]};
        double G[6];
        cell_metric<3>(X, xi, mu * wg[xq] * wg[yq] * wg[k], G);
        fx[k] = G[0] * gx + G[1] * gy + G[2] * gz;
        fy[k] = G[1] * gx + G[3] * gy + G[4] * gz;
        fz[k] = G[2] * gx + G[4] * gy + G[5] * gz;
      }
      for (int a = 0; a < n; ++a) {
        double wx = 0, wy = 0, wz = 0;
        for (int k = 0; k < n; ++k) {
          wx = fma(B[k * n + a], fx[k], wx);
          wy = fma(B[k * n + a], fy[k], wy);
          wz = fma(E[k * n + a], fz[k], wz);
        }
        const int o = (a * n + yq) * n + xq;
        w1[o] = wx;
        w1[N + o] = wy;
        w1[2 * N + o] = wz;
      }
    }
    __syncthreads();
    // YT: line (xq, z) along y
    for (int it = tid; it < n2; it += NTS) {
      const int xq = it % n, z = it / n;
      double wx[n], wy[n], wz[n];
      for (int k = 0; k < n; ++k) {
        const int o = (z * n + k) * n + xq;
        wx[k] = w1[o];
        wy[k] = w1[N + o];
        wz[k] = w1[2 * N + o];
      }
      for (int a = 0; a < n; ++a) {
        double y0 = 0, y1 = 0;
        for (int k = 0; k < n; ++k) {
          y0 = fma(B[k * n + a], wx[k], y0);
          y1 = fma(E[k * n + a], wy[k], y1);
          y1 = fma(B[k * n + a], wz[k], y1);
        }
        const int o = (z * n + a) * n + xq;
        w2[o] = y0;
        w2[N + o] = y1;
      }
    }
    __syncthreads();
    // XT: line (y, z) along x
    for (int it = tid; it < n2; it += NTS) {
      double y0[n], y1[n];
      for (int k = 0; k < n; ++k) {
        y0[k] = w2[it * n + k];
        y1[k] = w2[N + it * n + k];
      }
      for (int a = 0; a < n; ++a) {
        double acc = 0;
        for (int k = 0; k < n; ++k) {
          acc = fma(E[k * n + a], y0[k], acc);
          acc = fma(B[k * n + a], y1[k], acc);
        }
        co[it * n + a] = acc;
      }
    }
    __syncthreads();
  }
}

// y = A_l v over the patch unknowns (v, y in LDS; epi(i, y_i) per row).
// Cells in order: every unknown's sum runs in the same order on every run.
template <int DIM, class LV, int L, class Epi>
__device__ void level_apply(const SCtx& s, const double* v, Epi epi) {
  using Lay = SLayout<DIM, LV>;
  constexpr int Q = LV::q[L], n = Q + 1, N = spow(n, DIM), NL = Lay::size(L);
  double* out = s.lds + Lay::out_off;
  double* u = s.lds + Lay::u_off;
  double* co = s.lds + Lay::co_off;
  const int32_t* gat = s.a->gat[L];
  const int tid = threadIdx.x;
  for (int i = tid; i < NL; i += NTS) out[i] = 0.0;
  for (int c = 0; c < Lay::ncell; ++c) {
    for (int a = tid; a < N; a += NTS) {
      const int g = gat[c * N + a];
      u[a] = g >= 0 ? v[g >> 1] : 0.0;
    }
    __syncthreads();
    cell_apply<DIM, LV, L>(s, c, u, co);
    for (int a = tid; a < N; a += NTS) {
      const int g = gat[c * N + a];
      if (g >= 0) out[g >> 1] += co[a];
    }
    __syncthreads();
  }
  for (int i = tid; i < NL; i += NTS) epi(i, out[i]);
  __syncthreads();
}

struct SEpiStore {
  double* y;
  __device__ void operator()(int i, double v) const { y[i] = v; }
};
struct SEpiResidual {
  const double* f;
  double* res;
  __device__ void operator()(int i, double v) const { res[i] = f[i] - v; }
};
struct SEpiChebStart {
  const double *f, *dinv;
  double *res, *z;
  double inv_theta;
  __device__ void operator()(int i, double v) const {
    const double r = f[i] - v;
    res[i] = r;
    z[i] = dinv[i] * r * inv_theta;
  }
};
struct SEpiChebStep {
  double *x, *res, *z;
  const double* dinv;
  double c1, c2;
  __device__ void operator()(int i, double v) const {
    const double zi = z[i];
    x[i] += zi;
    const double r = res[i] - v;
    res[i] = r;
    z[i] = c1 * zi + c2 * dinv[i] * r;
  }
};

// Chebyshev-accelerated Jacobi (Saad, Algorithm 12.1, D^{-1} on the
// residuals) on level L: degree k, interval [theta - delta, theta + delta];
// degree 1 on an interval with theta = 2 is the damped Jacobi step with
// omega = 1/2 of Section 3.2
template <int DIM, class LV, int L>
__device__ void schebyshev(const SCtx& s, bool x_zero) {
  using Lay = SLayout<DIM, LV>;
  constexpr int NL = Lay::size(L);
  double* f = s.lds + Lay::vr(L);
  double* x = s.lds + Lay::vd(L);
  const double* dinv = s.lds + Lay::vdinv(L);
  double* res = s.lds + Lay::res_off;
  double* z = s.lds + Lay::z_off;
  const double* ch = s.a->cheb + ((int64_t)s.patch * (LV::count - 1) + L) * 2;
  const double theta = ch[0], delta = ch[1];
  const double sigma = theta / delta;
  double rho = 1.0 / sigma;
  const int tid = threadIdx.x;
  if (x_zero) {
    for (int i = tid; i < NL; i += NTS) {
      res[i] = f[i];
      z[i] = dinv[i] * f[i] / theta;
      x[i] = 0.0;
    }
    __syncthreads();
  } else {
    level_apply<DIM, LV, L>(s, x, SEpiChebStart{f, dinv, res, z, 1.0 / theta});
  }
  for (int it = 0; it + 1 < s.a->cheb_degree; ++it) {
    const double rho_new = 1.0 / (2.0 * sigma - rho);
    level_apply<DIM, LV, L>(s, z, SEpiChebStep{x, res, z, dinv, rho_new * rho, 2.0 * rho_new / delta});
    rho = rho_new;
  }
  for (int i = tid; i < NL; i += NTS) x[i] += z[i];
  __syncthreads();
}

// cell-local tensor transfer of one direction, out[.., s, ..] = sum_t
// M[s][t] in[.., t, ..] (M: rows x cols, row-major) along direction dir of a
// tensor whose extents are ext[0..DIM)
template <int DIM>
__device__ void tensor_pass(const double* in, double* out, const double* M, int rows, int cols, int dir,
                            const int* ext_in) {
  int ext_out[3] = {ext_in[0], DIM > 1 ? ext_in[1] : 1, DIM > 2 ? ext_in[2] : 1};
  ext_out[dir] = rows;
  const int total = ext_out[0] * ext_out[1] * ext_out[2];
  int stride_in = 1;
  for (int i = 0; i < dir; ++i) stride_in *= ext_in[i];
  for (int o = threadIdx.x; o < total; o += NTS) {
    int idx[3] = {o % ext_out[0], (o / ext_out[0]) % ext_out[1], o / (ext_out[0] * ext_out[1])};
    const int srow = idx[dir];
    idx[dir] = 0;
    const int base = idx[0] + ext_in[0] * (idx[1] + (DIM > 1 ? ext_in[1] : 1) * idx[2]);
    double acc = 0;
    for (int t = 0; t < cols; ++t) acc = fma(M[srow * cols + t], in[base + t * stride_in], acc);
    out[o] = acc;
  }
}

// rc = P^T rf (restriction from level L to L+1): per cell, the fine unknowns
// the cell owns, contracted with the transposed 1D embedding per direction,
// added into the coarse unknowns; cells in order
template <int DIM, class LV, int L>
__device__ void srestrict(const SCtx& s, const double* rf, double* rc) {
  using Lay = SLayout<DIM, LV>;
  constexpr int qf = LV::q[L], qc = LV::q[L + 1], nf = qf + 1, nc = qc + 1;
  constexpr int Nf = spow(nf, DIM), Nc = spow(nc, DIM), NLc = Lay::size(L + 1);
  const double* P1 = s.a->tab + kMaxLevels * kTabLevelStride + L * kTabTransferStride;  // nf x nc
  double* t0 = s.lds + Lay::u_off;
  double* t1 = s.lds + Lay::w1_off;
  double* t2 = s.lds + Lay::w2_off;
  const int32_t* gf = s.a->gat[L];
  const int32_t* gc = s.a->gat[L + 1];
  const int tid = threadIdx.x;
  // P1^T as a (nc x nf) matrix, in the work area's tail
  double* PT = s.lds + Lay::co_off;
  for (int i = tid; i < nc * nf; i += NTS) PT[i] = P1[(i % nf) * nc + i / nf];
  for (int i = tid; i < NLc; i += NTS) rc[i] = 0.0;
  __syncthreads();
  for (int c = 0; c < Lay::ncell; ++c) {
    for (int a = tid; a < Nf; a += NTS) {
      const int g = gf[c * Nf + a];
      t0[a] = (g >= 0 && (g & 1)) ? rf[g >> 1] : 0.0;
    }
    __syncthreads();
    int ext[3] = {nf, DIM > 1 ? nf : 1, DIM > 2 ? nf : 1};
    const double* src = t0;
    double* bufs[2] = {t1, t2};
    for (int d = 0; d < DIM; ++d) {
      tensor_pass<DIM>(src, bufs[d & 1], PT, nc, nf, d, ext);
      ext[d] = nc;
      __syncthreads();
      src = bufs[d & 1];
    }
    for (int b = tid; b < Nc; b += NTS) {
      const int g = gc[c * Nc + b];
      if (g >= 0) rc[g >> 1] += src[b];
    }
    __syncthreads();
  }
}

// df += P dc (prolongation from level L+1 to L and correction): per cell,
// the coarse function's values at the fine nodes, written to the fine
// unknowns the cell owns
template <int DIM, class LV, int L>
__device__ void sprolong_add(const SCtx& s, const double* dc, double* df) {
  using Lay = SLayout<DIM, LV>;
  constexpr int qf = LV::q[L], qc = LV::q[L + 1], nf = qf + 1, nc = qc + 1;
  constexpr int Nf = spow(nf, DIM), Nc = spow(nc, DIM);
  const double* P1 = s.a->tab + kMaxLevels * kTabLevelStride + L * kTabTransferStride;  // nf x nc
  double* t0 = s.lds + Lay::u_off;
  double* t1 = s.lds + Lay::w1_off;
  double* t2 = s.lds + Lay::w2_off;
  const int32_t* gf = s.a->gat[L];
  const int32_t* gc = s.a->gat[L + 1];
  const int tid = threadIdx.x;
  for (int c = 0; c < Lay::ncell; ++c) {
    for (int b = tid; b < Nc; b += NTS) {
      const int g = gc[c * Nc + b];
      t0[b] = g >= 0 ? dc[g >> 1] : 0.0;
    }
    __syncthreads();
    int ext[3] = {nc, DIM > 1 ? nc : 1, DIM > 2 ? nc : 1};
    const double* src = t0;
    double* bufs[2] = {t1, t2};
    for (int d = 0; d < DIM; ++d) {
      tensor_pass<DIM>(src, bufs[d & 1], P1, nf, nc, d, ext);
      ext[d] = nf;
      __syncthreads();
      src = bufs[d & 1];
    }
    for (int a = tid; a < Nf; a += NTS) {
      const int g = gf[c * Nf + a];
      if (g >= 0 && (g & 1)) df[g >> 1] += src[a];
    }
    __syncthreads();
  }
}

// The V-cycle of Algorithm 2 from level L: Chebyshev pre-smoothing,
// residual, restriction, recursion, prolongation and correction,
// post-smoothing; the coarsest level (degree 1: the patch vertex alone) is
// solved exactly
template <int DIM, class LV, int L>
__device__ void svcycle(const SCtx& s, bool d_zero) {
  using Lay = SLayout<DIM, LV>;
  if constexpr (L == LV::count - 1) {
    static_assert(Lay::size(L) == 1, "the coarsest level holds the patch vertex alone");
    if (threadIdx.x == 0) s.lds[Lay::vd(L)] = s.lds[Lay::vdinv(L)] * s.lds[Lay::vr(L)];
    __syncthreads();
  } else {
    schebyshev<DIM, LV, L>(s, d_zero);
    double* res = s.lds + Lay::res_off;
    level_apply<DIM, LV, L>(s, s.lds + Lay::vd(L), SEpiResidual{s.lds + Lay::vr(L), res});
    srestrict<DIM, LV, L>(s, res, s.lds + Lay::vr(L + 1));
    svcycle<DIM, LV, L + 1>(s, true);
    sprolong_add<DIM, LV, L>(s, s.lds + Lay::vd(L + 1), s.lds + Lay::vd(L));
    schebyshev<DIM, LV, L>(s, false);
  }
}

__device__ double sblock_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = 0;
  for (int w = 0; w < NTS / 64; ++w) t += red[w];
  __syncthreads();
  return t;
}

// the patch's geometry and inverse diagonals into LDS
template <int DIM, class LV>
__device__ void sload(const SCtx& s, bool with_dinv) {
  using Lay = SLayout<DIM, LV>;
  const int tid = threadIdx.x;
  const double* geo = s.a->geo + (int64_t)s.patch * s.a->geo_stride;
  for (int i = tid; i < Lay::ncell * Lay::nb * DIM + Lay::ncell; i += NTS) s.lds[i] = geo[i];
  if (with_dinv) {
    for (int l = 0; l < LV::count; ++l) {
      const int NL = simplex_unknowns(DIM, LV::q[l]);
      const double* src = s.a->dinv[l] + (int64_t)s.patch * NL;
      for (int i = tid; i < NL; i += NTS) s.lds[Lay::vdinv(l) + i] = src[i];
    }
  }
  __syncthreads();
}

template <int DIM, class LV, int MODE>
__global__ __launch_bounds__(NTS) void simplex_kernel(SimplexArgs a) {
  using Lay = SLayout<DIM, LV>;
  extern __shared__ __align__(16) double slds[];
  SCtx s{slds, &a, a.patch_begin + (int)blockIdx.x};
  const int tid = threadIdx.x;
  if constexpr (MODE == kSimplexDiag) {
    // inverse diagonal of level a.level: sum over cells and Gauss points of
    // grad phi_a^T G grad phi_a, with the metric of every Gauss point of a
    // cell kept in the work area
    sload<DIM, LV>(s, false);
    auto run = [&](auto Lc) {
      constexpr int L = decltype(Lc)::value;
      constexpr int Q = LV::q[L], n = Q + 1, N = spow(n, DIM), NG = DIM == 3 ? 6 : 3;
      constexpr int NL = Lay::size(L);
      const double* tab = a.tab + L * kTabLevelStride;
      const double* B = tab;
      const double* E = tab + n * n;
      const double* xg = tab + 2 * n * n;
      const double* wg = xg + n;
      double* diag = slds + Lay::out_off;
      double* G = slds + Lay::w1_off;  // NG x N (fits the two work buffers)
      double* co = slds + Lay::co_off;
      for (int i = tid; i < NL; i += NTS) diag[i] = 0.0;
      for (int c = 0; c < Lay::ncell; ++c) {
        const double* X = slds + Lay::geo_off + c * Lay::nb * DIM;
        const double mu = slds[Lay::mu_off + c];
        for (int k = tid; k < N; k += NTS) {
          double xi[3], w = mu;
          for (int i = 0; i < DIM; ++i) {
            const int ki = (k / spow(n, i)) % n;
            xi[i] = xg[ki];
            w *= wg[ki];
          }
          double g[6];
          cell_metric<DIM>(X, xi, w, g);
          for (int j = 0; j < NG; ++j) G[j * N + k] = g[j];
        }
        __syncthreads();
        for (int b = tid; b < N; b += NTS) {
          int bi[3] = {b % n, DIM > 1 ? (b / n) % n : 0, DIM > 2 ? b / (n * n) : 0};
          double acc = 0;
          for (int k = 0; k < N; ++k) {
            int ki[3] = {k % n, DIM > 1 ? (k / n) % n : 0, DIM > 2 ? k / (n * n) : 0};
            double gr[3];
            for (int i = 0; i < DIM; ++i) {
              double v = 1.0;
              for (int j = 0; j < DIM; ++j) v *= (j == i ? E : B)[ki[j] * n + bi[j]];
              gr[i] = v;
            }
            if constexpr (DIM == 2) {
              acc += gr[0] * (G[k] * gr[0] + G[N + k] * gr[1]) + gr[1] * (G[N + k] * gr[0] + G[2 * N + k] * gr[1]);
            } else {
              const double f0 = G[k] * gr[0] + G[N + k] * gr[1] + G[2 * N + k] * gr[2];
              const double f1 = G[N + k] * gr[0] + G[3 * N + k] * gr[1] + G[4 * N + k] * gr[2];
              const double f2 = G[2 * N + k] * gr[0] + G[4 * N + k] * gr[1] + G[5 * N + k] * gr[2];
              acc += gr[0] * f0 + gr[1] * f1 + gr[2] * f2;
            }
          }
          co[b] = acc;
        }
        __syncthreads();
        const int32_t* gat = a.gat[L];
        for (int b = tid; b < N; b += NTS) {
          const int g = gat[c * N + b];
          if (g >= 0) diag[g >> 1] += co[b];
        }
        __syncthreads();
      }
      double* out = a.out + (int64_t)s.patch * NL;
      for (int i = tid; i < NL; i += NTS) out[i] = 1.0 / diag[i];
    };
    if (a.level == 0) run(std::integral_constant<int, 0>{});
    if constexpr (LV::count > 1)
      if (a.level == 1) run(std::integral_constant<int, 1>{});
    if constexpr (LV::count > 2)
      if (a.level == 2) run(std::integral_constant<int, 2>{});
    if constexpr (LV::count > 3)
      if (a.level == 3) run(std::integral_constant<int, 3>{});
    return;
  } else if constexpr (MODE == kSimplexApply) {
    sload<DIM, LV>(s, false);
    auto run = [&](auto Lc) {
      constexpr int L = decltype(Lc)::value;
      constexpr int NL = Lay::size(L);
      double* v = slds + Lay::z_off;
      const double* in = a.in + (int64_t)s.patch * NL;
      for (int i = tid; i < NL; i += NTS) v[i] = in[i];
      __syncthreads();
      level_apply<DIM, LV, L>(s, v, SEpiStore{a.out + (int64_t)s.patch * NL});
    };
    if (a.level == 0) run(std::integral_constant<int, 0>{});
    if constexpr (LV::count > 1)
      if (a.level == 1) run(std::integral_constant<int, 1>{});
    if constexpr (LV::count > 2)
      if (a.level == 2) run(std::integral_constant<int, 2>{});
    if constexpr (LV::count > 3)
      if (a.level == 3) run(std::integral_constant<int, 3>{});
    return;
  } else if constexpr (MODE == kSimplexSolve) {
    // N_MG V-cycles from zero on the given right-hand side
    sload<DIM, LV>(s, true);
    constexpr int N0 = Lay::size(0);
    const double* r = a.in + (int64_t)s.patch * N0;
    for (int i = tid; i < N0; i += NTS) slds[Lay::vr(0) + i] = r[i];
    __syncthreads();
    for (int it = 0; it < a.n_vcycles; ++it) svcycle<DIM, LV, 0>(s, it == 0);
    double* d = a.out + (int64_t)s.patch * N0;
    for (int i = tid; i < N0; i += NTS) d[i] = slds[Lay::vd(0) + i];
    return;
  } else {
    // CG on A_p x = b preconditioned by N_MG V-cycles (Section 3.2; Saad,
    // Algorithm 9.1); x, the residual and the direction in global memory,
    // one thread per row, exit tests on workgroup sums every thread holds
    sload<DIM, LV>(s, true);
    constexpr int N = Lay::size(0);
    double* red = slds + Lay::red_off;
    const double* b = a.in + (int64_t)s.patch * N;
    double* x = a.out + (int64_t)s.patch * N;
    double* r = a.work + (int64_t)s.patch * 2 * N;
    double* p = r + N;
    double* r0 = slds + Lay::vr(0);
    const double* d0 = slds + Lay::vd(0);
    double* v = slds + Lay::z_off;
    double* Ap = slds + Lay::res_off;
    auto precondition = [&]() {
      for (int it = 0; it < a.n_vcycles; ++it) svcycle<DIM, LV, 0>(s, it == 0);
    };
    double bb = 0;
    for (int i = tid; i < N; i += NTS) {
      const double bi = b[i];
      x[i] = 0.0;
      r[i] = bi;
      r0[i] = bi;
      bb += bi * bi;
    }
    bb = sblock_sum(bb, red);
    const double stop = a.rtol * a.rtol * bb;
    double rr = bb;
    int k = 0;
    if (bb > 0.0 && a.maxit > 0) {
      precondition();
      double rz = 0;
      for (int i = tid; i < N; i += NTS) {
        p[i] = d0[i];
        rz += r[i] * d0[i];
      }
      rz = sblock_sum(rz, red);
#pragma unroll 1
      for (;;) {
        for (int i = tid; i < N; i += NTS) v[i] = p[i];
        __syncthreads();
        level_apply<DIM, LV, 0>(s, v, SEpiStore{Ap});
        double pap = 0;
        for (int i = tid; i < N; i += NTS) pap += p[i] * Ap[i];
        pap = sblock_sum(pap, red);
        const double alpha = rz / pap;
        double rn = 0;
        for (int i = tid; i < N; i += NTS) {
          x[i] += alpha * p[i];
          const double ri = r[i] - alpha * Ap[i];
          r[i] = ri;
          r0[i] = ri;
          rn += ri * ri;
        }
        rr = sblock_sum(rn, red);
        ++k;
        if (rr <= stop || k >= a.maxit) break;
        precondition();
        double rzn = 0;
        for (int i = tid; i < N; i += NTS) rzn += r[i] * d0[i];
        rzn = sblock_sum(rzn, red);
        const double beta = rzn / rz;
        rz = rzn;
        for (int i = tid; i < N; i += NTS) p[i] = d0[i] + beta * p[i];
      }
    }
    if (tid == 0) {
      a.iters[s.patch] = k;
      a.relres[s.patch] = bb > 0.0 ? sqrt(rr / bb) : 0.0;
    }
  }
}

template <typename K>
hipError_t sallow_lds(K kernel, size_t bytes) {
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
  }
  return e;
}

template <int DIM, class LV>
struct SVariant {
  using Lay = SLayout<DIM, LV>;
  template <int MODE>
  static hipError_t go(const SimplexArgs& a, hipStream_t st) {
    const size_t lds = (size_t)Lay::total * sizeof(double);
    hipError_t e = sallow_lds(simplex_kernel<DIM, LV, MODE>, lds);
    if (e) return e;
    (void)hipGetLastError();
    hipLaunchKernelGGL((simplex_kernel<DIM, LV, MODE>), dim3(a.n_patch), dim3(NTS), lds, st, a);
    return hipGetLastError();
  }
  static hipError_t launch(int mode, const SimplexArgs& a, hipStream_t st) {
    if (a.n_patch <= 0) return hipSuccess;
    switch (mode) {
      case kSimplexDiag: return go<kSimplexDiag>(a, st);
      case kSimplexApply: return go<kSimplexApply>(a, st);
      case kSimplexSolve: return go<kSimplexSolve>(a, st);
      case kSimplexPcg: return go<kSimplexPcg>(a, st);
      default: return hipErrorInvalidValue;
    }
  }
  static hipError_t prime() {
    const size_t lds = (size_t)Lay::total * sizeof(double);
    hipError_t e = sallow_lds(simplex_kernel<DIM, LV, kSimplexDiag>, lds);
    if (!e) e = sallow_lds(simplex_kernel<DIM, LV, kSimplexApply>, lds);
    if (!e) e = sallow_lds(simplex_kernel<DIM, LV, kSimplexSolve>, lds);
    if (!e) e = sallow_lds(simplex_kernel<DIM, LV, kSimplexPcg>, lds);
    return e;
  }
};

template <int DIM, int... Qs>
SimplexVariant make_svariant() {
  using LV = SLevels<Qs...>;
  using V = SVariant<DIM, LV>;
  SimplexVariant v{};
  v.dim = DIM;
  v.n_levels = LV::count;
  const int q[] = {Qs...};
  for (int i = 0; i < kMaxLevels; ++i) v.levels[i] = i < LV::count ? q[i] : 0;
  v.launch = &V::launch;
  v.prime = &V::prime;
  v.lds_bytes = (size_t)SLayout<DIM, LV>::total * sizeof(double);
  v.cell_nodes = SLayout<DIM, LV>::cellN;
  return v;
}

}  // namespace

const SimplexVariant* find_simplex_variant(int dim, int n_levels, const int* levels) {
  static const SimplexVariant table[] = {
      make_svariant<2, 3, 1>(), make_svariant<2, 7, 3, 1>(), make_svariant<2, 15, 7, 3, 1>(),
      make_svariant<3, 3, 1>(), make_svariant<3, 7, 3, 1>()};
  for (const SimplexVariant& v : table) {
    if (v.dim != dim || v.n_levels != n_levels) continue;
    bool same = true;
    for (int l = 0; l < n_levels; ++l) same = same && v.levels[l] == levels[l];
    if (same) return &v;
  }
  return nullptr;
}

}  // namespace pmgi
