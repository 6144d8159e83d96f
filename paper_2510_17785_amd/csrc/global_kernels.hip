// FP64 kernels of the outer geometric multigrid and CG (Section 2, Section 4):
// the cell-wise matrix-free operator A_l, the h-transfers, vector updates,
// deterministic dot products and the dense coarse-level solve.
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace pmgi {
namespace {

constexpr int kCellThreads = 256;

// Geometry of one multilinear cell at reference point (x, y, z):
// G = scale * adj(J) adj(J)^T / det J.  C holds the 2^dim corners, corner
// c = sum_i b_i 2^i at C[c*dim + r].
__device__ __forceinline__ void cell_metric3(const double* C, double x, double y, double z,
                                             double scale, double* G) {
  double J[3][3];
  for (int r = 0; r < 3; ++r) {
    for (int s = 0; s < 3; ++s) J[r][s] = 0;
    for (int c = 0; c < 8; ++c) {
      const int bx = c & 1, by = (c >> 1) & 1, bz = (c >> 2) & 1;
      const double lx = bx ? x : 1 - x, ly = by ? y : 1 - y, lz = bz ? z : 1 - z;
      const double sx = bx ? 1 : -1, sy = by ? 1 : -1, sz = bz ? 1 : -1;
      const double v = C[c * 3 + r];
      J[r][0] += v * sx * ly * lz;
      J[r][1] += v * lx * sy * lz;
      J[r][2] += v * lx * ly * sz;
    }
  }
  double a[3][3];
  a[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  a[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
  a[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
  a[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  a[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
  a[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
  a[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  a[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
  a[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  const double det = J[0][0] * a[0][0] + J[0][1] * a[1][0] + J[0][2] * a[2][0];
  const double s = scale / det;
  G[0] = s * (a[0][0] * a[0][0] + a[0][1] * a[0][1] + a[0][2] * a[0][2]);
  G[1] = s * (a[0][0] * a[1][0] + a[0][1] * a[1][1] + a[0][2] * a[1][2]);
  G[2] = s * (a[0][0] * a[2][0] + a[0][1] * a[2][1] + a[0][2] * a[2][2]);
  G[3] = s * (a[1][0] * a[1][0] + a[1][1] * a[1][1] + a[1][2] * a[1][2]);
  G[4] = s * (a[1][0] * a[2][0] + a[1][1] * a[2][1] + a[1][2] * a[2][2]);
  G[5] = s * (a[2][0] * a[2][0] + a[2][1] * a[2][1] + a[2][2] * a[2][2]);
}

__device__ __forceinline__ void cell_metric2(const double* C, double x, double y, double scale,
                                             double* G) {
  double J[2][2] = {{0, 0}, {0, 0}};
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 4; ++c) {
      const int bx = c & 1, by = (c >> 1) & 1;
      const double lx = bx ? x : 1 - x, ly = by ? y : 1 - y;
      const double v = C[c * 2 + r];
      J[r][0] += v * (bx ? 1 : -1) * ly;
      J[r][1] += v * lx * (by ? 1 : -1);
    }
  const double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  const double s = scale / det;
  G[0] = s * (J[1][1] * J[1][1] + J[0][1] * J[0][1]);
  G[1] = -s * (J[1][1] * J[1][0] + J[0][1] * J[0][0]);
  G[2] = s * (J[1][0] * J[1][0] + J[0][0] * J[0][0]);
}

__device__ void load_cell(const CellArgs& a, int cell, double* C, double* mu) {
  const int N = a.N, N1 = N + 1, dim = a.dim;
  const int ex = cell % N, ey = (cell / N) % N, ez = dim == 3 ? cell / (N * N) : 0;
  const int tid = threadIdx.x;
  for (int i = tid; i < (1 << dim) * dim; i += blockDim.x) {
    const int c = i / dim, r = i % dim;
    const int bx = c & 1, by = (c >> 1) & 1, bz = (c >> 2) & 1;
    int g = (ex + bx) + (ey + by) * N1;
    if (dim == 3) g += (ez + bz) * N1 * N1;
    C[i] = a.verts[g * dim + r];
  }
  if (tid == 0) *mu = a.mu[cell];
}

// cellbuf[cell][a] = (A^K x_K)_a for every cell K, by sum factorisation with
// the collocation derivative at the Gauss points (degree p, p+1 points).
__global__ __launch_bounds__(kCellThreads) void cell_apply_kernel(CellArgs a, const double* x,
                                                                  double* cellbuf) {
  extern __shared__ __align__(16) double sm[];
  const int p = a.p, n = p + 1, dim = a.dim;
  const int npt = dim == 3 ? n * n * n : n * n;
  const double* B = a.tab64;
  const double* Dc = a.tab64 + n * n;
  const double* xg = a.tab64 + 3 * n * n;
  const double* wg = xg + n;
  double* u = sm;              // npt
  double* t0 = u + npt;        // npt
  double* t1 = t0 + npt;       // npt
  double* f0 = t1 + npt;       // 3 * npt
  double* f1 = f0 + npt;
  double* f2 = f1 + npt;
  double* C = f2 + npt;        // 24
  double* mu = C + 24;
  const int cell = blockIdx.x;
  const int tid = threadIdx.x;
  const int N = a.N, M = N * p + 1;
  load_cell(a, cell, C, mu);
  const int ex = cell % N, ey = (cell / N) % N, ez = dim == 3 ? cell / (N * N) : 0;
  for (int i = tid; i < npt; i += blockDim.x) {
    const int ix = i % n, iy = (i / n) % n, iz = dim == 3 ? i / (n * n) : 0;
    const int gx = ex * p + ix, gy = ey * p + iy, gz = ez * p + iz;
    bool bd = gx == 0 || gx == M - 1 || gy == 0 || gy == M - 1;
    if (dim == 3) bd = bd || gz == 0 || gz == M - 1;
    int64_t g = gx + (int64_t)gy * M;
    if (dim == 3) g += (int64_t)gz * M * M;
    u[i] = bd ? 0.0 : x[g];
  }
  __syncthreads();
  // values at the Gauss points: contract x, then y, then z with B
  for (int i = tid; i < npt; i += blockDim.x) {
    const int kx = i % n, r = i / n;
    double s = 0;
    for (int q = 0; q < n; ++q) s += B[kx * n + q] * u[r * n + q];
    t0[i] = s;
  }
  __syncthreads();
  for (int i = tid; i < npt; i += blockDim.x) {
    const int ix = i % n, ky = (i / n) % n, r = i / (n * n);
    double s = 0;
    for (int q = 0; q < n; ++q) s += B[ky * n + q] * t0[(r * n + q) * n + ix];
    t1[i] = s;
  }
  __syncthreads();
  double* val = t1;
  if (dim == 3) {
    for (int i = tid; i < npt; i += blockDim.x) {
      const int kz = i / (n * n), rem = i % (n * n);
      double s = 0;
      for (int q = 0; q < n; ++q) s += B[kz * n + q] * t1[q * n * n + rem];
      t0[i] = s;
    }
    __syncthreads();
    val = t0;
  }
  for (int i = tid; i < npt; i += blockDim.x) {
    const int kx = i % n, ky = (i / n) % n, kz = dim == 3 ? i / (n * n) : 0;
    double g0 = 0, g1 = 0, g2 = 0;
    for (int q = 0; q < n; ++q) {
      g0 += Dc[kx * n + q] * val[i - kx + q];
      g1 += Dc[ky * n + q] * val[i + (q - ky) * n];
      if (dim == 3) g2 += Dc[kz * n + q] * val[i + (q - kz) * n * n];
    }
    if (dim == 3) {
      double G[6];
      cell_metric3(C, xg[kx], xg[ky], xg[kz], *mu * wg[kx] * wg[ky] * wg[kz], G);
      f0[i] = G[0] * g0 + G[1] * g1 + G[2] * g2;
      f1[i] = G[1] * g0 + G[3] * g1 + G[4] * g2;
      f2[i] = G[2] * g0 + G[4] * g1 + G[5] * g2;
    } else {
      double G[3];
      cell_metric2(C, xg[kx], xg[ky], *mu * wg[kx] * wg[ky], G);
      f0[i] = G[0] * g0 + G[1] * g1;
      f1[i] = G[1] * g0 + G[2] * g1;
    }
  }
  __syncthreads();
  double* w = (dim == 3) ? t1 : t0;
  for (int i = tid; i < npt; i += blockDim.x) {
    const int kx = i % n, ky = (i / n) % n, kz = dim == 3 ? i / (n * n) : 0;
    double s = 0;
    for (int q = 0; q < n; ++q) {
      s += Dc[q * n + kx] * f0[i - kx + q];
      s += Dc[q * n + ky] * f1[i + (q - ky) * n];
      if (dim == 3) s += Dc[q * n + kz] * f2[i + (q - kz) * n * n];
    }
    w[i] = s;
  }
  __syncthreads();
  // transposed interpolation back to the nodes
  double* src = w;
  double* tmp = (dim == 3) ? t0 : t1;
  if (dim == 3) {
    for (int i = tid; i < npt; i += blockDim.x) {
      const int iz = i / (n * n), rem = i % (n * n);
      double s = 0;
      for (int q = 0; q < n; ++q) s += B[q * n + iz] * src[q * n * n + rem];
      tmp[i] = s;
    }
    __syncthreads();
    src = tmp;
    tmp = f0;
  }
  for (int i = tid; i < npt; i += blockDim.x) {
    const int ix = i % n, iy = (i / n) % n, r = i / (n * n);
    double s = 0;
    for (int q = 0; q < n; ++q) s += B[q * n + iy] * src[(r * n + q) * n + ix];
    tmp[i] = s;
  }
  __syncthreads();
  double* out = cellbuf + (int64_t)cell * npt;
  for (int i = tid; i < npt; i += blockDim.x) {
    const int ix = i % n, r = i / n;
    double s = 0;
    for (int q = 0; q < n; ++q) s += B[q * n + ix] * tmp[r * n + q];
    out[i] = s;
  }
}

// y[g] = sum over the cells containing node g of cellbuf (fixed order), 0 on
// Dirichlet nodes.
__global__ void cell_gather_kernel(int dim, int N, int p, const double* cellbuf, double* y) {
  const int M = N * p + 1, n = p + 1;
  const int npt = dim == 3 ? n * n * n : n * n;
  const int64_t total = dim == 3 ? (int64_t)M * M * M : (int64_t)M * M;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int gi[3] = {(int)(g % M), (int)((g / M) % M), dim == 3 ? (int)(g / ((int64_t)M * M)) : 0};
    bool bd = false;
    for (int d = 0; d < dim; ++d) bd = bd || gi[d] == 0 || gi[d] == M - 1;
    if (bd) {
      y[g] = 0.0;
      continue;
    }
    // candidate cells per direction
    int ce[3][2], le[3][2], ne[3];
    for (int d = 0; d < 3; ++d) {
      if (d >= dim) {
        ne[d] = 1;
        ce[d][0] = 0;
        le[d][0] = 0;
        continue;
      }
      const int c = gi[d] / p, l = gi[d] - c * p;
      if (l == 0) {
        ne[d] = 2;
        ce[d][0] = c - 1;
        le[d][0] = p;
        ce[d][1] = c;
        le[d][1] = 0;
      } else {
        ne[d] = 1;
        ce[d][0] = c;
        le[d][0] = l;
      }
    }
    double s = 0;
    for (int kz = 0; kz < ne[2]; ++kz)
      for (int ky = 0; ky < ne[1]; ++ky)
        for (int kx = 0; kx < ne[0]; ++kx) {
          int cell = ce[0][kx] + ce[1][ky] * N;
          int loc = le[0][kx] + le[1][ky] * n;
          if (dim == 3) {
            cell += ce[2][kz] * N * N;
            loc += le[2][kz] * n * n;
          }
          s += cellbuf[(int64_t)cell * npt + loc];
        }
    y[g] = s;
  }
}

// Element matrices Ke[cell][a][b] = sum_k grad phi_a . G_k grad phi_b.
__global__ __launch_bounds__(kCellThreads) void element_matrix_kernel(CellArgs a, double* Ke) {
  extern __shared__ __align__(16) double sm[];
  const int p = a.p, n = p + 1, dim = a.dim;
  const int npt = dim == 3 ? n * n * n : n * n;
  const int NG = dim == 3 ? 6 : 3;
  const double* B = a.tab64;
  const double* D = a.tab64 + 2 * n * n;
  const double* xg = a.tab64 + 3 * n * n;
  const double* wg = xg + n;
  double* G = sm;             // NG * npt
  double* C = G + NG * npt;   // 24
  double* mu = C + 24;
  const int cell = blockIdx.x, row = blockIdx.y;
  load_cell(a, cell, C, mu);
  __syncthreads();
  for (int k = threadIdx.x; k < npt; k += blockDim.x) {
    const int kx = k % n, ky = (k / n) % n, kz = dim == 3 ? k / (n * n) : 0;
    if (dim == 3)
      cell_metric3(C, xg[kx], xg[ky], xg[kz], *mu * wg[kx] * wg[ky] * wg[kz], G + NG * k);
    else
      cell_metric2(C, xg[kx], xg[ky], *mu * wg[kx] * wg[ky], G + NG * k);
  }
  __syncthreads();
  const int ax = row % n, ay = (row / n) % n, az = dim == 3 ? row / (n * n) : 0;
  for (int col = threadIdx.x; col < npt; col += blockDim.x) {
    const int bx = col % n, by = (col / n) % n, bz = dim == 3 ? col / (n * n) : 0;
    double s = 0;
    for (int k = 0; k < npt; ++k) {
      const int kx = k % n, ky = (k / n) % n, kz = dim == 3 ? k / (n * n) : 0;
      const double* g = G + NG * k;
      if (dim == 3) {
        const double a0 = D[kx * n + ax] * B[ky * n + ay] * B[kz * n + az];
        const double a1 = B[kx * n + ax] * D[ky * n + ay] * B[kz * n + az];
        const double a2 = B[kx * n + ax] * B[ky * n + ay] * D[kz * n + az];
        const double b0 = D[kx * n + bx] * B[ky * n + by] * B[kz * n + bz];
        const double b1 = B[kx * n + bx] * D[ky * n + by] * B[kz * n + bz];
        const double b2 = B[kx * n + bx] * B[ky * n + by] * D[kz * n + bz];
        s += a0 * (g[0] * b0 + g[1] * b1 + g[2] * b2) + a1 * (g[1] * b0 + g[3] * b1 + g[4] * b2) +
             a2 * (g[2] * b0 + g[4] * b1 + g[5] * b2);
      } else {
        const double a0 = D[kx * n + ax] * B[ky * n + ay];
        const double a1 = B[kx * n + ax] * D[ky * n + ay];
        const double b0 = D[kx * n + bx] * B[ky * n + by];
        const double b1 = B[kx * n + bx] * D[ky * n + by];
        s += a0 * (g[0] * b0 + g[1] * b1) + a1 * (g[1] * b0 + g[2] * b1);
      }
    }
    Ke[((int64_t)cell * npt + row) * npt + col] = s;
  }
}

// One axis of a Kronecker h-transfer on full nodal tensors.
// forward (transpose = 0): out[.., i, ..] = sum_t w[i][t] in[.., first[i] + t, ..]
// transpose (1):           out[.., t, ..] = sum_i w[i][t - first[i]] in[.., i, ..]
__global__ void h_axis_kernel(int dim, int axis, int3 sin, int3 sout, const int* first,
                              const double* w, int p, const double* in, double* out,
                              int transpose, int nf) {
  const int64_t total = (int64_t)sout.x * sout.y * (dim == 3 ? sout.z : 1);
  for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < total;
       o += (int64_t)gridDim.x * blockDim.x) {
    int idx[3] = {(int)(o % sout.x), (int)((o / sout.x) % sout.y),
                  dim == 3 ? (int)(o / ((int64_t)sout.x * sout.y)) : 0};
    const int t = idx[axis];
    double s = 0;
    int ii[3] = {idx[0], idx[1], idx[2]};
    if (!transpose) {
      for (int k = 0; k <= p; ++k) {
        ii[axis] = first[t] + k;
        s += w[t * (p + 1) + k] * in[ii[0] + (int64_t)sin.x * (ii[1] + (int64_t)sin.y * ii[2])];
      }
    } else {
      // fine rows i whose support contains coarse column t
      const int c = t / p;
      int lo = 2 * (c - 1) * p, hi = 2 * (c + 1) * p;
      if (lo < 0) lo = 0;
      if (hi > nf - 1) hi = nf - 1;
      for (int i = lo; i <= hi; ++i) {
        const int k = t - first[i];
        if (k < 0 || k > p) continue;
        ii[axis] = i;
        s += w[i * (p + 1) + k] * in[ii[0] + (int64_t)sin.x * (ii[1] + (int64_t)sin.y * ii[2])];
      }
    }
    out[o] = s;
  }
}

__global__ void mask_kernel(int dim, int M, double* x) {
  const int64_t total = dim == 3 ? (int64_t)M * M * M : (int64_t)M * M;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int gx = g % M, gy = (g / M) % M, gz = dim == 3 ? g / ((int64_t)M * M) : 1;
    bool bd = gx == 0 || gx == M - 1 || gy == 0 || gy == M - 1;
    if (dim == 3) bd = bd || gz == 0 || gz == M - 1;
    if (bd) x[g] = 0.0;
  }
}

__global__ void axpby_kernel(int64_t n, double a, const double* x, double b, double* y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a * x[i] + b * y[i];
}

__global__ void xpay_to_kernel(int64_t n, const double* x, double a, const double* y, double* z) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    z[i] = x[i] + a * y[i];
}

// deterministic two-stage dot product: fixed grid, fixed reduction order
__global__ __launch_bounds__(256) void dot_partial_kernel(int64_t n, const double* x,
                                                          const double* y, double* partial) {
  __shared__ double red[4];
  double s = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    s += x[i] * y[i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ __launch_bounds__(256) void dot_final_kernel(const double* partial, int nb,
                                                        double* out) {
  __shared__ double red[4];
  double s = 0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) s += partial[i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *out = red[0] + red[1] + red[2] + red[3];
}

// y = A x, A dense row-major n x n: one wavefront per row
__global__ __launch_bounds__(256) void gemv_kernel(int n, const double* A, const double* x,
                                                   double* y) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  double s = 0;
  const double* a = A + (int64_t)row * n;
  for (int j = lane; j < n; j += 64) s += a[j] * x[j];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) y[row] = s;
}

__global__ void gather_interior_kernel(int dim, int M, const double* full, double* packed) {
  const int mi = M - 2;
  const int64_t total = dim == 3 ? (int64_t)mi * mi * mi : (int64_t)mi * mi;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int x = i % mi + 1, y = (i / mi) % mi + 1, z = dim == 3 ? i / ((int64_t)mi * mi) + 1 : 0;
    packed[i] = full[x + (int64_t)M * (y + (int64_t)M * z)];
  }
}

__global__ void scatter_interior_kernel(int dim, int M, const double* packed, double* full) {
  const int mi = M - 2;
  const int64_t total = dim == 3 ? (int64_t)mi * mi * mi : (int64_t)mi * mi;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int x = i % mi + 1, y = (i / mi) % mi + 1, z = dim == 3 ? i / ((int64_t)mi * mi) + 1 : 0;
    full[x + (int64_t)M * (y + (int64_t)M * z)] = packed[i];
  }
}

__global__ void convert_kernel(int64_t n, const double* in, float* out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (float)in[i];
}

int grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (int)g;
}

size_t cell_lds(int dim, int p) {
  const int n = p + 1;
  const int npt = dim == 3 ? n * n * n : n * n;
  return (size_t)(6 * npt + 32) * sizeof(double);
}

}  // namespace

hipError_t launch_cell_apply(const CellArgs& a, const double* x, double* cellbuf, hipStream_t s) {
  const int ncell = a.dim == 3 ? a.N * a.N * a.N : a.N * a.N;
  (void)hipGetLastError();
  hipLaunchKernelGGL(cell_apply_kernel, dim3(ncell), dim3(kCellThreads), cell_lds(a.dim, a.p), s,
                     a, x, cellbuf);
  return hipGetLastError();
}

hipError_t launch_cell_gather(int dim, int N, int p, const double* cellbuf, double* y,
                              hipStream_t s) {
  const int64_t M = (int64_t)N * p + 1;
  (void)hipGetLastError();
  hipLaunchKernelGGL(cell_gather_kernel, dim3(grid_for(dim == 3 ? M * M * M : M * M)), dim3(256),
                     0, s, dim, N, p, cellbuf, y);
  return hipGetLastError();
}

hipError_t launch_element_matrices(const CellArgs& a, double* Ke, hipStream_t s) {
  const int n = a.p + 1;
  const int npt = a.dim == 3 ? n * n * n : n * n;
  const int ncell = a.dim == 3 ? a.N * a.N * a.N : a.N * a.N;
  const size_t lds = (size_t)((a.dim == 3 ? 6 : 3) * npt + 32) * sizeof(double);
  (void)hipGetLastError();
  hipLaunchKernelGGL(element_matrix_kernel, dim3(ncell, npt), dim3(kCellThreads), lds, s, a, Ke);
  return hipGetLastError();
}

hipError_t launch_h_prolong_axis(int dim, int axis, const int* sizes_in, const int* sizes_out,
                                 const int* first, const double* w, int p, const double* in,
                                 double* out, int transpose, hipStream_t s) {
  int3 si = make_int3(sizes_in[0], sizes_in[1], sizes_in[2]);
  int3 so = make_int3(sizes_out[0], sizes_out[1], sizes_out[2]);
  const int64_t total = (int64_t)so.x * so.y * (dim == 3 ? so.z : 1);
  // number of fine rows of the 1D matrix: the larger extent along the axis
  const int nf = transpose ? sizes_in[axis] : sizes_out[axis];
  (void)hipGetLastError();
  hipLaunchKernelGGL(h_axis_kernel, dim3(grid_for(total)), dim3(256), 0, s, dim, axis, si, so,
                     first, w, p, in, out, transpose, nf);
  return hipGetLastError();
}

// u[global node of interior node i of patch j] += theta d[j][i] for the
// patches begin .. begin + count - 1 (patch order; one colour, so their
// interiors are disjoint and every node is written by one thread): the
// scatter of the additive smoother, interior-vertex patches of a structured
// mesh with N cells per direction at degree p, interiors x fastest.
template <int DIM>
__global__ void patch_scatter_kernel(int N, int p, const int32_t* vertex, int begin, int count,
                                     const double* d, double theta, double* u) {
  const int mi = 2 * p - 1;
  const int64_t n0 = DIM == 3 ? (int64_t)mi * mi * mi : (int64_t)mi * mi;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)count * n0) return;
  const int j = begin + (int)(t / n0);
  const int i = (int)(t % n0);
  const int N1 = N + 1;
  const int64_t M = (int64_t)N * p + 1;
  const int v = vertex[j];
  const int vx = v % N1, vy = (v / N1) % N1, vz = DIM == 3 ? v / (N1 * N1) : 0;
  const int x = i % mi + 1, y = (i / mi) % mi + 1, z = DIM == 3 ? i / (mi * mi) + 1 : 0;
  const int64_t gx = (int64_t)(vx - 1) * p + x, gy = (int64_t)(vy - 1) * p + y,
                gz = DIM == 3 ? (int64_t)(vz - 1) * p + z : 0;
  // nodes of a boundary-vertex patch on or beyond the boundary are masked
  if (gx <= 0 || gx >= M - 1 || gy <= 0 || gy >= M - 1 || (DIM == 3 && (gz <= 0 || gz >= M - 1))) return;
  u[gx + M * gy + M * M * gz] += theta * d[(int64_t)j * n0 + i];
}

hipError_t launch_patch_scatter(int dim, int N, int p, const int32_t* vertex, int begin, int count,
                                const double* d, double theta, double* u, hipStream_t s) {
  const int mi = 2 * p - 1;
  const int64_t total = (int64_t)count * (dim == 3 ? (int64_t)mi * mi * mi : (int64_t)mi * mi);
  if (total <= 0) return hipSuccess;
  (void)hipGetLastError();
  if (dim == 3)
    hipLaunchKernelGGL(patch_scatter_kernel<3>, dim3(grid_for(total)), dim3(256), 0, s, N, p, vertex, begin,
                       count, d, theta, u);
  else
    hipLaunchKernelGGL(patch_scatter_kernel<2>, dim3(grid_for(total)), dim3(256), 0, s, N, p, vertex, begin,
                       count, d, theta, u);
  return hipGetLastError();
}

hipError_t launch_mask_dirichlet(int dim, int M, double* x, hipStream_t s) {
  const int64_t total = dim == 3 ? (int64_t)M * M * M : (int64_t)M * M;
  (void)hipGetLastError();
  hipLaunchKernelGGL(mask_kernel, dim3(grid_for(total)), dim3(256), 0, s, dim, M, x);
  return hipGetLastError();
}

hipError_t launch_axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t s) {
  (void)hipGetLastError();
  hipLaunchKernelGGL(axpby_kernel, dim3(grid_for(n)), dim3(256), 0, s, n, a, x, b, y);
  return hipGetLastError();
}

hipError_t launch_xpay_to(int64_t n, const double* x, double a, const double* y, double* z,
                          hipStream_t s) {
  (void)hipGetLastError();
  hipLaunchKernelGGL(xpay_to_kernel, dim3(grid_for(n)), dim3(256), 0, s, n, x, a, y, z);
  return hipGetLastError();
}

hipError_t launch_dot_partial(int64_t n, const double* x, const double* y, double* partial,
                              int nblocks, hipStream_t s) {
  (void)hipGetLastError();
  hipLaunchKernelGGL(dot_partial_kernel, dim3(nblocks), dim3(256), 0, s, n, x, y, partial);
  return hipGetLastError();
}

hipError_t launch_dot_final(const double* partial, int nblocks, double* out, hipStream_t s) {
  (void)hipGetLastError();
  hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(256), 0, s, partial, nblocks, out);
  return hipGetLastError();
}

hipError_t launch_gemv(int n, const double* A, const double* x, double* y, hipStream_t s) {
  (void)hipGetLastError();
  hipLaunchKernelGGL(gemv_kernel, dim3((n + 3) / 4), dim3(256), 0, s, n, A, x, y);
  return hipGetLastError();
}

hipError_t launch_gather_interior(int dim, int M, const double* full, double* packed,
                                  hipStream_t s) {
  const int64_t mi = M - 2;
  (void)hipGetLastError();
  hipLaunchKernelGGL(gather_interior_kernel, dim3(grid_for(dim == 3 ? mi * mi * mi : mi * mi)),
                     dim3(256), 0, s, dim, M, full, packed);
  return hipGetLastError();
}

hipError_t launch_scatter_interior(int dim, int M, const double* packed, double* full,
                                   hipStream_t s) {
  const int64_t mi = M - 2;
  (void)hipGetLastError();
  hipLaunchKernelGGL(scatter_interior_kernel, dim3(grid_for(dim == 3 ? mi * mi * mi : mi * mi)),
                     dim3(256), 0, s, dim, M, packed, full);
  return hipGetLastError();
}

hipError_t launch_convert_to_float(int64_t n, const double* in, float* out, hipStream_t s) {
  (void)hipGetLastError();
  hipLaunchKernelGGL(convert_kernel, dim3(grid_for(n)), dim3(256), 0, s, n, in, out);
  return hipGetLastError();
}

}  // namespace pmgi
