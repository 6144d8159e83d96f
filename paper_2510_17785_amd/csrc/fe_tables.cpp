#include "fe_tables.hpp"

#include <algorithm>
#include <cmath>

namespace pmgi {

namespace {

// Legendre P_q(t) and P_q'(t) on [-1,1] by the three-term recurrence
// (k+1) P_{k+1} = (2k+1) t P_k - k P_{k-1}.
void legendre(int q, double t, double& P, double& dP) {
  double p0 = 1.0, p1 = t;
  if (q == 0) {
    P = 1.0;
    dP = 0.0;
    return;
  }
  for (int k = 1; k < q; ++k) {
    double p2 = ((2.0 * k + 1.0) * t * p1 - k * p0) / (k + 1.0);
    p0 = p1;
    p1 = p2;
  }
  P = p1;
  // P_q' from q (P_{q-1} - t P_q) / (1 - t^2), valid off the end points
  dP = q * (p0 - t * p1) / (1.0 - t * t);
}

}  // namespace

std::vector<double> gll_nodes(int q) {
  std::vector<double> x(q + 1);
  x[0] = 0.0;
  x[q] = 1.0;
  // interior points: roots of P_q'; Newton with P_q'' from the Legendre
  // equation (1 - t^2) P'' = 2 t P' - q (q+1) P; start at the
  // Chebyshev-Gauss-Lobatto points.
  for (int j = 1; j < q; ++j) {
    double t = -std::cos(M_PI * j / q);
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(q, t, P, dP);
      double d2P = (2.0 * t * dP - q * (q + 1.0) * P) / (1.0 - t * t);
      double step = dP / d2P;
      t -= step;
      if (std::fabs(step) < 1e-16) break;
    }
    x[j] = 0.5 * (t + 1.0);
  }
  std::sort(x.begin(), x.end());
  // exact symmetry about 1/2
  for (int j = 0; j <= q / 2; ++j) {
    double s = 0.5 * (x[j] + 1.0 - x[q - j]);
    x[j] = s;
    x[q - j] = 1.0 - s;
  }
  return x;
}

void gauss_rule(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int j = 0; j < n; ++j) {
    double t = -std::cos(M_PI * (j + 0.75) / (n + 0.5));
    double P = 0.0, dP = 1.0;
    for (int it = 0; it < 100; ++it) {
      legendre(n, t, P, dP);
      double step = P / dP;
      t -= step;
      if (std::fabs(step) < 1e-16) break;
    }
    legendre(n, t, P, dP);
    x[j] = 0.5 * (t + 1.0);
    w[j] = 1.0 / ((1.0 - t * t) * dP * dP);  // 2 / ((1-t^2) P'^2), halved for [0,1]
  }
  std::vector<int> idx(n);
  for (int j = 0; j < n; ++j) idx[j] = j;
  std::sort(idx.begin(), idx.end(), [&](int a, int b) { return x[a] < x[b]; });
  std::vector<double> xs(n), ws(n);
  for (int j = 0; j < n; ++j) {
    xs[j] = x[idx[j]];
    ws[j] = w[idx[j]];
  }
  for (int j = 0; j < n / 2; ++j) {
    double s = 0.5 * (xs[j] + 1.0 - xs[n - 1 - j]);
    xs[j] = s;
    xs[n - 1 - j] = 1.0 - s;
    double ww = 0.5 * (ws[j] + ws[n - 1 - j]);
    ws[j] = ws[n - 1 - j] = ww;
  }
  if (n % 2) xs[n / 2] = 0.5;
  x = xs;
  w = ws;
}

double lagrange(const std::vector<double>& nodes, int i, double x) {
  double v = 1.0;
  for (size_t j = 0; j < nodes.size(); ++j)
    if ((int)j != i) v *= (x - nodes[j]) / (nodes[i] - nodes[j]);
  return v;
}

double lagrange_deriv(const std::vector<double>& nodes, int i, double x) {
  double s = 0.0;
  for (size_t m = 0; m < nodes.size(); ++m) {
    if ((int)m == i) continue;
    double t = 1.0 / (nodes[i] - nodes[m]);
    for (size_t j = 0; j < nodes.size(); ++j)
      if ((int)j != i && j != m) t *= (x - nodes[j]) / (nodes[i] - nodes[j]);
    s += t;
  }
  return s;
}

DegreeTables degree_tables(int q) {
  DegreeTables t;
  t.q = q;
  t.n = q + 1;
  const int n = t.n;
  std::vector<double> nodes = gll_nodes(q);
  gauss_rule(n, t.xg, t.wg);
  t.B.resize(n * n);
  t.Dc.resize(n * n);
  t.D.resize(n * n);
  for (int k = 0; k < n; ++k)
    for (int a = 0; a < n; ++a) {
      t.B[k * n + a] = lagrange(nodes, a, t.xg[k]);
      t.D[k * n + a] = lagrange_deriv(nodes, a, t.xg[k]);
      t.Dc[k * n + a] = lagrange_deriv(t.xg, a, t.xg[k]);
    }
  return t;
}

std::vector<double> patch_prolongation_1d(int p, int q, int ncell) {
  const int rows = ncell * p - 1, cols = ncell * q - 1;
  std::vector<double> P(std::max(rows * cols, 0), 0.0);
  std::vector<double> xp = gll_nodes(p), xq = gll_nodes(q);
  for (int s = 1; s < ncell * p; ++s) {
    int c = std::min(s / p, ncell - 1);
    double xi = xp[s - c * p];
    for (int t = 1; t < ncell * q; ++t) {
      int a = t - c * q;
      if (a >= 0 && a <= q) P[(s - 1) * cols + (t - 1)] = lagrange(xq, a, xi);
    }
  }
  return P;
}

void h_prolongation_1d(int nc, int p, std::vector<int>& first, std::vector<double>& w) {
  const int nf = 2 * nc, rows = nf * p + 1;
  std::vector<double> x = gll_nodes(p);
  first.assign(rows, 0);
  w.assign(rows * (p + 1), 0.0);
  for (int g = 0; g < rows; ++g) {
    int f = std::min(g / p, nf - 1);
    double xi_f = x[g - f * p];
    int c = f / 2;
    double xi = ((f % 2) + xi_f) * 0.5;
    first[g] = c * p;
    for (int t = 0; t <= p; ++t) w[g * (p + 1) + t] = lagrange(x, t, xi);
  }
}

FdmTables fdm_tables(int q, int ncell) {
  FdmTables f;
  const int n = q + 1, m = ncell * q - 1, nt = ncell * q + 1;
  f.m = m;
  if (m <= 0) return f;
  DegreeTables t = degree_tables(q);
  // one cell: M_ab = sum_k w_k l_a(x_k) l_b(x_k), K_ab = sum_k w_k l_a'(x_k) l_b'(x_k);
  // neighbouring cells share a node; the interior nodes are 1 .. ncell q - 1
  std::vector<double> M2(nt * nt, 0.0), K2(M2.size(), 0.0);
  for (int c = 0; c < ncell; ++c)
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) {
        double mv = 0, kv = 0;
        for (int k = 0; k < n; ++k) {
          mv += t.wg[k] * t.B[k * n + a] * t.B[k * n + b];
          kv += t.wg[k] * t.D[k * n + a] * t.D[k * n + b];
        }
        const int r = c * q + a, s2 = c * q + b;
        M2[r * nt + s2] += mv;
        K2[r * nt + s2] += kv;
      }
  std::vector<double> M(m * m), K(m * m);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      M[i * m + j] = M2[(i + 1) * nt + (j + 1)];
      K[i * m + j] = K2[(i + 1) * nt + (j + 1)];
    }
  f.dM.resize(m);
  f.dK.resize(m);
  for (int i = 0; i < m; ++i) {
    f.dM[i] = M[i * m + i];
    f.dK[i] = K[i * m + i];
  }
  // Cholesky M = L L^T (M is symmetric positive definite)
  std::vector<double> Lc(m * m, 0.0);
  for (int j = 0; j < m; ++j) {
    double d = M[j * m + j];
    for (int k = 0; k < j; ++k) d -= Lc[j * m + k] * Lc[j * m + k];
    Lc[j * m + j] = std::sqrt(d);
    for (int i = j + 1; i < m; ++i) {
      double v = M[i * m + j];
      for (int k = 0; k < j; ++k) v -= Lc[i * m + k] * Lc[j * m + k];
      Lc[i * m + j] = v / Lc[j * m + j];
    }
  }
  // C = L^{-1} K L^{-T}: solve L Y = K, then L C^T = Y^T (C symmetric)
  std::vector<double> Y(m * m), C(m * m);
  for (int col = 0; col < m; ++col)
    for (int i = 0; i < m; ++i) {
      double v = K[i * m + col];
      for (int k = 0; k < i; ++k) v -= Lc[i * m + k] * Y[k * m + col];
      Y[i * m + col] = v / Lc[i * m + i];
    }
  for (int col = 0; col < m; ++col)
    for (int i = 0; i < m; ++i) {
      double v = Y[col * m + i];
      for (int k = 0; k < i; ++k) v -= Lc[i * m + k] * C[col * m + k];
      C[col * m + i] = v / Lc[i * m + i];
    }
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < i; ++j) C[i * m + j] = C[j * m + i] = 0.5 * (C[i * m + j] + C[j * m + i]);
  // cyclic Jacobi rotations (Golub and Van Loan, Algorithm 8.5.3): C = V diag(lam) V^T
  std::vector<double> V(m * m, 0.0);
  for (int i = 0; i < m; ++i) V[i * m + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0, tot = 0;
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) (i == j ? tot : off) += C[i * m + j] * C[i * m + j];
    if (off <= 1e-30 * (tot + off)) break;
    for (int p = 0; p < m - 1; ++p)
      for (int r = p + 1; r < m; ++r) {
        const double apr = C[p * m + r];
        if (apr == 0.0) continue;
        const double tau = (C[r * m + r] - C[p * m + p]) / (2.0 * apr);
        const double tt = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double cs = 1.0 / std::sqrt(1.0 + tt * tt), sn = tt * cs;
        for (int k = 0; k < m; ++k) {  // C <- C J (columns p, r)
          const double ckp = C[k * m + p], ckr = C[k * m + r];
          C[k * m + p] = cs * ckp - sn * ckr;
          C[k * m + r] = sn * ckp + cs * ckr;
        }
        for (int k = 0; k < m; ++k) {  // C <- J^T C (rows p, r)
          const double cpk = C[p * m + k], crk = C[r * m + k];
          C[p * m + k] = cs * cpk - sn * crk;
          C[r * m + k] = sn * cpk + cs * crk;
        }
        for (int k = 0; k < m; ++k) {  // V <- V J
          const double vkp = V[k * m + p], vkr = V[k * m + r];
          V[k * m + p] = cs * vkp - sn * vkr;
          V[k * m + r] = sn * vkp + cs * vkr;
        }
      }
  }
  f.lam.resize(m);
  for (int k = 0; k < m; ++k) f.lam[k] = C[k * m + k];
  // S = L^{-T} V: solve L^T S = V column by column
  f.S.assign(m * m, 0.0);
  for (int col = 0; col < m; ++col)
    for (int i = m - 1; i >= 0; --i) {
      double v = V[i * m + col];
      for (int k = i + 1; k < m; ++k) v -= Lc[k * m + i] * f.S[k * m + col];
      f.S[i * m + col] = v / Lc[i * m + i];
    }
  return f;
}

}  // namespace pmgi
