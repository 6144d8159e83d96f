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

}  // namespace pmgi
