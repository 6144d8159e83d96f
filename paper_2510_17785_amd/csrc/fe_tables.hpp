// One-dimensional finite element tables on the reference interval [0, 1],
// computed on the host in FP64 and uploaded once per handle.
//
// Readings of the paper (which fixes only "polynomials of degree up to p" on
// tensor-product cells, Section 3.1): the nodal basis of degree q is Lagrange
// on the q+1 Gauss-Lobatto-Legendre points; level q integrates with the
// (q+1)-point Gauss-Legendre rule.
#pragma once

#include <vector>

namespace pmgi {

constexpr int kMaxDegree = 15;
constexpr int kMaxN = kMaxDegree + 1;  // nodes (and Gauss points) per cell per direction

// q+1 GLL points of degree q on [0,1], ascending.
std::vector<double> gll_nodes(int q);
// n-point Gauss-Legendre rule on [0,1].
void gauss_rule(int n, std::vector<double>& x, std::vector<double>& w);
// l_i(x) and l_i'(x) for the Lagrange polynomials of `nodes`.
double lagrange(const std::vector<double>& nodes, int i, double x);
double lagrange_deriv(const std::vector<double>& nodes, int i, double x);

// Per-degree tables used by the sum-factorised operator:
//   B[k*n + a]  = l_a(xg_k)          (GLL basis at Gauss points)
//   Dc[k*n + j] = lg_j'(xg_k)        (derivative of the Gauss-point Lagrange
//                                     basis at the Gauss points: collocation
//                                     derivative)
//   D[k*n + a]  = l_a'(xg_k)         (GLL basis derivative at Gauss points)
struct DegreeTables {
  int q = 0, n = 0;
  std::vector<double> B, Dc, D, xg, wg;
};
DegreeTables degree_tables(int q);

// Embedding of the degree-q interior space of a patch direction with `ncell`
// cells into the degree-p one: (ncell p - 1) x (ncell q - 1), row-major.
std::vector<double> patch_prolongation_1d(int p, int q, int ncell);

// Embedding of the 1D degree-p space on nc cells into the one on 2 nc cells,
// all nodes: row g of the (2 nc p + 1) x (nc p + 1) matrix has its non-zeros
// in columns first[g] .. first[g] + p, values w[g*(p+1) + t].
void h_prolongation_1d(int nc, int p, std::vector<int>& first, std::vector<double>& w);

// Fast diagonalisation of the degree-q operator of the Cartesian reference
// patch with `ncell` unit cells per direction (2 for an interior vertex, 1
// along a direction where the boundary cuts the patch), coefficient 1: the
// A_b of the Cartesian-reinforced smoother (Section 3.1).  M, K: the 1D mass
// and stiffness matrices on the m = ncell q - 1 interior nodes (m = 0: empty
// tables); S (m x m, row-major,
// column k the k-th eigenvector) and lam solve K S = M S diag(lam) with
// S^T M S = I, so that A_b = sum_i M (x) .. K_i .. (x) M has the inverse
// S^(x d) diag(1 / sum_i lam_{k_i}) (S^T)^(x d); dM, dK are the diagonals of
// M and K (diag A_b = sum_i dM (x) .. dK_i .. (x) dM).
struct FdmTables {
  int m = 0;
  std::vector<double> S, lam, dM, dK;
};
FdmTables fdm_tables(int q, int ncell = 2);

}  // namespace pmgi
