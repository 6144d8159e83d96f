"""One-dimensional finite element ingredients on the reference interval [0, 1].

TEST INFRASTRUCTURE (oracle): see oracle/__init__.py.

The paper fixes only "polynomials of degree up to p" on tensor-product cells
(Section 3.1, p-multigrid components) and sum-factorised evaluation with
O(p^d) quadrature points per cell (Section 3.1, level operators).  Readings
used here:
  * the nodal basis of degree q is Lagrange on the q+1 Gauss-Lobatto-Legendre
    (GLL) points;
  * the quadrature at degree q is Gauss-Legendre with q+1 points.
"""
from __future__ import annotations

import numpy as np


def gll_nodes(q: int) -> np.ndarray:
    """The q+1 Gauss-Lobatto-Legendre points on [0,1]: the end points and the
    roots of P_q' (Legendre polynomial derivative), sorted ascending."""
    if q < 1:
        raise ValueError("degree must be >= 1")
    if q == 1:
        return np.array([0.0, 1.0])
    dP = np.polynomial.legendre.Legendre.basis(q).deriv()
    r = np.sort(np.real(dP.roots()))
    # polish the roots of P_q' with Newton steps
    d2P = dP.deriv()
    for _ in range(3):
        r = r - dP(r) / d2P(r)
    t = np.concatenate([[-1.0], r, [1.0]])
    return 0.5 * (t + 1.0)


def gauss_rule(n: int):
    """n-point Gauss-Legendre rule on [0,1]: (points, weights)."""
    t, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (t + 1.0), 0.5 * w


def lagrange_values(nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """L[i, k] = l_i(x_k): the Lagrange polynomials of `nodes` evaluated at x,
    l_i(x) = prod_{j != i} (x - x_j) / (x_i - x_j)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    L = np.ones((n, len(x)))
    for i in range(n):
        for j in range(n):
            if j != i:
                L[i] *= (x - nodes[j]) / (nodes[i] - nodes[j])
    return L


def lagrange_derivatives(nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """D[i, k] = l_i'(x_k), by the product rule:
    l_i'(x) = sum_{m != i} 1/(x_i - x_m) prod_{j != i, m} (x - x_j)/(x_i - x_j)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    D = np.zeros((n, len(x)))
    for i in range(n):
        for m in range(n):
            if m == i:
                continue
            term = np.full(len(x), 1.0 / (nodes[i] - nodes[m]))
            for j in range(n):
                if j != i and j != m:
                    term *= (x - nodes[j]) / (nodes[i] - nodes[j])
            D[i] += term
    return D
