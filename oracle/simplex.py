"""Simplicial (unstructured) vertex patches and their p-multigrid local solver
(Section 3.2: besides Cartesian patches the paper tests patches of 3
quadrilaterals in 2D and 4 hexahedra in 3D around one vertex).

TEST INFRASTRUCTURE (oracle): see oracle/__init__.py.

A patch is given by its vertices and the corner lists of its cells (x
fastest, corner 0 on the patch boundary, the last corner the patch vertex;
`synth.simplex_patch`).  The cells are multilinear, as everywhere else, so
the element matrices are those of `fem.element_matrices`; only the
numbering differs from a tensor-product patch:

  * the degree-q nodes of a cell are the images of its GLL tensor points;
    nodes of neighbouring cells that map to the same point are one degree
    of freedom (the conforming space, Section 2);
  * a node is on the patch boundary when it has a zero local index in some
    direction (the cell's faces through corner 0 lie on the patch boundary,
    those through the patch vertex inside it); the interior nodes are the
    patch's unknowns (zero Dirichlet values on the boundary, Section 2.1);
  * unknowns are numbered in order of first appearance, cells in order and
    the nodes of a cell x fastest.

Level operators are rediscretisations at every degree (Section 3.1), the
transfer P_{q->p} is the embedding of the degree-q patch space into the
degree-p one (a fine unknown takes the coarse function's value at its node,
evaluated in the first cell that holds it), R = P^T; the V-cycle is that of
`pmg.LocalSolver` (Algorithm 2) on these matrices.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import fe1d
from .fem import _multi, element_matrices
from .pmg import CHEB_RANGE, CHEB_SAFETY, chebyshev, chebyshev_interval, pcg


def cell_nodes(Xc: np.ndarray, q: int) -> np.ndarray:
    """Physical positions of the (q+1)^dim GLL nodes of a multilinear cell
    with corners Xc (2^dim, dim), x fastest."""
    dim = Xc.shape[1]
    x = fe1d.gll_nodes(q)
    out = []
    for a in _multi(q + 1, dim):
        w = np.ones(2 ** dim)
        for b in range(2 ** dim):
            for i in range(dim):
                w[b] *= x[a[i]] if (b >> i) & 1 else 1.0 - x[a[i]]
        out.append(w @ Xc)
    return np.array(out)


def numbering(X: np.ndarray, cells: np.ndarray, q: int):
    """gather (ncell, (q+1)^dim): unknown of every cell node, -1 on the patch
    boundary; and the number of unknowns."""
    dim = X.shape[1]
    scale = np.abs(X).max() + 1.0
    key_of = {}
    gather = np.full((len(cells), (q + 1) ** dim), -1, dtype=np.int64)
    count = 0
    for c, corners in enumerate(cells):
        P = cell_nodes(X[corners], q)
        for a, aa in enumerate(_multi(q + 1, dim)):
            if min(aa) == 0:
                continue
            key = tuple(np.round(P[a] / scale, 9))
            if key not in key_of:
                key_of[key] = count
                count += 1
            gather[c, a] = key_of[key]
    return gather, count


def level_matrix(X, cells, mu, q):
    """A_q: a(.,.) on the unknowns of the patch at degree q (explicit assembly)."""
    gather, n = numbering(X, cells, q)
    Ke = element_matrices(X[cells], np.asarray(mu, dtype=np.float64), q)
    A = np.zeros((n, n))
    for c in range(len(cells)):
        g = gather[c]
        m = g >= 0
        A[np.ix_(g[m], g[m])] += Ke[c][np.ix_(m, m)]
    return A


def prolongation(X, cells, p, q):
    """P_{q->p} (n_p x n_q): row of a fine unknown = the degree-q basis
    functions of the first cell holding it, at its reference point there."""
    dim = X.shape[1]
    gp, n_p = numbering(X, cells, p)
    gq, n_q = numbering(X, cells, q)
    xp, xq = fe1d.gll_nodes(p), fe1d.gll_nodes(q)
    L = fe1d.lagrange_values(xq, xp)           # L[b, s] = l^q_b(x^p_s)
    P = np.zeros((n_p, n_q))
    done = np.zeros(n_p, dtype=bool)
    fine_idx, coarse_idx = _multi(p + 1, dim), _multi(q + 1, dim)
    for c in range(len(cells)):
        for a, aa in enumerate(fine_idx):
            f = gp[c, a]
            if f < 0 or done[f]:
                continue
            done[f] = True
            for b, bb in enumerate(coarse_idx):
                if gq[c, b] >= 0:
                    P[f, gq[c, b]] = np.prod([L[bb[i], aa[i]] for i in range(dim)])
    return P


class SimplexSolver:
    """The p-multigrid V-cycle (Algorithm 2) for A_p d = r on one simplicial
    patch; Chebyshev-Jacobi smoothing with the intervals of pmg (degree 1 on
    an interval with a + b = 4 is the paper's damped Jacobi, omega = 1/2)."""

    def __init__(self, X, cells, mu, levels, cheb_degree=3, n_vcycles=1):
        self.levels = tuple(levels)
        self.k, self.n_vcycles = cheb_degree, n_vcycles
        self.A = [level_matrix(X, cells, mu, q) for q in self.levels]
        self.dinv = [1.0 / np.diag(A) for A in self.A]
        self.P = [prolongation(X, cells, self.levels[l], self.levels[l + 1])
                  for l in range(len(self.levels) - 1)]
        self.chol = sla.cho_factor(self.A[-1], lower=True)
        self.intervals = None

    def set_bounds(self, bounds, safety=CHEB_SAFETY, rng=CHEB_RANGE):
        self.intervals = [chebyshev_interval(lo, hi, safety, rng) for (lo, hi) in bounds]

    def vcycle(self, level, d, r, d_is_zero=False):
        if level == len(self.levels) - 1:
            return sla.cho_solve(self.chol, r)
        A, dinv = self.A[level], self.dinv[level]
        a, b = self.intervals[level]
        d = chebyshev(A, dinv, r, d, a, b, self.k, x_is_zero=d_is_zero)       # pre-smoothing
        rc = self.P[level].T @ (r - A @ d)                                     # residual, restriction
        e = self.vcycle(level + 1, np.zeros_like(rc), rc, d_is_zero=True)     # recursion
        d = d + self.P[level] @ e                                              # correction
        return chebyshev(A, dinv, r, d, a, b, self.k)                          # post-smoothing

    def solve(self, r):
        d = np.zeros_like(r)
        for it in range(self.n_vcycles):
            d = self.vcycle(0, d, r, d_is_zero=(it == 0))
        return d

    def pcg(self, b, rtol, maxit):
        """CG on A_p x = b preconditioned by solve(); (x, iterations, ||r||/||b||)."""
        return pcg(lambda v: self.A[0] @ v, self.solve, b, rtol, maxit)
