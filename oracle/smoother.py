"""The multiplicative vertex-patch smoother (Section 2.1, Algorithm 1).

TEST INFRASTRUCTURE (oracle): see oracle/__init__.py.

For every patch j, in a fixed order, with the global u updated after each
patch (Section 2.1):
    gather    u-bar_j = Pi-bar_j u, b_j = Pi_j b              (eq. gather)
    evaluate  r_j = b_j - Pi_j A-bar_j u-bar_j                (eq. main:4)
    solve     d_j ~ A~_j^{-1} r_j  (p-multigrid V-cycles)     (eq. main:5)
    scatter   u += Pi_j^T d_j                                 (eq. scatter)

Order: patches sit at the interior vertices v of the mesh.  Vertex v has
colour sum_i 2^i (v_i mod 2); a forward sweep visits colours 0 .. 2^d-1 and,
within a colour, vertices in lexicographic order (x fastest); a backward sweep
visits the reverse order.  Two vertices of one colour differ by at least 2 in
some coordinate, so the interior of one patch never meets the closure of the
other; the patches of one colour can therefore be updated in any order with
the same result.
"""
from __future__ import annotations

import itertools

import numpy as np

from .fem import Mesh, PatchGeometry, _multi, global_node, patch_closure_matrix
from .pmg import LocalSolver
from . import lanczos


def vertex_color(v) -> int:
    return sum(((v[i] % 2) << i) for i in range(len(v)))


def interior_vertices(dim: int, n: int):
    """Interior vertices in x-fastest order."""
    return [tuple(t + 1 for t in v) for v in _multi(n - 1, dim)]


def all_vertices(dim: int, n: int):
    """Every vertex, boundary included, in x-fastest order."""
    return [tuple(v) for v in _multi(n + 1, dim)]


def patch_order(dim: int, n: int, with_boundary: bool = False):
    """Forward sweep order: colours ascending, lexicographic within a colour;
    with_boundary adds the patches of the boundary vertices (cut to the cells
    inside the mesh)."""
    verts = all_vertices(dim, n) if with_boundary else interior_vertices(dim, n)
    return [v for c in range(2 ** dim) for v in verts if vertex_color(v) == c]


def patch_indices(v, p: int, n: int, dim: int):
    """(closure global indices, interior global indices) of the patch around
    vertex v at degree p: node offsets s in [0, k_i p] from start_i p per
    direction (k_i cells, start_i = max(v_i - 1, 0)), interior s in
    [1, k_i p - 1], both x-fastest."""
    m = n * p + 1
    st = [max(v[i] - 1, 0) for i in range(dim)]
    nc = [2 if 0 < v[i] < n else 1 for i in range(dim)]
    clo, inn = [], []
    for s in itertools.product(*[range(nc[i] * p + 1) for i in reversed(range(dim))]):
        s = tuple(reversed(s))
        g = global_node([st[i] * p + s[i] for i in range(dim)], m, dim)
        clo.append(g)
        if all(0 < s[i] < nc[i] * p for i in range(dim)):
            inn.append(g)
    return np.array(clo), np.array(inn)


class PatchSmoother:
    """All patches of one mesh with their local p-multigrid solvers.

    bounds: "lanczos" (computed here with the given seed and step count), or a
    dict {vertex: [(lam_min, lam_max) per smoothed level]}.
    global_matrix: if given, the evaluate step uses its rows at the patch
    interior (the same numbers as the interior rows of A-bar_j); else A-bar_j
    is assembled per patch, or taken from the cache when keep_closure is set.
    vertices: restrict the smoother to these patches (sweep order kept), for
    timing a sample of a large mesh.
    """

    def __init__(self, mesh: Mesh, p: int, levels, cheb_degree=3, n_vcycles=1,
                 bounds="lanczos", lanczos_steps=12, seed=0, global_matrix=None,
                 keep_closure=False, vertices=None, with_boundary=False, smoother="chebyshev",
                 omega=0.5):
        self.mesh, self.p, self.levels = mesh, p, tuple(levels)
        self.dim, self.n = mesh.dim, mesh.n
        self.order = patch_order(self.dim, self.n, with_boundary)
        if vertices is not None:
            keep = set(tuple(v) for v in vertices)
            self.order = [v for v in self.order if v in keep]
        self.solvers = {}
        self.idx = {}
        self.closure = {}
        self.A = global_matrix
        for v in self.order:
            P = mesh.patch(v)
            s = LocalSolver(P, self.levels, cheb_degree=cheb_degree, n_vcycles=n_vcycles,
                            smoother=smoother, omega=omega)
            if smoother == "cartesian":
                b = None                 # the Cartesian-reinforced smoother uses no interval
            elif bounds == "lanczos":
                vlin = sum(v[i] * (self.n + 1) ** i for i in range(self.dim))
                b = [lanczos.bounds(s.A[l], s.dinv[l], lanczos_steps, seed, vlin, l)
                     for l in range(len(s.levels) - 1)]
            else:
                b = bounds[v]
            if b is not None:
                s.set_bounds(b)
            self.solvers[v] = s
            self.idx[v] = patch_indices(v, p, self.n, self.dim)
            if keep_closure and global_matrix is None:
                mask = P.interior_mask(p)
                self.closure[v] = patch_closure_matrix(P, p)[mask]

    def local_residual(self, v, u, b):
        """r_j = b_j - Pi_j A-bar_j u-bar_j (evaluate step)."""
        clo, inn = self.idx[v]
        if self.A is not None:
            # rows of the global operator at the patch interior: every interior
            # basis function is supported inside the patch, so these rows only
            # see the patch cells and equal the interior rows of A-bar_j.
            return b[inn] - self.A[inn] @ u
        if v in self.closure:
            return b[inn] - self.closure[v] @ u[clo]
        Abar = patch_closure_matrix(self.solvers[v].patch, self.p)
        mask = self.solvers[v].patch.interior_mask(self.p)
        return b[inn] - (Abar @ u[clo])[mask]

    def additive_sweep(self, u, b, theta):
        """The additive variant: every patch's correction from the same
        iterate u, u + theta sum_j Pi_j^T d_j with d_j the local V-cycle
        solution for the local residual of u (all patches in one phase,
        damped by theta); returns the updated copy of u."""
        u = np.array(u, dtype=np.float64, copy=True)
        corr = np.zeros_like(u)
        for v in self.order:
            d = self.solvers[v].solve(self.local_residual(v, u, b))
            corr[self.idx[v][1]] += d
        return u + theta * corr

    def sweep(self, u, b, direction=+1, exact=False):
        """One multiplicative sweep; returns the updated copy of u."""
        u = np.array(u, dtype=np.float64, copy=True)
        order = self.order if direction > 0 else list(reversed(self.order))
        for v in order:
            r = self.local_residual(v, u, b)
            s = self.solvers[v]
            d = s.exact_solve(r) if exact else s.solve(r)
            u[self.idx[v][1]] += d
        return u
