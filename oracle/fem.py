"""Multilinear cells, element matrices and their assembly on patches and meshes.

TEST INFRASTRUCTURE (oracle): see oracle/__init__.py.

The operator is the variable-coefficient Poisson form of the paper
(Section 2, bilinear form): a(u, v) = int mu grad u . grad v, with A the
matrix of a(.,.) on the nodal basis (Section 2, discrete problem).  Every
matrix below is formed explicitly from that definition:

    A^K_ab = sum_k w_k mu_K det J_k (J_k^{-T} grad phi_a(xi_k)) . (J_k^{-T} grad phi_b(xi_k))

with J_k the Jacobian of the cell's multilinear map at Gauss point xi_k.

Index conventions (all x fastest):
  * reference tensor basis a = sum_i a_i n^i, n = q+1;
  * cell corners c = sum_i b_i 2^i;
  * global node g = sum_i g_i (N q + 1)^i with g_i = e_i q + a_i on cell e.
"""
from __future__ import annotations

import functools
import itertools

import numpy as np
import scipy.sparse as sp

from . import fe1d


def _multi(n: int, dim: int):
    """All multi-indices of [0,n)^dim in x-fastest order."""
    return [tuple(reversed(t)) for t in itertools.product(range(n), repeat=dim)]


@functools.lru_cache(maxsize=None)
def reference_gradients(q: int, dim: int):
    """Reference gradients of the degree-q tensor basis at the (q+1)^dim Gauss
    points.  Returns (grad (npts, nbasis, dim), weights (npts,), points
    (npts, dim))."""
    nodes = fe1d.gll_nodes(q)
    xg, wg = fe1d.gauss_rule(q + 1)
    L = fe1d.lagrange_values(nodes, xg)       # L[a, k] = l_a(x_k)
    D = fe1d.lagrange_derivatives(nodes, xg)  # D[a, k] = l_a'(x_k)
    idx = _multi(q + 1, dim)
    npt = len(idx)
    grad = np.zeros((npt, npt, dim))
    w = np.zeros(npt)
    pts = np.zeros((npt, dim))
    for k, kk in enumerate(idx):
        w[k] = np.prod([wg[kk[i]] for i in range(dim)])
        pts[k] = [xg[kk[i]] for i in range(dim)]
        for a, aa in enumerate(idx):
            for i in range(dim):
                val = 1.0
                for j in range(dim):
                    val *= D[aa[j], kk[j]] if j == i else L[aa[j], kk[j]]
                grad[k, a, i] = val
    return grad, w, pts


def corner_shape_gradients(points: np.ndarray) -> np.ndarray:
    """Reference gradients of the 2^dim multilinear corner functions
    N_c(xi) = prod_i (b_i ? xi_i : 1 - xi_i) at the given points:
    shape (npts, 2^dim, dim)."""
    npt, dim = points.shape
    out = np.zeros((npt, 2 ** dim, dim))
    for c in range(2 ** dim):
        bits = [(c >> i) & 1 for i in range(dim)]
        for k in range(dim):
            val = np.ones(npt)
            for i in range(dim):
                if i == k:
                    val *= 1.0 if bits[i] else -1.0
                else:
                    val *= points[:, i] if bits[i] else 1.0 - points[:, i]
            out[:, c, k] = val
    return out


def jacobians(X: np.ndarray, points: np.ndarray) -> np.ndarray:
    """Jacobians dF/dxi of multilinear cells at reference points.
    X: (ncell, 2^dim, dim) corner coordinates.  Returns (ncell, npts, dim, dim)
    with J[..., r, s] = d x_r / d xi_s."""
    dN = corner_shape_gradients(points)              # (npt, 2^d, d)
    return np.einsum("ecr,kcs->ekrs", X, dN)


@functools.lru_cache(maxsize=None)
def subcell_gradients(q: int, dim: int, s: int, sub: tuple):
    """The degree-q tensor basis of a cell and its reference gradients at
    the Gauss points of the sub-box sub of its reference cube cut into s^dim
    boxes (q+1 points per direction in each, weights scaled by 1/s per
    direction): the composite rule of a coarse cell whose coefficient is
    piecewise constant on those boxes.  Same returns as reference_gradients."""
    nodes = fe1d.gll_nodes(q)
    xg, wg = fe1d.gauss_rule(q + 1)
    per = [((sub[i] + xg) / s, wg / s) for i in range(dim)]
    Ls = [fe1d.lagrange_values(nodes, per[i][0]) for i in range(dim)]
    Ds = [fe1d.lagrange_derivatives(nodes, per[i][0]) for i in range(dim)]
    idx = _multi(q + 1, dim)
    npt = len(idx)
    grad = np.zeros((npt, npt, dim))
    w = np.zeros(npt)
    pts = np.zeros((npt, dim))
    for k, kk in enumerate(idx):
        w[k] = np.prod([per[i][1][kk[i]] for i in range(dim)])
        pts[k] = [per[i][0][kk[i]] for i in range(dim)]
        for a, aa in enumerate(idx):
            for i in range(dim):
                val = 1.0
                for j in range(dim):
                    val *= Ds[j][aa[j], kk[j]] if j == i else Ls[j][aa[j], kk[j]]
                grad[k, a, i] = val
    return grad, w, pts


def element_matrices(X: np.ndarray, mu: np.ndarray, q: int) -> np.ndarray:
    """Element matrices of a(.,.) for a batch of cells.

    X : (ncell, 2^dim, dim) corner coordinates, mu : (ncell,) coefficients,
    or (ncell, s^dim) coefficients constant on the s^dim boxes of each cell's
    reference cube (x fastest), integrated box by box with the q+1-point
    Gauss rule (the octant rule of coarse cells).
    Returns (ncell, n^dim, n^dim) with n = q+1, rows/columns in reference
    tensor order.
    """
    X = np.asarray(X, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    dim = X.shape[2]
    if mu.ndim == 2:
        s = int(round(mu.shape[1] ** (1.0 / dim)))
        if s ** dim != mu.shape[1]:
            raise ValueError("box coefficients must come in s^dim per cell")
        out = 0.0
        for b, sub in enumerate(_multi(s, dim)):
            out = out + _element_matrices_rule(X, mu[:, b], subcell_gradients(q, dim, s, sub))
        return out
    return _element_matrices_rule(X, mu, reference_gradients(q, dim))


def _element_matrices_rule(X: np.ndarray, mu: np.ndarray, rule) -> np.ndarray:
    """sum_k mu w_k (J_k^{-T} grad phi_a) . (J_k^{-T} grad phi_b) det J_k over
    the points of the rule (grad, w, pts)."""
    ncell = X.shape[0]
    grad, w, pts = rule
    npt, nb, dim = grad.shape
    out = np.zeros((ncell, nb, nb))
    J = jacobians(X, pts)                           # (ncell, npt, d, d)
    detJ = np.linalg.det(J)
    if np.any(detJ <= 0.0):
        raise ValueError("cell with non-positive Jacobian determinant")
    Jinv = np.linalg.inv(J)                         # d xi / d x
    # G_k = mu w_k det J_k J_k^{-1} J_k^{-T}
    G = np.einsum("eksr,ektr->ekst", Jinv, Jinv) * (mu[:, None, None, None]
                                                      * (w[None, :] * detJ)[:, :, None, None])
    # A_ab = sum_k sum_st grad[k,a,s] G[k,s,t] grad[k,b,t]
    gr = grad.transpose(1, 0, 2).reshape(nb, npt * dim)          # (a, k s)
    for e in range(ncell):
        M = np.einsum("kst,kbt->ksb", G[e], grad).reshape(npt * dim, nb)
        out[e] = gr @ M
    return out


# ---------------------------------------------------------------------------
# patches
# ---------------------------------------------------------------------------

class PatchGeometry:
    """A vertex patch: the cells around one vertex (Section 2.1).

    verts : (3^dim, dim) patch vertices, x fastest (entry t = sum t_i 3^i is
            the vertex at offset t in {0,1,2}^dim); in a direction with only
            one cell (a patch cut by the domain boundary) only offsets 0, 1
            are used
    mu    : (2^dim,) coefficient of cell c = sum c_i 2^i, or (2^dim, s^dim)
            coefficients per box of each cell (see element_matrices)
    ncell : cells per direction, each 1 or 2 (2 for a vertex in the interior)
    """

    def __init__(self, verts, mu, ncell=None):
        self.verts = np.asarray(verts, dtype=np.float64)
        self.dim = self.verts.shape[1]
        self.mu = np.asarray(mu, dtype=np.float64)
        self.ncell = tuple(ncell) if ncell is not None else (2,) * self.dim

    def cells(self):
        """Cells as multi-indices c in x-fastest order."""
        return [c for c in _multi(2, self.dim)
                if all(c[i] < self.ncell[i] for i in range(self.dim))]

    def cell_corners(self, c):
        rows = []
        for k in range(2 ** self.dim):
            t = [c[i] + ((k >> i) & 1) for i in range(self.dim)]
            rows.append(self.verts[sum(t[i] * 3 ** i for i in range(self.dim))])
        return np.array(rows)

    def cell_mu(self, c):
        return self.mu[sum(c[i] * 2 ** i for i in range(self.dim))]

    def closure_shape(self, q):
        return tuple(self.ncell[i] * q + 1 for i in range(self.dim))

    def interior_mask(self, q):
        """Closure nodes that are not on the patch boundary."""
        shp = self.closure_shape(q)
        idx = _multi_shape(shp)
        return np.array([all(0 < s[i] < shp[i] - 1 for i in range(self.dim)) for s in idx])


def _multi_shape(shp):
    dim = len(shp)
    return [tuple(reversed(t)) for t in itertools.product(*[range(shp[i]) for i in reversed(range(dim))])]


def patch_closure_matrix(P: PatchGeometry, q: int) -> np.ndarray:
    """A-bar_j: a(.,.) assembled on all closure nodes of the patch at degree q
    (Section 2.1, evaluate step).  Rows/columns in x-fastest closure order."""
    dim = P.dim
    shp = P.closure_shape(q)
    ntot = int(np.prod(shp))
    A = np.zeros((ntot, ntot))
    cells = P.cells()
    X = np.array([P.cell_corners(c) for c in cells])
    mu = np.array([P.cell_mu(c) for c in cells])
    Ke = element_matrices(X, mu, q)
    loc = _multi(q + 1, dim)
    for e, c in enumerate(cells):
        g = []
        for a in loc:
            s = [c[i] * q + a[i] for i in range(dim)]
            idx = 0
            for i in reversed(range(dim)):
                idx = idx * shp[i] + s[i]
            g.append(idx)
        g = np.array(g)
        A[np.ix_(g, g)] += Ke[e]
    return A


def patch_matrix(P: PatchGeometry, q: int) -> np.ndarray:
    """A_{j,q}: the patch operator on the interior nodes of the patch at degree
    q, i.e. the level operator obtained by rediscretising with the degree-q
    basis (Section 3.1, level operators)."""
    A = patch_closure_matrix(P, q)
    m = P.interior_mask(q)
    return A[np.ix_(m, m)]


# ---------------------------------------------------------------------------
# global meshes
# ---------------------------------------------------------------------------

class Mesh:
    """Structured mesh with n cells per direction and vertices from synth."""

    def __init__(self, dim: int, n: int, verts: np.ndarray, mu: np.ndarray):
        self.dim, self.n = dim, n
        self.verts = np.asarray(verts, dtype=np.float64)
        self.mu = np.asarray(mu, dtype=np.float64)

    def vertex(self, v):
        return self.verts[sum(v[i] * (self.n + 1) ** i for i in range(self.dim))]

    def cell_corners(self, e):
        return np.array([self.vertex([e[i] + ((k >> i) & 1) for i in range(self.dim)])
                         for k in range(2 ** self.dim)])

    def cell_mu(self, e):
        return self.mu[sum(e[i] * self.n ** i for i in range(self.dim))]

    def cells(self):
        return _multi(self.n, self.dim)

    def patch_start(self, v):
        """First cell index of the patch of vertex v per direction: the cells
        of the patch are {v_i - 1, v_i} intersected with the mesh (Section
        2.1), one cell in a direction where v lies on the boundary."""
        return [max(v[i] - 1, 0) for i in range(self.dim)]

    def patch_ncell(self, v):
        return tuple(2 if 0 < v[i] < self.n else 1 for i in range(self.dim))

    def patch(self, v) -> PatchGeometry:
        """The vertex patch around vertex v: all 2^dim cells for an interior
        vertex, the cells inside the mesh for a boundary vertex (entries of
        unused offsets are left at zero and never read)."""
        st, nc = self.patch_start(v), self.patch_ncell(v)
        verts = np.zeros((3 ** self.dim, self.dim))
        for t in _multi(3, self.dim):
            if all(t[i] <= nc[i] for i in range(self.dim)):
                verts[sum(t[i] * 3 ** i for i in range(self.dim))] = \
                    self.vertex([st[i] + t[i] for i in range(self.dim)])
        mu = np.zeros((2 ** self.dim,) + self.mu.shape[1:])
        for c in _multi(2, self.dim):
            if all(c[i] < nc[i] for i in range(self.dim)):
                mu[sum(c[i] * 2 ** i for i in range(self.dim))] = \
                    self.cell_mu([st[i] + c[i] for i in range(self.dim)])
        return PatchGeometry(verts, mu, nc)

    def coarsen(self, rule: str = "arithmetic") -> "Mesh":
        """Parent mesh with n/2 cells: vertices are the fine vertices with even
        indices (topological nesting, Section 2); a parent cell's coefficient
        is the arithmetic, geometric or harmonic mean of its 2^dim children,
        or with rule "octant" the children's coefficients themselves, kept
        per box of the parent's reference cube (s^dim boxes after k
        coarsenings, s = 2^k: the finest cells' coefficients), which
        element_matrices integrates box by box."""
        if self.n % 2:
            raise ValueError("odd mesh cannot be coarsened")
        nc = self.n // 2
        verts = np.array([self.vertex([2 * v[i] for i in range(self.dim)])
                          for v in _multi(nc + 1, self.dim)])
        if rule == "octant":
            fine = self.mu if self.mu.ndim == 2 else self.mu[:, None]
            s = int(round(fine.shape[1] ** (1.0 / self.dim)))
            mu = np.zeros((nc ** self.dim, (2 * s) ** self.dim))
            for e in _multi(nc, self.dim):
                ei = sum(e[i] * nc ** i for i in range(self.dim))
                for c in _multi(2, self.dim):
                    child = sum((2 * e[i] + c[i]) * self.n ** i for i in range(self.dim))
                    for t in _multi(s, self.dim):
                        box = sum((c[i] * s + t[i]) * (2 * s) ** i for i in range(self.dim))
                        mu[ei, box] = fine[child, sum(t[i] * s ** i for i in range(self.dim))]
            return Mesh(self.dim, nc, verts, mu)
        means = {"arithmetic": lambda x: np.mean(x),
                 "geometric": lambda x: np.exp(np.mean(np.log(x))),
                 "harmonic": lambda x: 1.0 / np.mean(1.0 / np.asarray(x))}
        mu = np.array([means[rule]([self.cell_mu([2 * e[i] + c[i] for i in range(self.dim)])
                                    for c in _multi(2, self.dim)])
                       for e in _multi(nc, self.dim)])
        return Mesh(self.dim, nc, verts, mu)


def global_node(g, m, dim):
    idx = 0
    for i in reversed(range(dim)):
        idx = idx * m + g[i]
    return idx


def dirichlet_mask(dim: int, n: int, p: int) -> np.ndarray:
    """True on interior (non-Dirichlet) global nodes."""
    m = n * p + 1
    return np.array([all(0 < g[i] < m - 1 for i in range(dim)) for g in _multi(m, dim)])


def assemble_global(mesh: Mesh, p: int, cell_batch: int = 512) -> sp.csr_matrix:
    """The full matrix of a(.,.) on all (N p + 1)^dim nodes, Dirichlet rows and
    columns included (they are masked by the caller)."""
    dim, n = mesh.dim, mesh.n
    m = n * p + 1
    cells = mesh.cells()
    loc = _multi(p + 1, dim)
    rows, cols, vals = [], [], []
    for start in range(0, len(cells), cell_batch):
        chunk = cells[start:start + cell_batch]
        X = np.array([mesh.cell_corners(e) for e in chunk])
        mu = np.array([mesh.cell_mu(e) for e in chunk])
        Ke = element_matrices(X, mu, p)
        for k, e in enumerate(chunk):
            g = np.array([global_node([e[i] * p + a[i] for i in range(dim)], m, dim) for a in loc])
            rows.append(np.repeat(g, len(g)))
            cols.append(np.tile(g, len(g)))
            vals.append(Ke[k].reshape(-1))
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(m ** dim, m ** dim))
    return A.tocsr()


def dirichlet_operator(mesh: Mesh, p: int) -> sp.csr_matrix:
    """A with Dirichlet rows and columns zeroed: x -> (A (x restricted to
    interior)) restricted to interior, on the full-length nodal vector."""
    A = assemble_global(mesh, p)
    mask = dirichlet_mask(mesh.dim, mesh.n, p).astype(np.float64)
    D = sp.diags(mask)
    return (D @ A @ D).tocsr()
