"""Seeded workloads: structured quad/hex meshes with perturbed interior vertices,
per-cell coefficients and random right-hand sides.

The problem class is the variable-coefficient Poisson problem of the paper
(Section 2, bilinear form a(u,v) = int mu grad u . grad v) on the unit square
or cube, with homogeneous Dirichlet conditions.  The paper's experiments are
all synthetic (random vertex displacements, coefficient jumps, random
right-hand sides; Section 3.2 and Section 4), so every input here is drawn from
a fixed seed with numpy's PCG64.

Conventions shared by every consumer of these arrays:
  * vertices: shape ((N+1)^d, d), lexicographic with x fastest; vertex
    v = (v_0, .., v_{d-1}) sits at row sum_i v_i (N+1)^i.  Boundary vertices are
    never moved.
  * coefficients: shape (N^d,), one value per cell, lexicographic, x fastest.
  * right-hand side: shape ((N p + 1)^d,), the global nodal vector of a
    continuous Q_p space, x fastest, zero on Dirichlet nodes.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Tuple

import numpy as np


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic test problem.

    name      : short identifier used by tests and the bench
    dim       : 2 or 3
    n         : cells per direction of the finest mesh
    p         : polynomial degree of the fine space
    levels    : local p-multigrid degrees, descending, ending in 1
    alpha     : vertex perturbation, as a fraction of h, per coordinate
    mu_log10  : None for mu = 1, else (lo, hi) for mu = 10^U(lo, hi) per cell
    rtol      : relative residual tolerance of the outer CG
    cfg       : index used to derive the seeds (mesh 1000+cfg, mu 2000+cfg,
                rhs 3000+cfg)
    """

    name: str
    dim: int
    n: int
    p: int
    levels: Tuple[int, ...]
    alpha: float
    mu_log10: Optional[Tuple[float, float]]
    rtol: float
    cfg: int

    @property
    def mesh_seed(self) -> int:
        return 1000 + self.cfg

    @property
    def coef_seed(self) -> int:
        return 2000 + self.cfg

    @property
    def rhs_seed(self) -> int:
        return 3000 + self.cfg

    @property
    def n_dofs(self) -> int:
        return (self.n * self.p + 1) ** self.dim

    @property
    def n_interior_dofs(self) -> int:
        return (self.n * self.p - 1) ** self.dim

    @property
    def n_patches(self) -> int:
        return (self.n - 1) ** self.dim

    def scaled(self, n: int, name: Optional[str] = None) -> "Workload":
        """Same degree, levels, distortion and coefficient law on an n^d mesh."""
        return dataclasses.replace(self, n=n, name=name or f"{self.name}-n{n}")


WORKLOADS: List[Workload] = [
    # 2D, 8x8 affine quads, Q3, mu = 1, levels 3 -> 2 -> 1, CG to 1e-10.
    Workload("2d-n8-q3", 2, 8, 3, (3, 2, 1), 0.0, None, 1e-10, 1),
    # 3D, 16^3 hexes perturbed by up to 0.2 h per coordinate, Q4, mu = 1.
    Workload("3d-n16-q4", 3, 16, 4, (4, 2, 1), 0.2, None, 1e-8, 2),
    # 3D, 32^3 hexes perturbed by 0.25 h, Q7, mu log-uniform in [1e-4, 1e4].
    Workload("3d-n32-q7-jump", 3, 32, 7, (7, 3, 1), 0.25, (-4.0, 4.0), 1e-8, 3),
    # 3D, 24^3 hexes perturbed by 0.2 h, one instance per degree 2, 4, 6, 8.
    Workload("3d-n24-q8-batch", 3, 24, 8, (8, 4, 2, 1), 0.2, None, 1e-8, 4),
    # 3D, 32^3 hexes perturbed by 0.3 h, Q6, mu log-uniform in [1e-2, 1e2].
    Workload("3d-n32-q6-learned", 3, 32, 6, (6, 3, 1), 0.3, (-2.0, 2.0), 1e-8, 5),
]


def workload(name_or_index) -> Workload:
    if isinstance(name_or_index, int):
        return WORKLOADS[name_or_index]
    for w in WORKLOADS:
        if w.name == name_or_index:
            return w
    raise KeyError(name_or_index)


# ---------------------------------------------------------------------------
# mesh
# ---------------------------------------------------------------------------

def _corner_rows(dim: int, n1: int, cells: np.ndarray) -> np.ndarray:
    """Vertex rows of the 2^dim corners of each cell; cells has shape (k, dim)
    (x index first).  Corner c = sum_i b_i 2^i."""
    out = np.zeros((cells.shape[0], 2 ** dim), dtype=np.int64)
    for k in range(2 ** dim):
        idx = np.zeros(cells.shape[0], dtype=np.int64)
        for i in reversed(range(dim)):
            idx = idx * n1 + cells[:, i] + ((k >> i) & 1)
        out[:, k] = idx
    return out


def _min_jacobian(X: np.ndarray, dim: int) -> np.ndarray:
    """Smallest Jacobian determinant of multilinear cells, sampled at their
    corners and at a 3-point Gauss grid.  X has shape (k, 2^dim, dim).  Used
    only to reject tangled cells while drawing a mesh."""
    g = 0.5 * np.sqrt(3.0 / 5.0)
    pts1 = [0.0, 0.5 - g, 0.5, 0.5 + g, 1.0]
    best = np.full(X.shape[0], np.inf)
    for xi in np.array(np.meshgrid(*([pts1] * dim), indexing="ij")).reshape(dim, -1).T:
        J = np.zeros((X.shape[0], dim, dim))
        for c in range(2 ** dim):
            bits = [(c >> i) & 1 for i in range(dim)]
            for k in range(dim):
                dphi = 1.0
                for i in range(dim):
                    if i == k:
                        dphi *= 1.0 if bits[i] else -1.0
                    else:
                        dphi *= xi[i] if bits[i] else 1.0 - xi[i]
                J[:, :, k] += X[:, c, :] * dphi
        best = np.minimum(best, np.linalg.det(J))
    return best


def _min_jacobian_batched(X: np.ndarray, dim: int, chunk: int = 4096) -> np.ndarray:
    """Same sample points and result as _min_jacobian, computed with one
    contraction per chunk of cells."""
    g = 0.5 * np.sqrt(3.0 / 5.0)
    pts1 = np.array([0.0, 0.5 - g, 0.5, 0.5 + g, 1.0])
    P = np.array(np.meshgrid(*([pts1] * dim), indexing="ij")).reshape(dim, -1).T   # (npt, d)
    dN = np.zeros((P.shape[0], 2 ** dim, dim))
    for c in range(2 ** dim):
        bits = [(c >> i) & 1 for i in range(dim)]
        for k in range(dim):
            v = np.ones(P.shape[0])
            for i in range(dim):
                if i == k:
                    v = v * (1.0 if bits[i] else -1.0)
                else:
                    v = v * (P[:, i] if bits[i] else 1.0 - P[:, i])
            dN[:, c, k] = v
    out = np.empty(X.shape[0])
    for s0 in range(0, X.shape[0], chunk):
        Xc = X[s0:s0 + chunk]
        dNm = dN.transpose(1, 0, 2).reshape(2 ** dim, -1)          # (corner, point*d)
        J = np.stack([(Xc[:, :, r] @ dNm).reshape(Xc.shape[0], P.shape[0], dim)
                      for r in range(dim)], axis=2)                 # (cell, point, r, s)
        if dim == 3:
            det = (J[..., 0, 0] * (J[..., 1, 1] * J[..., 2, 2] - J[..., 1, 2] * J[..., 2, 1])
                   - J[..., 0, 1] * (J[..., 1, 0] * J[..., 2, 2] - J[..., 1, 2] * J[..., 2, 0])
                   + J[..., 0, 2] * (J[..., 1, 0] * J[..., 2, 1] - J[..., 1, 1] * J[..., 2, 0]))
        else:
            det = J[..., 0, 0] * J[..., 1, 1] - J[..., 0, 1] * J[..., 1, 0]
        out[s0:s0 + chunk] = det.min(axis=1)
    return out


def _all_cells(dim: int, n: int) -> np.ndarray:
    g = np.array(np.meshgrid(*([np.arange(n)] * dim), indexing="ij"))
    return np.stack([g[i].transpose(tuple(reversed(range(dim)))).reshape(-1)
                     for i in range(dim)], axis=1)


def make_vertices(dim: int, n: int, alpha: float, seed: int,
                  det_floor: float = 0.05, max_redraws: int = 10000) -> np.ndarray:
    """Structured mesh of the unit square/cube with n cells per direction.

    Every interior vertex is moved by an independent U(-alpha h, alpha h) draw
    per coordinate (the paper moves each interior vertex randomly, Section 3.2
    and Section 4; the per-coordinate law is the workload recipe of this package).
    Draws happen for all vertices in lexicographic order, coordinates innermost;
    boundary draws are discarded.  Cells whose sampled Jacobian determinant
    falls to det_floor * h^dim or below get the displacements of their interior
    vertices redrawn from the continuing stream, cells in lexicographic order
    and corners in order (the paper excludes degenerate patches, Section 3.2),
    until no such cell is left.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    h = 1.0 / n
    n1 = n + 1
    coords = _all_cells(dim, n1)
    base = coords.astype(np.float64) * h
    interior = np.all((coords > 0) & (coords < n), axis=1)
    delta = rng.uniform(-alpha * h, alpha * h, size=base.shape)
    delta[~interior] = 0.0
    if alpha == 0.0:
        return base.copy()
    cells = _all_cells(dim, n)
    corners = _corner_rows(dim, n1, cells)
    floor = det_floor * h ** dim
    check = np.arange(cells.shape[0])
    for _ in range(max_redraws):
        verts = base + delta
        # only cells touching a redrawn vertex can change; the others passed
        bad = check[_min_jacobian(verts[corners[check]], dim) <= floor]
        if bad.size == 0:
            return verts
        moved = []
        for c in bad:
            for vi in corners[c]:
                if interior[vi]:
                    delta[vi] = rng.uniform(-alpha * h, alpha * h, size=dim)
                    moved.append(vi)
        touched = set()
        for vi in set(moved):
            v = coords[vi]
            for k in range(2 ** dim):
                c = v - np.array([(k >> i) & 1 for i in range(dim)])
                if np.all((c >= 0) & (c < n)):
                    touched.add(int(sum(int(c[i]) * n ** i for i in range(dim))))
        check = np.array(sorted(touched), dtype=np.int64)
    raise RuntimeError("could not draw a mesh without degenerate cells")


def make_coefficients(dim: int, n: int, mu_log10, seed: int) -> np.ndarray:
    """Per-cell coefficient mu: 1 everywhere, or 10^U(lo, hi) i.i.d. per cell
    (the paper's coefficient-jump studies use piecewise constant mu,
    Section 3.2)."""
    if mu_log10 is None:
        return np.ones(n ** dim)
    rng = np.random.Generator(np.random.PCG64(seed))
    lo, hi = mu_log10
    return 10.0 ** rng.uniform(lo, hi, size=n ** dim)


def make_rhs(dim: int, n: int, p: int, seed: int) -> np.ndarray:
    """Random right-hand side: N(0,1) i.i.d. on interior nodes, zero on the
    Dirichlet boundary (the paper solves with a random right-hand side,
    Section 4)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = n * p + 1
    b = rng.standard_normal(m ** dim)
    g = np.array(np.meshgrid(*([np.arange(m)] * dim), indexing="ij"))
    on_bdry = np.zeros(m ** dim, dtype=bool)
    for i in range(dim):
        gi = g[i].transpose(tuple(reversed(range(dim)))).reshape(-1)
        on_bdry |= (gi == 0) | (gi == m - 1)
    b[on_bdry] = 0.0
    return b


def make_case(w: Workload, n: Optional[int] = None):
    """(vertices, coefficients, rhs) for workload w, optionally on an n^d mesh
    with the same seeds."""
    nn = w.n if n is None else n
    X = make_vertices(w.dim, nn, w.alpha, w.mesh_seed)
    mu = make_coefficients(w.dim, nn, w.mu_log10, w.coef_seed)
    b = make_rhs(w.dim, nn, w.p, w.rhs_seed)
    return X, mu, b


def make_random_patch(dim: int, alpha: float, mu_log10, rng: np.random.Generator,
                      det_floor: float = 0.05):
    """One isolated 2^dim-cell vertex patch on [0, 1]^dim (h = 1/2) with all
    3^dim vertices moved by U(-alpha h, alpha h) per coordinate, and per-cell
    mu.  Returns (vertices (3^dim, dim), mu (2^dim,)).  Used to build
    training sets of independent patches."""
    h = 0.5
    coords = _all_cells(dim, 3).astype(np.float64) * h
    corners = _corner_rows(dim, 3, _all_cells(dim, 2))
    while True:
        X = coords + rng.uniform(-alpha * h, alpha * h, size=coords.shape)
        if np.all(_min_jacobian(X[corners], dim) > det_floor * h ** dim):
            break
    if mu_log10 is None:
        mu = np.ones(2 ** dim)
    else:
        mu = 10.0 ** rng.uniform(mu_log10[0], mu_log10[1], size=2 ** dim)
    return X, mu


def make_random_patches(dim: int, n: int, alpha: float, mu_log10, seed: int,
                        det_floor: float = 0.05):
    """n independent patches as make_random_patch draws them, vectorised:
    all displacements are drawn first (patch-major, vertex, coordinate), then
    patches with a tangled cell are redrawn in index order from the continuing
    stream until none is left; the coefficients come last.  Returns
    (vertices (n, 3^dim, dim), mu (n, 2^dim))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    h = 0.5
    coords = _all_cells(dim, 3).astype(np.float64) * h
    corners = _corner_rows(dim, 3, _all_cells(dim, 2))      # (2^d cells, 2^d corners)
    X = coords[None] + rng.uniform(-alpha * h, alpha * h, size=(n,) + coords.shape)
    floor = det_floor * h ** dim
    todo = np.arange(n)
    for _ in range(10000):
        dets = _min_jacobian_batched(X[todo][:, corners].reshape(-1, 2 ** dim, dim), dim).reshape(todo.size, -1)
        todo = todo[dets.min(axis=1) <= floor]
        if todo.size == 0:
            break
        X[todo] = coords[None] + rng.uniform(-alpha * h, alpha * h, size=(todo.size,) + coords.shape)
    else:
        raise RuntimeError("could not draw untangled patches")
    if mu_log10 is None:
        mu = np.ones((n, 2 ** dim))
    else:
        mu = 10.0 ** rng.uniform(mu_log10[0], mu_log10[1], size=(n, 2 ** dim))
    return X, mu


def make_sphere_distorted_patches(dim: int, n: int, delta: float, seed: int,
                                  mu_cell: Optional[float] = None, det_floor: float = 0.01):
    """n independent patches (2^dim cells of width h = 0.5, as
    make_random_patches lays them out) whose 3^dim vertices are each moved
    by delta h in a direction drawn uniformly on the unit sphere (a normalised
    standard Gaussian vector): the distortion model of the single-patch study
    in Section 3.2.  A patch with a cell whose sampled Jacobian determinant is
    at most det_floor h^dim is redrawn from the continuing stream.
    Coefficients: 1 in every cell, cell 0 set to mu_cell when given.
    Returns (vertices (n, 3^dim, dim), mu (n, 2^dim))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    h = 0.5
    coords = _all_cells(dim, 3).astype(np.float64) * h
    corners = _corner_rows(dim, 3, _all_cells(dim, 2))

    def draw(k):
        d = rng.standard_normal((k,) + coords.shape)
        d /= np.linalg.norm(d, axis=-1, keepdims=True)
        return coords[None] + delta * h * d

    X = draw(n)
    floor = det_floor * h ** dim
    todo = np.arange(n)
    for _ in range(10000):
        dets = _min_jacobian_batched(X[todo][:, corners].reshape(-1, 2 ** dim, dim), dim).reshape(todo.size, -1)
        todo = todo[dets.min(axis=1) <= floor]
        if todo.size == 0:
            break
        X[todo] = draw(todo.size)
    else:
        raise RuntimeError("could not draw untangled patches")
    mu = np.ones((n, 2 ** dim))
    if mu_cell is not None:
        mu[:, 0] = mu_cell
    return X, mu


def make_sphere_distorted_mesh(dim: int, n: int, delta: float, seed: int,
                               det_floor: float = 0.01, max_redraws: int = 10000) -> np.ndarray:
    """Structured mesh of the unit square/cube with n cells per direction whose
    interior vertices are each moved by delta h (h = 1/n, the length of every
    edge at a vertex of the uniform mesh) in a direction drawn uniformly on
    the unit sphere (a normalised standard Gaussian vector): the distortion
    model of the global experiments in Section 4.  Draws happen for all
    vertices in lexicographic order; boundary draws are discarded.  Cells whose
    sampled Jacobian determinant falls to det_floor h^dim or below get the
    directions of their interior vertices redrawn from the continuing stream,
    until no such cell is left."""
    rng = np.random.Generator(np.random.PCG64(seed))
    h = 1.0 / n
    n1 = n + 1
    coords = _all_cells(dim, n1)
    base = coords.astype(np.float64) * h
    if delta == 0.0:
        return base.copy()
    interior = np.all((coords > 0) & (coords < n), axis=1)

    def draw(k):
        d = rng.standard_normal((k, dim))
        return delta * h * d / np.linalg.norm(d, axis=1, keepdims=True)

    disp = draw(base.shape[0])
    disp[~interior] = 0.0
    cells = _all_cells(dim, n)
    corners = _corner_rows(dim, n1, cells)
    floor = det_floor * h ** dim
    for _ in range(max_redraws):
        verts = base + disp
        bad = np.flatnonzero(_min_jacobian_batched(verts[corners], dim) <= floor)
        if bad.size == 0:
            return verts
        move = sorted({int(vi) for c in bad for vi in corners[c] if interior[vi]})
        disp[move] = draw(len(move))
    raise RuntimeError("could not draw a mesh without degenerate cells")


def simplex_patch(dim: int):
    """The undeformed simplicial vertex patch (Section 3.2): a triangle cut into
    3 quadrilaterals (2D) or a tetrahedron cut into 4 hexahedra (3D) around its
    centroid, the patch vertex.  Unit edge length; vertices in this order:
      2D: corners T0, T1, T2 (counter-clockwise), edge midpoints M01, M12,
          M20, centroid C  (7 vertices);
      3D: corners T0..T3 (positively oriented), edge midpoints M01, M02, M03,
          M12, M13, M23, face centroids F012, F013, F023, F123, centroid C
          (15 vertices).
    Cell k belongs to corner Tk; its corners are listed x fastest (corner
    sum_i b_i 2^i), corner 0 being Tk and the last one C; the edge (2D) or
    face (3D) midpoints follow in the order that makes the cell map
    positively oriented.  Returns (vertices (nv, dim), cells (dim + 1,
    2^dim) int), the cell corner lists indexing the vertices."""
    if dim == 2:
        T = np.array([[0.0, 0.0], [1.0, 0.0], [0.5, np.sqrt(3.0) / 2.0]])
        M = np.array([(T[0] + T[1]) / 2, (T[1] + T[2]) / 2, (T[2] + T[0]) / 2])
        C = T.mean(axis=0)
        V = np.vstack([T, M, C[None]])
        cells = np.array([[k, 3 + k, 3 + (k + 2) % 3, 6] for k in range(3)], dtype=np.int64)
        return V, cells
    if dim != 3:
        raise ValueError("dim must be 2 or 3")
    T = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.5, np.sqrt(3.0) / 2.0, 0.0],
                  [0.5, np.sqrt(3.0) / 6.0, np.sqrt(2.0 / 3.0)]])
    pairs = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    triples = [(0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)]
    M = np.array([(T[i] + T[j]) / 2 for i, j in pairs])
    F = np.array([(T[i] + T[j] + T[k]) / 3 for i, j, k in triples])
    C = T.mean(axis=0)
    V = np.vstack([T, M, F, C[None]])
    mid = {pr: 4 + i for i, pr in enumerate(pairs)}
    cen = {tr: 10 + i for i, tr in enumerate(triples)}
    cells = []
    for k in range(4):
        a, b, c = [j for j in range(4) if j != k]
        e = lambda j: mid[tuple(sorted((k, j)))]
        f = lambda i, j: cen[tuple(sorted((k, i, j)))]
        if np.linalg.det(np.array([V[e(a)] - V[k], V[e(b)] - V[k], V[e(c)] - V[k]])) < 0:
            b, c = c, b
        cells.append([k, e(a), e(b), f(a, b), e(c), f(a, c), f(b, c), 14])
    return V, np.array(cells, dtype=np.int64)


def make_simplex_patches(dim: int, n: int, delta: float, seed: int,
                         mu_cell: Optional[float] = None, det_floor: float = 0.01):
    """n simplicial patches (simplex_patch) whose vertices are each moved by
    delta h in a direction drawn uniformly on the unit sphere, h the shortest
    edge of the undeformed patch (the centroid's edges); a patch with a cell
    whose sampled Jacobian determinant is at most det_floor h^dim is redrawn
    from the continuing stream (the paper excludes degenerate patches,
    Section 3.2).  Coefficients 1, cell 0 set to mu_cell when given.
    Returns (vertices (n, nv, dim), cells (dim + 1, 2^dim), mu (n, dim + 1))."""
    V, cells = simplex_patch(dim)
    rng = np.random.Generator(np.random.PCG64(seed))
    edges = set()
    for c in cells:
        for b in range(2 ** dim):
            for i in range(dim):
                if not (b >> i) & 1:
                    edges.add(tuple(sorted((int(c[b]), int(c[b | (1 << i)])))))
    h = min(float(np.linalg.norm(V[i] - V[j])) for i, j in edges)

    def draw(k):
        d = rng.standard_normal((k,) + V.shape)
        d /= np.linalg.norm(d, axis=-1, keepdims=True)
        return V[None] + delta * h * d

    X = draw(n)
    floor = det_floor * h ** dim
    todo = np.arange(n)
    for _ in range(10000):
        dets = _min_jacobian_batched(X[todo][:, cells].reshape(-1, 2 ** dim, dim), dim).reshape(todo.size, -1)
        todo = todo[dets.min(axis=1) <= floor]
        if todo.size == 0:
            break
        X[todo] = draw(todo.size)
    else:
        raise RuntimeError("could not draw untangled simplicial patches")
    mu = np.ones((n, len(cells)))
    if mu_cell is not None:
        mu[:, 0] = mu_cell
    return X, cells, mu
