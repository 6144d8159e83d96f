"""Pins of the oracle's 1D ingredients, element matrices and patch assembly
against closed forms, exact integrals and invariants (no GPU)."""
import itertools
import math

import numpy as np
import pytest

from oracle import fe1d, fem
import synth


# ---------------------------------------------------------------------------
# 1D ingredients
# ---------------------------------------------------------------------------

def test_gll_nodes_closed_forms():
    assert np.allclose(fe1d.gll_nodes(1), [0.0, 1.0], atol=0, rtol=0)
    assert np.allclose(fe1d.gll_nodes(2), [0.0, 0.5, 1.0], atol=1e-15)
    s5 = 1.0 / math.sqrt(5.0)
    assert np.allclose(fe1d.gll_nodes(3), [0.0, (1 - s5) / 2, (1 + s5) / 2, 1.0], atol=1e-15)
    s37 = math.sqrt(3.0 / 7.0)
    assert np.allclose(fe1d.gll_nodes(4), [0.0, (1 - s37) / 2, 0.5, (1 + s37) / 2, 1.0], atol=1e-15)


@pytest.mark.parametrize("q", range(1, 16))
def test_gll_nodes_symmetric_sorted(q):
    x = fe1d.gll_nodes(q)
    assert len(x) == q + 1
    assert np.all(np.diff(x) > 0)
    assert np.allclose(x + x[::-1], 1.0, atol=1e-14)


def test_gauss_closed_forms():
    x, w = fe1d.gauss_rule(2)
    g = 1.0 / math.sqrt(3.0)
    assert np.allclose(x, [(1 - g) / 2, (1 + g) / 2], atol=1e-15)
    assert np.allclose(w, [0.5, 0.5], atol=1e-15)
    x, w = fe1d.gauss_rule(3)
    g = math.sqrt(3.0 / 5.0)
    assert np.allclose(x, [(1 - g) / 2, 0.5, (1 + g) / 2], atol=1e-15)
    assert np.allclose(w, [5 / 18, 8 / 18, 5 / 18], atol=1e-15)


@pytest.mark.parametrize("n", range(1, 17))
def test_gauss_exact_monomials(n):
    # n-point Gauss integrates x^k exactly on [0,1] for k <= 2n-1 (in particular
    # every degree-q polynomial at n = q+1 points), and not x^{2n}.
    x, w = fe1d.gauss_rule(n)
    for k in range(2 * n):
        assert abs(w @ x ** k - 1.0 / (k + 1)) < 1e-14
    if n <= 8:
        assert abs(w @ x ** (2 * n) - 1.0 / (2 * n + 1)) > 1e-12


@pytest.mark.parametrize("q", [1, 2, 3, 5, 8, 15])
def test_lagrange_partition_of_unity_and_derivatives(q):
    nodes = fe1d.gll_nodes(q)
    x = np.linspace(0, 1, 37)
    L = fe1d.lagrange_values(nodes, x)
    D = fe1d.lagrange_derivatives(nodes, x)
    assert np.allclose(L.sum(axis=0), 1.0, atol=1e-12)
    assert np.allclose(D.sum(axis=0), 0.0, atol=1e-9 * q ** 2)
    # Kronecker property at the nodes
    assert np.allclose(fe1d.lagrange_values(nodes, nodes), np.eye(q + 1), atol=1e-13)
    # reproduce a random polynomial of degree q and its derivative
    rng = np.random.default_rng(q)
    c = rng.standard_normal(q + 1)
    f = np.polynomial.Polynomial(c)
    assert np.allclose(f(nodes) @ L, f(x), atol=1e-10)
    assert np.allclose(f(nodes) @ D, f.deriv()(x), atol=1e-8 * q ** 2)


# ---------------------------------------------------------------------------
# element matrices
# ---------------------------------------------------------------------------

def _unit_cell(dim, h=1.0, shift=None):
    X = np.array([[h * ((c >> i) & 1) for i in range(dim)] for c in range(2 ** dim)], dtype=float)
    if shift is not None:
        X = X + shift
    return X


def test_q1_element_matrix_closed_form_2d():
    # bilinear stiffness on the unit square: diagonal 2/3, edge neighbours -1/6,
    # opposite corner -1/3 (standard Q1 Laplacian stencil)
    K = fem.element_matrices(_unit_cell(2)[None], np.ones(1), 1)[0]
    ref = np.array([[4, -1, -1, -2], [-1, 4, -2, -1], [-1, -2, 4, -1], [-2, -1, -1, 4]]) / 6.0
    assert np.allclose(K, ref, atol=1e-15)


@pytest.mark.parametrize("dim,q", [(2, 1), (2, 3), (3, 1), (3, 2)])
def test_element_matrix_symmetric_kernel_constants(dim, q):
    rng = np.random.default_rng(7)
    X = _unit_cell(dim) + 0.2 * rng.uniform(-1, 1, (2 ** dim, dim))
    K = fem.element_matrices(X[None], np.array([3.0]), q)[0]
    assert np.abs(K - K.T).max() <= 1e-14 * np.abs(K).max()
    assert np.abs(K @ np.ones(K.shape[0])).max() <= 1e-13 * np.abs(K).max()
    ev = np.linalg.eigvalsh(K)
    assert ev[0] > -1e-12 * ev[-1] and ev[1] > 1e-8 * ev[-1]   # only constants in the kernel


def test_element_matrix_scaling_3d():
    # on a cube of side h the Laplacian element matrix scales like h^{d-2}
    K1 = fem.element_matrices(_unit_cell(3)[None], np.ones(1), 2)[0]
    Kh = fem.element_matrices(_unit_cell(3, h=0.25)[None], np.ones(1), 2)[0]
    assert np.allclose(Kh, 0.25 * K1, atol=1e-14)


# ---------------------------------------------------------------------------
# patches
# ---------------------------------------------------------------------------

def _random_patch(dim, alpha=0.2, mu_log10=(-2, 2), seed=0):
    rng = np.random.Generator(np.random.PCG64(seed))
    X, mu = synth.make_random_patch(dim, alpha, mu_log10, rng)
    return fem.PatchGeometry(X, mu)


@pytest.mark.parametrize("dim,q", [(2, 1), (2, 3), (2, 5), (3, 1), (3, 2), (3, 3)])
def test_patch_matrix_spd(dim, q):
    A = fem.patch_matrix(_random_patch(dim, seed=q), q)
    assert A.shape == ((2 * q - 1) ** dim,) * 2
    assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()
    np.linalg.cholesky(A)
    assert np.linalg.eigvalsh(A)[0] > 0


@pytest.mark.parametrize("dim,q", [(2, 2), (2, 4), (3, 2), (3, 3)])
def test_patch_linear_functions(dim, q):
    # patch test: with constant mu on a multilinear patch, the interpolant of
    # any linear function is annihilated by the interior rows (the Gauss rule
    # with q+1 points is exact for these integrands)
    P = _random_patch(dim, alpha=0.25, mu_log10=None, seed=11 + q)
    Abar = fem.patch_closure_matrix(P, q)
    mask = P.interior_mask(q)
    # physical coordinates of the closure nodes
    nodes = fe1d.gll_nodes(q)
    shp = P.closure_shape(q)
    coords = []
    for s in fem._multi_shape(shp):
        c = tuple(min(s[i] // q, P.ncell[i] - 1) for i in range(dim))
        xi = np.array([nodes[s[i] - c[i] * q] for i in range(dim)])
        N = [np.prod([xi[i] if (k >> i) & 1 else 1 - xi[i] for i in range(dim)]) for k in range(2 ** dim)]
        coords.append(np.array(N) @ P.cell_corners(c))
    coords = np.array(coords)
    a = np.array([0.3, -1.2, 0.7][:dim])
    u = coords @ a + 0.4
    res = (Abar @ u)[mask]
    assert np.abs(res).max() <= 1e-12 * np.abs(Abar).max() * np.abs(u).max()
    # the same function is not annihilated by the boundary rows in general
    assert np.abs((Abar @ u)[~mask]).max() > 1e-6


def test_patch_matrix_equals_global_block():
    # A_{j,p} = Pi_j A Pi_j^T: assembling on the patch cells equals the
    # interior block of the globally assembled matrix (independent indexing)
    from oracle.smoother import patch_indices
    w = synth.workload(1)
    X, mu, _ = synth.make_case(w, n=3)
    mu = 10.0 ** np.random.default_rng(1).uniform(-1, 1, mu.shape)
    mesh = fem.Mesh(3, 3, X, mu)
    A = fem.assemble_global(mesh, 2)
    for v in [(1, 1, 1), (2, 1, 2), (2, 2, 2)]:
        clo, inn = patch_indices(v, 2, 3, 3)
        Pj = fem.patch_matrix(mesh.patch(v), 2)
        assert np.allclose(A[np.ix_(inn, inn)].toarray(), Pj, atol=1e-13, rtol=0)
        Abar = fem.patch_closure_matrix(mesh.patch(v), 2)
        m = mesh.patch(v).interior_mask(2)
        assert np.allclose(A[np.ix_(inn, clo)].toarray(), Abar[m], atol=1e-13, rtol=0)


def test_coarse_scalar_closed_form():
    # Q1 patch on a Cartesian grid: the single interior entry is
    # (2/3) sum mu_K in 2D (any h) and (h/3) sum mu_K in 3D (coarse solver,
    # Section 3.1: the p = 1 operator is the scalar diagonal entry)
    mu2 = np.array([1.0, 2.0, 5.0, 0.5])
    h = 0.3
    X2 = np.array([[h * i, h * j] for j in range(3) for i in range(3)])
    A = fem.patch_matrix(fem.PatchGeometry(X2, mu2), 1)
    assert A.shape == (1, 1) and abs(A[0, 0] - 2.0 / 3.0 * mu2.sum()) < 1e-14
    mu3 = np.arange(1.0, 9.0)
    X3 = np.array([[h * i, h * j, h * k] for k in range(3) for j in range(3) for i in range(3)])
    A = fem.patch_matrix(fem.PatchGeometry(X3, mu3), 1)
    assert abs(A[0, 0] - h / 3.0 * mu3.sum()) < 1e-14
    A = fem.patch_matrix(fem.PatchGeometry(X3, np.ones(8)), 1)
    assert abs(A[0, 0] - 8.0 * h / 3.0) < 1e-15


def test_table1_dof_counts():
    # (2^L p + 1)^d reproduces every entry of the paper's Table 1
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "table1_dofs.txt")
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        d, p, L, printed = line.split()
        d, p, L = int(d), int(p), int(L)
        n = 2 ** L
        total = (n * p + 1) ** d
        if total <= 20000:
            # the oracle's global numbering has exactly this many nodes
            assert len(fem.dirichlet_mask(d, n, p)) == total
        scale = {"k": 1e3, "M": 1e6}.get(printed[-1], 1.0)
        val = float(printed.rstrip("kM")) * scale
        digits = len(printed.rstrip("kM").replace(".", "").lstrip("0"))
        assert abs(total - val) <= 0.5 * 10 ** (math.floor(math.log10(val)) - digits + 1), (line, total)


def test_boundary_patch_matrix_equals_global_block():
    # patches of boundary vertices keep only the cells inside the mesh
    # (Section 2.1): their interior block and evaluate rows still equal the
    # globally assembled matrix; face / edge / corner patches in 3D and edge /
    # corner patches in 2D
    from oracle.smoother import patch_indices
    for dim, n, verts in [(3, 3, [(0, 1, 2), (3, 0, 1), (0, 3, 0), (3, 3, 3), (1, 0, 2)]),
                          (2, 4, [(0, 2), (4, 0), (0, 0), (2, 4)])]:
        X = synth.make_vertices(dim, n, 0.2, 5)
        mu = 10.0 ** np.random.default_rng(2).uniform(-1, 1, n ** dim)
        mesh = fem.Mesh(dim, n, X, mu)
        A = fem.assemble_global(mesh, 2)
        for v in verts:
            clo, inn = patch_indices(v, 2, n, dim)
            P = mesh.patch(v)
            k = [2 if 0 < v[i] < n else 1 for i in range(dim)]
            assert len(inn) == np.prod([k[i] * 2 - 1 for i in range(dim)])
            Pj = fem.patch_matrix(P, 2)
            assert np.allclose(A[np.ix_(inn, inn)].toarray(), Pj, atol=1e-13, rtol=0), v
            Abar = fem.patch_closure_matrix(P, 2)
            m = P.interior_mask(2)
            assert np.allclose(A[np.ix_(inn, clo)].toarray(), Abar[m], atol=1e-13, rtol=0), v
