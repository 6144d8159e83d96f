"""Pins of the oracle's simplicial patches (Section 3.2: 3 quadrilaterals in
2D, 4 hexahedra in 3D around one vertex), no GPU."""
import numpy as np
import pytest

import synth
from oracle import fe1d, fem, simplex
from oracle.fem import _multi
from oracle.pmg import LocalSolver


def _patch(dim, delta=0.2, seed=1):
    X, cells, mu = synth.make_simplex_patches(dim, 1, delta, seed)
    return X[0], cells, mu[0]


@pytest.mark.parametrize("dim,q", [(2, 1), (2, 2), (2, 3), (2, 7), (3, 1), (3, 2), (3, 3)])
def test_unknown_counts(dim, q):
    # interior of the patch: cell interiors, the faces and edges the cells
    # share, and the patch vertex
    X, cells, _ = _patch(dim)
    _, n = simplex.numbering(X, cells, q)
    m = q - 1
    expect = 3 * m * m + 3 * m + 1 if dim == 2 else 4 * m ** 3 + 6 * m * m + 4 * m + 1
    assert n == expect


def test_undeformed_cells_are_positively_oriented_and_cover_the_simplex():
    for dim in (2, 3):
        V, cells = synth.simplex_patch(dim)
        vol = 0.0
        for c in cells:
            J = fem.jacobians(V[c][None], np.full((1, dim), 0.5))[0, 0]
            assert np.linalg.det(J) > 0
            x, w = fe1d.gauss_rule(2)
            pts = np.array([[x[(g >> i) & 1] for i in range(dim)] for g in range(2 ** dim)])
            wt = np.array([np.prod([w[(g >> i) & 1] for i in range(dim)]) for g in range(2 ** dim)])
            vol += (np.linalg.det(fem.jacobians(V[c][None], pts)[0]) * wt).sum()
        # unit-edge triangle sqrt(3)/4, tetrahedron sqrt(2)/12
        assert vol == pytest.approx(np.sqrt(3) / 4 if dim == 2 else np.sqrt(2) / 12, rel=1e-13)


@pytest.mark.parametrize("dim,q", [(2, 3), (2, 5), (3, 2), (3, 3)])
def test_spd(dim, q):
    X, cells, mu = _patch(dim, 0.25, 3)
    A = simplex.level_matrix(X, cells, mu * np.array([1.0, 30.0, 0.2, 4.0][:len(cells)]), q)
    assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()
    assert np.linalg.eigvalsh(A).min() > 0


@pytest.mark.parametrize("dim,q", [(2, 2), (2, 4), (3, 2), (3, 3)])
def test_patch_test(dim, q):
    # a physically linear function lies in the space on multilinear cells;
    # the interior rows of the operator applied to it vanish (the integrand
    # adj(J) grad phi is a polynomial the Gauss rule integrates exactly)
    X, cells, _ = _patch(dim, 0.25, 5)
    gather, n = simplex.numbering(X, cells, q)
    a_lin = np.array([0.7, -1.3, 0.4][:dim])
    Ke = fem.element_matrices(X[cells], np.ones(len(cells)), q)
    rows = np.zeros(n)
    scale = 0.0
    for c, corners in enumerate(cells):
        u = simplex.cell_nodes(X[corners], q) @ a_lin + 2.0
        f = Ke[c] @ u
        m = gather[c] >= 0
        np.add.at(rows, gather[c][m], f[m])
        scale = max(scale, np.abs(Ke[c]).max() * np.abs(u).max())
    assert np.abs(rows).max() <= 1e-12 * scale


def test_undeformed_triangle_patch_is_invariant_under_rotation():
    # the 120-degree rotation maps cell k onto cell k+1 node by node (the
    # construction is cyclic); the operator of the undeformed patch with one
    # coefficient commutes with the induced permutation of the unknowns
    V, cells = synth.simplex_patch(2)
    for q in (2, 3, 5):
        gather, n = simplex.numbering(V, cells, q)
        A = simplex.level_matrix(V, cells, np.ones(3), q)
        perm = np.full(n, -1)
        for c in range(3):
            for a in range((q + 1) ** 2):
                if gather[c, a] >= 0:
                    perm[gather[c, a]] = gather[(c + 1) % 3, a]
        assert sorted(perm) == list(range(n))
        assert np.abs(A[np.ix_(perm, perm)] - A).max() <= 1e-13 * np.abs(A).max()
        # a Cartesian-style assembly would not see this symmetry with a wrong
        # identification of the shared edges: the permutation is a bijection


@pytest.mark.parametrize("dim,p", [(2, 3), (2, 7), (3, 3)])
def test_degree_one_prolongation_is_the_vertex_hat(dim, p):
    # the one unknown at degree 1 is the patch vertex, the last corner of
    # every cell: its basis function is prod_i xi_i in each cell, so P_{1->p}
    # holds that product at every fine node
    X, cells, _ = _patch(dim)
    P = simplex.prolongation(X, cells, p, 1)
    gather, n = simplex.numbering(X, cells, p)
    assert P.shape == (n, 1)
    x = fe1d.gll_nodes(p)
    for c in range(len(cells)):
        for a, aa in enumerate(_multi(p + 1, dim)):
            if gather[c, a] >= 0:
                assert P[gather[c, a], 0] == pytest.approx(np.prod([x[i] for i in aa]), abs=1e-14)


def test_prolongations_nest():
    X, cells, _ = _patch(2, 0.2, 7)
    P73 = simplex.prolongation(X, cells, 7, 3)
    P31 = simplex.prolongation(X, cells, 3, 1)
    P71 = simplex.prolongation(X, cells, 7, 1)
    assert np.abs(P73 @ P31 - P71).max() <= 1e-13
    X3, cells3, _ = _patch(3, 0.2, 8)
    P42 = simplex.prolongation(X3, cells3, 4, 2)
    P21 = simplex.prolongation(X3, cells3, 2, 1)
    assert np.abs(P42 @ P21 - simplex.prolongation(X3, cells3, 4, 1)).max() <= 1e-13


def test_vcycle_symmetric_linear_and_convergent():
    X, cells, mu = _patch(2, 0.2, 9)
    s = simplex.SimplexSolver(X, cells, mu, (3, 1))
    s.set_bounds([(0.2, 2.0)])
    n = s.A[0].shape[0]
    rng = np.random.default_rng(0)
    r1, r2 = rng.standard_normal(n), rng.standard_normal(n)
    assert r2 @ s.solve(r1) == pytest.approx(r1 @ s.solve(r2), rel=1e-12)
    assert np.allclose(s.solve(2 * r1 + r2), 2 * s.solve(r1) + s.solve(r2), atol=1e-13)
    s.n_vcycles = 80
    assert np.abs(s.solve(r1) - np.linalg.solve(s.A[0], r1)).max() <= 1e-8 * np.abs(np.linalg.solve(s.A[0], r1)).max()


def test_cg_iterations_grow_with_degree_like_the_cartesian_patch():
    # Section 3.2: on the undeformed simplicial 2D patch the Jacobi-smoothed
    # V-cycle preconditioner shows a growth with p similar to the Cartesian
    # patch's (no numbers are printed for either: the counts of both are
    # compared here, and the Cartesian ones are pinned to the paper's
    # "about 10 to 23" elsewhere)
    V, cells = synth.simplex_patch(2)
    omega = [(0.5, 3.5 / 1.1)]
    counts = {}
    for levels in ((3, 1), (7, 3, 1), (15, 7, 3, 1)):
        s = simplex.SimplexSolver(V, cells, np.ones(3), levels, cheb_degree=1)
        s.set_bounds(omega * (len(levels) - 1))
        b = np.random.default_rng(levels[0]).standard_normal(s.A[0].shape[0])
        _, k, rel = s.pcg(b, 1e-8, 100)
        assert rel <= 1e-8
        g = np.array(np.meshgrid(np.arange(3.0), np.arange(3.0), indexing="ij"))
        Xc = np.stack([g[1].reshape(-1), g[0].reshape(-1)], 1) * 0.5
        c = LocalSolver(fem.PatchGeometry(Xc, np.ones(4)), levels, cheb_degree=1)
        c.set_bounds(omega * (len(levels) - 1))
        bc = np.random.default_rng(levels[0]).standard_normal(c.A[0].shape[0])
        counts[levels[0]] = (k, c.pcg(bc, 1e-8, 100)[1])
    ks, kc = [counts[p][0] for p in (3, 7, 15)], [counts[p][1] for p in (3, 7, 15)]
    assert ks[0] < ks[1] < ks[2]
    growth_s, growth_c = ks[2] / ks[0], kc[2] / kc[0]
    assert 0.6 * growth_c <= growth_s <= 1.6 * growth_c, (ks, kc)
