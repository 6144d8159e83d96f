"""Pins of the oracle's local p-multigrid, Chebyshev smoother, Lanczos bounds,
patch sweep and global multigrid (no GPU)."""
import os

import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import fe1d, fem, gmg, lanczos, pmg
from oracle.smoother import PatchSmoother, patch_order, vertex_color


def _patch(dim, alpha=0.2, mu_log10=(-2, 2), seed=0):
    rng = np.random.Generator(np.random.PCG64(seed))
    X, mu = synth.make_random_patch(dim, alpha, mu_log10, rng)
    return fem.PatchGeometry(X, mu)


def _affine_patch(dim, seed=0):
    # an affine image of the Cartesian patch (every cell a parallelogram)
    rng = np.random.default_rng(seed)
    B = np.eye(dim) + 0.3 * rng.uniform(-1, 1, (dim, dim))
    g = np.array(np.meshgrid(*([np.arange(3)] * dim), indexing="ij"))
    ref = np.stack([g[i].transpose(tuple(reversed(range(dim)))).reshape(-1)
                    for i in range(dim)], axis=1) * 0.5
    mu = 10.0 ** rng.uniform(-2, 2, 2 ** dim)
    return fem.PatchGeometry(ref @ B.T + 0.1, mu)


# ---------------------------------------------------------------------------
# transfers and level operators
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("p,q,r", [(4, 2, 1), (7, 3, 1), (8, 4, 2), (6, 3, 2), (15, 7, 3)])
def test_prolongation_nested(p, q, r):
    # V_r < V_q < V_p: embedding r->p equals embedding q->p after r->q
    A = pmg.prolongation_1d(p, q) @ pmg.prolongation_1d(q, r)
    assert np.allclose(A, pmg.prolongation_1d(p, r), atol=1e-13)
    if r >= 2:   # one-cell directions of boundary-cut patches
        A1 = pmg.prolongation_1d(p, q, 1) @ pmg.prolongation_1d(q, r, 1)
        assert np.allclose(A1, pmg.prolongation_1d(p, r, 1), atol=1e-13)


@pytest.mark.parametrize("p,q", [(3, 2), (4, 2), (7, 3), (5, 1)])
def test_prolongation_reproduces_piecewise_polynomials(p, q):
    # the coarse function with nodal values f(x_t) of a cellwise degree-q
    # polynomial f vanishing at the patch ends is reproduced at the fine nodes
    xq, xp = fe1d.gll_nodes(q), fe1d.gll_nodes(p)
    rng = np.random.default_rng(p * 10 + q)

    def fvals(nodes, deg):
        out = []
        for s in range(1, 2 * deg):
            c = min(s // deg, 1)
            xi = nodes[s - c * deg]
            out.append(cell_f(c, xi))
        return np.array(out)
    # cellwise polynomial of degree q with f(0)=f(2)=0 and continuity at 1:
    # f_0(xi) = xi * g0(xi), f_1(xi) = (1 - xi) * g1(xi), with g0(1) = g1(0)
    g0 = np.polynomial.Polynomial(rng.standard_normal(q))
    g1 = np.polynomial.Polynomial(rng.standard_normal(q))
    g1 = g1 - g1(0.0) + g0(1.0)
    X = np.polynomial.Polynomial([0, 1])
    f0, f1 = X * g0, (1 - X) * g1
    def cell_f(c, xi):
        return f0(xi) if c == 0 else f1(xi)
    coarse = fvals(xq, q)
    fine = fvals(xp, p)
    assert np.allclose(pmg.prolongation_1d(p, q) @ coarse, fine, atol=1e-12)


@pytest.mark.parametrize("dim,p,q", [(2, 3, 2), (2, 4, 2), (3, 2, 1), (3, 4, 2)])
def test_galerkin_equals_rediscretisation_affine(dim, p, q):
    # Section 3.1, level operators: P^T A_{j,p} P = A_{j,q} holds exactly on
    # affine patches with piecewise constant mu (exact quadrature)
    P = _affine_patch(dim, seed=p + q)
    Ap, Aq = fem.patch_matrix(P, p), fem.patch_matrix(P, q)
    Pr = pmg.prolongation(p, q, P.ncell)
    assert np.abs(Pr.T @ Ap @ Pr - Aq).max() <= 1e-12 * np.abs(Aq).max()


def test_galerkin_differs_on_distorted_patch():
    # on a genuinely trilinear patch the two differ (quadrature of rational
    # integrands); the method uses rediscretisation
    P = _patch(2, alpha=0.3, mu_log10=None, seed=3)
    Ap, Aq = fem.patch_matrix(P, 4), fem.patch_matrix(P, 2)
    Pr = pmg.prolongation(4, 2, P.ncell)
    assert np.abs(Pr.T @ Ap @ Pr - Aq).max() > 1e-8 * np.abs(Aq).max()


def test_coarse_level_equals_galerkin_diagonal_affine():
    # Section 3.1, coarse solver: the p = 1 scalar is the degree-one diagonal
    # entry, equal to the Galerkin projection of the fine operator
    P = _affine_patch(3, seed=5)
    A1 = fem.patch_matrix(P, 1)
    A3 = fem.patch_matrix(P, 3)
    Pr = pmg.prolongation(3, 1, P.ncell)
    assert A1.shape == (1, 1)
    assert abs((Pr.T @ A3 @ Pr)[0, 0] - A1[0, 0]) <= 1e-12 * A1[0, 0]


# ---------------------------------------------------------------------------
# Chebyshev smoothing
# ---------------------------------------------------------------------------

def test_chebyshev_error_polynomial():
    # e_k = tau_k(D^{-1}A) e_0, tau_k(lam) = T_k((theta - lam)/delta) / T_k(theta/delta)
    A = fem.patch_matrix(_patch(2, seed=4), 3)
    dinv = 1.0 / np.diag(A)
    lam, V = sla.eigh(A, np.diag(np.diag(A)))      # A v = lam D v
    rng = np.random.default_rng(0)
    xstar = rng.standard_normal(A.shape[0])
    f = A @ xstar
    x0 = rng.standard_normal(A.shape[0])
    a, b = 0.3, 1.1 * lam[-1]
    theta, delta = (a + b) / 2, (b - a) / 2
    for k in (1, 2, 3, 5):
        xk = pmg.chebyshev(A, dinv, f, x0, a, b, k)
        c0 = np.linalg.solve(V, xstar - x0)
        ck = np.linalg.solve(V, xstar - xk)
        Tk = np.polynomial.chebyshev.Chebyshev.basis(k)
        tau = Tk((theta - lam) / delta) / Tk(theta / delta)
        assert np.allclose(ck, tau * c0, atol=1e-9 * np.abs(c0).max())


def _eigen_contraction(A, dinv, a, b, k):
    """|tau_k(lambda)| of every eigenvector of D^{-1} A, measured by running
    the smoother on the error e_0 = v (f = 0)."""
    lam, V = sla.eigh(A, np.diag(1.0 / dinv))
    out = []
    for i in range(len(lam)):
        xk = pmg.chebyshev(A, dinv, np.zeros(len(lam)), V[:, i], a, b, k)
        out.append(np.linalg.norm(xk) / np.linalg.norm(V[:, i]))
    return lam, np.array(out)


def test_chebyshev_interval_targets_the_upper_spectrum():
    # Reading R5: the interval [max(lam_min, b/rho), b], b = s lam_max, makes
    # the degree-k smoother damp every eigenvector of D^{-1} A whose eigenvalue
    # lies in [b/rho, lam_max] by at least the Chebyshev minimax factor
    # 1/T_k((rho+1)/(rho-1)) (1/T_3(8/7) = 0.39334 for rho = 15) and amplify
    # none.  A patch whose D^{-1} A has eigenvalues far below b/rho exercises
    # the clamp: with a = lam_min instead, the polynomial equioscillates over
    # the whole spectrum and leaves part of the upper range almost undamped.
    A = fem.patch_matrix(_patch(2, seed=11), 4)
    dinv = 1.0 / np.diag(A)
    lam = sla.eigh(A, np.diag(np.diag(A)), eigvals_only=True)
    a, b = pmg.chebyshev_interval(lam[0], lam[-1])
    assert lam[0] < b / 15 / 2                     # the clamp is active here
    k = 3
    lam_v, tau = _eigen_contraction(A, dinv, a, b, k)
    T3 = lambda x: 4 * x ** 3 - 3 * x
    bound = 1.0 / T3(16.0 / 14.0)
    assert bound == pytest.approx(0.39334, abs=1e-5)
    upper = lam_v >= b / 15
    assert upper.sum() >= 10
    assert tau[upper].max() <= bound * (1 + 1e-9)
    assert tau.max() <= 1.0 + 1e-12
    # the factor is reached on the upper range (equioscillation), so the
    # interval is no wider than it needs to be
    assert tau[upper].max() >= 0.8 * bound


def test_chebyshev_interval_uses_lambda_min_when_it_is_large():
    # When the spectrum of D^{-1} A already lies inside [b/rho, b], the interval
    # starts at lam_min, and every eigenvector is damped by the minimax factor
    # of the tight interval, 1/T_k(theta/delta) with theta/delta =
    # (s lam_max + lam_min)/(s lam_max - lam_min): 1/T_3(8/3) = 0.014738 for
    # the spectrum [1, 2], far below the clamped interval's 0.393.
    rng = np.random.default_rng(5)
    n = 30
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.concatenate([[1.0, 2.0], rng.uniform(1.0, 2.0, n - 2)])
    d = rng.uniform(0.5, 4.0, n)                    # D = diag(A)
    M = Q @ np.diag(lam) @ Q.T                      # D^{-1/2} A D^{-1/2}
    A = np.sqrt(d)[:, None] * M * np.sqrt(d)[None, :]
    dinv = 1.0 / d                                  # scaling only: D^{-1} A ~ M
    a, b = pmg.chebyshev_interval(1.0, 2.0)
    assert a == pytest.approx(1.0)
    _, tau = _eigen_contraction(A, dinv, a, b, 3)
    T3 = lambda x: 4 * x ** 3 - 3 * x
    bound = 1.0 / T3((2.2 + 1.0) / (2.2 - 1.0))
    assert bound == pytest.approx(0.014738, abs=1e-6)
    assert tau.max() <= bound * (1 + 1e-9)


def test_chebyshev_degree_one_is_damped_jacobi():
    # k = 1 on an interval with a + b = 4 is the paper's Jacobi step with
    # omega = 1/2 (Section 3.1, smoothers; Section 3.2)
    A = fem.patch_matrix(_patch(3, seed=2), 2)
    dinv = 1.0 / np.diag(A)
    rng = np.random.default_rng(1)
    f, x0 = rng.standard_normal(A.shape[0]), rng.standard_normal(A.shape[0])
    x1 = pmg.chebyshev(A, dinv, f, x0, 0.5, 3.5, 1)
    assert np.allclose(x1, x0 + 0.5 * dinv * (f - A @ x0), atol=1e-14)


def test_chebyshev_zero_start_skips_apply():
    A = fem.patch_matrix(_patch(2, seed=8), 3)
    dinv = 1.0 / np.diag(A)
    f = np.random.default_rng(2).standard_normal(A.shape[0])
    x_a = pmg.chebyshev(A, dinv, f, np.zeros_like(f), 0.2, 2.0, 3, x_is_zero=True)
    x_b = pmg.chebyshev(A, dinv, f, np.zeros_like(f), 0.2, 2.0, 3)
    assert np.allclose(x_a, x_b, atol=1e-14)


# ---------------------------------------------------------------------------
# Lanczos bounds
# ---------------------------------------------------------------------------

def test_splitmix64_published_outputs():
    # reference outputs of SplitMix64 seeded with 0 and with 1234567
    assert [lanczos.splitmix64(0, i) for i in range(3)] == [
        0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    assert [lanczos.splitmix64(1234567, i) for i in range(3)] == [
        6457827717110365317, 3203168211198807973, 9817491932198370423]


def test_start_vector_range_and_independence():
    v = lanczos.start_vector(5, 100, 0, 4096)
    assert v.min() >= -1.0 and v.max() < 1.0 and abs(v.mean()) < 0.05
    w = lanczos.start_vector(5, 100, 1, 4096)
    assert abs(np.corrcoef(v, w)[0, 1]) < 0.1


@pytest.mark.parametrize("dim,q,m", [(2, 3, 12), (2, 4, 20), (3, 2, 12), (3, 2, 30)])
def test_lanczos_inside_spectrum(dim, q, m):
    A = fem.patch_matrix(_patch(dim, seed=q + m), q)
    dinv = 1.0 / np.diag(A)
    lo, hi = lanczos.bounds(A, dinv, m, seed=9, vertex=3, level=0)
    ev = np.linalg.eigvals(dinv[:, None] * A).real
    assert ev.min() - 1e-12 <= lo <= hi <= ev.max() + 1e-12
    # Gershgorin bound of D^{-1} A
    assert hi <= np.max(np.abs(A).sum(axis=1) * dinv) + 1e-12
    # the largest Ritz value converges fast
    assert hi >= 0.97 * ev.max()


def test_lanczos_exact_when_steps_reach_dimension():
    A = fem.patch_matrix(_patch(2, seed=1), 2)   # 9 x 9
    dinv = 1.0 / np.diag(A)
    lo, hi = lanczos.bounds(A, dinv, 9, seed=1, vertex=0, level=0)
    ev = np.sort(np.linalg.eigvals(dinv[:, None] * A).real)
    assert abs(lo - ev[0]) < 1e-10 and abs(hi - ev[-1]) < 1e-10


# ---------------------------------------------------------------------------
# V-cycle
# ---------------------------------------------------------------------------

def _solver(dim, levels, seed=0, k=3, nmg=1):
    P = _patch(dim, seed=seed)
    s = pmg.LocalSolver(P, levels, cheb_degree=k, n_vcycles=nmg)
    s.set_bounds([lanczos.bounds(s.A[l], s.dinv[l], 12, 1, seed, l) for l in range(len(levels) - 1)])
    return s


@pytest.mark.parametrize("dim,levels", [(2, (3, 2, 1)), (3, (4, 2, 1)), (3, (3, 1))])
def test_vcycle_linear_and_symmetric(dim, levels):
    s = _solver(dim, levels, seed=sum(levels))
    n = s.A[0].shape[0]
    rng = np.random.default_rng(3)
    r1, r2 = rng.standard_normal(n), rng.standard_normal(n)
    d1, d2 = s.solve(r1), s.solve(r2)
    assert np.allclose(s.solve(2.0 * r1 - 3.0 * r2), 2.0 * d1 - 3.0 * d2, atol=1e-12 * np.abs(d1).max())
    assert abs(r2 @ d1 - r1 @ d2) <= 1e-12 * abs(r1 @ d1)


def test_two_level_error_operator():
    # levels {p, 1}: the V-cycle error operator is S (I - P A_1^{-1} P^T A) S
    # with S the Chebyshev error polynomial in D^{-1} A (Algorithm 2)
    s = _solver(2, (3, 1), seed=4)
    A, dinv = s.A[0], s.dinv[0]
    n = A.shape[0]
    a, b = s.intervals[0]
    S = np.zeros((n, n))
    for j in range(n):        # error propagation of one Chebyshev pass
        e0 = np.eye(n)[j]
        S[:, j] = e0 - pmg.chebyshev(A, dinv, A @ e0, np.zeros(n), a, b, 3, x_is_zero=True)
    P = s.P[0]
    C = np.eye(n) - P @ np.linalg.solve(s.A[1], P.T @ A)   # rediscretised coarse operator
    E = S @ C @ S
    Minv = np.column_stack([s.solve(A @ np.eye(n)[j]) for j in range(n)])
    assert np.allclose(np.eye(n) - Minv, E, atol=1e-11)


def test_many_vcycles_converge_to_lu():
    s = _solver(3, (4, 2, 1), seed=2, nmg=40)
    r = np.random.default_rng(5).standard_normal(s.A[0].shape[0])
    d = s.solve(r)
    x = s.exact_solve(r)
    assert np.linalg.norm(d - x) <= 1e-8 * np.linalg.norm(x)


def test_paper_single_patch_pcg_counts():
    # Section 3.2: CG with one V-cycle (Jacobi, omega = 1/2, levels 1,3,7,15)
    # as preconditioner on an undeformed Cartesian 2D patch needs about 10
    # iterations at p = 3 and about 23 at p = 15 (to 1e-8).  omega = 1/2 is a
    # degree-1 Chebyshev step on any interval with a + b = 4.
    path = os.path.join(os.path.dirname(__file__), "golden", "single_patch_pcg.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    for d, p, iters in rows:
        d, p, iters = int(d), int(p), int(iters)
        levels = tuple(q for q in (15, 7, 3) if q < p) + (1,)
        levels = (p,) + tuple(q for q in levels if q < p)
        g = np.array(np.meshgrid(*([np.arange(3)] * d), indexing="ij"))
        X = np.stack([g[i].transpose(tuple(reversed(range(d)))).reshape(-1) for i in range(d)], 1) * 0.5
        s = pmg.LocalSolver(fem.PatchGeometry(X, np.ones(2 ** d)), levels, cheb_degree=1)
        s.bounds = None
        s.intervals = [(0.5, 3.5)] * (len(levels) - 1)
        b = np.random.default_rng(p).standard_normal(s.A[0].shape[0])
        x, k, rel = s.pcg(b, 1e-8, 100)
        assert rel <= 1e-8
        assert 0.7 * iters <= k <= 1.3 * iters, (p, k)


def _spd(n, eigs, seed):
    Q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((n, n)))
    return (Q * np.asarray(eigs)) @ Q.T


def test_pcg_reaches_the_direct_solution():
    # a random SPD matrix of condition 1e3 with the Jacobi preconditioner:
    # the returned x is the LU solution to within cond x rtol
    eigs = np.geomspace(1.0, 1e3, 40)
    A = _spd(40, eigs, 1) + np.diag(np.linspace(0, 5, 40))
    b = np.random.default_rng(2).standard_normal(40)
    x, k, rel = pmg.pcg(lambda v: A @ v, lambda r: r / np.diag(A), b, 1e-13, 500)
    xs = np.linalg.solve(A, b)
    assert rel <= 1e-13 and k < 500
    assert np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)
    assert abs(np.linalg.norm(b - A @ x) / np.linalg.norm(b) - rel) <= 1e-12


def test_pcg_finite_termination():
    # unpreconditioned CG ends in at most as many iterations as A has
    # distinct eigenvalues (the Krylov space then holds the solution), and
    # in one iteration with the exact inverse as preconditioner
    A = _spd(30, np.repeat([1.0, 3.0, 7.0, 20.0], [5, 10, 8, 7]), 3)
    b = np.random.default_rng(4).standard_normal(30)
    _, k, rel = pmg.pcg(lambda v: A @ v, lambda r: r, b, 1e-10, 100)
    assert k == 4 and rel <= 1e-10
    Ainv = np.linalg.inv(A)
    x, k, rel = pmg.pcg(lambda v: A @ v, lambda r: Ainv @ r, b, 1e-10, 100)
    assert k == 1 and rel <= 1e-10
    # maxit and a zero right-hand side
    x, k, rel = pmg.pcg(lambda v: A @ v, lambda r: r, b, 0.0, 2)
    assert k == 2 and 0 < rel < 1
    x, k, rel = pmg.pcg(lambda v: A @ v, lambda r: r, np.zeros(30), 1e-10, 100)
    assert k == 0 and rel == 0.0 and not x.any()
    x, k, rel = pmg.pcg(lambda v: A @ v, lambda r: r, b, 1e-10, 0)
    assert k == 0 and rel == 1.0 and not x.any()


def test_pcg_of_the_local_solver_is_monotone_in_energy():
    # CG minimises the A-norm of the error over growing Krylov spaces: the
    # error energy of x_k never increases with k (distorted Q4 patch, the
    # V-cycle as preconditioner)
    s = _solver(3, (4, 2, 1), seed=7)
    b = np.random.default_rng(8).standard_normal(s.A[0].shape[0])
    xs = s.exact_solve(b)
    prev = np.inf
    for kmax in range(1, 8):
        x, k, _ = s.pcg(b, 0.0, kmax)
        e = x - xs
        en = e @ (s.A[0] @ e)
        assert k == kmax and en <= prev * (1 + 1e-12)
        prev = en


# ---------------------------------------------------------------------------
# sweep
# ---------------------------------------------------------------------------

def test_colour_classes_disjoint():
    from oracle.smoother import patch_indices
    dim, n, p = 3, 5, 2
    order = patch_order(dim, n)
    for c in range(8):
        vs = [v for v in order if vertex_color(v) == c]
        for i, v in enumerate(vs):
            clo_v, inn_v = patch_indices(v, p, n, dim)
            for w in vs[i + 1:]:
                clo_w, inn_w = patch_indices(w, p, n, dim)
                assert not set(inn_v) & set(clo_w)
                assert not set(inn_w) & set(clo_v)


def test_sweep_order_within_colour_irrelevant():
    w = synth.workload(1)
    X, mu, _ = synth.make_case(w, n=4)
    b = synth.make_rhs(3, 4, 2, 7)
    mesh = fem.Mesh(3, 4, X, mu)
    S = PatchSmoother(mesh, 2, (2, 1))
    u0 = np.random.default_rng(0).standard_normal(b.shape) * fem.dirichlet_mask(3, 4, 2)
    u1 = S.sweep(u0, b)
    # permute patches inside each colour
    S.order = [v for c in range(8) for v in reversed([x for x in S.order if vertex_color(x) == c])]
    u2 = S.sweep(u0, b)
    assert np.allclose(u1, u2, atol=1e-13 * np.abs(u1).max())


def test_sweep_global_rows_equal_patch_closure():
    w = synth.workload(1)
    X, mu, _ = synth.make_case(w, n=3)
    b = synth.make_rhs(3, 3, 2, 8)
    mesh = fem.Mesh(3, 3, X, mu)
    A = fem.dirichlet_operator(mesh, 2)
    S1 = PatchSmoother(mesh, 2, (2, 1), global_matrix=A)
    S2 = PatchSmoother(mesh, 2, (2, 1))
    u0 = np.random.default_rng(1).standard_normal(b.shape) * fem.dirichlet_mask(3, 3, 2)
    assert np.allclose(S1.sweep(u0, b), S2.sweep(u0, b), atol=1e-12)


def test_one_patch_mesh_exact_solve():
    # N = 2: one patch covers every interior node, so an exact local solve
    # gives the discrete solution in one sweep
    w = synth.workload(1)
    X, mu, _ = synth.make_case(w, n=2)
    b = synth.make_rhs(3, 2, 3, 9)
    mesh = fem.Mesh(3, 2, X, mu)
    A = fem.dirichlet_operator(mesh, 3)
    S = PatchSmoother(mesh, 3, (3, 1))
    u = S.sweep(np.zeros_like(b), b, exact=True)
    m = fem.dirichlet_mask(3, 2, 3)
    assert np.linalg.norm((b - A @ u)[m]) <= 1e-12 * np.linalg.norm(b)


def _additive_case(n=3, p=2, seed=10):
    X = synth.make_vertices(2, n, 0.2, seed)
    mesh = fem.Mesh(2, n, X, np.ones(n * n))
    return mesh, PatchSmoother(mesh, p, (p, 1)), fem.dirichlet_operator(mesh, p), fem.dirichlet_mask(2, n, p)


def test_additive_sweep_ignores_patch_order():
    # every correction comes from the same iterate: any order, even across
    # colours, gives the same result (the multiplicative sweep does not)
    mesh, S, A, m = _additive_case(4)
    b = np.random.default_rng(1).standard_normal(m.size) * m
    u0 = np.random.default_rng(2).standard_normal(m.size) * m
    a1, s1 = S.additive_sweep(u0, b, 0.5), S.sweep(u0, b)
    S.order = list(reversed(S.order))
    a2, s2 = S.additive_sweep(u0, b, 0.5), S.sweep(u0, b)
    assert np.abs(a1 - a2).max() <= 1e-13 * np.abs(a1).max()
    assert np.abs(s1 - s2).max() > 1e-6 * np.abs(s1).max()


def test_additive_preconditioner_is_symmetric_and_linear():
    # u = 0: the sweep is theta B b with B = sum_j Pi_j^T M_j Pi_j, M_j the
    # (symmetric) local V-cycle: B is symmetric and linear in b
    mesh, S, A, m = _additive_case(3)
    idx = np.flatnonzero(m)
    cols = []
    for j in idx:
        e = np.zeros(m.size); e[j] = 1.0
        cols.append(S.additive_sweep(np.zeros(m.size), e, 0.7)[idx])
    B = np.array(cols).T / 0.7
    assert np.abs(B - B.T).max() <= 1e-11 * np.abs(B).max()
    r = np.random.default_rng(3).standard_normal(m.size) * m
    assert np.allclose(S.additive_sweep(np.zeros(m.size), r, 0.7)[idx], 0.7 * B @ r[idx], atol=1e-12)
    # the exact solution is a fixed point
    xs = np.zeros(m.size)
    xs[idx] = np.linalg.solve(A.toarray()[np.ix_(idx, idx)], r[idx])
    assert np.abs(S.additive_sweep(xs, r, 0.7) - xs).max() <= 1e-11 * np.abs(xs).max()


def test_additive_equals_multiplicative_on_one_patch():
    mesh, S, A, m = _additive_case(2, p=3)
    b = np.random.default_rng(4).standard_normal(m.size) * m
    u0 = np.random.default_rng(5).standard_normal(m.size) * m
    assert np.allclose(S.additive_sweep(u0, b, 1.0), S.sweep(u0, b), atol=1e-13)
    # the damping scales the correction
    assert np.allclose(S.additive_sweep(u0, b, 0.4) - u0, 0.4 * (S.sweep(u0, b) - u0), atol=1e-13)


# ---------------------------------------------------------------------------
# global multigrid and CG
# ---------------------------------------------------------------------------

def test_hierarchy_sizes():
    assert gmg.hierarchy_sizes(8) == [2, 4, 8]
    assert gmg.hierarchy_sizes(16) == [2, 4, 8, 16]
    assert gmg.hierarchy_sizes(24) == [3, 6, 12, 24]
    assert gmg.hierarchy_sizes(32) == [2, 4, 8, 16, 32]


@pytest.mark.parametrize("dim,p", [(2, 3), (3, 2)])
def test_h_prolongation_galerkin_cartesian(dim, p):
    # on Cartesian meshes with constant mu the embedding is exact, so
    # P^T A_fine P = A_coarse (Section 2, transfers)
    nc = 2
    def mesh_of(n):
        g = np.array(np.meshgrid(*([np.arange(n + 1)] * dim), indexing="ij"))
        X = np.stack([g[i].transpose(tuple(reversed(range(dim)))).reshape(-1)
                      for i in range(dim)], axis=1) / n
        return fem.Mesh(dim, n, X, np.ones(n ** dim))
    Af = fem.dirichlet_operator(mesh_of(2 * nc), p)
    Ac = fem.dirichlet_operator(mesh_of(nc), p)
    P = gmg.prolongation_h(dim, nc, p)
    assert abs(P.T @ Af @ P - Ac).max() <= 1e-12 * abs(Ac).max()


def test_h_prolongation_reproduces_polynomials():
    p, nc = 3, 3
    P1 = gmg.prolongation_h_1d(nc, p)
    x = fe1d.gll_nodes(p)
    xc = np.concatenate([[(c + t) / nc for t in x[:-1]] for c in range(nc)] + [[1.0]])
    xf = np.concatenate([[(c + t) / (2 * nc) for t in x[:-1]] for c in range(2 * nc)] + [[1.0]])
    f = np.polynomial.Polynomial([0.3, -1.0, 2.0, 0.7])
    assert np.allclose(P1 @ f(xc), f(xf), atol=1e-13)


def test_gmg_cg_2d_converges_to_direct_solution():
    w = synth.workload(0)
    X, mu, b = synth.make_case(w)
    mesh = fem.Mesh(w.dim, w.n, X, mu)
    G = gmg.GMG(mesh, w.p, w.levels)
    x, it, hist = G.cg(b, rtol=w.rtol)
    m = fem.dirichlet_mask(w.dim, w.n, w.p)
    A = G.A[-1].toarray()[np.ix_(m, m)]
    xs = np.linalg.solve(A, b[m])
    assert it <= 10
    assert np.linalg.norm(x[m] - xs) <= 1e-8 * np.linalg.norm(xs)
    # the preconditioner is symmetric (reversed sweep order after the coarse
    # correction), which CG relies on
    rng = np.random.default_rng(0)
    r1, r2 = rng.standard_normal(b.shape) * m, rng.standard_normal(b.shape) * m
    assert abs(r2 @ G.precondition(r1) - r1 @ G.precondition(r2)) <= 1e-11 * abs(r1 @ G.precondition(r1))


def test_boundary_patches_cover_and_colour():
    # with boundary vertices there are (n+1)^d patches; same-colour interiors
    # avoid each other's closures; every interior DoF lies in some patch
    # interior, and nodes near the boundary lie in more patches than without
    from oracle.smoother import patch_indices
    dim, n, p = 3, 4, 2
    order = patch_order(dim, n, with_boundary=True)
    assert len(order) == (n + 1) ** dim
    cover = np.zeros((n * p + 1) ** dim, dtype=int)
    for c in range(8):
        vs = [v for v in order if vertex_color(v) == c]
        idx = [patch_indices(v, p, n, dim) for v in vs]
        for i in range(len(vs)):
            cover[idx[i][1]] += 1
            for j in range(i + 1, len(vs)):
                assert not set(idx[i][1]) & set(idx[j][0])
                assert not set(idx[j][1]) & set(idx[i][0])
    mask = fem.dirichlet_mask(dim, n, p)
    assert np.all(cover[mask] >= 1) and np.all(cover[~mask] == 0)


def test_truncated_patch_levels_and_coarse_solve():
    # a corner patch has (q-1)^d interior nodes: empty at q = 1, so the
    # coarsest level is the lowest non-empty one, solved by Cholesky
    X = synth.make_vertices(3, 4, 0.2, 3)
    mesh = fem.Mesh(3, 4, X, np.ones(64))
    corner, edge, face = mesh.patch((0, 0, 0)), mesh.patch((4, 0, 2)), mesh.patch((2, 2, 4))
    s = pmg.LocalSolver(corner, (4, 2, 1))
    assert s.levels == (4, 2) and s.A[1].shape == (1, 1)
    s = pmg.LocalSolver(edge, (4, 2, 1))
    assert s.levels == (4, 2) and s.A[1].shape == (3, 3) and s.A[0].shape == (7 * 9, 7 * 9)
    s = pmg.LocalSolver(face, (2, 1))
    assert s.levels == (2,)
    r = np.random.default_rng(0).standard_normal(s.A[0].shape[0])
    assert np.allclose(s.solve(r), np.linalg.solve(s.A[0], r), rtol=1e-12, atol=1e-12)


def test_gmg_cg_with_boundary_patches():
    # the smoother with boundary patches is still symmetric in the V-cycle
    # and the outer CG converges
    from oracle.gmg import GMG
    X = synth.make_vertices(2, 8, 0.2, 9)
    mesh = fem.Mesh(2, 8, X, np.ones(64))
    b = synth.make_rhs(2, 8, 2, 3)
    G = GMG(mesh, 2, (2, 1), with_boundary=True)
    r1 = np.random.default_rng(1).standard_normal(b.shape) * fem.dirichlet_mask(2, 8, 2)
    r2 = np.random.default_rng(2).standard_normal(b.shape) * fem.dirichlet_mask(2, 8, 2)
    assert abs(r2 @ G.precondition(r1) - r1 @ G.precondition(r2)) <= 1e-10 * abs(r1 @ G.precondition(r1))
    x, it, hist = G.cg(b, rtol=1e-10)
    assert it <= 30


@pytest.mark.parametrize("rule,expect", [("arithmetic", 21.25), ("geometric", 8.0),
                                         ("harmonic", 1.0 / 0.33203125)])
def test_coarse_coefficient_means(rule, expect):
    # one parent cell of 2x2x2 children with mu = 1, 4, 16, 64 (twice): the
    # three means in closed form
    X = synth.make_vertices(3, 2, 0.0, 1)
    mu = np.array([1.0, 4.0, 16.0, 64.0, 1.0, 4.0, 16.0, 64.0])
    c = fem.Mesh(3, 2, X, mu).coarsen(rule)
    assert c.n == 1 and np.isclose(c.mu[0], expect, rtol=1e-14)


def _affine_mesh(dim, n, mu, skew=0.0):
    # a uniform mesh of the unit box sheared by an affine map: every cell
    # and every coarse cell is affine, so the coarse spaces are nested
    g = np.array(np.meshgrid(*([np.arange(n + 1)] * dim), indexing="ij"))
    X = np.stack([g[i].transpose(tuple(reversed(range(dim)))).reshape(-1)
                  for i in range(dim)], axis=1) / n
    X[:, 0] += skew * X[:, dim - 1]
    return fem.Mesh(dim, n, X, mu)


@pytest.mark.parametrize("dim,p,n,levels", [(2, 3, 4, 1), (2, 2, 8, 2), (3, 2, 4, 1), (3, 1, 4, 2)])
def test_octant_coarse_operator_is_galerkin_on_affine_meshes(dim, p, n, levels):
    # reading R11: a coarse cell integrates box by box with its descendants'
    # coefficients; on affine nested meshes that is exactly the Galerkin
    # product P^T A_fine P (the integrand is a polynomial on every box),
    # over one and two coarsenings, for coefficients jumping by 1e6
    mu = 10.0 ** np.random.default_rng(dim + n).uniform(-3, 3, n ** dim)
    fine = _affine_mesh(dim, n, mu, skew=0.3)
    A = fem.dirichlet_operator(fine, p)
    mesh, nc = fine, n
    for _ in range(levels):
        nc //= 2
        mesh = mesh.coarsen("octant")
        P = gmg.prolongation_h(dim, nc, p)
        A = (P.T @ A @ P).tocsr()
    Ac = fem.dirichlet_operator(mesh, p)
    assert mesh.n == nc and mesh.mu.shape == (nc ** dim, (n // nc) ** dim)
    assert abs(Ac - A).max() <= 1e-11 * abs(A).max()
    # the arithmetic mean does not give it
    Aa = fem.dirichlet_operator(_affine_mesh(dim, n, mu, skew=0.3).coarsen("arithmetic"), p) \
        if levels == 1 else None
    if Aa is not None:
        assert abs(Aa - A).max() > 1e-3 * abs(A).max()


def test_octant_rule_with_equal_box_coefficients_is_the_cell_rule():
    # boxes of one coefficient on a distorted mesh: the composite rule and the
    # cell rule differ only by quadrature error, which vanishes for an
    # undistorted cell and stays small on a distorted one
    dim, p, n = 2, 3, 4
    X = synth.make_vertices(dim, n, 0.2, 3)
    mu = np.full(n ** dim, 2.5)
    A1 = fem.dirichlet_operator(fem.Mesh(dim, n, X, mu).coarsen("arithmetic"), p)
    A2 = fem.dirichlet_operator(fem.Mesh(dim, n, X, mu).coarsen("octant"), p)
    rel = abs(A1 - A2).max() / abs(A1).max()
    assert 0 < rel < 1e-2


# ---------------------------------------------------------------------------
# Cartesian-reinforced smoother
# ---------------------------------------------------------------------------

def _cartesian_patch(dim, h, mu):
    g = np.array(np.meshgrid(*([np.arange(3.0)] * dim), indexing="ij"))
    X = np.stack([g[i].transpose(tuple(reversed(range(dim)))).reshape(-1) for i in range(dim)], 1) * h
    return fem.PatchGeometry(X, np.full(2 ** dim, mu))


def _two_cell_1d(q):
    # 1D mass and stiffness of two unit cells, interior nodes only, built
    # here from the GLL basis and the (q+1)-point Gauss rule directly
    x, w = fe1d.gauss_rule(q + 1)
    L = fe1d.lagrange_values(fe1d.gll_nodes(q), x)
    D = fe1d.lagrange_derivatives(fe1d.gll_nodes(q), x)
    Mc, Kc = (L * w) @ L.T, (D * w) @ D.T
    M = np.zeros((2 * q + 1, 2 * q + 1))
    K = np.zeros_like(M)
    for c in range(2):
        s = slice(c * q, c * q + q + 1)
        M[s, s] += Mc
        K[s, s] += Kc
    return M[1:-1, 1:-1], K[1:-1, 1:-1]


@pytest.mark.parametrize("dim,q", [(2, 1), (2, 3), (2, 7), (3, 2), (3, 3)])
def test_reference_patch_matrix_is_a_kronecker_sum(dim, q):
    # the reference patch operator is sum_i M x .. K_i .. x M (x fastest, so
    # the x factor is the right-most Kronecker factor), which is what makes
    # its fast diagonalisation exact
    M, K = _two_cell_1d(q)
    A = np.zeros((M.shape[0] ** dim,) * 2)
    for i in range(dim):
        T = np.ones((1, 1))
        for j in range(dim):
            T = np.kron(K if j == i else M, T)
        A += T
    assert np.abs(pmg.reference_patch_matrix(dim, q) - A).max() <= 1e-12 * np.abs(A).max()


@pytest.mark.parametrize("dim,q", [(2, 3), (2, 7), (3, 3)])
def test_cartesian_preconditioner_inverts_undeformed_patches(dim, q):
    # on an undeformed patch of any cell size with one coefficient, A_j is a
    # multiple of A_b and D diag(A_b) undoes that multiple: P A = I
    s = pmg.LocalSolver(_cartesian_patch(dim, 0.37, 5.3), (q, 1), smoother="cartesian")
    Ab = s.Ab[0]
    PA = (s.dinv[0] * np.diag(Ab))[:, None] * np.linalg.solve(Ab, s.A[0])
    assert np.abs(PA - np.eye(len(PA))).max() <= 1e-10
    # a distorted patch: P A is no longer the identity
    s2 = _solver(dim, (q, 1), seed=3)
    s2 = pmg.LocalSolver(s2.patch, (q, 1), smoother="cartesian")
    PA2 = (s2.dinv[0] * np.diag(s2.Ab[0]))[:, None] * np.linalg.solve(s2.Ab[0], s2.A[0])
    assert np.abs(PA2 - np.eye(len(PA2))).max() > 1e-2


@pytest.mark.parametrize("dim,q,ncell", [(2, 3, (1, 2)), (2, 4, (2, 1)), (3, 3, (1, 2, 1)), (3, 2, (2, 2, 1))])
def test_cartesian_preconditioner_inverts_cut_undeformed_patches(dim, q, ncell):
    # a patch of a boundary vertex keeps its cells inside the domain (one per
    # cut direction); its reference patch has the same cell counts, so on an
    # undeformed mesh P A = I there too, and the reference operator is the
    # Kronecker sum of the 1D matrices of one or two cells per direction
    P = _cartesian_patch(dim, 0.25, 3.0)
    P = fem.PatchGeometry(P.verts, P.mu, ncell)
    Ab = pmg.reference_patch_matrix(dim, q, ncell)
    Aj = fem.patch_matrix(P, q)
    PA = (np.diag(Ab) / np.diag(Aj))[:, None] * np.linalg.solve(Ab, Aj)
    assert np.abs(PA - np.eye(len(PA))).max() <= 1e-10
    M2, K2 = _two_cell_1d(q)
    M1, K1 = M2[:q - 1, :q - 1], K2[:q - 1, :q - 1]     # one cell: its interior nodes 1 .. q-1
    # (the first cell's block of the two-cell matrices holds exactly the one-cell ones)
    x, w = fe1d.gauss_rule(q + 1)
    L = fe1d.lagrange_values(fe1d.gll_nodes(q), x)
    assert np.allclose(M1, ((L * w) @ L.T)[1:-1, 1:-1], atol=1e-14)
    A = np.zeros_like(Ab)
    for i in range(dim):
        T = np.ones((1, 1))
        for j in range(dim):
            Mj, Kj = (M2, K2) if ncell[j] == 2 else (M1, K1)
            T = np.kron(Kj if j == i else Mj, T)
        A += T
    assert np.abs(Ab - A).max() <= 1e-12 * np.abs(A).max()


def test_cartesian_sweep_on_undeformed_mesh_reduces_the_error_by_four():
    # on a one-patch mesh (N = 2) with an undeformed patch, the sweep is one
    # V-cycle with the exact level inverses as smoothers: levels (q, 1) give
    # B A the eigenvalues 3/4 and 1, so the error propagation I - B A has
    # 1/4 and 0 and a sweep from zero reduces the energy norm of the error by
    # at least 4 (equality on the fine complement)
    mesh = fem.Mesh(2, 2, _cartesian_patch(2, 0.5, 1.0).verts, np.ones(4))
    S = PatchSmoother(mesh, 3, (3, 1), smoother="cartesian", omega=0.5)
    A = fem.dirichlet_operator(mesh, 3).toarray()
    mask = fem.dirichlet_mask(2, 2, 3)
    Ai = A[np.ix_(mask, mask)]
    rng = np.random.default_rng(2)
    b = np.zeros(mask.size)
    b[mask] = rng.standard_normal(mask.sum())
    xs = np.zeros(mask.size)
    xs[mask] = np.linalg.solve(Ai, b[mask])
    u = S.sweep(np.zeros_like(b), b, +1)
    e0, e1 = xs[mask], (xs - u)[mask]
    ratio = np.sqrt(e1 @ Ai @ e1 / (e0 @ Ai @ e0))
    assert ratio <= 0.25 + 1e-12
    assert ratio >= 0.2                  # not an exact solve


@pytest.mark.parametrize("dim,levels", [(2, (3, 1)), (3, (3, 1)), (2, (7, 3, 1)), (3, (7, 3, 1)),
                                        (2, (15, 7, 3, 1))])
def test_cartesian_vcycle_cg_iterations_equal_level_count(dim, levels):
    # with P = A^{-1} on every level and omega = 1/2, one V-cycle B gives
    # B A = 3/4 on the A-orthogonal complement of the first coarse space,
    # 1 - 1/4^k on the k-th complement below and 1 on the coarsest space:
    # one distinct eigenvalue per level, so CG ends after exactly as many
    # iterations as there are levels
    s = pmg.LocalSolver(_cartesian_patch(dim, 0.5, 2.0), levels, smoother="cartesian")
    b = np.random.default_rng(len(levels)).standard_normal(s.A[0].shape[0])
    x, k, rel = s.pcg(b, 1e-12, 50)
    assert k == len(levels) and rel <= 1e-12
    # the spectrum of B A itself
    n = s.A[0].shape[0]
    BA = np.column_stack([s.solve(s.A[0][:, j]) for j in range(n)]) if n <= 400 else None
    if BA is not None:
        ev = np.sort(np.linalg.eigvals(BA).real)
        expect = sorted({1.0 - 0.25 ** (len(levels) - 1 - l) if l < len(levels) - 1 else 1.0
                         for l in range(len(levels))})
        assert all(np.min(np.abs(ev - e)) <= 1e-10 for e in expect)
        assert all(np.min(np.abs(np.array(expect) - e)) <= 1e-10 for e in ev)


def test_cartesian_step_uses_the_reference_patch():
    # on a distorted patch one step from zero is omega D diag(A_b) A_b^{-1} r
    # with A_b the Kronecker sum of the 1D two-cell matrices (not the
    # distorted patch's own operator)
    M, K = _two_cell_1d(3)
    Ab = np.kron(M, K) + np.kron(K, M)
    s = pmg.LocalSolver(_solver(2, (3, 1), seed=3).patch, (3, 1), smoother="cartesian", omega=0.5)
    r = np.random.default_rng(4).standard_normal(Ab.shape[0])
    d = s.cartesian_step(0, r, np.zeros_like(r), d_is_zero=True)
    expect = 0.5 * s.dinv[0] * np.diag(Ab) * np.linalg.solve(Ab, r)
    assert np.abs(d - expect).max() <= 1e-12 * np.abs(expect).max()
    # and from a nonzero start it acts on the residual r - A d
    d0 = np.random.default_rng(5).standard_normal(Ab.shape[0])
    d1 = s.cartesian_step(0, r, d0)
    expect1 = d0 + 0.5 * s.dinv[0] * np.diag(Ab) * np.linalg.solve(Ab, r - s.A[0] @ d0)
    assert np.abs(d1 - expect1).max() <= 1e-12 * np.abs(expect1).max()


# ---------------------------------------------------------------------------
# GMRES and the paper's sweep order
# ---------------------------------------------------------------------------

def test_gmres_reaches_the_direct_solution_with_monotone_residuals():
    rng = np.random.default_rng(11)
    A = np.eye(40) * 4 + rng.standard_normal((40, 40))      # non-symmetric
    b = rng.standard_normal(40)
    x, k, rel = gmg.gmres(lambda v: A @ v, lambda r: r / np.diag(A), b, 1e-12, 40)
    xs = np.linalg.solve(A, b)
    assert k <= 40 and rel <= 1e-12
    assert np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)
    assert abs(np.linalg.norm(b - A @ x) / np.linalg.norm(b) - rel) <= 1e-12
    # minimal residual over growing Krylov spaces: true residuals never increase
    prev = np.inf
    for kmax in range(1, 12):
        x, _, _ = gmg.gmres(lambda v: A @ v, lambda r: r, b, 0.0, kmax)
        res = np.linalg.norm(b - A @ x)
        assert res <= prev * (1 + 1e-12)
        prev = res


def test_gmres_finite_termination():
    # a diagonalisable matrix with 3 distinct eigenvalues: 3 iterations;
    # the exact inverse as preconditioner: 1
    rng = np.random.default_rng(12)
    Q = rng.standard_normal((25, 25))
    A = Q @ np.diag(np.repeat([1.0, 2.5, 6.0], [10, 8, 7])) @ np.linalg.inv(Q)
    b = rng.standard_normal(25)
    _, k, rel = gmg.gmres(lambda v: A @ v, lambda r: r, b, 1e-9, 50)
    assert k == 3 and rel <= 1e-9
    Ainv = np.linalg.inv(A)
    _, k, rel = gmg.gmres(lambda v: A @ v, lambda r: Ainv @ r, b, 1e-9, 50)
    assert k == 1
    x, k, rel = gmg.gmres(lambda v: A @ v, lambda r: r, np.zeros(25), 1e-9, 50)
    assert k == 0 and rel == 0.0 and not x.any()
    _, k, rel = gmg.gmres(lambda v: A @ v, lambda r: r, b, 0.0, 2)
    assert k == 3 and 0 < rel < 1      # maxit + 1: not converged


def test_paper_order_vcycle_is_not_symmetric_and_gmres_converges():
    w = synth.workload("2d-n8-q3")
    X = synth.make_vertices(2, 4, 0.2, 5)
    mesh = fem.Mesh(2, 4, X, np.ones(16))
    G = gmg.GMG(mesh, 3, (3, 1), cheb_degree=1, post_direction=+1)
    G1 = gmg.GMG(mesh, 3, (3, 1), cheb_degree=1, post_direction=-1)
    n = G.A[-1].shape[0]
    mask = fem.dirichlet_mask(2, 4, 3)
    idx = np.flatnonzero(mask)[:12]
    def mat(GG):
        cols = []
        for j in idx:
            e = np.zeros(n); e[j] = 1.0
            cols.append(GG.precondition(e)[idx])
        return np.array(cols).T
    B, B1 = mat(G), mat(G1)
    assert np.abs(B1 - B1.T).max() <= 1e-10 * np.abs(B1).max()     # opposite orders: symmetric
    assert np.abs(B - B.T).max() > 1e-4 * np.abs(B).max()          # one order: not symmetric
    b = np.random.default_rng(3).standard_normal(n) * mask
    x, k, rel = G.gmres(b, 1e-10, 50)
    assert rel <= 1e-10 and k <= 50
    xs = sla.solve(G.A[-1].toarray()[np.ix_(mask, mask)], b[mask])
    assert np.abs(x[mask] - xs).max() <= 1e-8 * np.abs(xs).max()


def test_gmg_with_additive_smoothing_is_symmetric_and_solves():
    X = synth.make_vertices(2, 4, 0.2, 6)
    mesh = fem.Mesh(2, 4, X, np.ones(16))
    G = gmg.GMG(mesh, 3, (3, 1), additive_theta=0.25)
    n = G.A[-1].shape[0]
    mask = fem.dirichlet_mask(2, 4, 3)
    idx = np.flatnonzero(mask)[:15]
    cols = []
    for j in idx:
        e = np.zeros(n); e[j] = 1.0
        cols.append(G.precondition(e)[idx])
    B = np.array(cols).T
    assert np.abs(B - B.T).max() <= 1e-10 * np.abs(B).max()
    b = np.random.default_rng(7).standard_normal(n) * mask
    x, k, hist = G.cg(b, 1e-10, 200)
    assert k <= 200 and hist[-1] <= 1e-10
    xs = sla.solve(G.A[-1].toarray()[np.ix_(mask, mask)], b[mask])
    assert np.abs(x[mask] - xs).max() <= 1e-8 * np.abs(xs).max()
