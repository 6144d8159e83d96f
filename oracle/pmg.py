"""The local p-multigrid solver on one vertex patch (Section 3.1, Algorithm 2).

TEST INFRASTRUCTURE (oracle): see oracle/__init__.py.

Components, each formed explicitly:
  * level spaces V_{j,q} on the fixed patch geometry, one per degree in a
    descending list (p = q_0 > q_1 > ... > q_m) (Section 3.1);
  * prolongation = embedding of V_{j,q'} into V_{j,q}, restriction = its
    transpose; both Kronecker products of a 1D patch matrix (Section 3.1,
    transfer operators);
  * level operators by rediscretisation with the degree-q basis (Section 3.1,
    level operators);
  * coarse solve: dense Cholesky of the coarsest level operator, a 1x1 matrix
    for interior patches at degree 1 (Section 3.1, coarse solver);
  * smoother: Chebyshev acceleration of Jacobi (the paper's damped Jacobi
    Richardson step, Section 3.1 smoothers, is its degree-1 case) on the
    interval [a, b] with b = s lambda_max, a = max(lambda_min, b / rho).
    The recurrence is the standard Chebyshev iteration (Saad, Iterative
    Methods for Sparse Linear Systems, 2nd ed., Algorithm 12.1) with D^{-1}
    applied to the residuals;
  * V-cycle: pre-smooth, residual, restrict, recurse, prolongate, correct,
    post-smooth (Algorithm 2);
  * the Cartesian-reinforced smoother (Section 3.1, smoothers): Richardson
    steps d += omega P (r - A d) with P = D diag(A_b) A_b^{-1}, A_b the
    operator of the undeformed Cartesian reference patch (unit cells,
    coefficient 1) at the level's degree and D the level's inverse
    diagonal; one step before and one after the coarse correction;
  * the local solver's measure of quality in Section 3.2: conjugate gradients
    on the patch problem, preconditioned by one V-cycle.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import fe1d
from .fem import PatchGeometry, patch_matrix

CHEB_SAFETY = 1.1   # s: b = s * lambda_max
CHEB_RANGE = 15.0   # rho: a >= b / rho


def prolongation_1d(p: int, q: int, ncell: int = 2) -> np.ndarray:
    """Embedding of the degree-q interior patch space into the degree-p one
    along one direction with `ncell` cells: shape (ncell p - 1, ncell q - 1).

    Fine interior node s lies in cell c = floor(s / p) (a node shared by two
    cells has the same value from either side) at local coordinate
    xi = x^p_{s - c p} (GLL point); its entry for coarse node t is the degree-q
    Lagrange polynomial l^q_{t - c q}(xi) when 0 <= t - c q <= q, else 0.
    """
    xp = fe1d.gll_nodes(p)
    xq = fe1d.gll_nodes(q)
    P = np.zeros((ncell * p - 1, ncell * q - 1))
    for s in range(1, ncell * p):
        c = min(s // p, ncell - 1)
        xi = xp[s - c * p]
        L = fe1d.lagrange_values(xq, [xi])[:, 0]
        for t in range(1, ncell * q):
            a = t - c * q
            if 0 <= a <= q:
                P[s - 1, t - 1] = L[a]
    return P


def prolongation(p: int, q: int, ncell) -> np.ndarray:
    """Kronecker product of the 1D factors, x fastest:
    P = P_{d-1} (x) ... (x) P_0."""
    P = np.ones((1, 1))
    for i in range(len(ncell)):
        P = np.kron(prolongation_1d(p, q, ncell[i]), P)
    return P


def chebyshev_interval(lam_min: float, lam_max: float,
                       safety: float = CHEB_SAFETY, rng: float = CHEB_RANGE):
    b = safety * lam_max
    a = max(lam_min, b / rng)
    return a, b


def chebyshev(A, dinv, f, x, a, b, k, x_is_zero=False):
    """k steps of Chebyshev-accelerated Jacobi for A x = f on [a, b]:

        theta = (b+a)/2, delta = (b-a)/2, sigma = theta/delta, rho_0 = 1/sigma
        r_0 = f - A x_0,  z_0 = D^{-1} r_0 / theta
        for i = 0 .. k-1:
            x <- x + z_i
            if i < k-1:
                r_{i+1} = r_i - A z_i
                rho_{i+1} = 1 / (2 sigma - rho_i)
                z_{i+1} = rho_{i+1} rho_i z_i + (2 rho_{i+1} / delta) D^{-1} r_{i+1}
    """
    theta = 0.5 * (b + a)
    delta = 0.5 * (b - a)
    sigma = theta / delta
    rho = 1.0 / sigma
    x = np.array(x, dtype=np.float64, copy=True)
    r = f.copy() if x_is_zero else f - A @ x
    z = dinv * r / theta
    for i in range(k):
        x = x + z
        if i < k - 1:
            r = r - A @ z
            rho_new = 1.0 / (2.0 * sigma - rho)
            z = rho_new * rho * z + (2.0 * rho_new / delta) * (dinv * r)
            rho = rho_new
    return x


def reference_patch_matrix(dim: int, q: int, ncell=None) -> np.ndarray:
    """A_{b,q}: the degree-q operator of the undeformed Cartesian patch with
    unit cells and coefficient 1 (the reference patch of the
    Cartesian-reinforced smoother, Section 3.1), assembled like any patch."""
    ncell = tuple(ncell) if ncell is not None else (2,) * dim
    g = np.array(np.meshgrid(*([np.arange(3.0)] * dim), indexing="ij"))
    X = np.stack([g[i].transpose(tuple(reversed(range(dim)))).reshape(-1) for i in range(dim)], 1)
    return patch_matrix(PatchGeometry(X, np.ones(2 ** dim), ncell), q)


def _level_size(patch: PatchGeometry, q: int) -> int:
    return int(np.prod([patch.ncell[i] * q - 1 for i in range(patch.dim)]))


class LocalSolver:
    """p-multigrid V-cycle for A_{j,p} d = r on one patch.

    levels : descending degrees, e.g. (4, 2, 1)
    bounds : list of (lambda_min, lambda_max) of D^{-1} A per smoothed level
             (all levels but the coarsest), or None to fill in later
    """

    def __init__(self, patch: PatchGeometry, levels, bounds=None, cheb_degree=3,
                 n_vcycles=1, safety=CHEB_SAFETY, rng=CHEB_RANGE, smoother="chebyshev",
                 omega=0.5):
        self.patch = patch
        # a patch cut by the boundary has no interior node at low degrees
        # (q - 1 = 0 nodes along a one-cell direction at q = 1): the coarsest
        # level is the lowest one with a node, solved by Cholesky there
        self.levels = tuple(q for q in levels if _level_size(patch, q) > 0)
        self.k = cheb_degree
        self.n_vcycles = n_vcycles
        self.safety, self.rng = safety, rng
        self.A = [patch_matrix(patch, q) for q in self.levels]
        self.dinv = [1.0 / np.diag(A) for A in self.A]
        self.P = [prolongation(self.levels[l], self.levels[l + 1], patch.ncell)
                  for l in range(len(self.levels) - 1)]
        self.chol = sla.cho_factor(self.A[-1], lower=True)
        if smoother not in ("chebyshev", "cartesian"):
            raise ValueError(smoother)
        self.smoother, self.omega = smoother, omega
        if smoother == "cartesian":
            self.Ab = [reference_patch_matrix(patch.dim, q, patch.ncell) for q in self.levels[:-1]]
            self.Ab_chol = [sla.cho_factor(Ab, lower=True) for Ab in self.Ab]
        self.bounds = None
        if bounds is not None:
            self.set_bounds(bounds)

    def set_bounds(self, bounds):
        self.bounds = [tuple(b) for b in bounds]
        self.intervals = [chebyshev_interval(lo, hi, self.safety, self.rng)
                          for (lo, hi) in self.bounds]

    def vcycle(self, level, d, r, d_is_zero=False):
        """One V-cycle at `level` (index into self.levels), Algorithm 2."""
        if level == len(self.levels) - 1:
            return sla.cho_solve(self.chol, r)
        A, dinv = self.A[level], self.dinv[level]
        if self.smoother == "cartesian":
            d = self.cartesian_step(level, r, d, d_is_zero)                # pre-smoothing
        else:
            a, b = self.intervals[level]
            d = chebyshev(A, dinv, r, d, a, b, self.k, x_is_zero=d_is_zero)
        res = r - A @ d                                                    # residual
        rc = self.P[level].T @ res                                         # restriction
        e = self.vcycle(level + 1, np.zeros_like(rc), rc, d_is_zero=True)  # recursion
        d = d + self.P[level] @ e                                          # prolongation + correction
        if self.smoother == "cartesian":
            d = self.cartesian_step(level, r, d)                           # post-smoothing
        else:
            d = chebyshev(A, dinv, r, d, a, b, self.k)
        return d

    def cartesian_step(self, level, r, d, d_is_zero=False):
        """One Richardson step d += omega P (r - A d) with the
        Cartesian-reinforced preconditioner P = D diag(A_b) A_b^{-1}."""
        res = r if d_is_zero else r - self.A[level] @ d
        Ab = self.Ab[level]
        return d + self.omega * self.dinv[level] * np.diag(Ab) * sla.cho_solve(self.Ab_chol[level], res)

    def solve(self, r):
        """d ~ A_{j,p}^{-1} r by n_vcycles V-cycles from d = 0."""
        d = np.zeros_like(r)
        for it in range(self.n_vcycles):
            d = self.vcycle(0, d, r, d_is_zero=(it == 0))
        return d

    def exact_solve(self, r):
        """The exact local solve (the limit of many V-cycles): LU of A_{j,p}."""
        return np.linalg.solve(self.A[0], r)

    def pcg(self, b, rtol, maxit):
        """CG on A_{j,p} x = b preconditioned by solve() (Section 3.2 measures
        the local solver by the iterations of exactly this combination)."""
        return pcg(lambda v: self.A[0] @ v, self.solve, b, rtol, maxit)


def pcg(apply_A, precondition, b, rtol, maxit):
    """Preconditioned conjugate gradients from x = 0 (Hestenes and Stiefel,
    1952; Saad, Iterative Methods for Sparse Linear Systems, 2nd ed.,
    Algorithm 9.1).  Stops after the first iteration k with
    ||r_k|| <= rtol ||b||, or after maxit iterations.
    Returns (x_k, k, ||r_k|| / ||b||); b = 0 gives (0, 0, 0)."""
    x = np.zeros_like(b)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x, 0, 0.0
    r = b.copy()
    k = 0
    if maxit <= 0:
        return x, 0, 1.0
    z = precondition(r)
    p = z.copy()
    rz = r @ z
    while True:
        Ap = apply_A(p)
        alpha = rz / (p @ Ap)          # step length along p
        x = x + alpha * p
        r = r - alpha * Ap
        k += 1
        if np.linalg.norm(r) <= rtol * bnorm or k >= maxit:
            break
        z = precondition(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p      # next direction, A-conjugate to the previous ones
        rz = rz_new
    return x, k, np.linalg.norm(r) / bnorm
