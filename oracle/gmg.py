"""Global geometric multigrid with the patch smoother, and the outer CG.

TEST INFRASTRUCTURE (oracle): see oracle/__init__.py.

Hierarchy (Section 2): meshes M_1 < ... < M_L, each a uniform refinement of
the previous one; the fine mesh has N cells per direction and N is halved
while it stays even and the halved mesh still has an interior vertex.  The
coarse vertices are the shared fine vertices (topological nesting suffices,
Section 2); a coarse cell's coefficient is the mean of its children.  Every
level uses the same degree p.

Transfers (Section 2): prolongation is the embedding of the coarse space in
reference coordinates (a fine node at local coordinate xi of fine cell f lies
at (f mod 2 + xi) / 2 of the parent cell), restriction is its transpose.

V-cycle, one smoothing step each way (Section 4): on the coarsest level an
exact solve (dense Cholesky); otherwise
    u = sweep_forward(0, f);  r = f - A u;  u += P V(R r);  u = sweep_backward(u, f).
Pre- and post-smoothing visit the patches in opposite orders, which keeps the
preconditioner symmetric so that CG applies; with additive_theta set, both
are additive sweeps with that damping (symmetric as well).  With post_direction = +1 both
sweeps use the same colour order, as the paper does (Section 4), and the
preconditioner is not symmetric.

Outer solvers: preconditioned CG, or GMRES with the preconditioner on the
right (Section 4 runs GMRES), from x = 0, stopped at ||r_k|| <= rtol ||b||.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import fe1d
from .fem import Mesh, dirichlet_mask, dirichlet_operator
from .smoother import PatchSmoother


def hierarchy_sizes(n: int):
    """Cells per direction from coarsest to finest."""
    sizes = [n]
    while sizes[-1] % 2 == 0 and sizes[-1] // 2 >= 2:
        sizes.append(sizes[-1] // 2)
    return list(reversed(sizes))


def prolongation_h_1d(nc: int, p: int) -> np.ndarray:
    """Embedding of the 1D degree-p space on nc cells into the one on 2 nc
    cells, all nodes included: shape (2 nc p + 1, nc p + 1)."""
    x = fe1d.gll_nodes(p)
    nf = 2 * nc
    P = np.zeros((nf * p + 1, nc * p + 1))
    for g in range(nf * p + 1):
        f = min(g // p, nf - 1)
        xi_f = x[g - f * p]
        c = f // 2
        xi = ((f % 2) + xi_f) / 2.0
        L = fe1d.lagrange_values(x, [xi])[:, 0]
        for t in range(p + 1):
            P[g, c * p + t] = L[t]
    return P


def prolongation_h(dim: int, nc: int, p: int) -> sp.csr_matrix:
    P1 = sp.csr_matrix(prolongation_h_1d(nc, p))
    P = P1
    for _ in range(dim - 1):
        P = sp.kron(P1, P, format="csr")
    mf = sp.diags(dirichlet_mask(dim, 2 * nc, p).astype(np.float64))
    mc = sp.diags(dirichlet_mask(dim, nc, p).astype(np.float64))
    return (mf @ P @ mc).tocsr()


class GMG:
    def __init__(self, mesh: Mesh, p: int, levels, cheb_degree=3, n_vcycles=1,
                 lanczos_steps=12, seed=0, bounds=None, with_boundary=False,
                 coarse_mean="arithmetic", post_direction=-1, additive_theta=None,
                 smoother="chebyshev", omega=0.5):
        self.dim, self.p = mesh.dim, p
        self.post_direction = post_direction
        self.additive_theta = additive_theta
        sizes = hierarchy_sizes(mesh.n)
        meshes = [mesh]
        while meshes[-1].n != sizes[0]:
            meshes.append(meshes[-1].coarsen(coarse_mean))
        self.meshes = list(reversed(meshes))            # coarsest first
        self.A = [dirichlet_operator(m, p) for m in self.meshes]
        self.P = [prolongation_h(self.dim, m.n, p) for m in self.meshes[:-1]]
        self.smoothers = [None]
        for li, m in enumerate(self.meshes[1:], start=1):
            bl = "lanczos" if bounds is None else bounds[li]
            self.smoothers.append(PatchSmoother(m, p, levels, cheb_degree, n_vcycles, bl,
                                                lanczos_steps, seed, global_matrix=self.A[li],
                                                with_boundary=with_boundary, smoother=smoother,
                                                omega=omega))
        mask = dirichlet_mask(self.dim, self.meshes[0].n, p)
        self.coarse_mask = mask
        Ac = self.A[0].toarray()[np.ix_(mask, mask)]
        self.coarse_chol = sla.cho_factor(Ac, lower=True)

    def coarse_solve(self, f):
        u = np.zeros_like(f)
        u[self.coarse_mask] = sla.cho_solve(self.coarse_chol, f[self.coarse_mask])
        return u

    def vcycle(self, level, f):
        if level == 0:
            return self.coarse_solve(f)
        S = self.smoothers[level]
        th = self.additive_theta
        u = S.sweep(np.zeros_like(f), f, +1) if th is None else S.additive_sweep(np.zeros_like(f), f, th)
        r = f - self.A[level] @ u
        u = u + self.P[level - 1] @ self.vcycle(level - 1, self.P[level - 1].T @ r)
        u = S.sweep(u, f, self.post_direction) if th is None else S.additive_sweep(u, f, th)
        return u

    def precondition(self, r):
        return self.vcycle(len(self.meshes) - 1, r)

    def cg(self, b, rtol=1e-8, maxit=100):
        """Preconditioned CG.  Returns (x, iterations, relative residual
        history); iterations = maxit + 1 signals no convergence."""
        A = self.A[-1]
        x = np.zeros_like(b)
        r = b.copy()
        nb = np.linalg.norm(b)
        hist = [1.0]
        z = self.precondition(r)
        d = z.copy()
        rz = r @ z
        for k in range(1, maxit + 1):
            Ad = A @ d
            alpha = rz / (d @ Ad)
            x += alpha * d
            r -= alpha * Ad
            rel = np.linalg.norm(r) / nb
            hist.append(rel)
            if rel <= rtol:
                return x, k, hist
            z = self.precondition(r)
            rz_new = r @ z
            d = z + (rz_new / rz) * d
            rz = rz_new
        return x, maxit + 1, hist

    def gmres(self, b, rtol=1e-8, maxit=100):
        """GMRES preconditioned on the right by one V-cycle.  Returns
        (x, iterations, relative residual); iterations = maxit + 1 signals no
        convergence."""
        return gmres(lambda v: self.A[-1] @ v, self.precondition, b, rtol, maxit)


def gmres(apply_A, precondition, b, rtol, maxit):
    """Flexible GMRES with the preconditioner on the right, from x = 0, no
    restart (Saad, Iterative Methods for Sparse Linear Systems, 2nd ed.,
    Algorithm 9.6): Arnoldi with modified Gram-Schmidt on A M^{-1}, Givens
    rotations for the least-squares problem, x = Z y with z_j = M^{-1} v_j.
    Stops after the first iteration k with ||b - A x_k|| <= rtol ||b|| (the
    rotated right-hand side gives that norm), or after maxit.
    Returns (x_k, k or maxit + 1, ||b - A x_k|| / ||b||)."""
    n = b.shape[0]
    beta = np.linalg.norm(b)
    if beta == 0.0:
        return np.zeros_like(b), 0, 0.0
    V = [b / beta]
    Z = []
    H = np.zeros((maxit + 1, maxit))
    cs, sn = np.zeros(maxit), np.zeros(maxit)
    g = np.zeros(maxit + 1)
    g[0] = beta
    k_done = maxit + 1
    for j in range(maxit):
        Z.append(precondition(V[j]))
        w = apply_A(Z[j])
        for i in range(j + 1):                 # modified Gram-Schmidt
            H[i, j] = w @ V[i]
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        V.append(w / H[j + 1, j] if H[j + 1, j] != 0.0 else w)
        for i in range(j):                     # earlier rotations on the new column
            hi = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
            H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
            H[i, j] = hi
        den = np.hypot(H[j, j], H[j + 1, j])
        cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
        H[j, j] = den
        H[j + 1, j] = 0.0
        g[j + 1] = -sn[j] * g[j]
        g[j] = cs[j] * g[j]
        if abs(g[j + 1]) <= rtol * beta:
            k_done = j + 1
            break
    k = min(k_done, maxit)
    y = sla.solve_triangular(H[:k, :k], g[:k])
    x = sum(y[i] * Z[i] for i in range(k))
    return x, k_done, abs(g[k]) / beta

