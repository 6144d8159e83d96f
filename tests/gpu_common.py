"""Shared helpers of the GPU parity tests: seeded cases, oracle-side
reference values and the device handles."""
import numpy as np

import synth
from oracle import fem, lanczos, pmg
from oracle.smoother import patch_indices, patch_order


def case(name, n=None, p=None, levels=None):
    w = synth.workload(name)
    if n is not None:
        w = w.scaled(n)
    p = p or w.p
    levels = tuple(levels or w.levels)
    X = synth.make_vertices(w.dim, w.n, w.alpha, w.mesh_seed)
    mu = synth.make_coefficients(w.dim, w.n, w.mu_log10, w.coef_seed)
    b = synth.make_rhs(w.dim, w.n, p, w.rhs_seed)
    return w, p, levels, X, mu, b


def vlin(v, n):
    return sum(v[i] * (n + 1) ** i for i in range(len(v)))


def oracle_solver(mesh, v, levels, seed=0, steps=12, k=3, nmg=1):
    """LocalSolver of the patch at vertex v with Lanczos bounds computed by
    the oracle from the same start-vector definition."""
    s = pmg.LocalSolver(mesh.patch(v), levels, cheb_degree=k, n_vcycles=nmg)
    b = [lanczos.bounds(s.A[l], s.dinv[l], steps, seed, vlin(v, mesh.n), l)
         for l in range(len(levels) - 1)]
    s.set_bounds(b)
    return s


def rel_err(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)
