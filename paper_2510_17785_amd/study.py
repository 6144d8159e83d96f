"""The single-patch study of the local solver (Section 3.2) on the GPU.

CG to a relative residual of 1e-8, preconditioned by one p-multigrid V-cycle
with damped Jacobi smoothing (omega = 1/2: the degree-1 Chebyshev step on
the interval [0.5, 3.5]) and the nested p-levels 1, 3, 7, 15
(p_{k+1} = 2 p_k + 1),
at most 100 iterations per patch.  For one (dim, p), three sweeps are run as
one batch in one pmg_patch_pcg call:

* distortion: every patch vertex moved by delta h in a uniformly random
  direction, `realizations` patches per delta, coefficient 1;
* jump: an undeformed patch with coefficient mu in cell 0 and 1 elsewhere,
  `realizations` right-hand sides per mu;
* jump under distortion: mu = `fixed_jump` in cell 0 and the distortion sweep.

Right-hand sides are N(0, 1).  A patch that does not reach the tolerance in
`maxit` iterations is counted as not converged.  Each row reports the mean
over the converged patches with the number that did not converge, and the
mean the paper plots, in which every non-converged run enters with a large
sentinel count (SENTINEL_ITERATIONS) so that the point lies off the axes
(Section 3.2).
The patches and right-hand sides come from the seeded generators in `synth`;
all arithmetic runs in the library's kernels.
"""
from __future__ import annotations

import time
from typing import Dict, List, Sequence

import numpy as np
import torch

import synth

from .api import PatchBatch

# lambda bounds whose Chebyshev interval (b = 1.1 lambda_max, a = lambda_min)
# is [0.5, 3.5]: centre 2, so the degree-1 step is omega = 1/2 Jacobi
OMEGA_HALF_BOUNDS = (0.5, 3.5 / 1.1)

# the count a non-converged run enters the paper's means with
SENTINEL_ITERATIONS = 10000


def paper_levels(p: int) -> tuple:
    """p followed by the members of the nested sequence 1, 3, 7, 15 below it."""
    return (p,) + tuple(q for q in (15, 7, 3, 1) if q < p)


def study_patches(dim: int, distortions: Sequence[float], jumps: Sequence[float],
                  fixed_jump: float, realizations: int, seed: int):
    """The batch of one study: (groups, vertices, coefficients), where each
    group is (sweep, value, first patch, patch count)."""
    groups, Xs, mus = [], [], []
    start = 0

    def add(sweep, value, X, mu):
        nonlocal start
        groups.append((sweep, float(value), start, len(X)))
        Xs.append(X)
        mus.append(mu)
        start += len(X)

    for i, d in enumerate(distortions):
        add("distortion", d, *synth.make_sphere_distorted_patches(dim, realizations, d, seed + i))
    for i, m in enumerate(jumps):
        add("jump", m, *synth.make_sphere_distorted_patches(dim, realizations, 0.0, seed + 100 + i,
                                                             mu_cell=m))
    for i, d in enumerate(distortions):
        add("jump+distortion", d, *synth.make_sphere_distorted_patches(dim, realizations, d, seed + 200 + i,
                                                                        mu_cell=fixed_jump))
    return groups, np.concatenate(Xs), np.concatenate(mus)


def run_study(dim: int, p: int, distortions: Sequence[float] = (0.0, 0.05, 0.1, 0.15, 0.2, 0.25, 0.3),
              jumps: Sequence[float] = (1.0, 1e2, 1e4, 1e6, 1e8), fixed_jump: float = 1e4,
              realizations: int = 20, rtol: float = 1e-8, maxit: int = 100, seed: int = 7000,
              smoother: str = "jacobi", device=None) -> Dict:
    """Run the three sweeps for one (dim, p) with the damped Jacobi
    (`smoother="jacobi"`) or the Cartesian-reinforced smoother
    (`"cartesian"`, omega = 1/2 as well); returns the per-group rows, the
    per-patch iteration counts and residuals, and the time of the CG call."""
    dev = torch.device("cuda", 0) if device is None else device
    levels = paper_levels(p)
    groups, X, mu = study_patches(dim, distortions, jumps, fixed_jump, realizations, seed)
    B = PatchBatch(dim, p, X, mu, levels=levels, precision="fp64", cheb_degree=1, bounds="fixed")
    if smoother == "cartesian":
        B.set_smoother("cartesian", 0.5)
    elif smoother == "jacobi":
        B.set_bounds(np.broadcast_to(np.array(OMEGA_HALF_BOUNDS), (B.n_patches, len(levels) - 1, 2)).copy())
    else:
        raise ValueError(smoother)
    b = np.random.default_rng(seed + 300).standard_normal((B.n_patches, B.level_sizes[0]))
    bd = torch.tensor(b, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, it, rel = B.pcg(bd, rtol, maxit)
    torch.cuda.synchronize()
    seconds = time.perf_counter() - t0
    its, rels = it.cpu().numpy(), rel.cpu().numpy()
    rows: List[Dict] = []
    for sweep, value, s0, n in groups:
        k, r = its[s0:s0 + n], rels[s0:s0 + n]
        ok = r <= rtol
        rows.append({"sweep": sweep, "value": value, "patches": n,
                     "mean_iterations": float(k[ok].mean()) if ok.any() else None,
                     "mean_with_sentinel": float(np.where(ok, k, SENTINEL_ITERATIONS).mean()),
                     "min": int(k.min()), "max": int(k.max()),
                     "not_converged": int((~ok).sum())})
    B.close()
    return {"dim": dim, "p": p, "levels": levels, "smoother": smoother, "rows": rows,
            "iterations": its, "relres": rels,
            "X": X, "mu": mu, "b": b, "groups": groups, "seconds": seconds,
            "patch_dofs": int(b.shape[1]), "v_cycles": int(its.sum())}
