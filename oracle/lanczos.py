"""Eigenvalue bounds of D^{-1} A for the Chebyshev interval.

TEST INFRASTRUCTURE (oracle): see oracle/__init__.py.

The paper smooths with damped Jacobi and a fixed damping (Section 3.1,
smoothers); the Chebyshev interval used by this project needs the extreme
eigenvalues of D^{-1} A_{j,q} on each smoothed level.  They are estimated by m
steps of the Lanczos process on the symmetric matrix M = D^{-1/2} A D^{-1/2}
(same spectrum as D^{-1} A), with full reorthogonalisation, and the extreme
eigenvalues of the tridiagonal matrix T_m.

Start vector: entry i is uniform on (-1, 1), drawn from a SplitMix64 stream
(Steele, Lea and Flood, "Fast splittable pseudorandom number generators",
OOPSLA 2014): the n-th output of the stream seeded with s is
mix(s + (n + 1) * 0x9E3779B97F4A7C15 mod 2^64), with
    mix(z): z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
            z = (z ^ (z >> 27)) * 0x94D049BB133111EB
            return z ^ (z >> 31)
The counter for entry i of the vector of the patch at vertex number v
(lexicographic vertex index) and smoothed level l is
n = (v * 16 + l) * 2^24 + i, and the entry is (top 53 bits) * 2^-52 - 1.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

M64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def splitmix64(seed: int, n: int) -> int:
    z = (seed + (n + 1) * GAMMA) & M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def start_vector(seed: int, vertex: int, level: int, size: int) -> np.ndarray:
    base = (vertex * 16 + level) << 24
    return np.array([(splitmix64(seed, base + i) >> 11) * 2.0 ** -52 - 1.0
                     for i in range(size)])


def lanczos_tridiagonal(M: np.ndarray, v0: np.ndarray, m: int):
    """(alpha, beta) of m Lanczos steps on symmetric M from v0, with full
    reorthogonalisation; stops early when beta_{j+1} < 1e-12 |alpha_j|."""
    n = M.shape[0]
    m = min(m, n)
    V = np.zeros((m, n))
    alpha, beta = [], []
    v = v0 / np.linalg.norm(v0)
    v_prev = np.zeros(n)
    b_prev = 0.0
    for j in range(m):
        V[j] = v
        w = M @ v - b_prev * v_prev
        a = float(w @ v)
        w = w - a * v
        for _ in range(2):  # full reorthogonalisation, twice
            w = w - V[: j + 1].T @ (V[: j + 1] @ w)
        alpha.append(a)
        bnext = float(np.linalg.norm(w))
        if j == m - 1 or bnext < 1e-12 * abs(a):
            break
        beta.append(bnext)
        v_prev, v, b_prev = v, w / bnext, bnext
    return np.array(alpha), np.array(beta)


def extreme_eigenvalues(alpha, beta):
    if len(alpha) == 1:
        return float(alpha[0]), float(alpha[0])
    ev = sla.eigvalsh_tridiagonal(alpha, beta)
    return float(ev[0]), float(ev[-1])


def bounds(A: np.ndarray, dinv: np.ndarray, m: int, seed: int, vertex: int, level: int):
    """(lambda_min, lambda_max) estimates of D^{-1} A from m Lanczos steps."""
    s = np.sqrt(dinv)
    M = s[:, None] * A * s[None, :]
    v0 = start_vector(seed, vertex, level, A.shape[0])
    a, b = lanczos_tridiagonal(M, v0, m)
    return extreme_eigenvalues(a, b)
