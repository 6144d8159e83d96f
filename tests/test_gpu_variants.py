"""Every compiled patch-kernel variant against the FP64 oracle.

The variants (level list x precision) are read from the variant tables of
paper_2510_17785_amd/csrc/patch_variants_*.hip, so a level list added there
is covered here without editing this file.  Each runs on a small distorted
mesh with coefficient jumps of two decades (2D: 4 x 4 cells, 9 patches; 3D:
3 x 3 x 3 cells, 8 patches): the operator of every level and the inverse
diagonals on one patch, and one local solve (Algorithm 2 with Lanczos
intervals) on another.  The level operators follow Section 3.1 (level
operators), the local solver Algorithm 2.

Tolerances (relative, max-norm): FP64 1e-11 for an apply and 1e-10 for a
solve; FP32 2e-5 and 1e-4 (the bars of the main parity tests); BF16 operands
2.5e-2 and 5e-2, split BF16 2e-4 and 4e-4 (BF16 rounds the top level's
interpolation operands to 8 bits of mantissa, split BF16 to about 16); the
inverse diagonals come from the FP64 setup kernel for every precision: 1e-11.
"""
import functools
import os
import re

import numpy as np
import pytest

import synth
from oracle import fem
from oracle.smoother import patch_order

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                    "paper_2510_17785_amd", "csrc")
_ENTRY = re.compile(r"make_variant<(double|float),\s*(\d)((?:,\s*\d+)+)>\(\)"
                    r"|make_variant_bf16<(true|false),\s*(\d)((?:,\s*\d+)+)>\(\)")


def compiled_variants():
    """(precision, dim, levels) of every entry of the variant tables."""
    out = []
    for f in sorted(os.listdir(CSRC)):
        if not (f.startswith("patch_variants_") and f.endswith(".hip")):
            continue
        for m in _ENTRY.finditer(open(os.path.join(CSRC, f)).read()):
            if m.group(1):
                prec, dim, lv = {"double": "fp64", "float": "fp32"}[m.group(1)], m.group(2), m.group(3)
            else:
                prec, dim, lv = ("bf16x3" if m.group(4) == "true" else "bf16"), m.group(5), m.group(6)
            out.append((prec, int(dim), tuple(int(x) for x in lv.split(",")[1:])))
    return out


VARIANTS = compiled_variants()
APPLY_TOL = {"fp64": 1e-11, "fp32": 2e-5, "bf16": 2.5e-2, "bf16x3": 2e-4}
SOLVE_TOL = {"fp64": 1e-10, "fp32": 1e-4, "bf16": 5e-2, "bf16x3": 4e-4}


def test_variant_tables_parse():
    # every variant file contributes entries, each level list strictly
    # decreasing to degree 1, and FP64 and FP32 exist for every level list
    files = [f for f in os.listdir(CSRC) if f.startswith("patch_variants_") and f.endswith(".hip")]
    assert len(files) >= 1
    for f in files:
        assert _ENTRY.search(open(os.path.join(CSRC, f)).read()), f
    for prec, dim, levels in VARIANTS:
        assert dim in (2, 3) and levels[-1] == 1
        assert all(a > b for a, b in zip(levels, levels[1:])), levels
    lists = {(d, lv) for _, d, lv in VARIANTS}
    for d, lv in lists:
        assert ("fp64", d, lv) in VARIANTS and ("fp32", d, lv) in VARIANTS, (d, lv)


@functools.lru_cache(maxsize=None)
def _mesh(dim):
    n = 4 if dim == 2 else 3
    X = synth.make_vertices(dim, n, 0.2, 31 + dim)
    mu = synth.make_coefficients(dim, n, (-1.0, 1.0), 41 + dim)
    return n, X, mu


@functools.lru_cache(maxsize=None)
def _oracle(dim, levels):
    """Products with the patch matrices of every level on patch 0, their
    inverse diagonals, and the oracle's local solve on patch 1 (patches in
    sweep order)."""
    from gpu_common import oracle_solver
    n, X, mu = _mesh(dim)
    mesh = fem.Mesh(dim, n, X, mu)
    order = patch_order(dim, n)
    A = [fem.patch_matrix(mesh.patch(order[0]), q) for q in levels]
    rng = np.random.default_rng(11)
    xs = [rng.standard_normal(a.shape[0]) for a in A]
    ys = [a @ x for a, x in zip(A, xs)]
    dg = [1.0 / np.diag(a) for a in A]
    s = oracle_solver(mesh, order[1], levels)
    r = rng.standard_normal(A[0].shape[0])
    return xs, ys, dg, r, s.solve(r)


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.gpu
@pytest.mark.parametrize("precision,dim,levels", VARIANTS,
                         ids=[f"{p}-{d}d-{'-'.join(map(str, lv))}" for p, d, lv in VARIANTS])
def test_variant_against_oracle(precision, dim, levels):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_17785_amd import PatchSmoother
    dev = torch.device("cuda", 0)
    n, X, mu = _mesh(dim)
    p = levels[0]
    S = PatchSmoother(dim, n, p, X, mu, levels=levels, precision=precision)
    assert S.n_patches == (n - 1) ** dim
    xs, ys, dg, r, ref = _oracle(dim, levels)
    for l in range(len(levels)):
        x = np.zeros((S.n_patches, S.level_sizes[l]))
        x[0] = xs[l]
        y = S.apply(l, torch.tensor(x, device=dev)).cpu().numpy()
        # BF16 operands are used on the top level only
        tol = APPLY_TOL[precision] if l == 0 else APPLY_TOL["fp32" if precision != "fp64" else "fp64"]
        assert _rel(y[0], ys[l]) <= tol, (l, _rel(y[0], ys[l]))
        assert _rel(S.inv_diag(l).cpu().numpy()[0], dg[l]) <= 1e-11, l
    rr = np.zeros((S.n_patches, S.level_sizes[0]))
    rr[1] = r
    d = S.local_solve(torch.tensor(rr, device=dev)).cpu().numpy()
    assert _rel(d[1], ref) <= SOLVE_TOL[precision], _rel(d[1], ref)
