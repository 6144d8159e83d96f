"""Patches of boundary vertices (cut to the cells inside the mesh) against the
FP64 oracle, through the C ABI.

The device keeps the two-cell shape per direction, with ghost cells of zero
coefficient and masked nodes on or beyond the boundary; the oracle assembles
the cut patch directly.  Compared on the unmasked nodes, in the cut patch's
own numbering; masked entries must be exactly zero.  Tolerances as in the
interior-patch parity tests (FP64 1e-11 per apply, 1e-10 per solve; FP32
2e-5 / 1e-4).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import fem, lanczos, pmg  # noqa: E402
from oracle.gmg import GMG  # noqa: E402
from oracle.smoother import PatchSmoother as OracleSmoother  # noqa: E402
from oracle.smoother import patch_indices, patch_order  # noqa: E402

from gpu_common import case, rel_err, vlin  # noqa: E402

pytestmark = pytest.mark.gpu

CASES = [("2d-n8-q3", 4, 3, (3, 2, 1)), ("3d-n16-q4", 3, 4, (4, 2, 1)),
         ("3d-n32-q6-learned", 2, 6, (6, 3, 1)), ("3d-n24-q8-batch", 2, 2, (2, 1))]


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def unmasked(v, n, q, dim):
    """Positions (x fastest over (2q-1)^dim) of the cut patch's interior
    nodes, in the cut patch's own order."""
    mi = 2 * q - 1
    rng = []
    for i in range(dim):
        if v[i] == 0:
            rng.append(range(q + 1, 2 * q))
        elif v[i] == n:
            rng.append(range(1, q))
        else:
            rng.append(range(1, 2 * q))
    out = []
    if dim == 2:
        for y in rng[1]:
            for x in rng[0]:
                out.append((x - 1) + mi * (y - 1))
    else:
        for z in rng[2]:
            for y in rng[1]:
                for x in rng[0]:
                    out.append((x - 1) + mi * ((y - 1) + mi * (z - 1)))
    return np.array(out, dtype=np.int64)


def _setup(name, n, p, levels, precision):
    from paper_2510_17785_amd import PatchSmoother
    w, p, levels, X, mu, b = case(name, n, p, levels)
    S = PatchSmoother(w.dim, w.n, p, X, mu, levels=levels, precision=precision, with_boundary=True)
    return w, p, levels, X, mu, b, S, fem.Mesh(w.dim, w.n, X, mu)


def _boundary_sample(order, n, dim):
    kinds = {}
    for j, v in enumerate(order):
        k = sum(1 for i in range(dim) if v[i] in (0, n))
        kinds.setdefault(k, j)
    return [kinds[k] for k in sorted(kinds)]   # one interior, face, edge, corner patch


@pytest.mark.parametrize("name,n,p,levels", CASES)
def test_boundary_order_apply_diag_bounds(dev, name, n, p, levels):
    w, p, levels, X, mu, b, S, mesh = _setup(name, n, p, levels, "fp64")
    order = patch_order(w.dim, w.n, with_boundary=True)
    assert S.n_patches == (w.n + 1) ** w.dim
    assert list(S.patch_vertices()) == [vlin(v, w.n) for v in order]
    rng = np.random.default_rng(3)
    lam = S.bounds()
    for j in _boundary_sample(order, w.n, w.dim):
        v = order[j]
        P = mesh.patch(v)
        s = pmg.LocalSolver(P, levels)
        for l, q in enumerate(levels):
            if l >= len(s.levels):
                break
            idx = unmasked(v, w.n, q, w.dim)
            x = np.zeros((S.n_patches, S.level_sizes[l]))
            x[j, idx] = rng.standard_normal(len(idx))
            y = S.apply(l, torch.tensor(x, device=dev)).cpu().numpy()[j]
            assert rel_err(y[idx], s.A[l] @ x[j, idx]) <= 1e-11, (v, l)
            dg = S.inv_diag(l).cpu().numpy()[j]
            assert rel_err(dg[idx], s.dinv[l]) <= 1e-11, (v, l)
            mask = np.ones(S.level_sizes[l], bool)
            mask[idx] = False
            assert np.all(dg[mask] == 0.0), (v, l)
        for l in range(len(s.levels) - 1):     # smoothed levels of the cut patch
            ref = lanczos.bounds(s.A[l], s.dinv[l], 12, 0, vlin(v, w.n), l)
            assert np.allclose(lam[j, l], ref, rtol=1e-9, atol=0), (v, l, lam[j, l], ref)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name,n,p,levels", CASES)
def test_boundary_residual_and_solve(dev, name, n, p, levels, precision):
    w, p, levels, X, mu, b, S, mesh = _setup(name, n, p, levels, precision)
    order = patch_order(w.dim, w.n, with_boundary=True)
    rng = np.random.default_rng(7)
    u = rng.standard_normal(b.shape) * fem.dirichlet_mask(w.dim, w.n, p)
    r = S.residual(torch.tensor(u, device=dev), torch.tensor(b, device=dev)).cpu().numpy()
    rr = np.zeros((S.n_patches, S.level_sizes[0]))
    for j, v in enumerate(order):
        idx = unmasked(v, w.n, p, w.dim)
        rr[j, idx] = rng.standard_normal(len(idx))
    d = S.local_solve(torch.tensor(rr, device=dev)).cpu().numpy()
    tol_apply = 1e-11 if precision == "fp64" else 2e-5
    tol_solve = 1e-10 if precision == "fp64" else 1e-4
    for j in _boundary_sample(order, w.n, w.dim):
        v = order[j]
        P = mesh.patch(v)
        idx = unmasked(v, w.n, p, w.dim)
        clo, inn = patch_indices(v, p, w.n, w.dim)
        ref = b[inn] - (fem.patch_closure_matrix(P, p) @ u[clo])[P.interior_mask(p)]
        assert rel_err(r[j, idx], ref) <= 50 * tol_apply, v
        mask = np.ones(S.level_sizes[0], bool)
        mask[idx] = False
        assert np.all(r[j, mask] == 0.0) and np.all(d[j, mask] == 0.0), v
        s = pmg.LocalSolver(P, levels)
        s.set_bounds([lanczos.bounds(s.A[l], s.dinv[l], 12, 0, vlin(v, w.n), l)
                      for l in range(len(s.levels) - 1)])
        assert rel_err(d[j, idx], s.solve(rr[j, idx])) <= tol_solve, v


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name,n,p,levels", CASES[:2])
def test_boundary_sweep(dev, name, n, p, levels, precision):
    w, p, levels, X, mu, b, S, mesh = _setup(name, n, p, levels, precision)
    ref = OracleSmoother(mesh, p, levels, with_boundary=True)
    u0 = np.random.default_rng(1).standard_normal(b.shape) * fem.dirichlet_mask(w.dim, w.n, p)
    u = torch.tensor(u0, device=dev)
    S.smooth(u, torch.tensor(b, device=dev), +1)
    S.smooth(u, torch.tensor(b, device=dev), -1)
    expect = ref.sweep(ref.sweep(u0, b, +1), b, -1)
    tol = 1e-10 if precision == "fp64" else 1e-4
    assert rel_err(u.cpu().numpy() - u0, expect - u0) <= tol


@pytest.mark.parametrize("name,n", [("2d-n8-q3", 8), ("3d-n16-q4", 4)])
def test_boundary_gmg_cg(dev, name, n):
    from paper_2510_17785_amd import GMGSolver
    w, p, levels, X, mu, b = case(name, n)
    G = GMGSolver(w.dim, w.n, p, X, mu, levels=levels, with_boundary=True)
    x, it, rel = G.cg(torch.tensor(b, device=dev), rtol=w.rtol)
    xo, ito, hist = GMG(fem.Mesh(w.dim, w.n, X, mu), p, levels, with_boundary=True).cg(b, rtol=w.rtol)
    assert it == ito
    assert rel_err(x.cpu().numpy(), xo) <= 1e-10
