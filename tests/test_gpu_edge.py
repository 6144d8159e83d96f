"""Edge cases of the patch smoother through the C ABI, against the FP64
oracle: the smallest mesh (2 cells per direction: one interior vertex, one
patch), an empty range of colours, and independent-patch batches of one
patch and of a ragged count.  Tolerances as in the interior-patch parity
tests (FP64 1e-11 per apply, 1e-10 per solve or sweep; FP32 2e-5 / 1e-4)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth  # noqa: E402
from oracle import fem, lanczos, pmg  # noqa: E402
from oracle.smoother import PatchSmoother as OracleSmoother  # noqa: E402

from gpu_common import case, rel_err  # noqa: E402

pytestmark = pytest.mark.gpu

TOL_APPLY = {"fp64": 1e-11, "fp32": 2e-5}
TOL_SOLVE = {"fp64": 1e-10, "fp32": 1e-4}


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name,p,levels", [("3d-n16-q4", 4, (4, 2, 1)), ("2d-n8-q3", 3, (3, 2, 1))])
def test_single_patch_mesh(dev, name, p, levels, precision):
    from paper_2510_17785_amd import PatchSmoother
    w, p, levels, X, mu, b = case(name, 2, p, levels)
    S = PatchSmoother(w.dim, 2, p, X, mu, levels=levels, precision=precision)
    assert S.n_patches == 1 and S.n_colors == 2 ** w.dim
    ref = OracleSmoother(fem.Mesh(w.dim, 2, X, mu), p, levels)
    u0 = np.random.default_rng(5).standard_normal(b.shape) * fem.dirichlet_mask(w.dim, 2, p)
    u = torch.tensor(u0, device=dev)
    S.smooth(u, torch.tensor(b, device=dev), +1)
    expect = ref.sweep(u0, b, +1)
    assert rel_err(u.cpu().numpy() - u0, expect - u0) <= TOL_SOLVE[precision]


def test_empty_colour_range_is_a_no_op(dev):
    from paper_2510_17785_amd import PatchSmoother
    w, p, levels, X, mu, b = case("3d-n16-q4", 4)
    S = PatchSmoother(w.dim, w.n, p, X, mu, levels=levels, precision="fp32")
    u = torch.tensor(np.random.default_rng(2).standard_normal(b.shape) * fem.dirichlet_mask(w.dim, w.n, p),
                     device=dev)
    before = u.clone()
    for c in range(S.n_colors + 1):
        S.smooth_colors(u, torch.tensor(b, device=dev), c, c)
    torch.cuda.synchronize()
    assert torch.equal(u, before)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("n", [1, 13])
def test_independent_patches_one_and_ragged(dev, n, precision):
    from paper_2510_17785_amd import PatchBatch
    X, mu = synth.make_random_patches(3, n, 0.25, (-1, 1), 40 + n)
    B = PatchBatch(3, 4, X, mu, levels=(4, 2, 1), precision=precision)
    assert B.n_patches == n
    rng = np.random.default_rng(n)
    x = rng.standard_normal((n, B.level_sizes[0]))
    r = rng.standard_normal((n, B.level_sizes[0]))
    y = B.apply(0, torch.tensor(x, device=dev)).cpu().numpy()
    d = B.local_solve(torch.tensor(r, device=dev)).cpu().numpy()
    for j in range(n):
        s = pmg.LocalSolver(fem.PatchGeometry(X[j], mu[j]), (4, 2, 1))
        s.set_bounds([lanczos.bounds(s.A[l], s.dinv[l], 12, 0, j, l) for l in range(2)])
        assert rel_err(y[j], s.A[0] @ x[j]) <= TOL_APPLY[precision], j
        assert rel_err(d[j], s.solve(r[j])) <= TOL_SOLVE[precision], j
