"""The launch shapes the benchmark times, bit for bit against the default.

The smoothing kernel runs either one workgroup per patch of a colour or a
persistent grid whose workgroups take several patches in turn, with the
patches dealt linearly or in eight contiguous ranges (one per XCD).  Every
shape runs the same patch updates, so a colour of a sweep must give the same
bits in every shape.  Checked at the full 16^3 Q4 and 32^3 Q7 jump sizes in
FP32 for every candidate of pmg_autotune (including persistent grids below
the colour size) and for the tuner's own pick, over one colour and over a
whole forward sweep.  The default shape itself is pinned to the oracle in
test_gpu_fullsize.py.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth  # noqa: E402

pytestmark = pytest.mark.gpu

# the candidates of pmg_autotune on a 256-CU device: (grid, map)
CANDIDATES = [(0, 0), (0, 1), (256, 1), (512, 1), (1024, 1), (512, 0)]


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


@pytest.mark.parametrize("name", ["3d-n16-q4", "3d-n32-q7-jump"])
def test_launch_shapes_bitwise(dev, name):
    from paper_2510_17785_amd import PatchSmoother
    w = synth.workload(name)
    X, mu, b = synth.make_case(w)
    u0 = np.random.default_rng(3).standard_normal(b.shape) * (b != 0)
    S = PatchSmoother(w.dim, w.n, w.p, X, mu, levels=w.levels, precision="fp32", bounds="fixed")
    # one interval for every patch and level: the shapes do not depend on it
    S.set_bounds(np.broadcast_to(np.array([0.05, 2.5]), (S.n_patches, S.n_levels - 1, 2)).copy())
    sizes = np.diff(S.color_offsets)
    c = int(np.argmax(sizes))                       # the colour the tuner times
    assert any(0 < g < sizes[c] for g, _ in CANDIDATES), "no persistent grid below the colour size"
    bd = torch.tensor(b, device=dev)

    def colour(grid, mp):
        S.set_launch(grid, mp)
        u = torch.tensor(u0, device=dev)
        S.smooth_colors(u, bd, c, c + 1)
        torch.cuda.synchronize()
        return u

    def sweep(grid, mp):
        S.set_launch(grid, mp)
        u = torch.tensor(u0, device=dev)
        S.smooth(u, bd, +1)
        torch.cuda.synchronize()
        return u

    ref_c, ref_s = colour(0, 0), sweep(0, 0)
    assert not torch.equal(ref_c, torch.tensor(u0, device=dev))
    for grid, mp in CANDIDATES[1:]:
        print(f"{name}: grid {grid}, map {mp}", flush=True)
        assert torch.equal(colour(grid, mp), ref_c), (grid, mp)
    # a persistent grid that is not a multiple of the XCD count, linear mapping
    assert torch.equal(colour(37, 0), ref_c)
    # the tuner's pick, over one colour and over a whole sweep
    u = torch.tensor(u0, device=dev)
    S.autotune(u, bd)
    assert torch.equal(u, torch.tensor(u0, device=dev))   # the tuner works on a copy
    pick = S.launch
    print(f"{name}: tuned launch shape {pick}", flush=True)
    assert torch.equal(colour(*pick), ref_c), pick
    assert torch.equal(sweep(*pick), ref_s), pick
    S.close()
