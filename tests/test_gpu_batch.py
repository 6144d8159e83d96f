"""Mixed-degree batches: four independent meshes of degrees 2, 4, 6 and 8
with boundary-vertex patches, smoothed together (instances concurrent per
colour), and hand-set launch shapes.  Every path runs the same patch
updates, so results are compared bit for bit: batch against each instance
smoothed on its own, other launch shapes against the default one.  Graph
sweeps and the batch tuner are switched off in the library (host crashes of
unknown cause); their tests stay in this file, skipped.  Each instance's
own smoother is pinned to the oracle elsewhere (boundary-patch and parity
tests); here the outer FP64 GMG-CG of every degree converges and, at
degrees 2 and 4, takes the oracle's iteration count.  (pytest's own
faulthandler prints the stacks of a crash to the terminal.)"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth  # noqa: E402
from oracle import fem  # noqa: E402
from oracle.gmg import GMG  # noqa: E402

pytestmark = pytest.mark.gpu

PS = (2, 4, 6, 8)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def _inputs(n, seed0=0):
    w = synth.workload("3d-n24-q8-batch")
    X = [synth.make_vertices(3, n, w.alpha, w.mesh_seed + 10 * k) for k in range(len(PS))]
    mu = [np.ones(n ** 3) for _ in PS]
    b = [synth.make_rhs(3, n, p, w.rhs_seed + 10 * k) for k, p in enumerate(PS)]
    u0 = [np.random.default_rng(seed0 + k).standard_normal(bk.shape) * (bk != 0) for k, bk in enumerate(b)]
    return X, mu, b, u0


@pytest.mark.skip(reason="a host crash (segmentation fault) inside pmg_batch_autotune's timing of "
                         "graph replays of tuned launch shapes occurred twice, the second time after "
                         "the kernel attributes were set at setup and the capture error paths were "
                         "fixed; its cause is not known, so the tuner and graphs of non-default "
                         "shapes are switched off in the library and this test stays off the GPU")
def test_batch_graph_and_autotune_bitwise(dev):
    from paper_2510_17785_amd import SmootherBatch
    n = 6
    X, mu, b, u0 = _inputs(n)
    B = SmootherBatch(3, [n] * 4, PS, X, mu, precision="fp32")
    bd = [torch.tensor(x, device=dev) for x in b]
    # reference: each instance alone, forward then backward sweep
    ref = []
    for k, S in enumerate(B.instances):
        u = torch.tensor(u0[k], device=dev)
        S.smooth(u, bd[k], +1)
        S.smooth(u, bd[k], -1)
        ref.append(u.clone())
    assert all(S.n_boundary_patches == 7 ** 3 - 5 ** 3 for S in B.instances)
    # batch, direct
    us = [torch.tensor(x, device=dev) for x in u0]
    B.smooth(us, bd, +1, graph=False)
    B.smooth(us, bd, -1, graph=False)
    for k in range(4):
        assert torch.equal(us[k], ref[k]), PS[k]
    # batch, graph: several replays with host work and synchronisation between
    for rep in range(3):
        for k in range(4):
            us[k].copy_(torch.tensor(u0[k], device=dev))
        torch.cuda.synchronize()
        B.smooth(us, bd, +1, graph=True)
        B.smooth(us, bd, -1, graph=True)
        torch.cuda.synchronize()
        for k in range(4):
            assert torch.equal(us[k], ref[k]), (rep, PS[k])
    assert B.captures == 2 and B.replays == 4
    # other addresses: captured again
    vs = [u.clone() for u in us]
    B.smooth(vs, bd, +1, graph=True)
    torch.cuda.synchronize()
    assert B.captures == 3
    # autotuned launch shapes give the same numbers
    B.autotune(us, bd)
    shapes = [S.launch for S in B.instances]
    for k in range(4):
        us[k].copy_(torch.tensor(u0[k], device=dev))
    B.smooth(us, bd, +1, graph=True)
    B.smooth(us, bd, -1, graph=True)
    torch.cuda.synchronize()
    for k in range(4):
        assert torch.equal(us[k], ref[k]), (PS[k], shapes[k])
    # every launch shape by hand as well (persistent grids, XCD mapping)
    S = B.instances[1]
    for grid, mp in [(0, 1), (64, 1), (8, 0), (3, 0)]:
        S.set_launch(grid, mp)
        u = torch.tensor(u0[1], device=dev)
        S.smooth(u, bd[1], +1)
        S.smooth(u, bd[1], -1)
        assert torch.equal(u, ref[1]), (grid, mp)
    # a launch shape changed after capture makes the batch capture again
    S.set_launch(64, 1)
    c0 = B.captures
    for k in range(4):
        us[k].copy_(torch.tensor(u0[k], device=dev))
    B.smooth(us, bd, +1, graph=True)
    B.smooth(us, bd, -1, graph=True)
    torch.cuda.synchronize()
    assert B.captures == c0 + 2
    for k in range(4):
        assert torch.equal(us[k], ref[k]), PS[k]
    print(f"\ntuned launch shapes (grid, map) per degree {PS}: {shapes}")
    B.close()


@pytest.mark.skip(reason="a host crash (segmentation fault) occurred in this test in one of three "
                         "full GPU runs with unchanged code (graph capture, replays and recaptures "
                         "of the batch sweep); its cause is not known, so graph sweeps are switched "
                         "off in the library and this test stays off the GPU")
def test_batch_graph_replays_and_recapture_bitwise(dev):
    # the sweeps of the test above without the launch-shape tuner: direct
    # batch = each instance alone, graph replays (with host work and
    # synchronisation between) = direct, new vector addresses captured again
    # (the previous graph is destroyed only after its replay has finished)
    from paper_2510_17785_amd import SmootherBatch
    n = 6
    X, mu, b, u0 = _inputs(n)
    B = SmootherBatch(3, [n] * 4, PS, X, mu, precision="fp32")
    bd = [torch.tensor(x, device=dev) for x in b]
    ref = []
    for k, S in enumerate(B.instances):
        u = torch.tensor(u0[k], device=dev)
        S.smooth(u, bd[k], +1)
        S.smooth(u, bd[k], -1)
        ref.append(u.clone())
    us = [torch.tensor(x, device=dev) for x in u0]
    B.smooth(us, bd, +1, graph=False)
    B.smooth(us, bd, -1, graph=False)
    for k in range(4):
        assert torch.equal(us[k], ref[k]), PS[k]
    for rep in range(3):
        for k in range(4):
            us[k].copy_(torch.tensor(u0[k], device=dev))
        torch.cuda.synchronize()
        B.smooth(us, bd, +1, graph=True)
        B.smooth(us, bd, -1, graph=True)
        torch.cuda.synchronize()
        for k in range(4):
            assert torch.equal(us[k], ref[k]), (rep, PS[k])
    assert B.captures == 2 and B.replays == 4
    # other addresses, queued right behind a replay: captured again
    vs = [torch.tensor(x, device=dev) for x in u0]
    for k in range(4):
        us[k].copy_(vs[k])
    B.smooth(us, bd, +1, graph=True)
    B.smooth(vs, bd, +1, graph=True)
    B.smooth(vs, bd, -1, graph=True)
    torch.cuda.synchronize()
    assert B.captures == 4
    for k in range(4):
        assert torch.equal(vs[k], ref[k]), PS[k]
    # an instance's smoother changed after capture: the same addresses are
    # captured again, and the graph sweep equals the direct one
    B.instances[1].set_smoother("cartesian", 0.5)
    es = [torch.tensor(x, device=dev) for x in u0]
    B.smooth(es, bd, +1, graph=False)
    for k in range(4):
        vs[k].copy_(torch.tensor(u0[k], device=dev))
    torch.cuda.synchronize()
    B.smooth(vs, bd, +1, graph=True)
    torch.cuda.synchronize()
    assert B.captures == 5
    for k in range(4):
        assert torch.equal(vs[k], es[k]), PS[k]
    B.close()


def test_batch_eager_with_launch_shapes_and_graph_refusal(dev):
    # hand-set launch shapes (persistent grids, XCD mapping) on the
    # instances: the direct batch sweep gives the default shape's bits; the
    # graph sweep refuses non-default shapes and the tuner is switched off,
    # both without device work
    from paper_2510_17785_amd import SmootherBatch
    from paper_2510_17785_amd._lib import PmgError
    n = 6
    X, mu, b, u0 = _inputs(n)
    B = SmootherBatch(3, [n] * 4, PS, X, mu, precision="fp32")
    bd = [torch.tensor(x, device=dev) for x in b]
    us = [torch.tensor(x, device=dev) for x in u0]
    B.smooth(us, bd, +1, graph=False)
    B.smooth(us, bd, -1, graph=False)
    ref = [u.clone() for u in us]
    for k, (grid, mp) in enumerate([(0, 1), (64, 1), (8, 0), (3, 0)]):
        B.instances[k].set_launch(grid, mp)
    for k in range(4):
        us[k].copy_(torch.tensor(u0[k], device=dev))
    B.smooth(us, bd, +1, graph=False)
    B.smooth(us, bd, -1, graph=False)
    torch.cuda.synchronize()
    for k in range(4):
        assert torch.equal(us[k], ref[k]), PS[k]
    with pytest.raises(PmgError):
        B.smooth(us, bd, +1, graph=True)
    with pytest.raises(PmgError):
        B.autotune(us, bd)
    assert B.captures == 0
    B.close()


@pytest.mark.parametrize("k", range(4))
def test_batch_instance_outer_cg(dev, k):
    from paper_2510_17785_amd import GMGSolver
    p = PS[k]
    n = 4
    X, mu, b, _ = _inputs(n)
    G = GMGSolver(3, n, p, X[k], mu[k], precision="fp32", with_boundary=True)
    G64 = GMGSolver(3, n, p, X[k], mu[k], precision="fp64", with_boundary=True)
    bd = torch.tensor(b[k], device=dev)
    _, it32, rel32 = G.cg(bd, rtol=1e-8)
    x, it64, rel64 = G64.cg(bd, rtol=1e-8)
    assert rel32 <= 1e-8 and rel64 <= 1e-8
    assert it32 <= it64 + 1
    if p <= 4:
        levels = tuple(q for q in (p, p // 2, p // 4) if q >= 1)
        levels = tuple(dict.fromkeys(levels + (1,)))
        xo, ito, _ = GMG(fem.Mesh(3, n, X[k], mu[k]), p, levels, with_boundary=True).cg(b[k], rtol=1e-8)
        assert it64 == ito
        assert np.abs(x.cpu().numpy() - xo).max() <= 1e-10 * np.abs(xo).max()
    print(f"\ndegree {p}: outer CG iterations FP64 {it64}, FP32 {it32}")


def test_batch_instance_outer_cg_fullsize(dev):
    """The degree-6 instance at its full 24^3 size (GMG levels 24^3, 12^3,
    6^3 and the dense coarse solve of the 17^3 unknowns on 3^3): FP32 local
    solver within one outer iteration of FP64."""
    from paper_2510_17785_amd import GMGSolver
    w = synth.workload("3d-n24-q8-batch")
    k, p, n = 2, 6, w.n
    X = synth.make_vertices(3, n, w.alpha, w.mesh_seed + k)
    b = torch.tensor(synth.make_rhs(3, n, p, w.rhs_seed + k), device=dev)
    its = {}
    for prec in ("fp64", "fp32"):
        G = GMGSolver(3, n, p, X, np.ones(n ** 3), precision=prec, with_boundary=True)
        _, its[prec], rel = G.cg(b, rtol=1e-8)
        G.close()
        assert rel <= 1e-8, (prec, rel)
    print(f"\n24^3 Q6 instance: outer CG iterations {its}")
    assert its["fp32"] <= its["fp64"] + 1
