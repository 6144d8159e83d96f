"""Parity at the full workload sizes, in the default launch shape (one
workgroup per patch; the shapes the benchmark's autotuner picks are checked
bit for bit against it in test_gpu_launch_shapes.py).

One colour of a forward sweep runs on the whole mesh; sampled patches of
that colour are recomputed one by one by the oracle from the same u and b
(same-colour patches are independent, so each update depends only on the
starting vector), and every node outside the colour's patch interiors must
keep its value bit for bit.  At the 32^3 Q7 jump size the outer GMG-CG of the
FP32 and split-BF16 local solvers must converge within one iteration of the
FP64 one, plain BF16 is reported (the FP64 path itself is pinned to the
oracle on down-scaled meshes).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth  # noqa: E402
from oracle import fem  # noqa: E402
from oracle.smoother import PatchSmoother as OracleSmoother  # noqa: E402
from oracle.smoother import patch_indices, patch_order, vertex_color  # noqa: E402

pytestmark = pytest.mark.gpu

# relative to the largest entry of the local correction
TOL = {"fp64": 1e-11, "fp32": 1e-4, "bf16": 5e-2, "bf16x3": 4e-4}

FULL = [("3d-n16-q4", "fp64"), ("3d-n16-q4", "fp32"), ("3d-n32-q7-jump", "fp64"),
        ("3d-n32-q7-jump", "fp32"), ("3d-n32-q7-jump", "bf16"), ("3d-n32-q7-jump", "bf16x3"),
        ("3d-n32-q6-learned", "fp32"),
        ("3d-n24-q8-batch", "fp32")]

_inputs = {}


def _case(name):
    if name not in _inputs:
        _inputs.clear()
        w = synth.workload(name)
        X, mu, b = synth.make_case(w)
        u0 = np.random.default_rng(7).standard_normal(b.shape)
        u0[b == 0.0] = 0.0            # Dirichlet nodes (b is zero exactly there)
        _inputs[name] = (w, X, mu, b, u0)
    return _inputs[name]


def _colour_interior_mask(dim, n, p, c):
    """Nodes inside the interior of some patch of colour c (a product of 1D
    masks: the colour fixes the parity of each vertex coordinate)."""
    m = n * p + 1
    masks = []
    for i in range(dim):
        mk = np.zeros(m, dtype=bool)
        for v in range(1, n):
            if v % 2 == (c >> i) & 1:
                mk[(v - 1) * p + 1:(v + 1) * p] = True
        masks.append(mk)
    full = masks[0][None, :]
    for i in range(1, dim):
        full = (masks[i][:, None] & full.reshape(1, -1)).reshape(-1)[None, :]
    return full.reshape(-1)


@pytest.mark.parametrize("name,precision", FULL)
def test_full_size_colour_sweep(name, precision):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_17785_amd import PatchSmoother
    w, X, mu, b, u0 = _case(name)
    dev = torch.device("cuda", 0)
    S = PatchSmoother(w.dim, w.n, w.p, X, mu, levels=w.levels, precision=precision)
    bd = torch.tensor(b, device=dev)
    order = patch_order(w.dim, w.n)
    mesh = fem.Mesh(w.dim, w.n, X, mu)
    rng = np.random.default_rng(11)
    for c in (0, 2 ** w.dim - 1):
        ud = torch.tensor(u0, device=dev)
        S.smooth_colors(ud, bd, c, c + 1)
        u1 = ud.cpu().numpy()
        inside = _colour_interior_mask(w.dim, w.n, w.p, c)
        assert np.array_equal(u1[~inside], u0[~inside])
        of_c = [v for v in order if vertex_color(v) == c]
        sample = [of_c[i] for i in sorted(rng.choice(len(of_c), 3, replace=False))]
        ref = OracleSmoother(mesh, w.p, w.levels, vertices=sample)
        for v in sample:
            d = ref.solvers[v].solve(ref.local_residual(v, u0, b))
            inn = patch_indices(v, w.p, w.n, w.dim)[1]
            err = np.abs(u1[inn] - u0[inn] - d).max() / np.abs(d).max()
            assert err <= TOL[precision], (name, precision, c, v, err)
    S.close()


def test_full_size_gmg_cg_within_one():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_17785_amd import GMGSolver
    w, X, mu, b, _ = _case("3d-n32-q7-jump")
    bd = torch.tensor(b, device="cuda")
    its = {}
    for prec in ("fp64", "fp32", "bf16", "bf16x3"):
        G = GMGSolver(w.dim, w.n, w.p, X, mu, levels=w.levels, precision=prec)
        _, its[prec], rel = G.cg(bd, rtol=w.rtol)
        G.close()
        # plain BF16 operands may stall above the tolerance at this size: reported only
        assert prec == "bf16" or rel <= w.rtol, (prec, rel)
    print(f"\n32^3 Q7 jump GMG-CG iterations (101 = not converged in 100): {its}")
    assert its["fp32"] <= its["fp64"] + 1
    assert its["bf16x3"] <= its["fp64"] + 1
