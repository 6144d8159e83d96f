"""The single-patch study of the local solver (Section 3.2) on the GPU:
batched patch CG with one omega = 1/2 Jacobi V-cycle (levels from 1, 3, 7)
over distortion and coefficient-jump sweeps.

Parity: every patch's CG iteration count equals the oracle's `pcg` on the
same patch and right-hand side, and the final relative residuals agree to
1e-4 of their value (FP64; a count may differ by one only where an oracle
residual lies within 1% of the 1e-8 threshold).

Trends, as the paper states them in the text (its figures' data are not
printed): with the Jacobi smoother the counts grow only gradually with
distortion, depend only weakly on a jump of up to 1e8 in one cell of an
undeformed patch, and with a jump of 1e4 stay close to the
constant-coefficient counts under distortion.  Checked in 2D, where the
paper runs these sweeps; the bars (ratios 1.6, 1.5, 1.3) are this test's
reading of "gradual", "weak" and "close".
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import fem, pmg  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def _oracle_counts(res, rtol=1e-8, maxit=100):
    from paper_2510_17785_amd.study import OMEGA_HALF_BOUNDS
    out = []
    for j in range(len(res["X"])):
        s = pmg.LocalSolver(fem.PatchGeometry(res["X"][j], res["mu"][j]), res["levels"], cheb_degree=1)
        s.set_bounds([OMEGA_HALF_BOUNDS] * (len(res["levels"]) - 1))
        _, k, r = s.pcg(res["b"][j], rtol, maxit)
        near = False
        if k < maxit:
            prev = s.pcg(res["b"][j], 0.0, k - 1)[2] if k > 1 else 1.0
            near = abs(r / rtol - 1) < 0.01 or abs(prev / rtol - 1) < 0.01
        out.append((k, r, near))
    return out


@pytest.mark.parametrize("dim,p,reals", [(2, 3, 3), (2, 7, 3), (2, 15, 1), (3, 3, 3), (3, 7, 1)])
def test_study_matches_oracle(dev, dim, p, reals):
    from paper_2510_17785_amd.study import run_study
    dist = (0.0, 0.2, 0.35) if dim == 2 else (0.0, 0.15, 0.28)
    res = run_study(dim, p, distortions=dist, jumps=(1.0, 1e4, 1e8), realizations=reals, seed=50 + p)
    assert res["levels"] == {3: (3, 1), 7: (7, 3, 1), 15: (15, 7, 3, 1)}[p]
    for j, (k, r, near) in enumerate(_oracle_counts(res)):
        kg, rg = int(res["iterations"][j]), float(res["relres"][j])
        if near:
            assert abs(kg - k) <= 1, (j, kg, k)
        else:
            assert kg == k, (j, kg, k)
            assert abs(rg - r) <= 1e-4 * r, (j, rg, r)
    assert all(row["not_converged"] == 0 for row in res["rows"])


@pytest.mark.parametrize("p", [3, 7, 15])
def test_study_trends_2d(dev, p):
    from paper_2510_17785_amd.study import run_study
    dist = (0.0, 0.1, 0.2, 0.3, 0.35)
    jumps = (1.0, 1e2, 1e4, 1e6, 1e8)
    res = run_study(2, p, distortions=dist, jumps=jumps, realizations=20)
    rows = res["rows"]
    assert all(r["not_converged"] == 0 for r in rows)
    mean = {(r["sweep"], r["value"]): r["mean_iterations"] for r in rows}
    d = [mean[("distortion", x)] for x in dist]
    j = [mean[("jump", x)] for x in jumps]
    jd = [mean[("jump+distortion", x)] for x in dist]
    print(f"\n2D p={p}: distortion {dist} -> {np.round(d, 2).tolist()}; jump {jumps} -> "
          f"{np.round(j, 2).tolist()}; jump 1e4 + distortion -> {np.round(jd, 2).tolist()}")
    # gradual growth with distortion
    assert d[-1] >= d[0] and d[-1] <= 1.6 * d[0]
    # weak dependence on the jump over eight decades
    assert max(j) <= 1.5 * min(j)
    # a jump of 1e4 under distortion stays close to the constant-coefficient counts
    for a, b in zip(jd, d):
        assert a <= 1.3 * b
