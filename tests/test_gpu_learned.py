"""GPU tests of the learned Chebyshev bounds: features, network forward,
gradient and training against the FP64 oracle, and what the trained network
gains over per-patch Lanczos and over one fixed interval.

Tolerances: features are computed in FP64 and stored in FP32 (relative
rounding 6e-8), compared to 1e-5 relative; the network runs in FP32, so
outputs agree to 1e-4 and gradients to 1e-3 of their largest entry (sums of
up to 64 x 200 FP32 products); after 30 Adam steps predictions agree to 2e-3
(Adam normalises every step, so FP32 rounding in near-zero gradients moves
parameters by up to the learning rate).
"""
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth  # noqa: E402
from oracle import fem, lanczos, mlp, pmg  # noqa: E402
from oracle.smoother import patch_order  # noqa: E402

from gpu_common import rel_err, vlin  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def test_batch_features_bounds_apply(dev):
    from paper_2510_17785_amd import PatchBatch
    X, mu = synth.make_random_patches(3, 12, 0.3, (-2, 2), 11)
    B = PatchBatch(3, 4, X, mu, levels=(4, 2, 1))
    F = B.features().cpu().numpy()
    lam = B.bounds()
    x = np.random.default_rng(1).standard_normal((12, B.level_sizes[0]))
    y = B.apply(0, torch.tensor(x, device=dev)).cpu().numpy()
    for j in range(12):
        P = fem.PatchGeometry(X[j], mu[j])
        assert rel_err(F[j], mlp.features(P)) <= 1e-5, j
        s = pmg.LocalSolver(P, (4, 2, 1))
        for l in range(2):
            ref = lanczos.bounds(s.A[l], s.dinv[l], 12, 0, j, l)   # patch number as vertex id
            assert np.allclose(lam[j, l], ref, rtol=1e-9), (j, l)
        assert rel_err(y[j], s.A[0] @ x[j]) <= 1e-11


def test_mesh_features(dev):
    from paper_2510_17785_amd import PatchSmoother
    w = synth.workload("3d-n32-q6-learned").scaled(4)
    X = synth.make_vertices(3, 4, w.alpha, w.mesh_seed)
    mu = synth.make_coefficients(3, 4, w.mu_log10, w.coef_seed)
    S = PatchSmoother(3, 4, w.p, X, mu, levels=w.levels)
    F = S.features().cpu().numpy()
    mesh = fem.Mesh(3, 4, X, mu)
    for j, v in enumerate(patch_order(3, 4)):
        assert rel_err(F[j], mlp.features(mesh.patch(v))) <= 1e-5, j


def _net_case(n=64, n_in=200, n_out=4, seed=3):
    rng = np.random.default_rng(seed)
    theta = mlp.glorot_init(n_in, n_out, rng) + 0.02 * rng.standard_normal(mlp.n_params(n_in, n_out))
    X = rng.standard_normal((n, n_in)) * rng.uniform(0.5, 3.0, n_in) + rng.uniform(-2, 2, n_in)
    T = rng.standard_normal((n, n_out))
    return theta, X, T


def test_forward_and_gradient_parity(dev):
    from paper_2510_17785_amd import BoundNet
    theta, X, T = _net_case()
    net = BoundNet(200, 4, theta.astype(np.float32), max_batch=256)
    Xd = torch.tensor(X, dtype=torch.float32, device=dev)
    Td = torch.tensor(T, dtype=torch.float32, device=dev)
    net.fit_standardizer(Xd)
    mean, inv = net.standardizer()
    m_ref, s_ref = mlp.standardiser(X.astype(np.float32).astype(np.float64))
    assert rel_err(mean, m_ref) <= 1e-5 and rel_err(inv, 1.0 / s_ref) <= 1e-4
    Xs = (X - mean.astype(np.float64)) * inv.astype(np.float64)
    th64 = net.params().astype(np.float64)
    Y = net.predict(Xd).cpu().numpy()
    assert rel_err(Y, mlp.forward(th64, Xs, 4)[0]) <= 1e-4
    g, loss = net.gradient(Xd, Td)
    assert rel_err(g, mlp.gradient(th64, Xs, T)) <= 1e-3
    assert abs(loss - mlp.loss(th64, Xs, T)) <= 1e-4 * mlp.loss(th64, Xs, T)


def test_training_matches_oracle(dev):
    from paper_2510_17785_amd import BoundNet
    theta, X, T = _net_case(n=480, n_in=52, n_out=4, seed=5)
    theta = theta.astype(np.float32)
    net = BoundNet(52, 4, theta, max_batch=512)
    Xd = torch.tensor(X, dtype=torch.float32, device=dev)
    Td = torch.tensor(T, dtype=torch.float32, device=dev)
    net.fit_standardizer(Xd)
    mean, inv = net.standardizer()
    order = np.random.default_rng(6).permutation(480).astype(np.int32)[None]
    hist = net.train(Xd, Td, torch.tensor(order, device=dev), 1, 16, 1e-3)
    Xs = (X - mean.astype(np.float64)) * inv.astype(np.float64)
    batches = [order[0][s:s + 16] for s in range(0, 480, 16)]
    th_ref = mlp.train(theta.astype(np.float64), Xs, T, batches, lr=1e-3)
    Y = net.predict(Xd).cpu().numpy()
    assert np.abs(Y - mlp.forward(th_ref, Xs, 4)[0]).max() <= 2e-3
    assert np.isfinite(hist).all()


def _gmg_iterations(w, X, mu, b, dev, precision, setter=None):
    from paper_2510_17785_amd import GMGSolver
    G = GMGSolver(w.dim, w.n, w.p, X, mu, levels=w.levels, precision=precision)
    t = 0.0
    if setter is not None:
        for l in range(1, G.n_mesh_levels):
            S = G.smoother(l)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            setter(S)
            torch.cuda.synchronize()
            t += time.perf_counter() - t0
    _, it, rel = G.cg(torch.tensor(b, device=dev), rtol=w.rtol)
    return it, t


def test_learned_bounds_gain(dev):
    """Train on random patches of the 16^3 Q4 workload's distribution (0.2 h,
    mu = 1), then compare on that mesh: bound setup time and accuracy against
    per-patch Lanczos, and outer CG iterations with Lanczos, learned and one
    fixed interval for all patches."""
    from paper_2510_17785_amd import PatchSmoother
    from paper_2510_17785_amd.learned import train_bound_network
    w = synth.workload("3d-n16-q4")
    Xt, mut = synth.make_random_patches(3, 6000, w.alpha, w.mu_log10, 123)
    res = train_bound_network(3, w.p, w.levels, Xt, mut, epochs=30, batch=256, lr=2e-3, seed=1)
    assert res.epoch_loss[-1] < 0.1 * res.epoch_loss[0]
    assert res.val_rmse.max() < 0.1
    X, mu, b = synth.make_case(w)
    # accuracy and setup time on the mesh, FP32 smoother: the handle's setup
    # with and without per-patch Lanczos (after a warm-up setup), the
    # difference being the Lanczos bounds' cost
    PatchSmoother(3, w.n, w.p, X, mu, levels=w.levels, precision="fp32", bounds="fixed").close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S0 = PatchSmoother(3, w.n, w.p, X, mu, levels=w.levels, precision="fp32", bounds="fixed")
    torch.cuda.synchronize()
    t_fixed_setup = time.perf_counter() - t0
    S0.close()
    t0 = time.perf_counter()
    S = PatchSmoother(3, w.n, w.p, X, mu, levels=w.levels, precision="fp32")
    torch.cuda.synchronize()
    t_lanczos_setup = time.perf_counter() - t0
    t_lanczos = t_lanczos_setup - t_fixed_setup
    lam_l = S.bounds()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nfb = S.set_bounds_mlp(res.net, res.margin)
    torch.cuda.synchronize()
    t_mlp = time.perf_counter() - t0
    lam_m = S.bounds()
    err = np.abs(np.log(lam_m[..., 0]) - np.log(lam_l[..., 0]))
    err_max = np.abs(np.log(lam_m[..., 1]) - res.margin - np.log(lam_l[..., 1]))
    assert nfb == 0
    assert np.median(err_max) < 0.05 and np.quantile(err_max, 0.99) < 0.2
    # the learned lambda_max with its margin covers the Lanczos estimate
    assert np.mean(lam_m[..., 1] >= lam_l[..., 1]) > 0.99
    # outer CG: learned vs Lanczos vs one fixed interval (the largest Lanczos
    # interval over all patches and levels)
    it_l, _ = _gmg_iterations(w, X, mu, b, dev, "fp32")
    it_m, t_set = _gmg_iterations(w, X, mu, b, dev, "fp32", lambda S: S.set_bounds_mlp(res.net, res.margin))
    fixed = lambda S: S.set_bounds(np.broadcast_to(np.array([lam_l[..., 0].min(), lam_l[..., 1].max()]),
                                                   (S.n_patches, S.n_levels - 1, 2)).copy())
    it_f, _ = _gmg_iterations(w, X, mu, b, dev, "fp32", fixed)
    print(f"\nlearned bounds: train {res.train_seconds:.2f} s on 6000 patches (labels "
          f"{res.label_seconds:.2f} s), val rmse {res.val_rmse}, margin {res.margin:.3f}; "
          f"mesh: median |dln lmax| {np.median(err_max):.4f}, p99 {np.quantile(err_max, 0.99):.4f}, "
          f"max {err_max.max():.4f}; lmin median {np.median(err):.4f}; "
          f"bounds setup: Lanczos handle {t_lanczos_setup:.4f} s (Lanczos {t_lanczos:.4f} s), "
          f"network {t_mlp:.4f} s; CG iterations: Lanczos {it_l}, learned {it_m}, fixed {it_f}")
    assert it_m <= it_l + 1
    assert it_m <= it_f
    # the gain: the network's bounds cost a fraction of per-patch Lanczos
    # (12 operator applies per smoothed level and patch) at equal iterations
    assert t_mlp < 0.5 * t_lanczos


def test_network_save_load_round_trip(dev, tmp_path):
    from paper_2510_17785_amd import BoundNet
    theta, X, T = _net_case(n=64, n_in=52, n_out=4, seed=9)
    net = BoundNet(52, 4, theta.astype(np.float32), max_batch=128)
    Xd = torch.tensor(X, dtype=torch.float32, device=dev)
    net.fit_standardizer(Xd)
    path = tmp_path / "net.bin"
    net.save(path, margin=0.125)
    net2, margin = BoundNet.load(path, max_batch=128)
    assert margin == 0.125 and net2.n_in == 52 and net2.n_out == 4
    assert np.array_equal(net2.params(), net.params())
    assert torch.equal(net2.predict(Xd), net.predict(Xd))
