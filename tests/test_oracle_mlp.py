"""Pins of the oracle's patch features and MLP (no GPU)."""
import numpy as np
import pytest

import synth
from oracle import fem, lanczos, mlp, pmg


def _patch(dim, seed, alpha=0.3, mu_log10=(-2, 2)):
    rng = np.random.Generator(np.random.PCG64(seed))
    X, mu = synth.make_random_patch(dim, alpha, mu_log10, rng)
    return fem.PatchGeometry(X, mu)


@pytest.mark.parametrize("dim", [2, 3])
def test_features_cartesian_closed_form(dim):
    # J = h I on a Cartesian patch: det J / h^d = 1, ||J||^2 / h^2 = d,
    # ||cof J||^2 / h^(2(d-1)) = d; constant mu gives zero log features
    h = 0.37
    g = np.array(np.meshgrid(*([np.arange(3)] * dim), indexing="ij"))
    X = np.stack([g[i].transpose(tuple(reversed(range(dim)))).reshape(-1) for i in range(dim)], 1) * h
    f = mlp.features(fem.PatchGeometry(X + 1.5, np.full(2 ** dim, 7.0)))
    n = 4 ** dim
    assert f.shape == (mlp.n_features(dim),)
    assert np.allclose(f[0:3 * n:3], 1.0) and np.allclose(f[1:3 * n:3], dim)
    assert np.allclose(f[2:3 * n:3], dim) and np.allclose(f[3 * n:], 0.0)


@pytest.mark.parametrize("dim", [2, 3])
def test_features_invariances(dim):
    # invariant under rotation, translation and scaling of the patch and under
    # scaling of mu (as the spectrum of D^{-1} A is)
    P = _patch(dim, 3)
    f0 = mlp.features(P)
    rng = np.random.default_rng(1)
    Q, _ = np.linalg.qr(rng.standard_normal((dim, dim)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    P2 = fem.PatchGeometry(2.5 * P.verts @ Q.T + 0.3, 40.0 * P.mu)
    assert np.allclose(mlp.features(P2), f0, atol=1e-12)


def test_spectrum_invariance_matches_features():
    # the labels share the invariances: D^{-1}A of a scaled, rotated patch with
    # scaled mu has the same eigenvalues
    P = _patch(2, 5)
    A = fem.patch_matrix(P, 3)
    ev = np.sort(np.linalg.eigvals(A / np.diag(A)[:, None]).real)
    th = 0.7
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    A2 = fem.patch_matrix(fem.PatchGeometry(3.0 * P.verts @ R.T, 5.0 * P.mu), 3)
    ev2 = np.sort(np.linalg.eigvals(A2 / np.diag(A2)[:, None]).real)
    assert np.allclose(ev, ev2, rtol=1e-10)


def test_gradient_central_differences():
    rng = np.random.default_rng(0)
    n_in, n_out, B = 12, 4, 9
    theta = mlp.glorot_init(n_in, n_out, rng) + 0.05 * rng.standard_normal(mlp.n_params(n_in, n_out))
    X = rng.standard_normal((B, n_in))
    T = rng.standard_normal((B, n_out))
    g = mlp.gradient(theta, X, T)
    eps = 1e-6
    idx = rng.choice(theta.size, 60, replace=False)
    for i in idx:
        e = np.zeros_like(theta)
        e[i] = eps
        fd = (mlp.loss(theta + e, X, T) - mlp.loss(theta - e, X, T)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-7 + 1e-5 * abs(fd), (i, fd, g[i])


def test_glorot_ranges_and_layout():
    rng = np.random.default_rng(2)
    th = mlp.glorot_init(200, 4, rng)
    W1, b1, W2, b2, W3, b3, W4, b4 = mlp.unpack(th, 200, 4)
    assert W1.shape == (200, 64) and W4.shape == (64, 4) and b4.shape == (4,)
    assert np.abs(W1).max() <= np.sqrt(6 / 264) and np.all(b1 == 0)
    assert th.size == 200 * 64 + 64 + 2 * (64 * 64 + 64) + 64 * 4 + 4


def test_adam_first_step_is_signed_lr():
    # with bias correction the first Adam step moves every parameter by lr
    # times the sign of its gradient (up to eps)
    opt = mlp.Adam(5, lr=1e-3)
    g = np.array([1.0, -2.0, 0.5, -1e-3, 3.0])
    th = opt.step(np.zeros(5), g)
    assert np.allclose(th, -1e-3 * np.sign(g), rtol=1e-4)


def test_training_reduces_loss_on_lanczos_labels():
    # small end-to-end check: labels from the oracle's Lanczos on random 2D
    # patches, a few epochs of Adam lower the loss
    levels = (3, 2, 1)
    rng = np.random.default_rng(4)
    Xf, T = [], []
    for s in range(48):
        P = _patch(2, 100 + s)
        sol = pmg.LocalSolver(P, levels)
        lab = [lanczos.bounds(sol.A[l], sol.dinv[l], 12, 0, s, l) for l in range(2)]
        Xf.append(mlp.features(P))
        T.append(np.log(np.array(lab).ravel()))
    Xf, T = np.array(Xf), np.array(T)
    mean, std = mlp.standardiser(Xf)
    Xs = (Xf - mean) / std
    theta = mlp.glorot_init(Xs.shape[1], T.shape[1], rng)
    l0 = mlp.loss(theta, Xs, T)
    batches = [rng.permutation(48)[:16] for _ in range(300)]
    theta = mlp.train(theta, Xs, T, batches, lr=3e-3)
    assert mlp.loss(theta, Xs, T) < 0.2 * l0


def _tanh(x):
    # tanh from its definition through the exponential, independent of numpy's tanh
    import math
    e = math.exp(2.0 * x)
    return (e - 1.0) / (e + 1.0)


def test_forward_hand_computed_network():
    # A 2-input, 2-output network whose weights route one chain through every
    # layer: unit 0 of each hidden layer carries tanh(x0 - 0.5 x1 + 0.1), then
    # tanh(0.8 h + 0.2), then tanh(-1.5 h), and the linear output layer reads
    # y0 = 2 h3 + 0.5 and y1 = -h3 + (unit 1 of layer 3 = tanh(0) = 0) - 1.
    # A dropped hidden layer, tanh on the output, a transposed weight matrix
    # or a bias in the wrong place each change the printed values.
    n_in, n_out = 2, 2
    theta = np.zeros(mlp.n_params(n_in, n_out))
    W1, b1, W2, b2, W3, b3, W4, b4 = mlp.unpack(theta, n_in, n_out)  # views into theta
    W1[0, 0], W1[1, 0], b1[0] = 1.0, -0.5, 0.1
    W2[0, 0], b2[0] = 0.8, 0.2
    W3[0, 0] = -1.5
    W4[0, 0], W4[0, 1], W4[1, 1] = 2.0, -1.0, 3.0
    b4[0], b4[1] = 0.5, -1.0
    X = np.array([[0.3, -0.4], [-1.2, 0.6], [0.0, 0.0]])
    Y, (_, h1, h2, h3) = mlp.forward(theta, X, n_out)
    for row, (x0, x1) in enumerate(X):
        t1 = _tanh(x0 - 0.5 * x1 + 0.1)
        t2 = _tanh(0.8 * t1 + 0.2)
        t3 = _tanh(-1.5 * t2)
        assert Y[row, 0] == pytest.approx(2.0 * t3 + 0.5, abs=1e-14)
        assert Y[row, 1] == pytest.approx(-t3 + 3.0 * _tanh(0.0) - 1.0, abs=1e-14)
        assert h1[row, 0] == pytest.approx(t1, abs=1e-15)
        # every other hidden unit has zero weights and bias: tanh(0) = 0
        assert np.all(h1[row, 1:] == 0) and np.all(h2[row, 1:] == 0) and np.all(h3[row, 1:] == 0)
    # the first row, by hand: t1 = tanh(0.6), t2 = tanh(0.8 t1 + 0.2), t3 = tanh(-1.5 t2)
    assert Y[0, 0] == pytest.approx(-0.8681209, abs=5e-7)
    assert Y[0, 1] == pytest.approx(-0.3159396, abs=5e-7)
