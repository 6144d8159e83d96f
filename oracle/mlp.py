"""Learned Chebyshev bounds: patch features and a small MLP, in FP64.

TEST INFRASTRUCTURE (oracle): see oracle/__init__.py.

The paper damps its Jacobi smoother with a fixed weight (Section 3.1); the
Chebyshev interval of this project needs eigenvalue bounds of D^{-1} A_{j,q}
per patch and smoothed level.  Besides Lanczos, a small network predicts them
from the patch's geometry and coefficients.

Features of a patch (all invariant under translation, rotation and scaling of
the patch and under scaling of mu, like the spectrum of D^{-1} A):
  * h = (mean cell volume)^(1/d), the cell volume integrated with the 2-point
    Gauss rule;
  * for every cell c (c = sum c_i 2^i) and every point g of the 2-point Gauss
    rule (g = sum g_i 2^i): det J / h^d, ||J||_F^2 / h^2 and
    ||cof J||_F^2 / h^(2(d-1)), at index (c 2^d + g) 3 + {0, 1, 2};
  * log10 mu_c minus the patch mean of log10 mu, at index 3 4^d + c.
That is 200 features in 3D and 52 in 2D.

Network: inputs standardised with the training-set mean and standard
deviation (a zero deviation counts as 1), three tanh hidden layers of width
64, a linear output of 2 values per smoothed level (ln lambda_min,
ln lambda_max); loss = mean squared error over outputs and samples; Adam
(Kingma and Ba 2015) with bias correction.

Parameter vector layout: W1 (n_in x 64, row-major), b1, W2, b2, W3, b3,
W4 (64 x n_out), b4.
"""
from __future__ import annotations

import numpy as np

from .fem import PatchGeometry, jacobians

HIDDEN = 64


def n_features(dim: int) -> int:
    return 3 * 4 ** dim + 2 ** dim


def features(P: PatchGeometry) -> np.ndarray:
    dim = P.dim
    g1 = np.array([0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)])
    pts = np.array([[g1[(g >> i) & 1] for i in range(dim)] for g in range(2 ** dim)])
    cells = [tuple((c >> i) & 1 for i in range(dim)) for c in range(2 ** dim)]
    X = np.array([P.cell_corners(c) for c in cells])           # (2^d, 2^d, d)
    J = jacobians(X, pts)                                      # (cell, point, d, d)
    det = np.linalg.det(J)
    vol = det.sum(axis=1) / 2 ** dim                           # cell volumes (weights 2^-d)
    h = vol.mean() ** (1.0 / dim)
    fro = (J ** 2).sum(axis=(2, 3))
    if dim == 3:
        cof = np.linalg.inv(J).transpose(0, 1, 3, 2) * det[:, :, None, None]
    else:
        cof = np.stack([np.stack([J[..., 1, 1], -J[..., 1, 0]], -1),
                        np.stack([-J[..., 0, 1], J[..., 0, 0]], -1)], -2)
    cfro = (cof ** 2).sum(axis=(2, 3))
    f = np.zeros(n_features(dim))
    for c in range(2 ** dim):
        for g in range(2 ** dim):
            k = (c * 2 ** dim + g) * 3
            f[k] = det[c, g] / h ** dim
            f[k + 1] = fro[c, g] / h ** 2
            f[k + 2] = cfro[c, g] / h ** (2 * (dim - 1))
    lm = np.log10(np.array([P.cell_mu(c) for c in cells]))
    f[3 * 4 ** dim:] = lm - lm.mean()
    return f


def param_shapes(n_in: int, n_out: int):
    return [(n_in, HIDDEN), (HIDDEN,), (HIDDEN, HIDDEN), (HIDDEN,), (HIDDEN, HIDDEN), (HIDDEN,),
            (HIDDEN, n_out), (n_out,)]


def n_params(n_in: int, n_out: int) -> int:
    return sum(int(np.prod(s)) for s in param_shapes(n_in, n_out))


def unpack(theta, n_in, n_out):
    out, o = [], 0
    for s in param_shapes(n_in, n_out):
        k = int(np.prod(s))
        out.append(theta[o:o + k].reshape(s))
        o += k
    return out


def glorot_init(n_in: int, n_out: int, rng: np.random.Generator) -> np.ndarray:
    """Glorot-uniform weights U(-a, a), a = sqrt(6 / (fan_in + fan_out)), zero biases."""
    parts = []
    for s in param_shapes(n_in, n_out):
        if len(s) == 2:
            a = np.sqrt(6.0 / (s[0] + s[1]))
            parts.append(rng.uniform(-a, a, size=s).ravel())
        else:
            parts.append(np.zeros(s))
    return np.concatenate(parts)


def standardiser(X):
    mean = X.mean(axis=0)
    std = X.std(axis=0)
    std[std == 0] = 1.0
    return mean, std


def forward(theta, Xs, n_out):
    """Xs: standardised inputs (B, n_in).  Returns (Y, cache)."""
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(theta, Xs.shape[1], n_out)
    h1 = np.tanh(Xs @ W1 + b1)
    h2 = np.tanh(h1 @ W2 + b2)
    h3 = np.tanh(h2 @ W3 + b3)
    Y = h3 @ W4 + b4
    return Y, (Xs, h1, h2, h3)


def loss(theta, Xs, T):
    Y, _ = forward(theta, Xs, T.shape[1])
    return float(np.mean((Y - T) ** 2))


def gradient(theta, Xs, T):
    """d loss / d theta by backpropagation."""
    n_in, n_out = Xs.shape[1], T.shape[1]
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(theta, n_in, n_out)
    Y, (X0, h1, h2, h3) = forward(theta, Xs, n_out)
    dY = 2.0 * (Y - T) / Y.size
    gW4 = h3.T @ dY
    gb4 = dY.sum(axis=0)
    d3 = (dY @ W4.T) * (1.0 - h3 ** 2)
    gW3 = h2.T @ d3
    gb3 = d3.sum(axis=0)
    d2 = (d3 @ W3.T) * (1.0 - h2 ** 2)
    gW2 = h1.T @ d2
    gb2 = d2.sum(axis=0)
    d1 = (d2 @ W2.T) * (1.0 - h1 ** 2)
    gW1 = X0.T @ d1
    gb1 = d1.sum(axis=0)
    return np.concatenate([g.ravel() for g in (gW1, gb1, gW2, gb2, gW3, gb3, gW4, gb4)])


class Adam:
    def __init__(self, n, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps

    def step(self, theta, g):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mhat = self.m / (1 - self.b1 ** self.t)
        vhat = self.v / (1 - self.b2 ** self.t)
        return theta - self.lr * mhat / (np.sqrt(vhat) + self.eps)


def train(theta, Xs, T, batches, lr=1e-3):
    """Adam over the given mini-batches (lists of row indices); returns theta."""
    opt = Adam(theta.size, lr=lr)
    for idx in batches:
        theta = opt.step(theta, gradient(theta, Xs[idx], T[idx]))
    return theta
