"""Thin Python interface to libpmg.so with the entry points of include/pmg.h.

Torch is used only to hold device memory and to name the stream; every
computation runs in the library's HIP kernels.  There is no CPU fallback:
constructing any object without the built library, or without a GPU, raises.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as L


def _dptr(t: torch.Tensor) -> int:
    if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError("expected a contiguous float64 device tensor")
    return t.data_ptr()


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream or None


def _opts(levels, precision, cheb_degree, n_vcycles, bounds, lanczos_steps, cheb_safety,
          cheb_range, seed, stream, with_boundary=False) -> L.PmgOpts:
    lib = L.load()
    o = L.PmgOpts()
    L.check(lib.pmg_default_opts(ctypes.byref(o)))
    o.precision = {"fp64": L.PMG_FP64, "fp32": L.PMG_FP32, "bf16": L.PMG_BF16_FP32ACC,
                    "bf16x3": L.PMG_BF16X3_FP32ACC}[precision]
    lv = list(levels) if levels is not None else []
    o.n_levels = len(lv)
    for i, q in enumerate(lv):
        o.levels[i] = int(q)
    o.cheb_degree = int(cheb_degree)
    o.n_vcycles = int(n_vcycles)
    o.bounds = {"lanczos": L.PMG_BOUNDS_LANCZOS, "fixed": L.PMG_BOUNDS_FIXED}[bounds]
    o.lanczos_steps = int(lanczos_steps)
    o.cheb_safety = float(cheb_safety)
    o.cheb_range = float(cheb_range)
    o.seed = int(seed)
    o.stream = _stream_handle(stream)
    o.patch_set = L.PMG_PATCH_WITH_BOUNDARY if with_boundary else L.PMG_PATCH_INTERIOR
    return o


def _fptr(t: torch.Tensor) -> int:
    if not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
        raise ValueError("expected a contiguous float32 device tensor")
    return t.data_ptr()


def _host_f(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def n_features(dim: int) -> int:
    return 3 * 4 ** dim + 2 ** dim


def _mesh(dim, n, vertices):
    v = np.ascontiguousarray(vertices, dtype=np.float64)
    if v.shape != ((n + 1) ** dim, dim):
        raise ValueError(f"vertices must have shape {((n + 1) ** dim, dim)}, got {v.shape}")
    m = L.PmgMesh(dim, n, v.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return m, v


class PatchSmoother:
    """pmg_patch_setup / pmg_patch_smooth and the batched local entry points."""

    def __init__(self, dim: int, n: int, p: int, vertices, coeff, levels: Sequence[int] = None,
                 precision: str = "fp64", cheb_degree: int = 3, n_vcycles: int = 1,
                 bounds: str = "lanczos", lanczos_steps: int = 12, cheb_safety: float = 1.1,
                 cheb_range: float = 15.0, seed: int = 0, stream=None, with_boundary: bool = False,
                 _handle=None, _owner=None):
        self._lib = L.load()
        if not torch.cuda.is_available():
            raise RuntimeError("PatchSmoother needs a GPU")
        self._owner = _owner
        if _handle is not None:
            self._h = _handle
        else:
            m, keep = _mesh(dim, n, vertices)
            mu = np.ascontiguousarray(coeff, dtype=np.float64)
            if mu.shape != (n ** dim,):
                raise ValueError("one coefficient per cell expected")
            o = _opts(levels, precision, cheb_degree, n_vcycles, bounds, lanczos_steps, cheb_safety,
                      cheb_range, seed, stream, with_boundary)
            h = ctypes.c_void_p()
            L.check(self._lib.pmg_patch_setup(ctypes.byref(m), mu.ctypes.data_as(
                ctypes.POINTER(ctypes.c_double)), int(p), ctypes.byref(o), ctypes.byref(h)))
            self._h = h
            del keep
        q = self.query
        self.dim = dim
        self.n_patches = q(L.PMG_Q_N_PATCHES)
        self.n_colors = q(L.PMG_Q_N_COLORS)
        self.n_levels = q(L.PMG_Q_N_LEVELS)
        self.levels = [q(L.PMG_Q_LEVEL_DEGREE + l) for l in range(self.n_levels)]
        self.level_sizes = [q(L.PMG_Q_LEVEL_SIZE + l) for l in range(self.n_levels)]
        self.color_offsets = [q(L.PMG_Q_COLOR_OFFSET + c) for c in range(self.n_colors + 1)]
        self.n_dofs = q(L.PMG_Q_N_DOFS)
        self.n_interior_dofs = q(L.PMG_Q_N_INTERIOR_DOFS)
        self.n_boundary_patches = q(L.PMG_Q_N_BOUNDARY_PATCHES)
        self.local_dofs = q(L.PMG_Q_LOCAL_DOFS)

    def query(self, what: int) -> int:
        v = ctypes.c_int64()
        L.check(self._lib.pmg_query(self._h, int(what), ctypes.byref(v)))
        return v.value

    @property
    def device_bytes(self) -> int:
        return self.query(L.PMG_Q_DEVICE_BYTES)

    def patch_vertices(self) -> np.ndarray:
        out = np.zeros(self.n_patches, dtype=np.int32)
        L.check(self._lib.pmg_get_patch_vertices(self._h, out.ctypes.data_as(
            ctypes.POINTER(ctypes.c_int32))))
        return out

    def smooth(self, u: torch.Tensor, b: torch.Tensor, direction: int = 1):
        L.check(self._lib.pmg_patch_smooth(self._h, _dptr(u), _dptr(b), int(direction)))

    def smooth_additive(self, u: torch.Tensor, b: torch.Tensor, theta: float):
        """pmg_patch_smooth_additive: all patches from the same u, damped by theta."""
        L.check(self._lib.pmg_patch_smooth_additive(self._h, _dptr(u), _dptr(b), float(theta)))

    def smooth_colors(self, u, b, c_begin, c_end):
        L.check(self._lib.pmg_patch_smooth_colors(self._h, _dptr(u), _dptr(b), int(c_begin),
                                                  int(c_end)))

    def residual(self, u: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
        r = torch.empty((self.n_patches, self.level_sizes[0]), dtype=torch.float64, device=u.device)
        L.check(self._lib.pmg_patch_residual(self._h, _dptr(u), _dptr(b), _dptr(r)))
        return r

    def apply(self, level: int, x: torch.Tensor) -> torch.Tensor:
        y = torch.empty_like(x)
        if tuple(x.shape) != (self.n_patches, self.level_sizes[level]):
            raise ValueError("x must have shape (n_patches, level size)")
        L.check(self._lib.pmg_patch_apply(self._h, int(level), _dptr(x), _dptr(y)))
        return y

    def local_solve(self, r: torch.Tensor) -> torch.Tensor:
        if tuple(r.shape) != (self.n_patches, self.level_sizes[0]):
            raise ValueError("r must have shape (n_patches, top level size)")
        d = torch.empty_like(r)
        L.check(self._lib.pmg_patch_local_solve(self._h, _dptr(r), _dptr(d)))
        return d

    def pcg(self, b: torch.Tensor, rtol: float = 1e-8, maxit: int = 200):
        """pmg_patch_pcg: CG on every patch problem A_{j,p} x = b[j],
        preconditioned by the V-cycle.  Returns device tensors (x, iterations
        int32, ||r_k|| / ||b[j]||)."""
        if tuple(b.shape) != (self.n_patches, self.level_sizes[0]):
            raise ValueError("b must have shape (n_patches, top level size)")
        x = torch.empty_like(b)
        it = torch.empty(self.n_patches, dtype=torch.int32, device=b.device)
        rel = torch.empty(self.n_patches, dtype=torch.float64, device=b.device)
        L.check(self._lib.pmg_patch_pcg(self._h, _dptr(b), _dptr(x), float(rtol), int(maxit),
                                        it.data_ptr(), _dptr(rel)))
        return x, it, rel

    def pcg_noalloc(self, b: torch.Tensor, x: torch.Tensor, iters: torch.Tensor, relres: torch.Tensor,
                    rtol: float = 1e-8, maxit: int = 200):
        """pmg_patch_pcg_noalloc: pcg into caller-provided outputs, with no
        device allocation in the library (its work memory is a fixed
        per-GPU array)."""
        n = (self.n_patches, self.level_sizes[0])
        if tuple(b.shape) != n or tuple(x.shape) != n:
            raise ValueError("b and x must have shape (n_patches, top level size)")
        if iters.dtype != torch.int32 or tuple(iters.shape) != (self.n_patches,) or not iters.is_cuda:
            raise ValueError("iters must be an int32 device tensor of n_patches entries")
        if tuple(relres.shape) != (self.n_patches,):
            raise ValueError("relres must have n_patches entries")
        L.check(self._lib.pmg_patch_pcg_noalloc(self._h, _dptr(b), _dptr(x), float(rtol), int(maxit),
                                                iters.data_ptr(), _dptr(relres)))

    def set_smoother(self, kind: str = "chebyshev", omega: float = 0.5):
        """pmg_set_smoother: "chebyshev" (default) or "cartesian" (the
        Cartesian-reinforced smoother with damping omega; pmg_patch_pcg only)."""
        k = {"chebyshev": L.PMG_SMOOTHER_CHEBYSHEV, "cartesian": L.PMG_SMOOTHER_CARTESIAN}[kind]
        L.check(self._lib.pmg_set_smoother(self._h, k, float(omega)))

    def inv_diag(self, level: int) -> torch.Tensor:
        out = torch.empty((self.n_patches, self.level_sizes[level]), dtype=torch.float64,
                          device="cuda")
        L.check(self._lib.pmg_get_inv_diag(self._h, int(level), _dptr(out)))
        return out

    def features(self) -> torch.Tensor:
        """pmg_patch_features: (n_patches, n_features) float32 on the device."""
        out = torch.empty((self.n_patches, n_features(self.dim)), dtype=torch.float32, device="cuda")
        L.check(self._lib.pmg_patch_features(self._h, _fptr(out)))
        return out

    def set_bounds_mlp(self, net: "BoundNet", margin: float, ood_z: float = 8.0) -> int:
        """pmg_set_bounds_mlp; returns the number of patches that fell back to Lanczos."""
        nf = ctypes.c_int64()
        L.check(self._lib.pmg_set_bounds_mlp(self._h, net._h, float(margin), float(ood_z),
                                             ctypes.byref(nf)))
        return nf.value

    def set_launch(self, grid: int, map_mode: int) -> None:
        """pmg_set_launch: smoothing-kernel launch shape (grid 0 = one
        workgroup per patch; map_mode 1 = XCD-aware ranges)."""
        L.check(self._lib.pmg_set_launch(self._h, int(grid), int(map_mode)))

    def autotune(self, u: torch.Tensor, b: torch.Tensor) -> float:
        """pmg_autotune; returns the best time per colour launch in ms."""
        ms = ctypes.c_float()
        L.check(self._lib.pmg_autotune(self._h, _dptr(u), _dptr(b), ctypes.byref(ms)))
        return ms.value

    @property
    def launch(self):
        return self.query(L.PMG_Q_TUNED_GRID), self.query(L.PMG_Q_TUNED_MAP)

    def bounds(self) -> np.ndarray:
        out = np.zeros((self.n_patches, self.n_levels - 1, 2))
        L.check(self._lib.pmg_get_bounds(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def set_bounds(self, lam) -> None:
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        if lam.shape != (self.n_patches, self.n_levels - 1, 2):
            raise ValueError("bounds must have shape (n_patches, n_levels - 1, 2)")
        L.check(self._lib.pmg_set_bounds(self._h, lam.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))

    def close(self):
        if getattr(self, "_h", None) is not None and self._owner is None:
            L.check(self._lib.pmg_patch_destroy(self._h))
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PatchBatch(PatchSmoother):
    """pmg_patches_setup: n independent vertex patches (vertices (n, 3^d, d),
    coefficients (n, 2^d)); no global vector, so no smooth/residual."""

    def __init__(self, dim: int, p: int, vertices, coeff, levels: Sequence[int] = None,
                 precision: str = "fp64", cheb_degree: int = 3, n_vcycles: int = 1,
                 bounds: str = "lanczos", lanczos_steps: int = 12, cheb_safety: float = 1.1,
                 cheb_range: float = 15.0, seed: int = 0, stream=None):
        lib = L.load()
        if not torch.cuda.is_available():
            raise RuntimeError("PatchBatch needs a GPU")
        v = np.ascontiguousarray(vertices, dtype=np.float64)
        mu = np.ascontiguousarray(coeff, dtype=np.float64)
        n = v.shape[0]
        if v.shape != (n, 3 ** dim, dim) or mu.shape != (n, 2 ** dim):
            raise ValueError("vertices (n, 3^d, d) and coefficients (n, 2^d) expected")
        o = _opts(levels, precision, cheb_degree, n_vcycles, bounds, lanczos_steps, cheb_safety,
                  cheb_range, seed, stream)
        h = ctypes.c_void_p()
        L.check(lib.pmg_patches_setup(int(dim), int(n), v.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                      mu.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(p),
                                      ctypes.byref(o), ctypes.byref(h)))
        super().__init__(dim, 2, p, None, None, _handle=h)
        self._owner = None


class BoundNet:
    """pmg_mlp_*: the bound-predicting network n_in -> 64 -> 64 -> 64 -> n_out."""

    def __init__(self, n_in: int, n_out: int, params, max_batch: int = 4096, stream=None):
        self._lib = L.load()
        self.n_in, self.n_out = int(n_in), int(n_out)
        cnt = ctypes.c_int64()
        L.check(self._lib.pmg_mlp_param_count(self.n_in, self.n_out, ctypes.byref(cnt)))
        self.n_params = cnt.value
        arr, ptr = _host_f(params)
        if arr.size != self.n_params:
            raise ValueError(f"{self.n_params} parameters expected")
        h = ctypes.c_void_p()
        L.check(self._lib.pmg_mlp_create(self.n_in, self.n_out, ptr, int(max_batch),
                                         _stream_handle(stream), ctypes.byref(h)))
        self._h = h

    def save(self, path: str, margin: float = 0.0) -> None:
        """pmg_mlp_save: parameters, standardiser and the lambda_max margin."""
        L.check(self._lib.pmg_mlp_save(self._h, float(margin), str(path).encode()))

    @classmethod
    def load(cls, path: str, max_batch: int = 4096, stream=None):
        """pmg_mlp_load; returns (network, margin)."""
        lib = L.load()
        h = ctypes.c_void_p()
        margin = ctypes.c_double()
        L.check(lib.pmg_mlp_load(str(path).encode(), int(max_batch), _stream_handle(stream),
                                 ctypes.byref(h), ctypes.byref(margin)))
        net = cls.__new__(cls)
        net._lib = lib
        net._h = h
        # sizes from the file header
        with open(path, "rb") as f:
            f.read(8)
            net.n_in, net.n_out = (int(x) for x in np.frombuffer(f.read(8), dtype="<i4"))
        cnt = ctypes.c_int64()
        L.check(lib.pmg_mlp_param_count(net.n_in, net.n_out, ctypes.byref(cnt)))
        net.n_params = cnt.value
        return net, margin.value

    def params(self) -> np.ndarray:
        out = np.zeros(self.n_params, dtype=np.float32)
        L.check(self._lib.pmg_mlp_get_params(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return out

    def set_params(self, params):
        arr, ptr = _host_f(params)
        L.check(self._lib.pmg_mlp_set_params(self._h, ptr))

    def fit_standardizer(self, X: torch.Tensor):
        L.check(self._lib.pmg_mlp_fit_standardizer(self._h, _fptr(X), int(X.shape[0])))

    def standardizer(self):
        mean = np.zeros(self.n_in, dtype=np.float32)
        inv = np.zeros(self.n_in, dtype=np.float32)
        L.check(self._lib.pmg_mlp_get_standardizer(self._h, mean.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                                   inv.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return mean, inv

    def set_standardizer(self, mean, inv_std):
        m, pm = _host_f(mean)
        s, ps = _host_f(inv_std)
        L.check(self._lib.pmg_mlp_set_standardizer(self._h, pm, ps))

    def predict(self, X: torch.Tensor) -> torch.Tensor:
        Y = torch.empty((X.shape[0], self.n_out), dtype=torch.float32, device=X.device)
        L.check(self._lib.pmg_mlp_predict(self._h, _fptr(X), int(X.shape[0]), _fptr(Y)))
        return Y

    def gradient(self, X: torch.Tensor, T: torch.Tensor):
        g = np.zeros(self.n_params, dtype=np.float32)
        loss = ctypes.c_double()
        L.check(self._lib.pmg_mlp_gradient(self._h, _fptr(X), _fptr(T), int(X.shape[0]),
                                           g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                           ctypes.byref(loss)))
        return g, loss.value

    def train(self, X: torch.Tensor, T: torch.Tensor, order: torch.Tensor, epochs: int, batch: int,
              lr: float = 1e-3) -> np.ndarray:
        """order: int32 device tensor (epochs, n) of sample indices."""
        if order.dtype != torch.int32 or not order.is_cuda or tuple(order.shape) != (epochs, X.shape[0]):
            raise ValueError("order must be an int32 device tensor of shape (epochs, n)")
        hist = np.zeros(epochs)
        L.check(self._lib.pmg_mlp_train(self._h, _fptr(X), _fptr(T), int(X.shape[0]),
                                        order.data_ptr(), int(epochs), int(batch), float(lr),
                                        hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return hist

    def fit_bounds(self, labels: "PatchSmoother", train_order: torch.Tensor, val_rows: torch.Tensor,
                   epochs: int, batch: int, lr: float = 1e-3):
        """pmg_mlp_fit_bounds: features and ln-bound targets of the patches of
        `labels`, standardiser, training and validation, all in the library.
        train_order: int32 device (epochs, n_train) patch numbers; val_rows:
        int32 device (n_val,).  Returns (epoch losses, validation RMSE per
        output, lambda_max margin)."""
        for t in (train_order, val_rows):
            if t.dtype != torch.int32 or not t.is_cuda or not t.is_contiguous():
                raise ValueError("row lists must be contiguous int32 device tensors")
        if train_order.dim() != 2 or train_order.shape[0] != epochs:
            raise ValueError("train_order must have shape (epochs, n_train)")
        hist = np.zeros(epochs)
        rmse = np.zeros(self.n_out, dtype=np.float32)
        margin = ctypes.c_double()
        L.check(self._lib.pmg_mlp_fit_bounds(
            self._h, labels._h, train_order.data_ptr(), int(train_order.shape[1]), val_rows.data_ptr(),
            int(val_rows.shape[0]), int(epochs), int(batch), float(lr),
            hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            rmse.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), ctypes.byref(margin)))
        return hist, rmse, margin.value

    def close(self):
        if getattr(self, "_h", None) is not None:
            L.check(self._lib.pmg_mlp_destroy(self._h))
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class GMGSolver:
    """gmg_setup / gmg_cg_solve: geometric multigrid with patch smoothers as the
    CG preconditioner."""

    def __init__(self, dim: int, n: int, p: int, vertices, coeff, levels: Sequence[int] = None,
                 precision: str = "fp64", cheb_degree: int = 3, n_vcycles: int = 1,
                 bounds: str = "lanczos", lanczos_steps: int = 12, cheb_safety: float = 1.1,
                 cheb_range: float = 15.0, seed: int = 0, stream=None, with_boundary: bool = False,
                 coarse_mean: str = "arithmetic"):
        self._lib = L.load()
        if not torch.cuda.is_available():
            raise RuntimeError("GMGSolver needs a GPU")
        m, keep = _mesh(dim, n, vertices)
        mu = np.ascontiguousarray(coeff, dtype=np.float64)
        o = _opts(levels, precision, cheb_degree, n_vcycles, bounds, lanczos_steps, cheb_safety,
                  cheb_range, seed, stream, with_boundary)
        o.coarse_mean = {"arithmetic": L.PMG_COARSE_ARITHMETIC, "geometric": L.PMG_COARSE_GEOMETRIC,
                         "harmonic": L.PMG_COARSE_HARMONIC}[coarse_mean]
        h = ctypes.c_void_p()
        L.check(self._lib.gmg_setup(ctypes.byref(m), mu.ctypes.data_as(
            ctypes.POINTER(ctypes.c_double)), int(p), ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        del keep
        v = ctypes.c_int64()
        L.check(self._lib.gmg_query(self._h, 0, ctypes.byref(v)))
        self.n_mesh_levels = v.value
        self.sizes = []
        for l in range(self.n_mesh_levels):
            L.check(self._lib.gmg_query(self._h, 16 + l, ctypes.byref(v)))
            self.sizes.append(v.value)
        self.dim, self.p = dim, p

    def smoother(self, level: int) -> PatchSmoother:
        h = ctypes.c_void_p()
        L.check(self._lib.gmg_level_smoother(self._h, int(level), ctypes.byref(h)))
        return PatchSmoother(self.dim, self.sizes[level], self.p, None, None, _handle=h, _owner=self)

    def apply(self, x: torch.Tensor) -> torch.Tensor:
        y = torch.empty_like(x)
        L.check(self._lib.gmg_apply(self._h, _dptr(x), _dptr(y)))
        return y

    def vcycle(self, r: torch.Tensor) -> torch.Tensor:
        z = torch.empty_like(r)
        L.check(self._lib.gmg_vcycle(self._h, _dptr(r), _dptr(z)))
        return z

    def cg(self, b: torch.Tensor, rtol: float = 1e-8, maxit: int = 100):
        """Returns (x, iterations, relative residual); iterations = maxit + 1
        when CG did not converge."""
        x = torch.empty_like(b)
        it = ctypes.c_int32()
        rel = ctypes.c_double()
        L.check(self._lib.gmg_cg_solve(self._h, _dptr(x), _dptr(b), float(rtol), int(maxit),
                                       ctypes.byref(it), ctypes.byref(rel)))
        return x, it.value, rel.value

    def gmres(self, b: torch.Tensor, rtol: float = 1e-8, maxit: int = 100):
        """gmg_gmres_solve: GMRES with one V-cycle as right preconditioner.
        Returns (x, iterations, relative residual); iterations = maxit + 1
        when it did not converge."""
        x = torch.empty_like(b)
        it = ctypes.c_int32()
        rel = ctypes.c_double()
        L.check(self._lib.gmg_gmres_solve(self._h, _dptr(x), _dptr(b), float(rtol), int(maxit),
                                          ctypes.byref(it), ctypes.byref(rel)))
        return x, it.value, rel.value

    def set_additive(self, theta: float):
        """gmg_set_additive: additive smoothing with damping theta (0: multiplicative)."""
        L.check(self._lib.gmg_set_additive(self._h, float(theta)))

    def set_post_direction(self, direction: int):
        """gmg_set_post_direction: -1 (reversed, symmetric) or +1 (the
        paper's same order)."""
        L.check(self._lib.gmg_set_post_direction(self._h, int(direction)))

    def close(self):
        if getattr(self, "_h", None) is not None:
            L.check(self._lib.gmg_destroy(self._h))
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SmootherBatch:
    """pmg_batch_*: independent meshes of mixed degree smoothed together, per
    colour every instance's launch on a stream of its own (graph sweeps are
    switched off in the library: smooth(graph=True) raises)."""

    def __init__(self, dim: int, ns, ps, vertices, coeffs, precision: str = "fp32",
                 bounds: str = "lanczos", with_boundary: bool = True, cheb_degree: int = 3,
                 lanczos_steps: int = 12, seed: int = 0, stream=None):
        self._lib = L.load()
        if not torch.cuda.is_available():
            raise RuntimeError("SmootherBatch needs a GPU")
        k = len(ps)
        meshes = (L.PmgMesh * k)()
        self._keep = []
        for i in range(k):
            m, v = _mesh(dim, ns[i], vertices[i])
            meshes[i] = m
            mu = np.ascontiguousarray(coeffs[i], dtype=np.float64)
            if mu.shape != (ns[i] ** dim,):
                raise ValueError("one coefficient per cell expected")
            self._keep += [v, mu]
        cptr = (ctypes.POINTER(ctypes.c_double) * k)(
            *[self._keep[2 * i + 1].ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for i in range(k)])
        pp = (ctypes.c_int32 * k)(*[int(x) for x in ps])
        o = _opts(None, precision, cheb_degree, 1, bounds, lanczos_steps, 1.1, 15.0, seed, stream,
                  with_boundary)
        h = ctypes.c_void_p()
        L.check(self._lib.pmg_batch_setup(meshes, cptr, pp, k, ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self.instances = []
        for i in range(k):
            hi = ctypes.c_void_p()
            L.check(self._lib.pmg_batch_instance(self._h, i, ctypes.byref(hi)))
            self.instances.append(PatchSmoother(dim, ns[i], ps[i], None, None, _handle=hi, _owner=self))

    @staticmethod
    def _ptrs(ts):
        return (ctypes.c_void_p * len(ts))(*[_dptr(t) for t in ts])

    def smooth(self, us, bs, direction: int = 1, graph: bool = False):
        f = self._lib.pmg_batch_smooth if graph else self._lib.pmg_batch_smooth_eager
        L.check(f(self._h, self._ptrs(us), self._ptrs(bs), int(direction)))

    def autotune(self, us, bs):
        L.check(self._lib.pmg_batch_autotune(self._h, self._ptrs(us), self._ptrs(bs)))

    def query(self, what: int) -> int:
        v = ctypes.c_int64()
        L.check(self._lib.pmg_batch_query(self._h, int(what), ctypes.byref(v)))
        return v.value

    @property
    def captures(self) -> int:
        return self.query(L.PMG_BQ_CAPTURES)

    @property
    def replays(self) -> int:
        return self.query(L.PMG_BQ_REPLAYS)

    def close(self):
        if getattr(self, "_h", None) is not None:
            self._lib.pmg_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def simplex_numbering(dim: int, cells, q: int):
    """pmg_simplex_numbering: (codes (dim+1, (q+1)^dim) with 2 g + first-holder
    flag or -1, number of unknowns); host only."""
    lib = L.load()
    c = np.ascontiguousarray(cells, dtype=np.int32)
    codes = np.zeros((dim + 1, (q + 1) ** dim), dtype=np.int32)
    cnt = ctypes.c_int32()
    L.check(lib.pmg_simplex_numbering(int(dim), c.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), int(q),
                                      codes.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(cnt)))
    return codes, cnt.value


class SimplexBatch:
    """pmg_simplex_*: independent simplicial vertex patches (vertices (n, nv,
    dim), cells (dim+1, 2^dim), coefficients (n, dim+1))."""

    def __init__(self, dim: int, p: int, vertices, cells, coeff, levels: Sequence[int] = None,
                 cheb_degree: int = 3, n_vcycles: int = 1, cheb_safety: float = 1.1,
                 cheb_range: float = 15.0, stream=None):
        self._lib = L.load()
        if not torch.cuda.is_available():
            raise RuntimeError("SimplexBatch needs a GPU")
        v = np.ascontiguousarray(vertices, dtype=np.float64)
        c = np.ascontiguousarray(cells, dtype=np.int32)
        mu = np.ascontiguousarray(coeff, dtype=np.float64)
        n = v.shape[0]
        nv = 7 if dim == 2 else 15
        if v.shape != (n, nv, dim) or c.shape != (dim + 1, 2 ** dim) or mu.shape != (n, dim + 1):
            raise ValueError("vertices (n, nv, dim), cells (dim+1, 2^dim), coefficients (n, dim+1) expected")
        o = _opts(levels, "fp64", cheb_degree, n_vcycles, "fixed", 12, cheb_safety, cheb_range, 0, stream)
        h = ctypes.c_void_p()
        L.check(self._lib.pmg_simplex_setup(int(dim), int(n), v.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                            c.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                            mu.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(p),
                                            ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self.dim, self.n_patches = dim, n
        self.n_levels = self.query(L.PMG_Q_N_LEVELS)
        self.levels = [self.query(L.PMG_Q_LEVEL_DEGREE + l) for l in range(self.n_levels)]
        self.level_sizes = [self.query(L.PMG_Q_LEVEL_SIZE + l) for l in range(self.n_levels)]

    def query(self, what: int) -> int:
        v = ctypes.c_int64()
        L.check(self._lib.pmg_simplex_query(self._h, int(what), ctypes.byref(v)))
        return v.value

    def set_bounds(self, lam) -> None:
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        if lam.shape != (self.n_patches, self.n_levels - 1, 2):
            raise ValueError("bounds must have shape (n_patches, n_levels - 1, 2)")
        L.check(self._lib.pmg_simplex_set_bounds(self._h, lam.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))

    def inv_diag(self, level: int) -> torch.Tensor:
        out = torch.empty((self.n_patches, self.level_sizes[level]), dtype=torch.float64, device="cuda")
        L.check(self._lib.pmg_simplex_get_inv_diag(self._h, int(level), _dptr(out)))
        return out

    def apply(self, level: int, x: torch.Tensor) -> torch.Tensor:
        if tuple(x.shape) != (self.n_patches, self.level_sizes[level]):
            raise ValueError("x must have shape (n_patches, level size)")
        y = torch.empty_like(x)
        L.check(self._lib.pmg_simplex_apply(self._h, int(level), _dptr(x), _dptr(y)))
        return y

    def local_solve(self, r: torch.Tensor) -> torch.Tensor:
        if tuple(r.shape) != (self.n_patches, self.level_sizes[0]):
            raise ValueError("r must have shape (n_patches, top level size)")
        d = torch.empty_like(r)
        L.check(self._lib.pmg_simplex_local_solve(self._h, _dptr(r), _dptr(d)))
        return d

    def pcg(self, b: torch.Tensor, rtol: float = 1e-8, maxit: int = 200):
        if tuple(b.shape) != (self.n_patches, self.level_sizes[0]):
            raise ValueError("b must have shape (n_patches, top level size)")
        x = torch.empty_like(b)
        it = torch.empty(self.n_patches, dtype=torch.int32, device=b.device)
        rel = torch.empty(self.n_patches, dtype=torch.float64, device=b.device)
        L.check(self._lib.pmg_simplex_pcg(self._h, _dptr(b), _dptr(x), float(rtol), int(maxit),
                                          it.data_ptr(), _dptr(rel)))
        return x, it, rel

    def close(self):
        if getattr(self, "_h", None) is not None:
            L.check(self._lib.pmg_simplex_destroy(self._h))
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
