"""Argument checks of pmg_patch_setup that run on the host before any device
work (no GPU needed): each invalid request returns its documented status and
a message that names the problem."""
import ctypes

import numpy as np
import pytest

import synth


def _setup(dim, n, p, verts, levels=None, prec="fp64", **kw):
    from paper_2510_17785_amd import _lib as L
    from paper_2510_17785_amd.api import _mesh
    lib = L.load()
    m, keep = _mesh(dim, n, verts)
    mu = np.ones(n ** dim)
    o = L.PmgOpts()
    L.check(lib.pmg_default_opts(ctypes.byref(o)))      # host only: stream stays NULL
    o.precision = {"fp64": L.PMG_FP64, "bf16": L.PMG_BF16_FP32ACC}[prec]
    lv = list(levels or [])
    o.n_levels = len(lv)
    for i, q in enumerate(lv):
        o.levels[i] = q
    for k, v in kw.items():
        setattr(o, k, v)
    h = ctypes.c_void_p()
    st = lib.pmg_patch_setup(ctypes.byref(m), mu.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                             int(p), ctypes.byref(o), ctypes.byref(h))
    return st, lib.pmg_last_error().decode(), h.value


def test_tangled_cell_is_reported():
    from paper_2510_17785_amd import _lib as L
    X = synth.make_vertices(3, 4, 0.0, 1).copy()
    v = 2 + 2 * 5 + 2 * 25             # interior vertex (2,2,2)
    X[v, 0] += 0.6                     # pushed past its neighbours in x
    st, msg, h = _setup(3, 4, 2, X, (2, 1))
    assert st == L.PMG_ERR_DEGENERATE and h is None
    assert "det J" in msg and "cell" in msg


@pytest.mark.parametrize("levels,fragment", [((5, 2, 1), "no kernel compiled"),
                                             ((5, 5, 1), "strictly decrease"),
                                             ((5, 2), "last level")])
def test_level_lists(levels, fragment):
    from paper_2510_17785_amd import _lib as L
    X = synth.make_vertices(3, 4, 0.0, 1)
    st, msg, _ = _setup(3, 4, 5, X, levels)
    want = L.PMG_ERR_UNSUPPORTED if fragment == "no kernel compiled" else L.PMG_ERR_INVALID_ARG
    assert st == want and fragment in msg


def test_bf16_only_where_compiled():
    from paper_2510_17785_amd import _lib as L
    X = synth.make_vertices(3, 4, 0.0, 1)
    st, msg, _ = _setup(3, 4, 4, X, (4, 2, 1), prec="bf16")
    assert st == L.PMG_ERR_UNSUPPORTED and "bf16 3D:7,3,1" in msg


def test_bad_scalars():
    from paper_2510_17785_amd import _lib as L
    X = synth.make_vertices(3, 4, 0.0, 1)
    assert _setup(3, 4, 16, X, None)[0] == L.PMG_ERR_INVALID_ARG          # p > 15
    assert _setup(3, 4, 4, X, (4, 2, 1), precision=7)[0] == L.PMG_ERR_INVALID_ARG
    assert _setup(3, 4, 4, X, (4, 2, 1), cheb_degree=0)[0] == L.PMG_ERR_INVALID_ARG
    assert _setup(3, 4, 4, X, (4, 2, 1), lanczos_steps=1)[0] == L.PMG_ERR_INVALID_ARG
    assert _setup(3, 4, 4, X, (4, 2, 1), n_vcycles=0)[0] == L.PMG_ERR_INVALID_ARG


def test_network_file_rejected_before_device_work(tmp_path):
    # a malformed network file is refused while parsing, with no GPU needed
    from paper_2510_17785_amd import _lib as L
    lib = L.load()
    bad = tmp_path / "bad.bin"
    bad.write_bytes(b"PMGMLP1\x00" + np.array([200, 4], dtype="<i4").tobytes() + b"\x00" * 20)
    h = ctypes.c_void_p()
    mg = ctypes.c_double()
    for path in (bad, tmp_path / "missing.bin"):
        st = lib.pmg_mlp_load(str(path).encode(), 64, None, ctypes.byref(h), ctypes.byref(mg))
        assert st == L.PMG_ERR_INVALID_ARG and h.value is None
    wrong = tmp_path / "wrong.bin"
    wrong.write_bytes(b"NOTANET\x00" + b"\x00" * 64)
    assert lib.pmg_mlp_load(str(wrong).encode(), 64, None, ctypes.byref(h), ctypes.byref(mg)) == L.PMG_ERR_INVALID_ARG


def test_mesh_size_and_degree_checked():
    from paper_2510_17785_amd import _lib as L
    X1 = synth.make_vertices(3, 1, 0.0, 1)
    st, msg, h = _setup(3, 1, 2, X1, (2, 1))
    assert st == L.PMG_ERR_INVALID_ARG and "at least 2 cells" in msg and h is None
    X = synth.make_vertices(3, 4, 0.0, 1)
    st, msg, _ = _setup(3, 4, 0, X, None)
    assert st == L.PMG_ERR_INVALID_ARG and "degree" in msg


@pytest.mark.parametrize("bad", [0.0, -1.0, float("nan"), float("inf")])
def test_coefficients_checked_before_device_work(bad):
    from paper_2510_17785_amd import _lib as L
    from paper_2510_17785_amd.api import _mesh
    lib = L.load()
    X = synth.make_vertices(3, 4, 0.0, 1)
    m, keep = _mesh(3, 4, X)
    mu = np.ones(4 ** 3)
    mu[37] = bad
    o = L.PmgOpts()
    L.check(lib.pmg_default_opts(ctypes.byref(o)))
    o.n_levels = 3
    for i, q in enumerate((4, 2, 1)):
        o.levels[i] = q
    h = ctypes.c_void_p()
    st = lib.pmg_patch_setup(ctypes.byref(m), mu.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 4,
                             ctypes.byref(o), ctypes.byref(h))
    assert st == L.PMG_ERR_INVALID_ARG and h.value is None
    assert "coefficient of cell 37" in lib.pmg_last_error().decode()


def test_independent_patch_and_batch_counts_checked():
    from paper_2510_17785_amd import _lib as L
    lib = L.load()
    o = L.PmgOpts()
    L.check(lib.pmg_default_opts(ctypes.byref(o)))
    V, mu = synth.make_random_patches(3, 2, 0.2, (-1, 1), 3)
    V = np.ascontiguousarray(V)
    mu = np.ascontiguousarray(mu)
    D = ctypes.POINTER(ctypes.c_double)
    h = ctypes.c_void_p()
    st = lib.pmg_patches_setup(3, 0, V.ctypes.data_as(D), mu.ctypes.data_as(D), 4, ctypes.byref(o),
                               ctypes.byref(h))
    assert st == L.PMG_ERR_INVALID_ARG and "patch count" in lib.pmg_last_error().decode()
    mu[1, 3] = -2.0
    st = lib.pmg_patches_setup(3, 2, V.ctypes.data_as(D), mu.ctypes.data_as(D), 4, ctypes.byref(o),
                               ctypes.byref(h))
    assert st == L.PMG_ERR_INVALID_ARG and "patch 1 cell 3" in lib.pmg_last_error().decode()
    st = lib.pmg_batch_setup(None, None, None, 0, ctypes.byref(o), ctypes.byref(h))
    assert st == L.PMG_ERR_INVALID_ARG and h.value is None


@pytest.mark.parametrize("dim,q", [(2, 1), (2, 2), (2, 3), (2, 7), (2, 15), (3, 1), (3, 2), (3, 3), (3, 5), (3, 7)])
def test_simplex_numbering_matches_the_oracle(dim, q):
    # the library numbers the unknowns of a simplicial patch topologically
    # (entities named by their vertices), the oracle by node position on a
    # distorted patch: both must give the same unknown for every cell node
    # and the same first holder (no GPU: host code only)
    import synth
    from oracle import simplex
    from paper_2510_17785_amd import simplex_numbering
    X, cells, _ = synth.make_simplex_patches(dim, 1, 0.2, 11)
    codes, count = simplex_numbering(dim, cells, q)
    gather, n = simplex.numbering(X[0], cells, q)
    assert count == n
    assert np.array_equal(np.where(codes >= 0, codes >> 1, -1), gather)
    first = np.zeros_like(codes)
    seen = set()
    for c in range(dim + 1):
        for a in range(codes.shape[1]):
            g = gather[c, a]
            if g >= 0 and g not in seen:
                seen.add(g)
                first[c, a] = 1
    assert np.array_equal(np.where(codes >= 0, codes & 1, 0), first)


def test_simplex_numbering_rejects_bad_cells():
    import synth
    from paper_2510_17785_amd import simplex_numbering
    from paper_2510_17785_amd._lib import PmgError
    _, cells = synth.simplex_patch(2)
    bad = cells.copy()
    bad[0, 0] = 9
    with pytest.raises(PmgError):
        simplex_numbering(2, bad, 3)
    with pytest.raises(PmgError):
        simplex_numbering(2, cells, 0)
