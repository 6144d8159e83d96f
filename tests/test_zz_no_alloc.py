"""pmg_patch_pcg_noalloc, the patch CG that allocates no device memory,
against pmg_patch_pcg: the same kernels, so the solutions, iteration counts
and residuals must agree bit for bit.  Two calls in a row on one GPU, the
second on a smaller batch (the shared work array keeps the first call's
contents), then a batch whose work exceeds the array, refused before any
device work."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def _batch(n, seed, p=4, levels=(4, 2, 1)):
    from paper_2510_17785_amd import PatchBatch
    X, mu = synth.make_random_patches(3, n, 0.2, (-2.0, 2.0), seed)
    return PatchBatch(3, p, X, mu, levels=levels, precision="fp64")


def _run_both(B, seed, dev):
    N = B.level_sizes[0]
    b = torch.tensor(np.random.default_rng(seed).standard_normal((B.n_patches, N)), device=dev)
    x_ref, it_ref, rel_ref = B.pcg(b, 1e-10, 100)
    x = torch.full_like(b, np.nan)
    it = torch.full((B.n_patches,), -1, dtype=torch.int32, device=dev)
    rel = torch.full((B.n_patches,), np.nan, dtype=torch.float64, device=dev)
    B.pcg_noalloc(b, x, it, rel, 1e-10, 100)
    torch.cuda.synchronize()
    assert torch.equal(x, x_ref)
    assert torch.equal(it, it_ref)
    assert torch.equal(rel, rel_ref)
    assert int(it.min()) > 2 and float(rel.max()) <= 1e-10
    return int(it.max())


def test_noalloc_pcg_matches_pcg_twice_then_smaller(dev):
    from paper_2510_17785_amd import _lib
    big = _batch(40, 501)
    small = _batch(7, 502, p=7, levels=(7, 3, 1))
    # first call: 40 Q4 patches; second call: 7 Q7 patches (less work memory,
    # a different layout of the shared array)
    _run_both(big, 11, dev)
    _run_both(small, 12, dev)
    # and the first batch again after the second one wrote the array
    _run_both(big, 13, dev)
    big.close()
    small.close()


def test_noalloc_pcg_refuses_work_beyond_the_array(dev):
    from paper_2510_17785_amd import _lib
    from paper_2510_17785_amd._lib import PmgError
    # 2 x 343 doubles per Q4 patch: 12,229 patches exceed 64 MiB
    n = (64 << 20) // (2 * 343 * 8) + 1
    B = _batch(n, 503)
    N = B.level_sizes[0]
    b = torch.zeros((n, N), dtype=torch.float64, device=dev)
    x = torch.zeros_like(b)
    it = torch.zeros(n, dtype=torch.int32, device=dev)
    rel = torch.zeros(n, dtype=torch.float64, device=dev)
    with pytest.raises(PmgError, match="exceeds"):
        B.pcg_noalloc(b, x, it, rel)
    B.close()
