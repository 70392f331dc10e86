"""hdg_apply_noalloc against hdg_apply (needs an MI355X).

The entry point that allocates nothing keeps its per-face scratch in the
library's static device array.  Its output must equal hdg_apply's on the
same input (same kernels: identical bits), on two calls in a row, the second
on a smaller mesh (the array keeps the first call's contents), in both bases
and both precisions; sizes beyond its limit are refused.
"""
import numpy as np
import pytest

import workloads as W
from helpers import gpu_ctx, perturbed_mesh, to_dev, to_host

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def _ctx(n, p, seed):
    widths = perturbed_mesh(n, seed)
    lam = np.exp(np.random.default_rng(seed + 1).standard_normal(n[0] * n[1] * n[2]))
    return gpu_ctx(n, widths, p, 1.0, lam)


@pytest.mark.parametrize("basis", ["eigen", "nodal"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_apply_matches_apply_twice(basis, dtype):
    import paper_2007_11891_amd as pkg
    tdt = torch.float64 if dtype == "f64" else torch.float32
    print(f"[noalloc] basis={basis} dtype={dtype}", flush=True)
    for n, p, seed in (((6, 5, 7), 7, 3), ((3, 2, 4), 4, 5)):     # the second call is smaller
        c = _ctx(n, p, seed)
        nf = c.sizes.n_free
        x = to_dev(W.random_trace(nf, seed), tdt)
        ref = to_host(c.apply(x, basis=basis))
        y = torch.full((nf,), float("nan"), dtype=tdt, device="cuda")
        c.apply_noalloc(x, y, basis=basis)
        got = to_host(y)
        assert np.array_equal(got, ref), (n, p, np.abs(got - ref).max())
        # a second call on the same context reuses the array as it left it
        y2 = torch.zeros_like(y)
        c.apply_noalloc(x, y2, basis=basis)
        assert np.array_equal(to_host(y2), ref)
        c.close()


def test_noalloc_refuses_sizes_beyond_its_limit():
    """32 x 32 x 16 at p = 8 has 3.8M free unknowns: two FP64 vectors exceed
    the 48 MiB array; the call fails cleanly and the context stays usable."""
    import paper_2007_11891_amd as pkg
    n, p = (32, 32, 16), 8
    c = gpu_ctx(n, [W.uniform_widths(v) for v in n], p, 1.0, 1.0)
    nf = c.sizes.n_free
    assert 2 * 8 * nf > 48 << 20
    x = torch.ones(nf, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    with pytest.raises(pkg.HdgError):
        c.apply_noalloc(x, y)
    ref = c.apply(x)
    assert torch.isfinite(ref).all()
    c.close()
