"""FP32-inner / FP64-outer defect correction (needs an MI355X).

The mixed-precision solve must reach the FP64 oracle to 1e-10 relative on
sub-meshes with the degrees and lambda values of the 32^3 sweep, and agree
with the plain FP64 GPU solve at the full 32^3 size.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from helpers import gpu_ctx, rel_err, to_dev, to_host

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def _manufactured(c, lam):
    vx, tx = c.coords()
    vx, tx = to_host(vx), to_host(tx)
    f = W.f_mixed(*vx.T, lam)
    g = W.u_mixed(*tx.T)
    return vx, tx, f, g


@pytest.mark.parametrize("variant", [1, 2])
@pytest.mark.parametrize("p", [4, 8])
@pytest.mark.parametrize("lam", [1e-2, 1.0, 1e2])
def test_mixed_precision_matches_oracle_submesh(p, lam, variant):
    """The FP32 inner CG in the plain two-kernel form (variant 1) and in the
    pencil form (variant 2, segments of two elements so that x3 faces are
    summed inside segments and split at their ends)."""
    import paper_2007_11891_amd as pkg
    n = (4, 4, 4) if p == 4 else (3, 3, 3)
    print(f"[mixed vs oracle] n={n} p={p} lam={lam} variant={variant}", flush=True)
    widths = [W.uniform_widths(v) for v in n]
    c = gpu_ctx(n, widths, p, 1.0, lam)
    c.set_cg_segment(2)
    vx, tx, f, g = _manufactured(c, lam)
    tr = to_dev(g)
    tr[:c.sizes.n_free] = 0
    tr, uv, info = c.solve_forcing(to_dev(f), tr, opts=pkg.default_opts(rtol=1e-11, mixed=1,
                                                                          variant=variant))
    assert info["outer_iters"] >= 1 and info["rel_res"] <= 1e-11
    o = oracle.HdgOracle(n, widths, p, 1.0, lam)
    ut = o.solve(f, g)
    uo = o.reconstruct(f, ut)
    assert rel_err(to_host(tr), ut) < 1e-10
    assert rel_err(to_host(uv), uo) < 1e-10


@pytest.mark.parametrize("p", [4, 8, 12])
@pytest.mark.parametrize("lam", [1e-2, 1.0, 1e2])
def test_mixed_precision_matches_fp64_full_size(p, lam):
    """32^3 mesh: FP32-inner / FP64-outer to relative residual 1e-10 agrees
    with the FP64 CG solve to 1e-8 (both are 1e-10-residual solutions)."""
    import paper_2007_11891_amd as pkg
    print(f"[mixed vs fp64] 32^3 p={p} lam={lam}", flush=True)
    prob = W.mixed(p, lam)
    c = gpu_ctx(prob.n, prob.widths, prob.p, prob.tau, lam)
    vx, tx, f, g = _manufactured(c, lam)
    fd = to_dev(f)
    tr64 = to_dev(g)
    tr64[:c.sizes.n_free] = 0
    tr64, u64, i64 = c.solve_forcing(fd, tr64, opts=pkg.default_opts(rtol=1e-10))
    trmx = to_dev(g)
    trmx[:c.sizes.n_free] = 0
    trmx, umx, imx = c.solve_forcing(fd, trmx, opts=pkg.default_opts(rtol=1e-10, mixed=1))
    assert i64["rel_res"] <= 1e-10 * 1.01 and imx["rel_res"] <= 1e-10 * 1.01
    nf = c.sizes.n_free
    assert rel_err(to_host(trmx)[:nf], to_host(tr64)[:nf]) < 1e-8
    # discretisation error against the manufactured solution is far above both
    err = np.abs(to_host(umx) - W.u_mixed(*vx.T)).max()
    assert err < 5e-2
    c.close()
