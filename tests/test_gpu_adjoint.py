"""Adjoint gradients of the HIP path (needs an MI355X).

J = 1/2 sum_e (u_e - u*_e)^T M_e (u_e - u*_e) (lumped GLL mass).  The GPU
gradients with respect to the per-element lambda field and the nodal forcing
are compared with the oracle's dense adjoint on a 3x3x3, p = 6 mesh with a
log-normal lambda field, and with central differences of the GPU's own J on
random directions (also at the full 24^3, p = 6 size).
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


def _setup(n, p, seed):
    prob = W.adjoint(n=n, p=p, seed=seed)
    c = gpu_ctx(prob.n, prob.widths, prob.p, prob.tau, prob.lam)
    vx, _ = c.coords()
    vx = to_host(vx)
    lam_nodes = np.repeat(prob.lam, (p + 1) ** 3)
    f = W.lambda_forcing_sin3(*vx.T, lam_nodes)
    ustar = W.target_with_noise(W.u_sin3(*vx.T), prob.extra["noise_seed"])
    return prob, c, vx, f, ustar


def _mass_diag(prob):
    from oracle.basis import gll_nodes_weights
    _, w = gll_nodes_weights(prob.p)
    wk = np.kron(w, np.kron(w, w))
    out = []
    n1, n2, n3 = prob.n
    for k in range(n3):
        for j in range(n2):
            for i in range(n1):
                out.append(prob.widths[0][i] * prob.widths[1][j] * prob.widths[2][k] / 8.0 * wk)
    return np.concatenate(out)


def test_adjoint_matches_oracle_3x3x3_p6():
    import paper_2007_11891_amd as pkg
    prob, c, vx, f, ustar = _setup(3, 6, 55)
    opts = pkg.default_opts(rtol=1e-14, maxit=5000, check_every=10)
    tr, uv, info = c.solve_forcing(to_dev(f), c.zeros_trace(), opts=opts, allow_noconv=True)
    Md = _mass_diag(prob)
    dJdu = Md * (to_host(uv) - ustar)
    dl, df, ainfo = c.adjoint(to_dev(f), tr, to_dev(dJdu), opts=opts)
    o = oracle.HdgOracle(prob.n, prob.widths, prob.p, prob.tau, prob.lam)
    g = np.zeros(o.layout.n_all)
    ut = o.solve(f, g)
    uo = o.reconstruct(f, ut)
    assert rel_err(to_host(uv), uo) < 1e-11
    dl_ref, df_ref = o.adjoint(f, ut, uo, Md * (uo - ustar))
    assert rel_err(to_host(dl), dl_ref) < 1e-10
    assert rel_err(to_host(df), df_ref) < 1e-10


def _J(c, lam, f, ustar, Md, opts):
    c.set_lambda(to_dev(lam))
    _, uv, _ = c.solve_forcing(to_dev(f), c.zeros_trace(), opts=opts, allow_noconv=True)
    d = to_host(uv) - ustar
    return 0.5 * float(d @ (Md * d))


@pytest.mark.parametrize("n,p,ndir", [(4, 3, 4), (24, 6, 20)])
def test_adjoint_matches_central_differences(n, p, ndir):
    """Directional derivatives of J in (lambda, f) against the adjoint
    gradient; the full-size case uses 20 random unit directions."""
    import paper_2007_11891_amd as pkg
    print(f"[adjoint FD] n={n} p={p} dirs={ndir}", flush=True)
    prob, c, vx, f, ustar = _setup(n, p, 5)
    Md = _mass_diag(prob)
    opts = pkg.default_opts(rtol=1e-13, maxit=20000)
    lam = prob.lam.copy()
    c.set_lambda(to_dev(lam))
    tr, uv, _ = c.solve_forcing(to_dev(f), c.zeros_trace(), opts=opts, allow_noconv=True)
    dl, df, _ = c.adjoint(to_dev(f), tr, to_dev(Md * (to_host(uv) - ustar)), opts=opts)
    dl, df = to_host(dl), to_host(df)
    dirs = W.fd_directions(lam.size, f.size, ndir, prob.extra["fd_seed"])
    eps = 1e-4
    for vl, vf in dirs:
        fd = (_J(c, lam + eps * vl, f + eps * vf, ustar, Md, opts)
              - _J(c, lam - eps * vl, f - eps * vf, ustar, Md, opts)) / (2 * eps)
        an = float(dl @ vl + df @ vf)
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-8), (fd, an)


def test_autograd_function_gradients():
    import paper_2007_11891_amd as pkg
    from paper_2007_11891_amd.autograd import hdg_solve
    prob, c, vx, f, ustar = _setup(3, 4, 7)
    Md = to_dev(_mass_diag(prob))
    opts = pkg.default_opts(rtol=1e-13, maxit=5000)
    lam = to_dev(prob.lam).requires_grad_(True)
    ft = to_dev(f).requires_grad_(True)
    u = hdg_solve(lam, ft, c, opts=opts)
    J = 0.5 * (Md * (u - to_dev(ustar)) ** 2).sum()
    J.backward()
    # same as the C entry point
    c.set_lambda(lam.detach())
    tr, uv, _ = c.solve_forcing(ft.detach(), c.zeros_trace(), opts=opts)
    dl, df, _ = c.adjoint(ft.detach(), tr, Md * (uv - to_dev(ustar)), opts=opts)
    assert rel_err(to_host(lam.grad), to_host(dl)) < 1e-12
    assert rel_err(to_host(ft.grad), to_host(df)) < 1e-12
