"""The paper's own solver test on the GPU (needs an MI355X).

Section "Definition of a test case for assessment": (0, 2 pi)^3 with 8^3
elements, Poisson (lambda = 0), tau_e = 25, inhomogeneous Dirichlet data and
forcing from the five-factor manufactured solution with k = 5.  Checked: the
solve against the oracle's direct solve at low degree, the discretization
error falling with p (the paper reports spectral convergence beyond
p ~ 12; degrees up to 16 are built here), and the iteration count of the transformed-basis Jacobi solver
staying near the paper's ~100 over the degrees it describes.
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


def _solve(p, rtol, maxit=20000, allow_noconv=False):
    import paper_2007_11891_amd as pkg
    pr = W.paper_case(p)
    c = gpu_ctx(pr.n, pr.widths, pr.p, pr.tau, pr.lam)
    vx, tx = c.coords()
    vx, tx = to_host(vx), to_host(tx)
    f = W.f_paper(*vx.T, 0.0)
    g = W.u_paper(*tx.T)
    tr = to_dev(g)
    tr[:c.sizes.n_free] = 0
    tr, uv, info = c.solve_forcing(to_dev(f), tr, opts=pkg.default_opts(rtol=rtol, maxit=maxit),
                                   allow_noconv=allow_noconv)
    return pr, c, vx, f, g, to_host(tr), to_host(uv), info


@pytest.mark.parametrize("p", [2, 4])
def test_paper_case_matches_oracle(p):
    print(f"[paper case vs oracle] p={p}", flush=True)
    pr, c, vx, f, g, tr, uv, info = _solve(p, 1e-15, maxit=8000, allow_noconv=True)
    o = oracle.HdgOracle(pr.n, pr.widths, pr.p, pr.tau, pr.lam)
    nf = o.layout.n_free
    ut = o.solve(f, g)
    uo = o.reconstruct(f, ut)
    print(f"[paper case vs oracle] p={p}: iters {info['iters']}, trace {rel_err(tr, ut):.2e}, "
          f"volume {rel_err(uv, uo):.2e}", flush=True)
    # Poisson with tau_e = 25 is ill-conditioned: the CG at stagnation holds
    # the solution to the conditioning times round-off; the residual of the
    # GPU trace in the oracle's assembled system is the sharper check
    K = o.assemble_K()
    F = o.lifted_rhs(f, g)
    res = np.linalg.norm(F - K[:nf, :nf] @ tr[:nf]) / np.linalg.norm(F)
    assert res < 1e-12, res
    assert rel_err(tr, ut) < 1e-10
    assert rel_err(uv, uo) < 1e-10


def test_paper_case_convergence_and_iterations():
    errs, its = {}, {}
    for p in (4, 8, 12, 16):
        pr, c, vx, f, g, tr, uv, info = _solve(p, 1e-10)
        errs[p] = float(np.max(np.abs(uv - W.u_paper(*vx.T))))
        its[p] = info["iters"]
        print(f"[paper case] p={p}: max error {errs[p]:.3e}, iterations {its[p]}", flush=True)
    # the product of five k = 5 waves has up to ~60 radians per unit length,
    # ~7 wavelengths per element: p <= 16 is still in the pre-asymptotic range
    # (the paper reaches its error floor only near p = 26..30)
    assert errs[8] < errs[4] and errs[12] < errs[8] and errs[16] < errs[12]
    assert errs[16] < 0.2 * errs[8]
    for p in (8, 12, 16):
        assert 50 <= its[p] <= 250, its          # the paper: about 100 over a wide range of p


def test_penalty_study_trends():
    """The paper's penalty study (tau_e in {1, 25, 625} on its test case):
    a larger penalty lowers the solution error and costs iterations, by
    about a factor 1.5 from 25 to 625 at p = 2 and much less at high p."""
    import paper_2007_11891_amd as pkg
    res = {}
    for tau_e in (1.0, 25.0, 625.0):
        for p in (2, 12):
            pr = W.paper_case(p, tau_e=tau_e)
            c = pkg.HdgContext(pr.n, pr.widths, pr.p, pr.tau, pr.lam)
            vx, tx = c.coords()
            vx, tx = vx.cpu().numpy(), tx.cpu().numpy()
            f = torch.as_tensor(W.f_paper(*vx.T, 0.0), device="cuda")
            g = torch.as_tensor(W.u_paper(*tx.T), device="cuda")
            u_ex = torch.as_tensor(W.u_paper(*vx.T), device="cuda")
            nf = c.sizes.n_free
            tr = g.clone()
            tr[:nf] = 0
            _, uv, info = c.solve_forcing(f, tr, opts=pkg.default_opts(rtol=1e-10))
            err = float(torch.max(torch.abs(uv - u_ex)))
            print(f"[penalty] tau_e={tau_e:g} p={p}: {info['iters']} it, error {err:.3e}", flush=True)
            assert info["rel_res"] < 1.5e-10
            res[tau_e, p] = (info["iters"], err)
            c.close()
    for p in (2, 12):
        assert res[625.0, p][1] < res[25.0, p][1] < res[1.0, p][1]
        assert res[1.0, p][0] <= res[25.0, p][0] <= res[625.0, p][0]
    grow2 = res[625.0, 2][0] / res[25.0, 2][0]
    grow12 = res[625.0, 12][0] / res[25.0, 12][0]
    assert 1.2 < grow2 < 2.5 and grow12 < grow2


def test_paper_protocol_start_matches_oracle_cg():
    """The paper's protocol: the initial trace is the flux (equation (fluxu))
    of a pseudo-random volume field with the exact values on the boundary,
    and the CG stops when the initial residual has dropped by 1e-10.  On the
    test case with 4^3 elements at p = 4, HDG-trans (guess = 2) stops within
    two iterations of the oracle's Jacobi CG on K^ from the oracle's own
    hybridized start, and reaches the direct solution."""
    import paper_2007_11891_amd as pkg
    from helpers import canonical_oracle_S, face_T
    from oracle.pcg import pcg
    pr = W.paper_case(4, n=4)
    o = oracle.HdgOracle(pr.n, pr.widths, pr.p, pr.tau, pr.lam)
    c = gpu_ctx(pr.n, pr.widths, pr.p, pr.tau, pr.lam)
    L = o.layout
    nf = L.n_free
    X, T = o.volume_coords(), o.trace_coords()
    f = W.f_paper(*X.T, 0.0)
    g = W.u_paper(*T.T)
    u0 = W.paper_initial_volume(X, 11)
    # oracle: start, CG in the eigen basis with the Jacobi preconditioner
    x0 = o.hybridize(u0, g)
    K = o.assemble_K()[:nf, :nf].toarray()
    F = o.lifted_rhs(f, g)
    S, _ = canonical_oracle_S(o.std)
    Tm = face_T(S, L, L.n_free_faces)
    Kh = Tm.T @ K @ Tm
    dinv = 1.0 / np.diag(Kh)
    xh0 = np.linalg.solve(Tm, x0)
    _, its, _ = pcg(Kh, Tm.T @ F, lambda r: dinv * r, rtol=1e-10, x0=xh0, relative_to="initial")
    # GPU: the same start from its own hybridization
    tr = to_dev(g)
    c.hybridize(to_dev(u0), tr, out=tr[:nf])
    assert rel_err(to_host(tr)[:nf], x0) < 1e-13
    tr, uv, info = c.solve_forcing(to_dev(f), tr, opts=pkg.default_opts(rtol=1e-10, guess=2))
    print(f"[paper protocol] GPU {info}, oracle {its} iterations", flush=True)
    assert abs(info["iters"] - its) <= 2, (info, its)
    ref = np.linalg.solve(K, F)
    assert rel_err(to_host(tr)[:nf], ref) < 1e-8
