"""Neumann sides and the initial-guess hybridization on the GPU against the
oracle (needs an MI355X).

* the operator (nodal and eigen basis), its transformed diagonal, the
  right-hand side with g_D and g_N, coordinates, the whole solution process
  with every solver (HDG-trans in both CG forms and mixed precision,
  HDG-unprec / -diag / -block) and the adjoint match the oracle at 1e-12
  (1e-10 after mixed precision) for several sets of Neumann sides, including
  meshes one element thick, where one element holds both faces of an axis;
* a tensor polynomial of degree <= p is reproduced with n . grad u = g_N;
* the hybridized trace equals the oracle's flux of equation (fluxu);
* a solve from the hybridized guess of a nearby solution needs fewer
  iterations and reaches the same solution; from the converged trace none.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from helpers import (bc_vector, canonical_oracle_S, face_T, max_rel, perturbed_mesh, rel_err,
                     to_dev, to_host)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

MASKS = [0b000001, 0b000010, 0b101010, 0b111110, 0b010101, 0b111111]
CASES = [((3, 2, 2), 3), ((1, 2, 3), 4), ((2, 1, 1), 2), ((4, 3, 2), 6)]


def _pair(n, p, mask, seed=31, tau=1.0):
    import paper_2007_11891_amd as pkg
    widths = perturbed_mesh(n, seed)
    ne = n[0] * n[1] * n[2]
    lam = np.exp(np.random.default_rng(seed + 1).standard_normal(ne))
    o = oracle.HdgOracle(n, widths, p, tau, lam, neumann=mask)
    c = pkg.HdgContext(n, widths, p, tau, lam, neumann=mask)
    return o, c


def _bc(o, seed=3):
    """Smooth g_D and g_N from u = sin(pi x) sin(pi y) sin(pi z) + 0.3 x."""
    u = lambda x, y, z: W.u_sin3(x, y, z) + 0.3 * x          # noqa: E731
    g = lambda x, y, z: W.grad_sin3(x, y, z) + np.array([0.3, 0.0, 0.0])   # noqa: E731
    return bc_vector(o.layout, u, g, o.trace_coords(), o.trace_normals())


@pytest.mark.parametrize("mask", MASKS)
@pytest.mark.parametrize("n,p", CASES)
def test_operator_and_diagonal(mask, n, p):
    import paper_2007_11891_amd as pkg
    print(f"[neumann operator] mask={mask:06b} n={n} p={p}", flush=True)
    o, c = _pair(n, p, mask)
    L = o.layout
    assert (c.sizes.n_free, c.sizes.n_all, c.sizes.n_vol) == (L.n_free, L.n_all, L.n_vol)
    nf = L.n_free
    Kff = o.assemble_K()[:nf, :nf].toarray()
    x = W.random_trace(nf, 5 + p)
    y = to_host(c.apply(to_dev(x), basis="nodal"))
    assert rel_err(y, Kff @ x) < 1e-12
    S, _ = canonical_oracle_S(o.std)
    T = face_T(S, L, L.n_free_faces)
    Kh = T.T @ Kff @ T
    xh = W.random_trace(nf, 6 + p)
    yh = to_host(c.apply(to_dev(xh), basis="eigen"))
    assert rel_err(yh, Kh @ xh) < 1e-12
    assert max_rel(to_host(c.diagonal()), np.diag(Kh)) < 1e-12
    vx, tx = c.coords()
    assert np.abs(to_host(tx) - o.trace_coords()).max() < 1e-14
    del pkg


@pytest.mark.parametrize("mask", MASKS)
def test_rhs_with_dirichlet_and_neumann_data(mask):
    o, c = _pair((3, 2, 2), 4, mask)
    X = o.volume_coords()
    f = W.f_sin3(*X.T, 1.0)
    bc = _bc(o)
    ref = o.lifted_rhs(f, bc)
    got = to_host(c.rhs(to_dev(f), to_dev(bc)))
    assert rel_err(got, ref) < 1e-12


SOLVERS = [dict(precond=1, variant=0), dict(precond=1, variant=1), dict(precond=1, variant=2),
           dict(precond=0),
           dict(precond=2), dict(precond=3)]


@pytest.mark.parametrize("solver", SOLVERS, ids=lambda s: "-".join(f"{k}{v}" for k, v in s.items()))
@pytest.mark.parametrize("mask", [0b000011, 0b101010, 0b111110, 0b111111])
@pytest.mark.parametrize("n,p", [((3, 2, 2), 4), ((1, 3, 2), 3)])
def test_solve_forcing_matches_oracle(solver, mask, n, p):
    import paper_2007_11891_amd as pkg
    print(f"[neumann solve] {solver} mask={mask:06b} n={n} p={p}", flush=True)
    o, c = _pair(n, p, mask)
    X = o.volume_coords()
    f = W.f_sin3(*X.T, 1.0)
    bc = _bc(o)
    ut = o.solve(f, bc)
    uv = o.reconstruct(f, ut)
    nf = o.layout.n_free
    tr, u_vol, info = c.solve_forcing(to_dev(f), to_dev(bc),
                                      opts=pkg.default_opts(rtol=1e-15, maxit=4000, check_every=7,
                                                            **solver),
                                      allow_noconv=True)
    tr = to_host(tr)
    assert rel_err(tr[:nf], ut[:nf]) < 1e-12, info
    assert np.array_equal(tr[nf:], bc[nf:])
    assert rel_err(to_host(u_vol), uv) < 1e-12, info


def test_mixed_precision_with_neumann():
    import paper_2007_11891_amd as pkg
    o, c = _pair((4, 3, 2), 5, 0b011010)
    X = o.volume_coords()
    f = W.f_sin3(*X.T, 1.0)
    bc = _bc(o)
    ut = o.solve(f, bc)
    nf = o.layout.n_free
    tr, _, info = c.solve_forcing(to_dev(f), to_dev(bc), want_volume=False,
                                  opts=pkg.default_opts(rtol=1e-13, mixed=1))
    assert rel_err(to_host(tr)[:nf], ut[:nf]) < 1e-10, info


@pytest.mark.parametrize("mask", [0b000001, 0b110100, 0b111111])
@pytest.mark.parametrize("p", [2, 3, 5])
def test_polynomial_reproduction_with_neumann_on_gpu(mask, p):
    import paper_2007_11891_amd as pkg
    rng = np.random.default_rng(40 + p)
    cf = rng.standard_normal((p + 1,) * 3)
    u, fu = W.poly_tensor(cf)
    g = W.poly_tensor_grad(cf)
    lam = 1.1
    widths = [np.array([0.3, 0.5, 0.2]), np.array([0.6, 0.4]), np.array([0.45, 0.55])]
    c = pkg.HdgContext((3, 2, 2), widths, p, 1.0, lam, neumann=mask)
    o = oracle.HdgOracle((3, 2, 2), widths, p, 1.0, lam, neumann=mask)
    X, T = o.volume_coords(), o.trace_coords()
    bc = bc_vector(o.layout, u, g, T, o.trace_normals())
    tr, uv, info = c.solve_forcing(to_dev(fu(*X.T, lam)), to_dev(bc),
                                   opts=pkg.default_opts(rtol=1e-14))
    nf = o.layout.n_free
    ref = u(*T[:nf].T)
    assert np.abs(to_host(tr)[:nf] - ref).max() < 1e-10 * np.abs(ref).max(), info
    assert np.abs(to_host(uv) - u(*X.T)).max() < 1e-10 * np.abs(u(*X.T)).max()


@pytest.mark.parametrize("mask", [0, 0b000001, 0b101101, 0b111111])
@pytest.mark.parametrize("n,p", [((3, 2, 2), 3), ((1, 2, 3), 5), ((2, 2, 2), 8)])
def test_hybridize_matches_oracle(mask, n, p):
    print(f"[hybridize] mask={mask:06b} n={n} p={p}", flush=True)
    o, c = _pair(n, p, mask, tau=2.5)
    L = o.layout
    uv = np.random.default_rng(9).standard_normal(L.n_vol)
    bc = np.random.default_rng(10).standard_normal(L.n_all)
    ref = o.hybridize(uv, bc)
    got = to_host(c.hybridize(to_dev(uv), to_dev(bc)))
    assert rel_err(got, ref) < 1e-13
    # without trace: g_N = 0
    bc0 = bc.copy()
    bc0[L.n_faces * L.np_ ** 2:] = 0.0
    got0 = to_host(c.hybridize(to_dev(uv)))
    assert rel_err(got0, o.hybridize(uv, bc0)) < 1e-13


@pytest.mark.parametrize("solver", SOLVERS[:2] + [dict(precond=3), dict(precond=1, mixed=1)],
                         ids=lambda s: "-".join(f"{k}{v}" for k, v in s.items()))
def test_solve_from_hybridized_guess(solver):
    """Start from the hybridized volume solution of lambda 10 % off: fewer
    iterations than from zero, same solution; from the converged trace the
    solver does no iteration."""
    import paper_2007_11891_amd as pkg
    print(f"[guess] {solver}", flush=True)
    n, p, mask = (4, 4, 3), 5, 0b000110
    widths = [W.uniform_widths(v) for v in n]
    c = pkg.HdgContext(n, widths, p, 1.0, 2.0, neumann=mask)
    c2 = pkg.HdgContext(n, widths, p, 1.0, 2.2, neumann=mask)
    o = oracle.HdgOracle(n, widths, p, 1.0, 2.0, neumann=mask)
    X = o.volume_coords()
    f = to_dev(W.f_sin3(*X.T, 2.0))
    bc = to_dev(_bc(o))
    nf = c.sizes.n_free
    opts = pkg.default_opts(rtol=1e-10, **solver)
    tr0, _, info0 = c.solve_forcing(f, bc.clone(), want_volume=False, opts=opts)
    _, u2, _ = c2.solve_forcing(f, bc.clone(), opts=pkg.default_opts(rtol=1e-12))
    tr = bc.clone()
    c.hybridize(u2, bc, out=tr[:nf])
    optg = pkg.default_opts(rtol=1e-10, guess=1, **solver)
    tr1, _, info1 = c.solve_forcing(f, tr, want_volume=False, opts=optg)
    print(f"  zero guess {info0}\n  hybridized guess {info1}", flush=True)
    assert info1["iters"] < info0["iters"]
    assert info1["rel_res"] < 1.5e-10
    ref = o.solve(to_host(f), to_host(bc))[:nf]
    for t in (tr0, tr1):
        assert rel_err(to_host(t)[:nf], ref) < 1e-7
    # from a converged trace (a looser tolerance than it was solved to):
    # nothing to do, the trace comes back through the two face transforms
    tr2 = tr1.clone()
    _, _, info2 = c.solve_forcing(f, tr2, want_volume=False,
                                  opts=pkg.default_opts(rtol=1e-9, guess=1, **solver))
    assert info2["iters"] == 0 and info2["rel_res"] <= 1e-9
    assert rel_err(to_host(tr2), to_host(tr1)) < 1e-14


def test_solve_entry_with_guess_matches_direct():
    import paper_2007_11891_amd as pkg
    o, c = _pair((3, 3, 2), 4, 0b100001)
    nf = o.layout.n_free
    K = o.assemble_K()[:nf, :nf].toarray()
    F = W.random_trace(nf, 77)
    ref = np.linalg.solve(K, F)
    x0 = ref + 1e-3 * W.random_trace(nf, 78)
    for pc in (1, 0, 2, 3):
        u = to_dev(x0)
        u, info = c.solve(to_dev(F), opts=pkg.default_opts(rtol=1e-12, precond=pc, guess=1),
                          u_free=u)
        assert rel_err(to_host(u), ref) < 1e-9, (pc, info)
        assert info["rel_res"] < 1.5e-12, (pc, info)
        if pc != 1:   # the nodal solvers report the nodal residual
            res = np.linalg.norm(F - K @ to_host(u)) / np.linalg.norm(F)
            assert abs(info["rel_res"] - res) <= 1e-2 * res + 1e-15, (pc, info, res)


def test_adjoint_with_neumann_sides():
    import paper_2007_11891_amd as pkg
    o, c = _pair((3, 2, 2), 4, 0b010011)
    X = o.volume_coords()
    f = W.f_sin3(*X.T, 1.0)
    bc = _bc(o)
    ut = o.solve(f, bc)
    uv = o.reconstruct(f, ut)
    target = W.target_with_noise(uv, 3)
    dJdu = o.mass_diag() * (uv - target)
    dl_ref, df_ref = o.adjoint(f, ut, uv, dJdu)
    dl, df, info = c.adjoint(to_dev(f), to_dev(ut), to_dev(dJdu),
                             opts=pkg.default_opts(rtol=1e-14))
    assert rel_err(to_host(dl), dl_ref) < 1e-10, info
    assert rel_err(to_host(df), df_ref) < 1e-10, info


def test_neumann_at_full_size_sampled():
    """16^3 elements, p = 7, four Neumann sides: sampled rows of the operator
    against the oracle, and HDG-trans equals HDG-block to the solve tolerance."""
    import paper_2007_11891_amd as pkg
    n, p, mask = (16, 16, 16), 7, 0b110011
    pr = W.perturbed(16, 7)
    c = pkg.HdgContext(n, pr.widths, p, pr.tau, pr.lam, neumann=mask)
    o = oracle.HdgOracle(n, pr.widths, p, pr.tau, pr.lam, neumann=mask)
    L = o.layout
    nf = L.n_free
    x = W.random_trace(nf, 12)
    y = to_host(c.apply(to_dev(x), basis="nodal"))
    npf = L.np_ ** 2
    rng = np.random.default_rng(3)
    faces = np.concatenate([rng.integers(0, L.n_int_faces, 6),
                            rng.integers(L.n_int_faces, L.n_free_faces, 6)])
    rows = (faces[:, None] * npf + rng.integers(0, npf, (faces.size, 3))).ravel()
    xa = np.zeros(L.n_all)
    xa[:nf] = x
    assert max_rel(y[rows], o.apply_rows(xa, rows)) < 1e-12
    X = c.coords()[0]
    f = torch.sin(X[:, 0]) * torch.cos(X[:, 1]) + X[:, 2]
    bc = c.zeros_trace()
    bc[nf:] = 0.5
    tr1, _, i1 = c.solve_forcing(f, bc.clone(), want_volume=False,
                                 opts=pkg.default_opts(rtol=1e-11))
    tr3, _, i3 = c.solve_forcing(f, bc.clone(), want_volume=False,
                                 opts=pkg.default_opts(rtol=1e-11, precond=3))
    print(f"[neumann 16^3 p=7] trans {i1}  block {i3}", flush=True)
    assert rel_err(to_host(tr1)[:nf], to_host(tr3)[:nf]) < 1e-8
