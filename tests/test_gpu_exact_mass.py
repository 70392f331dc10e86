"""The exact (non-lumped) GLL mass matrix on the GPU against the oracle
(needs an MI355X).

With exact mass the transformed face term couples the two opposite faces of
every element through the 2 x 2 matrix G + C^T M^-1 C.  Checked at 1e-12
against the oracle built with the same mass matrix: the operator in both
bases and every tile shape, its transformed diagonal, the right-hand side
with Dirichlet and Neumann data, the whole solution process with every
solver, polynomial reproduction, and the adjoint; the FP32 apply at 1e-5.
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


def _pair(n, p, mask=0, seed=51, tau=1.0):
    import paper_2007_11891_amd as pkg
    widths = perturbed_mesh(n, seed)
    ne = n[0] * n[1] * n[2]
    lam = np.exp(np.random.default_rng(seed + 1).standard_normal(ne))
    o = oracle.HdgOracle(n, widths, p, tau, lam, exact_mass=True, neumann=mask)
    c = pkg.HdgContext(n, widths, p, tau, lam, neumann=mask, exact_mass=True)
    return o, c


@pytest.mark.parametrize("n,p", [((2, 2, 2), 1), ((3, 2, 2), 2), ((2, 3, 2), 4), ((3, 3, 3), 7),
                                 ((2, 1, 2), 10), ((2, 2, 1), 16)])
def test_operator_every_tile_and_diagonal(n, p):
    print(f"[exact mass operator] n={n} p={p}", flush=True)
    o, c = _pair(n, p, mask=0b000010)
    L = o.layout
    nf = L.n_free
    Kff = o.assemble_K()[:nf, :nf].toarray()
    x = W.random_trace(nf, 3 + p)
    ref = Kff @ x
    for v in range(3):
        c.set_tile(v)
        assert rel_err(to_host(c.apply(to_dev(x), basis="nodal")), ref) < 1e-12, v
    S, _ = canonical_oracle_S(o.std)
    T = face_T(S, L, L.n_free_faces)
    Kh = T.T @ Kff @ T
    xh = W.random_trace(nf, 4 + p)
    assert rel_err(to_host(c.apply(to_dev(xh), basis="eigen")), Kh @ xh) < 1e-12
    assert max_rel(to_host(c.diagonal()), np.diag(Kh)) < 1e-12
    y32 = to_host(c.apply(to_dev(xh, torch.float32), basis="eigen")).astype(np.float64)
    assert rel_err(y32, Kh @ xh) < 1e-5


@pytest.mark.parametrize("mask", [0, 0b100101])
def test_rhs_with_boundary_data(mask):
    o, c = _pair((3, 2, 2), 5, mask)
    X = o.volume_coords()
    f = W.f_sin3(*X.T, 1.0)
    u = lambda x, y, z: W.u_sin3(x, y, z) + 0.2 * y      # noqa: E731
    g = lambda x, y, z: W.grad_sin3(x, y, z) + np.array([0.0, 0.2, 0.0])   # noqa: E731
    bc = bc_vector(o.layout, u, g, o.trace_coords(), o.trace_normals())
    assert rel_err(to_host(c.rhs(to_dev(f), to_dev(bc))), o.lifted_rhs(f, bc)) < 1e-12


SOLVERS = [dict(precond=1, variant=0), dict(precond=1, variant=1), dict(precond=1, variant=2),
           dict(precond=0),
           dict(precond=2), dict(precond=3)]


@pytest.mark.parametrize("solver", SOLVERS, ids=lambda s: "-".join(f"{k}{v}" for k, v in s.items()))
@pytest.mark.parametrize("mask", [0, 0b001100])
def test_solve_forcing_matches_oracle(solver, mask):
    import paper_2007_11891_amd as pkg
    print(f"[exact mass solve] {solver} mask={mask:06b}", flush=True)
    o, c = _pair((3, 3, 2), 4, mask)
    X = o.volume_coords()
    f = W.f_sin3(*X.T, 1.0)
    bc = bc_vector(o.layout, W.u_sin3, W.grad_sin3, o.trace_coords(), o.trace_normals())
    ut = o.solve(f, bc)
    uv = o.reconstruct(f, ut)
    nf = o.layout.n_free
    tr, u_vol, info = c.solve_forcing(to_dev(f), to_dev(bc),
                                      opts=pkg.default_opts(rtol=1e-15, maxit=4000, check_every=7,
                                                            **solver),
                                      allow_noconv=True)
    assert rel_err(to_host(tr)[:nf], ut[:nf]) < 1e-12, info
    assert rel_err(to_host(u_vol), uv) < 1e-12, info


def test_mixed_precision_exact_mass():
    import paper_2007_11891_amd as pkg
    o, c = _pair((4, 3, 3), 6)
    X = o.volume_coords()
    f = W.f_sin3(*X.T, 1.0)
    ut = o.solve(f, np.zeros(o.layout.n_all))
    nf = o.layout.n_free
    tr, _, info = c.solve_forcing(to_dev(f), c.zeros_trace(), want_volume=False,
                                  opts=pkg.default_opts(rtol=1e-13, mixed=1))
    assert rel_err(to_host(tr)[:nf], ut[:nf]) < 1e-10, info


@pytest.mark.parametrize("p", [2, 3, 6])
def test_polynomial_reproduction_exact_mass(p):
    import paper_2007_11891_amd as pkg
    rng = np.random.default_rng(70 + p)
    cf = rng.standard_normal((p + 1,) * 3)
    u, fu = W.poly_tensor(cf)
    g = W.poly_tensor_grad(cf)
    lam = 0.7
    widths = [np.array([0.3, 0.5, 0.2]), np.array([0.6, 0.4]), np.array([0.45, 0.55])]
    mask = 0b010001
    c = pkg.HdgContext((3, 2, 2), widths, p, 1.0, lam, neumann=mask, exact_mass=True)
    o = oracle.HdgOracle((3, 2, 2), widths, p, 1.0, lam, neumann=mask, exact_mass=True)
    X, T = o.volume_coords(), o.trace_coords()
    bc = bc_vector(o.layout, u, g, T, o.trace_normals())
    tr, uv, info = c.solve_forcing(to_dev(fu(*X.T, lam)), to_dev(bc),
                                   opts=pkg.default_opts(rtol=1e-14))
    nf = o.layout.n_free
    ref = u(*T[:nf].T)
    assert np.abs(to_host(tr)[:nf] - ref).max() < 1e-10 * np.abs(ref).max(), info
    assert np.abs(to_host(uv) - u(*X.T)).max() < 1e-10 * np.abs(u(*X.T)).max()


def test_adjoint_exact_mass():
    import paper_2007_11891_amd as pkg
    o, c = _pair((3, 2, 2), 4)
    X = o.volume_coords()
    f = W.f_sin3(*X.T, 1.0)
    ut = o.solve(f, np.zeros(o.layout.n_all))
    uv = o.reconstruct(f, ut)
    dJdu = W.target_with_noise(uv, 5) - uv
    dl_ref, df_ref = o.adjoint(f, ut, uv, dJdu)
    dl, df, info = c.adjoint(to_dev(f), to_dev(ut), to_dev(dJdu),
                             opts=pkg.default_opts(rtol=1e-14))
    assert rel_err(to_host(dl), dl_ref) < 1e-10, info
    assert rel_err(to_host(df), df_ref) < 1e-10, info


def test_exact_and_lumped_differ_and_converge_alike():
    """Control: the two mass matrices give different discrete solutions on
    smooth data, both close to the exact solution (spectral accuracy)."""
    import paper_2007_11891_amd as pkg
    n, p = (3, 3, 3), 6
    widths = [W.uniform_widths(3)] * 3
    out = []
    for em in (False, True):
        c = pkg.HdgContext(n, widths, p, 1.0, 1.0, exact_mass=em)
        vx, tx = c.coords()
        f = to_dev(W.f_sin3(*to_host(vx).T, 1.0))
        g = to_dev(W.u_sin3(*to_host(tx).T))
        tr = g.clone()
        tr[:c.sizes.n_free] = 0
        _, uv, _ = c.solve_forcing(f, tr, opts=pkg.default_opts(rtol=1e-13))
        out.append((to_host(uv), W.u_sin3(*to_host(vx).T)))
    (ul, ue), (um, _) = out
    assert np.abs(ul - um).max() > 1e-8
    assert np.abs(ul - ue).max() < 1e-3 and np.abs(um - ue).max() < 1e-3


@pytest.mark.parametrize("p", [10, 12])
def test_exact_mass_with_neumann_at_high_degree(p):
    """Exact mass and four Neumann sides at p = 10 and 12 on a 2 x 2 x 2 mesh
    (p = 16 is in the operator test above):
    the operator and the right-hand side (nodal basis: the eigen basis of
    each side carries its own rounding of S at this degree) and the whole
    solution process against the oracle."""
    import paper_2007_11891_amd as pkg
    mask = 0b110011
    o, c = _pair((2, 2, 2), p, mask)
    L = o.layout
    nf = L.n_free
    Kff = o.assemble_K()[:nf, :nf].toarray()
    x = W.random_trace(nf, 21)
    assert rel_err(to_host(c.apply(to_dev(x), basis="nodal")), Kff @ x) < 1e-12
    X = o.volume_coords()
    f = W.f_sin3(*X.T, 1.0)
    bc = bc_vector(L, W.u_sin3, W.grad_sin3, o.trace_coords(), o.trace_normals())
    F = o.lifted_rhs(f, bc)
    assert rel_err(to_host(c.rhs(to_dev(f), to_dev(bc), basis="nodal")), F) < 1e-12
    ut = np.linalg.solve(Kff, F)
    tr, uv, info = c.solve_forcing(to_dev(f), to_dev(bc),
                                   opts=pkg.default_opts(rtol=1e-15, maxit=5000, check_every=9),
                                   allow_noconv=True)
    assert rel_err(to_host(tr)[:nf], ut) < 1e-11, info
