"""Pins of the oracle's Neumann boundaries and initial-guess hybridization
(no GPU).

* layout: Neumann faces are free unknowns with one element each, the g_N
  block mirrors them, and no Neumann side gives the Dirichlet layout;
* a tensor polynomial of degree <= p per axis is reproduced to round-off
  with n . grad u = g_N on any set of Neumann sides (equation
  (neumann_flux)); the same data with the wrong sign, or a missing face
  measure, is not;
* with smooth data the Neumann problem converges spectrally in p like the
  Dirichlet one;
* the flux of equation (fluxu) with q = grad u: a continuous polynomial
  keeps its trace, a piecewise constant field gives the tau-weighted mean
  (tau = 2 tau_hat / h), and a Neumann face moves by (g_N - q.n) / tau;
* CG started from the hybridized guess of a nearby solution needs fewer
  iterations than from zero and reaches the same solution.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from helpers import bc_vector
from oracle.pcg import pcg

WIDTHS = [np.array([0.3, 0.5, 0.2]), np.array([0.6, 0.4]), np.array([0.45, 0.55])]
MASKS = [0b000001, 0b000010, 0b101010, 0b111110, 0b010101]


def test_layout_with_neumann_sides():
    for mask in [0] + MASKS + [63]:
        L = oracle.Layout((3, 2, 2), 2, mask)
        npf = L.np_ ** 2
        counts = np.zeros(L.n_faces, dtype=int)
        for e in range(L.n_elem):
            for f in np.unique(L.element_trace_map(e) // npf):
                counts[f] += 1
        side_total = sum(n for (a, s), n in L.side_faces.items() if (mask >> (2 * a + s)) & 1)
        assert L.n_neu_faces == side_total
        assert np.all(counts[: L.n_int_faces] == 2)
        assert np.all(counts[L.n_int_faces:] == 1)
        assert L.n_all == (L.n_faces + L.n_neu_faces) * npf
        for f in range(L.n_int_faces, L.n_free_faces):
            a, s = L.face_side(f)
            assert (mask >> (2 * a + s)) & 1
        for f in range(L.n_free_faces, L.n_faces):
            a, s = L.face_side(f)
            assert not (mask >> (2 * a + s)) & 1
    # no Neumann side: the plain Dirichlet layout
    L0 = oracle.Layout((3, 2, 2), 2)
    assert L0.n_free_faces == L0.n_int_faces and L0.n_all == L0.n_faces * L0.np_ ** 2


def test_neumann_data_block_mirrors_faces():
    o = oracle.HdgOracle((3, 2, 2), WIDTHS, 2, 1.0, 1.0, neumann=0b100110)
    L = o.layout
    npf = L.np_ ** 2
    T, nrm = o.trace_coords(), o.trace_normals()
    assert not np.isnan(T).any()
    for f in range(L.n_int_faces, L.n_free_faces):
        d = L.neumann_data_index(f)
        a, s = L.face_side(f)
        assert np.array_equal(T[d:d + npf], T[f * npf:(f + 1) * npf])
        assert np.all(nrm[d:d + npf, a] == 2 * s - 1)
        ext = np.cumsum(WIDTHS[a])[-1] if s else 0.0
        assert np.allclose(T[f * npf:(f + 1) * npf, a], ext)


def _poly(p, seed):
    rng = np.random.default_rng(seed)
    c = rng.standard_normal((p + 1,) * 3)
    u, f = W.poly_tensor(c)
    return u, f, W.poly_tensor_grad(c)


@pytest.mark.parametrize("mask", MASKS + [63])
@pytest.mark.parametrize("p", [1, 2, 3])
def test_polynomial_reproduction_with_neumann(mask, p):
    lam = 1.3
    u, f, g = _poly(p, 10 + p + mask)
    o = oracle.HdgOracle((3, 2, 2), WIDTHS, p, 1.0, lam, neumann=mask)
    X, T = o.volume_coords(), o.trace_coords()
    bc = bc_vector(o.layout, u, g, T, o.trace_normals())
    ut = o.solve(f(*X.T, lam), bc)
    nf = o.layout.n_free
    ref = u(*T[:nf].T)
    assert np.abs(ut[:nf] - ref).max() < 1e-11 * np.abs(ref).max()
    uv = o.reconstruct(f(*X.T, lam), ut)
    assert np.abs(uv - u(*X.T)).max() < 1e-11 * np.abs(u(*X.T)).max()


def test_polynomial_reproduction_pure_neumann_poisson_up_to_constant():
    """All sides Neumann, lambda = 0: K_ff is singular with the constants as
    kernel; the data is compatible, so a least-squares solution equals u up
    to a constant."""
    p = 2
    u, f, g = _poly(p, 4)
    o = oracle.HdgOracle((2, 2, 2), [np.array([0.4, 0.6])] * 3, p, 1.0, 0.0, neumann=63)
    X, T = o.volume_coords(), o.trace_coords()
    bc = bc_vector(o.layout, u, g, T, o.trace_normals())
    nf = o.layout.n_free
    K = o.assemble_K()[:nf, :nf].toarray()
    rhs = o.lifted_rhs(f(*X.T, 0.0), bc)
    assert abs(np.ones(nf) @ rhs) < 1e-10 * np.abs(rhs).sum()       # compatible data
    assert np.abs(K @ np.ones(nf)).max() < 1e-10 * np.abs(K).max()   # constants in the kernel
    x = np.linalg.lstsq(K, rhs, rcond=None)[0]
    d = x - u(*T[:nf].T)
    assert np.abs(d - d.mean()).max() < 1e-9


@pytest.mark.parametrize("flip", ["sign", "measure"])
def test_wrong_neumann_data_is_not_reproduced(flip):
    """Controls: the reproduction test fails for g_N of the wrong sign or
    with the face measure dropped (data scaled by 4 / (h_b h_c))."""
    p, lam, mask = 2, 1.3, 0b000011
    u, f, g = _poly(p, 7)
    o = oracle.HdgOracle((3, 2, 2), WIDTHS, p, 1.0, lam, neumann=mask)
    X, T = o.volume_coords(), o.trace_coords()
    bc = bc_vector(o.layout, u, g, T, o.trace_normals())
    L = o.layout
    gn = slice(L.n_faces * L.np_ ** 2, L.n_all)
    if flip == "sign":
        bc[gn] = -bc[gn]
    else:
        bc[gn] = bc[gn] * 4.0 / (0.6 * 0.45)
    ut = o.solve(f(*X.T, lam), bc)
    nf = L.n_free
    assert np.abs(ut[:nf] - u(*T[:nf].T)).max() > 1e-4


def test_neumann_spectral_convergence():
    errs = []
    for p in (3, 5, 7):
        o = oracle.HdgOracle((2, 2, 2), [W.uniform_widths(2)] * 3, p, 1.0, 1.0, neumann=0b011001)
        X, T = o.volume_coords(), o.trace_coords()
        bc = bc_vector(o.layout, W.u_sin3, W.grad_sin3, T, o.trace_normals())
        fv = W.f_sin3(*X.T, 1.0)
        uv = o.reconstruct(fv, o.solve(fv, bc))
        errs.append(np.abs(uv - W.u_sin3(*X.T)).max())
    assert errs[0] < 5e-2 and errs[1] < errs[0] / 10 and errs[2] < errs[1] / 10, errs


def test_hybridize_keeps_continuous_polynomial():
    p = 3
    u, f, g = _poly(p, 21)
    o = oracle.HdgOracle((3, 2, 2), WIDTHS, p, 2.0, 1.0, neumann=0b100101)
    X, T = o.volume_coords(), o.trace_coords()
    bc = bc_vector(o.layout, u, g, T, o.trace_normals())
    ut = o.hybridize(u(*X.T), bc)
    nf = o.layout.n_free
    ref = u(*T[:nf].T)
    assert np.abs(ut - ref).max() < 1e-11 * np.abs(ref).max()


def test_hybridize_piecewise_constant_is_tau_weighted_mean():
    """u = c_e on each element: q = 0, interior faces get the mean weighted
    with tau = 2 tau_hat / h, Neumann faces c_e + g_N / tau."""
    p, tau = 2, 3.0
    mask = 0b000001                       # x1 = 0 is Neumann
    o = oracle.HdgOracle((3, 2, 2), WIDTHS, p, tau, 1.0, neumann=mask)
    L = o.layout
    npn, npf = L.np_, L.np_ ** 2
    ce = np.random.default_rng(5).standard_normal(L.n_elem)
    uv = np.repeat(ce, npn ** 3)
    bc = np.zeros(L.n_all)
    bc[L.n_faces * npf:] = 0.7
    ut = o.hybridize(uv, bc)
    for e in range(L.n_elem):
        i, j, k = L.elem_ijk(e)
        if i + 1 < 3:                               # face to the x1 neighbour
            fid = L.face_id(0, i + 1, (i, j, k))
            e2 = L.elem_index(i + 1, j, k)
            t1, t2 = 2 * tau / WIDTHS[0][i], 2 * tau / WIDTHS[0][i + 1]
            want = (t1 * ce[e] + t2 * ce[e2]) / (t1 + t2)
            assert np.allclose(ut[fid * npf:(fid + 1) * npf], want, rtol=1e-14, atol=1e-14)
        if i == 0:
            fid = L.face_id(0, 0, (i, j, k))
            want = ce[e] + 0.7 / (2 * tau / WIDTHS[0][0])
            assert np.allclose(ut[fid * npf:(fid + 1) * npf], want, rtol=1e-14, atol=1e-14)


def test_hybridize_neumann_face_shift():
    """u = x1 on a mesh whose side x1 = 0 is Neumann with g_N = 0.25: there
    q.n = -1, so u~ = 0 - (-1 - 0.25) / tau."""
    p, tau = 3, 1.5
    o = oracle.HdgOracle((3, 2, 2), WIDTHS, p, tau, 1.0, neumann=0b000001)
    L = o.layout
    npf = L.np_ ** 2
    X = o.volume_coords()
    bc = np.zeros(L.n_all)
    bc[L.n_faces * npf:] = 0.25
    ut = o.hybridize(X[:, 0].copy(), bc)
    for f in range(L.n_int_faces, L.n_free_faces):
        want = (1.0 + 0.25) / (2 * tau / WIDTHS[0][0])
        assert np.allclose(ut[f * npf:(f + 1) * npf], want, rtol=1e-13)


def test_cg_from_hybridized_guess():
    """The solution of a nearby problem (lambda 10 % off), hybridized, starts
    CG closer: fewer iterations, same solution."""
    p, mask = 3, 0b000110
    o = oracle.HdgOracle((3, 3, 2), [W.uniform_widths(3), W.uniform_widths(3), W.uniform_widths(2)],
                         p, 1.0, 2.0, neumann=mask)
    o2 = oracle.HdgOracle((3, 3, 2), [W.uniform_widths(3), W.uniform_widths(3), W.uniform_widths(2)],
                          p, 1.0, 2.2, neumann=mask)
    X, T = o.volume_coords(), o.trace_coords()
    bc = bc_vector(o.layout, W.u_sin3, W.grad_sin3, T, o.trace_normals())
    fv = W.f_sin3(*X.T, 2.0)
    u2 = o2.reconstruct(fv, o2.solve(fv, bc))
    nf = o.layout.n_free
    K = o.assemble_K()[:nf, :nf].toarray()
    F = o.lifted_rhs(fv, bc)
    x_ref = np.linalg.solve(K, F)
    x0 = o.hybridize(u2, bc)
    x_a, it0, _ = pcg(K, F, None, rtol=1e-10)
    x_b, it1, _ = pcg(K, F, None, rtol=1e-10, x0=x0)
    assert it1 < it0
    for x in (x_a, x_b):
        assert np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref) < 1e-8
