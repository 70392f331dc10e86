"""Pins of the CPU oracle against facts fixed by mathematics and the paper.

Each test checks the oracle against something other than itself: closed forms,
exactness of the discretisation, invariants of the condensed operator, the
paper's own factorisation identities, or finite differences.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W
from oracle.basis import gll_nodes_weights, standard_matrices
from oracle.element import element_operator, ElementSystem, kron3
from oracle.fastdiag import eigen_1d, factorized_element_operator, face_transform, b_s
from oracle.layout import Layout

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _parse(s):
    return float(eval(s, {"sqrt": math.sqrt}))


@pytest.mark.parametrize("p", [2, 3, 4])
def test_gll_closed_forms(p):
    """GLL points and weights against the tabulated closed forms."""
    with open(os.path.join(GOLDEN, "gll_closed_forms.json")) as fh:
        g = json.load(fh)[f"p{p}"]
    x, w = gll_nodes_weights(p)
    np.testing.assert_allclose(x, [_parse(s) for s in g["nodes"]], atol=1e-15)
    np.testing.assert_allclose(w, [_parse(s) for s in g["weights"]], rtol=1e-14)


@pytest.mark.parametrize("p", range(1, 17))
def test_gll_quadrature_exactness(p):
    """GLL integrates x^k exactly for k <= 2p-1 and not for k = 2p."""
    x, w = gll_nodes_weights(p)
    assert abs(w.sum() - 2.0) < 1e-13
    for k in range(0, 2 * p):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(w @ x ** k - exact) < 1e-13
    # P_p^2 has degree 2p: GLL gives 2/p instead of the exact 2/(2p+1)
    Pp = np.polynomial.legendre.legval(x, [0.0] * p + [1.0])
    assert abs(w @ Pp ** 2 - 2.0 / p) < 1e-12


@pytest.mark.parametrize("p", [1, 2, 5, 9, 16])
def test_1d_matrices_structure(p):
    """D 1 = 0, summation by parts D + D^T = diag(-1,0..0,1), and the end-point
    forms of E, G, B, C for GLL Lagrange polynomials."""
    tau = 1.7
    s = standard_matrices(p, tau)
    n = p + 1
    D = s["D"]
    assert np.abs(D @ np.ones(n)).max() < 1e-12
    sbp = np.zeros((n, n))
    sbp[0, 0], sbp[-1, -1] = -1.0, 1.0
    assert np.abs(D + D.T - sbp).max() < 1e-12
    e0, ep = np.eye(n)[0], np.eye(n)[-1]
    assert np.abs(s["E"] - tau * (np.outer(e0, e0) + np.outer(ep, ep))).max() < 1e-13
    assert np.abs(s["G"] - tau * np.eye(2)).max() == 0
    assert np.abs(s["B"] + tau * np.stack([e0, ep], 1)).max() < 1e-13
    assert np.abs(s["C"] - np.stack([-e0, ep], 1)).max() < 1e-13
    # D_ij = int phi_i phi_j' is exact for the derivative of a polynomial:
    # sum_j D_ij x_j^k = int phi_i k x^(k-1) for k <= p
    x, w = s["x"], s["w"]
    for k in range(1, p + 1):
        lhs = D @ x ** k
        rhs = w * k * x ** (k - 1)       # GLL quadrature is exact here (deg <= 2p-1)
        assert np.abs(lhs - rhs).max() < 1e-12


@pytest.mark.parametrize("p", [1, 2, 4, 8])
def test_eigendecomposition_invariants(p):
    s = standard_matrices(p, 1.0)
    S, lam = eigen_1d(s)
    n = p + 1
    assert np.abs(S.T @ s["M"] @ S - np.eye(n)).max() < 1e-13
    assert np.abs(S.T @ s["L"] @ S - np.diag(lam)).max() < 1e-12 * np.abs(s["L"]).max()
    assert lam.min() > 0


H_PERT = (0.31, 0.52, 0.77)


@pytest.mark.parametrize("p", [1, 2, 3, 5])
@pytest.mark.parametrize("exact_mass", [False, True])
def test_element_operator_matches_paper_factorisation(p, exact_mass):
    """Schur complement (equation hdg_operator) == factorised form (equation
    hdg_operator_factorized) built from the generalized eigendecomposition."""
    s = standard_matrices(p, 1.3, exact_mass=exact_mass)
    K = element_operator(s, H_PERT, 2.5)
    Kf, _ = factorized_element_operator(s, H_PERT, 2.5)
    assert np.abs(K - Kf).max() <= 1e-13 * np.abs(K).max()


@pytest.mark.parametrize("p", [1, 2, 4])
def test_element_operator_symmetric_positive(p):
    s = standard_matrices(p, 1.0)
    K = element_operator(s, H_PERT, 1.7)
    assert np.abs(K - K.T).max() < 1e-13 * np.abs(K).max()
    assert np.linalg.eigvalsh(K).min() > 0
    # lambda = 0: constant traces are in the null space (u = const, q = 0)
    K0 = element_operator(s, H_PERT, 0.0)
    assert np.abs(K0 @ np.ones(K0.shape[0])).max() < 1e-12 * np.abs(K0).max()
    assert np.linalg.eigvalsh(K0).min() > -1e-12 * np.abs(K0).max()


@pytest.mark.parametrize("p", [2, 3])
def test_element_operator_scaling_law(p):
    """Scaling x -> s x maps lambda -> lambda s^2 and the element operator by s:
    K(s h, lambda) = s K(h, lambda s^2) (tau_e scales like 1/h)."""
    s = standard_matrices(p, 1.0)
    sc = 1.9
    K1 = element_operator(s, tuple(sc * v for v in H_PERT), 2.0)
    K2 = element_operator(s, H_PERT, 2.0 * sc * sc)
    assert np.abs(K1 - sc * K2).max() < 1e-12 * np.abs(K1).max()


@pytest.mark.parametrize("p", [2, 4])
def test_transformed_same_direction_block_is_diagonal(p):
    """In the face eigenbasis the face-to-opposite-face block of each direction
    is diagonal in the two tangential indices (section on preconditioners),
    and its entries have the closed form of the factorised operator,

        K^[(s,t),(s',t)] = d_a H[s,s'] - d_a^2 sum_k B_S[k,s] B_S[k,s'] / D_Z[k,t],

    D_Z[k,t] = lambda d0 + d_a Lambda_k + d_b Lambda_tb + d_c Lambda_tc
    (k the normal index, (tb, tc) the tangential pair).  The operator here is
    the dense Schur complement of the element system, so a wrong sign, a
    dropped face term or a transposed B_S in the closed form fails."""
    s = standard_matrices(p, 1.0)
    lam = 1.0
    K = element_operator(s, H_PERT, lam)
    S, Lam = eigen_1d(s)
    BS = b_s(s, S)
    Hm = s["G"] + s["C"].T @ np.linalg.inv(s["M"]) @ s["C"]
    h1, h2, h3 = H_PERT
    d0 = h1 * h2 * h3 / 8.0
    d = [d0 * (2.0 / h1) ** 2, d0 * (2.0 / h2) ** 2, d0 * (2.0 / h3) ** 2]
    T = face_transform(S, p + 1)
    Kh = T.T @ K @ T
    n = p + 1
    nf = 2 * n * n
    for a in range(3):
        blk = Kh[a * nf:(a + 1) * nf, a * nf:(a + 1) * nf]
        # local face index -> (side, tangential pair (tb, tc), lower axis first)
        idx = np.arange(nf)
        if a == 0:
            side, tb, tc = idx % 2, (idx // 2) % n, idx // (2 * n)
        elif a == 1:
            side, tb, tc = (idx // n) % 2, idx % n, idx // (2 * n)
        else:
            side, tb, tc = idx // (n * n), idx % n, (idx // n) % n
        t = tb + n * tc
        mask = t[:, None] != t[None, :]
        assert np.abs(blk[mask]).max() < 1e-12 * np.abs(blk).max()
        b, c = [ax for ax in range(3) if ax != a]
        for i in range(nf):
            for j in range(nf):
                if t[i] != t[j]:
                    continue
                dz = lam * d0 + d[a] * Lam + d[b] * Lam[tb[i]] + d[c] * Lam[tc[i]]
                ref = (d[a] * Hm[side[i], side[j]]
                       - d[a] ** 2 * np.sum(BS[:, side[i]] * BS[:, side[j]] / dz))
                assert abs(blk[i, j] - ref) < 1e-12 * np.abs(blk).max()


def test_layout_counts_and_coverage():
    L = Layout((3, 2, 4), 2)
    npf = 9
    assert L.n_free == npf * (2 * 2 * 4 + 3 * 1 * 4 + 3 * 2 * 3)
    assert L.n_all == L.n_free + npf * 2 * (2 * 4 + 3 * 4 + 3 * 2)
    count = np.zeros(L.n_all, dtype=int)
    for e in range(L.n_elem):
        count[L.element_trace_map(e)] += 1
    assert (count[: L.n_free] == 2).all()
    assert (count[L.n_free:] == 1).all()


def test_layout_face_nodes_coincide_with_element_boundary_nodes():
    """Element-local face DOF coordinates (taken from the element's own
    boundary volume nodes) equal the global trace coordinates."""
    n, p = (3, 2, 2), 2
    widths = [np.array([0.2, 0.5, 0.3]), np.array([0.4, 0.6]), np.array([0.7, 0.3])]
    o = oracle.HdgOracle(n, widths, p, 1.0, 1.0)
    X = o.volume_coords()
    T = o.trace_coords()
    npn = p + 1
    for e in range(o.layout.n_elem):
        xe = X[o.vol_slice(e)].reshape(npn, npn, npn, 3)   # [q3, q2, q1]
        m = o.layout.element_trace_map(e)
        loc = np.empty((6 * npn * npn, 3))
        for s in (0, 1):
            q = 0 if s == 0 else npn - 1
            for q3 in range(npn):
                for q2 in range(npn):
                    loc[s + 2 * (q2 + npn * q3)] = xe[q3, q2, q]
            for q3 in range(npn):
                for q1 in range(npn):
                    loc[2 * npn * npn + q1 + npn * (s + 2 * q3)] = xe[q3, q, q1]
            for q2 in range(npn):
                for q1 in range(npn):
                    loc[4 * npn * npn + q1 + npn * (q2 + npn * s)] = xe[q, q2, q1]
        assert np.abs(loc - T[m]).max() < 1e-14


def _poly_problem(p, exact_mass=False, lam=1.7, seed=0):
    rng = np.random.default_rng(seed)
    c = rng.standard_normal((p + 1,) * 3)
    u, f = W.poly_tensor(c)
    widths = [np.array([0.3, 0.5, 0.2]), np.array([0.6, 0.4]), np.array([0.45, 0.55])]
    o = oracle.HdgOracle((3, 2, 2), widths, p, 1.0, lam, exact_mass=exact_mass)
    X = o.volume_coords()
    T = o.trace_coords()
    return o, u(*X.T), f(*X.T, lam), u(*T.T)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_polynomial_reproduction(p):
    """A tensor polynomial of degree <= p per axis is reproduced to round-off,
    on the trace and in the element interiors, on a perturbed mesh."""
    o, uv, fv, g = _poly_problem(p)
    ut = o.solve(fv, g)
    assert np.abs(ut - g).max() < 1e-12 * np.abs(g).max()
    ur = o.reconstruct(fv, ut)
    assert np.abs(ur - uv).max() < 1e-12 * np.abs(uv).max()


def test_polynomial_degree_p_plus_1_is_not_reproduced():
    """Control for the previous test: degree p+1 data is not reproduced."""
    p = 2
    rng = np.random.default_rng(3)
    c = np.zeros((p + 2,) * 3)
    c[p + 1, 1, 0] = 1.0
    c[0, 0, 0] = rng.standard_normal()
    u, f = W.poly_tensor(c)
    widths = [np.array([0.3, 0.5, 0.2]), np.array([0.6, 0.4]), np.array([0.45, 0.55])]
    o = oracle.HdgOracle((3, 2, 2), widths, p, 1.0, 1.0)
    X, T = o.volume_coords(), o.trace_coords()
    ut = o.solve(f(*X.T, 1.0), u(*T.T))
    assert np.abs(ut - u(*T.T)).max() > 1e-6


def test_convergence_order_p2():
    """O(h^(p+1)) convergence of the reconstructed u for p = 2 (n = 4 -> 8)."""
    errs = []
    for n in (4, 8):
        o = oracle.HdgOracle((n, n, n), [W.uniform_widths(n)] * 3, 2, 1.0, 1.0)
        X, T = o.volume_coords(), o.trace_coords()
        fv = W.f_sin3(*X.T, 1.0)
        ut = o.solve(fv, W.u_sin3(*T.T))
        uv = o.reconstruct(fv, ut)
        errs.append(np.abs(uv - W.u_sin3(*X.T)).max())
    rate = math.log2(errs[0] / errs[1])
    assert 2.8 < rate < 3.3, rate


def test_convergence_order_p3():
    errs = []
    for n in (2, 4):
        o = oracle.HdgOracle((n, n, n), [W.uniform_widths(n)] * 3, 3, 1.0, 1.0)
        X, T = o.volume_coords(), o.trace_coords()
        fv = W.f_sin3(*X.T, 1.0)
        ut = o.solve(fv, W.u_sin3(*T.T))
        uv = o.reconstruct(fv, ut)
        errs.append(np.abs(uv - W.u_sin3(*X.T)).max())
    rate = math.log2(errs[0] / errs[1])
    assert 3.7 < rate < 4.4, rate


def test_global_operator_spd_tiny():
    prob = W.tiny()
    o = oracle.HdgOracle(prob.n, prob.widths, prob.p, prob.tau, prob.lam)
    K = o.assemble_K().toarray()
    nf = o.layout.n_free
    Kff = K[:nf, :nf]
    assert np.abs(Kff - Kff.T).max() < 1e-13 * np.abs(Kff).max()
    np.linalg.cholesky(Kff)
    # matrix-free element apply == assembled matrix
    x = W.random_trace(nf, 1)
    assert np.abs(o.apply_free(x) - Kff @ x).max() < 1e-13 * np.abs(Kff @ x).max()


def test_adjoint_matches_central_differences():
    """Oracle gradients dJ/dlambda_e and dJ/df against central differences of
    J = 1/2 ||u - u*||_M^2 computed by re-solving."""
    n, p = (2, 2, 2), 2
    rng = np.random.default_rng(11)
    lam = np.exp(rng.standard_normal(8))
    widths = [W.uniform_widths(2)] * 3
    o = oracle.HdgOracle(n, widths, p, 1.0, lam)
    X, T = o.volume_coords(), o.trace_coords()
    f = rng.standard_normal(o.layout.n_vol)
    g = np.zeros(o.layout.n_all)
    ustar = rng.standard_normal(o.layout.n_vol) * 0.1
    ut = o.solve(f, g)
    uv = o.reconstruct(f, ut)
    Md = o.mass_diag()
    dlam, df = o.adjoint(f, ut, uv, Md * (uv - ustar))

    def J(lam_, f_):
        oo = oracle.HdgOracle(n, widths, p, 1.0, lam_)
        tt = oo.solve(f_, g)
        return oo.loss(oo.reconstruct(f_, tt), ustar)

    for seed in range(3):
        r = np.random.default_rng(100 + seed)
        vl, vf = r.standard_normal(8), r.standard_normal(o.layout.n_vol)
        eps = 1e-5
        fd = (J(lam + eps * vl, f + eps * vf) - J(lam - eps * vl, f - eps * vf)) / (2 * eps)
        an = dlam @ vl + df @ vf
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (fd, an)


@pytest.mark.parametrize("neumann", [0, 0b100110])
def test_apply_rows_and_faces_elements(neumann):
    """The sampled-row operator of the oracle (used as the expected value of
    full-size GPU checks) equals rows of the assembled K = sum_e Q_e^T K_e Q_e
    (equation (hdg_system)), and the elements it sums are exactly the
    elements whose closed box contains the face (one on a side of the box,
    two inside), found from coordinates."""
    n, p = (3, 2, 4), 2
    widths = [np.array([0.2, 0.5, 0.3]), np.array([0.45, 0.55]), np.array([0.1, 0.2, 0.3, 0.4])]
    o = oracle.HdgOracle(n, widths, p, 1.0, 1.3, neumann=neumann)
    L = o.layout
    rng = np.random.default_rng(3)
    x = rng.uniform(-1, 1, L.n_all)
    y_full = o.assemble_K() @ x
    assert np.abs(o.apply(x) - y_full).max() < 1e-13 * np.abs(y_full).max()
    npf = (p + 1) ** 2
    faces = rng.choice(L.n_faces, size=12, replace=False)
    rows = np.concatenate([f * npf + rng.choice(npf, size=3, replace=False) for f in faces])
    rows = np.concatenate([rows, [0, L.n_free - 1, L.n_all - 1]])
    got = o.apply_rows(x, rows)
    assert np.abs(got - y_full[rows]).max() < 1e-13 * np.abs(y_full).max()
    # the same rows of the assembled right-hand side
    f = rng.uniform(-1, 1, L.n_vol)
    F_full = o.assemble_F(f)
    assert np.abs(o.rhs_rows(f, rows) - F_full[rows]).max() < 1e-13 * np.abs(F_full).max()
    # elements of each face from geometry: the face's nodes lie on the
    # element's closed box
    T = o.trace_coords()
    edges = [np.concatenate([[0.0], np.cumsum(w)]) for w in widths]
    for f in faces:
        pts = T[f * npf:(f + 1) * npf]
        want = []
        for e in range(L.n_elem):
            ijk = L.elem_ijk(e)
            lo = np.array([edges[a][ijk[a]] for a in range(3)])
            hi = np.array([edges[a][ijk[a] + 1] for a in range(3)])
            if ((pts >= lo - 1e-12) & (pts <= hi + 1e-12)).all():
                want.append(e)
        assert o.faces_elements([f]) == want
        on_side = any(np.allclose(pts[:, a], v) for a in range(3) for v in (0.0, edges[a][-1]))
        assert len(want) == (1 if on_side else 2)
