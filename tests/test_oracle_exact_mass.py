"""Pins of the oracle's exact (non-lumped) GLL mass matrix and of the
discretisation built on it (no GPU).

* M integrates the product of any two polynomials of degree <= p exactly
  (monomials against closed-form integrals); the lumped diag(w) does not
  when the degrees add up to 2p (control);
* row sums of M are the GLL weights, and M is not diagonal;
* a tensor polynomial of degree <= p is reproduced with exact mass too,
  with Dirichlet and with Neumann sides;
* in the eigen-face basis the faces of one axis still couple only at the
  same tangential index (S^T M S = I holds for the exact M as well), while
  H = G + C^T M^-1 C, the face term, is no longer diagonal (the paper's
  remark on dropping the lumping); the factorised operator with this H is
  pinned against the Schur complement in test_oracle_pins.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from helpers import bc_vector
from oracle.basis import standard_matrices
from oracle.fastdiag import eigen_1d


@pytest.mark.parametrize("p", [1, 2, 3, 5, 8, 12])
def test_exact_mass_integrates_polynomial_products(p):
    s = standard_matrices(p, 1.0, exact_mass=True)
    sl = standard_matrices(p, 1.0)
    x = s["x"]
    M, Ml = s["M"], sl["M"]
    for a in range(p + 1):
        for b in range(p + 1):
            want = 2.0 / (a + b + 1) if (a + b) % 2 == 0 else 0.0
            got = (x ** a) @ M @ (x ** b)
            assert abs(got - want) < 1e-13 * max(1.0, abs(want))
    # lumped: exact below degree 2p, wrong at 2p
    assert abs((x ** p) @ Ml @ (x ** p) - 2.0 / (2 * p + 1)) > 1e-8
    assert np.allclose(M.sum(axis=1), s["w"], rtol=0, atol=1e-14)
    assert np.abs(M - np.diag(np.diag(M))).max() > 1e-3


@pytest.mark.parametrize("mask", [0, 0b010011])
@pytest.mark.parametrize("p", [1, 2, 4])
def test_polynomial_reproduction_with_exact_mass(mask, p):
    lam = 0.9
    rng = np.random.default_rng(60 + p)
    c = rng.standard_normal((p + 1,) * 3)
    u, f = W.poly_tensor(c)
    g = W.poly_tensor_grad(c)
    widths = [np.array([0.3, 0.5, 0.2]), np.array([0.6, 0.4]), np.array([0.45, 0.55])]
    o = oracle.HdgOracle((3, 2, 2), widths, p, 1.0, lam, exact_mass=True, neumann=mask)
    X, T = o.volume_coords(), o.trace_coords()
    bc = bc_vector(o.layout, u, g, T, o.trace_normals())
    ut = o.solve(f(*X.T, lam), bc)
    nf = o.layout.n_free
    assert np.abs(ut[:nf] - u(*T[:nf].T)).max() < 1e-11 * np.abs(u(*T[:nf].T)).max()
    uv = o.reconstruct(f(*X.T, lam), ut)
    assert np.abs(uv - u(*X.T)).max() < 1e-11 * np.abs(u(*X.T)).max()


@pytest.mark.parametrize("p", [2, 4])
def test_transformed_faces_of_an_axis_couple_per_tangential_index(p):
    s = standard_matrices(p, 1.3, exact_mass=True)
    S, _ = eigen_1d(s)
    h = (0.7, 1.1, 0.5)
    K = oracle.element_operator(s, h, 0.8)
    npn = p + 1
    npf = npn * npn
    # element-local face order u1 (side, q2, q3), u2 (q1, side, q3), u3 (q1, q2, side)
    Q = np.zeros((6 * npf, 6 * npf))
    SS = np.kron(S, S)
    Q[0:2 * npf, 0:2 * npf] = np.kron(SS, np.eye(2))
    blk = np.kron(S, np.kron(np.eye(2), S))
    Q[2 * npf:4 * npf, 2 * npf:4 * npf] = blk
    Q[4 * npf:, 4 * npf:] = np.kron(np.eye(2), SS)
    Kh = Q.T @ K @ Q
    Minv = np.linalg.inv(s["M"])
    C = s["C"]
    H = s["G"] + C.T @ Minv @ C
    assert abs(H[0, 1]) > 1e-3                     # not diagonal with exact mass
    # no coupling between different tangential indices within the axis-1 faces
    A1 = Kh[:2 * npf, :2 * npf].reshape(npf, 2, npf, 2)
    for t1 in range(npf):
        for t2 in range(npf):
            if t1 != t2:
                assert np.abs(A1[t1, :, t2, :]).max() < 1e-11 * np.abs(Kh).max()
