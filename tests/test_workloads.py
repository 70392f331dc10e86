"""Pins of the synthetic input generators (CPU only).

The paper's test case (section "Definition of a test case for assessment")
needs f = lambda u - laplace u of its five-factor manufactured solution; the
analytic Laplacian is checked against central differences of u itself, and
the generator's geometry against the case's definition.
"""
import math

import numpy as np

import workloads as W


def test_paper_forcing_matches_finite_differences():
    rng = np.random.default_rng(12)
    pts = rng.uniform(0.0, 2 * math.pi, size=(200, 3))

    def fd_lap(h):
        lap = np.zeros(len(pts))
        for a in range(3):
            e = np.zeros(3)
            e[a] = h
            lap += (W.u_paper(*(pts + e).T) - 2 * W.u_paper(*pts.T)
                    + W.u_paper(*(pts - e).T)) / (h * h)
        return lap

    # Richardson extrapolation of the second-order central difference
    lap = (4.0 * fd_lap(1e-3) - fd_lap(2e-3)) / 3.0
    for lam in (0.0, 2.5):
        f = W.f_paper(*pts.T, lam)
        ref = lam * W.u_paper(*pts.T) - lap
        assert np.max(np.abs(f - ref)) <= 1e-6 * np.max(np.abs(ref))


def test_paper_forcing_negative_control():
    """Dropping the cross terms of the product rule must fail the check above."""
    rng = np.random.default_rng(13)
    pts = rng.uniform(0.0, 2 * math.pi, size=(50, 3))
    u = W.u_paper(*pts.T)
    k = 5.0
    only_diag = k * k * sum(float(np.dot(a, a)) for a, _, _ in W._PAPER_FACTORS) * u
    assert np.max(np.abs(W.f_paper(*pts.T, 0.0) - only_diag)) > 1.0


def test_paper_case_geometry():
    pr = W.paper_case(p=6)
    assert pr.n == (8, 8, 8)
    for w in pr.widths:
        assert np.allclose(w.sum(), 2 * math.pi)
    h = 2 * math.pi / 8
    assert math.isclose(2 * pr.tau / h, 25.0)           # tau_e = 2 tau_hat / h
    assert np.all(pr.lam == 0.0)
    assert not pr.dirichlet_zero
