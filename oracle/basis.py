"""One-dimensional basis and standard-element matrices (oracle, FP64).

TEST INFRASTRUCTURE ONLY: nothing in the product path may import this module.

Follows the paper's section "HDG operators in one dimension", equation
(element_matrices): Lagrange polynomials on the Gauss-Lobatto-Legendre (GLL)
points of degree p on [-1, 1] (the basis named in the section on operator
runtimes), the flux basis phi_1, phi_2 that is one on the left / right end,
and the matrices

    M_ij = int phi_i phi_j           D_ij = int phi_i d(phi_j)/dxi
    E_ij = +tau [phi_i phi_j](+-1)   G_ij = +tau [phit_i phit_j](+-1)
    B_ij = -tau [phi_i phit_j](+-1)  C_ij = [phi_i phit_j n](+-1)
    L    = E + D M^-1 D^T

where [.](+-1) sums the two end points and n = -1 on the left, +1 on the
right.  The mass matrix is the lumped GLL one, diag(w), unless ``exact_mass``
is requested (the paper allows both; the lumped one is the one for which the
face terms are diagonal).
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg


def gll_nodes_weights(p: int):
    """GLL nodes (ascending) and weights for degree p >= 1.

    Nodes: -1, +1 and the roots of P_p'.  Weights: 2 / (p (p+1) P_p(x_i)^2).
    The interior roots come from numpy's Legendre-series root finder and are
    polished by Newton steps on P_p'.
    """
    if p < 1:
        raise ValueError("p >= 1 required")
    cp = np.zeros(p + 1)
    cp[p] = 1.0                       # P_p as a Legendre series
    dcp = npleg.legder(cp)            # P_p'
    d2cp = npleg.legder(dcp)          # P_p''
    inner = np.sort(np.real(npleg.legroots(dcp))) if p >= 2 else np.zeros(0)
    for _ in range(3):
        inner = inner - npleg.legval(inner, dcp) / npleg.legval(inner, d2cp)
    x = np.concatenate(([-1.0], inner, [1.0]))
    w = 2.0 / (p * (p + 1) * npleg.legval(x, cp) ** 2)
    return x, w


def lagrange_eval(nodes: np.ndarray, xs: np.ndarray) -> np.ndarray:
    """V[k, j] = phi_j(xs[k]) by the product formula."""
    nodes = np.asarray(nodes, dtype=np.float64)
    xs = np.atleast_1d(np.asarray(xs, dtype=np.float64))
    n = nodes.size
    V = np.ones((xs.size, n))
    for j in range(n):
        for m in range(n):
            if m != j:
                V[:, j] *= (xs - nodes[m]) / (nodes[j] - nodes[m])
    return V


def lagrange_deriv_eval(nodes: np.ndarray, xs: np.ndarray) -> np.ndarray:
    """W[k, j] = phi_j'(xs[k]) by differentiating the product formula."""
    nodes = np.asarray(nodes, dtype=np.float64)
    xs = np.atleast_1d(np.asarray(xs, dtype=np.float64))
    n = nodes.size
    W = np.zeros((xs.size, n))
    for j in range(n):
        for l in range(n):
            if l == j:
                continue
            term = np.full(xs.size, 1.0 / (nodes[j] - nodes[l]))
            for m in range(n):
                if m != j and m != l:
                    term *= (xs - nodes[m]) / (nodes[j] - nodes[m])
            W[:, j] += term
    return W


def standard_matrices(p: int, tau: float, exact_mass: bool = False) -> dict:
    """Standard-element matrices of equation (element_matrices).

    Integrals of polynomial products are taken with Gauss-Legendre quadrature
    of p+2 points (exact to degree 2p+3).
    """
    x, w = gll_nodes_weights(p)
    gx, gw = npleg.leggauss(p + 2)
    Vg = lagrange_eval(x, gx)              # phi_j at Gauss points
    Wg = lagrange_deriv_eval(x, gx)        # phi_j' at Gauss points
    if exact_mass:
        M = Vg.T @ (gw[:, None] * Vg)
    else:
        M = np.diag(w)
    D = Vg.T @ (gw[:, None] * Wg)          # D_ij = int phi_i phi_j'
    ends = lagrange_eval(x, np.array([-1.0, 1.0]))   # ends[0] = phi(-1), ends[1] = phi(+1)
    phi_m, phi_p = ends[0], ends[1]
    E = tau * (np.outer(phi_m, phi_m) + np.outer(phi_p, phi_p))
    G = tau * np.eye(2)
    B = -tau * np.stack([phi_m, phi_p], axis=1)      # (p+1) x 2
    C = np.stack([-phi_m, phi_p], axis=1)            # normal -1 left, +1 right
    Minv = np.linalg.inv(M)
    L = E + D @ Minv @ D.T
    return {"x": x, "w": w, "M": M, "D": D, "E": E, "G": G, "B": B, "C": C, "L": L,
            "p": p, "tau": tau}
