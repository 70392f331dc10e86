"""Dense three-dimensional element system and its Schur complement (oracle).

TEST INFRASTRUCTURE ONLY: nothing in the product path may import this module.

Follows the paper's section "LDG operator structure in three dimensions":
the 7x7 block element system of equation (ldg_element_operator_threed), the
metric factors d_0..d_3 and the penalty tau_{i,e} = 2 tau / h_{i,e}, and the
tensor-product matrices of Table 1, built here as explicit Kronecker products
(np.kron(A3, np.kron(A2, A1)) acts with A1 on the fastest index, matching the
definition in equation (tp_definition)).  The condensed element operator is
the Schur complement of equation (hdg_operator),

    K_e = G_e - R_e^T A_e^-1 R_e,

formed with a dense LU solve.  The right-hand side and the recovery of u, q
follow from eliminating u, q from the same system (equation
(ldg_element_operator) and its 3D form):

    F_e = g_N,e - R_e^T A_e^-1 [M_e f_e; 0; 0; 0]
    [u; q1; q2; q3] = A_e^-1 ([M_e f_e; 0; 0; 0] - R_e u~_e)

(the reading of the signs is derived from the element system; the printed
solver listing has the opposite sign in both places).
"""
from __future__ import annotations

import numpy as np

from .basis import standard_matrices


def kron3(A3, A2, A1):
    return np.kron(A3, np.kron(A2, A1))


def metric_factors(h1, h2, h3):
    """(d0, d1, d2, d3) = h1 h2 h3 / 8 * (1, (2/h1)^2, (2/h2)^2, (2/h3)^2)."""
    d0 = h1 * h2 * h3 / 8.0
    return d0, d0 * (2.0 / h1) ** 2, d0 * (2.0 / h2) ** 2, d0 * (2.0 / h3) ** 2


class ElementSystem:
    """A_e, R_e, G_e and M_e of one Cartesian element."""

    def __init__(self, std: dict, h, lam: float):
        h1, h2, h3 = (float(v) for v in h)
        M, D, E, G, B, C = (std[k] for k in ("M", "D", "E", "G", "B", "C"))
        d0, d1, d2, d3 = metric_factors(h1, h2, h3)
        nv = M.shape[0] ** 3
        Me = d0 * kron3(M, M, M)
        D1 = (h1 / 2.0) * d1 * kron3(M, M, D)
        D2 = (h2 / 2.0) * d2 * kron3(M, D, M)
        D3 = (h3 / 2.0) * d3 * kron3(D, M, M)
        Ee = d1 * kron3(M, M, E) + d2 * kron3(M, E, M) + d3 * kron3(E, M, M)
        G1 = d1 * kron3(M, M, G)
        G2 = d2 * kron3(M, G, M)
        G3 = d3 * kron3(G, M, M)
        B1 = d1 * kron3(M, M, B)
        B2 = d2 * kron3(M, B, M)
        B3 = d3 * kron3(B, M, M)
        C1 = (h1 / 2.0) * d1 * kron3(M, M, C)
        C2 = (h2 / 2.0) * d2 * kron3(M, C, M)
        C3 = (h3 / 2.0) * d3 * kron3(C, M, M)
        Z = np.zeros((nv, nv))
        self.A = np.block([
            [lam * Me + Ee, -D1, -D2, -D3],
            [-D1.T, -Me, Z, Z],
            [-D2.T, Z, -Me, Z],
            [-D3.T, Z, Z, -Me],
        ])
        nf = G1.shape[0]
        Zf = np.zeros((nv, nf))
        self.R = np.block([
            [B1, B2, B3],
            [C1, Zf, Zf],
            [Zf, C2, Zf],
            [Zf, Zf, C3],
        ])
        Zg = np.zeros((nf, nf))
        self.G = np.block([[G1, Zg, Zg], [Zg, G2, Zg], [Zg, Zg, G3]])
        self.Me = Me
        self.nv = nv
        self.d = (d0, d1, d2, d3)
        self.lam = lam

    def volume_rhs(self, v):
        """[v; 0; 0; 0] for a volume vector v."""
        out = np.zeros(4 * self.nv)
        out[: self.nv] = v
        return out


def element_operator(std: dict, h, lam: float) -> np.ndarray:
    """K_e = G_e - R_e^T A_e^-1 R_e (equation (hdg_operator))."""
    es = ElementSystem(std, h, lam)
    return es.G - es.R.T @ np.linalg.solve(es.A, es.R)
