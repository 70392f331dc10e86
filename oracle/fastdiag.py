"""The paper's factorised element operator, written out densely (oracle).

TEST INFRASTRUCTURE ONLY: nothing in the product path may import this module.

Used only to pin the paper's factorisation claims against the Schur
complement of ``element``:

* generalized eigenproblem (generalized_eigenvalue_decomposition):
  S^T M S = I, S^T L S = Lambda, solved with scipy.linalg.eigh(L, M);
* B_S = S^T B - S^T D M^-1 C (equation (hdgbs));
* factorised operator (equation (hdg_operator_factorized)):
  K_e = blockdiag_i(d_i (M x M x (G + C^T M^-1 C))_i) - B_S,e^T D_Z^-1 B_S,e,
  with D_Z = lambda d0 + d1 Lambda_1 + d2 Lambda_2 + d3 Lambda_3 and
  B_S,e = [d1 S^TM x S^TM x B_S, d2 S^TM x B_S x S^TM, d3 B_S x S^TM x S^TM];
* the transformed operator K^ = T^T K T, T = S x S on every face (section
  "Product factorization of the HDG operator").
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .element import kron3, metric_factors


def eigen_1d(std: dict):
    lam, S = sla.eigh(std["L"], std["M"])
    return S, lam


def b_s(std: dict, S):
    Minv = np.linalg.inv(std["M"])
    return S.T @ std["B"] - S.T @ std["D"] @ Minv @ std["C"]


def factorized_element_operator(std: dict, h, lam: float):
    S, Lam = eigen_1d(std)
    BS = b_s(std, S)
    M, G, C = std["M"], std["G"], std["C"]
    H = G + C.T @ np.linalg.inv(M) @ C
    d0, d1, d2, d3 = metric_factors(*h)
    I = np.eye(M.shape[0])
    StM = S.T @ M
    one = np.ones(M.shape[0])
    DZ = (lam * d0 * kron3(one, one, one) + d1 * kron3(one, one, Lam)
          + d2 * kron3(one, Lam, one) + d3 * kron3(Lam, one, one))
    BSe = np.hstack([d1 * kron3(StM, StM, BS), d2 * kron3(StM, BS, StM), d3 * kron3(BS, StM, StM)])
    nf = 2 * M.shape[0] ** 2
    face = np.zeros((3 * nf, 3 * nf))
    face[:nf, :nf] = d1 * kron3(M, M, H)
    face[nf:2 * nf, nf:2 * nf] = d2 * kron3(M, H, M)
    face[2 * nf:, 2 * nf:] = d3 * kron3(H, M, M)
    return face - BSe.T @ (BSe / DZ[:, None]), {"S": S, "Lam": Lam, "BS": BS, "H": H, "I": I}


def face_transform(S, n_p):
    """Block-diagonal T over the six element faces: S x S on the tangential
    indices, identity on the side index (Table 1 face shapes)."""
    I2 = np.eye(2)
    T1 = kron3(S, S, I2)
    T2 = kron3(S, I2, S)
    T3 = kron3(I2, S, S)
    return sla.block_diag(T1, T2, T3)
