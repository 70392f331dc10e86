"""The paper's nodal-basis CG solvers of the condensed system (oracle).

TEST INFRASTRUCTURE ONLY: nothing in the product path may import this module.

Section "Summary of solution method" compares CG solvers of K_ff u = F_f
that all use the factorised operator: HDG-unprec (no preconditioner),
HDG-diag (diagonal preconditioner), HDG-block (block preconditioner,
algorithm "Block_Preconditioner") in the nodal trace basis, and HDG-trans
(the transformed system with its diagonal preconditioner).  Section
"Preconditioners" defines the two nodal preconditioners from the face
blocks of K:

* block: the exact inverse of every face's block of K_ff (the coupling of a
  face with itself, summed over its two elements) -- block Jacobi over the
  faces;
* diag: the main diagonal of that block inverse (the restrictor formula of
  the same section), applied as a pointwise scaling.

Here both are formed by definition: the dense n_p^2 x n_p^2 diagonal blocks
of the assembled K_ff are cut out and inverted with numpy.  The CG is the
textbook preconditioned CG with x_0 = 0, stopped when ||r||_2 <= rtol
||F||_2 (residual of the recursion, in the basis the CG runs in).
"""
from __future__ import annotations

import numpy as np


def face_block_inverses(K_ff, npf: int) -> np.ndarray:
    """Inverses of the diagonal face blocks of K_ff: [n_faces, npf, npf]."""
    K = K_ff.toarray() if hasattr(K_ff, "toarray") else np.asarray(K_ff)
    nfaces = K.shape[0] // npf
    out = np.empty((nfaces, npf, npf))
    for f in range(nfaces):
        s = slice(f * npf, (f + 1) * npf)
        out[f] = np.linalg.inv(K[s, s])
    return out


def block_preconditioner(K_ff, npf: int):
    """z = P^-1 r with P = block diagonal of K_ff over the faces."""
    inv = face_block_inverses(K_ff, npf)

    def apply(r):
        return np.einsum("fij,fj->fi", inv, r.reshape(-1, npf)).ravel()
    return apply


def diagonal_preconditioner(K_ff, npf: int):
    """z = d * r with d the main diagonal of the face-block inverses."""
    d = np.concatenate([np.diag(b) for b in face_block_inverses(K_ff, npf)])

    def apply(r):
        return d * r
    return apply, d


def pcg(K, F, apply_pinv=None, rtol: float = 1e-10, maxit: int = 100000, x0=None,
        relative_to: str = "rhs"):
    """Textbook preconditioned CG for the SPD matrix K (dense or sparse),
    from x0 (default 0); stops when ||r||_2 <= rtol ||F||_2, or with
    relative_to="initial" when ||r||_2 <= rtol ||r_0||_2 (the paper's test
    protocol).  Returns (x, iterations, history of ||r||_2 / ||F||_2)."""
    F = np.asarray(F, dtype=np.float64)
    x = np.zeros_like(F) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    r = F - K @ x if x0 is not None else F.copy()
    nF = np.linalg.norm(F)
    hist = [np.linalg.norm(r) / nF if nF > 0 else 0.0]
    if nF == 0.0:
        return x, 0, hist
    if relative_to == "initial":
        rtol = rtol * hist[0]
    elif relative_to != "rhs":
        raise ValueError("relative_to must be 'rhs' or 'initial'")
    if hist[0] <= rtol:
        return x, 0, hist
    z = r.copy() if apply_pinv is None else apply_pinv(r)
    p = z.copy()
    rho = r @ z
    for k in range(1, maxit + 1):
        q = K @ p
        alpha = rho / (p @ q)
        x += alpha * p
        r -= alpha * q
        hist.append(np.linalg.norm(r) / nF)
        if hist[-1] <= rtol:
            return x, k, hist
        z = r.copy() if apply_pinv is None else apply_pinv(r)
        rho_new = r @ z
        p = z + (rho_new / rho) * p
        rho = rho_new
    return x, maxit, hist
