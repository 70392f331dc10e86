"""Pins of the oracle's nodal-basis CG solvers (oracle/pcg.py) against the
paper's claims and textbook facts (no GPU).

* unpreconditioned CG reaches the direct solution;
* the inverse face blocks of K_ff equal the paper's factorised form
  (S x S) Y^-1 (S^T x S^T), Y the (diagonal) face blocks of the transformed
  operator (section "Preconditioners", algorithm "Block_Preconditioner");
* the diagonal preconditioner equals the restrictor formula of the same
  section, ((S o S) x (S o S)) Y^-1 per face (o: entrywise square);
* block-preconditioned CG in the nodal basis produces the same iterates as
  Jacobi-preconditioned CG on the transformed system (HDG-block and
  HDG-trans of section "Summary of solution method" are one solver).
"""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle.basis import standard_matrices
from oracle.fastdiag import eigen_1d
from oracle.pcg import block_preconditioner, diagonal_preconditioner, face_block_inverses, pcg


def _case(n=(3, 2, 2), p=3, lam=0.5, seed=4):
    rng = np.random.default_rng(seed)
    widths = [W.perturbed_widths(k, rng) for k in n]
    o = oracle.HdgOracle(n, widths, p, 1.0, lam)
    nf = o.layout.n_free
    K = o.assemble_K()[:nf, :nf].toarray()
    S, _ = eigen_1d(standard_matrices(p, 1.0))
    npf = (p + 1) ** 2
    Q = np.kron(np.eye(nf // npf), np.kron(S, S))   # eigen-face unknown -> nodal unknown
    return o, K, Q, S, npf


def test_unpreconditioned_cg_reaches_direct_solution():
    o, K, Q, S, npf = _case()
    F = W.random_trace(K.shape[0], 1)
    x, its, hist = pcg(K, F, None, rtol=1e-14, maxit=5000)
    ref = np.linalg.solve(K, F)
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) < 1e-10
    assert hist[-1] <= 1e-14 and its < 5000


def test_face_block_inverse_is_the_factorised_form():
    o, K, Q, S, npf = _case(p=4)
    Khat = Q.T @ K @ Q
    inv = face_block_inverses(K, npf)
    SS = np.kron(S, S)
    for f in range(K.shape[0] // npf):
        s = slice(f * npf, (f + 1) * npf)
        blk = Khat[s, s]
        y = np.diag(blk)
        # the transformed face block is diagonal
        assert np.max(np.abs(blk - np.diag(y))) < 1e-11 * np.max(np.abs(y))
        fact = SS @ np.diag(1.0 / y) @ SS.T
        assert np.max(np.abs(inv[f] - fact)) < 1e-10 * np.max(np.abs(fact))


def test_diagonal_preconditioner_is_the_restrictor_formula():
    o, K, Q, S, npf = _case(p=3)
    Khat = Q.T @ K @ Q
    _, d = diagonal_preconditioner(K, npf)
    S2 = S * S
    for f in range(K.shape[0] // npf):
        s = slice(f * npf, (f + 1) * npf)
        want = np.kron(S2, S2) @ (1.0 / np.diag(Khat[s, s]))
        assert np.max(np.abs(d[s] - want)) < 1e-10 * np.max(np.abs(want))


@pytest.mark.parametrize("m", [1, 5, 20])
def test_block_pcg_iterates_equal_transformed_jacobi_pcg(m):
    o, K, Q, S, npf = _case(n=(3, 3, 2), p=3, lam=0.0)
    F = W.random_trace(K.shape[0], 2)
    x, _, _ = pcg(K, F, block_preconditioner(K, npf), rtol=0.0, maxit=m)
    Khat = Q.T @ K @ Q
    dinv = 1.0 / np.diag(Khat)
    xh, _, _ = pcg(Khat, Q.T @ F, lambda r: dinv * r, rtol=0.0, maxit=m)
    assert np.linalg.norm(x - Q @ xh) / np.linalg.norm(x) < 1e-10


def test_preconditioners_reduce_iterations():
    o, K, Q, S, npf = _case(n=(3, 3, 3), p=4, lam=0.0)
    F = W.random_trace(K.shape[0], 3)
    _, it_u, _ = pcg(K, F, None, rtol=1e-10)
    _, it_d, _ = pcg(K, F, diagonal_preconditioner(K, npf)[0], rtol=1e-10)
    _, it_b, _ = pcg(K, F, block_preconditioner(K, npf), rtol=1e-10)
    assert it_b < it_u and it_d <= it_u + 2


def test_stopping_relative_to_initial_residual():
    """relative_to="initial" stops at ||r|| <= rtol ||r_0||: from x_0 = 0 it
    is the usual test (r_0 = F); from a start with ||r_0|| = 1e-3 ||F|| it
    stops at the first iterate that passes rtol * 1e-3 relative to ||F||."""
    o, K, Q, S, npf = _case(n=(3, 3, 2), p=3, lam=0.3)
    F = W.random_trace(K.shape[0], 9)
    x_a, it_a, _ = pcg(K, F, None, rtol=1e-8)
    x_b, it_b, _ = pcg(K, F, None, rtol=1e-8, relative_to="initial")
    assert it_a == it_b and np.array_equal(x_a, x_b)
    ref = np.linalg.solve(K, F)
    d = W.random_trace(K.shape[0], 10)
    x0 = ref + d * (1e-3 * np.linalg.norm(F) / np.linalg.norm(K @ d))
    r0 = np.linalg.norm(F - K @ x0) / np.linalg.norm(F)
    assert abs(r0 - 1e-3) < 1e-9
    _, it_c, hist = pcg(K, F, None, rtol=1e-6, x0=x0, relative_to="initial")
    assert hist[-1] <= 1e-6 * r0 and all(h > 1e-6 * r0 for h in hist[:-1])
    _, it_d, _ = pcg(K, F, None, rtol=1e-6, x0=x0)
    assert it_d < it_c
