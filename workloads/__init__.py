"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This module holds no arithmetic of the discretisation: it draws element
widths, Helmholtz parameters, forcing values and trace vectors from seeded
generators, and it defines the analytic manufactured solutions as plain
functions of the physical coordinates.  Whoever needs nodal values evaluates
these functions at node coordinates that it computes itself.

Workload recipes (the shapes follow the paper's experiments: Cartesian
hexahedral meshes, degrees p = 2..16, lambda over several decades; the paper
measures on an analytic test case, see its section on the test case, so no
dataset is involved):

* ``tiny``      unit cube, 2x2x2 uniform, p=4, lambda=1, tau=1,
                u = sin(pi x) sin(pi y) sin(pi z), f = (lambda + 3 pi^2) u,
                random trace U[-1,1] (seed 1).
* ``perturbed`` unit cube, 16^3, widths per axis w ~ U[0.7,1.3] drawn x, y, z
                in order (seed 2) and renormalised to sum 1; p=7,
                lambda=10, tau=1; f ~ U[-1,1] i.i.d. per element node (same
                generator, after the widths); homogeneous Dirichlet data.
* ``mixed``     unit cube, 32^3 uniform, p in {4,8,12}, lambda in
                {1e-2,1,1e2}, tau=1, u = sin(2 pi x) cos(3 pi y) exp(z),
                f = (lambda + 13 pi^2 - 1) u, Dirichlet data = u.
* ``batched``   256 problems (seed 4): per problem n1, n2, n3 ~ U{4..12},
                p ~ U{2..10}, log10 lambda ~ U[-2,2], then f ~ N(0,1) per
                node; uniform unit-cube meshes, tau=1, homogeneous Dirichlet.
* ``adjoint``   unit cube, 24^3 uniform, p=6, tau=1, ln lambda_e ~ N(0,1)
                (seed 5), u* = sin sin sin + N(0, 0.01^2) per node,
                f = (lambda_e + 3 pi^2) sin sin sin at the nodes, homogeneous
                Dirichlet data.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np


# ----------------------------------------------------------------------------
# Manufactured solutions (analytic functions of physical coordinates)
# ----------------------------------------------------------------------------

def u_sin3(x, y, z):
    """u = sin(pi x) sin(pi y) sin(pi z)."""
    return np.sin(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * z)


def f_sin3(x, y, z, lam):
    """lambda u - laplace u for u_sin3: (lambda + 3 pi^2) u."""
    return (lam + 3.0 * np.pi ** 2) * u_sin3(x, y, z)


def u_mixed(x, y, z):
    """u = sin(2 pi x) cos(3 pi y) exp(z)."""
    return np.sin(2 * np.pi * x) * np.cos(3 * np.pi * y) * np.exp(z)


def f_mixed(x, y, z, lam):
    """lambda u - laplace u for u_mixed: (lambda + 13 pi^2 - 1) u."""
    return (lam + 13.0 * np.pi ** 2 - 1.0) * u_mixed(x, y, z)


def u_paper(x, y, z, k=5.0):
    """The paper's manufactured solution on (0, 2 pi)^3 (test-case section)."""
    return (np.cos(k * (x - 3 * y + 2 * z)) * np.sin(k * (1 + x))
            * np.sin(k * (1 - y)) * np.sin(k * (2 * x + y))
            * np.sin(k * (3 * x - 2 * y + 2 * z)))


# u_paper as a product of five factors g_m(k (a_m . x + c_m)), g_m = cos for
# the first factor, sin for the others: (a_m, c_m, is_cos)
_PAPER_FACTORS = (((1.0, -3.0, 2.0), 0.0, True), ((1.0, 0.0, 0.0), 1.0, False),
                  ((0.0, -1.0, 0.0), 1.0, False), ((2.0, 1.0, 0.0), 0.0, False),
                  ((3.0, -2.0, 2.0), 0.0, False))


def f_paper(x, y, z, lam, k=5.0):
    """lambda u - laplace u for u_paper, evaluated analytically.

    For u = prod_m g_m(k (a_m . x + c_m)) with g'' = -g:
      laplace u = -k^2 sum_m |a_m|^2 u
                  + k^2 sum_{m != n} (a_m . a_n) g_m' g_n' prod_{l != m, n} g_l.
    """
    X = (np.asarray(x, dtype=np.float64), np.asarray(y, dtype=np.float64),
         np.asarray(z, dtype=np.float64))
    g, dg, a = [], [], []
    for am, cm, is_cos in _PAPER_FACTORS:
        t = k * (am[0] * X[0] + am[1] * X[1] + am[2] * X[2] + cm)
        g.append(np.cos(t) if is_cos else np.sin(t))
        dg.append(-np.sin(t) if is_cos else np.cos(t))
        a.append(np.asarray(am))
    m5 = len(g)
    u = np.prod(g, axis=0)
    lap = -k * k * sum(float(a[m] @ a[m]) for m in range(m5)) * u
    for m in range(m5):
        for n in range(m5):
            if m == n:
                continue
            rest = np.ones_like(u)
            for l in range(m5):
                if l != m and l != n:
                    rest = rest * g[l]
            lap = lap + k * k * float(a[m] @ a[n]) * dg[m] * dg[n] * rest
    return lam * u - lap


def paper_case(p: int, n: int = 8, tau_e: float = 25.0, lam: float = 0.0) -> Problem:
    """The paper's solver test: (0, 2 pi)^3, n^3 uniform elements, degree p,
    penalty tau_e = 2 tau_hat / h (so tau_hat = tau_e h / 2), Poisson
    (lambda = 0) by default, Dirichlet data and forcing from u_paper."""
    h = 2.0 * math.pi / n
    return Problem(f"paper_p{p}", (n, n, n), [np.full(n, h)] * 3, p=p, tau=tau_e * h / 2.0,
                   lam=np.full(n ** 3, float(lam)), u_exact=u_paper,
                   f_func=f_paper, dirichlet_zero=False)


def paper_initial_volume(coords: np.ndarray, seed: int, length: float = 2.0 * math.pi) -> np.ndarray:
    """The paper's initial guess for its test case: pseudo-random numbers
    U[0, 1) at the volume nodes inside the domain (0, length)^3, the exact
    solution u_paper at the nodes on its boundary."""
    out = np.random.default_rng(seed).uniform(0.0, 1.0, size=coords.shape[0])
    tol = 1e-12 * length
    bnd = np.any((np.abs(coords) < tol) | (np.abs(coords - length) < tol), axis=1)
    out[bnd] = u_paper(*coords[bnd].T)
    return out


def poly_tensor(coeffs: np.ndarray) -> Callable:
    """Tensor polynomial sum_{abc} c[a,b,c] x^a y^b z^c (degree <= p per axis).

    Returns (u, f_of_lambda) where f = lambda u - laplace u, evaluated exactly
    from the monomial coefficients.
    """
    c = np.asarray(coeffs, dtype=np.float64)
    P = c.shape[0]

    def _eval(cc, x, y, z):
        out = np.zeros(np.broadcast(x, y, z).shape)
        for a in range(cc.shape[0]):
            for b in range(cc.shape[1]):
                for g in range(cc.shape[2]):
                    if cc[a, b, g] != 0.0:
                        out = out + cc[a, b, g] * x ** a * y ** b * z ** g
        return out

    def _d2(cc, axis):
        d = np.zeros_like(cc)
        for m in range(2, P):
            src = [slice(None)] * 3
            dst = [slice(None)] * 3
            src[axis] = m
            dst[axis] = m - 2
            d[tuple(dst)] += m * (m - 1) * cc[tuple(src)]
        return d

    lap = _d2(c, 0) + _d2(c, 1) + _d2(c, 2)

    def u(x, y, z):
        return _eval(c, x, y, z)

    def f(x, y, z, lam):
        return lam * _eval(c, x, y, z) - _eval(lap, x, y, z)

    return u, f


def poly_tensor_grad(coeffs: np.ndarray) -> Callable:
    """Gradient of the tensor polynomial of ``poly_tensor``: returns g with
    g(x, y, z) of shape (..., 3)."""
    c = np.asarray(coeffs, dtype=np.float64)
    P = c.shape[0]

    def _d1(axis):
        d = np.zeros_like(c)
        for m in range(1, P):
            src = [slice(None)] * 3
            dst = [slice(None)] * 3
            src[axis] = m
            dst[axis] = m - 1
            d[tuple(dst)] += m * c[tuple(src)]
        return d

    parts = [_d1(0), _d1(1), _d1(2)]

    def g(x, y, z):
        out = []
        for cc in parts:
            v = np.zeros(np.broadcast(x, y, z).shape)
            for a in range(cc.shape[0]):
                for b in range(cc.shape[1]):
                    for e in range(cc.shape[2]):
                        if cc[a, b, e] != 0.0:
                            v = v + cc[a, b, e] * x ** a * y ** b * z ** e
            out.append(v)
        return np.stack(out, axis=-1)

    return g


def grad_sin3(x, y, z):
    """Gradient of u_sin3."""
    return np.stack([np.pi * np.cos(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * z),
                     np.pi * np.sin(np.pi * x) * np.cos(np.pi * y) * np.sin(np.pi * z),
                     np.pi * np.sin(np.pi * x) * np.sin(np.pi * y) * np.cos(np.pi * z)], axis=-1)


def boundary_data(u, grad, coords: np.ndarray, normals: np.ndarray) -> np.ndarray:
    """Full trace vector of boundary data: u at every node, replaced by the
    normal derivative n . grad u wherever ``normals`` marks a g_N slot
    (rows with a nonzero normal that the caller passes for the g_N block
    only).  coords / normals: (n_all, 3)."""
    out = u(*coords.T)
    rows = np.nonzero(np.any(normals != 0.0, axis=1))[0]
    if rows.size:
        out[rows] = np.einsum("ij,ij->i", normals[rows], grad(*coords[rows].T))
    return out


# ----------------------------------------------------------------------------
# Problem descriptions
# ----------------------------------------------------------------------------

@dataclass
class Problem:
    """A Helmholtz problem on a Cartesian mesh of the box [0, sum h_a]^3."""

    name: str
    n: tuple                      # elements per axis (n1, n2, n3)
    widths: list                  # three float64 arrays, element widths per axis
    p: int                        # polynomial degree
    tau: float                    # stabilisation tau_hat
    lam: np.ndarray               # per-element lambda, shape (n1*n2*n3,)
    u_exact: Optional[Callable] = None            # u(x, y, z) or None
    f_func: Optional[Callable] = None             # f(x, y, z, lam) or None
    f_values: Optional[np.ndarray] = None         # nodal f if drawn randomly
    dirichlet_zero: bool = True   # True: g_D = 0, else g_D = u_exact at faces
    extra: dict = field(default_factory=dict)

    @property
    def n_elem(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    @property
    def n_p(self) -> int:
        return self.p + 1

    def n_trace_free(self) -> int:
        n1, n2, n3 = self.n
        return self.n_p ** 2 * ((n1 - 1) * n2 * n3 + n1 * (n2 - 1) * n3 + n1 * n2 * (n3 - 1))

    def n_trace_all(self) -> int:
        n1, n2, n3 = self.n
        return self.n_trace_free() + self.n_p ** 2 * 2 * (n2 * n3 + n1 * n3 + n1 * n2)

    def n_vol(self) -> int:
        return self.n_elem * self.n_p ** 3


def uniform_widths(n: int, length: float = 1.0) -> np.ndarray:
    return np.full(n, length / n, dtype=np.float64)


def perturbed_widths(n: int, rng: np.random.Generator, lo=0.7, hi=1.3,
                     length: float = 1.0) -> np.ndarray:
    w = rng.uniform(lo, hi, size=n)
    return length * w / w.sum()


def random_trace(n: int, seed: int) -> np.ndarray:
    """Trace vector with entries U[-1, 1]."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=n)


def tiny() -> Problem:
    lam = 1.0
    return Problem("tiny", (2, 2, 2), [uniform_widths(2)] * 3, p=4, tau=1.0,
                   lam=np.full(8, lam), u_exact=u_sin3, f_func=f_sin3,
                   dirichlet_zero=False, extra={"trace_seed": 1})


def perturbed(n: int = 16, p: int = 7, lam: float = 10.0, seed: int = 2) -> Problem:
    rng = np.random.default_rng(seed)
    widths = [perturbed_widths(n, rng) for _ in range(3)]
    prob = Problem("perturbed", (n, n, n), widths, p=p, tau=1.0,
                   lam=np.full(n ** 3, float(lam)), dirichlet_zero=True)
    prob.f_values = rng.uniform(-1.0, 1.0, size=prob.n_vol())
    return prob


def mixed(p: int, lam: float, n: int = 32) -> Problem:
    return Problem(f"mixed_p{p}_lam{lam:g}", (n, n, n), [uniform_widths(n)] * 3,
                   p=p, tau=1.0, lam=np.full(n ** 3, float(lam)),
                   u_exact=u_mixed, f_func=f_mixed, dirichlet_zero=False)


def batched(count: int = 256, seed: int = 4, n_range=(4, 12), p_range=(2, 10)):
    """List of independent problems drawn in order per problem."""
    rng = np.random.default_rng(seed)
    probs = []
    for b in range(count):
        n = tuple(int(v) for v in rng.integers(n_range[0], n_range[1] + 1, size=3))
        p = int(rng.integers(p_range[0], p_range[1] + 1))
        lam = float(10.0 ** rng.uniform(-2.0, 2.0))
        pr = Problem(f"batch{b}", n, [uniform_widths(v) for v in n], p=p, tau=1.0,
                     lam=np.full(n[0] * n[1] * n[2], lam), dirichlet_zero=True)
        pr.f_values = rng.standard_normal(pr.n_vol())
        probs.append(pr)
    return probs


def adjoint(n: int = 24, p: int = 6, seed: int = 5) -> Problem:
    rng = np.random.default_rng(seed)
    lam = np.exp(rng.standard_normal(n ** 3))
    pr = Problem(f"adjoint{n}", (n, n, n), [uniform_widths(n)] * 3, p=p, tau=1.0,
                 lam=lam, u_exact=u_sin3, dirichlet_zero=True)
    pr.extra["noise_seed"] = seed * 1000 + 1
    pr.extra["fd_seed"] = seed * 1000 + 2
    return pr


def lambda_forcing_sin3(x, y, z, lam_nodes):
    """f = (lambda_e + 3 pi^2) u_sin3 with lambda given per node."""
    return (lam_nodes + 3.0 * np.pi ** 2) * u_sin3(x, y, z)


def target_with_noise(u_nodes: np.ndarray, seed: int, sigma: float = 0.01) -> np.ndarray:
    """u* = u + N(0, sigma^2) per node."""
    return u_nodes + sigma * np.random.default_rng(seed).standard_normal(u_nodes.shape)


def fd_directions(n_lambda: int, n_f: int, count: int, seed: int):
    """Random unit directions (v_lambda, v_f) for central finite differences."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        vl = rng.standard_normal(n_lambda)
        vf = rng.standard_normal(n_f)
        s = math.sqrt(float(vl @ vl + vf @ vf))
        out.append((vl / s, vf / s))
    return out
