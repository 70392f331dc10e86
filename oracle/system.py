"""Global condensed HDG system: assembly, direct solve, recovery, adjoint (oracle).

TEST INFRASTRUCTURE ONLY: nothing in the product path may import this module.

Follows equation (hdg_system): K u~ = F with K = sum_e Q_e^T K_e Q_e and
F = sum_e Q_e^T F_e, where Q_e scatters global trace unknowns to the element
faces (the element-local ordering of Table 1).  Dirichlet data is imposed
strongly: all trace nodes on Dirichlet faces are fixed to g_D (the values of
the Dirichlet function at the face nodes) and eliminated,

    K_ff u~_f = F_f - K_fD g_D.

On a Neumann side (equation (neumann_flux), n . grad u = g_N) the trace is
unknown and the flux row of the element system (the last row of equation
(ldg_element_operator)) carries the boundary data: there the numerical flux
equals g_N, which adds the face integral of mu g_N to F_e,

    g_N,e = (h_b h_c / 4) (M x M) g_N      (face normal to axis a, b, c the others)

with g_N sampled at the face nodes.

The initial guess of the solution process (section "Summary of solution
method") hybridizes a volume field u: q = grad u by differentiation, then
the flux of equation (fluxu) on every face,

    u~ = (tau+ u+ + tau- u-) / (tau+ + tau-) - (q+.n+ + q-.n-) / (tau+ + tau-),

tau = 2 tau_hat / h_a of the element on either side.  On a Neumann face
there is one element; the outside is read as tau- = 0 with the flux
q-.n- = -g_N it would bring, so u~ = u+ - (q+.n+ - g_N) / tau+.

Recovery of u per element uses the element system (see ``element``).  The
adjoint of u(lambda, f) is the dense transpose of the same steps:

    K_ff mu_f = -sum_e Q_e^T R_e^T A_e^-1 [r_e; 0],   mu_D = 0
    a_e       = A_e^-1 ([r_e; 0] - R_e mu_e)
    dJ/dlambda_e = -(u-part of a_e)^T M_e u_e,   dJ/df_e = M_e (u-part of a_e)

with r_e = dJ/du_e; this follows from dA_e/dlambda_e = diag(M_e, 0, 0, 0)
and the symmetry of A_e and K.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .basis import lagrange_deriv_eval, standard_matrices
from .element import ElementSystem
from .layout import Layout, trace_coords, trace_normals, volume_coords


def npf_of(layout):
    return layout.np_ ** 2


class HdgOracle:
    def __init__(self, n, widths, p, tau, lam, exact_mass=False, cache_limit=64, neumann=0):
        self.layout = Layout(n, p, neumann)
        self.widths = [np.asarray(w, dtype=np.float64) for w in widths]
        self.p = int(p)
        self.tau = float(tau)
        lam = np.asarray(lam, dtype=np.float64)
        if lam.ndim == 0:
            lam = np.full(self.layout.n_elem, float(lam))
        self.lam = lam
        self.std = standard_matrices(self.p, self.tau, exact_mass=exact_mass)
        self._cache = {}
        self._cache_limit = cache_limit
        self._maps = {}

    # -- element data --------------------------------------------------------
    def elem_h(self, e):
        i, j, k = self.layout.elem_ijk(e)
        return (self.widths[0][i], self.widths[1][j], self.widths[2][k])

    def _entry(self, e):
        h = self.elem_h(e)
        key = (float(h[0]), float(h[1]), float(h[2]), float(self.lam[e]))
        ent = self._cache.get(key)
        if ent is None:
            es = ElementSystem(self.std, h, float(self.lam[e]))
            AinvR = np.linalg.solve(es.A, es.R)
            K = es.G - es.R.T @ AinvR
            ent = {"sys": es, "K": K}
            if len(self._cache) >= self._cache_limit:
                self._cache.pop(next(iter(self._cache)))
            self._cache[key] = ent
        return ent

    def K_e(self, e):
        return self._entry(e)["K"]

    def system(self, e) -> ElementSystem:
        return self._entry(e)["sys"]

    def tmap(self, e):
        m = self._maps.get(e)
        if m is None:
            m = self.layout.element_trace_map(e)
            if len(self._maps) < 100000:
                self._maps[e] = m
        return m

    def vol_slice(self, e):
        nv = self.layout.np_ ** 3
        return slice(e * nv, (e + 1) * nv)

    # -- coordinates -----------------------------------------------------------
    def volume_coords(self):
        return volume_coords(self.layout, self.widths, self.std["x"])

    def trace_coords(self):
        return trace_coords(self.layout, self.widths, self.std["x"])

    def trace_normals(self):
        return trace_normals(self.layout)

    def mass_diag(self):
        """Diagonal of the lumped global mass matrix (volume ordering)."""
        w = self.std["w"]
        out = np.empty(self.layout.n_vol)
        wk = np.kron(w, np.kron(w, w))
        for e in range(self.layout.n_elem):
            h = self.elem_h(e)
            out[self.vol_slice(e)] = h[0] * h[1] * h[2] / 8.0 * wk
        return out

    # -- operator --------------------------------------------------------------
    def assemble_K(self):
        rows, cols, vals = [], [], []
        for e in range(self.layout.n_elem):
            m = self.tmap(e)
            K = self.K_e(e)
            rows.append(np.repeat(m, m.size))
            cols.append(np.tile(m, m.size))
            vals.append(K.ravel())
        n = self.layout.n_all
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(n, n))

    def apply(self, x_all):
        """y = K x element by element (all DOFs, no masking)."""
        y = np.zeros(self.layout.n_all)
        for e in range(self.layout.n_elem):
            m = self.tmap(e)
            y[m] += self.K_e(e) @ x_all[m]
        return y

    def apply_free(self, x_free):
        """y_f = K_ff x_f: Dirichlet entries of x are zero, of y dropped."""
        x = np.zeros(self.layout.n_all)
        x[: self.layout.n_free] = x_free
        return self.apply(x)[: self.layout.n_free]

    def faces_elements(self, face_ids):
        """Elements adjacent to the given global faces."""
        want = set(int(f) for f in face_ids)
        npf = self.layout.np_ ** 2
        out = []
        for e in range(self.layout.n_elem):
            fs = set((self.tmap(e) // npf).tolist())
            if fs & want:
                out.append(e)
        return out

    def apply_rows(self, x_all, dof_ids):
        """(K x)[dof_ids], summing only the elements that touch those DOFs."""
        dof_ids = np.asarray(dof_ids, dtype=np.int64)
        npf = self.layout.np_ ** 2
        elems = self.faces_elements(np.unique(dof_ids // npf))
        acc = {}
        for e in elems:
            m = self.tmap(e)
            ye = self.K_e(e) @ x_all[m]
            for loc, g in enumerate(m):
                acc[g] = acc.get(g, 0.0) + ye[loc]
        return np.array([acc.get(int(d), 0.0) for d in dof_ids])

    # -- right-hand side -----------------------------------------------------------
    def rhs_element(self, e, f_e):
        es = self.system(e)
        return -es.R.T @ np.linalg.solve(es.A, es.volume_rhs(es.Me @ f_e))

    def rhs_rows(self, f_vol, dof_ids):
        """F[dof_ids] of F = sum_e Q_e^T F_e (no Dirichlet lift, no Neumann
        load), summing only the elements that touch those DOFs."""
        dof_ids = np.asarray(dof_ids, dtype=np.int64)
        npf = self.layout.np_ ** 2
        acc = {}
        for e in self.faces_elements(np.unique(dof_ids // npf)):
            m = self.tmap(e)
            Fe = self.rhs_element(e, f_vol[self.vol_slice(e)])
            for loc, g in enumerate(m):
                acc[g] = acc.get(g, 0.0) + Fe[loc]
        return np.array([acc.get(int(d), 0.0) for d in dof_ids])

    def assemble_F(self, f_vol):
        F = np.zeros(self.layout.n_all)
        for e in range(self.layout.n_elem):
            m = self.tmap(e)
            F[m] += self.rhs_element(e, f_vol[self.vol_slice(e)])
        return F

    def neumann_load(self, g_all):
        """Sum of the g_N,e over the Neumann faces, as a free-trace vector
        (g_all: full trace vector whose g_N block holds n . grad u)."""
        L = self.layout
        npn = L.np_
        npf = npn * npn
        out = np.zeros(L.n_free)
        M = self.std["M"]
        Mf = np.kron(M, M)
        for e in range(L.n_elem):
            i, j, k = L.elem_ijk(e)
            h = self.elem_h(e)
            idx = (i, j, k)
            for a in range(3):
                b, c = [ax for ax in range(3) if ax != a]
                for s in (0, 1):
                    fid = L.face_id(a, idx[a] + s, idx)
                    if not L.n_int_faces <= fid < L.n_free_faces:
                        continue
                    d = L.neumann_data_index(fid)
                    out[fid * npf:(fid + 1) * npf] += h[b] * h[c] / 4.0 * (Mf @ g_all[d:d + npf])
        return out

    def lifted_rhs(self, f_vol, g_all):
        """F_f - K_fD g_D + g_N,f (g_all: Dirichlet values in the g_D block,
        Neumann data in the g_N block)."""
        L = self.layout
        nf = L.n_free
        F = self.assemble_F(f_vol)
        xD = np.zeros(L.n_all)
        end = L.n_faces * npf_of(L)
        xD[nf:end] = g_all[nf:end]
        rhs = F[:nf] - self.apply(xD)[:nf]
        if L.n_neu_faces:
            rhs = rhs + self.neumann_load(g_all)
        return rhs

    # -- initial guess -------------------------------------------------------------
    def hybridize(self, u_vol, g_all=None):
        """Free trace u~ of a volume field by the flux of equation (fluxu)
        with q = grad u (see the module docstring)."""
        L = self.layout
        npn = L.np_
        npf = npn * npn
        dphi = lagrange_deriv_eval(self.std["x"], np.array([-1.0, 1.0]))   # [end, k]
        num = np.zeros(L.n_free)
        den = np.zeros(L.n_free_faces)
        for e in range(L.n_elem):
            i, j, k = L.elem_ijk(e)
            idx = (i, j, k)
            h = self.elem_h(e)
            cube = u_vol[self.vol_slice(e)].reshape(npn, npn, npn)   # [q3][q2][q1]
            for a in range(3):
                ax = 2 - a                       # cube axis of x_{a+1}
                for s in (0, 1):
                    fid = L.face_id(a, idx[a] + s, idx)
                    if fid >= L.n_free_faces:
                        continue
                    end = s * (npn - 1)
                    uf = np.take(cube, end, axis=ax).ravel()
                    dn = (2.0 * s - 1.0) * (2.0 / h[a]) * np.tensordot(cube, dphi[s], axes=([ax], [0])).ravel()
                    tau_e = 2.0 * self.tau / h[a]
                    sl = slice(fid * npf, (fid + 1) * npf)
                    num[sl] += tau_e * uf - dn
                    den[fid] += tau_e
                    if fid >= L.n_int_faces and g_all is not None:
                        d = L.neumann_data_index(fid)
                        num[sl] += g_all[d:d + npf]
        return num / np.repeat(den, npf)

    # -- solve & recovery ------------------------------------------------------------
    def solve(self, f_vol, g_all):
        """Direct solve; returns the full trace (free part solved, tail = g_D)."""
        nf = self.layout.n_free
        rhs = self.lifted_rhs(f_vol, g_all)
        u = np.array(g_all, dtype=np.float64, copy=True)
        if nf == 0:
            return u
        K = self.assemble_K()[:nf, :nf].tocsc()
        if nf <= 6000:
            u[:nf] = np.linalg.solve(K.toarray(), rhs)
        else:
            u[:nf] = spla.spsolve(K, rhs)
        return u

    def reconstruct_element(self, e, f_e, trace_all):
        es = self.system(e)
        y = np.linalg.solve(es.A, es.volume_rhs(es.Me @ f_e) - es.R @ trace_all[self.tmap(e)])
        return y[: es.nv]

    def reconstruct(self, f_vol, trace_all):
        u = np.empty(self.layout.n_vol)
        for e in range(self.layout.n_elem):
            u[self.vol_slice(e)] = self.reconstruct_element(e, f_vol[self.vol_slice(e)], trace_all)
        return u

    # -- loss and adjoint -------------------------------------------------------------
    def loss(self, u_vol, u_target):
        d = u_vol - u_target
        return 0.5 * float(d @ (self.mass_diag() * d))

    def adjoint(self, f_vol, trace_all, u_vol, dJdu):
        """Gradients of J with respect to per-element lambda and nodal f."""
        L = self.layout
        nf = L.n_free
        j = np.zeros(L.n_all)
        for e in range(L.n_elem):
            es = self.system(e)
            j[self.tmap(e)] -= es.R.T @ np.linalg.solve(es.A, es.volume_rhs(dJdu[self.vol_slice(e)]))
        mu = np.zeros(L.n_all)
        if nf:
            K = self.assemble_K()[:nf, :nf].tocsc()
            mu[:nf] = np.linalg.solve(K.toarray(), j[:nf]) if nf <= 6000 else spla.spsolve(K, j[:nf])
        dlam = np.empty(L.n_elem)
        df = np.empty(L.n_vol)
        for e in range(L.n_elem):
            es = self.system(e)
            sl = self.vol_slice(e)
            a = np.linalg.solve(es.A, es.volume_rhs(dJdu[sl]) - es.R @ mu[self.tmap(e)])[: es.nv]
            dlam[e] = -a @ (es.Me @ u_vol[sl])
            df[sl] = es.Me @ a
        return dlam, df
