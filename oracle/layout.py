"""Trace and volume numbering of a Cartesian mesh (oracle side).

TEST INFRASTRUCTURE ONLY: nothing in the product path may import this module.

This is the canonical layout through which the oracle and the GPU library
exchange vectors; both implement it independently from this description.

Elements: axis a in {0,1,2} has n_a elements of widths h_a[0..n_a-1]; the box
starts at the origin.  Element e = i + n1 (j + n2 k).  Element nodes: GLL index
q1 + n_p (q2 + n_p q3), q1 fastest; the volume vector is element-major.

Faces: the faces normal to axis a sit on planes m = 0..n_a.  Interior planes
m = 1..n_a-1 carry the free unknowns, boundary planes m = 0 and m = n_a carry
Dirichlet data.  The trace vector is

    [free faces normal to x1][... x2][... x3][boundary faces]

Free faces of axis a are ordered lexicographically with x1 fastest over their
position (m along a, element indices along the two other axes):
    a=0: id = (m-1) + (n1-1) (j + n2 k)
    a=1: id = i + n1 ((m-1) + (n2-1) k)
    a=2: id = i + n1 (j + n2 (m-1))
The boundary tail holds, for a = 0, 1, 2, the low plane then the high plane,
each ordered t_b + n_b t_c over the tangential element indices (b < c).
Within a face: n_p x n_p GLL nodes, id = q_b + n_p q_c (lower axis fastest).

Element-local face vectors follow the paper's Table 1 shapes (first index
fastest): u1 is 2 x n_p x n_p (side, q2, q3), u2 is n_p x 2 x n_p (q1, side,
q3), u3 is n_p x n_p x 2 (q1, q2, side); they are concatenated u1, u2, u3.
"""
from __future__ import annotations

import numpy as np


class Layout:
    def __init__(self, n, p):
        self.n = tuple(int(v) for v in n)
        self.p = int(p)
        self.np_ = self.p + 1
        n1, n2, n3 = self.n
        npf = self.np_ ** 2
        self.face_counts_free = [(n1 - 1) * n2 * n3, n1 * (n2 - 1) * n3, n1 * n2 * (n3 - 1)]
        self.free_offset = [0, 0, 0]
        off = 0
        for a in range(3):
            self.free_offset[a] = off
            off += self.face_counts_free[a]
        self.n_free_faces = off
        tang = [(n2, n3), (n1, n3), (n1, n2)]
        self.bdry_offset = {}
        for a in range(3):
            for side in (0, 1):
                self.bdry_offset[(a, side)] = off
                off += tang[a][0] * tang[a][1]
        self.n_faces = off
        self.n_free = self.n_free_faces * npf
        self.n_all = self.n_faces * npf
        self.n_elem = n1 * n2 * n3
        self.n_vol = self.n_elem * self.np_ ** 3

    def face_id(self, a, m, t):
        """Global face index of the face normal to axis a on plane m; t = the
        element indices (i, j, k) with the a-th entry ignored."""
        n1, n2, n3 = self.n
        i, j, k = t
        na = self.n[a]
        if 1 <= m <= na - 1:
            if a == 0:
                loc = (m - 1) + (n1 - 1) * (j + n2 * k)
            elif a == 1:
                loc = i + n1 * ((m - 1) + (n2 - 1) * k)
            else:
                loc = i + n1 * (j + n2 * (m - 1))
            return self.free_offset[a] + loc
        side = 0 if m == 0 else 1
        if m not in (0, na):
            raise IndexError("face plane out of range")
        if a == 0:
            tb, tc, nb = j, k, n2
        elif a == 1:
            tb, tc, nb = i, k, n1
        else:
            tb, tc, nb = i, j, n1
        return self.bdry_offset[(a, side)] + tb + nb * tc

    def is_free_face(self, fid):
        return fid < self.n_free_faces

    def elem_index(self, i, j, k):
        n1, n2, _ = self.n
        return i + n1 * (j + n2 * k)

    def elem_ijk(self, e):
        n1, n2, _ = self.n
        return e % n1, (e // n1) % n2, e // (n1 * n2)

    def element_trace_map(self, e):
        """Global DOF index of every element-local face DOF (6 n_p^2 entries),
        in the order u1 (s, q2, q3), u2 (q1, s, q3), u3 (q1, q2, s)."""
        npn = self.np_
        npf = npn * npn
        i, j, k = self.elem_ijk(e)
        out = np.empty(6 * npf, dtype=np.int64)
        # direction 1: local index s + 2 (q2 + n_p q3)
        for s in (0, 1):
            f = self.face_id(0, i + s, (i, j, k))
            for q3 in range(npn):
                for q2 in range(npn):
                    out[0 * 2 * npf + s + 2 * (q2 + npn * q3)] = f * npf + q2 + npn * q3
        # direction 2: local index q1 + n_p (s + 2 q3)
        for s in (0, 1):
            f = self.face_id(1, j + s, (i, j, k))
            for q3 in range(npn):
                for q1 in range(npn):
                    out[1 * 2 * npf + q1 + npn * (s + 2 * q3)] = f * npf + q1 + npn * q3
        # direction 3: local index q1 + n_p (q2 + n_p s)
        for s in (0, 1):
            f = self.face_id(2, k + s, (i, j, k))
            for q2 in range(npn):
                for q1 in range(npn):
                    out[2 * 2 * npf + q1 + npn * (q2 + npn * s)] = f * npf + q1 + npn * q2
        return out


def axis_breaks(widths):
    """Plane coordinates X[0..n] of one axis."""
    return np.concatenate(([0.0], np.cumsum(np.asarray(widths, dtype=np.float64))))


def volume_coords(layout: Layout, widths, gll_x):
    """Physical coordinates of every volume node, shape (n_vol, 3)."""
    npn = layout.np_
    n1, n2, n3 = layout.n
    X = [axis_breaks(w) for w in widths]
    out = np.empty((layout.n_vol, 3))
    ref = (np.asarray(gll_x) + 1.0) / 2.0
    for e in range(layout.n_elem):
        i, j, k = layout.elem_ijk(e)
        x1 = X[0][i] + widths[0][i] * ref
        x2 = X[1][j] + widths[1][j] * ref
        x3 = X[2][k] + widths[2][k] * ref
        c3, c2, c1 = np.meshgrid(x3, x2, x1, indexing="ij")   # q1 fastest
        blk = slice(e * npn ** 3, (e + 1) * npn ** 3)
        out[blk, 0] = c1.ravel()
        out[blk, 1] = c2.ravel()
        out[blk, 2] = c3.ravel()
    return out


def trace_coords(layout: Layout, widths, gll_x):
    """Physical coordinates of every trace node, shape (n_all, 3)."""
    npn = layout.np_
    X = [axis_breaks(w) for w in widths]
    ref = (np.asarray(gll_x) + 1.0) / 2.0
    out = np.full((layout.n_all, 3), np.nan)
    for e in range(layout.n_elem):
        i, j, k = layout.elem_ijk(e)
        idx = [i, j, k]
        for a in range(3):
            b, c = [ax for ax in range(3) if ax != a]
            for s in (0, 1):
                m = idx[a] + s
                f = layout.face_id(a, m, (i, j, k))
                xb = X[b][idx[b]] + widths[b][idx[b]] * ref
                xc = X[c][idx[c]] + widths[c][idx[c]] * ref
                cc, cb = np.meshgrid(xc, xb, indexing="ij")   # q_b fastest
                rows = f * npn * npn + np.arange(npn * npn)
                out[rows, a] = X[a][m]
                out[rows, b] = cb.ravel()
                out[rows, c] = cc.ravel()
    return out
