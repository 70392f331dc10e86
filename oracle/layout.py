"""Trace and volume numbering of a Cartesian mesh (oracle side).

TEST INFRASTRUCTURE ONLY: nothing in the product path may import this module.

This is the canonical layout through which the oracle and the GPU library
exchange vectors; both implement it independently from this description.

Elements: axis a in {0,1,2} has n_a elements of widths h_a[0..n_a-1]; the box
starts at the origin.  Element e = i + n1 (j + n2 k).  Element nodes: GLL index
q1 + n_p (q2 + n_p q3), q1 fastest; the volume vector is element-major.

Faces: the faces normal to axis a sit on planes m = 0..n_a.  Interior planes
m = 1..n_a-1 always carry free unknowns.  Each of the six sides of the box
(axis a, side s: 0 the plane m = 0, 1 the plane m = n_a) is either a
Dirichlet side (u = g_D, the default) or a Neumann side (n . grad u = g_N,
equation (neumann_flux)); the set is a bit mask with bit 2a + s for a
Neumann side.  The trace of a Neumann side is unknown too.  The trace
vector is

    [interior faces normal to x1][... x2][... x3][Neumann faces]   (free part)
    [Dirichlet faces]                                              (g_D)
    [Neumann data]                                                 (g_N)

Interior faces of axis a are ordered lexicographically with x1 fastest over
their position (m along a, element indices along the two other axes):
    a=0: id = (m-1) + (n1-1) (j + n2 k)
    a=1: id = i + n1 ((m-1) + (n2-1) k)
    a=2: id = i + n1 (j + n2 (m-1))
Boundary faces come side by side in the order (a, s) = (0,0), (0,1), (1,0),
(1,1), (2,0), (2,1), each side ordered t_b + n_b t_c over the tangential
element indices (b < c); the Neumann sides in the free part, the Dirichlet
sides in the g_D block.  The g_N block repeats the Neumann faces' order: the
data of the i-th Neumann face follows the g_D block at offset i n_p^2.
Within a face: n_p x n_p GLL nodes, id = q_b + n_p q_c (lower axis fastest).
With no Neumann side this is the plain Dirichlet layout (free part = interior
faces, tail = all boundary faces).

Element-local face vectors follow the paper's Table 1 shapes (first index
fastest): u1 is 2 x n_p x n_p (side, q2, q3), u2 is n_p x 2 x n_p (q1, side,
q3), u3 is n_p x n_p x 2 (q1, q2, side); they are concatenated u1, u2, u3.
"""
from __future__ import annotations

import numpy as np


class Layout:
    def __init__(self, n, p, neumann: int = 0):
        self.n = tuple(int(v) for v in n)
        self.p = int(p)
        self.np_ = self.p + 1
        self.neumann = int(neumann)
        if not 0 <= self.neumann < 64:
            raise ValueError("neumann mask must be in [0, 63]")
        n1, n2, n3 = self.n
        npf = self.np_ ** 2
        self.face_counts_free = [(n1 - 1) * n2 * n3, n1 * (n2 - 1) * n3, n1 * n2 * (n3 - 1)]
        self.free_offset = [0, 0, 0]
        off = 0
        for a in range(3):
            self.free_offset[a] = off
            off += self.face_counts_free[a]
        self.n_int_faces = off
        tang = [(n2, n3), (n1, n3), (n1, n2)]
        self.side_faces = {(a, s): tang[a][0] * tang[a][1] for a in range(3) for s in (0, 1)}
        self.bdry_offset = {}
        for want_neumann in (True, False):
            for a in range(3):
                for side in (0, 1):
                    if self.is_neumann_side(a, side) == want_neumann:
                        self.bdry_offset[(a, side)] = off
                        off += self.side_faces[(a, side)]
            if want_neumann:
                self.n_free_faces = off
        self.n_faces = off
        self.n_neu_faces = self.n_free_faces - self.n_int_faces
        self.n_dir_faces = self.n_faces - self.n_free_faces
        self.n_free = self.n_free_faces * npf
        self.n_all = (self.n_faces + self.n_neu_faces) * npf
        self.n_elem = n1 * n2 * n3
        self.n_vol = self.n_elem * self.np_ ** 3

    def is_neumann_side(self, a, side):
        return bool((self.neumann >> (2 * a + side)) & 1)

    def neumann_data_index(self, fid):
        """First trace-vector index of the g_N data of Neumann face fid."""
        if not self.n_int_faces <= fid < self.n_free_faces:
            raise IndexError("not a Neumann face")
        return (self.n_faces + fid - self.n_int_faces) * self.np_ ** 2

    def face_side(self, fid):
        """(a, s) of a boundary face, None for an interior face."""
        for key, off in self.bdry_offset.items():
            if off <= fid < off + self.side_faces[key]:
                return key
        return None

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
    """Physical coordinates of every trace node, shape (n_all, 3); the g_N
    block repeats the coordinates of its Neumann faces."""
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
    npf = npn * npn
    for f in range(layout.n_int_faces, layout.n_free_faces):
        d = layout.neumann_data_index(f)
        out[d:d + npf] = out[f * npf:(f + 1) * npf]
    return out


def trace_normals(layout: Layout):
    """Outward unit normal of the boundary at every trace node (rows of the
    Neumann faces, the g_D block and the g_N block), zero elsewhere."""
    npf = layout.np_ ** 2
    out = np.zeros((layout.n_all, 3))
    for (a, s), off in layout.bdry_offset.items():
        nf = layout.side_faces[(a, s)]
        out[off * npf:(off + nf) * npf, a] = 2.0 * s - 1.0
        if layout.is_neumann_side(a, s):
            d = layout.neumann_data_index(off)
            out[d:d + nf * npf, a] = 2.0 * s - 1.0
    return out
