"""Oracle grid layer: canonical and derived connectivity, orientation, SFC renumbering.

Test infrastructure only.  Neighbour access on the icosahedral grid is by
index lookup (Section 4.2.1 of the paper, "stencil-like" access through
lookup tables); the grid itself is the RnBk construction of Section 5.1.
The canonical orders below are readings (the paper fixes none); the library
must reproduce every integer table of this module bit for bit.

Canonical rules, applied to the (possibly renumbered) input tables:
  e2v_t[e]   = e2v[e] swapped if needed so that (x_v1 - x_v0) . t_e > 0,
               with t_e = x_e x n_e (so (n, t, r) is right-handed).
  c2e[c]     = input order (e0, e1, e2) if the triangle it implies is
               counter-clockwise seen from outside, else (e0, e2, e1);
               c2e[c][i] joins c2v[c][i] and c2v[c][(i+1)%3].
  c2v[c][i]  = common vertex of c2e[c][i-1] and c2e[c][i].
  c2e2c[c][i]= the cell across c2e[c][i].
  s[c][i]    = +1 if c == e2c[c2e[c][i]][0] else -1 (outward normal sign).
  v2e[v]     = incident edges counter-clockwise around v, starting at the
               smallest edge id; slot 5 = -1 at the 12 pentagons.
  v2c[v][i]  = cell between v2e[v][i] and v2e[v][i+1] (cyclic); -1 padded.
  sig[v][i]  = +1 if v == e2v_t[v2e[v][i]][1] else -1 (counter-clockwise
               circulation sign).
  e2c2e[e]   = [c2e(c0) without e, in c2e order] ++ [c2e(c1) without e].
  e2c2v[e]   = [v0, v1, vertex of c0 off e, vertex of c1 off e].
SFC renumbering (optional): cells sorted by (triangle-tree key, old id);
edges sorted by (min new cell, max new cell, old id); vertices by
(min new id of the cells around it, old id).  The key of a unit vector x
walks a recursive subdivision of a fixed icosahedron (poles on the z axis,
the upper ring at longitudes 72 i degrees and z = 1/sqrt 5, the lower ring
36 degrees further and z = -1/sqrt 5): the face is the one whose smallest
great-circle side test det(x, B, C), det(A, x, C), det(A, B, x) is largest
(the first on ties); then, 16 times, the triangle (A, B, C) is split at the
normalised midpoints ab, bc, ca into the corner children (A, ab, ca),
(ab, B, bc), (ca, bc, C), taken when x lies inside the first of them
(det(x, ab, ca), det(x, bc, ab), det(x, ca, bc) > 0, tested in that order),
else the middle child (ab, bc, ca); key = face * 4^16 + the base-4 digits of
the children.  Blocks of 4^j consecutive keys are spherical triangles, so a
block of cells touches few cache lines of its neighbours' data.
"""
from __future__ import annotations

import numpy as np


def _common(a, b):
    """Row-wise common element of two (N, 2) arrays (exactly one expected)."""
    m00 = a[:, 0] == b[:, 0]
    m01 = a[:, 0] == b[:, 1]
    return np.where(m00 | m01, a[:, 0], a[:, 1])


def _ico():
    """The icosahedron of the tree key: 12 unit vertices, 20 faces
    counter-clockwise seen from outside (written out with square roots only,
    so that every implementation builds the same bits)."""
    s5 = np.sqrt(5.0)
    c1, s1 = (s5 - 1.0) / 2.0, np.sqrt(10.0 + 2.0 * s5) / 2.0  # 2 cos 72, 2 sin 72
    c2, s2 = (s5 + 1.0) / 2.0, np.sqrt(10.0 - 2.0 * s5) / 2.0  # 2 cos 36, 2 sin 36
    v = np.array([[0.0, 0.0, s5],
                  [2.0, 0.0, 1.0], [c1, s1, 1.0], [-c2, s2, 1.0], [-c2, -s2, 1.0], [c1, -s1, 1.0],
                  [c2, s2, -1.0], [-c1, s1, -1.0], [-2.0, 0.0, -1.0], [-c1, -s1, -1.0], [c2, -s2, -1.0],
                  [0.0, 0.0, -s5]]) / s5
    faces = np.array([[0, 1, 2], [1, 6, 2], [2, 6, 7], [11, 7, 6], [0, 2, 3], [2, 7, 3], [3, 7, 8],
                      [11, 8, 7], [0, 3, 4], [3, 8, 4], [4, 8, 9], [11, 9, 8], [0, 4, 5], [4, 9, 5],
                      [5, 9, 10], [11, 10, 9], [0, 5, 1], [5, 10, 1], [1, 10, 6], [11, 6, 10]])
    return v, faces


TREE_LEVELS = 16


def _det(a, b, c):
    """a . (b x c), summed in this order."""
    return ((a[..., 0] * (b[..., 1] * c[..., 2] - b[..., 2] * c[..., 1])
             + a[..., 1] * (b[..., 2] * c[..., 0] - b[..., 0] * c[..., 2]))
            + a[..., 2] * (b[..., 0] * c[..., 1] - b[..., 1] * c[..., 0]))


def _mid(p, q):
    s = p + q
    return s / np.sqrt((s[..., 0] * s[..., 0] + s[..., 1] * s[..., 1]) + s[..., 2] * s[..., 2])[..., None]


def tree_key(xyz):
    """Triangle-tree key (int64) of each row of xyz (any positive length:
    every decision is the sign or the order of triple products with x)."""
    v, faces = _ico()
    n = xyz.shape[0]
    best = np.full(n, -np.inf)
    face = np.zeros(n, dtype=np.int64)
    for f in range(20):
        a, b, c = v[faces[f, 0]], v[faces[f, 1]], v[faces[f, 2]]
        m = np.minimum(np.minimum(_det(xyz, b, c), _det(a, xyz, c)), _det(a, b, xyz))
        up = m > best
        best[up] = m[up]
        face[up] = f
    a, b, c = v[faces[face, 0]], v[faces[face, 1]], v[faces[face, 2]]
    key = face.copy()
    for _ in range(TREE_LEVELS):
        ab, bc, ca = _mid(a, b), _mid(b, c), _mid(c, a)
        ch = np.where(_det(xyz, ab, ca) > 0, 0,
                      np.where(_det(xyz, bc, ab) > 0, 1, np.where(_det(xyz, ca, bc) > 0, 2, 3)))[:, None]
        a, b, c = (np.where(ch == 0, a, np.where(ch == 1, ab, np.where(ch == 2, ca, ab))),
                   np.where(ch == 0, ab, np.where(ch == 1, b, bc)),
                   np.where(ch == 0, ca, np.where(ch == 1, bc, np.where(ch == 2, c, ca))))
        key = key * 4 + ch[:, 0]
    return key


def sfc_permutation(g):
    """Return new->old permutations (cells, edges, vertices)."""
    nc, ne, nv = g["n_cells"], g["n_edges"], g["n_verts"]
    key = tree_key(g["cell_xyz"])
    pc = np.lexsort((np.arange(nc), key))
    old2new_c = np.empty(nc, dtype=np.int64)
    old2new_c[pc] = np.arange(nc)
    ec = old2new_c[g["e2c"].astype(np.int64)]
    lo, hi = ec.min(axis=1), ec.max(axis=1)
    pe = np.lexsort((np.arange(ne), hi, lo))
    # vertices: minimum new cell id over the cells containing the vertex
    c2e = g["c2e"].astype(np.int64)
    e2v = g["e2v"].astype(np.int64)
    vmin = np.full(nv, np.iinfo(np.int64).max)
    for i in range(3):
        for j in range(2):
            np.minimum.at(vmin, e2v[c2e[:, i], j], old2new_c)
    pv = np.lexsort((np.arange(nv), vmin))
    return pc, pe, pv


def renumber(g, pc, pe, pv):
    """Apply new->old permutations to the input tables and geometry."""
    nc, ne, nv = g["n_cells"], g["n_edges"], g["n_verts"]
    inv = lambda p: np.argsort(p)  # old->new
    oc, oe, ov = inv(pc), inv(pe), inv(pv)
    h = dict(g)
    h["e2c"] = oc[g["e2c"][pe]].astype(np.int32)
    h["c2e"] = oe[g["c2e"][pc]].astype(np.int32)
    h["e2v"] = ov[g["e2v"][pe]].astype(np.int32)
    h["c2e2c"] = oc[g["c2e2c"][pc]].astype(np.int32)
    for name in ("cell_xyz", "cell_area"):
        h[name] = g[name][pc]
    for name in ("edge_xyz", "edge_length", "dual_edge_length", "edge_normal_xyz"):
        h[name] = g[name][pe]
    for name in ("vert_xyz", "dual_area"):
        h[name] = g[name][pv]
    return h


def derive(g):
    """Canonical and derived tables plus orientation signs (see module docstring)."""
    nc, ne, nv = g["n_cells"], g["n_edges"], g["n_verts"]
    xv, xe, xc = g["vert_xyz"], g["edge_xyz"], g["cell_xyz"]
    nrm = g["edge_normal_xyz"]
    e2c = g["e2c"].astype(np.int64)
    e2v = g["e2v"].astype(np.int64)
    c2e_in = g["c2e"].astype(np.int64)

    # edge tangents and vertex order along them
    tan = np.cross(xe, nrm)
    along = np.einsum("ij,ij->i", xv[e2v[:, 1]] - xv[e2v[:, 0]], tan)
    e2v_t = np.where((along > 0)[:, None], e2v, e2v[:, ::-1])

    # counter-clockwise cell -> edge order and cell -> vertex order
    def c2v_of(c2e):
        ev = e2v_t[c2e]  # (C, 3, 2)
        return np.stack([_common(ev[:, (i - 1) % 3], ev[:, i]) for i in range(3)], axis=1)

    c2v = c2v_of(c2e_in)
    a, b, c = xv[c2v[:, 0]], xv[c2v[:, 1]], xv[c2v[:, 2]]
    ccw = np.einsum("ij,ij->i", np.cross(b - a, c - a), xc) > 0
    c2e = np.where(ccw[:, None], c2e_in, c2e_in[:, [0, 2, 1]])
    c2v = c2v_of(c2e)
    cells = np.arange(nc)
    c2e2c = np.where(e2c[c2e, 0] == cells[:, None], e2c[c2e, 1], e2c[c2e, 0])
    sgn_c = np.where(e2c[c2e, 0] == cells[:, None], 1, -1)

    # counter-clockwise walk around each vertex: in a counter-clockwise cell
    # (p_i, p_i+1, p_i+2) the edge (p_i, p_i+1) is followed by (p_i, p_i-1)
    nxt_e = np.full((ne, 2), -1, dtype=np.int64)
    nxt_c = np.full((ne, 2), -1, dtype=np.int64)
    for ci in range(3):
        v = c2v[:, ci]
        e_from = c2e[:, ci]
        side = (e2v_t[e_from, 0] != v).astype(np.int64)
        nxt_e[e_from, side] = c2e[:, (ci - 1) % 3]
        nxt_c[e_from, side] = cells
    v2e = np.full((nv, 6), -1, dtype=np.int64)
    v2c = np.full((nv, 6), -1, dtype=np.int64)
    emin = np.full(nv, np.iinfo(np.int64).max)
    np.minimum.at(emin, e2v_t[:, 0], np.arange(ne))
    np.minimum.at(emin, e2v_t[:, 1], np.arange(ne))
    verts = np.arange(nv)
    cur = emin.copy()
    active = np.ones(nv, dtype=bool)
    for i in range(6):
        v2e[active, i] = cur[active]
        side = (e2v_t[cur, 0] != verts).astype(np.int64)
        nx = nxt_e[cur, side]
        v2c[active, i] = nxt_c[cur, side][active]
        active &= nx != emin
        cur = nx
    if active.any():
        raise ValueError("a vertex has more than 6 edges")
    valid = v2e >= 0
    sgn_v = np.where(valid, np.where(e2v_t[np.maximum(v2e, 0), 1] == np.arange(nv)[:, None], 1, -1), 0)

    # edge -> neighbouring edges and rhombus vertices
    e2c2e = np.empty((ne, 4), dtype=np.int64)
    e2c2v = np.empty((ne, 4), dtype=np.int64)
    e2c2v[:, 0:2] = e2v_t
    for side in range(2):
        cc = e2c[:, side]
        ce = c2e[cc]  # (E, 3)
        keep = ce != np.arange(ne)[:, None]
        e2c2e[:, 2 * side:2 * side + 2] = ce[keep].reshape(ne, 2)
        cv = c2v[cc]
        off = (cv != e2v_t[:, 0:1]) & (cv != e2v_t[:, 1:2])
        e2c2v[:, 2 + side] = cv[off]

    i32 = np.int32
    return {
        "e2v": e2v_t.astype(i32),
        "c2e": c2e.astype(i32),
        "c2v": c2v.astype(i32),
        "c2e2c": c2e2c.astype(i32),
        "e2c": e2c.astype(i32),
        "v2e": v2e.astype(i32),
        "v2c": v2c.astype(i32),
        "e2c2e": e2c2e.astype(i32),
        "e2c2v": e2c2v.astype(i32),
        "sgn_c": sgn_c.astype(i32),
        "sgn_v": sgn_v.astype(i32),
        "tangent": tan,
    }


class Grid:
    """Everything the oracle's operators need, in plain arrays."""

    def __init__(self, g, vert, sfc=False):
        if sfc:
            pc, pe, pv = sfc_permutation(g)
            g = renumber(g, pc, pe, pv)
            self.perm = (pc, pe, pv)
        else:
            self.perm = None
        d = derive(g)
        self.raw = g
        self.tables = d
        self.nc, self.ne, self.nv = g["n_cells"], g["n_edges"], g["n_verts"]
        self.radius = g["radius"]
        R = self.radius
        self.e2c = d["e2c"].astype(np.int64)
        self.e2v = d["e2v"].astype(np.int64)
        self.c2e = d["c2e"].astype(np.int64)
        self.c2v = d["c2v"].astype(np.int64)
        self.c2e2c = d["c2e2c"].astype(np.int64)
        self.v2e = d["v2e"].astype(np.int64)
        self.v2c = d["v2c"].astype(np.int64)
        self.e2c2e = d["e2c2e"].astype(np.int64)
        self.e2c2v = d["e2c2v"].astype(np.int64)
        self.sgn_c = d["sgn_c"].astype(np.float64)
        self.sgn_v = d["sgn_v"].astype(np.float64)
        self.xv, self.xe, self.xc = g["vert_xyz"], g["edge_xyz"], g["cell_xyz"]
        self.nrm = g["edge_normal_xyz"]
        self.tan = d["tangent"]
        self.l_e = g["edge_length"]
        self.d_e = g["dual_edge_length"]
        self.a_c = g["cell_area"]
        self.a_v = g["dual_area"]
        self.a_e = 0.5 * self.l_e * self.d_e
        self.mean_area = 4.0 * np.pi * R * R / self.nc
        # vertical column
        self.n_lev = vert["z_half"].size - 1
        self.z_half = vert["z_half"]
        self.z_full = 0.5 * (self.z_half[:-1] + self.z_half[1:])
        self.dz_full = self.z_half[:-1] - self.z_half[1:]
        self.dz_half = np.zeros(self.n_lev + 1)
        self.dz_half[1:-1] = self.z_full[:-1] - self.z_full[1:]
        self.ex_ref = vert["exner_ref_full"]
        self.th_ref = vert["theta_ref_full"]
        self.th_ref_ic = vert["theta_ref_half"]
        self.dex_dz_ref_ic = vert["dexner_dz_ref_half"]

    def permute_state(self, state):
        """Original numbering -> this grid's numbering (identity without SFC)."""
        if self.perm is None:
            return {k: v.copy() for k, v in state.items()}
        pc, pe, _ = self.perm
        return {k: (v[:, pe] if k == "vn" else v[:, pc]).copy() for k, v in state.items()}

    def unpermute_state(self, state):
        if self.perm is None:
            return {k: v.copy() for k, v in state.items()}
        pc, pe, _ = self.perm
        out = {}
        for k, v in state.items():
            p = pe if k == "vn" else pc
            o = np.empty_like(v)
            o[:, p] = v
            out[k] = o
        return out
