"""Icosahedral RnBk grid generator (seeded-input side, shared by oracle and GPU path).

Builds the triangular grid described in the paper's Results section
("Experimental setup"): the 20 faces of an icosahedron are root-divided into
n^2 triangles (Sadourny), then every triangle is bisected k times into four.
Only n in {1, 2} is supported; for n = 2 the root division is one midpoint
split of every icosahedron edge.  Every new point is the great-circle midpoint
normalize(a + b), projected at every level.

The output is the *input* of ``dc_grid_create``: the four given connectivity
tables (e2c, c2e, e2v, c2e2c) and the geometry (positions, primal and dual
edge lengths, primal and dual areas, edge normals).  Nothing of the dynamical
core's arithmetic lives here; derived tables (v2e, v2c, e2c2e, e2c2v,
orientation) are computed independently by the oracle and by the library.

Conventions of the generated tables (the library re-derives canonical forms
and must not rely on them beyond what its validation checks):
  * cells are numbered in quadtree order (children of triangle t are 4t..4t+3);
  * c2v (internal) is counter-clockwise seen from outside;
    c2e[c][i] joins c2v[c][i] and c2v[c][(i+1)%3]; c2e2c[c][i] is across c2e[c][i];
  * edges are numbered by first appearance in the scan (c, i), c = 0.. C-1;
    e2c[e] = (first cell, second cell); the normal points e2c[e][0] -> e2c[e][1];
  * e2v[e] = (min vertex id, max vertex id)  (NOT ordered along the tangent);
  * vertices are numbered by first appearance in the c2v scan.
"""
from __future__ import annotations

import numpy as np

EARTH_RADIUS = 6.371e6  # m


def _normalize(x):
    return x / np.linalg.norm(x, axis=-1, keepdims=True)


def _icosahedron():
    """12 unit vertices (two at the poles) and 20 faces, counter-clockwise seen from outside."""
    lat = np.arctan(0.5)
    pts = [np.array([0.0, 0.0, 1.0])]
    for i in range(5):
        lon = 2.0 * np.pi * i / 5.0
        pts.append(np.array([np.cos(lat) * np.cos(lon), np.cos(lat) * np.sin(lon), np.sin(lat)]))
    for i in range(5):
        lon = 2.0 * np.pi * (i + 0.5) / 5.0
        pts.append(np.array([np.cos(lat) * np.cos(lon), np.cos(lat) * np.sin(lon), -np.sin(lat)]))
    pts.append(np.array([0.0, 0.0, -1.0]))
    x = _normalize(np.array(pts))
    U = [1 + i for i in range(5)]
    L = [6 + i for i in range(5)]
    faces = []
    for i in range(5):
        j = (i + 1) % 5
        faces.append((0, U[i], U[j]))
        faces.append((U[i], L[i], U[j]))
        faces.append((U[j], L[i], L[j]))
        faces.append((11, L[j], L[i]))
    faces = np.array(faces, dtype=np.int64)
    # orient counter-clockwise seen from outside
    a, b, c = x[faces[:, 0]], x[faces[:, 1]], x[faces[:, 2]]
    s = np.einsum("ij,ij->i", np.cross(b - a, c - a), a + b + c)
    flip = s < 0
    faces[flip] = faces[flip][:, [0, 2, 1]]
    return x, faces


def _bisect(x, tri):
    """One bisection: every triangle (a, b, c) -> (a,ab,ca), (ab,b,bc), (ca,bc,c), (ab,bc,ca)."""
    nv = x.shape[0]
    a, b, c = tri[:, 0], tri[:, 1], tri[:, 2]
    pairs = np.stack([np.stack([a, b], 1), np.stack([b, c], 1), np.stack([c, a], 1)], 1)  # (T,3,2)
    lo = pairs.min(axis=2)
    hi = pairs.max(axis=2)
    key = (lo * nv + hi).ravel()
    ukey, inv = np.unique(key, return_inverse=True)
    mid = _normalize(x[ukey // nv] + x[ukey % nv])
    mid_id = (nv + inv).reshape(-1, 3)  # midpoint of (a,b), (b,c), (c,a)
    ab, bc, ca = mid_id[:, 0], mid_id[:, 1], mid_id[:, 2]
    children = np.stack(
        [
            np.stack([a, ab, ca], 1),
            np.stack([ab, b, bc], 1),
            np.stack([ca, bc, c], 1),
            np.stack([ab, bc, ca], 1),
        ],
        1,
    ).reshape(-1, 3)
    return np.concatenate([x, mid], 0), children


def _sph_tri_area(a, b, c):
    """Spherical excess of unit-vector triangles (Van Oosterom-Strackee)."""
    num = np.abs(np.einsum("ij,ij->i", a, np.cross(b, c)))
    den = 1.0 + np.einsum("ij,ij->i", a, b) + np.einsum("ij,ij->i", b, c) + np.einsum("ij,ij->i", c, a)
    return 2.0 * np.arctan2(num, den)


def _arc(a, b):
    return np.arctan2(np.linalg.norm(np.cross(a, b), axis=1), np.einsum("ij,ij->i", a, b))


def make_grid(n: int, k: int, radius: float = EARTH_RADIUS):
    """Return a dict with the RnBk grid tables (int32) and geometry (float64)."""
    if n not in (1, 2):
        raise ValueError("only root divisions n = 1 and n = 2 are supported")
    if k < 0:
        raise ValueError("k must be >= 0")
    x, tri = _icosahedron()
    for _ in range((1 if n == 2 else 0) + k):
        x, tri = _bisect(x, tri)

    # renumber vertices by first appearance in the c2v scan
    order = np.unique(tri.ravel(), return_index=True)[1]
    first = np.full(x.shape[0], -1, dtype=np.int64)
    first[tri.ravel()[np.sort(order)]] = np.arange(order.size)
    # tri.ravel()[np.sort(order)] lists vertices in first-appearance order
    c2v = first[tri]
    xv = np.empty_like(x)
    xv[first] = x
    nc = c2v.shape[0]
    nv = xv.shape[0]

    # edges by first appearance in the (c, i) scan; c2e[c][i] joins c2v[i], c2v[i+1]
    p = c2v
    q = np.roll(c2v, -1, axis=1)
    lo = np.minimum(p, q).ravel()
    hi = np.maximum(p, q).ravel()
    key = lo * nv + hi
    ukey, first_idx, inv = np.unique(key, return_index=True, return_inverse=True)
    rank = np.empty(ukey.size, dtype=np.int64)
    rank[np.argsort(first_idx, kind="stable")] = np.arange(ukey.size)
    c2e = rank[inv].reshape(nc, 3)
    ne = ukey.size
    e2v = np.empty((ne, 2), dtype=np.int64)
    e2v[rank, 0] = ukey // nv
    e2v[rank, 1] = ukey % nv

    # e2c: first and second cell seen in the scan
    slot_cell = np.repeat(np.arange(nc), 3)
    flat_e = c2e.ravel()
    srt = np.argsort(flat_e, kind="stable")
    cells_sorted = slot_cell[srt].reshape(ne, 2)
    e2c = cells_sorted  # stable sort keeps scan order: first seen, then second
    # c2e2c: the cell across each edge
    other = np.where(e2c[c2e, 0] == np.arange(nc)[:, None], e2c[c2e, 1], e2c[c2e, 0])
    c2e2c = other

    # geometry (unit vectors, then metric scaling by radius)
    a, b, c = xv[c2v[:, 0]], xv[c2v[:, 1]], xv[c2v[:, 2]]
    cc = _normalize(np.cross(b - a, c - a))
    sgn = np.sign(np.einsum("ij,ij->i", cc, a + b + c))
    xc = cc * sgn[:, None]
    xe = _normalize(xv[e2v[:, 0]] + xv[e2v[:, 1]])
    l_e = radius * _arc(xv[e2v[:, 0]], xv[e2v[:, 1]])
    d_e = radius * _arc(xc[e2c[:, 0]], xc[e2c[:, 1]])
    area_c = radius**2 * _sph_tri_area(a, b, c)
    # dual area: fan from the vertex over each dual edge (c0(e), c1(e)) of its edges
    ve = np.concatenate([e2v[:, 0], e2v[:, 1]])
    ee = np.concatenate([np.arange(ne), np.arange(ne)])
    tri_a = radius**2 * _sph_tri_area(xv[ve], xc[e2c[ee, 0]], xc[e2c[ee, 1]])
    area_v = np.bincount(ve, weights=tri_a, minlength=nv)
    nrm = _normalize(np.cross(xv[e2v[:, 0]], xv[e2v[:, 1]]))
    s = np.sign(np.einsum("ij,ij->i", nrm, xc[e2c[:, 1]] - xc[e2c[:, 0]]))
    nrm = nrm * s[:, None]

    i32 = np.int32
    return {
        "n": n,
        "k": k,
        "radius": float(radius),
        "n_cells": nc,
        "n_edges": ne,
        "n_verts": nv,
        "e2c": e2c.astype(i32),
        "c2e": c2e.astype(i32),
        "e2v": e2v.astype(i32),
        "c2e2c": c2e2c.astype(i32),
        "vert_xyz": xv,
        "cell_xyz": xc,
        "edge_xyz": xe,
        "edge_length": l_e,
        "dual_edge_length": d_e,
        "cell_area": area_c,
        "dual_area": area_v,
        "edge_normal_xyz": nrm,
    }


def expected_counts(n: int, k: int):
    """Closed-form entity counts of RnBk: C = 20 n^2 4^k, E = 30 n^2 4^k, V = 10 n^2 4^k + 2."""
    f = n * n * 4**k
    return 20 * f, 30 * f, 10 * f + 2
