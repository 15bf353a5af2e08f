"""Pins of the grid generator and the oracle's derived tables (CPU).

Closed forms: RnBk counts, Euler characteristic, areas tiling the sphere,
primal/dual orthogonality; brute force: neighbour sets recomputed by plain
loops on small grids; geometry checks of the canonical orientations.
"""
import numpy as np
import pytest

from synth import expected_counts
from oracle.grid import TREE_LEVELS, _ico, derive, renumber, sfc_permutation, tree_key

SMALL = [(1, 0), (2, 0), (2, 1), (2, 2)]


@pytest.mark.parametrize("n,k", SMALL + [(2, 3)])
def test_counts_and_euler(grids, n, k):
    g = grids(n, k)
    C, E, V = expected_counts(n, k)
    assert (g["n_cells"], g["n_edges"], g["n_verts"]) == (C, E, V)
    assert V - E + C == 2
    assert {(1, 0): (20, 30, 12), (2, 0): (80, 120, 42), (2, 1): (320, 480, 162),
            (2, 2): (1280, 1920, 642), (2, 3): (5120, 7680, 2562)}[(n, k)] == (C, E, V)


@pytest.mark.parametrize("n,k", SMALL)
def test_areas_tile_sphere(grids, n, k):
    g = grids(n, k)
    s = 4 * np.pi * g["radius"] ** 2
    assert abs(g["cell_area"].sum() / s - 1) < 1e-13
    assert abs(g["dual_area"].sum() / s - 1) < 1e-13
    assert (g["cell_area"] > 0).all() and (g["dual_area"] > 0).all()
    assert (g["edge_length"] > 0).all() and (g["dual_edge_length"] > 0).all()


@pytest.mark.parametrize("n,k", SMALL)
def test_orthogonality_and_normals(grids, n, k):
    g = grids(n, k)
    d = derive(g)
    xc, xv = g["cell_xyz"], g["vert_xyz"]
    e2c = g["e2c"]
    t = d["tangent"]
    chord = xc[e2c[:, 1]] - xc[e2c[:, 0]]
    dn = np.linalg.norm(chord, axis=1)
    assert np.max(np.abs(np.einsum("ij,ij->i", t, chord)) / dn) < 1e-12
    assert (np.einsum("ij,ij->i", g["edge_normal_xyz"], chord) > 0).all()
    ev = d["e2v"]
    assert (np.einsum("ij,ij->i", xv[ev[:, 1]] - xv[ev[:, 0]], t) > 0).all()
    # (n, t, r) right-handed
    assert np.allclose(np.cross(g["edge_normal_xyz"], t), g["edge_xyz"], atol=1e-14)


@pytest.mark.parametrize("n,k", SMALL)
def test_connectivity_brute_force(grids, n, k):
    g = grids(n, k)
    d = derive(g)
    nc, ne, nv = g["n_cells"], g["n_edges"], g["n_verts"]
    c2e, e2c, c2e2c, e2v = d["c2e"], d["e2c"], d["c2e2c"], d["e2v"]
    # every edge has two distinct cells, and each lists it
    cells_of_edge = [[] for _ in range(ne)]
    for c in range(nc):
        for e in c2e[c]:
            cells_of_edge[e].append(c)
    for e in range(ne):
        assert sorted(cells_of_edge[e]) == sorted(e2c[e].tolist())
        assert e2c[e, 0] != e2c[e, 1] and e2v[e, 0] != e2v[e, 1]
    # c2e2c symmetric
    for c in range(nc):
        for i in range(3):
            o = c2e2c[c, i]
            assert c in c2e2c[o]
            assert c2e[c, i] in c2e[o]
    # vertex incidence: 12 pentagons, the rest hexagons; v2e/v2c consistent
    v2e, v2c = d["v2e"], d["v2c"]
    inc = [set() for _ in range(nv)]
    for e in range(ne):
        for v in e2v[e]:
            inc[v].add(e)
    npent = 0
    for v in range(nv):
        ev = [e for e in v2e[v] if e >= 0]
        assert set(ev) == inc[v]
        assert ev[0] == min(inc[v])
        npent += len(ev) == 5
        m = len(ev)
        for i in range(m):
            c = v2c[v, i]
            assert ev[i] in c2e[c] and ev[(i + 1) % m] in c2e[c]
    assert npent == 12
    # e2c2e / e2c2v
    for e in range(ne):
        c0, c1 = e2c[e]
        want = [x for x in c2e[c0] if x != e] + [x for x in c2e[c1] if x != e]
        assert d["e2c2e"][e].tolist() == want
        r = d["e2c2v"][e]
        assert r[0] == e2v[e, 0] and r[1] == e2v[e, 1]
        assert r[2] in d["c2v"][c0] and r[2] not in e2v[e]
        assert r[3] in d["c2v"][c1] and r[3] not in e2v[e]


@pytest.mark.parametrize("n,k", SMALL)
def test_counter_clockwise_orders(grids, n, k):
    """Geometric check (independent of the combinatorial walk): orders turn counter-clockwise."""
    g = grids(n, k)
    d = derive(g)
    xv, xe = g["vert_xyz"], g["edge_xyz"]
    c2v = d["c2v"]
    a, b, c = xv[c2v[:, 0]], xv[c2v[:, 1]], xv[c2v[:, 2]]
    assert (np.einsum("ij,ij->i", np.cross(b - a, c - a), a + b + c) > 0).all()
    for i in range(3):  # c2e[i] joins c2v[i] and c2v[i+1]
        ev = d["e2v"][d["c2e"][:, i]]
        pair = np.sort(np.stack([c2v[:, i], c2v[:, (i + 1) % 3]], 1), axis=1)
        assert (np.sort(ev, axis=1) == pair).all()
    for v in range(g["n_verts"]):
        ev = [e for e in d["v2e"][v] if e >= 0]
        dirs = xe[ev] - xv[v]
        dirs = dirs - np.outer(dirs @ xv[v], xv[v])  # tangent-plane projection
        m = len(ev)
        total = 0.0
        for i in range(m):
            cr = np.dot(np.cross(dirs[i], dirs[(i + 1) % m]), xv[v])
            assert cr > 0
            total += np.arctan2(cr, np.dot(dirs[i], dirs[(i + 1) % m]))
        assert abs(total - 2 * np.pi) < 1e-6


def test_tree_icosahedron_is_regular():
    """The key's icosahedron: 12 unit vertices with the poles on the z axis
    and the rings at latitude +-atan(1/2), longitudes 72 i and 72 i + 36
    degrees; 30 edges of one length (the central angle atan 2), each shared
    by two faces; all 20 faces counter-clockwise seen from outside."""
    v, faces = _ico()
    assert np.allclose(np.linalg.norm(v, axis=1), 1.0, atol=1e-15)
    assert np.allclose(v[0], [0, 0, 1]) and np.allclose(v[11], [0, 0, -1])
    lon = np.degrees(np.arctan2(v[1:11, 1], v[1:11, 0])) % 360.0
    assert np.allclose(lon[:5], [0, 72, 144, 216, 288]) and np.allclose(lon[5:], [36, 108, 180, 252, 324])
    assert np.allclose(np.abs(np.arcsin(v[1:11, 2])), np.arctan(0.5))
    edges = {}
    for f in faces:
        a, b, c = v[f]
        assert np.dot(np.cross(b - a, c - a), a + b + c) > 0
        for i in range(3):
            e = tuple(sorted((f[i], f[(i + 1) % 3])))
            edges[e] = edges.get(e, 0) + 1
    assert len(edges) == 30 and set(edges.values()) == {2}
    ang = [np.arccos(np.clip(np.dot(v[i], v[j]), -1, 1)) for i, j in edges]
    assert np.allclose(ang, np.arctan(2.0))


def _leaves(depth):
    """Brute force: every triangle of the subdivided icosahedron `depth`
    levels down, as (centroid direction, face, child digits), built by plain
    recursion over explicit triangles."""
    v, faces = _ico()
    out = []

    def rec(a, b, c, face, digits, d):
        if d == 0:
            g = a + b + c
            out.append((g / np.linalg.norm(g), face, digits))
            return
        m = lambda p, q: (p + q) / np.linalg.norm(p + q)
        ab, bc, ca = m(a, b), m(b, c), m(c, a)
        for i, (x, y, z) in enumerate(((a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca))):
            rec(x, y, z, face, digits + [i], d - 1)

    for f, (i, j, k) in enumerate(faces):
        rec(v[i], v[j], v[k], f, [], depth)
    return out


def test_tree_key_against_explicit_subdivision():
    """The key of each leaf triangle's centroid, three levels down, starts
    with that leaf's face and child digits; every face centroid stays in the
    middle child at all levels (the middle child of an equilateral spherical
    triangle shares its centre), so its digits are all 3."""
    leaves = _leaves(3)
    keys = tree_key(np.array([x for x, _, _ in leaves]))
    shift = 2 * (TREE_LEVELS - 3)
    for key, (_, f, d) in zip(keys.tolist(), leaves):
        assert key >> shift == ((f * 4 + d[0]) * 4 + d[1]) * 4 + d[2]
    v, faces = _ico()
    cen = v[faces].sum(axis=1)
    assert (tree_key(cen) == np.arange(20) * 4**TREE_LEVELS + (4**TREE_LEVELS - 1)).all()
    # positive scaling of x does not change the key
    assert (tree_key(7.0 * cen) == tree_key(cen)).all()


def test_sfc_blocks_are_compact(grids):
    """Runs of 64 = 4^3 consecutive cells in the curve's order are connected
    patches of the mesh (over c2e2c), as the locality of neighbour gathers
    needs."""
    g = grids(2, 3)
    pc, _, _ = sfc_permutation(g)
    oc = np.empty_like(pc)
    oc[pc] = np.arange(pc.size)
    nb = oc[g["c2e2c"]]
    for b0 in range(0, pc.size, 64):
        members = set(range(b0, b0 + 64))
        seen, stack = {b0}, [b0]
        while stack:
            c = stack.pop()
            for n in nb[pc[c]]:
                if n in members and n not in seen:
                    seen.add(int(n))
                    stack.append(int(n))
        assert len(seen) == 64, b0


@pytest.mark.parametrize("n,k", [(2, 1), (2, 2)])
def test_sfc_renumbering(grids, n, k):
    g = grids(n, k)
    pc, pe, pv = sfc_permutation(g)
    for p, m in ((pc, g["n_cells"]), (pe, g["n_edges"]), (pv, g["n_verts"])):
        assert np.array_equal(np.sort(p), np.arange(m))
    keys = tree_key(g["cell_xyz"][pc])
    assert (np.diff(keys) >= 0).all()
    h = renumber(g, pc, pe, pv)
    d = derive(h)  # renumbered grid is still a consistent grid
    assert abs(h["cell_area"].sum() - g["cell_area"].sum()) / g["cell_area"].sum() < 1e-13
    ec = d["e2c"]
    lo = np.minimum(ec[:, 0], ec[:, 1]).astype(np.int64)
    assert (np.diff(lo) >= 0).all()
    # same edges (as cell pairs) before and after
    oc = np.argsort(pc)
    before = {tuple(sorted(oc[c] for c in row)) for row in g["e2c"]}
    after = {tuple(sorted(row)) for row in d["e2c"].tolist()}
    assert before == after
