"""Pins of the grid generator and the oracle's derived tables (CPU).

Closed forms: RnBk counts, Euler characteristic, areas tiling the sphere,
primal/dual orthogonality; brute force: neighbour sets recomputed by plain
loops on small grids; geometry checks of the canonical orientations.
"""
import numpy as np
import pytest

from synth import expected_counts
from oracle.grid import derive, morton_key, renumber, sfc_permutation

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


def test_morton_key_brute_force():
    rng = np.random.default_rng(3)
    x = rng.normal(size=(50, 3))
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    keys = morton_key(x)
    for row, key in zip(x, keys):
        q = [int(np.floor((u + 1.0) * 0.5 * 2097151.0)) for u in row]
        want = 0
        for bit in range(21):
            for axis, shift in ((0, 2), (1, 1), (2, 0)):
                want |= ((q[axis] >> bit) & 1) << (3 * bit + shift)
        assert int(key) == want
        assert want < 2**63


@pytest.mark.parametrize("n,k", [(2, 1), (2, 2)])
def test_sfc_renumbering(grids, n, k):
    g = grids(n, k)
    pc, pe, pv = sfc_permutation(g)
    for p, m in ((pc, g["n_cells"]), (pe, g["n_edges"]), (pv, g["n_verts"])):
        assert np.array_equal(np.sort(p), np.arange(m))
    keys = morton_key(g["cell_xyz"][pc])
    assert (np.diff(keys.astype(np.float64)) >= 0).all()
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
