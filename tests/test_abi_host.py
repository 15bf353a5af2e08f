"""Host-side tests of the C-ABI library (no GPU): load, exported symbols,
bit-exact derived tables and permutations against the oracle, validation
errors without side effects."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle.grid import derive, renumber, sfc_permutation
from synth import make_grid, initial_state

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

D = pytest.importorskip("paper_2608_21150_amd.dycore", reason="libdycore.so not built")

TABLES = ["e2c", "c2e", "e2v", "c2e2c", "c2v", "v2e", "v2c", "e2c2e", "e2c2v"]


def test_every_declared_symbol_is_exported():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            names |= set(re.findall(r"^\s*(?:dc_status|const char \*|dc_status)\s*(dc_\w+)\s*\(", txt, re.M))
            names |= set(re.findall(r"\b(dc_\w+)\s*\(", txt)) - {"dc_grid_desc", "dc_params"}
    assert len(names) >= 18
    lib = ctypes.CDLL(D.LIB_PATH)
    for n in sorted(names):
        assert hasattr(lib, n), n


def test_c_driver_is_built_and_checks_its_arguments():
    """The plain-C host driver links the library; without arguments it prints
    its usage and touches no GPU."""
    import subprocess

    drv = os.path.join(ROOT, "paper_2608_21150_amd", "examples", "c_driver")
    assert os.access(drv, os.X_OK), "build() builds the C driver"
    r = subprocess.run([drv], capture_output=True, text=True, timeout=60)
    assert r.returncode == 2 and "usage: c_driver IN OUT" in r.stderr


@pytest.mark.parametrize("n,k,sfc", [(1, 0, False), (2, 0, False), (2, 1, True), (2, 2, False), (2, 3, True)])
def test_tables_bit_exact(grids, n, k, sfc):
    g = grids(n, k)
    _, vert = initial_state(g, 3, 10e3, seed=0)
    G = D.Grid(g, vert, sfc=sfc)
    if sfc:
        pc, pe, pv = sfc_permutation(g)
        ref = derive(renumber(g, pc, pe, pv))
        assert np.array_equal(G.table("perm_cell"), pc)
        assert np.array_equal(G.table("perm_edge"), pe)
        assert np.array_equal(G.table("perm_vert"), pv)
    else:
        ref = derive(g)
        assert np.array_equal(G.table("perm_cell"), np.arange(g["n_cells"]))
    for t in TABLES:
        assert np.array_equal(G.table(t), ref[t]), t
    info = G.info
    assert info["cell_stride"] % 64 == 0 and info["cell_stride"] >= g["n_cells"]
    G.close()


def test_input_orders_are_canonicalised(grids):
    """Shuffled c2e/c2e2c slot orders and swapped e2v give the same canonical tables."""
    g = dict(grids(2, 1))
    _, vert = initial_state(g, 2, 10e3, seed=0)
    ref = derive(g)
    rng = np.random.default_rng(0)
    h = dict(g)
    h["c2e"] = np.array([row[rng.permutation(3)] for row in g["c2e"]], dtype=np.int32)
    h["c2e2c"] = np.array([row[rng.permutation(3)] for row in g["c2e2c"]], dtype=np.int32)
    h["e2v"] = g["e2v"][:, ::-1].copy()
    G = D.Grid(h, vert)
    ref2 = derive(h)
    for t in ("e2v", "c2v", "v2e", "v2c", "e2c2v"):
        assert np.array_equal(G.table(t), ref2[t]), t
        assert np.array_equal(G.table(t), ref[t]) or t in ("c2v",), t  # e2v/v2e independent of input order
    for t in ("c2e", "c2e2c", "e2c2e"):
        assert np.array_equal(G.table(t), ref2[t]), t


def _expect(code, fn):
    with pytest.raises(D.DycoreError) as ei:
        fn()
    assert ei.value.code == code, str(ei.value)


def test_validation_errors(grids):
    g = grids(2, 1)
    _, vert = initial_state(g, 2, 10e3, seed=0)

    def bad(**mod):
        h = dict(g)
        h.update(mod)
        return lambda: D.Grid(h, vert)

    e2c = g["e2c"].copy()
    e2c[5, 0] = g["n_cells"]
    _expect(D.DC_EGRID, bad(e2c=e2c))
    e2c = g["e2c"].copy()
    e2c[5, 1] = e2c[5, 0]
    _expect(D.DC_EGRID, bad(e2c=e2c))
    c2e2c = g["c2e2c"].copy()
    c2e2c[3, 0] = (c2e2c[3, 0] + 1) % g["n_cells"]
    _expect(D.DC_EGRID, bad(c2e2c=c2e2c))
    area = g["cell_area"].copy()
    area[7] = 0.0
    _expect(D.DC_EGRID, bad(cell_area=area))
    nrm = g["edge_normal_xyz"].copy()
    nrm[11] *= -1
    _expect(D.DC_EGRID, bad(edge_normal_xyz=nrm))
    v = dict(vert)
    zh = vert["z_half"].copy()
    zh[1] = zh[0] + 1
    v["z_half"] = zh
    _expect(D.DC_EGRID, lambda: D.Grid(g, v))
    _expect(D.DC_EGRID, bad(n_verts=g["n_verts"] + 1,
                            vert_xyz=np.vstack([g["vert_xyz"], [[0, 0, 1]]]),
                            dual_area=np.append(g["dual_area"], 1.0)))
    # the column solver's depth limit: 129 levels accepted, 130 refused
    _, v129 = initial_state(g, 129, 60e3, seed=0)
    D.Grid(g, v129).close()
    _, v130 = initial_state(g, 130, 60e3, seed=0)
    _expect(D.DC_EINVAL, lambda: D.Grid(g, v130))
    xc = g["cell_xyz"].copy()
    xc[4, 1] = np.nan
    _expect(D.DC_EGRID, bad(cell_xyz=xc))
    # NULL description and NULL output
    assert D.lib.dc_grid_create(None, None) == D.DC_EINVAL
    assert D.lib.dc_params_default(None) == D.DC_EINVAL


def test_params_defaults():
    p = D.default_params()
    from oracle.constants import default_params
    q = default_params()
    for k in ("eta", "adv_w0", "adv_w1", "divdamp_c4", "rayleigh_tau0", "rayleigh_zfrac", "smag_cs", "smag_cap",
              "hdiff_k4", "rd", "cpd", "cvd", "omega", "diffuse_w", "diffuse_theta", "theta_enh_nlev",
              "theta_enh_thresh", "miura", "vt_rbf"):
        assert getattr(p, k) == q[k], k
    # the last member sits where the C struct has it: the binding's layout matches
    assert ctypes.sizeof(D.Params) == 13 * 8 + 4 * 4 + 8 + 2 * 4


def test_sizes_and_workspace(grids):
    g = grids(2, 2)
    _, vert = initial_state(g, 30, 30e3, seed=0)
    G = D.Grid(g, vert)
    nb = ctypes.c_size_t()
    D.check(D.lib.dc_field_bytes(G.handle, 0, 0, ctypes.byref(nb)))
    assert nb.value == 30 * G.info["edge_stride"] * 8
    D.check(D.lib.dc_field_bytes(G.handle, 1, 0, ctypes.byref(nb)))
    assert nb.value == 30 * G.info["edge_stride"] * 4
    D.check(D.lib.dc_field_bytes(G.handle, 0, 1, ctypes.byref(nb)))
    assert nb.value == 31 * G.info["cell_stride"] * 8
    assert D.lib.dc_field_bytes(G.handle, 0, 9, ctypes.byref(nb)) == D.DC_EINVAL
    assert D.lib.dc_state_workspace_bytes(G.handle, 7, 0, ctypes.byref(nb)) == D.DC_EINVAL
    D.check(D.lib.dc_state_workspace_bytes(G.handle, 0, 0, ctypes.byref(nb)))
    assert nb.value > 0
    # state creation rejects NULL / misaligned buffers before touching the GPU
    f = D.Fields(0, 0, 0, 0, 0)
    h = ctypes.c_void_p()
    assert D.lib.dc_state_create(G.handle, ctypes.byref(D.default_params()), 0, 0, f, f, None, 0, None,
                                 ctypes.byref(h)) == D.DC_EINVAL
    G.close()
