"""The host grid layer (validation, canonical tables, space-filling curve,
stencil coefficients, fused-edge tiles, the optional schemes' tables) built
with AddressSanitizer and UndefinedBehaviorSanitizer by the host compiler
(no GPU code), run on valid grids and on every malformed case the
validation must refuse: each valid grid builds, each malformed one returns
DC_EGRID or DC_EINVAL, and no sanitizer reports anything."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from synth import initial_state, make_grid

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2608_21150_amd", "csrc")
DC_OK, DC_EINVAL, DC_EGRID = 0, -1, -2

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


def _write(path, g, vert, sfc=0):
    K = len(vert["z_half"]) - 1
    with open(path, "wb") as f:
        np.array([g["n_cells"], g["n_edges"], g["n_verts"], K, sfc], dtype="<i4").tofile(f)
        np.array([g["radius"]], dtype="<f8").tofile(f)
        for name in ("e2c", "c2e", "e2v", "c2e2c"):
            np.ascontiguousarray(g[name], dtype="<i4").tofile(f)
        for name in ("vert_xyz", "cell_xyz", "edge_xyz", "edge_length", "dual_edge_length", "cell_area",
                     "dual_area", "edge_normal_xyz"):
            np.ascontiguousarray(g[name], dtype="<f8").tofile(f)
        for name in ("z_half", "exner_ref_full", "theta_ref_full", "theta_ref_half", "dexner_dz_ref_half"):
            np.ascontiguousarray(vert[name], dtype="<f8").tofile(f)


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    d = tmp_path_factory.mktemp("san")
    exe = str(d / "grid_harness")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(ROOT, "tests", "sanitize", "grid_harness.cpp"), os.path.join(CSRC, "grid.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe, d


def _run(exe, files):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe, *files], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    out = {}
    for line in r.stdout.strip().splitlines():
        name, rc, rbf, tiles = line.split()
        out[os.path.basename(name)] = (int(rc), int(rbf), int(tiles))
    return out


def test_valid_grids_build_clean(harness):
    exe, d = harness
    files = []
    for (n, k), K, sfc in (((1, 0), 1, 0), ((2, 0), 3, 1), ((2, 2), 30, 0), ((2, 3), 12, 1), ((2, 4), 5, 1)):
        g = make_grid(n, k)
        _, vert = initial_state(g, K, 20e3, seed=0)
        p = str(d / f"ok_{n}_{k}_{sfc}.bin")
        _write(p, g, vert, sfc)
        files.append(p)
    out = _run(exe, files)
    assert len(out) == len(files)
    for name, (rc, rbf, tiles) in out.items():
        assert rc == DC_OK and rbf == 1 and tiles == 1, (name, rc, rbf, tiles)


def test_malformed_grids_are_refused_clean(harness):
    exe, d = harness
    g = make_grid(2, 1)
    _, vert = initial_state(g, 4, 10e3, seed=0)
    cases = {}

    def case(name, gm=None, vm=None, **mod):
        h = dict(g)
        h.update(mod)
        cases[name] = (h if gm is None else gm, vert if vm is None else vm)

    e2c = g["e2c"].copy(); e2c[5, 0] = g["n_cells"]
    case("e2c_out_of_range", e2c=e2c)
    e2c = g["e2c"].copy(); e2c[5, 0] = -1
    case("e2c_negative", e2c=e2c)
    e2c = g["e2c"].copy(); e2c[5, 1] = e2c[5, 0]
    case("e2c_degenerate", e2c=e2c)
    c2e = g["c2e"].copy(); c2e[2, 1] = g["n_edges"] + 7
    case("c2e_out_of_range", c2e=c2e)
    e2v = g["e2v"].copy(); e2v[9, 1] = g["n_verts"]
    case("e2v_out_of_range", e2v=e2v)
    c2e2c = g["c2e2c"].copy(); c2e2c[3, 0] = (c2e2c[3, 0] + 1) % g["n_cells"]
    case("c2e2c_inconsistent", c2e2c=c2e2c)
    area = g["cell_area"].copy(); area[7] = 0.0
    case("zero_area", cell_area=area)
    length = g["edge_length"].copy(); length[4] = np.nan
    case("nan_length", edge_length=length)
    nrm = g["edge_normal_xyz"].copy(); nrm[11] *= -1
    case("flipped_normal", edge_normal_xyz=nrm)
    xc = g["cell_xyz"].copy(); xc[4, 1] = np.inf
    case("inf_cell_position", cell_xyz=xc)
    case("extra_vertex", n_verts=g["n_verts"] + 1, vert_xyz=np.vstack([g["vert_xyz"], [[0, 0, 1]]]),
         dual_area=np.append(g["dual_area"], 1.0))
    v = dict(vert); zh = vert["z_half"].copy(); zh[1] = zh[0] + 1; v["z_half"] = zh
    case("z_not_decreasing", vm=v)
    _, v130 = initial_state(g, 130, 60e3, seed=0)
    case("too_many_levels", vm=v130)
    files = []
    for name, (gm, vm) in cases.items():
        p = str(d / f"bad_{name}.bin")
        _write(p, gm, vm)
        files.append(p)
    out = _run(exe, files)
    for name in cases:
        rc = out[f"bad_{name}.bin"][0]
        assert rc in (DC_EGRID, DC_EINVAL), (name, rc)
