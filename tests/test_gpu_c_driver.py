"""The plain-C host driver (paper_2608_21150_amd/examples/c_driver.c) runs
the step through the C ABI with its own device allocations and no Python in
the process.  Its results must match the FP64 oracle (relative L2 <= 1e-11
after the ten steps of the R2B2 / 30-level parity case; the mixed form within
1e-4 of it) and equal the Python binding's bit for bit (the same library on
the same inputs)."""
import os
import subprocess

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2608_21150_amd import dycore as D  # noqa: E402
from oracle import dycore as O  # noqa: E402
from oracle.grid import Grid as OGrid  # noqa: E402
from synth import build_workload  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = os.path.join(ROOT, "paper_2608_21150_amd", "examples", "c_driver")
FIELDS = ("vn", "w", "rho", "exner", "theta_v")


def write_input(path, g, vert, S, dt, nsub, steps, precision, sfc):
    C, E, V = g["n_cells"], g["n_edges"], g["n_verts"]
    K = len(vert["z_half"]) - 1
    with open(path, "wb") as f:
        np.array([C, E, V, K, precision == "mixed", int(sfc), nsub, steps], dtype="<i4").tofile(f)
        np.array([g["radius"], dt], dtype="<f8").tofile(f)
        for name in ("e2c", "c2e", "e2v", "c2e2c"):
            np.ascontiguousarray(g[name], dtype="<i4").tofile(f)
        for name in ("vert_xyz", "cell_xyz", "edge_xyz", "edge_length", "dual_edge_length", "cell_area",
                     "dual_area", "edge_normal_xyz"):
            np.ascontiguousarray(g[name], dtype="<f8").tofile(f)
        for name in ("z_half", "exner_ref_full", "theta_ref_full", "theta_ref_half", "dexner_dz_ref_half"):
            np.ascontiguousarray(vert[name], dtype="<f8").tofile(f)
        for name in FIELDS:
            np.ascontiguousarray(S[name], dtype="<f8").tofile(f)


def read_output(path, g, K):
    C, E = g["n_cells"], g["n_edges"]
    a = np.fromfile(path, dtype="<f8")
    shapes = {"vn": (K, E), "w": (K + 1, C), "rho": (K, C), "exner": (K, C), "theta_v": (K, C)}
    out, o = {}, 0
    for name in FIELDS:
        n = int(np.prod(shapes[name]))
        out[name] = a[o:o + n].reshape(shapes[name])
        o += n
    assert a.size == o + 5
    return out, a[o:]


@pytest.fixture(scope="module")
def oracle_r2b2():
    g0, S, vert, spec = build_workload("r2b2_k30")
    og = OGrid(g0, vert)
    ref = S
    for _ in range(spec["steps"]):
        ref = O.step(og, ref, spec["dt"], spec["nsub"])
    return ref


@pytest.mark.parametrize("precision,sfc", [("fp64", False), ("mixed", True)])
def test_c_driver_matches_oracle_and_python_binding(tmp_path, precision, sfc, oracle_r2b2):
    g0, S, vert, spec = build_workload("r2b2_k30")
    K, steps = spec["n_lev"], spec["steps"]
    fin, fout = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    write_input(fin, g0, vert, S, spec["dt"], spec["nsub"], steps, precision, sfc)
    print("running", DRIVER, precision, "sfc" if sfc else "", flush=True)
    r = subprocess.run([DRIVER, fin, fout], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr)
    assert r.returncode == 0
    out, diag = read_output(fout, g0, K)
    tol = 1e-11 if precision == "fp64" else 1e-4
    for name in FIELDS:
        ref = oracle_r2b2[name]
        err = np.linalg.norm(out[name] - ref) / np.linalg.norm(ref)
        print(precision, name, f"rel L2 vs oracle {err:.3e}")
        assert err <= tol, (precision, name, err)
    G = D.Grid(g0, vert, sfc=sfc)
    st = D.State(G, precision=precision)
    st.write(S)
    for _ in range(steps):
        st.step(spec["dt"], spec["nsub"])
    ref = st.read()
    d = st.diag()
    st.close()
    G.close()
    for name in FIELDS:
        assert np.array_equal(out[name], ref[name]), name
    assert diag[0] == d["mass"] and diag[1] == d["theta_mass"] and diag[4] == 0


def test_c_driver_reports_bad_input(tmp_path):
    fin = str(tmp_path / "bad.bin")
    np.array([0, 0, 0, 0, 0, 0, 1, 1], dtype="<i4").tofile(fin)
    np.array([6.371e6, 60.0], dtype="<f8").tofile(open(fin, "ab"))
    r = subprocess.run([DRIVER, fin, str(tmp_path / "o.bin")], capture_output=True, text=True, timeout=60)
    assert r.returncode == 1 and "bad counts" in r.stderr
