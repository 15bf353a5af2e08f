"""Launch tiles through the C ABI: the tuner restores the state it times on,
no result depends on the tiles, and selective profiling records only the
chosen kernel."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2608_21150_amd import dycore as D  # noqa: E402
from synth import build_workload, initial_state, make_grid  # noqa: E402

FIELDS = ("vn", "w", "rho", "exner", "theta_v")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_autotune_restores_state_and_results_do_not_depend_on_tiles(precision):
    g0, S, vert, spec = build_workload("r2b2_k30")
    G = D.Grid(g0, vert)
    a = D.State(G, precision=precision)
    b = D.State(G, precision=precision)
    a.write(S)
    b.write(S)
    a.step(spec["dt"], spec["nsub"])  # parity 1: the tuner must restore it too
    b.step(spec["dt"], spec["nsub"])
    before = a.read()
    t0 = a.tiles()
    a.autotune(spec["dt"], spec["nsub"])
    t1 = a.tiles()
    print("default tiles", t0, "tuned", t1)
    after = a.read()
    for k in FIELDS:
        assert np.array_equal(before[k], after[k]), k
    assert a.current() == b.current()
    for th, kb in t1.values():
        assert th in (64, 128, 256) and 1 <= kb <= 30
    for _ in range(3):
        a.step(spec["dt"], spec["nsub"])
        b.step(spec["dt"], spec["nsub"])
    x, y = a.read(), b.read()
    for k in FIELDS:
        assert np.array_equal(x[k], y[k]), k
    a.close()
    b.close()
    G.close()


def test_profile_select_records_one_kernel():
    g0, S, vert, spec = build_workload("r2b2_k30")
    G = D.Grid(g0, vert)
    st = D.State(G)
    st.write(S)
    st.profile_select(["column_corr"])
    st.profile(True)
    st.step(spec["dt"], spec["nsub"])
    p = st.profile_read()
    assert p["column_corr"][0] == spec["nsub"] and p["column_corr"][1] > 0
    assert all(c == 0 for n, (c, _) in p.items() if n != "column_corr")
    st.profile_select(None)
    st.profile(True)
    st.step(spec["dt"], spec["nsub"])
    p = st.profile_read()
    assert p["edge_pred"][0] == spec["nsub"] and p["diff_edge2"][0] == 1
    with pytest.raises(D.DycoreError):
        st.autotune(-1.0, 2)
    st.close()
    G.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_padding_contents_do_not_matter(precision):
    """Padding entries of the field buffers belong to the library: NaN in all
    of them, in both buffer sets, changes no result."""
    g0 = make_grid(2, 0)  # 80 cells, 120 edges: both strides padded
    S, vert = initial_state(g0, 12, 20.0e3, seed=5, vn_sigma=1.0, jet_u0=20.0)
    spec = {"dt": 300.0, "nsub": 3}
    G = D.Grid(g0, vert)
    a = D.State(G, precision=precision)
    b = D.State(G, precision=precision)
    K = G.info["n_lev"]
    nc, ne = G.info["n_cells"], G.info["n_edges"]
    cs, es = G.info["cell_stride"], G.info["edge_stride"]
    assert cs > nc and es > ne  # the test needs padding
    for bufs in b.bufs:
        for name, t in bufs.items():
            if name == "vn":
                v = t.view(torch.float32 if precision == "mixed" else torch.float64).view(K, es)
                v[:, ne:] = float("nan")
            else:
                rows = K + 1 if name == "w" else K
                t.view(torch.float64).view(rows, cs)[:, nc:] = float("nan")
    a.write(S)
    b.write(S)
    for _ in range(3):
        a.step(spec["dt"], spec["nsub"])
        b.step(spec["dt"], spec["nsub"])
    x, y = a.read(), b.read()
    for name in FIELDS:
        assert np.array_equal(x[name], y[name]), name
    assert b.diag()["n_nonfinite"] == 0
    a.close()
    b.close()
    G.close()
