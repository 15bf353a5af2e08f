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
from synth import build_workload  # noqa: E402

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
