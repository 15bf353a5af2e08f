"""The R2B8 / 90-level workload at its full size (5,242,880 cells, one GPU's
share of a production grid), curve-ordered as the benchmark runs it: the
oracle cannot step a grid this size, so the checks are properties that hold
at any size.  Two steps of dt 30 s with 5 substeps from the jet state, in the
mixed form (the benchmark's) and in FP64: total mass conserved to round-off,
no non-finite value, theta-mass conserved to round-off, and mixed within
1e-4 relative L2 of FP64 on vn, rho, exner and theta_v (the bound asserted
on R2B5 after 10 steps); w, still tiny after 60 s, within its stated 5e-3.
The step's parts at the same size: the area-weighted sum of the
predictor's div vn* vanishes on the closed sphere at every level (each
edge's flux leaves one cell and enters the other), w* keeps its boundary
rows at zero, and predictor then corrector equals one substep (equal
fixed-order diagnostics)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2608_21150_amd import dycore as D  # noqa: E402
from synth import WORKLOADS, initial_state, make_grid  # noqa: E402


def rel_l2(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.timeout(600)
def test_r2b8_full_size_invariants():
    spec = WORKLOADS["r2b8_k90"]
    g0 = make_grid(spec["n"], spec["k"])
    S, vert = initial_state(g0, spec["n_lev"], spec["z_top"], **spec["state"])
    G = D.Grid(g0, vert, sfc=True)
    out = {}
    for prec in ("mixed", "fp64"):
        st = D.State(G, precision=prec)
        st.write(S)
        d0 = st.diag()
        for _ in range(2):
            st.step(spec["dt"], spec["nsub"])
        d1 = st.diag()
        assert d1["n_nonfinite"] == 0, prec
        assert abs(d1["mass"] / d0["mass"] - 1) <= 1e-13, (prec, d1["mass"] / d0["mass"] - 1)
        assert abs(d1["theta_mass"] / d0["theta_mass"] - 1) <= 1e-13, (prec, d1["theta_mass"] / d0["theta_mass"] - 1)
        out[prec] = st.read()
        st.close()
    G.close()
    errs = {k: rel_l2(out["mixed"][k], out["fp64"][k]) for k in ("vn", "w", "rho", "exner", "theta_v")}
    print("R2B8 mixed vs FP64 after 2 steps:", errs)
    for k, e in errs.items():
        if k != "w":
            assert e <= 1e-4, (k, e)
    # w is a few mm/s this early in the balanced jet, and the FP32 storage
    # of vn alone sets an absolute floor on its error (the divergence of vn's
    # rounding): its relative error is stated separately (2.5e-3 measured)
    assert errs["w"] <= 5e-3, errs["w"]


@pytest.mark.timeout(600)
def test_r2b8_full_size_parts():
    spec = WORKLOADS["r2b8_k90"]
    g0 = make_grid(spec["n"], spec["k"])
    S, vert = initial_state(g0, spec["n_lev"], spec["z_top"], **spec["state"])
    K = spec["n_lev"]
    dtau = spec["dt"] / spec["nsub"]
    G = D.Grid(g0, vert, sfc=True)
    a = D.State(G, diffusion="none")
    a.write(S)
    m0 = a.diag()["mass"]
    a.part("predictor", dtau, 1)
    div = a.read_work("div")
    area = np.asarray(g0["cell_area"], dtype=np.float64)
    net = np.abs(div @ area)
    scale = np.abs(div) @ area
    print("R2B8 sum A div vn* / sum A |div vn*|: max over levels", float(np.max(net / scale)))
    assert np.all(net <= 1e-12 * scale), float(np.max(net / scale))
    del div
    wp = a.read_work("w_pred")
    assert np.all(np.isfinite(wp))
    assert not np.any(wp[0]) and not np.any(wp[K])
    del wp
    assert a.diag()["mass"] == m0  # the predictor leaves the state alone
    a.part("corrector", dtau, 1)
    b = D.State(G, diffusion="none")
    b.write(S)
    b.step(dtau, 1)
    da, db = a.diag(), b.diag()
    for k in ("mass", "theta_mass", "max_abs_w", "max_abs_vn"):
        assert da[k] == db[k], (k, da[k], db[k])
    a.close()
    b.close()
    G.close()
