"""The step in parts against the oracle's parts, through the C ABI: the
first level of the paper's verification hierarchy (Section 4.4), which
checks each segment between halo exchanges on the same input fields with a
relative-error tolerance of 1e-12; and its second level, whole steps run
beside the reference on copies of the reference's fields at every step.

Segments: the predictor (advective tendencies at the substep start, the
momentum update to vn*, the implicit solve for w*, with its intermediates
Y, T_w and div vn* read back), the corrector (predictor then corrector is
one substep), the diffusion (plain, and with the theta_v option).  Inputs:
the R2B2 workload state with seeded noise added to w on the interior half
levels, so that every term of T_w is active.  FP64 fields are compared by
relative L2 at <= 1e-12 (the paper's standard tolerance), mixed precision
at <= 1e-5 (FP32 storage of vn and the stencil intermediates).
"""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2608_21150_amd import dycore as D  # noqa: E402
from oracle import dycore as O  # noqa: E402
from oracle import operators as op  # noqa: E402
from oracle.constants import default_params  # noqa: E402
from oracle.grid import Grid as OGrid  # noqa: E402
from synth import build_workload, initial_state, make_grid  # noqa: E402

FIELDS = ("vn", "w", "rho", "exner", "theta_v")
TOL = 1e-12


def rel_l2(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a - b)


def case(name="r2b2_k30", seed=7):
    g0, S, vert, spec = build_workload(name)
    S = {k: v.copy() for k, v in S.items()}
    K = S["rho"].shape[0]
    rng = np.random.default_rng(seed)
    S["w"][1:K] += 0.05 * rng.standard_normal(S["w"][1:K].shape)
    return g0, S, vert, spec


def oracle_predictor(og, p, S, dtau):
    pred, saved = O.predictor(og, p, S, dtau)
    y = S["vn"] + dtau * (p["adv_w0"] * saved["t_vn0"] - p["cpd"] * saved["th_e"] * saved["grad_ex"])
    return {"vn_pred": pred["vn"], "y": y, "w_pred": pred["w"], "t_w": saved["t_w0"],
            "div": op.div(og, pred["vn"])}


@pytest.mark.parametrize("opts", [{}, {"miura": 1}, {"vt_rbf": 1}], ids=["plain", "miura", "vt_rbf"])
@pytest.mark.parametrize("sfc", [False, True], ids=["gen", "curve"])
def test_predictor_part_matches_oracle(opts, sfc):
    g0, S, vert, spec = case()
    dt, nsub = spec["dt"], spec["nsub"]
    og = OGrid(g0, vert)
    p = default_params()
    p.update(opts)
    ref = oracle_predictor(og, p, S, dt / nsub)
    G = D.Grid(g0, vert, sfc=sfc)
    st = D.State(G, params=D.default_params(**opts))
    st.write(S)
    st.part("predictor", dt, nsub)
    for name, r in ref.items():
        got = st.read_work(name)
        err = rel_l2(got, r)
        print(opts, sfc, name, err)
        assert err <= TOL, (opts, sfc, name, err)
    # the predictor leaves the state alone
    out = st.read()
    for k in FIELDS:
        assert np.array_equal(out[k], S[k]), k
    assert st.current() == 0
    st.close()
    G.close()


def test_corrector_part_completes_the_substep():
    """Predictor then corrector equals one substep bit for bit and matches
    the oracle's substep (<= 1e-12); a step of one substep without diffusion
    is the same substep."""
    g0, S, vert, spec = case()
    dt = spec["dt"] / spec["nsub"]
    og = OGrid(g0, vert)
    ref = O.substep(og, default_params(), S, dt)
    G = D.Grid(g0, vert)
    a = D.State(G, diffusion="none")
    b = D.State(G, diffusion="none")
    a.write(S)
    b.write(S)
    a.part("predictor", dt, 1)
    a.part("corrector", dt, 1)
    b.step(dt, 1)
    assert a.current() == 1 and b.current() == 1
    ra, rb = a.read(), b.read()
    for k in FIELDS:
        assert np.array_equal(ra[k], rb[k]), k
        assert rel_l2(ra[k], ref[k]) <= TOL, (k, rel_l2(ra[k], ref[k]))
    # the predictor's fields stay readable after the corrector
    assert rel_l2(a.read_work("vn_pred"), oracle_predictor(og, default_params(), S, dt)["vn_pred"]) <= TOL
    a.close()
    b.close()
    G.close()


@pytest.mark.parametrize("theta", [0, 1], ids=["plain", "theta"])
def test_diffusion_part_matches_oracle(theta):
    g0, S, vert, spec = case()
    dt = spec["dt"]
    og = OGrid(g0, vert)
    p = default_params()
    p["diffuse_theta"] = theta
    ref = O.diffusion(og, p, S, dt)
    G = D.Grid(g0, vert)
    st = D.State(G, params=D.default_params(diffuse_theta=theta))
    st.write(S)
    st.part("diffusion", dt, spec["nsub"])
    out = st.read()
    for k in FIELDS:
        err = rel_l2(out[k], ref[k])
        print(theta, k, err)
        assert err <= TOL, (theta, k, err)
    if not theta:
        for k in ("rho", "exner", "theta_v"):
            assert np.array_equal(out[k], S[k]), k
    assert st.current() == 0
    st.close()
    G.close()


@pytest.mark.parametrize("name", ["r1b0_k4", "r2b1_k7"])
def test_parts_on_small_and_ragged_grids(name):
    """Grids smaller than one tile and with ragged last tiles."""
    g0, S, vert, spec = case(name)
    dt, nsub = spec["dt"], spec["nsub"]
    og = OGrid(g0, vert)
    p = default_params()
    ref = oracle_predictor(og, p, S, dt / nsub)
    G = D.Grid(g0, vert)
    st = D.State(G)
    st.write(S)
    st.part("predictor", dt, nsub)
    for n, r in ref.items():
        got = st.read_work(n)
        if np.linalg.norm(r) == 0:
            assert np.max(np.abs(got)) <= 1e-13, (name, n)
        else:
            assert rel_l2(got, r) <= TOL, (name, n, rel_l2(got, r))
    st.close()
    G.close()


@pytest.mark.parametrize("n_lev", [90, 129])
def test_predictor_part_deep_columns(n_lev):
    """The column predictor's chunking at the R2B8 depth and the maximum."""
    g0 = make_grid(2, 1)
    S, vert = initial_state(g0, n_lev, 75.0e3, seed=21, vn_sigma=1.0, jet_u0=35.0, n_bumps=4,
                            bump_radius=2000.0e3)
    rng = np.random.default_rng(3)
    S["w"][1:n_lev] += 0.05 * rng.standard_normal(S["w"][1:n_lev].shape)
    og = OGrid(g0, vert)
    ref = oracle_predictor(og, default_params(), S, 100.0)
    G = D.Grid(g0, vert)
    st = D.State(G)
    st.write(S)
    st.part("predictor", 300.0, 3)
    for n, r in ref.items():
        assert rel_l2(st.read_work(n), r) <= TOL, (n_lev, n, rel_l2(st.read_work(n), r))
    st.close()
    G.close()


def test_mixed_precision_parts():
    g0, S, vert, spec = case()
    dt, nsub = spec["dt"], spec["nsub"]
    og = OGrid(g0, vert)
    ref = oracle_predictor(og, default_params(), S, dt / nsub)
    G = D.Grid(g0, vert)
    st = D.State(G, precision="mixed")
    st.write(S)
    st.part("predictor", dt, nsub)
    for n, r in ref.items():
        err = rel_l2(st.read_work(n), r)
        print("mixed", n, err)
        assert err <= 1e-5, (n, err)
    st.close()
    st = D.State(G, precision="mixed")
    st.write(S)
    st.part("diffusion", dt, nsub)
    out = st.read()
    dref = O.diffusion(og, default_params(), S, dt)
    for k in FIELDS:
        assert rel_l2(out[k], dref[k]) <= 1e-5, k
    st.close()
    G.close()


def test_part_errors():
    g0, S, vert, spec = case("r1b0_k4")
    G = D.Grid(g0, vert)
    st = D.State(G)
    st.write(S)
    h = st.handle
    buf = np.empty(S["vn"].size)
    ptr = buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert D.lib.dc_state_read_work(h, 0, ptr, buf.size) == D.DC_ESTATE
    assert D.lib.dc_dycore_part(h, 1, 60.0, 1) == D.DC_ESTATE       # corrector without predictor
    assert D.lib.dc_dycore_part(h, 3, 60.0, 1) == D.DC_EINVAL       # no such part
    assert D.lib.dc_dycore_part(h, 0, -1.0, 1) == D.DC_EINVAL
    assert D.lib.dc_dycore_part(h, 0, 60.0, 0) == D.DC_EINVAL
    st.part("predictor", 60.0, 1)
    assert D.lib.dc_state_read_work(h, 0, ptr, buf.size - 1) == D.DC_EINVAL
    assert D.lib.dc_state_read_work(h, 9, ptr, buf.size) == D.DC_EINVAL
    D.check(D.lib.dc_state_read_work(h, 0, ptr, buf.size))
    st.part("corrector", 60.0, 1)
    assert D.lib.dc_dycore_part(h, 1, 60.0, 1) == D.DC_ESTATE       # a second corrector
    st.step(60.0, 1)
    assert D.lib.dc_state_read_work(h, 0, ptr, buf.size) == D.DC_ESTATE
    st.close()
    none = D.State(G, diffusion="none")
    assert D.lib.dc_dycore_part(none.handle, 2, 60.0, 1) == D.DC_ESTATE
    none.close()
    G.close()


@pytest.mark.parametrize("precision,tol", [("fp64", TOL), ("mixed", 1e-5)])
def test_second_level_step_by_step(precision, tol):
    """The paper's second verification level (Section 4.4): the GPU step runs
    beside the reference on copies of the reference's fields, so that each
    step is checked on its own and errors do not accumulate.  Five whole
    steps (substeps and diffusion) of config 1 from the seeded state: at
    every step the GPU state is overwritten with the oracle's, both advance
    one step, and every field agrees within the tolerance."""
    g0, S, vert, spec = case()
    dt, nsub = spec["dt"], spec["nsub"]
    og = OGrid(g0, vert)
    p = default_params()
    wts = O.vertex_lsq_weights(og)
    G = D.Grid(g0, vert)
    st = D.State(G, precision=precision)
    worst = {k: 0.0 for k in FIELDS}
    for _ in range(5):
        st.write(S)
        st.step(dt, nsub)
        got = st.read()
        S = O.step(og, S, dt, nsub, p, wts=wts)
        for k in FIELDS:
            worst[k] = max(worst[k], rel_l2(got[k], S[k]))
    print(precision, "worst per-step rel L2:", worst)
    for k in FIELDS:
        assert worst[k] <= tol, (precision, k, worst[k])
    st.close()
    G.close()


@pytest.mark.parametrize("dtau", [600.0, 3000.0])
def test_predictor_part_large_courant(dtau):
    """The column solve at large vertical Courant numbers (sound crosses
    many layers per substep: c dtau / dz up to ~1000 on config 1's 1 km
    layers): w* from the partition-method solve matches the oracle's Thomas
    solve, itself pinned against dense LU, at 1e-12."""
    g0, S, vert, spec = case()
    og = OGrid(g0, vert)
    ref = oracle_predictor(og, default_params(), S, dtau)
    G = D.Grid(g0, vert)
    st = D.State(G)
    st.write(S)
    st.part("predictor", dtau, 1)
    for n in ("w_pred", "vn_pred", "t_w"):
        err = rel_l2(st.read_work(n), ref[n])
        print(dtau, n, err)
        assert err <= TOL, (dtau, n, err)
    st.close()
    G.close()
