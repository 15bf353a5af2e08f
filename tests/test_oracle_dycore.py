"""Pins of the oracle's time step against invariants and physics (CPU).

Each pin targets a part of the step where a plausible slip would show:
  * resting isothermal atmosphere stays bitwise at rest (whole step);
  * total mass conserved to round-off (flux form, column increments);
  * horizontally uniform fields produce no horizontal tendencies (bitwise);
  * a balanced zonal jet stays steady, and does not with the Coriolis sign
    flipped (Coriolis, kinetic-energy gradient, pressure gradient signs);
  * a column balanced by the input generator's own discrete hydrostatic
    integration keeps w ~ 0, an unbalanced one does not (implicit solver,
    buoyancy and vertical pressure-gradient signs);
  * vertical advection signs, diffusion and divergence damping dissipate,
    Smagorinsky sees no deformation in rigid rotation, the least-squares
    vertex vector is exact for a uniform tangent vector.
"""
import numpy as np
import pytest

from oracle import dycore
from oracle import operators as op
from oracle.constants import default_params
from oracle.grid import Grid
from synth import build_workload, initial_state, make_grid


@pytest.fixture(scope="module")
def r2b2_case():
    g0, S, vert, spec = build_workload("r2b2_k30")
    return Grid(g0, vert), S, spec


@pytest.fixture(scope="module")
def r2b3():
    return make_grid(2, 3)


def test_rest_state_bitwise(r2b2_case):
    g, _, spec = r2b2_case
    g0, S, vert, _ = build_workload("r2b2_k30_rest")
    S1 = S
    for _ in range(10):
        S1 = dycore.step(g, S1, spec["dt"], spec["nsub"])
    for k in S:
        assert np.array_equal(S1[k], S[k]), k


def test_mass_conservation(r2b2_case):
    g, S, spec = r2b2_case
    m0 = dycore.diag(g, S)["mass"]
    S1 = S
    for _ in range(10):
        S1 = dycore.step(g, S1, spec["dt"], spec["nsub"])
    d = dycore.diag(g, S1)
    assert abs(d["mass"] / m0 - 1.0) <= 1e-13
    assert d["n_nonfinite"] == 0
    assert d["max_abs_vn"] < 10.0 and d["max_abs_w"] < 1.0  # stays bounded


def test_horizontally_uniform_symmetry(r2b3):
    S, vert = initial_state(r2b3, 12, 20e3, seed=0)
    g = Grid(r2b3, vert)
    S["theta_v"] = S["theta_v"] + np.linspace(0.0, 3.0, 12)[:, None]  # unbalanced, uniform
    S1 = dycore.step(g, S, 300.0, 3)
    assert np.all(S1["vn"] == 0.0)
    for k in ("w", "rho", "exner", "theta_v"):
        assert np.all(S1[k] == S1[k][:, :1]), k
    assert np.abs(S1["w"]).max() > 1e-3  # the column did evolve


def test_balanced_jet_steady_and_coriolis_sign(r2b3):
    S, vert = initial_state(r2b3, 20, 30e3, seed=0, jet_u0=35.0)
    g = Grid(r2b3, vert)
    p = default_params()
    S1 = dycore.step(g, S, 300.0, 5, p)
    assert np.abs(S1["vn"] - S["vn"]).max() < 0.05
    p2 = dict(p)
    p2["omega"] = -p["omega"]
    S2 = dycore.step(g, S, 300.0, 5, p2)
    assert np.abs(S2["vn"] - S["vn"]).max() > 0.5


def test_balanced_warm_column_keeps_w_zero(r2b3):
    prof = 4.0 * np.sin(np.linspace(0.0, np.pi, 16))
    S, vert = initial_state(r2b3, 16, 20e3, seed=0, t_profile=prof)
    g = Grid(r2b3, vert)
    S1 = dycore.step(g, S, 300.0, 5)
    assert np.abs(S1["w"]).max() < 1e-9
    # the same temperatures with the reference Exner (not balanced) must move
    Sb = dict(S)
    Sb["exner"] = np.repeat(g.ex_ref[:, None], g.nc, axis=1)
    Sb["rho"] = 1.0e5 * Sb["exner"] ** (717.6 / 287.04) / (287.04 * Sb["theta_v"])
    S2 = dycore.step(g, Sb, 300.0, 5)
    assert np.abs(S2["w"]).max() > 1e-3


def test_vertical_advection_signs(r2b3):
    S, vert = initial_state(r2b3, 10, 10e3, seed=0)
    g = Grid(r2b3, vert)
    p = default_params()
    K = 10
    # vn increasing with height (k = 0 is the top), w > 0 in the interior
    vn = np.repeat(np.linspace(10.0, 1.0, K)[:, None], g.ne, axis=1)
    w = np.zeros((K + 1, g.nc))
    w[1:K] = 0.5
    t_vn, _ = dycore.velocity_advection(g, p, vn, w)
    t_vn0, _ = dycore.velocity_advection(g, p, vn, np.zeros_like(w))
    vert_part = (t_vn - t_vn0)[1:K - 1]
    assert np.all(vert_part < 0.0)  # upward motion brings slower air from below
    w2 = np.zeros((K + 1, g.nc))
    w2[1:K] = np.linspace(1.0, 0.1, K - 1)[:, None]  # w decreasing downward, upward motion
    _, t_w = dycore.velocity_advection(g, p, np.zeros((K, g.ne)), w2)
    # -w dw/dz with dw/dz > 0 and w > 0 -> negative
    assert np.all(t_w[2:K - 1] < 0.0)
    assert np.all(t_w[0] == 0.0) and np.all(t_w[K] == 0.0)


def test_diffusion_and_divergence_damping_dissipate(r2b3):
    S, vert = initial_state(r2b3, 6, 10e3, seed=4, vn_sigma=2.0, jet_u0=20.0)
    g = Grid(r2b3, vert)
    p = default_params()
    e0 = np.sum(g.a_e * S["vn"] ** 2)
    S1 = dycore.diffusion(g, p, S, 600.0)
    assert np.sum(g.a_e * S1["vn"] ** 2) < e0
    # the corrector's damping increment alone reduces the divergence
    inc = -p["divdamp_c4"] * g.mean_area**2 * dycore.divergence_damping(g, S["vn"])
    d0 = np.sum(g.a_c * op.div(g, S["vn"]) ** 2)
    d1 = np.sum(g.a_c * op.div(g, S["vn"] + inc) ** 2)
    assert d1 < d0


def test_smagorinsky_rigid_rotation_vs_shear(r2b3):
    _, vert = initial_state(r2b3, 1, 10e3, seed=0)
    g = Grid(r2b3, vert)
    p = default_params()
    w = dycore.vertex_lsq_weights(g)
    om = 1e-5
    u = om * g.radius * np.cross(np.array([0.0, 0.0, 1.0]), g.xe)
    vn = np.einsum("ej,ej->e", u, g.nrm)[None]
    vv = np.einsum("vjs,kvs->kvj", w, np.where(g.v2e[None] >= 0, vn[:, np.maximum(g.v2e, 0)], 0.0))
    nu_rot = dycore.smagorinsky_nu(g, p, vv, 1.0)
    # zonal shear flow u = U z (z = sin lat), deformation ~ U / R
    u2 = 10.0 * g.xe[:, 2:3] * np.cross(np.array([0.0, 0.0, 1.0]), g.xe)
    vn2 = np.einsum("ej,ej->e", u2, g.nrm)[None]
    vv2 = np.einsum("vjs,kvs->kvj", w, np.where(g.v2e[None] >= 0, vn2[:, np.maximum(g.v2e, 0)], 0.0))
    nu_sh = dycore.smagorinsky_nu(g, p, vv2, 1.0)
    def_rot = np.median(nu_rot / (p["smag_cs"] * g.a_e)) / om
    def_sh = np.median(nu_sh / (p["smag_cs"] * g.a_e)) / (10.0 / g.radius)
    assert def_rot < 0.05
    assert 0.3 < def_sh < 3.0


def test_lsq_vertex_vector_exact_for_tangent_vector(r2b3):
    _, vert = initial_state(r2b3, 1, 10e3, seed=0)
    g = Grid(r2b3, vert)
    w = dycore.vertex_lsq_weights(g)
    rng = np.random.default_rng(0)
    U = rng.normal(size=(g.nv, 3))
    U -= np.einsum("vj,vj->v", U, g.xv)[:, None] * g.xv  # tangent at each vertex
    ok = g.v2e >= 0
    vn_v = np.where(ok, np.einsum("vsj,vj->vs", g.nrm[np.maximum(g.v2e, 0)], U), 0.0)
    rec = np.einsum("vjs,vs->vj", w, vn_v)
    assert np.abs(rec - U).max() < 1e-12 * np.abs(U).max()


def test_smagorinsky_cap(r2b3):
    S, vert = initial_state(r2b3, 3, 10e3, seed=9, vn_sigma=50.0)
    g = Grid(r2b3, vert)
    p = default_params()
    w = dycore.vertex_lsq_weights(g)
    vv = np.einsum("vjs,kvs->kvj", w, np.where(g.v2e[None] >= 0, S["vn"][:, np.maximum(g.v2e, 0)], 0.0))
    dt = 1.0e5
    nu = dycore.smagorinsky_nu(g, p, vv, dt)
    assert np.all(nu >= 0.0)
    assert np.all(nu <= g.a_e / (p["smag_cap"] * dt))
    assert np.any(nu == g.a_e / (p["smag_cap"] * dt))


def test_equation_of_state_round_trip():
    g = make_grid(2, 1)
    S, vert = initial_state(g, 8, 20e3, seed=3, jet_u0=35.0, n_bumps=4, bump_radius=2000e3)
    ex = (287.04 * S["rho"] * S["theta_v"] / 1.0e5) ** (287.04 / 717.6)
    assert np.max(np.abs(ex / S["exner"] - 1)) < 1e-14
    # jet surface pressure: equator/pole ratio of the gradient-wind balance
    from synth.state import _surface_pressure_jet
    r = _surface_pressure_jet(np.array([0.0]), 35.0, 6.371e6)[0] / _surface_pressure_jet(np.array([np.pi / 2]), 35.0, 6.371e6)[0]
    assert abs(r - 1.168) < 1e-3


def _theta_diffusion(g, S, dt=600.0):
    p = default_params()
    p["diffuse_theta"] = 1
    out = dycore.diffusion(g, p, S, dt)
    return p, out


def test_theta_diffusion_leaves_uniform_levels_alone(r2b3):
    """A theta_v that is constant on every level has no horizontal Laplacian:
    theta_v and exner come out bitwise unchanged however large nu is."""
    S, vert = initial_state(r2b3, 4, 10e3, seed=3, vn_sigma=20.0)
    g = Grid(r2b3, vert)
    _, out = _theta_diffusion(g, S)
    assert np.all(np.ptp(S["theta_v"], axis=1) == 0.0)  # the generator's reference column
    assert np.array_equal(out["theta_v"], S["theta_v"])
    assert np.array_equal(out["exner"], S["exner"])


def test_theta_diffusion_maximum_principle_and_pressure(r2b3):
    """theta_v bumps: a cell hotter than its three neighbours cools and a
    colder one warms (nu >= 0, positive Laplacian weights); exner moves with
    theta_v as the equation of state at fixed rho says, pi ~ (rho theta_v)^(R_d/c_vd),
    to second order in the increment."""
    S, vert = initial_state(r2b3, 4, 10e3, seed=4, vn_sigma=20.0, t_sigma=1.0)
    g = Grid(r2b3, vert)
    p, out = _theta_diffusion(g, S)
    th, dth = S["theta_v"], out["theta_v"] - S["theta_v"]
    nb = th[:, g.c2e2c]  # [K][C][3]
    hot = np.all(th[:, :, None] > nb, axis=2)
    cold = np.all(th[:, :, None] < nb, axis=2)
    assert hot.sum() > 10 and cold.sum() > 10
    assert np.all(dth[hot] <= 0.0) and np.any(dth[hot] < 0.0)
    assert np.all(dth[cold] >= 0.0) and np.any(dth[cold] > 0.0)
    a = p["rd"] / p["cvd"]
    x = dth / th
    assert np.max(np.abs(x)) > 1e-6
    resid = out["exner"] / S["exner"] - (1.0 + x) ** a
    assert np.max(np.abs(resid)) <= 0.2 * np.max(x * x) + 1e-15
    assert np.array_equal(out["rho"], S["rho"])


def _cold_pool_increment(g, S, cell, level, d_theta, n_enh, p_extra=None):
    """theta_v increment of `cell` at `level` after one diffusion step of a
    resting state (vn = 0, so the Smagorinsky viscosity is zero everywhere)
    whose theta_v is the reference column except at that one point, shifted
    by d_theta.  Returns the increment, the output and the input."""
    S = {k: v.copy() for k, v in S.items()}
    S["theta_v"][level, cell] += d_theta
    p = default_params()
    p["diffuse_theta"] = 1
    p["theta_enh_nlev"] = n_enh
    p.update(p_extra or {})
    out = dycore.diffusion(g, p, S, 600.0)
    return out["theta_v"][level, cell] - S["theta_v"][level, cell], out, S


def test_near_surface_enhancement_ramp_and_band(r2b3):
    """The near-surface floor on the theta_v coefficient (Section 4.1): with
    no wind only the floor diffuses.  A cold point anomaly -dT relaxes by
    s(dT) * f * dT, s ramping from 0 at dT = T to 1 at dT = 2T; f, the
    fraction one step at the stability cap removes, is geometry alone
    (3 / (8 sqrt 3) on an equilateral mesh with A_e = l d / 2 and the cap
    A_e / (16 dt)), so increment ratios between anomalies fix the ramp.  Warm
    anomalies, anomalies above the band of lowest levels and the cold cell's
    neighbours (warmer than their own neighbours) stay untouched."""
    S, vert = initial_state(r2b3, 4, 10e3, seed=5)
    g = Grid(r2b3, vert)
    assert np.all(S["vn"] == 0.0) and np.all(np.ptp(S["theta_v"], axis=1) == 0.0)
    T = default_params()["theta_enh_thresh"]
    K, c = 4, 17
    inc = {}
    for m in (0.9, 1.5, 2.0, 3.0):
        inc[m], out, S1 = _cold_pool_increment(g, S, c, K - 1, -m * T, 1)
        # nothing else moves: every other cell has zero coefficient
        mask = np.ones_like(S1["theta_v"], dtype=bool)
        mask[K - 1, c] = False
        assert np.array_equal(out["theta_v"][mask], S1["theta_v"][mask])
    assert inc[0.9] == 0.0
    f = inc[2.0] / (2.0 * T)
    assert abs(f / (3.0 / (8.0 * np.sqrt(3.0))) - 1) < 0.15, f
    assert abs(inc[3.0] / inc[2.0] - 1.5) < 1e-12  # s saturates at 1
    assert abs(inc[1.5] / inc[2.0] - 0.375) < 1e-12  # s = 0.5 at dT = 1.5 T
    # warm anomaly: no floor
    assert _cold_pool_increment(g, S, c, K - 1, 3.0 * T, 1)[0] == 0.0
    # the level above the band of one level is left alone; with a band of two
    # it relaxes like the lowest level (same horizontal geometry)
    assert _cold_pool_increment(g, S, c, K - 2, -3.0 * T, 1)[0] == 0.0
    up = _cold_pool_increment(g, S, c, K - 2, -3.0 * T, 2)[0]
    assert abs(up / inc[3.0] - 1) < 1e-12
    # no overshoot past the surrounding value (the cap keeps f < 1)
    assert 0.0 < f < 1.0
    # a larger threshold moves the ramp: dT = 3 T with threshold 2 T gives s = 0.5
    half = _cold_pool_increment(g, S, c, K - 1, -3.0 * T, 1, {"theta_enh_thresh": 2.0 * T})[0]
    assert abs(half / inc[3.0] - 0.5) < 1e-12
