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
    vertex vector is exact for a uniform tangent vector;
  * theta-mass conserved to round-off, and the column update keeps the
    equation of state to second order in the pressure increment (theta_v
    increment);
  * the sponge profile's zeros, top value, midpoint and layer mean;
  * the horizontal advection of w converges to -u . grad w for a
    solid-body rotation;
  * the w diffusion: uniform levels untouched, the capped-viscosity
    increment of a degree-1 harmonic in closed form, energy not growing.
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


# ----------------------------------------------------------------------------
# pins of the theta_v increment, the sponge profile, the horizontal advection
# of w and the w diffusion (each fails under the slip named in its docstring)
# ----------------------------------------------------------------------------
def test_theta_mass_conserved(r2b2_case):
    """The increment form of the column update (Section 4.1, vertically
    implicit solver) changes rho theta_v by the divergence of the theta flux
    only: rho* theta_v* = rho theta_v (1 + (c_vd/R_d) d_pi/pi), and
    (c_vd/R_d) rho theta_v b / pi = dtau.  So the total theta-mass telescopes
    like the mass.  An inverted c_vd/R_d, or a theta_v update that drops the
    -theta_v d_rho term, breaks it at first order."""
    g, S, spec = r2b2_case
    t0 = dycore.diag(g, S)["theta_mass"]
    S1 = S
    for _ in range(10):
        S1 = dycore.step(g, S1, spec["dt"], spec["nsub"])
    assert abs(dycore.diag(g, S1)["theta_mass"] / t0 - 1.0) <= 1e-13


def test_column_update_keeps_equation_of_state_to_second_order(r2b3):
    """Exner is advanced by the equation of state linearised in the pressure
    increment (Section 4.1; the linearised form of the Exner equation).  With
    x = d_pi / pi and a = c_vd / R_d, the update gives pi* = pi (1 + x) and
    rho* theta_v* = rho theta_v (1 + a x), so the full equation of state
    pi(rho theta_v) = (R_d rho theta_v / p0)^(1/a) differs from pi* by
    pi ((1 + x) - (1 + a x)^(1/a)) = pi (a - 1) x^2 / 2 + O(x^3) at every
    point.  Any first-order slip in the rho, exner or theta_v increments
    (a wrong c_vd/R_d, a lost theta_v d_rho term) leaves a residual of order x."""
    S, vert = initial_state(r2b3, 20, 30e3, seed=3, jet_u0=35.0, n_bumps=10, bump_amp=3.0,
                            bump_radius=1000e3, vn_sigma=2.0)
    g = Grid(r2b3, vert)
    p = default_params()
    a = p["cvd"] / p["rd"]
    # the initial state satisfies the equation of state to round-off
    eos0 = (p["rd"] * S["rho"] * S["theta_v"] / 1.0e5) ** (1.0 / a)
    assert np.max(np.abs(eos0 / S["exner"] - 1.0)) < 1e-14
    for dtau in (40.0, 10.0):
        pred, _ = dycore.predictor(g, p, S, dtau)
        x = pred["exner"] / S["exner"] - 1.0
        eos = (p["rd"] * pred["rho"] * pred["theta_v"] / 1.0e5) ** (1.0 / a)
        resid = pred["exner"] - eos
        lead = S["exner"] * (a - 1.0) * x * x / 2.0
        m = np.abs(x) > 1e-5
        assert m.sum() > 1000
        ratio = resid[m] / lead[m]
        assert np.max(np.abs(ratio - 1.0)) < 2e-3, (dtau, ratio.min(), ratio.max())
        # and nowhere a first-order residual
        assert np.max(np.abs(resid)) <= 1.01 * np.max(np.abs(lead)) + 1e-15


def test_sponge_profile():
    """Rayleigh damping (the upper sponge of the column solver): zero at and
    below z_d = 2/3 z_top, tau0 at the model top, tau0/2 halfway between
    (sin^2(pi/4) = 1/2), and a layer mean of tau0/2 (the mean of sin^2 over a
    quarter period).  A sin profile instead of sin^2 gives 0.71 and 0.64;
    a wrong z_d moves the zeros."""
    g0 = make_grid(1, 0)
    K = 300
    _, vert = initial_state(g0, K, 30e3, seed=0)
    g = Grid(g0, vert)
    p = default_params()
    tau0 = p["rayleigh_tau0"]
    tau = dycore.rayleigh_tau(g, p)
    z = g.z_half
    z_d = 20e3
    assert np.all(tau[z <= z_d + 1e-6] == 0.0)
    assert np.all(tau[z > z_d + 1e-6] > 0.0)
    assert tau[0] == tau0  # model top
    mid = np.argmin(np.abs(z - 25e3))
    assert abs(z[mid] - 25e3) < 1e-6
    assert abs(tau[mid] / tau0 - 0.5) < 1e-12
    # layer mean over [z_d, z_top] by the trapezoid rule on the half levels
    band = z >= z_d - 1e-6
    zz, tt = z[band][::-1], tau[band][::-1]
    mean = np.sum(0.5 * (tt[1:] + tt[:-1]) * np.diff(zz)) / (zz[-1] - zz[0])
    assert abs(mean / tau0 - 0.5) < 1e-4
    # the solver divides w* by (1 + dtau tau): a resting column with w only
    # at the top half level loses it at that rate, compare the damped and
    # undamped columns' w after one predictor
    S, vert = initial_state(g0, 30, 30e3, seed=0)
    g30 = Grid(g0, vert)
    S = dict(S)
    S["w"] = S["w"].copy()
    S["w"][1] = 0.1
    p0 = dict(p)
    p0["rayleigh_tau0"] = 0.0
    dtau = 10.0
    w_damped = dycore.predictor(g30, p, S, dtau)[0]["w"]
    w_free = dycore.predictor(g30, p0, S, dtau)[0]["w"]
    tau30 = dycore.rayleigh_tau(g30, p)
    assert np.allclose(w_damped[1:30], w_free[1:30] / (1.0 + dtau * tau30[1:30, None]), rtol=1e-14, atol=0.0)


def _solid_body_vn(g, axis, omega, n_lev):
    u = omega * g.radius * np.cross(np.asarray(axis, dtype=float), g.xe)
    return np.repeat(np.einsum("ej,ej->e", u, g.nrm)[None], n_lev, axis=0)


def test_horizontal_w_advection_converges_to_closed_form():
    """Horizontal part of the vertical-wind advection (velocity advection,
    Section 4.1).  For a solid-body rotation about the x axis,
    u = omega R (x_hat x r_hat), and w = W sin(lat) = W z_hat . r_hat, the
    continuous term is -u . grad w = -omega W y.  With w uniform in the
    vertical the vertical part vanishes, so T_w is the horizontal part
    alone; its relative RMS error against -omega W y_c must fall with every
    refinement R2B2 -> R2B5.  A lost factor 1/2 or a flipped sign leaves an
    error of 1 or 2."""
    errs = []
    om, W, K = 1e-5, 2.0, 3
    for k in (2, 3, 4, 5):
        g0 = make_grid(2, k)
        _, vert = initial_state(g0, K, 10e3, seed=0)
        g = Grid(g0, vert)
        vn = _solid_body_vn(g, (1.0, 0.0, 0.0), om, K)
        w = np.repeat((W * g.xc[:, 2])[None], K + 1, axis=0)
        _, t_w = dycore.velocity_advection(g, default_params(), vn, w)
        exact = -om * W * g.xc[:, 1]
        for j in range(1, K):
            assert np.array_equal(t_w[j], t_w[1])
        errs.append(np.sqrt(np.mean((t_w[1] - exact) ** 2) / np.mean(exact**2)))
    assert errs[0] < 0.1
    for a, b in zip(errs[:-1], errs[1:]):
        assert b < 0.8 * a, errs
    assert errs[-1] < 0.025, errs


def test_w_diffusion_pins():
    """Second-order Smagorinsky diffusion of w (the diffusion granule,
    Section 4.1): w(k) += dt nu_c(k) laps(w)(k) with nu_c the cell mean of
    nu at half levels.  Pins:
      * a horizontally uniform w is left bitwise unchanged (laps of a
        constant is exactly zero), and so are the boundaries w(0), w(K);
      * with nu on its stability cap A_e / (16 dt) at one full level j and
        zero elsewhere, only half levels j and j+1 move, by the same amount,
        and for w = W sin(lat) (a degree-1 harmonic, laps = -2 w / R^2) the
        increment is -(mean_e A_e) / (16 R^2) w: the half-level mean (1/2),
        the cell mean (1/3), dt and the sign are all fixed by this value;
      * sum A_c w^2 does not grow for a random w under a random flow."""
    g0 = make_grid(2, 3)
    K = 5
    S, vert = initial_state(g0, K, 10e3, seed=0)
    g = Grid(g0, vert)
    p = default_params()
    dt = 600.0
    rng = np.random.default_rng(1)
    S2 = dict(S)
    S2["vn"] = rng.normal(0.0, 20.0, (K, g.ne))
    S2["w"] = np.zeros((K + 1, g.nc))
    S2["w"][1:K] = rng.normal(0.0, 1.0, (K - 1, 1))  # uniform on every half level
    out = dycore.diffusion(g, p, S2, dt)
    assert np.array_equal(out["w"], S2["w"])
    # capped viscosity at full level 1 only (not the middle one, so that a
    # level mix-up shows)
    p_cap = dict(p)
    p_cap["smag_cs"] = 1e9
    W = 3.0
    S3 = dict(S)
    S3["vn"] = np.zeros((K, g.ne))
    S3["vn"][1] = rng.normal(0.0, 1.0, g.ne)
    S3["w"] = np.zeros((K + 1, g.nc))
    S3["w"][1:K] = W * g.xc[:, 2][None]
    S3["w"][0] = S3["w"][K] = 1.0  # boundary values must stay as they are
    out = dycore.diffusion(g, p_cap, S3, dt)
    inc = out["w"] - S3["w"]
    for k in (0, 3, 4, 5):
        assert np.all(inc[k] == 0.0), k
    assert np.array_equal(inc[1], inc[2])
    ae_c = (g.a_e[g.c2e[:, 0]] + g.a_e[g.c2e[:, 1]] + g.a_e[g.c2e[:, 2]]) / 3.0
    exact = -ae_c / (16.0 * g.radius**2) * W * g.xc[:, 2]
    rms = np.sqrt(np.mean((inc[1] - exact) ** 2) / np.mean(exact**2))
    assert rms < 0.04, rms
    big = np.abs(exact) > 0.1 * np.abs(exact).max()
    assert abs(np.median(inc[1][big] / exact[big]) - 1.0) < 0.01
    # energy of a random w under a random flow
    S4 = dict(S)
    S4["vn"] = rng.normal(0.0, 20.0, (K, g.ne))
    S4["w"] = np.zeros((K + 1, g.nc))
    S4["w"][1:K] = rng.normal(0.0, 1.0, (K - 1, g.nc))
    out = dycore.diffusion(g, p, S4, dt)
    e0 = np.sum(g.a_c * S4["w"] ** 2)
    e1 = np.sum(g.a_c * out["w"] ** 2)
    assert e1 < e0
    assert np.abs(out["w"] - S4["w"]).max() > 1e-6  # it did act


@pytest.mark.parametrize("opts", [{"miura": 1}, {"vt_rbf": 1}, {"miura": 1, "vt_rbf": 1}])
def test_fuller_numerics_options_keep_invariants(opts, r2b2_case, r2b3):
    """Miura upwind edge values and the RBF tangential wind (Section 4.1:
    ICON's discretisation) keep the step's invariants: the resting
    atmosphere stays bitwise at rest, mass and theta-mass are conserved to
    round-off over 10 steps of the parity case, a horizontally uniform state
    gets no horizontal tendencies, and the balanced jet stays steady."""
    g, S, spec = r2b2_case
    p = default_params()
    p.update(opts)
    _, Sr, _, _ = build_workload("r2b2_k30_rest")
    S1 = Sr
    for _ in range(3):
        S1 = dycore.step(g, S1, spec["dt"], spec["nsub"], p)
    for k in Sr:
        assert np.array_equal(S1[k], Sr[k]), k
    d0 = dycore.diag(g, S)
    S1 = S
    for _ in range(10):
        S1 = dycore.step(g, S1, spec["dt"], spec["nsub"], p)
    d1 = dycore.diag(g, S1)
    assert abs(d1["mass"] / d0["mass"] - 1.0) <= 1e-13
    assert abs(d1["theta_mass"] / d0["theta_mass"] - 1.0) <= 1e-13
    assert d1["n_nonfinite"] == 0 and d1["max_abs_vn"] < 10.0
    Su, vert = initial_state(r2b3, 12, 20e3, seed=0)
    gu = Grid(r2b3, vert)
    Su["theta_v"] = Su["theta_v"] + np.linspace(0.0, 3.0, 12)[:, None]
    S2 = dycore.step(gu, Su, 300.0, 3, p)
    assert np.all(S2["vn"] == 0.0)
    for k in ("w", "rho", "exner", "theta_v"):
        assert np.all(S2[k] == S2[k][:, :1]), k
    Sj, vert = initial_state(r2b3, 20, 30e3, seed=0, jet_u0=35.0)
    gj = Grid(r2b3, vert)
    S3 = dycore.step(gj, Sj, 300.0, 5, p)
    assert np.abs(S3["vn"] - Sj["vn"]).max() < 0.05
