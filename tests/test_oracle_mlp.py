"""Pins of the oracle surrogate MLP (CPU): gradients against central finite
differences, GELU against its closed form and derivative, Adam against a
hand-worked first step, features against their definitions on a grid."""
import math

import numpy as np
import pytest

from oracle import mlp as M


def test_gelu_values_and_derivative():
    x = np.array([-3.0, -1.0, 0.0, 0.5, 2.0])
    want = [v * 0.5 * (1 + math.erf(v / math.sqrt(2))) for v in x]
    assert np.allclose(M.gelu(x), want, rtol=0, atol=1e-15)
    h = 1e-6
    fd = (M.gelu(x + h) - M.gelu(x - h)) / (2 * h)
    assert np.allclose(M.gelu_grad(x), fd, rtol=0, atol=1e-9)
    assert M.gelu(np.array([0.0]))[0] == 0.0 and abs(M.gelu_grad(np.array([0.0]))[0] - 0.5) < 1e-15


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(0)
    p = M.init_params(1)
    x = rng.normal(size=(7, 18))
    t = rng.normal(size=7)
    _, g = M.loss_and_grads(p, x, t)
    h = 1e-6
    worst = 0.0
    for k in p:
        flat = p[k].reshape(-1)
        for idx in rng.choice(flat.size, size=min(12, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp, _ = M.loss_and_grads(p, x, t)
            flat[idx] = old - h
            lm, _ = M.loss_and_grads(p, x, t)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = g[k].reshape(-1)[idx]
            worst = max(worst, abs(fd - an) / max(1e-3, abs(fd)))
    assert worst < 1e-6


def test_adam_first_step_is_signed_lr():
    p = {"w": np.array([1.0, -2.0, 3.0])}
    g = {"w": np.array([0.5, -0.25, 0.0])}
    m = {"w": np.zeros(3)}
    v = {"w": np.zeros(3)}
    M.adam_step(p, g, m, v, 1, lr=0.1)
    # first bias-corrected step: lr * g / (|g| + eps)
    assert np.allclose(p["w"], [1.0 - 0.1, -2.0 + 0.1, 3.0], atol=1e-7)


def test_cosine_schedule_end_points():
    assert M.cosine_lr(0, 100) == pytest.approx(1e-3)
    assert M.cosine_lr(100, 100) == pytest.approx(1e-5)
    assert M.cosine_lr(50, 100) == pytest.approx(0.5 * (1e-3 + 1e-5))


def test_init_is_kaiming_uniform_and_seeded():
    a, b = M.init_params(3), M.init_params(3)
    for k in a:
        assert np.array_equal(a[k], b[k])
    assert np.max(np.abs(a["w1"])) <= math.sqrt(6 / 18)
    assert np.max(np.abs(a["w2"])) <= math.sqrt(6 / 64)
    assert np.all(a["b1"] == 0)


def test_features_definitions():
    from oracle.grid import Grid
    from synth import initial_state, make_grid
    from oracle import operators as op

    g0 = make_grid(2, 1)
    S, vert = initial_state(g0, 3, 10e3, seed=2, vn_sigma=1.0)
    g = Grid(g0, vert)
    vn = S["vn"]
    f = M.features(g, vn)
    e, k = 17, 1
    vt = op.recon_vt(g, vn)
    assert f[k, e, 0] == vn[k, e] and f[k, e, 1] == vt[k, e]
    D = op.div(g, vn)
    c0, c1 = g.e2c[e]
    assert f[k, e, 2] == 0.5 * (D[k, c0] + D[k, c1]) and f[k, e, 3] == (D[k, c1] - D[k, c0]) / g.d_e[e]
    z = op.curl(g, vn)
    v0, v1, v2, v3 = g.e2c2v[e]
    assert f[k, e, 5] == (z[k, v1] - z[k, v0]) / g.l_e[e] and f[k, e, 14] == 0.5 * (z[k, v2] + z[k, v3])
    # the tangent-ordered end vertices are e2c2v[:, :2], the same as e2v
    assert np.array_equal(g.e2c2v[:, :2], g.e2v)
    assert np.allclose(f[0, :, 16].mean(), 1.0) and np.allclose(f[0, :, 17].mean(), 1.0)
    # odd in the flow: flipping vn flips the 16 flow features, keeps geometry
    f2 = M.features(g, -vn)
    assert np.allclose(f2[..., :16], -f[..., :16], rtol=0, atol=1e-12)
    assert np.array_equal(f2[..., 16:], f[..., 16:])


def test_features_of_a_solid_body_rotation():
    """A rigid rotation u = Omega x r: no divergence, vorticity 2 Omega
    sin(latitude), no deformation (closed forms, up to discretisation)."""
    from oracle.grid import Grid
    from synth import initial_state, make_grid

    g0 = make_grid(2, 2)
    _, vert = initial_state(g0, 1, 10e3, seed=0)
    g = Grid(g0, vert)
    om = 1.0e-5
    u = np.cross(np.array([0.0, 0.0, om * g.radius]), g.xe)  # (E, 3) metres/s
    vn = np.einsum("ej,ej->e", u, g.nrm)[None, :]
    f = M.features(g, vn)
    scale_d = om  # natural size of the divergence and vorticity
    assert np.max(np.abs(f[0, :, 2])) < 2e-2 * scale_d  # discretely almost divergence-free
    lat = g.xv[:, 2]
    z_ref = 2.0 * om * lat  # curl of a rigid rotation
    zz = f[0, :, 4]
    z_mid = 0.5 * (z_ref[g.e2c2v[:, 0]] + z_ref[g.e2c2v[:, 1]])
    assert np.max(np.abs(zz - z_mid)) < 2e-2 * 2 * om
    # and the along-edge vorticity gradient is that of 2 Omega sin(lat)
    dz_ref = (z_ref[g.e2c2v[:, 1]] - z_ref[g.e2c2v[:, 0]]) / g.l_e
    assert np.max(np.abs(f[0, :, 5] - dz_ref)) < 0.1 * np.max(np.abs(dz_ref))
    # deformation of a rigid rotation vanishes (the least-squares vertex
    # vectors leave a discretisation error, largest near the 12 pentagons),
    # while each shear derivative is of the size of the rotation rate: a sign
    # error in the shearing combination would give |b| ~ Omega
    a = f[0, :, 12] - f[0, :, 11]
    b = f[0, :, 13] + f[0, :, 10]
    d = np.hypot(a, b)
    assert np.sqrt(np.mean(d**2)) < 0.1 * 2 * om and np.max(d) < 0.2 * 2 * om
    assert np.median(np.abs(f[0, :, 13])) > 0.1 * om


def test_features_determine_the_plain_tendency():
    """The plain diffusion tendency is an exact function of the features and
    the geometry: nu L1 - k4 A_e^2 L2 / dt with L1 = f3 - f5 (grad D -
    gradt Z), L2 = f7 - f9 (grad div L1 - gradt curl L1) and nu from the
    deformation of features 10..13."""
    from oracle import dycore as dy
    from oracle.constants import default_params
    from oracle.grid import Grid
    from synth import initial_state, make_grid

    g0 = make_grid(2, 1)
    S, vert = initial_state(g0, 3, 10e3, seed=5, vn_sigma=2.0, jet_u0=20.0)
    g = Grid(g0, vert)
    p = default_params()
    dt = 300.0
    f = M.features(g, S["vn"])
    T = M.diffusion_tendency(g, p, S, dt, dy.diffusion)
    L1 = f[..., 3] - f[..., 5]
    L2 = f[..., 7] - f[..., 9]
    deform = np.hypot(f[..., 12] - f[..., 11], f[..., 13] + f[..., 10])
    nu = np.minimum(p["smag_cs"] * g.a_e * deform, g.a_e / (p["smag_cap"] * dt))
    T_f = nu * L1 - p["hdiff_k4"] * g.a_e**2 * L2 / dt
    assert np.max(np.abs(T_f - T)) <= 1e-9 * np.max(np.abs(T))
