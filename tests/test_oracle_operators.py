"""Pins of the oracle's C-grid operators against mathematics (CPU).

Each test is chosen so that a plausible slip in an operator (wrong sign,
transposed index, wrong length or area) fails: discrete identities that hold
to round-off (constant gradient, summation by parts, curl-grad, div-gradt),
and convergence to closed forms of solid-body rotation on the sphere.
"""
import numpy as np
import pytest

from oracle import operators as op
from oracle.grid import Grid
from synth import make_grid, vertical, reference


def _grid(n, k, K=3):
    zh, zf = vertical(K, 10e3)
    return Grid(make_grid(n, k), {"z_half": zh, **reference(zh, zf)})


@pytest.fixture(scope="module")
def g2():
    return _grid(2, 2)


def _solid_body(g, omega=1e-5):
    """Normal wind of rigid rotation about z: u = omega z_hat x r."""
    u = omega * g.radius * np.cross(np.array([0.0, 0.0, 1.0]), g.xe)
    return np.einsum("ej,ej->e", u, g.nrm)[None, :], u


def test_grad_constant_is_zero(g2):
    p = np.full((3, g2.nc), 987.654321)
    assert np.all(op.grad(g2, p) == 0.0)


def test_summation_by_parts(g2):
    rng = np.random.default_rng(0)
    phi = rng.normal(size=(3, g2.nc))
    F = rng.normal(size=(3, g2.ne))
    lhs = np.sum(g2.a_c * phi * op.div(g2, F), axis=1)
    rhs = np.sum(g2.l_e * g2.d_e * F * op.grad(g2, phi), axis=1)
    scale = np.sum(np.abs(g2.l_e * g2.d_e * F * op.grad(g2, phi)), axis=1)
    assert np.all(np.abs(lhs + rhs) / scale < 1e-13)


def test_curl_grad_and_div_gradt_vanish(g2):
    rng = np.random.default_rng(1)
    phi = rng.normal(size=(2, g2.nc))
    psi = rng.normal(size=(2, g2.nv))
    gp = op.grad(g2, phi)
    c = op.curl(g2, gp) * g2.a_v
    ref = np.abs(g2.d_e * gp).max()
    assert np.abs(c).max() < 1e-13 * ref
    gt = op.gradt(g2, psi)
    d = op.div(g2, gt) * g2.a_c
    assert np.abs(d).max() < 1e-13 * np.abs(g2.l_e * gt).max()


def test_solid_body_curl_converges():
    errs = []
    omega = 1e-5
    for k in (2, 3, 4, 5):
        g = _grid(2, k, K=1)
        vn, _ = _solid_body(g, omega)
        z = op.curl(g, vn)[0]
        errs.append(np.max(np.abs(z - 2 * omega * g.xv[:, 2])) / (2 * omega))
    assert all(b < a for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 2e-3


def test_solid_body_divergence_converges_and_lapv_bounded():
    """Div of a rigid rotation converges to 0 (first order); the plain triangular
    vector Laplacian is only zeroth-order accurate, so only a bound is pinned."""
    omega = 1e-5
    dmax = []
    for k in (2, 3, 4, 5):
        g = _grid(2, k, K=1)
        vn, _ = _solid_body(g, omega)
        dmax.append(np.max(np.abs(op.div(g, vn)[0])) / omega)
        L = op.lapv(g, vn)[0]
        want = -2.0 / g.radius**2 * vn[0]
        rms = np.sqrt(np.mean((L - want) ** 2) / np.mean(want**2))
        assert rms < 0.06
    assert all(b < 0.6 * a for a, b in zip(dmax, dmax[1:]))


def test_lapv_adjoint_identity(g2):
    """<F, lapv G>_e = -<div F, div G>_c - <curl F, curl G>_v (both summations by parts)."""
    rng = np.random.default_rng(5)
    F = rng.normal(size=(2, g2.ne))
    G = rng.normal(size=(2, g2.ne))
    lhs = np.sum(g2.l_e * g2.d_e * F * op.lapv(g2, G), axis=1)
    rhs = -(np.sum(g2.a_c * op.div(g2, F) * op.div(g2, G), axis=1)
            + np.sum(g2.a_v * op.curl(g2, F) * op.curl(g2, G), axis=1))
    assert np.all(np.abs(lhs - rhs) < 1e-12 * np.abs(rhs).max())


def test_perot_tangential_converges():
    omega = 1e-5
    errs = []
    for k in (2, 3, 4, 5):
        g = _grid(2, k, K=1)
        vn, u = _solid_body(g, omega)
        vt = op.recon_vt(g, vn)[0]
        want = np.einsum("ej,ej->e", u, g.tan)
        errs.append(np.max(np.abs(vt - want)) / (omega * g.radius))
    assert all(b < a for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 5e-3


def test_scalar_laplacian_is_div_grad(g2):
    """laps must equal div(grad): the same telescoping, written the other way round."""
    rng = np.random.default_rng(2)
    phi = rng.normal(size=(2, g2.nc))
    a = op.laps(g2, phi)
    b = op.div(g2, op.grad(g2, phi))
    assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(b))


def test_level_averages():
    q = np.arange(12.0).reshape(4, 3)
    h = op.ih(q)
    assert h.shape == (5, 3)
    assert np.all(h[0] == q[0]) and np.all(h[-1] == q[-1])
    assert np.all(h[2] == 0.5 * (q[1] + q[2]))
    assert np.all(op.fh(h)[1] == 0.5 * (h[1] + h[2]))


def test_cell_and_edge_means(g2):
    c = np.full((1, g2.nc), 3.0)
    e = np.full((1, g2.ne), 5.0)
    assert np.all(op.avg_e(g2, c) == 3.0)
    assert np.all(op.avg_c(g2, e) == 5.0)


def test_scalar_laplacian_spherical_harmonics():
    """Closed form: on the sphere of radius R a spherical harmonic of degree l
    is an eigenfunction of the Laplacian, lap Y = -l(l+1)/R^2 Y.  The cell
    Laplacian (two-point fluxes l_e/d_e across triangle edges) converges to
    it in the area-weighted L2 norm, about half an order per bisection on
    these grids (pointwise it keeps an O(1) error at irregular cells, as
    such triangle-based Laplacians do), and its Rayleigh quotient gives the
    eigenvalue to within 2 % from R2B4 on: a swapped l_e/d_e, a lost area or a
    flipped sign fails by far."""
    zh, zf = vertical(1, 10e3)
    errs = {1: [], 2: [], 3: []}
    for k in (2, 3, 4):
        g = Grid(make_grid(2, k), {"z_half": zh, **reference(zh, zf)})
        x = g.xc / np.linalg.norm(g.xc, axis=1, keepdims=True)
        for l, phi in ((1, x[:, 2]), (2, x[:, 0] * x[:, 1]), (3, x[:, 2] * (5 * x[:, 2] ** 2 - 3))):
            lap = op.laps(g, phi[None])[0]
            lam = -l * (l + 1) / g.radius**2
            errs[l].append(np.sqrt(np.sum(g.a_c * (lap - lam * phi) ** 2) / np.sum(g.a_c * (lam * phi) ** 2)))
            if k == 4:
                rq = np.sum(g.a_c * phi * lap) / np.sum(g.a_c * phi * phi)
                assert abs(rq / lam - 1) < 0.02, (l, rq / lam)
    for l, e in errs.items():
        assert e[0] > e[1] > e[2], (l, e)
        assert e[2] < 0.03, (l, e)


# ----------------------------------------------------------------------------
# optional operators: least-squares gradient, Miura upwind edge values, RBF vt
# ----------------------------------------------------------------------------
def test_cell_gradient_exact_for_plane_linear_data(g2):
    """The least-squares gradient reproduces data that is linear in the
    tangent-plane coordinates of the cell exactly: sum_i W_i d_i^T is the
    tangent projector at x_c (so grad (g . d) = P g), and it is tangent."""
    W = op.cell_gradient_weights(g2)
    d = g2.radius * (g2.xc[g2.c2e2c] - g2.xc[:, None, :])
    P = np.eye(3)[None] - g2.xc[:, :, None] * g2.xc[:, None, :]
    dp = np.einsum("cij,ckj->cki", P, d)  # offsets projected on the plane
    M = np.einsum("cji,cik->cjk", W, dp)
    assert np.max(np.abs(M - P)) < 1e-12
    assert np.max(np.abs(np.einsum("cji,cj->ci", W, g2.xc))) < 1e-12 * np.max(np.abs(W)) * g2.radius
    # a uniform field has zero gradient, bitwise
    q = np.full((2, g2.nc), 3.5)
    assert np.all(op.cell_gradient(g2, q, W) == 0.0)


def test_miura_second_order_and_upwind():
    """Miura edge values: a uniform field comes out unchanged (bitwise); for
    q = a . x (linear in space) the value at the departure point
    x* = R x_e - dtau (vn n + vt t) is reached to second order (the error
    falls about fourfold per refinement, R2B2 -> R2B5; a first-order or
    centred value would not); the value depends only on the upwind cell and
    its neighbours."""
    om, dtau = 1e-5, 60.0
    a = np.array([0.2, -0.7, 0.4])
    errs = []
    for k in (2, 3, 4, 5):
        g = _grid(2, k, K=1)
        u = om * g.radius * np.cross(np.array([0.3, 0.5, 0.8]) / np.linalg.norm([0.3, 0.5, 0.8]), g.xe)
        vn = np.einsum("ej,ej->e", u, g.nrm)[None]
        vt = np.einsum("ej,ej->e", u, g.tan)[None]
        q = 100.0 * (g.xc @ a)[None]
        qe = op.miura_edge(g, q, vn, vt, dtau)
        xs = g.radius * g.xe - dtau * (vn[0][:, None] * g.nrm + vt[0][:, None] * g.tan)
        want = 100.0 * (xs / np.linalg.norm(xs, axis=1, keepdims=True)) @ a
        errs.append(np.sqrt(np.mean((qe[0] - want) ** 2)))
        if k == 2:
            assert np.all(op.miura_edge(g, np.full((1, g.nc), 7.25), vn, vt, dtau) == 7.25)
            # upwind locality: a spike at one cell reaches only edges whose
            # upwind cell is that cell or one of its neighbours
            c = 100
            spike = np.zeros((1, g.nc))
            spike[0, c] = 1.0
            se = op.miura_edge(g, spike, vn, vt, dtau)[0]
            up = np.where(vn[0] >= 0, g.e2c[:, 0], g.e2c[:, 1])
            near = (up == c) | np.any(g.c2e2c[up] == c, axis=1)
            assert np.all(se[~near] == 0.0) and np.any(se[near] != 0.0)
            # reversing the wind switches the upwind cell
            se2 = op.miura_edge(g, spike, -vn, -vt, dtau)[0]
            up2 = np.where(-vn[0] >= 0, g.e2c[:, 0], g.e2c[:, 1])
            assert np.all(up2 != up)
            near2 = (up2 == c) | np.any(g.c2e2c[up2] == c, axis=1)
            assert np.all(se2[~near2] == 0.0)
    for e0, e1 in zip(errs, errs[1:]):
        assert e1 < 0.35 * e0, errs
    assert errs[-1] < 2e-3, errs


def test_rbf_vt_exact_for_uniform_tangent_flow_and_converges():
    """RBF tangential wind: with the constant term, every flow uniform in the
    tangent plane at the edge is reproduced exactly (the weights map the
    stencil normals onto t_e in that plane); for solid-body rotation on the
    sphere the error falls with refinement R2B2 -> R2B5, below Perot's."""
    errs, errs_p = [], []
    for k in (2, 3, 4, 5):
        g = _grid(2, k, K=1)
        w = op.rbf_vt_weights(g)
        if k == 2:
            st = np.concatenate([np.arange(g.ne)[:, None], g.e2c2e], axis=1)
            s = np.einsum("es,esj->ej", w, g.nrm[st])
            P = np.eye(3)[None] - g.xe[:, :, None] * g.xe[:, None, :]
            assert np.max(np.abs(np.einsum("eij,ej->ei", P, s) - g.tan)) < 1e-10
        om = 1e-5
        ax = np.array([0.3, 0.5, 0.8]) / np.linalg.norm([0.3, 0.5, 0.8])
        u = om * g.radius * np.cross(ax, g.xe)
        vn = np.einsum("ej,ej->e", u, g.nrm)[None]
        want = np.einsum("ej,ej->e", u, g.tan)
        errs.append(np.max(np.abs(op.recon_vt_rbf(g, vn, w)[0] - want)) / (om * g.radius))
        errs_p.append(np.max(np.abs(op.recon_vt(g, vn)[0] - want)) / (om * g.radius))
    for e0, e1 in zip(errs, errs[1:]):
        assert e1 < 0.6 * e0, errs
    assert all(a < b for a, b in zip(errs, errs_p)), (errs, errs_p)
    assert errs[-1] < 1e-3
