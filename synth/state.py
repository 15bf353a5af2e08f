"""Seeded initial states and the vertical reference column (seeded-input side).

The vertical grid is height based with uniform spacing and level 0 at the
model top: z_half(k) = z_top (K - k) / K for k = 0..K, z_full the midpoints.
The reference atmosphere is isothermal at T0: pi0(z) = exp(-g z / (cpd T0)),
theta0 = T0 / pi0 and d pi0/dz = -g pi0 / (cpd T0) evaluated at half levels.
These four reference profiles are handed to the solver as inputs (as the
vertical metric fields are in the host model), so that oracle and library
see bit-identical reference values.

Initial states follow one recipe for every workload:
  1. analytic T (T0 plus optional bumps and noise) and surface pressure p_s
     (p0 at rest; the gradient-wind balanced value for the zonal jet);
     pi_a = (p_s / p0)^(Rd/cpd) * pi0(z_full), theta_v = T / pi_a;
  2. the Exner perturbation pi' is integrated upward from its bottom value so
     that every column is discretely hydrostatic for the solver's vertical
     pressure-gradient/buoyancy balance (the state is "balanced");
  3. rho from the equation of state, vn from the jet plus noise, w = 0.
Draw order of the PCG64 stream: vn noise (K, E), then temperature noise
(K, C), then bump centres (n_bumps x 3 normals, normalised).

Nothing of the time step's arithmetic lives here.
"""
from __future__ import annotations

import numpy as np

# physical constants of the dry, shallow, traditional atmosphere
GRAV = 9.80665
RD = 287.04
CPD = 1004.64
CVD = CPD - RD
P0 = 1.0e5
T0 = 250.0
OMEGA = 7.29212e-5


def vertical(n_lev: int, z_top: float):
    k = np.arange(n_lev + 1, dtype=np.float64)
    z_half = z_top * (n_lev - k) / n_lev
    z_full = 0.5 * (z_half[:-1] + z_half[1:])
    return z_half, z_full


def reference(z_half, z_full):
    """Isothermal reference column at T0."""
    ex_full = np.exp(-GRAV * z_full / (CPD * T0))
    ex_half = np.exp(-GRAV * z_half / (CPD * T0))
    return {
        "exner_ref_full": ex_full,
        "theta_ref_full": T0 / ex_full,
        "theta_ref_half": T0 / ex_half,
        "dexner_dz_ref_half": -GRAV * ex_half / (CPD * T0),
    }


def _surface_pressure_jet(lat, u0, radius):
    """Closed-form gradient-wind balance of u = u0 cos^2(lat) at constant T0; p_s(pole) = p0."""
    cl = np.cos(lat)
    return P0 * np.exp((radius / (RD * T0)) * (2.0 * OMEGA * u0 * cl**3 / 3.0 + u0**2 * cl**4 / (4.0 * radius)))


def initial_state(
    grid,
    n_lev: int,
    z_top: float,
    seed: int,
    vn_sigma: float = 0.0,
    t_sigma: float = 0.0,
    jet_u0: float = 0.0,
    n_bumps: int = 0,
    bump_amp: float = 1.0,
    bump_radius: float = 500.0e3,
    t_profile=None,
):
    """Return (state dict of float64 arrays, vertical dict).

    state: vn (K, E), w (K+1, C), rho, exner, theta_v (K, C); unpadded, [level][entity].
    """
    rng = np.random.default_rng(seed)
    ne, nc = grid["n_edges"], grid["n_cells"]
    radius = grid["radius"]
    z_half, z_full = vertical(n_lev, z_top)
    ref = reference(z_half, z_full)

    vn_noise = rng.normal(0.0, vn_sigma, size=(n_lev, ne)) if vn_sigma > 0 else None
    t_noise = rng.normal(0.0, t_sigma, size=(n_lev, nc)) if t_sigma > 0 else None
    centres = None
    if n_bumps > 0:
        centres = rng.normal(size=(n_bumps, 3))
        centres /= np.linalg.norm(centres, axis=1, keepdims=True)

    xc = grid["cell_xyz"]
    lat_c = np.arcsin(np.clip(xc[:, 2], -1.0, 1.0))

    # 1. analytic temperature and surface pressure
    temp = np.full((n_lev, nc), T0)
    if centres is not None:
        dist = radius * np.arctan2(
            np.linalg.norm(np.cross(xc[:, None, :], centres[None, :, :]), axis=2),
            xc @ centres.T,
        )
        temp = temp + bump_amp * np.exp(-((dist / bump_radius) ** 2)).sum(axis=1)[None, :]
    if t_noise is not None:
        temp = temp + t_noise
    if t_profile is not None:  # horizontally uniform temperature offset per level
        temp = temp + np.asarray(t_profile, dtype=np.float64)[:, None]
    if jet_u0 != 0.0:
        ps = _surface_pressure_jet(lat_c, jet_u0, radius)
        fac = (ps / P0) ** (RD / CPD)
    else:
        fac = np.ones(nc)
    pi_a = fac[None, :] * ref["exner_ref_full"][:, None]
    theta_v = temp / pi_a

    # 2. discrete hydrostatic pi' from the bottom value, upward
    th_pr = theta_v - ref["theta_ref_full"][:, None]
    ex_pr = np.empty((n_lev, nc))
    ex_pr[n_lev - 1] = pi_a[n_lev - 1] - ref["exner_ref_full"][n_lev - 1]
    for k in range(n_lev - 1, 0, -1):
        th_pr_ic = 0.5 * (th_pr[k - 1] + th_pr[k])
        th_ic = ref["theta_ref_half"][k] + th_pr_ic
        dzk = z_full[k - 1] - z_full[k]
        ex_pr[k - 1] = ex_pr[k] - dzk * th_pr_ic * ref["dexner_dz_ref_half"][k] / th_ic
    exner = ref["exner_ref_full"][:, None] + ex_pr

    # 3. density from the equation of state, winds
    rho = P0 * exner ** (CVD / RD) / (RD * theta_v)
    vn = np.zeros((n_lev, ne))
    if jet_u0 != 0.0:
        xe = grid["edge_xyz"]
        nrm = grid["edge_normal_xyz"]
        cosl = np.sqrt(xe[:, 0] ** 2 + xe[:, 1] ** 2)
        # u0 cos^2(lat) * e_east . n, with e_east = (-y, x, 0) / cos(lat)
        vn = vn + (jet_u0 * cosl * (-xe[:, 1] * nrm[:, 0] + xe[:, 0] * nrm[:, 1]))[None, :]
    if vn_noise is not None:
        vn = vn + vn_noise
    w = np.zeros((n_lev + 1, nc))
    state = {"vn": vn, "w": w, "rho": rho, "exner": exner, "theta_v": theta_v}
    vert = {"z_half": z_half, "z_full": z_full, **ref}
    return state, vert


def add_cold_pools(state, n_cells: int, n_levels: int, d_theta: float, seed: int):
    """Copy of `state` with cold pools: n_cells cells drawn without
    replacement (PCG64 with `seed`) have theta_v lowered by d_theta in their
    n_levels lowest levels, rho raised so that rho * theta_v, and with it the
    pressure and exner of the equation of state, is unchanged.  Strong
    near-surface temperature contrasts of this kind are what the diffusion's
    near-surface coefficient floor acts on."""
    out = {k: v.copy() for k, v in state.items()}
    n_lev, nc = out["rho"].shape
    cells = np.random.default_rng(seed).choice(nc, n_cells, replace=False)
    for k in range(n_lev - n_levels, n_lev):
        th = out["theta_v"][k, cells]
        cold = th - d_theta
        out["rho"][k, cells] *= th / cold
        out["theta_v"][k, cells] = cold
    return out
