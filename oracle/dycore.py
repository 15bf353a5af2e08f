"""The dynamical-core time step, plain FP64 NumPy (oracle, test infrastructure).

Structure from the paper (Section 4.1 and the Fig. 1 caption; Section 5.1 for
the nh_solve / nh_diff split): a time step of length dt runs nsub dynamic
substeps of length dtau = dt / nsub, then one diffusion step.  Each substep
is a predictor followed by a corrector; each of them starts with the
advective tendencies, updates the horizontal momentum with pressure gradient
and advection, and advances w and the thermodynamic state with a vertically
implicit column solver; divergence damping is applied in the corrector only.
Diffusion is Smagorinsky plus fourth-order background on vn, second order on
w.  The discretisation of each step is a reading, stated where it is coded;
symbols follow the usual non-hydrostatic ICON notation:

  state      vn [K][E], w [K+1][C], rho, exner, theta_v [K][C]
  reference  pi0, theta0 at full levels, theta0 and d pi0/dz at half levels
  pi' = exner - pi0,  theta' = theta_v - theta0

Every function takes the state as a dict of arrays and returns new arrays.
"""
from __future__ import annotations

import numpy as np

from . import operators as op
from .constants import default_params


# ----------------------------------------------------------------------------
# velocity advection (start of every predictor and corrector pass)
# ----------------------------------------------------------------------------
def tangential_wind(g, p, vn):
    """vt at the edges: Perot reconstruction, or (option vt_rbf) the RBF
    vector reconstruction of ICON's discretisation (Section 4.1)."""
    if p.get("vt_rbf", 0):
        return op.recon_vt_rbf(g, vn)
    return op.recon_vt(g, vn)


def velocity_advection(g, p, vn, w):
    """Advective tendencies (T_vn [K][E], T_w [K+1][C]) in vector-invariant form."""
    K = g.n_lev
    vt = tangential_wind(g, p, vn)
    vn_ie = op.ih(vn)
    ke_e = 0.5 * (vn * vn + vt * vt)
    ke_c = op.avg_c(g, ke_e)
    zeta_v = op.curl(g, vn)
    zeta_e = 0.5 * (zeta_v[:, g.e2v[:, 0]] + zeta_v[:, g.e2v[:, 1]])
    f_e = 2.0 * p["omega"] * g.xe[:, 2]
    w_ef = op.fh(op.avg_e(g, w))
    dvn_dz = (vn_ie[:-1] - vn_ie[1:]) / g.dz_full[:, None]
    t_vn = (zeta_e + f_e) * vt - op.grad(g, ke_c) - w_ef * dvn_dz

    t_w = np.zeros((K + 1, g.nc))
    if K >= 2:
        horiz = np.zeros((K - 1, g.nc))
        wi = w[1:K]
        for i in range(3):
            e = g.c2e[:, i]
            horiz += g.sgn_c[:, i] * g.l_e[e] * vn_ie[1:K][:, e] * (wi[:, g.c2e2c[:, i]] - wi)
        horiz *= -1.0 / (2.0 * g.a_c)
        dzc = (g.z_half[0:K - 1] - g.z_half[2:K + 1])[:, None]
        vert = -wi * (w[0:K - 1] - w[2:K + 1]) / dzc
        t_w[1:K] = horiz + vert
    return t_vn, t_w


# ----------------------------------------------------------------------------
# vertically implicit column solver
# ----------------------------------------------------------------------------
def thomas(a, b, c, r):
    """Tridiagonal solve without pivoting, vectorised over columns.

    a, b, c, r have shape (n, ncol): a[i] x[i-1] + b[i] x[i] + c[i] x[i+1] = r[i].
    """
    n = b.shape[0]
    cp = np.empty_like(b)
    dp = np.empty_like(b)
    den = b[0]
    cp[0] = c[0] / den
    dp[0] = r[0] / den
    for i in range(1, n):
        den = b[i] - a[i] * cp[i - 1]
        cp[i] = c[i] / den
        dp[i] = (r[i] - a[i] * dp[i - 1]) / den
    x = np.empty_like(b)
    x[n - 1] = dp[n - 1]
    for i in range(n - 2, -1, -1):
        x[i] = dp[i] - cp[i] * x[i + 1]
    return x


def column_coefficients(g, p, S, dtau):
    """Column quantities that depend only on the state at the start of the substep."""
    K = g.n_lev
    eta = p["eta"]
    rho, exner, th = S["rho"], S["exner"], S["theta_v"]
    ex_pr = exner - g.ex_ref[:, None]
    th_pr = th - g.th_ref[:, None]
    rho_ic = op.ih(rho)
    th_pr_ic = op.ih(th_pr)
    th_ic = g.th_ref_ic[:, None] + th_pr_ic
    a_til = th_ic * rho_ic
    a_til[0] = 0.0
    a_til[K] = 0.0
    a_eta = eta * a_til
    b = dtau * (p["rd"] / p["cvd"]) * exner / (rho * th)
    beta = b / g.dz_full[:, None]
    gamma = np.zeros((K + 1, g.nc))
    z_th = np.zeros((K + 1, g.nc))
    if K >= 2:
        dzh = g.dz_half[1:K][:, None]
        gamma[1:K] = dtau * p["cpd"] * eta * th_ic[1:K] / dzh
        z_th[1:K] = ((1.0 - eta) * th_ic[1:K] * (ex_pr[0:K - 1] - ex_pr[1:K]) / dzh
                     + th_pr_ic[1:K] * g.dex_dz_ref_ic[1:K][:, None])
    return {"ex_pr": ex_pr, "rho_ic": rho_ic, "a_til": a_til, "a_eta": a_eta,
            "b": b, "beta": beta, "gamma": gamma, "z_th": z_th}


def rayleigh_tau(g, p):
    """Sponge rate at half levels: tau0 sin^2(pi/2 (z - z_d)/(z_top - z_d)) above z_d."""
    z = g.z_half
    z_top = z[0]
    z_d = p["rayleigh_zfrac"] * z_top
    s = np.sin(0.5 * np.pi * (z - z_d) / (z_top - z_d))
    return np.where(z > z_d, p["rayleigh_tau0"] * s * s, 0.0)


def column_solve(g, p, S, cf, dm, dth, w_x, dtau):
    """Explicit parts, tridiagonal w solve, sponge, increment updates of rho, exner, theta_v."""
    K = g.n_lev
    eta = p["eta"]
    w = S["w"]
    dzf = g.dz_full[:, None]
    rw = cf["rho_ic"] * w
    aw = cf["a_til"] * w
    drho_x = -dtau * (dm + (1.0 - eta) * (rw[:-1] - rw[1:]) / dzf)
    dex_x = -cf["b"] * (dth + (1.0 - eta) * (aw[:-1] - aw[1:]) / dzf)
    e_ex = cf["ex_pr"] + dex_x

    w_new = np.zeros((K + 1, g.nc))
    if K >= 2:
        gam, bet, ae = cf["gamma"], cf["beta"], cf["a_eta"]
        ks = np.arange(1, K)
        A = -gam[ks] * bet[ks - 1] * ae[ks - 1]
        B = 1.0 + gam[ks] * ae[ks] * (bet[ks - 1] + bet[ks])
        C = -gam[ks] * bet[ks] * ae[ks + 1]
        r = w_x[ks] - gam[ks] * (e_ex[ks - 1] - e_ex[ks])
        w_new[1:K] = thomas(A, B, C, r)
        tau = rayleigh_tau(g, p)
        w_new[1:K] = w_new[1:K] / (1.0 + dtau * tau[1:K, None])

    drho = drho_x - dtau * eta * (cf["rho_ic"][:-1] * w_new[:-1] - cf["rho_ic"][1:] * w_new[1:]) / dzf
    dex = dex_x - cf["beta"] * (cf["a_eta"][:-1] * w_new[:-1] - cf["a_eta"][1:] * w_new[1:])
    rho, exner, th = S["rho"], S["exner"], S["theta_v"]
    rho_new = rho + drho
    ex_new = exner + dex
    th_new = th + (rho * th * (p["cvd"] / p["rd"]) * dex / exner - th * drho) / rho_new
    return {"w": w_new, "rho": rho_new, "exner": ex_new, "theta_v": th_new}


def mass_fluxes(g, vn, rho_e, th_e):
    fm = rho_e * vn
    ft = fm * th_e
    return op.div(g, fm), op.div(g, ft)


# ----------------------------------------------------------------------------
# predictor and corrector
# ----------------------------------------------------------------------------
def predictor(g, p, S, dtau):
    t_vn0, t_w0 = velocity_advection(g, p, S["vn"], S["w"])
    cf = column_coefficients(g, p, S, dtau)
    if p.get("miura", 0):
        # Section 4.1 keeps ICON's discretisation: the edge values of density
        # and theta_v by second-order upwind (Miura) reconstruction with the
        # substep's start winds, used for the fluxes of both passes and for
        # the pressure-gradient term
        vt = tangential_wind(g, p, S["vn"])
        wts = op.cell_gradient_weights(g)
        rho_e = op.miura_edge(g, S["rho"], S["vn"], vt, dtau, wts)
        th_e = op.miura_edge(g, S["theta_v"], S["vn"], vt, dtau, wts)
    else:
        rho_e = op.avg_e(g, S["rho"])
        th_e = op.avg_e(g, S["theta_v"])
    grad_ex = op.grad(g, cf["ex_pr"])
    vn_s = S["vn"] + dtau * (t_vn0 - p["cpd"] * th_e * grad_ex)
    dm, dth = mass_fluxes(g, vn_s, rho_e, th_e)
    w_x = S["w"] + dtau * (t_w0 - p["cpd"] * cf["z_th"])
    col = column_solve(g, p, S, cf, dm, dth, w_x, dtau)
    pred = {"vn": vn_s, **col}
    saved = {"t_vn0": t_vn0, "t_w0": t_w0, "cf": cf, "rho_e": rho_e, "th_e": th_e, "grad_ex": grad_ex}
    return pred, saved


def divergence_damping(g, vn):
    """Fourth-order damping operator grad(div(grad(div vn)))."""
    return op.grad(g, op.div(g, op.grad(g, op.div(g, vn))))


def corrector(g, p, S, pred, saved, dtau):
    t_vn1, t_w1 = velocity_advection(g, p, pred["vn"], pred["w"])
    a0, a1 = p["adv_w0"], p["adv_w1"]
    dd = divergence_damping(g, pred["vn"])
    vn_new = (S["vn"]
              + dtau * (a0 * saved["t_vn0"] + a1 * t_vn1 - p["cpd"] * saved["th_e"] * saved["grad_ex"])
              - p["divdamp_c4"] * g.mean_area**2 * dd)
    dm, dth = mass_fluxes(g, vn_new, saved["rho_e"], saved["th_e"])
    w_x = S["w"] + dtau * (a0 * saved["t_w0"] + a1 * t_w1 - p["cpd"] * saved["cf"]["z_th"])
    col = column_solve(g, p, S, saved["cf"], dm, dth, w_x, dtau)
    return {"vn": vn_new, **col}


def substep(g, p, S, dtau):
    pred, saved = predictor(g, p, S, dtau)
    return corrector(g, p, S, pred, saved, dtau)


# ----------------------------------------------------------------------------
# diffusion granule (once per time step)
# ----------------------------------------------------------------------------
def vertex_lsq_weights(g):
    """(V, 3, 6) weights of the least-squares vertex vector fitting the v2e normal winds.

    V_v minimises sum_e (V . n_e - vn_e)^2 subject to V . x_v = 0; written as
    V = P a with P an orthonormal tangent basis, a = pinv(N P) vn.
    """
    xv = g.xv
    ax = np.where(np.abs(xv[:, 0:1]) < 0.9, np.array([[1.0, 0.0, 0.0]]), np.array([[0.0, 1.0, 0.0]]))
    e1 = np.cross(ax, xv)
    e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
    e2 = np.cross(xv, e1)
    P = np.stack([e1, e2], axis=2)  # (V, 3, 2)
    ok = g.v2e >= 0
    N = np.where(ok[:, :, None], g.nrm[np.maximum(g.v2e, 0)], 0.0)  # (V, 6, 3)
    NP = N @ P  # (V, 6, 2)
    return P @ np.linalg.pinv(NP)  # (V, 3, 6)


def rhombus_diagonal(g):
    """Great-circle distance (m) between the two vertices of each edge's
    rhombus that are not on the edge."""
    v2, v3 = g.e2c2v[:, 2], g.e2c2v[:, 3]
    return g.radius * np.arctan2(np.linalg.norm(np.cross(g.xv[v2], g.xv[v3]), axis=1),
                                 np.einsum("ij,ij->i", g.xv[v2], g.xv[v3]))


def rhombus_derivatives(g, vv):
    """Derivatives of the normal and tangential wind across the rhombus of
    each edge, from the vertex vectors vv (K, V, 3): along the edge (between
    its end vertices, over l_e) and across it (between the two opposite
    vertices, over their great-circle distance).  Returns dvn_dt, dvt_dt,
    dvn_dn, dvt_dn, each (K, E)."""
    v0, v1, v2, v3 = (g.e2c2v[:, i] for i in range(4))
    big_l = rhombus_diagonal(g)
    d_t = vv[:, v1] - vv[:, v0]  # (K, E, 3)
    d_n = vv[:, v3] - vv[:, v2]
    dvn_dt = np.einsum("kej,ej->ke", d_t, g.nrm) / g.l_e
    dvt_dt = np.einsum("kej,ej->ke", d_t, g.tan) / g.l_e
    dvn_dn = np.einsum("kej,ej->ke", d_n, g.nrm) / big_l
    dvt_dn = np.einsum("kej,ej->ke", d_n, g.tan) / big_l
    return dvn_dt, dvt_dt, dvn_dn, dvt_dn


def vertex_vectors(g, vn, wts):
    """Least-squares vertex vectors (K, V, 3) of the normal winds vn."""
    ok = g.v2e >= 0
    vn_v = np.where(ok[None], vn[:, np.maximum(g.v2e, 0)], 0.0)  # (K, V, 6)
    return np.einsum("vjs,kvs->kvj", wts, vn_v)


def smagorinsky_nu(g, p, vv, dt):
    """Smagorinsky viscosity from the rhombus deformation (edges), capped for stability."""
    dvn_dt, dvt_dt, dvn_dn, dvt_dn = rhombus_derivatives(g, vv)
    deform = np.sqrt((dvn_dn - dvt_dt) ** 2 + (dvt_dn + dvn_dt) ** 2)
    return np.minimum(p["smag_cs"] * g.a_e * deform, g.a_e / (p["smag_cap"] * dt))


def near_surface_nu(g, p, th, dt):
    """Section 4.1: the theta_v diffusion coefficient is raised where the
    near-surface temperature contrast is strong.  Reading: a cell colder
    than the mean of its three neighbours by more than the threshold T
    (delta = theta_c - mean_n theta_n < -T; the reference profile is the
    same in every cell of a level here, so it drops out) gets a floor on
    its coefficient that grows linearly from 0 at delta = -T to the
    stability cap at delta = -2T and stays there:
        s = clip((-delta - T) / T, 0, 1),  floor = s * mean_e(A_e) / (smag_cap dt),
    the cap being the one of the Smagorinsky viscosity, averaged over the
    cell's edges like nu.  th holds the affected levels (the lowest ones)."""
    mean_n = (th[:, g.c2e2c[:, 0]] + th[:, g.c2e2c[:, 1]] + th[:, g.c2e2c[:, 2]]) / 3.0
    delta = th - mean_n
    thr = p["theta_enh_thresh"]
    s = np.clip((-delta - thr) / thr, 0.0, 1.0)
    cap_c = (g.a_e[g.c2e[:, 0]] + g.a_e[g.c2e[:, 1]] + g.a_e[g.c2e[:, 2]]) / 3.0 / (p["smag_cap"] * dt)
    return s * cap_c


def diffusion(g, p, S, dt, wts=None):
    if wts is None:
        wts = vertex_lsq_weights(g)
    K = g.n_lev
    vn = S["vn"]
    vv = vertex_vectors(g, vn, wts)
    nu = smagorinsky_nu(g, p, vv, dt)
    l1 = op.lapv(g, vn)
    l2 = op.lapv(g, l1)
    vn_new = vn + dt * nu * l1 - p["hdiff_k4"] * g.a_e**2 * l2
    w_new = S["w"].copy()
    if p["diffuse_w"] and K >= 2:
        nu_c = op.avg_c(g, op.ih(nu))
        lw = op.laps(g, S["w"])
        w_new[1:K] = S["w"][1:K] + dt * nu_c[1:K] * lw[1:K]
    out = dict(S)
    out["vn"] = vn_new
    out["w"] = w_new
    if p.get("diffuse_theta", 0):
        # Section 4.1: diffusion optionally acts on temperature and Exner too.
        # Reading: theta_v takes the same second-order Smagorinsky form as w,
        # at full levels with nu averaged over the cell's edges; Exner follows
        # the equation of state linearised at fixed rho, dpi/pi = (R_d/c_vd)
        # dtheta_v/theta_v, so that pressure changes only at second order.
        nu_f = op.avg_c(g, nu)
        n_enh = p.get("theta_enh_nlev", 0)
        if n_enh > 0:
            assert n_enh <= K
            nu_f[K - n_enh:] = np.maximum(nu_f[K - n_enh:],
                                          near_surface_nu(g, p, S["theta_v"][K - n_enh:], dt))
        dth = dt * nu_f * op.laps(g, S["theta_v"])
        out["theta_v"] = S["theta_v"] + dth
        out["exner"] = S["exner"] * (1.0 + p["rd"] / p["cvd"] * dth / S["theta_v"])
    return out


# ----------------------------------------------------------------------------
# time step and diagnostics
# ----------------------------------------------------------------------------
def step(g, S, dt, nsub, p=None, diffuse=True, wts=None):
    p = default_params() if p is None else p
    dtau = dt / nsub
    for _ in range(nsub):
        S = substep(g, p, S, dtau)
    if diffuse:
        S = diffusion(g, p, S, dt, wts)
    return S


def diag(g, S):
    """Total mass, theta-mass, max |w|, max |vn|, non-finite count."""
    dz = g.dz_full[:, None]
    mass = float(np.sum(g.a_c * np.sum(S["rho"] * dz, axis=0)))
    theta_mass = float(np.sum(g.a_c * np.sum(S["rho"] * S["theta_v"] * dz, axis=0)))
    nonfinite = int(sum(np.count_nonzero(~np.isfinite(S[k])) for k in ("vn", "w", "rho", "exner", "theta_v")))
    return {
        "mass": mass,
        "theta_mass": theta_mass,
        "max_abs_w": float(np.max(np.abs(S["w"]))),
        "max_abs_vn": float(np.max(np.abs(S["vn"]))),
        "n_nonfinite": nonfinite,
    }
