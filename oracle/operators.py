"""C-grid operators on the triangular icosahedral grid (oracle, test infrastructure).

The paper states that the dynamical core keeps ICON's numerical
discretisation (Section 4.1, citing Wan et al. 2013); these are the standard
triangular C-grid operators of that discretisation, with two simplifications
that are readings (arithmetic means instead of ICON's bilinear/RBF weights,
Perot reconstruction for the tangential wind).  All arrays are
[level][entity]; every operator acts level by level.

  div_c(F)   = (1/A_c) sum_i s_ci l_ei F_ei
  grad_e(p)  = (p_c1 - p_c0) / d_e
  curl_v(F)  = (1/A_v) sum_{e in v2e} sig_ve d_e F_e
  gradt_e(q) = (q_v1 - q_v0) / l_e
  lapv(F)    = grad(div F) - gradt(curl F)
  laps_c(p)  = (1/A_c) sum_i l_ei (p_{c2e2c ci} - p_c) / d_ei
  vt_e       = 1/2 (V_c0 + V_c1) . t_e,  V_c = (1/A_c) sum_i s l F (x_ei - x_c)
  avg_c(q)   = mean over the three edges of a cell
  avg_e(p)   = mean over the two cells of an edge
  ih(q)      = full -> half levels: interior means, copied end values
  fh(w)      = half -> full levels: means
"""
from __future__ import annotations

import numpy as np


def div(g, F):
    out = np.zeros((F.shape[0], g.nc))
    for i in range(3):
        e = g.c2e[:, i]
        out += g.sgn_c[:, i] * g.l_e[e] * F[:, e]
    return out / g.a_c


def grad(g, p):
    return (p[:, g.e2c[:, 1]] - p[:, g.e2c[:, 0]]) / g.d_e


def curl(g, F):
    out = np.zeros((F.shape[0], g.nv))
    for i in range(6):
        e = g.v2e[:, i]
        ok = e >= 0
        es = np.where(ok, e, 0)
        out += np.where(ok, g.sgn_v[:, i] * g.d_e[es], 0.0) * F[:, es]
    return out / g.a_v


def gradt(g, q):
    return (q[:, g.e2v[:, 1]] - q[:, g.e2v[:, 0]]) / g.l_e


def lapv(g, F):
    return grad(g, div(g, F)) - gradt(g, curl(g, F))


def laps(g, p):
    out = np.zeros_like(p)
    for i in range(3):
        e = g.c2e[:, i]
        out += g.l_e[e] * (p[:, g.c2e2c[:, i]] - p) / g.d_e[e]
    return out / g.a_c


def recon_vt(g, F):
    """Tangential wind from normal components (Perot reconstruction at cells, averaged to edges)."""
    R = g.radius
    vc = np.zeros((F.shape[0], g.nc, 3))
    for i in range(3):
        e = g.c2e[:, i]
        arm = R * (g.xe[e] - g.xc)  # (C, 3) metres
        vc += (g.sgn_c[:, i] * g.l_e[e] / g.a_c)[None, :, None] * F[:, e][:, :, None] * arm[None]
    ve = 0.5 * (vc[:, g.e2c[:, 0]] + vc[:, g.e2c[:, 1]])
    return np.einsum("kej,ej->ke", ve, g.tan)


def avg_c(g, q):
    return (q[:, g.c2e[:, 0]] + q[:, g.c2e[:, 1]] + q[:, g.c2e[:, 2]]) / 3.0


def avg_e(g, p):
    return 0.5 * (p[:, g.e2c[:, 0]] + p[:, g.e2c[:, 1]])


def ih(q):
    out = np.empty((q.shape[0] + 1,) + q.shape[1:])
    out[1:-1] = 0.5 * (q[:-1] + q[1:])
    out[0] = q[0]
    out[-1] = q[-1]
    return out


def fh(w):
    return 0.5 * (w[:-1] + w[1:])
