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


# ----------------------------------------------------------------------------
# optional operators of the fuller ICON discretisation (Section 4.1: the
# dynamical core keeps ICON's numerics): least-squares cell gradients and
# the second-order upwind (Miura) edge values of cell scalars, and the
# tangential wind by radial-basis-function vector reconstruction
# ----------------------------------------------------------------------------
def tangent_basis(x):
    """Two orthonormal vectors spanning the tangent plane at each unit vector
    x (N, 3): e1 = normalize(a x x) with a = z_hat (x_hat near the poles),
    e2 = x x e1."""
    a = np.where(np.abs(x[:, 2:3]) < 0.9, np.array([[0.0, 0.0, 1.0]]), np.array([[1.0, 0.0, 0.0]]))
    e1 = np.cross(a, x)
    e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
    e2 = np.cross(x, e1)
    return e1, e2


def cell_gradient_weights(g):
    """(C, 3, 3) weights W of the least-squares gradient at the cell centres:
    grad q_c = sum_i W[c, :, i] (q_{c2e2c[c][i]} - q_c), a vector in the
    tangent plane at x_c (per metre).  It minimises
    sum_i (grad . d_i - (q_i - q_c))^2 with d_i the neighbour's offset
    R (x_i - x_c) projected on that plane, so it reproduces every field that
    is linear in the plane's coordinates exactly."""
    e1, e2 = tangent_basis(g.xc)
    E = np.stack([e1, e2], axis=2)                      # (C, 3, 2)
    d = g.radius * (g.xc[g.c2e2c] - g.xc[:, None, :])   # (C, 3 nbrs, 3)
    D = np.einsum("cij,cjk->cik", d, E)                 # (C, 3 nbrs, 2): plane coordinates
    return np.einsum("cjk,cki->cji", E, np.linalg.pinv(D))  # (C, 3, 3 nbrs)


def cell_gradient(g, q, wts=None):
    """Least-squares gradient (K, C, 3) of a cell field q (K, C)."""
    if wts is None:
        wts = cell_gradient_weights(g)
    dq = q[:, g.c2e2c] - q[:, :, None]                  # (K, C, 3 nbrs)
    return np.einsum("cji,kci->kcj", wts, dq)


def miura_edge(g, q, vn, vt, dtau, wts=None):
    """Second-order upwind edge value of the cell scalar q (K, C) for the
    normal and tangential winds vn, vt (K, E) over dtau: the value at the
    departure point x* = R x_e - dtau (vn n_e + vt t_e) of the edge
    midpoint, extrapolated linearly with the least-squares gradient of the
    upwind cell (c0 when vn >= 0, the normal pointing c0 -> c1, else c1):
        q_e = q_up + grad q_up . (x* - R x_up)."""
    K = q.shape[0]
    grad = cell_gradient(g, q, wts)
    up = np.where(vn >= 0.0, g.e2c[:, 0][None, :], g.e2c[:, 1][None, :])  # (K, E)
    k = np.arange(K)[:, None]
    xstar = g.radius * g.xe[None] - dtau * (vn[..., None] * g.nrm[None] + vt[..., None] * g.tan[None])
    off = xstar - g.radius * g.xc[up]
    return q[k, up] + np.einsum("kej,kej->ke", grad[k, up], off)


def rbf_vt_weights(g, scale=0.5):
    """(E, 5) weights of the tangential wind by vector radial-basis-function
    interpolation over the edge and its four e2c2e neighbours (stencil order
    [e, e2c2e[e][0..3]]): the field v(x) = sum_j a_j phi(|x - x_j|) n_j + c,
    c a constant vector in the tangent plane at x_e, takes the normal winds
    at the stencil's midpoints (v(x_i) . n_i = vn_i) with sum_j a_j (n_j . b) = 0
    for both tangent directions b; vt_e = v(x_e) . t_e.  Kernel: the inverse
    multiquadric phi(r) = (1 + (r / eps)^2)^(-1/2), eps = scale * l_e;
    positions in metres.  The constant term makes the reconstruction exact
    for every flow that is uniform in the tangent plane at the edge."""
    R = g.radius
    st = np.concatenate([np.arange(g.ne)[:, None], g.e2c2e], axis=1)  # (E, 5)
    x = R * g.xe[st]                                                  # (E, 5, 3)
    n = g.nrm[st]
    eps = scale * g.l_e
    def phi(r):
        return 1.0 / np.sqrt(1.0 + (r / eps[:, None, None]) ** 2)
    r = np.linalg.norm(x[:, :, None, :] - x[:, None, :, :], axis=3)  # (E, 5, 5)
    A = phi(r) * np.einsum("eik,ejk->eij", n, n)
    e1, e2 = tangent_basis(g.xe)
    B = np.stack([np.einsum("eik,ek->ei", n, e1), np.einsum("eik,ek->ei", n, e2)], axis=2)  # (E, 5, 2)
    M = np.zeros((g.ne, 7, 7))
    M[:, :5, :5] = A
    M[:, :5, 5:] = B
    M[:, 5:, :5] = np.transpose(B, (0, 2, 1))
    # right-hand side: the evaluation functional v(x_e) . t_e
    re = np.linalg.norm(x - R * g.xe[:, None, :], axis=2)              # (E, 5)
    b = np.zeros((g.ne, 7))
    b[:, :5] = (1.0 / np.sqrt(1.0 + (re / eps[:, None]) ** 2)) * np.einsum("eik,ek->ei", n, g.tan)
    b[:, 5] = np.einsum("ek,ek->e", g.tan, e1)
    b[:, 6] = np.einsum("ek,ek->e", g.tan, e2)
    # M is symmetric: the weights of vn are the first five entries of M^-1 b
    return np.linalg.solve(M, b[:, :, None])[:, :5, 0]


def recon_vt_rbf(g, F, wts=None):
    """Tangential wind (K, E) of the normal field F (K, E) by the RBF weights."""
    if wts is None:
        wts = rbf_vt_weights(g)
    st = np.concatenate([np.arange(g.ne)[:, None], g.e2c2e], axis=1)
    return np.einsum("es,kes->ke", wts, F[:, st])
