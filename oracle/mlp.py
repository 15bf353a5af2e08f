"""FP64 reference of the learned diffusion surrogate (test infrastructure).

The paper motivates a modular Python dynamical core with integration of
machine-learning workflows (Section 3, Section 6); the surrogate itself is a
reading of this project: an 18 -> 64 -> 64 -> 1 multilayer perceptron with exact
(erf) GELU, predicting the vn tendency of the diffusion step from stencil
features of one (edge, level).

Everything here is plain NumPy in float64: forward pass, the hand-derived
backward pass (checked against central finite differences in the tests),
mean-squared-error loss, Adam and the 18 input features written from their
definitions with the oracle's operators.
"""
from __future__ import annotations

import math

import numpy as np

from . import operators as op

N_IN, N_H = 18, 64
# features whose sign flips with the flow (all but the two geometric ratios)
FLOW_FEATURES = np.arange(16)


def gelu(x):
    return 0.5 * x * (1.0 + _erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + _erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


_erf = np.vectorize(math.erf, otypes=[np.float64])


def init_params(seed: int):
    """Kaiming-uniform (fan-in, gain sqrt(2)) weights, zero biases, float64."""
    rng = np.random.default_rng(seed)

    def ku(fan_in, shape):
        bound = math.sqrt(6.0 / fan_in)
        return rng.uniform(-bound, bound, size=shape)

    return {
        "w1": ku(N_IN, (N_IN, N_H)), "b1": np.zeros(N_H),
        "w2": ku(N_H, (N_H, N_H)), "b2": np.zeros(N_H),
        "w3": ku(N_H, (N_H,)), "b3": np.zeros(1),
    }


def forward(p, x):
    """x (B, 18) -> (y (B,), cache)."""
    z1 = x @ p["w1"] + p["b1"]
    h1 = gelu(z1)
    z2 = h1 @ p["w2"] + p["b2"]
    h2 = gelu(z2)
    y = h2 @ p["w3"] + p["b3"][0]
    return y, (x, z1, h1, z2, h2)


def loss_and_grads(p, x, t):
    """Mean squared error and its gradients with respect to every parameter."""
    y, (x, z1, h1, z2, h2) = forward(p, x)
    B = x.shape[0]
    r = y - t
    loss = float(np.mean(r * r))
    dy = 2.0 * r / B
    g = {"w3": h2.T @ dy, "b3": np.array([dy.sum()])}
    dh2 = np.outer(dy, p["w3"])
    dz2 = dh2 * gelu_grad(z2)
    g["w2"] = h1.T @ dz2
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ p["w2"].T
    dz1 = dh1 * gelu_grad(z1)
    g["w1"] = x.T @ dz1
    g["b1"] = dz1.sum(axis=0)
    return loss, g


def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); p, m, v updated in place."""
    for k in p:
        m[k] = b1 * m[k] + (1.0 - b1) * g[k]
        v[k] = b2 * v[k] + (1.0 - b2) * g[k] * g[k]
        mh = m[k] / (1.0 - b1**t)
        vh = v[k] / (1.0 - b2**t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)


def cosine_lr(step, total, lr0=1e-3, lr1=1e-5):
    return lr1 + 0.5 * (lr0 - lr1) * (1.0 + math.cos(math.pi * step / max(total, 1)))


def features(g, vn, wts=None):
    """The 18 features of every (level, edge): (K, E, 18).  Stencil values
    enter as centred pairs (mean over the two points, difference over their
    distance), so that the differences that decide the tendency are formed
    before the network's BF16 rounding:
      0 vn_e, 1 vt_e;
      2 mean of D = div vn at c0, c1,      3 (D_c1 - D_c0) / d_e;
      4 mean of Z = curl vn at v0, v1,     5 (Z_v1 - Z_v0) / l_e;
      6 mean of div L1 at c0, c1,          7 its difference / d_e;
      8 mean of curl L1 at v0, v1,         9 its difference / l_e;
        with L1 = lapv(vn) = grad D - gradt Z;
      10..13 the rhombus derivatives dvn_dt, dvt_dt, dvn_dn, dvt_dn of the
        least-squares vertex vectors;
      14 mean of Z at the opposite rhombus vertices v2, v3,
      15 (Z_v3 - Z_v2) / (their distance);
      16 l_e / mean l, 17 d_e / mean d.
    Features 0..15 are linear in vn (odd in the flow).  The plain tendency
    is nu L1 - k4 A_e^2 L2 / dt with L1 = f3 - f5, L2 = f7 - f9 and nu a
    function of f10..f13 and A_e."""
    from . import dycore as dy

    if wts is None:
        wts = dy.vertex_lsq_weights(g)
    vt = op.recon_vt(g, vn)
    D = op.div(g, vn)
    z = op.curl(g, vn)
    L1 = op.lapv(g, vn)
    dL1 = op.div(g, L1)
    cL1 = op.curl(g, L1)
    der = dy.rhombus_derivatives(g, dy.vertex_vectors(g, vn, wts))
    K, E = vn.shape
    c0, c1 = g.e2c[:, 0], g.e2c[:, 1]
    v0, v1, v2, v3 = (g.e2c2v[:, i] for i in range(4))
    f = np.empty((K, E, 18))
    f[:, :, 0] = vn
    f[:, :, 1] = vt
    f[:, :, 2], f[:, :, 3] = 0.5 * (D[:, c0] + D[:, c1]), (D[:, c1] - D[:, c0]) / g.d_e
    f[:, :, 4], f[:, :, 5] = 0.5 * (z[:, v0] + z[:, v1]), (z[:, v1] - z[:, v0]) / g.l_e
    f[:, :, 6], f[:, :, 7] = 0.5 * (dL1[:, c0] + dL1[:, c1]), (dL1[:, c1] - dL1[:, c0]) / g.d_e
    f[:, :, 8], f[:, :, 9] = 0.5 * (cL1[:, v0] + cL1[:, v1]), (cL1[:, v1] - cL1[:, v0]) / g.l_e
    for i in range(4):
        f[:, :, 10 + i] = der[i]
    f[:, :, 14] = 0.5 * (z[:, v2] + z[:, v3])
    f[:, :, 15] = (z[:, v3] - z[:, v2]) / dy.rhombus_diagonal(g)
    f[:, :, 16] = (g.l_e / g.l_e.mean())[None, :]
    f[:, :, 17] = (g.d_e / g.d_e.mean())[None, :]
    return f


def diffusion_tendency(g, p, S, dt, diffusion):
    """Target of the surrogate: (vn after the vn diffusion - vn before) / dt."""
    out = diffusion(g, p, S, dt)
    return (out["vn"] - S["vn"]) / dt
