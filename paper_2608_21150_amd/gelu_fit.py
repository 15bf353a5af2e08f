"""Coefficients of the polynomial GELU that the surrogate's inference kernels
evaluate (mlp.hip, gelu_poly).

GELU(x) = x Phi(x) with Phi the standard normal CDF.  Phi(x) - 1/2 is odd, so
Phi(x) = 1/2 + x Q(x^2) with Q smooth in s = x^2; on s in [0, T^2] the kernel
evaluates Q as a degree-8 polynomial in s (Horner with FP32 fused
multiply-adds), clamps s to T^2 beyond it and clamps Phi to [0, 1], so that
GELU(x) -> x for large x and -> 0 for very negative x.  The fit minimises the
largest GELU error x^2 |Q_fit(s) - Q(s)| by Lawson's iteratively reweighted
least squares on Chebyshev nodes.  Run this file to print the coefficients
and the largest error of the FP32 evaluation against the erf form.
"""
import numpy as np
from numpy.polynomial import polynomial as P
from scipy.special import erf

T = 4.25
DEG = 8


def fit(T=T, deg=DEG, nodes=6000, iters=40):
    S = T * T
    t = np.cos(np.linspace(0.0, np.pi, nodes))
    s = (t + 1.0) * 0.5 * S
    x = np.sqrt(s)
    q = np.where(x > 1e-7, 0.5 * erf(x / np.sqrt(2.0)) / np.maximum(x, 1e-30), 1.0 / np.sqrt(2.0 * np.pi))
    w = s + 0.02
    cf = P.polyfit(s, q, deg, w=w)
    for _ in range(iters):
        r = np.abs(s * (P.polyval(s, cf) - q)) + 1e-12
        w = w * np.sqrt(r / r.max())
        w /= w.max()
        cf = P.polyfit(s, q, deg, w=w * (s + 0.02))
    return cf.astype(np.float32)


def gelu_poly_f32(x, cf, T=T):
    """The kernel's arithmetic in FP32; a fused multiply-add rounds once."""
    f = np.float32
    x = np.asarray(x, np.float32)
    s = np.minimum(x * x, f(T * T))
    acc = np.full_like(s, cf[-1])
    for c in cf[-2::-1]:
        acc = (acc.astype(np.float64) * s + np.float64(c)).astype(np.float32)
    ph = np.clip((x.astype(np.float64) * acc + 0.5).astype(np.float32), 0.0, 1.0)
    return (x * ph).astype(np.float32)


def main():
    cf = fit()
    x = np.linspace(-12.0, 12.0, 2_400_001)
    ref = x * 0.5 * (1.0 + erf(x / np.sqrt(2.0)))
    err = np.abs(gelu_poly_f32(x, cf).astype(np.float64) - ref)
    print("constexpr float kGeluT2 = %.9ef;  // T^2" % (T * T))
    print("constexpr float kGeluQ[%d] = {%s};" % (DEG + 1, ", ".join("%.9ef" % c for c in cf)))
    print("max |GELU_poly - GELU| = %.3e at x = %.4f" % (err.max(), x[err.argmax()]))


if __name__ == "__main__":
    main()
