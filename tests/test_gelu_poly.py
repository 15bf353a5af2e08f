"""The inference kernels' polynomial GELU: its coefficients in mlp.hip are the
ones gelu_fit.py produces, and its FP32 evaluation stays within 5e-5 of the
erf form everywhere (GELU is defined with the normal CDF)."""
import os
import re

import numpy as np
from scipy.special import erf

from paper_2608_21150_amd import gelu_fit

SRC = os.path.join(os.path.dirname(__file__), "..", "paper_2608_21150_amd", "csrc", "mlp.hip")


def _kernel_constants():
    s = open(SRC).read()
    t2 = float(re.search(r"kGeluT2 = ([0-9.eE+-]+)f;", s).group(1))
    body = re.search(r"kGeluQ\[\d+\] = \{([^}]*)\}", s, re.S).group(1)
    q = np.array([float(v.strip().rstrip("f")) for v in body.split(",") if v.strip()], np.float32)
    return t2, q


def test_kernel_coefficients_are_the_fit():
    t2, q = _kernel_constants()
    assert t2 == gelu_fit.T * gelu_fit.T
    assert len(q) == gelu_fit.DEG + 1
    np.testing.assert_allclose(q, gelu_fit.fit(), rtol=1e-6, atol=0)


def test_polynomial_gelu_within_bound_of_erf_form():
    _, q = _kernel_constants()
    x = np.linspace(-20.0, 20.0, 800_001)
    ref = x * 0.5 * (1.0 + erf(x / np.sqrt(2.0)))
    g = gelu_fit.gelu_poly_f32(x, q).astype(np.float64)
    assert np.abs(g - ref).max() < 5e-5
    # limits: identity for large x, zero for very negative x, exact at 0
    assert gelu_fit.gelu_poly_f32(np.array([0.0]), q)[0] == 0.0
    np.testing.assert_allclose(gelu_fit.gelu_poly_f32(np.array([8.0, 50.0]), q), [8.0, 50.0], rtol=1e-6)
    assert np.all(gelu_fit.gelu_poly_f32(np.array([-8.0, -50.0]), q) == 0.0)
