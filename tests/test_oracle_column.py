"""Pins of the oracle's vertically implicit column solver (CPU).

The tridiagonal matrix of the scheme is M = I + G D^T diag(beta) D diag(a_eta)
(G, beta, a_eta > 0, D the half-to-full level difference), diagonally similar
to I + (symmetric positive semi-definite): elimination without pivoting is
safe and every pivot is >= 1.  Thomas is checked against dense LU, against a
known solution, and the pivots against ratios of leading principal minors.
"""
import numpy as np
import pytest

from oracle.dycore import thomas


def _system(rng, n, courant):
    """Random tridiagonal system with the scheme's structure, n unknowns (half levels 1..n)."""
    K = n + 1
    gam = rng.uniform(0.2, 1.0, size=K + 1) * courant
    bet = rng.uniform(0.2, 1.0, size=K) * courant
    ae = rng.uniform(0.5, 2.0, size=K + 1)
    ae[0] = ae[K] = 0.0
    ks = np.arange(1, K)
    A = -gam[ks] * bet[ks - 1] * ae[ks - 1]
    B = 1.0 + gam[ks] * ae[ks] * (bet[ks - 1] + bet[ks])
    C = -gam[ks] * bet[ks] * ae[ks + 1]
    M = np.diag(B) + np.diag(A[1:], -1) + np.diag(C[:-1], 1)
    return A, B, C, M


@pytest.mark.parametrize("n", [1, 2, 3, 9, 29])
@pytest.mark.parametrize("courant", [0.01, 1.0, 40.0])
def test_thomas_matches_dense_lu(n, courant):
    rng = np.random.default_rng(n * 100 + int(courant))
    A, B, C, M = _system(rng, n, courant)
    x_true = rng.normal(size=n)
    r = M @ x_true
    x = thomas(A[:, None], B[:, None], C[:, None], r[:, None])[:, 0]
    x_lu = np.linalg.solve(M, r)
    scale = np.linalg.norm(x_lu)
    assert np.linalg.norm(x - x_lu) <= 1e-13 * scale * max(1.0, np.linalg.cond(M) / 1e3)
    assert np.linalg.norm(x - x_true) <= 1e-12 * np.linalg.norm(x_true) * max(1.0, np.linalg.cond(M) / 1e2)


@pytest.mark.parametrize("courant", [0.1, 5.0, 40.0])
def test_pivots_at_least_one(courant):
    rng = np.random.default_rng(7)
    n = 12
    _, _, _, M = _system(rng, n, courant)
    dets = [1.0] + [np.linalg.det(M[:i, :i]) for i in range(1, n + 1)]
    piv = np.array(dets[1:]) / np.array(dets[:-1])
    assert np.all(piv >= 1.0 - 1e-12)


def test_thomas_vectorised_columns_independent():
    rng = np.random.default_rng(11)
    cols = []
    for j in range(5):
        A, B, C, M = _system(rng, 6, 3.0)
        r = rng.normal(size=6)
        cols.append((A, B, C, r, np.linalg.solve(M, r)))
    A = np.stack([c[0] for c in cols], 1)
    B = np.stack([c[1] for c in cols], 1)
    C = np.stack([c[2] for c in cols], 1)
    R = np.stack([c[3] for c in cols], 1)
    X = thomas(A, B, C, R)
    for j, c in enumerate(cols):
        assert np.allclose(X[:, j], c[4], rtol=1e-13, atol=1e-14)
