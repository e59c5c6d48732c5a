"""Pins of the oracle's 1D operators (nodes, weights, D, Q = W D).

Pinned against library routines and closed forms, never against the oracle
itself: numpy's Gauss-Legendre rule, scipy's Jacobi roots for the Lobatto
interior nodes, exact polynomial integration/differentiation, textbook
closed-form nodes, and the summation-by-parts property of Q (the property
that Eq. (5)'s weighted derivative relies on).
"""
import numpy as np
import pytest
from scipy.special import roots_jacobi


@pytest.mark.parametrize("n", list(range(1, 17)))
def test_gl_nodes_match_numpy(orc, n):
    x, w = orc.nodes(n, "gl")
    xr, wr = np.polynomial.legendre.leggauss(n)
    np.testing.assert_allclose(x, xr, rtol=0, atol=2e-15)
    # numpy's own weights carry up to ~5e-14 relative error at n = 15 (checked
    # against mpmath below), so the library comparison is at 1e-13
    np.testing.assert_allclose(w, wr, rtol=1e-13, atol=0)


@pytest.mark.parametrize("n", [5, 8, 12, 15, 16])
def test_gl_weights_mpmath(orc, n):
    """Weights 2 / ((1-x^2) P_n'(x)^2) at 40 digits on mpmath-polished roots."""
    import mpmath as mp
    mp.mp.dps = 40
    x, w = orc.nodes(n, "gl")
    P = lambda t: mp.legendre(n, t)
    for i in range(n):
        xm = mp.findroot(P, mp.mpf(float(x[i])))
        wm = 2 / ((1 - xm ** 2) * mp.diff(P, xm) ** 2)
        assert abs(float(x[i] - xm)) < 1e-16
        assert abs(float((w[i] - wm) / wm)) < 1e-14


@pytest.mark.parametrize("n", list(range(2, 17)))
def test_gll_nodes_match_jacobi_roots(orc, n):
    x, w = orc.nodes(n, "gll")
    interior = np.sort(roots_jacobi(n - 2, 1, 1)[0]) if n > 2 else np.zeros(0)
    xr = np.concatenate([[-1.0], interior, [1.0]])
    np.testing.assert_allclose(x, xr, rtol=0, atol=4e-15)
    # weights from the closed form 2 / (N (N+1) P_N(x)^2), N = n-1, with numpy's Legendre
    N = n - 1
    PN = np.polynomial.legendre.Legendre.basis(N)(xr)
    np.testing.assert_allclose(w, 2.0 / (N * (N + 1) * PN ** 2), rtol=3e-14)


def test_closed_form_nodes(orc):
    # textbook closed forms
    x, w = orc.nodes(3, "gl")
    np.testing.assert_allclose(x, [-np.sqrt(0.6), 0.0, np.sqrt(0.6)], atol=1e-16)
    np.testing.assert_allclose(w, [5 / 9, 8 / 9, 5 / 9], rtol=1e-15)
    x, w = orc.nodes(4, "gll")
    np.testing.assert_allclose(x, [-1, -1 / np.sqrt(5), 1 / np.sqrt(5), 1], atol=1e-16)
    np.testing.assert_allclose(w, [1 / 6, 5 / 6, 5 / 6, 1 / 6], rtol=1e-15)
    x, w = orc.nodes(3, "gll")
    np.testing.assert_allclose(x, [-1, 0, 1], atol=1e-16)
    np.testing.assert_allclose(w, [1 / 3, 4 / 3, 1 / 3], rtol=1e-15)


@pytest.mark.parametrize("kind,exact_deg", [("gl", lambda n: 2 * n - 1), ("gll", lambda n: 2 * n - 3)])
@pytest.mark.parametrize("n", [2, 3, 4, 5, 8, 12, 16])
def test_quadrature_exactness(orc, kind, exact_deg, n):
    x, w = orc.nodes(n, kind)
    for k in range(exact_deg(n) + 1):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, x ** k) - exact) < 1e-14 * max(1.0, n), (k, n, kind)


@pytest.mark.parametrize("kind", ["gl", "gll"])
@pytest.mark.parametrize("n", [2, 3, 4, 5, 8, 12, 16])
def test_D_differentiates_polynomials_exactly(orc, kind, n):
    x, w, D, Q = orc.operator_1d(n, kind)
    scale = np.abs(D).max()
    for k in range(n):
        d = D @ (x ** k)
        ref = k * x ** (k - 1) if k > 0 else np.zeros(n)
        assert np.abs(d - ref).max() <= 2e-14 * scale * max(1, k), (n, kind, k)
    assert np.abs(D @ np.ones(n)).max() <= 4e-15 * scale
    np.testing.assert_array_equal(Q, np.diag(w) @ D)


def _lagrange_at(x, t):
    """Values l_j(t) of the Lagrange basis on nodes x (direct product formula)."""
    n = len(x)
    out = np.ones(n)
    for j in range(n):
        for k in range(n):
            if k != j:
                out[j] *= (t - x[k]) / (x[j] - x[k])
    return out


@pytest.mark.parametrize("kind", ["gl", "gll"])
@pytest.mark.parametrize("n", [2, 3, 4, 5, 8, 12, 16])
def test_Q_summation_by_parts(orc, kind, n):
    """Q + Q^T = t_R t_R^T - t_L t_L^T (t = Lagrange values at +1 / -1)."""
    x, w, D, Q = orc.operator_1d(n, kind)
    tR = _lagrange_at(x, 1.0)
    tL = _lagrange_at(x, -1.0)
    B = np.outer(tR, tR) - np.outer(tL, tL)
    err = np.abs(Q + Q.T - B).max()
    assert err <= 1e-15 * n * n * np.abs(Q).max(), err
    if kind == "gll":
        np.testing.assert_allclose(np.diag(B), np.r_[-1.0, np.zeros(n - 2), 1.0], atol=1e-14)


def test_diff_matrix_mpmath(orc):
    """D against mpmath differentiation (50 digits) of the Lagrange product formula."""
    import mpmath as mp
    mp.mp.dps = 50
    for n, kind in [(4, "gl"), (5, "gll"), (8, "gl")]:
        x, w = orc.nodes(n, kind)
        D = orc.diff_matrix(x)
        xs = [mp.mpf(float(v)) for v in x]
        for j in range(n):
            denom = mp.fprod([xs[j] - xs[k] for k in range(n) if k != j])
            lj = lambda t, j=j, denom=denom: mp.fprod([t - xs[k] for k in range(n) if k != j]) / denom
            for i in range(n):
                ref = mp.diff(lj, xs[i])
                assert abs(float(ref) - D[i, j]) <= 1e-13 * max(1.0, abs(float(ref))), (n, kind, i, j)
