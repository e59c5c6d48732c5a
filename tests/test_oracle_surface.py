"""Pins of the oracle's surface term (the Remark after Eq. (5): the Hadamard
product with alpha = 0 on facet cubature nodes).

The facet operator is the quadrature-weighted interpolation to the facet,
so the pins are what interpolation and the two-point flux fix: the Lagrange
end values reproduce polynomials, the product flux turns the facet rows into
an interpolated polynomial times the facet state, GLL end values pick the
boundary nodes, a constant state gives the weighted physical flux, and for
the entropy-conservative Euler flux the entropy-weighted sums telescope into
entropy potentials (Tadmor's identity summed over every facet-volume pair).
"""
import numpy as np
import pytest
from numpy.polynomial import polynomial as P

from test_oracle_flux import _entropy_vars, _rand_states, GAMMA


def tangential(n, d, m):
    """(index arrays) of the facet nodes of direction m: for t = 0..n^(d-1)-1
    the node indices (i_0, .., i_{d-1}) with i_m left out, first fastest."""
    others = [k for k in range(d) if k != m]
    T = n ** (d - 1)
    idx = np.zeros((T, d), dtype=int)
    for t in range(T):
        r = t
        for k in others:
            idx[t, k] = r % n
            r //= n
    return idx, others


@pytest.mark.parametrize("n", [2, 3, 5, 8, 13])
@pytest.mark.parametrize("kind", ["gl", "gll"])
def test_lagrange_end_values_reproduce_polynomials(orc, n, kind):
    x, _ = orc.nodes(n, kind)
    lm, lp = orc.lagrange_endpoints(n, kind)
    for j in range(n):
        assert abs(lm @ x ** j - (-1.0) ** j) < 1e-13 * n
        assert abs(lp @ x ** j - 1.0) < 1e-13 * n
    if kind == "gll":
        assert np.array_equal(np.abs(lm), np.eye(n)[0]) and np.array_equal(np.abs(lp), np.eye(n)[-1])


@pytest.mark.parametrize("n,d", [(3, 2), (4, 3), (5, 3), (6, 2)])
@pytest.mark.parametrize("kind", ["gl", "gll"])
def test_product_flux_facet_rows_interpolate(orc, n, d, kind):
    """f(a, b) = a b: y_face[t] = u_face[t] w_perp(t) p(facet point t) for
    volume data sampled from a polynomial p of degree n - 1 per direction,
    with p at the facet point evaluated by numpy."""
    rng = np.random.default_rng(n + 7 * d)
    x, w = orc.nodes(n, kind)
    coef = rng.normal(size=(n,) * d)                  # coef[i_x, i_y(, i_z)]
    E = 2
    grid = np.meshgrid(*([x] * d), indexing="ij")      # grid[k][i_x, i_y, ..]
    if d == 2:
        vals = P.polyval2d(grid[0], grid[1], coef)
    else:
        vals = P.polyval3d(grid[0], grid[1], grid[2], coef)
    u = np.stack([vals.transpose().ravel()] * E)[None]          # node = i_x + n i_y (+ n^2 i_z)
    uf = rng.uniform(0.5, 2.0, size=(1, E, 2 * d, n ** (d - 1)))
    _, yf = orc.surface(u, uf, n, d, "product", nodes_kind=kind)
    for m in range(d):
        idx, others = tangential(n, d, m)
        for s, xm in ((0, -1.0), (1, 1.0)):
            pt = np.zeros((idx.shape[0], d))
            for k in range(d):
                pt[:, k] = xm if k == m else x[idx[:, k]]
            pv = P.polyval2d(pt[:, 0], pt[:, 1], coef) if d == 2 else P.polyval3d(pt[:, 0], pt[:, 1], pt[:, 2], coef)
            wp = np.prod([w[idx[:, k]] for k in others], axis=0)
            ref = uf[0, :, 2 * m + s, :] * (wp * pv)[None, :]
            got = yf[0, :, 2 * m + s, :]
            assert np.abs(got - ref).max() < 1e-12 * max(1.0, np.abs(ref).max()), (m, s)


@pytest.mark.parametrize("n,d", [(3, 2), (4, 3)])
def test_gll_product_flux_hits_boundary_nodes_only(orc, n, d):
    """GLL end values are unit vectors: with u_face = 1 the volume output is
    u times the sum of w_perp over the facets the node lies on (interior 0)."""
    rng = np.random.default_rng(5)
    x, w = orc.nodes(n, "gll")
    u = rng.uniform(0.5, 2.0, size=(1, 3, n ** d))
    uf = np.ones((1, 3, 2 * d, n ** (d - 1)))
    yv, _ = orc.surface(u, uf, n, d, "product", nodes_kind="gll")
    for node in range(n ** d):
        ii = [(node // n ** k) % n for k in range(d)]
        s = 0.0
        for m in range(d):
            wp = np.prod([w[ii[k]] for k in range(d) if k != m])
            s += wp * ((ii[m] == 0) + (ii[m] == n - 1))
        np.testing.assert_allclose(yv[0, :, node], u[0, :, node] * s, rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("kind", ["gl", "gll"])
def test_constant_state_gives_weighted_physical_flux(orc, kind):
    n, d = 4, 3
    rng = np.random.default_rng(8)
    st = _rand_states(rng, 1)[0]
    _, w = orc.nodes(n, kind)
    lm, lp = orc.lagrange_endpoints(n, kind)
    u = np.broadcast_to(st[:, None, None], (5, 2, n ** 3)).copy()
    uf = np.broadcast_to(st[:, None, None, None], (5, 2, 6, n * n)).copy()
    yv, yf = orc.surface(u, uf, n, d, "euler", nodes_kind=kind)
    for m in range(3):
        f = orc.physical_flux_euler(st, m, GAMMA)
        idx, others = tangential(n, d, m)
        wp = np.prod([w[idx[:, k]] for k in others], axis=0)
        for s in range(2):
            ref = f[:, None, None] * wp[None, None, :]
            assert np.abs(yf[:, :, 2 * m + s, :] - ref).max() < 1e-13 * np.abs(f).max()
    # volume side: each node gets sum over faces of w_perp l_s[k] f_m
    for node in [0, 5, n ** 3 - 1]:
        ii = [(node // n ** k) % n for k in range(3)]
        ref = np.zeros(5)
        for m in range(3):
            wp = np.prod([w[ii[k]] for k in range(3) if k != m])
            ref += wp * (lm[ii[m]] + lp[ii[m]]) * orc.physical_flux_euler(st, m, GAMMA)
        assert np.abs(yv[:, 0, node] - ref).max() < 1e-13 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("kind", ["gl", "gll"])
def test_euler_surface_entropy_identity(orc, kind):
    """Tadmor's identity (v_f - v_v) . F = psi_m(u_f) - psi_m(u_v), summed with
    the facet weights B_f over every facet-volume pair:
      sum_f sum_t v(u_f[t]) . y_face_f[t] - sum_v v(u_v) . y_vol[v]
        = sum_f sum_t w_perp(t) (psi_m(u_f[t]) - sum_k l_s[k] psi_m(u_v[line t, k]))."""
    n, d = 4, 3
    rng = np.random.default_rng(21)
    x, w = orc.nodes(n, kind)
    lm, lp = orc.lagrange_endpoints(n, kind)
    u = _rand_states(rng, n ** 3).T[:, None, :].copy()            # (5, 1, 64)
    uf = _rand_states(rng, 6 * n * n).T.reshape(5, 1, 6, n * n).copy()
    yv, yf = orc.surface(u, uf, n, d, "euler", nodes_kind=kind)
    lhs = 0.0
    rhs = 0.0
    for node in range(n ** 3):
        v, _ = _entropy_vars(u[:, 0, node])
        lhs -= v @ yv[:, 0, node]
    for m in range(3):
        idx, others = tangential(n, d, m)
        for s, ls in ((0, lm), (1, lp)):
            f = 2 * m + s
            for t in range(n * n):
                vf, psif = _entropy_vars(uf[:, 0, f, t])
                lhs += vf @ yf[:, 0, f, t]
                wp = np.prod([w[idx[t, k]] for k in others])
                inner = 0.0
                for k in range(n):
                    ii = idx[t].copy(); ii[m] = k
                    node = ii[0] + n * ii[1] + n * n * ii[2]
                    inner += ls[k] * _entropy_vars(u[:, 0, node])[1][m]
                rhs += wp * (psif[m] - inner)
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(rhs)), (lhs, rhs)
