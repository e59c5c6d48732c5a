"""Pins of the oracle's entropy variables and entropy-projected facet states.

v = dU/du for the entropy U = -rho s/(gamma - 1) is checked against a
finite-difference gradient of U (not against a retyped formula); the inverse
map by the round trip; the facet states by constant data (unchanged), GLL end
nodes (the boundary value itself) and entropy variables that are polynomials
of the node coordinates, whose facet interpolation numpy evaluates exactly.
"""
import numpy as np
import pytest
from numpy.polynomial import polynomial as P

GAMMA = 1.4


def entropy(u, g=GAMMA):
    rho = u[0]; vel = u[1:4] / rho
    p = (g - 1) * (u[4] - 0.5 * rho * vel @ vel)
    return -rho * (np.log(p) - g * np.log(rho)) / (g - 1)


def states(rng, k):
    from paper_2306_11665_amd import workloads as W
    return W.primitives_to_conserved(rng.uniform(0.5, 1.5, k), rng.uniform(-0.5, 0.5, (3, k)),
                                     rng.uniform(0.5, 1.5, k), GAMMA).T


def test_entropy_vars_are_the_gradient_of_the_entropy(orc):
    rng = np.random.default_rng(1)
    for u in states(rng, 20):
        v = orc.entropy_vars(u)
        g = np.zeros(5)
        for k in range(5):
            h = 1e-6 * max(1.0, abs(u[k]))
            up, um = u.copy(), u.copy()
            up[k] += h; um[k] -= h
            g[k] = (entropy(up) - entropy(um)) / (2 * h)
        assert np.abs(v - g).max() < 1e-7 * max(1.0, np.abs(v).max())


def test_inverse_map_round_trip(orc):
    rng = np.random.default_rng(2)
    for u in states(rng, 50):
        back = orc.conserved_from_entropy(orc.entropy_vars(u))
        assert np.abs(back - u).max() < 4e-15 * np.abs(u).max()


@pytest.mark.parametrize("kind", ["gl", "gll"])
def test_constant_state_traces_unchanged(orc, kind):
    n = 5
    st = np.array([1.1, 0.2, -0.3, 0.15, 2.9])
    u = np.broadcast_to(st[:, None, None], (5, 2, n ** 3)).copy()
    uf = orc.entropy_trace(u, n, kind)
    assert np.abs(uf - st[:, None, None, None]).max() < 1e-14 * np.abs(st).max()


def test_gll_traces_are_the_boundary_values(orc):
    n = 4
    rng = np.random.default_rng(3)
    u = states(rng, n ** 3).T[:, None, :].copy()
    uf = orc.entropy_trace(u, n, "gll")
    for t in range(n * n):
        a, b = t % n, t // n
        # face x = -1 (f = 0): node (0, a, b); face z = +1 (f = 5): node (a, b, n-1)
        assert np.abs(uf[:, 0, 0, t] - u[:, 0, 0 + n * a + n * n * b]).max() < 1e-14 * 4
        assert np.abs(uf[:, 0, 5, t] - u[:, 0, a + n * b + n * n * (n - 1)]).max() < 1e-14 * 4


@pytest.mark.parametrize("kind", ["gl", "gll"])
def test_polynomial_entropy_variables_interpolate_exactly(orc, kind):
    """Nodal states whose entropy variables are polynomials of degree n - 1
    per direction: the facet state is u of the polynomial at the facet point
    (numpy evaluates it)."""
    n = 4
    x, _ = orc.nodes(n, kind)
    rng = np.random.default_rng(4)
    base = orc.entropy_vars(np.array([1.0, 0.1, -0.1, 0.05, 2.6]))
    coef = rng.normal(size=(5, n, n, n)) * 0.02
    coef[:, 0, 0, 0] += base
    node = np.arange(n ** 3)
    X, Y, Z = x[node % n], x[(node // n) % n], x[node // (n * n)]
    vnodes = np.stack([P.polyval3d(X, Y, Z, coef[k]) for k in range(5)])
    u = np.stack([orc.conserved_from_entropy(vnodes[:, i]) for i in range(n ** 3)], axis=1)[:, None, :]
    uf = orc.entropy_trace(u, n, kind)
    t = np.arange(n * n)
    a, b = x[t % n], x[t // n]
    for m in range(3):
        for s, xm in ((0, -1.0), (1, 1.0)):
            pts = [None, None, None]
            others = [k for k in range(3) if k != m]
            pts[m] = np.full(n * n, xm); pts[others[0]] = a; pts[others[1]] = b
            vf = np.stack([P.polyval3d(pts[0], pts[1], pts[2], coef[k]) for k in range(5)])
            ref = np.stack([orc.conserved_from_entropy(vf[:, i]) for i in range(n * n)], axis=1)
            assert np.abs(uf[:, 0, 2 * m + s] - ref).max() < 1e-12 * np.abs(ref).max(), (m, s)
