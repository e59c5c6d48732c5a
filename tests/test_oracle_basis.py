"""Pins of the oracle's basis transformation (Eq. (6) and the proof of
Theorem 1): the modal basis values, the projection with P V = I, and the
d-fold Kronecker-power application, checked against library routines and
closed forms rather than against a retyped formula."""
import numpy as np
import pytest
from numpy.polynomial import legendre as npleg


def norms(n):
    return np.sqrt((2 * np.arange(n) + 1) / 2.0)


@pytest.mark.parametrize("n", [2, 3, 5, 8, 12, 16])
@pytest.mark.parametrize("kind", ["gl", "gll"])
def test_basis_values_match_numpy_legvander(orc, n, kind):
    x, _ = orc.nodes(n, kind)
    V, P = orc.basis_1d(n, kind)
    ref = npleg.legvander(x, n - 1) * norms(n)[None, :]
    assert np.abs(V - ref).max() < 1e-13 * max(1.0, np.abs(ref).max())
    assert np.abs(P @ V - np.eye(n)).max() < 1e-12
    assert np.abs(V @ P - np.eye(n)).max() < 1e-12


@pytest.mark.parametrize("n", [2, 4, 8, 16])
def test_gauss_legendre_discrete_orthonormality(orc, n):
    # GL with n nodes integrates degree 2n - 1 exactly: V^T W V = I, so P = V^T W
    _, w = orc.nodes(n, "gl")
    V, P = orc.basis_1d(n, "gl")
    assert np.abs(V.T @ np.diag(w) @ V - np.eye(n)).max() < 1e-13
    assert np.abs(P - V.T @ np.diag(w)).max() < 1e-12


@pytest.mark.parametrize("n", [3, 5, 8])
def test_gauss_lobatto_last_mode_norm(orc, n):
    # GLL integrates degree 2n - 3 exactly; the last mode's discrete squared
    # norm is 2/N for P_N (N = n - 1), i.e. (2N + 1)/N once normalised
    _, w = orc.nodes(n, "gll")
    V, _ = orc.basis_1d(n, "gll")
    G = V.T @ np.diag(w) @ V
    N = n - 1
    expect = np.eye(n)
    expect[N, N] = (2 * N + 1) / N
    assert np.abs(G - expect).max() < 1e-13


@pytest.mark.parametrize("n,d", [(2, 2), (3, 3), (4, 3), (6, 2), (8, 3)])
@pytest.mark.parametrize("kind", ["gl", "gll"])
def test_modal_to_nodal_reproduces_the_polynomial(orc, n, d, kind):
    """u(xi) = sum_k u_hat_k L_k(xi) at the node grid, evaluated by numpy's
    legval2d/legval3d (x fastest in the node index, as in the volume term)."""
    rng = np.random.default_rng(100 + n + 10 * d)
    x, _ = orc.nodes(n, kind)
    V, _ = orc.basis_1d(n, kind)
    E = 3
    uh = rng.uniform(-1, 1, (2, E, n ** d))
    u = orc.tensor_apply(uh, n, d, V)
    s = norms(n)
    for v in range(2):
        for e in range(E):
            if d == 2:
                c = uh[v, e].reshape(n, n).T * s[:, None] * s[None, :]          # c[kx, ky]
                gx, gy = np.meshgrid(x, x, indexing="xy")                        # node ix + n iy
                ref = npleg.legval2d(gx.ravel(), gy.ravel(), c)
            else:
                c = uh[v, e].reshape(n, n, n).transpose(2, 1, 0) * s[:, None, None] * s[None, :, None] * s[None, None, :]
                gz, gy, gx = np.meshgrid(x, x, x, indexing="ij")                 # node ix + n iy + n^2 iz
                ref = npleg.legval3d(gx.ravel(), gy.ravel(), gz.ravel(), c)
            assert np.abs(u[v, e] - ref).max() < 1e-13 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("n,d", [(3, 2), (5, 3), (8, 3)])
def test_projection_round_trip(orc, n, d):
    # Pi chi = I: projecting the interpolated values gives the coefficients back
    rng = np.random.default_rng(7)
    V, P = orc.basis_1d(n, "gl")
    uh = rng.normal(size=(1, 4, n ** d))
    back = orc.tensor_apply(orc.tensor_apply(uh, n, d, V), n, d, P)
    assert np.abs(back - uh).max() < 1e-12


def test_kronecker_power_tiny_brute_force(orc):
    # n = 2, d = 2 with a non-symmetric M written out entry by entry:
    # out[i + 2 j] = sum_{k, l} M[i][k] M[j][l] in[k + 2 l]
    M = np.array([[1.0, 2.0], [3.0, 5.0]])
    u = np.array([[[7.0, 11.0, 13.0, 17.0]]])
    out = orc.tensor_apply(u, 2, 2, M)[0, 0]
    a, b, c, dd = 7.0, 11.0, 13.0, 17.0      # in[0], in[1], in[2], in[3] = (k,l) = (0,0),(1,0),(0,1),(1,1)
    expect = [
        1 * 1 * a + 2 * 1 * b + 1 * 2 * c + 2 * 2 * dd,      # (i, j) = (0, 0)
        3 * 1 * a + 5 * 1 * b + 3 * 2 * c + 5 * 2 * dd,      # (1, 0)
        1 * 3 * a + 2 * 3 * b + 1 * 5 * c + 2 * 5 * dd,      # (0, 1)
        3 * 3 * a + 5 * 3 * b + 3 * 5 * c + 5 * 5 * dd,      # (1, 1)
    ]
    assert np.array_equal(out, np.array(expect))


@pytest.mark.parametrize("n,m,d", [(3, 5, 2), (4, 6, 3), (5, 8, 3), (8, 12, 3)])
@pytest.mark.parametrize("kind", ["gl", "gll"])
def test_modal_to_more_quadrature_nodes(orc, n, m, d, kind):
    """n modes evaluated on m > n nodes (over-integration): the rectangular
    Kronecker power reproduces the polynomial at the m-node grid (numpy's
    legval2d/legval3d), and the L2 projection returns the coefficients."""
    rng = np.random.default_rng(n * 13 + m + d)
    V, P = orc.basis_rect(n, m, kind)
    x, w = orc.nodes(m, kind)
    ref_V = npleg.legvander(x, n - 1) * norms(n)[None, :]
    assert np.abs(V - ref_V).max() < 1e-13 * max(1.0, np.abs(ref_V).max())
    # the quadrature of m >= n + 1 nodes integrates the mass matrix exactly: P = V^T W
    assert np.abs(P - V.T @ np.diag(w)).max() < 1e-12
    uh = rng.uniform(-1, 1, (2, 3, n ** d))
    u = orc.tensor_apply(uh, n, d, V)
    assert u.shape == (2, 3, m ** d)
    s = norms(n)
    for v in range(2):
        for e in range(3):
            if d == 2:
                c = uh[v, e].reshape(n, n).T * s[:, None] * s[None, :]
                gx, gy = np.meshgrid(x, x, indexing="xy")
                ref = npleg.legval2d(gx.ravel(), gy.ravel(), c)
            else:
                c = uh[v, e].reshape(n, n, n).transpose(2, 1, 0) * s[:, None, None] * s[None, :, None] * s[None, None, :]
                gz, gy, gx = np.meshgrid(x, x, x, indexing="ij")
                ref = npleg.legval3d(gx.ravel(), gy.ravel(), gz.ravel(), c)
            assert np.abs(u[v, e] - ref).max() < 1e-13 * max(1.0, np.abs(ref).max())
    back = orc.tensor_apply(u, m, d, P)
    assert np.abs(back - uh).max() < 1e-12


def test_rectangular_kronecker_tiny_brute_force(orc):
    # n_in = 2, n_out = 3, d = 2: out[i + 3 j] = sum_{k, l} M[i][k] M[j][l] in[k + 2 l]
    M = np.array([[1.0, 2.0], [3.0, 5.0], [7.0, 11.0]])
    u = np.array([[[2.0, 3.0, 5.0, 7.0]]])
    out = orc.tensor_apply(u, 2, 2, M)[0, 0]
    expect = np.zeros(9)
    for i in range(3):
        for j in range(3):
            for k in range(2):
                for l in range(2):
                    expect[i + 3 * j] += M[i, k] * M[j, l] * u[0, 0, k + 2 * l]
    assert np.array_equal(out, expect)
