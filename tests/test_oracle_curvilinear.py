"""Pins of the oracle's curvilinear volume term (metric-averaged two-point
flux, sum_k f_k(u_i, u_j) (Ja^m_k(i) + Ja^m_k(j)) / 2).

Identity metrics give the Cartesian term; a rotated frame rotates the
momentum result (rotational invariance of the Euler flux, the metric terms
being the rotated axes); and a constant state on a warped element whose
metric terms satisfy the discrete metric identities (conservative curl
form, built here from the oracle's own derivative matrix) gives zero.
"""
import numpy as np
import pytest

GAMMA = 1.4


def rand_state(rng, E, N):
    from paper_2306_11665_amd import workloads as W
    rho = rng.uniform(0.5, 1.5, (E, N))
    vel = rng.uniform(-0.5, 0.5, (3, E, N))
    p = rng.uniform(0.5, 1.5, (E, N))
    return W.primitives_to_conserved(rho, vel, p, GAMMA)


def test_identity_metrics_give_the_cartesian_term(orc):
    n, E = 4, 3
    rng = np.random.default_rng(1)
    u = rand_state(rng, E, n ** 3)
    Ja = np.zeros((3, 3, E, n ** 3))
    for m in range(3):
        Ja[m, m] = 1.0
    y = orc.curv_volume(u, Ja, n, "euler")
    ref = orc.dense_volume(u, n, 3, "euler")
    assert np.array_equal(y, ref)


@pytest.mark.parametrize("seed", [2, 3])
def test_rotated_frame_rotates_the_momentum(orc, seed):
    """Mapping x = R xi: J = 1, Ja^m = R e_m.  With velocities rotated by R
    the mass and energy results are unchanged and the momentum result is R
    times the Cartesian one."""
    n, E = 3, 2
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(3, 3))
    R, _ = np.linalg.qr(A)
    if np.linalg.det(R) < 0:
        R[:, 0] = -R[:, 0]
    u = rand_state(rng, E, n ** 3)
    ur = u.copy()
    ur[1:4] = np.einsum("kj,jen->ken", R, u[1:4])
    Ja = np.zeros((3, 3, E, n ** 3))
    for m in range(3):
        for k in range(3):
            Ja[m, k] = R[k, m]
    y = orc.curv_volume(ur, Ja, n, "euler")
    ref = orc.dense_volume(u, n, 3, "euler")
    scale = np.abs(ref).max()
    assert np.abs(y[0] - ref[0]).max() < 1e-13 * scale
    assert np.abs(y[4] - ref[4]).max() < 1e-13 * scale
    assert np.abs(y[1:4] - np.einsum("kj,jen->ken", R, ref[1:4])).max() < 1e-13 * scale


def curl_form_metrics(orc, n, kind, X):
    """Ja^i_n (conservative curl form) from nodal coordinates X (3, n^3) of
    one element: Ja^i_n = d_k (x_m d_j x_l) - d_j (x_m d_k x_l), (i, j, k) and
    (n, m, l) cyclic, with d_j the collocated derivative along xi_j."""
    _, _, D, _ = orc.operator_1d(n, kind)
    I = np.eye(n)
    Dxi = [np.kron(np.kron(I, I), D), np.kron(np.kron(I, D), I), np.kron(np.kron(D, I), I)]
    Ja = np.zeros((3, 3, n ** 3))
    for i in range(3):
        j, k = (i + 1) % 3, (i + 2) % 3
        for nn in range(3):
            m, l = (nn + 1) % 3, (nn + 2) % 3
            Ja[i, nn] = Dxi[k] @ (X[m] * (Dxi[j] @ X[l])) - Dxi[j] @ (X[m] * (Dxi[k] @ X[l]))
    return Ja


@pytest.mark.parametrize("kind", ["gl", "gll"])
def test_free_stream_on_warped_element(orc, kind):
    n = 5
    x, _ = orc.nodes(n, kind)
    node = np.arange(n ** 3)
    xi = np.stack([x[node % n], x[(node // n) % n], x[node // (n * n)]])
    X = xi + 0.1 * np.stack([np.sin(np.pi * xi[1]) * np.sin(1.5 * xi[2]),
                             np.sin(0.7 * xi[0] + 0.3) * np.cos(xi[2]),
                             np.cos(1.3 * xi[0]) * np.sin(np.pi * xi[1] / 2)])
    Ja = curl_form_metrics(orc, n, kind, X)[:, :, None, :]
    rng = np.random.default_rng(4)
    st = rand_state(rng, 1, 1)[:, 0, 0]
    u = np.broadcast_to(st[:, None, None], (5, 1, n ** 3)).copy()
    y = orc.curv_volume(u, Ja, n, "euler", nodes_kind=kind)
    f = max(np.abs(orc.physical_flux_euler(st, m, GAMMA)).max() for m in range(3))
    assert np.abs(y).max() < 1e-12 * f * np.abs(Ja).max()
    # and the same metrics with a non-constant state do not vanish
    u2 = rand_state(rng, 1, n ** 3)
    assert np.abs(orc.curv_volume(u2, Ja, n, "euler", nodes_kind=kind)).max() > 1e-3
