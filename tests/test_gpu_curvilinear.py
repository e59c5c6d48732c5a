"""GPU parity of the curvilinear volume term (metric-averaged Chandrashekar
flux) against the oracle's dense definition, on a non-symmetrically warped
mesh (analytic metric terms), with identity metrics against the Cartesian
kernel, and free-stream preservation with curl-form metric terms.

Tolerance: per variable ||y_gpu - y_ref||_inf / ||y_ref||_inf <= 1e-12.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    return torch


@pytest.fixture(scope="module")
def sf(torch_dev):
    from paper_2306_11665_amd import sfhad
    sfhad.lib()
    return sfhad


def relerr(y, ref):
    return max(np.abs(y[v] - ref[v]).max() / max(np.abs(ref[v]).max(), 1e-300) for v in range(ref.shape[0]))


def gpu(torch, sf, u, Ja, n, **kw):
    y = sf.volume_curvilinear(torch.from_numpy(np.ascontiguousarray(u)).cuda(),
                              torch.from_numpy(np.ascontiguousarray(Ja)).cuda(), n, **kw)
    torch.cuda.synchronize()
    return y.cpu().numpy()


@pytest.mark.parametrize("n", list(range(2, 11)))
@pytest.mark.parametrize("kind", ["gl", "gll"])
def test_warped_mesh_every_n(torch_dev, sf, orc, n, kind):
    from paper_2306_11665_amd import workloads as W
    E = 9 if n <= 6 else 2
    u = W.euler_state(E, n, seed=1200 + n, freestream_frac=0.25)
    Ja = W.warped_mesh_metrics(E, n, nodes=kind, amp=0.03)
    y = gpu(torch_dev, sf, u, Ja, n, nodes=kind)
    ref = orc.curv_volume(u, Ja, n, "euler", nodes_kind=kind)
    err = relerr(y, ref)
    print(f"curvilinear n={n} {kind}: {err:.2e}")
    assert err <= TOL, err


def test_identity_metrics_match_the_cartesian_kernel(torch_dev, sf):
    from paper_2306_11665_amd import workloads as W
    torch = torch_dev
    n, E = 8, 40
    u = W.euler_state(E, n, seed=5, freestream_frac=0.1)
    Ja = np.zeros((3, 3, E, n ** 3))
    for m in range(3):
        Ja[m, m] = 1.0
    y = gpu(torch, sf, u, Ja, n)
    yc = sf.volume(torch.from_numpy(u).cuda(), n, 3, "euler")
    torch.cuda.synchronize()
    assert relerr(y, yc.cpu().numpy()) <= TOL


def test_free_stream_with_curl_form_metrics(torch_dev, sf, orc):
    """Discrete metric identities (curl form) + constant state -> y = 0."""
    import test_oracle_curvilinear as T
    n, kind = 6, "gl"
    x, _ = orc.nodes(n, kind)
    node = np.arange(n ** 3)
    xi = np.stack([x[node % n], x[(node // n) % n], x[node // (n * n)]])
    X = xi + 0.1 * np.stack([np.sin(np.pi * xi[1]) * np.sin(1.5 * xi[2]),
                             np.sin(0.7 * xi[0] + 0.3) * np.cos(xi[2]),
                             np.cos(1.3 * xi[0]) * np.sin(np.pi * xi[1] / 2)])
    Ja = T.curl_form_metrics(orc, n, kind, X)[:, :, None, :]
    st = np.array([1.1, 0.2, -0.3, 0.15, 2.9])
    u = np.broadcast_to(st[:, None, None], (5, 1, n ** 3)).copy()
    y = gpu(torch_dev, sf, u, Ja, n, nodes=kind)
    f = max(np.abs(orc.physical_flux_euler(st, m)).max() for m in range(3))
    assert np.abs(y).max() < 1e-12 * f * np.abs(Ja).max()


def test_full_size_sampled(torch_dev, sf, orc):
    """The benchmark's curvilinear shape (n = 8, 32768 elements, warped mesh):
    sampled elements against the oracle."""
    from paper_2306_11665_amd import workloads as W
    w = W.WORKLOADS["euler3d_n8_gl_e32768"]
    n, E = w.n, w.E
    u = w.state()
    Ja = W.warped_mesh_metrics(E, n)
    y = gpu(torch_dev, sf, u, Ja, n)
    idx = np.sort(np.random.default_rng(13).choice(E, 10, replace=False))
    idx[-1] = E - 1
    ref = orc.curv_volume(np.ascontiguousarray(u[:, idx]), np.ascontiguousarray(Ja[:, :, idx]), n, "euler")
    assert relerr(y[:, idx], ref) <= TOL
