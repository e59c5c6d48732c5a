"""GPU parity of the surface term (the Remark after Eq. (5): alpha = 0 on the
facet cubature nodes) and of the fused volume + surface pass, against the
oracle's dense definitions (every facet-volume pair, explicit Kronecker
facet operators).

Tolerance: per variable ||y_gpu - y_ref||_inf / ||y_ref||_inf <= 1e-12 for
both y_vol and y_face.  Facet states: independent random states of the
volume-state distribution, traces interpolated from the volume state (the
near-equal regime of smooth data), and constant states.
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


def states(flux, E, n, d, seed, faces=False):
    from paper_2306_11665_amd import workloads as W
    k = 2 * d * n ** (d - 1) if faces else n ** d
    if flux == "euler":
        rng = np.random.default_rng(seed)
        rho = rng.uniform(0.5, 1.5, (E, k))
        vel = rng.uniform(-0.5, 0.5, (3, E, k))
        p = rng.uniform(0.5, 1.5, (E, k))
        u = W.primitives_to_conserved(rho, vel, p)
    elif flux == "product":
        u = np.random.default_rng(seed).uniform(1e-8, 30.0, (1, E, k))
    else:
        u = np.random.default_rng(seed).uniform(-1.0, 1.0, (1, E, k))
    if faces:
        return np.ascontiguousarray(u.reshape(u.shape[0], E, 2 * d, n ** (d - 1)))
    return np.ascontiguousarray(u)


def gpu_surface(torch, sf, u, uf, n, d, flux, **kw):
    ut = torch.from_numpy(u).cuda()
    uft = torch.from_numpy(uf).cuda()
    yv, yf = sf.surface(ut, uft, n, d, flux, **kw)
    torch.cuda.synchronize()
    return yv.cpu().numpy(), yf.cpu().numpy()


@pytest.mark.parametrize("n", list(range(2, 14)))
@pytest.mark.parametrize("kind", ["gl", "gll"])
def test_euler_surface_every_n(torch_dev, sf, orc, n, kind):
    E = 37 if n <= 5 else (9 if n <= 9 else 3)
    u = states("euler", E, n, 3, seed=600 + n)
    uf = states("euler", E, n, 3, seed=700 + n, faces=True)
    yv, yf = gpu_surface(torch_dev, sf, u, uf, n, 3, "euler", nodes=kind)
    rv, rf = orc.surface(u, uf, n, 3, "euler", nodes_kind=kind)
    ev, ef = relerr(yv, rv), relerr(yf, rf)
    print(f"euler n={n} {kind}: y_vol {ev:.2e} y_face {ef:.2e}")
    assert ev <= TOL and ef <= TOL, (ev, ef)


@pytest.mark.parametrize("flux,d,n", [("burgers", 2, 4), ("burgers", 3, 5), ("product", 2, 16), ("product", 3, 8),
                                      ("product", 3, 16), ("burgers", 2, 13)])
def test_scalar_surface(torch_dev, sf, orc, flux, d, n):
    E = 23 if n ** d <= 512 else 2
    u = states(flux, E, n, d, seed=800 + n)
    uf = states(flux, E, n, d, seed=900 + n, faces=True)
    for kind in ("gl", "gll"):
        yv, yf = gpu_surface(torch_dev, sf, u, uf, n, d, flux, nodes=kind)
        rv, rf = orc.surface(u, uf, n, d, flux, nodes_kind=kind)
        assert relerr(yv, rv) <= TOL and relerr(yf, rf) <= TOL, (kind, relerr(yv, rv), relerr(yf, rf))


def traces(u, n, lm, lp):
    """Facet states interpolated from the volume state (3D)."""
    nv, E, _ = u.shape
    U = u.reshape(nv, E, n, n, n)                       # [v, e, iz, iy, ix]
    uf = np.zeros((nv, E, 6, n * n))
    for s, l in ((0, lm), (1, lp)):
        uf[:, :, 0 + s] = np.einsum("veabk,k->veab", U, l).reshape(nv, E, n * n)   # x faces: t = iy + n iz
        uf[:, :, 2 + s] = np.einsum("veakb,k->veab", U, l).reshape(nv, E, n * n)   # y faces: t = ix + n iz
        uf[:, :, 4 + s] = np.einsum("vekab,k->veab", U, l).reshape(nv, E, n * n)   # z faces: t = ix + n iy
    return np.ascontiguousarray(uf)


def test_traces_and_free_stream(torch_dev, sf, orc):
    """Facet states equal to the interpolated trace of smooth (linear) or
    constant volume data: the near-equal log-mean branch on the facet pairs.
    (Random per-node data would interpolate to non-physical traces.)"""
    from paper_2306_11665_amd import workloads as W
    n, E = 6, 8
    x, _ = orc.nodes(n, "gl")
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")           # node = ix + n iy + n^2 iz
    X, Y, Z = X.ravel(), Y.ravel(), Z.ravel()
    rng = np.random.default_rng(31)
    rho = np.zeros((E, n ** 3)); p = np.zeros((E, n ** 3)); vel = np.zeros((3, E, n ** 3))
    for e in range(E):
        amp = 0.0 if e % 2 else 0.2                           # every other element constant
        g = rng.uniform(-1, 1, (5, 3)) * amp
        rho[e] = 1.0 + g[0] @ np.stack([X, Y, Z])
        p[e] = 1.0 + g[1] @ np.stack([X, Y, Z])
        for k in range(3):
            vel[k, e] = 0.1 * (k + 1) + g[2 + k] @ np.stack([X, Y, Z])
    u = np.ascontiguousarray(W.primitives_to_conserved(rho, vel, p))
    lm, lp = orc.lagrange_endpoints(n, "gl")
    uf = traces(u, n, lm, lp)
    yv, yf = gpu_surface(torch_dev, sf, u, uf, n, 3, "euler")
    rv, rf = orc.surface(u, uf, n, 3, "euler")
    assert np.isfinite(rv).all() and np.isfinite(rf).all()
    assert relerr(yv, rv) <= TOL and relerr(yf, rf) <= TOL, (relerr(yv, rv), relerr(yf, rf))


def test_fused_volume_and_surface(torch_dev, sf, orc):
    torch = torch_dev
    for n, kind in ((4, "gl"), (7, "gll"), (8, "gl")):
        E = 11
        u = states("euler", E, n, 3, seed=40 + n)
        uf = states("euler", E, n, 3, seed=50 + n, faces=True)
        yv, yf = gpu_surface(torch, sf, u, uf, n, 3, "euler", nodes=kind, with_volume=True)
        rv, rf = orc.surface(u, uf, n, 3, "euler", nodes_kind=kind)
        rv = rv + orc.dense_volume(u, n, 3, "euler", nodes_kind=kind)
        assert relerr(yv, rv) <= TOL and relerr(yf, rf) <= TOL, (n, relerr(yv, rv), relerr(yf, rf))


def test_full_size_sampled(torch_dev, sf, orc):
    """At the benchmark's shape (n = 8, 32768 elements, fused pass): sampled
    elements against the oracle."""
    torch = torch_dev
    from paper_2306_11665_amd import workloads as W
    w = W.WORKLOADS["euler3d_n8_gl_e32768"]
    n, E = w.n, w.E
    u = w.state()
    uf = states("euler", E, n, 3, seed=77, faces=True)
    yv, yf = gpu_surface(torch, sf, u, uf, n, 3, "euler", with_volume=True)
    idx = np.sort(np.random.default_rng(12).choice(E, 24, replace=False))
    idx[-1] = E - 1
    us, ufs = np.ascontiguousarray(u[:, idx]), np.ascontiguousarray(uf[:, idx])
    rv, rf = orc.surface(us, ufs, n, 3, "euler")
    rv = rv + orc.sf_volume(us, n, 3, "euler")
    assert relerr(yv[:, idx], rv) <= TOL and relerr(yf[:, idx], rf) <= TOL


def test_empty(torch_dev, sf):
    torch = torch_dev
    u = torch.zeros((5, 0, 512), dtype=torch.float64, device="cuda")
    uf = torch.zeros((5, 0, 6, 64), dtype=torch.float64, device="cuda")
    yv, yf = sf.surface(u, uf, 8, 3, "euler")
    assert yv.shape == u.shape and yf.shape == uf.shape
