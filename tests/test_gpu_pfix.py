"""GPU parity of the pressure-fix flux variant (SF_FLUX_EULER_CHANDRASHEKAR_PFIX:
Chandrashekar's flux with Ranocha's pressure fix, the flux of the Results
section's Taylor-Green runs) against the oracle's euler_pfix definition, in
every entry point that builds it: the sum-factorized volume term (every n,
both node sets), the dense path, the surface term alone and fused with the
volume term, and the curvilinear volume term; plus pressure equilibrium on
the GPU and the refusals of the forms that do not build it.

Tolerance: per variable ||y_gpu - y_ref||_inf / ||y_ref||_inf <= 1e-12.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL = 1e-12
FLUX = "euler_pfix"


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


def cuda(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("kind", ["gl", "gll"])
@pytest.mark.parametrize("n", list(range(2, 14)))
def test_volume_every_n(torch_dev, sf, orc, n, kind):
    from paper_2306_11665_amd import workloads as W
    E = 9 if n <= 6 else 3
    u = W.euler_state(E, n, seed=1600 + n, freestream_frac=0.2)
    y = sf.volume(cuda(torch_dev, u), n, 3, FLUX, nodes=kind).cpu().numpy()
    ref = orc.dense_volume(u, n, 3, FLUX, nodes_kind=kind)
    err = relerr(y, ref)
    assert err <= TOL, (n, kind, err)


def test_volume_n8_mesh_and_wide_ratios(torch_dev, sf, orc):
    """n = 8, 2000 elements with free-stream ones, against the oracle's CPU
    method on every element; and in-element ratios of 1e4 with near-switch
    pairs against the dense definition."""
    from paper_2306_11665_amd import workloads as W
    n = 8
    u = W.euler_state(2000, n, seed=1700, freestream_frac=0.1)
    y = sf.volume(cuda(torch_dev, u), n, 3, FLUX).cpu().numpy()
    assert relerr(y, orc.sf_volume(u, n, 3, FLUX)) <= TOL
    uw = W.wide_ratio_euler_state(4, n, 1e4, seed=1701, switch_tau=2e-3)
    yw = sf.volume(cuda(torch_dev, uw), n, 3, FLUX).cpu().numpy()
    assert relerr(yw, orc.dense_volume(uw, n, 3, FLUX)) <= TOL


@pytest.mark.parametrize("n", [4, 8])
def test_dense_path(torch_dev, sf, orc, n):
    from paper_2306_11665_amd import workloads as W
    u = W.euler_state(3, n, seed=1800 + n)
    y = sf.dense_volume(cuda(torch_dev, u), n, 3, FLUX).cpu().numpy()
    assert relerr(y, orc.dense_volume(u, n, 3, FLUX)) <= TOL


@pytest.mark.parametrize("n,kind", [(3, "gl"), (5, "gll"), (8, "gl"), (11, "gll")])
def test_surface_alone_and_fused(torch_dev, sf, orc, n, kind):
    from paper_2306_11665_amd import workloads as W
    E = 7 if n <= 8 else 2
    u = W.euler_state(E, n, seed=1900 + n)
    rng = np.random.default_rng(1950 + n)
    k = 6 * n * n
    uf = W.primitives_to_conserved(rng.uniform(0.5, 1.5, (E, k)), rng.uniform(-0.5, 0.5, (3, E, k)),
                                   rng.uniform(0.5, 1.5, (E, k))).reshape(5, E, 6, n * n)
    rv, rf = orc.surface(u, np.ascontiguousarray(uf), n, 3, FLUX, nodes_kind=kind)
    for fused in (False, True):
        yv, yf = sf.surface(cuda(torch_dev, u), cuda(torch_dev, uf), n, 3, FLUX, nodes=kind, with_volume=fused)
        want_v = rv + orc.dense_volume(u, n, 3, FLUX, nodes_kind=kind) if fused else rv
        assert relerr(yv.cpu().numpy(), want_v) <= TOL, (n, kind, fused)
        assert relerr(yf.cpu().numpy(), rf) <= TOL, (n, kind, fused)


@pytest.mark.parametrize("n,kind", [(2, "gl"), (4, "gll"), (8, "gl"), (10, "gll")])
def test_curvilinear(torch_dev, sf, orc, n, kind):
    from paper_2306_11665_amd import workloads as W
    E = 5 if n <= 6 else 2
    u = W.euler_state(E, n, seed=2000 + n, freestream_frac=0.2)
    Ja = W.warped_mesh_metrics(E, n, nodes=kind, amp=0.03)
    y = sf.volume_curvilinear(cuda(torch_dev, u), cuda(torch_dev, Ja), n, FLUX, nodes=kind).cpu().numpy()
    ref = orc.curv_volume(u, Ja, n, FLUX, nodes_kind=kind)
    assert relerr(y, ref) <= TOL, (n, kind)


def test_pressure_equilibrium_on_the_gpu(torch_dev, sf):
    """Constant velocity and pressure, random density: the momentum and energy
    results are the velocity and |v|^2/2 times the mass result (to rounding
    of the fluxes, whose O(p) pressure terms cancel in y)."""
    from paper_2306_11665_amd import workloads as W
    n, E = 6, 20
    rng = np.random.default_rng(2100)
    rho = rng.uniform(0.5, 1.5, (E, n ** 3))
    v = np.array([-0.25, 0.4, 0.15])
    u = np.ascontiguousarray(W.primitives_to_conserved(
        rho, np.broadcast_to(v[:, None, None], (3, E, n ** 3)), np.full((E, n ** 3), 1.2)))
    y = sf.volume(cuda(torch_dev, u), n, 3, FLUX).cpu().numpy()
    scale = 1.2 + rho.max() * (v @ v) * 2                 # p + rho |v|^2 (flux size), with margin
    for k in range(3):
        assert np.abs(y[1 + k] - v[k] * y[0]).max() <= 1e-13 * scale
    assert np.abs(y[4] - 0.5 * (v @ v) * y[0]).max() <= 1e-13 * scale


def test_forms_without_the_variant_refuse_it(torch_dev, sf):
    from paper_2306_11665_amd import serving, workloads as W
    u = cuda(torch_dev, W.euler_state(2, 4, seed=2200))
    with pytest.raises(sf.SFError) as ex:
        sf.volume(u, 4, 3, FLUX, precision="fp32_split")
    assert ex.value.status == -2
    L = serving._lib()
    import ctypes
    h = ctypes.c_void_p()
    assert L.sf_server_create(1 << 26, 4, ctypes.byref(h)) == 0
    try:
        m = ctypes.c_int64()
        host = np.ascontiguousarray(W.euler_state(2, 4, seed=2201))
        st = L.sf_mesh_register(h, host.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 2, 4,
                                sf.FLUX[FLUX], 0, ctypes.byref(m))
        assert st == -2
    finally:
        L.sf_server_destroy(h)
