"""GPU parity over the state domain the C-ABI states (include/sfhad.h):
in-element density and pressure ratios of 1e2, 1e4 and 1e6 with node pairs
either side of the logarithmic mean's series switch, the end points of the
FP64 domain (rho, beta down to 1e-30 and up to 1e30), the narrower FP32-split
domain, and the dense path at the largest Euler sizes it accepts.

Every case is checked per element and per conserved variable:
max_nodes |y - y_ref| / max_nodes |y_ref| <= 1e-12 (FP64) or 1e-5
(FP32-split), y_ref from the oracle's dense definition (Eq. (1)).  The
element-wise norm is stricter than the mesh-wide one: a wide-ratio element
cannot hide behind a larger neighbour.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5
# the kernels take the series form of the logarithmic mean below
# |ln a - ln b| = 2e-3 (FP64 form)
SWITCH = 2e-3


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


def elementwise(y, ref):
    """max over elements and variables of the element's normwise error."""
    d = np.abs(y - ref).max(axis=2)
    s = np.maximum(np.abs(ref).max(axis=2), 1e-300)
    return float((d / s).max())


def gpu(torch, sf, u, n, **kw):
    y = sf.volume(torch.from_numpy(u).cuda(), n, 3, "euler", **kw)
    torch.cuda.synchronize()
    return y.cpu().numpy()


@pytest.mark.parametrize("ratio", [1e2, 1e4, 1e6])
@pytest.mark.parametrize("n", [4, 5, 8])
def test_wide_in_element_ratios(torch_dev, sf, orc, ratio, n):
    """rho and p spread over `ratio` inside every element, and on every x-line
    a node pair at |ln a - ln b| = 2e-3 (1 +- 1e-3, 1e-2) for both rho and
    beta: the element-relative logarithms and the direct / series switch."""
    from paper_2306_11665_amd import workloads as W
    E = 6
    u = W.wide_ratio_euler_state(E, n, ratio, seed=1200 + n, switch_tau=SWITCH)
    ref = orc.dense_volume(u, n, 3, "euler")
    err64 = elementwise(gpu(torch_dev, sf, u, n), ref)
    err32 = elementwise(gpu(torch_dev, sf, u, n, precision="fp32_split"), ref)
    print(f"wide ratio {ratio:.0e} n={n}: fp64 {err64:.2e} fp32-split {err32:.2e}")
    assert err64 <= TOL64, err64
    assert err32 <= TOL32, err32


@pytest.mark.parametrize("rho_scale,p_scale", [(1e-29, 1.0), (1e29, 1.0), (1.0, 1e-29), (1e-29, 1e-29),
                                               (1e29, 1e29)])
def test_fp64_domain_end_points(torch_dev, sf, orc, rho_scale, p_scale):
    """States at the ends of the FP64 domain: rho and beta = rho/(2p) between
    about 1e-30 and 1e30 (an in-element ratio of 1e2 around each scale, the
    velocity scaled with the sound speed), with near-switch pairs."""
    from paper_2306_11665_amd import workloads as W
    n, E = 5, 4
    u = W.wide_ratio_euler_state(E, n, 1e2, seed=1300, rho_scale=rho_scale, p_scale=p_scale,
                                 switch_tau=SWITCH, vel_scale=np.sqrt(p_scale / rho_scale))
    ref = orc.dense_volume(u, n, 3, "euler")
    assert np.isfinite(ref).all()
    err = elementwise(gpu(torch_dev, sf, u, n), ref)
    print(f"end points rho~{rho_scale:.0e} p~{p_scale:.0e}: fp64 {err:.2e}")
    assert err <= TOL64, err


@pytest.mark.parametrize("rho_scale,p_scale", [(1e-10, 1.0), (1e10, 1.0), (1.0, 1e-10), (1.0, 1e10),
                                               (1e10, 1e10), (1e-10, 1e-10)])
def test_fp32split_domain(torch_dev, sf, orc, rho_scale, p_scale):
    """The FP32-split form's narrower domain: rho and beta between about
    1e-10 and 1e10 (it multiplies up to three FP32 means)."""
    from paper_2306_11665_amd import workloads as W
    n, E = 5, 4
    u = W.wide_ratio_euler_state(E, n, 1e2, seed=1400, rho_scale=rho_scale, p_scale=p_scale,
                                 switch_tau=SWITCH, vel_scale=np.sqrt(p_scale / rho_scale))
    ref = orc.dense_volume(u, n, 3, "euler")
    err = elementwise(gpu(torch_dev, sf, u, n, precision="fp32_split"), ref)
    print(f"fp32-split rho~{rho_scale:.0e} p~{p_scale:.0e}: {err:.2e}")
    assert err <= TOL32, err


@pytest.mark.parametrize("n", [9, 13])
def test_dense_euler_largest(torch_dev, sf, orc, n):
    """The dense O(n^(2d)) path at the largest Euler sizes it accepts
    (n^3 <= 4096: up to 123 KB of staged LDS at n = 13)."""
    from paper_2306_11665_amd import workloads as W
    E = 2
    u = W.euler_state(E, n, seed=1500 + n, freestream_frac=0.0)
    y = sf.dense_volume(torch_dev.from_numpy(u).cuda(), n, 3, "euler")
    torch_dev.cuda.synchronize()
    ref = orc.dense_volume(u, n, 3, "euler")
    err = elementwise(y.cpu().numpy(), ref)
    print(f"dense n={n}: {err:.2e}")
    assert err <= TOL64, err
