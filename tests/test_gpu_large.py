"""Index width at large meshes: n = 8 with 1.1 million elements puts the
variable offsets of the SoA arrays past 2^31 doubles (about 22.5 GB per
array), so every kernel's 64-bit address arithmetic is exercised.  Sampled
elements (the last ones included) against the oracle: volume term (FP64 and
FP32-split), basis transformation and entropy-projected facet states."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

N, E = 8, 1_100_000


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


@pytest.fixture(scope="module")
def big_state(torch_dev):
    """Per-node random physical states drawn on the device from a seeded
    generator (rho, p in [0.5, 1.5], velocity in [-0.5, 0.5]^3), stored as
    conserved variables."""
    torch = torch_dev
    assert 5 * E * N ** 3 > 2 ** 31 and 4 * E * N ** 3 > 2 ** 31
    g = torch.Generator(device="cuda")
    g.manual_seed(2024)
    u = torch.empty((5, E, N ** 3), dtype=torch.float64, device="cuda")
    chunk = 100_000
    for e0 in range(0, E, chunk):
        k = min(chunk, E - e0)
        r = torch.rand((5, k, N ** 3), generator=g, dtype=torch.float64, device="cuda")
        rho = 0.5 + r[0]
        vel = r[1:4] - 0.5
        p = 0.5 + r[4]
        u[0, e0:e0 + k] = rho
        u[1:4, e0:e0 + k] = rho * vel
        u[4, e0:e0 + k] = p / 0.4 + 0.5 * rho * (vel * vel).sum(0)
        del r, rho, vel, p
    torch.cuda.synchronize()
    idx = np.unique(np.concatenate([np.random.default_rng(5).choice(E, 24, replace=False),
                                    np.arange(E - 8, E)]))
    return u, idx


def relerr(y, ref):
    return max(np.abs(y[v] - ref[v]).max() / max(np.abs(ref[v]).max(), 1e-300) for v in range(ref.shape[0]))


def test_volume_at_large_offsets(torch_dev, sf, orc, big_state):
    torch = torch_dev
    u, idx = big_state
    us = u[:, idx].cpu().numpy()
    ref = orc.dense_volume(us, N, 3, "euler")
    for prec, tol in (("fp64", 1e-12), ("fp32_split", 1e-5)):
        y = sf.volume(u, N, 3, "euler", precision=prec)
        torch.cuda.synchronize()
        err = relerr(y[:, idx].cpu().numpy(), ref)
        del y
        torch.cuda.empty_cache()
        assert err <= tol, (prec, err)


def test_tensor_and_trace_at_large_offsets(torch_dev, sf, orc, big_state):
    torch = torch_dev
    u, idx = big_state
    us = np.ascontiguousarray(u[:, idx].cpu().numpy())
    _, P = sf.basis_1d(N, "gl")
    uh = sf.tensor_apply(u, N, 3, P)
    torch.cuda.synchronize()
    assert relerr(uh[:, idx].cpu().numpy(), orc.tensor_apply(us, N, 3, P)) <= 1e-12
    del uh
    torch.cuda.empty_cache()
    uf = sf.entropy_trace(u, N, nodes="gll")
    torch.cuda.synchronize()
    assert relerr(uf[:, idx].cpu().numpy(), orc.entropy_trace(us, N, "gll")) <= 1e-12
    del uf
    torch.cuda.empty_cache()
