"""The entry points under HIP graph capture: volume (FP64 and FP32-split),
volume + surface, entropy trace and basis transformation captured into one
graph on a side stream, replayed several times with new inputs written by
eager work between the replays; every replay must equal the eager calls bit
for bit (same kernels, same launch shapes, fixed summation order).  The
calls allocate nothing and clear nothing, so they capture as plain kernel
nodes."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


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


def test_graph_replays_match_eager(torch_dev, sf):
    torch = torch_dev
    from paper_2306_11665_amd import workloads as W
    n, E = 4, 96
    states = [W.smooth_euler_state(E, n, seed=40 + k, nodes="gll") for k in range(3)]
    u = torch.from_numpy(states[0]).cuda()
    _, P = sf.basis_1d(n, "gll")
    s = torch.cuda.Stream()
    outs = {
        "vol": torch.empty_like(u), "vol32": torch.empty_like(u),
        "uf": torch.empty((5, E, 6, n * n), dtype=torch.float64, device="cuda"),
        "yv": torch.empty_like(u), "yf": torch.empty((5, E, 6, n * n), dtype=torch.float64, device="cuda"),
        "uh": torch.empty_like(u),
    }

    def calls(o, stream):
        sf.volume(u, n, 3, "euler", nodes="gll", out=o["vol"], stream=stream)
        sf.volume(u, n, 3, "euler", nodes="gll", precision="fp32_split", out=o["vol32"], stream=stream)
        sf.entropy_trace(u, n, nodes="gll", out=o["uf"], stream=stream)
        sf.surface(u, o["uf"], n, 3, "euler", nodes="gll", with_volume=True, y_vol=o["yv"], y_face=o["yf"],
                   stream=stream)
        sf.tensor_apply(u, n, 3, P, out=o["uh"], stream=stream)

    with torch.cuda.stream(s):
        calls(outs, s)                     # warm (operator cache, module load) before capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        calls(outs, s)
    ref = {k: torch.empty_like(v) for k, v in outs.items()}
    for k in range(3):
        u.copy_(torch.from_numpy(states[k]).cuda())      # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        calls(ref, torch.cuda.current_stream())
        torch.cuda.synchronize()
        for name in outs:
            a, b = outs[name].cpu().numpy(), ref[name].cpu().numpy()
            assert np.isfinite(a).all(), (k, name)
            assert np.array_equal(a, b), (k, name, np.abs(a - b).max())
