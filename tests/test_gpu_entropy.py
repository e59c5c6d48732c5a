"""GPU parity of the entropy-projected facet states (sf_entropy_trace)
against the oracle's definition (explicit facet interpolation of the entropy
variables), and of the chain entropy trace -> volume + surface term against
the oracle's chain.  Tolerance 1e-12 normwise per variable."""
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


def smooth_state(orc, E, n, kind, seed):
    """Linear primitive fields per element (their facet values stay physical)."""
    from paper_2306_11665_amd import workloads as W
    x, _ = orc.nodes(n, kind)
    node = np.arange(n ** 3)
    X = np.stack([x[node % n], x[(node // n) % n], x[node // (n * n)]])
    rng = np.random.default_rng(seed)
    rho = np.zeros((E, n ** 3)); p = np.zeros((E, n ** 3)); vel = np.zeros((3, E, n ** 3))
    for e in range(E):
        g = rng.uniform(-0.2, 0.2, (5, 3))
        rho[e] = 1.0 + g[0] @ X
        p[e] = 1.0 + g[1] @ X
        for k in range(3):
            vel[k, e] = rng.uniform(-0.3, 0.3) + g[2 + k] @ X
    return np.ascontiguousarray(W.primitives_to_conserved(rho, vel, p))


@pytest.mark.parametrize("n", list(range(2, 14)))
@pytest.mark.parametrize("kind", ["gl", "gll"])
def test_entropy_trace_every_n(torch_dev, sf, orc, n, kind):
    torch = torch_dev
    E = 13 if n <= 8 else 3
    u = smooth_state(orc, E, n, kind, seed=100 + n)
    y = sf.entropy_trace(torch.from_numpy(u).cuda(), n, nodes=kind)
    torch.cuda.synchronize()
    ref = orc.entropy_trace(u, n, kind)
    err = relerr(y.cpu().numpy(), ref)
    assert err <= TOL, (n, kind, err)


def test_chain_trace_then_volume_surface(torch_dev, sf, orc):
    """u -> entropy-projected facet states -> volume + surface term, both on
    the GPU, against the same chain in the oracle."""
    torch = torch_dev
    n, E = 6, 7
    u = smooth_state(orc, E, n, "gl", seed=9)
    ut = torch.from_numpy(u).cuda()
    uf = sf.entropy_trace(ut, n)
    yv, yf = sf.surface(ut, uf, n, 3, "euler", with_volume=True)
    torch.cuda.synchronize()
    uf_ref = orc.entropy_trace(u, n)
    rv, rf = orc.surface(u, uf_ref, n, 3, "euler")
    rv = rv + orc.dense_volume(u, n, 3, "euler")
    assert relerr(yv.cpu().numpy(), rv) <= TOL and relerr(yf.cpu().numpy(), rf) <= TOL


def test_full_size_sampled(torch_dev, sf, orc):
    """At the benchmark's shape (n = 8, 32768 elements of the random
    per-node state; GLL, whose end values pick the boundary nodes, so the
    facet states stay physical): sampled elements against the oracle."""
    torch = torch_dev
    from paper_2306_11665_amd import workloads as W
    w = W.WORKLOADS["euler3d_n8_gl_e32768"]
    u = w.state()
    y = sf.entropy_trace(torch.from_numpy(u).cuda(), 8, nodes="gll").cpu().numpy()
    idx = np.sort(np.random.default_rng(14).choice(w.E, 32, replace=False))
    ref = orc.entropy_trace(np.ascontiguousarray(u[:, idx]), 8, "gll")
    assert relerr(y[:, idx], ref) <= TOL


def physical_states(count, seed):
    from paper_2306_11665_amd import workloads as W
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.2, 3.0, count)
    p = rng.uniform(0.2, 3.0, count)
    vel = rng.uniform(-1.5, 1.5, (3, count))
    return np.ascontiguousarray(W.primitives_to_conserved(rho, vel, p))


@pytest.mark.parametrize("count", [1, 255, 256, 257, 100_003])
def test_entropy_variable_maps(torch_dev, sf, orc, count):
    """Pointwise u -> v and v -> u against the oracle's maps on sampled
    states (every state when few), and the round trip on all of them;
    counts around one block and a ragged multi-block one."""
    torch = torch_dev
    u = physical_states(count, seed=count)
    ut = torch.from_numpy(u).cuda()
    v = sf.entropy_variables(ut)
    back = sf.conserved_variables(v)
    torch.cuda.synchronize()
    vn, bn = v.cpu().numpy(), back.cpu().numpy()
    idx = np.arange(count) if count <= 300 else np.random.default_rng(1).choice(count, 300, replace=False)
    for i in idx:
        rv = orc.entropy_vars(u[:, i])
        assert np.abs(vn[:, i] - rv).max() <= TOL * np.abs(rv).max(), i
        ru = orc.conserved_from_entropy(vn[:, i])
        assert np.abs(bn[:, i] - ru).max() <= TOL * np.abs(ru).max(), i
    assert relerr(bn, u) <= 1e-12


def test_entropy_variable_maps_in_place(torch_dev, sf):
    torch = torch_dev
    u = physical_states(1000, seed=4)
    ut = torch.from_numpy(u).cuda()
    v = sf.entropy_variables(ut)
    w = ut.clone()
    sf.entropy_variables(w, out=w)
    sf.conserved_variables(w, out=w)
    torch.cuda.synchronize()
    assert relerr(w.cpu().numpy(), u) <= 1e-12
    assert relerr(sf.entropy_variables(ut).cpu().numpy(), v.cpu().numpy()) == 0.0


@pytest.mark.parametrize("n,m", [(4, 6), (6, 9)])
def test_over_integrated_entropy_projection(torch_dev, sf, orc, n, m):
    """The entropy projection on m > n over-integration nodes,
    u(V P v(u)) with v projected from the n collocated nodes to modes and
    evaluated on the m^3 nodes: the GPU chain (map, two basis
    transformations, inverse map) against the oracle's chain."""
    torch = torch_dev
    E = 9
    u = smooth_state(orc, E, n, "gl", seed=n * m)
    _, Pn = orc.basis_rect(n, n, "gl")
    Vm, _ = orc.basis_rect(n, m, "gl")
    ut = torch.from_numpy(u).cuda()
    v = sf.entropy_variables(ut)
    vh = sf.tensor_apply(v, n, 3, Pn)
    vq = sf.tensor_apply(vh, n, 3, Vm)
    uq = sf.conserved_variables(vq)
    torch.cuda.synchronize()
    vo = np.zeros_like(u)
    for e in range(E):
        for k in range(n ** 3):
            vo[:, e, k] = orc.entropy_vars(u[:, e, k])
    vqo = orc.tensor_apply(orc.tensor_apply(vo, n, 3, Pn), n, 3, Vm)
    uqo = np.zeros_like(vqo)
    for e in range(E):
        for k in range(m ** 3):
            uqo[:, e, k] = orc.conserved_from_entropy(vqo[:, e, k])
    assert relerr(uq.cpu().numpy(), uqo) <= TOL
