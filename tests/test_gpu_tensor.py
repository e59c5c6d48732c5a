"""GPU parity of the basis transformation (sf_tensor_apply, FP64 matrix
cores) against the oracle's Kronecker-power matrix-vector product.

Tolerance: per variable, ||out_gpu - out_ref||_inf / ||out_ref||_inf <= 1e-12
(sums of n^d products in a different order).  Inputs: seeded modal
coefficients u_hat ~ N(0, 1) decaying like 1/(1 + |k|) (smooth modal data),
and the n = 8, 32768-element Euler state as nodal data for the projection.
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


def slabs_per_block(n, d):
    nodes = n ** d
    return 1 if nodes >= 2048 else 2048 // nodes


def modal(nvar, E, n, d, seed):
    rng = np.random.default_rng(seed)
    k = np.arange(n)
    if d == 2:
        decay = 1.0 / (1.0 + k[None, :] + k[:, None])
    else:
        decay = 1.0 / (1.0 + k[None, None, :] + k[None, :, None] + k[:, None, None])
    return rng.normal(size=(nvar, E, n ** d)) * decay.ravel()[None, None, :]


def relerr(y, ref):
    return max(np.abs(y[v] - ref[v]).max() / max(np.abs(ref[v]).max(), 1e-300) for v in range(ref.shape[0]))


def gpu_apply(torch, sf, u, n, d, M, inplace=False, stream=None):
    ut = torch.from_numpy(np.ascontiguousarray(u)).cuda()
    y = sf.tensor_apply(ut, n, d, M, out=ut if inplace else None, stream=stream)
    torch.cuda.synchronize()
    return y.cpu().numpy()


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("n", list(range(2, 17)))
def test_modal_to_nodal_every_n(torch_dev, sf, orc, n, d):
    # several blocks and a ragged last block: 3 full blocks plus one slab
    G = slabs_per_block(n, d)
    nvar = 5
    slabs = 3 * G + 1
    E = -(-slabs // nvar)
    if n ** d >= 1024:
        E = min(E, 3)                                  # keep the dense oracle to seconds
    uh = modal(nvar, E, n, d, seed=1000 + 17 * n + d)
    for kind in ("gl", "gll"):
        V, P = sf.basis_1d(n, kind)
        ref = orc.tensor_apply(uh, n, d, V)
        y = gpu_apply(torch_dev, sf, uh, n, d, V)
        err = relerr(y, ref)
        print(f"n={n} d={d} {kind} E={E}: {err:.2e}")
        assert err <= TOL, (n, d, kind, err)


@pytest.mark.parametrize("n,d", [(3, 2), (4, 3), (7, 3), (8, 3), (16, 2), (13, 3)])
def test_general_matrix_and_projection(torch_dev, sf, orc, n, d):
    """A non-symmetric M catches a transposed operand or swapped directions;
    the projection P returns the coefficients (Pi chi = I)."""
    rng = np.random.default_rng(n * 31 + d)
    M = rng.normal(size=(n, n))
    E = 5
    u = rng.normal(size=(2, E, n ** d))
    ref = orc.tensor_apply(u, n, d, M)
    assert relerr(gpu_apply(torch_dev, sf, u, n, d, M), ref) <= TOL
    V, P = sf.basis_1d(n, "gl")
    uh = modal(1, E, n, d, seed=3)
    back = gpu_apply(torch_dev, sf, gpu_apply(torch_dev, sf, uh, n, d, V), n, d, P)
    assert np.abs(back - uh).max() <= 1e-12 * np.abs(uh).max()


def test_in_place_and_side_stream(torch_dev, sf, orc):
    torch = torch_dev
    n, d = 6, 3
    V, _ = sf.basis_1d(n, "gl")
    uh = modal(5, 40, n, d, seed=9)
    ref = orc.tensor_apply(uh, n, d, V)
    assert relerr(gpu_apply(torch, sf, uh, n, d, V, inplace=True), ref) <= TOL
    s = torch.cuda.Stream()
    assert relerr(gpu_apply(torch, sf, uh, n, d, V, stream=s), ref) <= TOL


def test_empty_and_single(torch_dev, sf, orc):
    torch = torch_dev
    n, d = 8, 3
    V, _ = sf.basis_1d(n, "gl")
    u0 = torch.zeros((5, 0, n ** d), dtype=torch.float64, device="cuda")
    assert sf.tensor_apply(u0, n, d, V).shape == u0.shape
    uh = modal(1, 1, n, d, seed=4)
    assert relerr(gpu_apply(torch, sf, uh, n, d, V), orc.tensor_apply(uh, n, d, V)) <= TOL


def test_full_size_sampled_and_round_trip(torch_dev, sf, orc):
    """At the benchmark's shape (5 x 32768 elements, n = 8), in the launch
    configuration the benchmark times: sampled elements against the oracle,
    and the projection of the nodal state back and forth on every element."""
    torch = torch_dev
    from paper_2306_11665_amd import workloads as W
    w = W.WORKLOADS["euler3d_n8_gl_e32768"]
    n, d, E = w.n, 3, w.E
    u = w.state()
    V, P = sf.basis_1d(n, "gl")
    ut = torch.from_numpy(u).cuda()
    uh = sf.tensor_apply(ut, n, d, P)                 # nodal -> modal
    back = sf.tensor_apply(uh, n, d, V)               # modal -> nodal
    torch.cuda.synchronize()
    b = back.cpu().numpy()
    assert relerr(b, u) <= TOL
    idx = np.sort(np.random.default_rng(11).choice(E, 48, replace=False))
    idx[-1] = E - 1
    uh_np = uh.cpu().numpy()
    ref = orc.tensor_apply(np.ascontiguousarray(u[:, idx, :]), n, d, P)
    assert relerr(uh_np[:, idx, :], ref) <= TOL


# the (n_in, n_out) pairs built with compile-time sizes (3D), each with its
# own LDS stage of `rect_stage` doubles; other pairs take 4096
CT_PAIRS = [(3, 5), (5, 3), (4, 6), (6, 4), (5, 7), (7, 5), (6, 8), (8, 6), (7, 9), (9, 7), (8, 10), (10, 8)]


def rect_block_slabs(ni, no, d):
    """Slabs per block of the rectangular kernel's launch: the LDS stage
    (3072 doubles for 10 -> 8 and larger projections, 6144 for the other
    compile-time pairs, 4096 otherwise) over the larger shape, at most 512
    lines of a pass."""
    mx = max(ni, no)
    if d == 3 and (ni, no) in CT_PAIRS:
        stage = 3072 if (ni > no and ni ** 3 >= 1000) else 6144
    else:
        stage = 4096
    return max(1, min(stage // mx ** d, 512 // mx ** (d - 1)))


@pytest.mark.parametrize("ni,no,d", [(3, 5, 2), (2, 16, 2), (8, 12, 3), (16, 9, 3), (7, 8, 3), (4, 16, 3)]
                         + [(a, b, 3) for a, b in CT_PAIRS])
def test_rectangular_every_shape_class(torch_dev, sf, orc, ni, no, d):
    """n_in != n_out (modes to more or fewer nodes): several blocks and a
    ragged last one, a non-symmetric matrix, against the oracle; every
    compile-time pair and the run-time kernel in 2D and 3D."""
    rng = np.random.default_rng(ni * 31 + no + d)
    M = rng.normal(size=(no, ni))
    nvar = 5
    G = rect_block_slabs(ni, no, d)
    slabs = 3 * G + 1
    E = -(-slabs // nvar)
    u = rng.normal(size=(nvar, E, ni ** d))
    ref = orc.tensor_apply(u, ni, d, M)
    y = gpu_apply(torch_dev, sf, u, ni, d, M)
    assert y.shape == ref.shape
    err = relerr(y, ref)
    print(f"rect {ni}->{no} d={d}: {err:.2e}")
    assert err <= TOL, err


@pytest.mark.parametrize("n,m", [(4, 6), (8, 12), (5, 16)])
@pytest.mark.parametrize("kind", ["gl", "gll"])
def test_over_integration_round_trip(torch_dev, sf, orc, n, m, kind):
    """n modes to m > n quadrature nodes and back with the library's basis:
    the interpolation matches the oracle and the projection returns the
    coefficients (P V = I)."""
    V, P = sf.basis_rect(n, m, kind)
    Vo, Po = orc.basis_rect(n, m, kind)
    assert np.abs(V - Vo).max() < 1e-13 and np.abs(P - Po).max() < 1e-12
    uh = modal(2, 37, n, 3, seed=n + m)
    uq = gpu_apply(torch_dev, sf, uh, n, 3, V)
    assert relerr(uq, orc.tensor_apply(uh, n, 3, V)) <= TOL
    back = gpu_apply(torch_dev, sf, uq, m, 3, P)
    assert np.abs(back - uh).max() <= 1e-12 * np.abs(uh).max()
