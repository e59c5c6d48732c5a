"""GPU parity: the HIP kernels (through the C-ABI) against the CPU oracle.

Tolerances.  FP64 paths: normwise relative error per conserved variable,
max_v ||y_gpu - y_ref||_inf / ||y_ref||_inf <= 1e-12.  FP32-split:
<= 1e-5 with the same metric.  Free-stream elements must also give
|y| <= 1e-13 max|f(u)|.  Inputs are the seeded synthetic workloads.
"""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


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


def normwise(y, ref):
    """Per-variable (max, mean) normwise relative errors."""
    nv = ref.shape[0]
    mx, mn = [], []
    for v in range(nv):
        d = np.abs(y[v] - ref[v])
        s_inf = max(np.abs(ref[v]).max(), 1e-300)
        s_1 = max(np.abs(ref[v]).sum(), 1e-300)
        mx.append(d.max() / s_inf)
        mn.append(d.sum() / s_1)
    return np.array(mx), np.array(mn)


def run_gpu(torch, sf, u, n, d, flux, dense=False, **kw):
    ut = torch.from_numpy(u).cuda()
    fn = sf.dense_volume if dense else sf.volume
    y = fn(ut, n, d, flux, **kw)
    torch.cuda.synchronize()
    return y.cpu().numpy()


def state(flux, E, n, d, seed, fs=0.0):
    from paper_2306_11665_amd import workloads as W
    if flux == "euler":
        return W.euler_state(E, n, seed, fs, d=d)
    if flux == "product":
        return W.scalar_state(E, n, d, seed, 1e-8, 30.0)
    return W.scalar_state(E, n, d, seed)


# ----------------------------------------------------------------- workloads
def test_burgers2d_n4_gll_e64(torch_dev, sf, orc):
    from paper_2306_11665_amd import workloads as W
    w = W.WORKLOADS["burgers2d_n4_gll_e64"]
    u = w.state()
    y = run_gpu(torch_dev, sf, u, w.n, w.d, w.flux, nodes=w.nodes)
    ref = orc.dense_volume(u, w.n, w.d, w.flux, nodes_kind=w.nodes)
    mx, _ = normwise(y, ref)
    print("burgers2d_n4_gll_e64 max normwise", mx)
    assert mx.max() <= TOL64


def test_euler3d_n4_gl_e4096(torch_dev, sf, orc):
    from paper_2306_11665_amd import workloads as W
    w = W.WORKLOADS["euler3d_n4_gl_e4096"]
    u = w.state()
    y = run_gpu(torch_dev, sf, u, w.n, w.d, w.flux, nodes=w.nodes)
    ref = orc.dense_volume(u, w.n, w.d, w.flux, nodes_kind=w.nodes)
    mx, mn = normwise(y, ref)
    print("euler3d_n4_gl_e4096 max", mx, "mean", mn)
    assert mx.max() <= TOL64


@pytest.fixture(scope="module")
def cfg_n8(torch_dev, sf):
    """The n = 8, 32768-element workload on the GPU (FP64 and FP32-split)."""
    from paper_2306_11665_amd import workloads as W
    w = W.WORKLOADS["euler3d_n8_gl_e32768"]
    u = w.state()
    ut = torch_dev.from_numpy(u).cuda()
    y64 = sf.volume(ut, w.n, w.d, w.flux).cpu().numpy()
    y32 = sf.volume(ut, w.n, w.d, w.flux, precision="fp32_split").cpu().numpy()
    fs = W.freestream_index(w)
    sample = W.sample_elements(w.E, 48, seed=33, must_include=fs[:8].tolist() + [0, w.E - 1])
    return w, u, y64, y32, fs, sample


def test_euler3d_n8_gl_e32768_sampled(cfg_n8, orc):
    w, u, y64, y32, fs, sample = cfg_n8
    us = np.ascontiguousarray(u[:, sample, :])
    ref = orc.dense_volume(us, w.n, w.d, w.flux, nodes_kind=w.nodes)
    mx, mn = normwise(y64[:, sample, :], ref)
    print(f"euler3d_n8 FP64 on {len(sample)} sampled elements: max {mx} mean {mn}")
    assert mx.max() <= TOL64


def test_euler3d_n8_freestream_elements_vanish(cfg_n8, orc):
    w, u, y64, y32, fs, sample = cfg_n8
    assert len(fs) == round(0.1 * w.E)
    fscale = max(np.abs(orc.physical_flux_euler(u[:, e, 0], m)).max() for e in fs[:64] for m in range(3))
    assert np.abs(y64[:, fs, :]).max() <= 1e-13 * fscale
    assert np.abs(y32[:, fs, :]).max() <= 1e-5 * fscale


def test_euler3d_n8_full_mesh_vs_oracle_method(cfg_n8, orc):
    """Every element, against the oracle's CPU sum-factorized method (itself
    pinned to the dense definition on the CPU)."""
    w, u, y64, y32, fs, sample = cfg_n8
    ref = orc.sf_volume(u, w.n, w.d, w.flux, nodes_kind=w.nodes)
    mx, mn = normwise(y64, ref)
    print("euler3d_n8 FP64 full mesh max", mx, "mean", mn)
    assert mx.max() <= TOL64
    mx32, mn32 = normwise(y32, ref)
    print("euler3d_n8 FP32-split full mesh max", mx32, "mean", mn32)
    assert mx32.max() <= TOL32


def test_fp32split_sampled_vs_dense_oracle(cfg_n8, orc):
    w, u, y64, y32, fs, sample = cfg_n8
    us = np.ascontiguousarray(u[:, sample, :])
    ref = orc.dense_volume(us, w.n, w.d, w.flux, nodes_kind=w.nodes)
    mx, mn = normwise(y32[:, sample, :], ref)
    print("FP32-split sampled: max", mx, "mean", mn)
    assert mx.max() <= TOL32


# ------------------------------------------------------------------ sweeps
@pytest.mark.parametrize("nodes", ["gl", "gll"])
@pytest.mark.parametrize("n", list(range(2, 14)))
def test_euler_all_n(torch_dev, sf, orc, n, nodes):
    E = 7 if n <= 6 else 3                       # ragged: not a multiple of the block size
    u = state("euler", E, n, 3, seed=100 + n)
    y = run_gpu(torch_dev, sf, u, n, 3, "euler", nodes=nodes)
    ref = orc.dense_volume(u, n, 3, "euler", nodes_kind=nodes)
    mx, _ = normwise(y, ref)
    assert mx.max() <= TOL64, (n, nodes, mx)


@pytest.mark.parametrize("flux", ["burgers", "product"])
@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 7, 8, 9, 11, 12, 16])
def test_scalar_all_n(torch_dev, sf, orc, flux, d, n):
    if d == 3 and n >= 12:
        E = 2
    else:
        E = 37 if d == 2 else 5
    u = state(flux, E, n, d, seed=200 + n)
    nodes = "gll" if n % 2 else "gl"
    y = run_gpu(torch_dev, sf, u, n, d, flux, nodes=nodes)
    ref = orc.dense_volume(u, n, d, flux, nodes_kind=nodes)
    mx, _ = normwise(y, ref)
    assert mx.max() <= TOL64, (flux, d, n, mx)


@pytest.mark.parametrize("flux,d,n", [("euler", 3, 2), ("euler", 3, 4), ("euler", 3, 5), ("euler", 3, 8),
                                      ("burgers", 2, 4), ("burgers", 3, 6), ("product", 3, 8),
                                      ("product", 2, 16), ("product", 3, 12), ("product", 3, 16)])
def test_dense_gpu_path(torch_dev, sf, orc, flux, d, n):
    E = 3
    u = state(flux, E, n, d, seed=300 + n)
    y = run_gpu(torch_dev, sf, u, n, d, flux, dense=True)
    ref = orc.dense_volume(u, n, d, flux)
    mx, _ = normwise(y, ref)
    assert mx.max() <= TOL64, mx


@pytest.mark.parametrize("nodes", ["gl", "gll"])
@pytest.mark.parametrize("n", list(range(2, 14)))
def test_fp32split_all_n(torch_dev, sf, orc, n, nodes):
    """The FP32-split form at every built n and both node sets (ragged
    element counts), against the FP64 dense oracle at the form's tolerance."""
    E = 9 if n <= 6 else 3
    u = state("euler", E, n, 3, seed=400 + n)
    y = run_gpu(torch_dev, sf, u, n, 3, "euler", nodes=nodes, precision="fp32_split")
    ref = orc.dense_volume(u, n, 3, "euler", nodes_kind=nodes)
    mx, _ = normwise(y, ref)
    assert mx.max() <= TOL32, (n, nodes, mx)


# ------------------------------------------------------------- edge cases
def test_near_equal_states(torch_dev, sf, orc):
    """Elements whose nodal densities and pressures differ by 1e-12..1e-1
    relative: exact equality, the near-equal series, the direct form and the
    switch between them (|ln a - ln b| = 2e-3 in FP64, |d| = 1e-6 s in the FP32 form)."""
    from paper_2306_11665_amd import workloads as W
    n, E = 6, 12
    base = W.euler_state(E, n, seed=500, freestream_frac=1.0)
    rng = np.random.default_rng(501)
    u = base.copy()
    for e in range(E):
        rel = 10.0 ** (-12 + e)                       # 1e-12 ... 1e-1
        r = base[0, e] * (1 + rel * rng.uniform(-1, 1, n ** 3))
        pr = (0.4 * (base[4, e] - 0.5 * (base[1, e] ** 2 + base[2, e] ** 2 + base[3, e] ** 2) / base[0, e]))
        pr = pr * (1 + rel * rng.uniform(-1, 1, n ** 3))
        v = base[1:4, e] / base[0, e]
        u[:, e, :] = W.primitives_to_conserved(r, v, pr)
    for nodes in ("gl", "gll"):
        y = run_gpu(torch_dev, sf, u, n, 3, "euler", nodes=nodes)
        ref = orc.dense_volume(u, n, 3, "euler", nodes_kind=nodes)
        _, w1, _, Q1 = orc.operator_1d(n, nodes)
        # rounding bound: a nearly uniform element has |y| << |F|, and the
        # rounding of each F (a few ulp of |F|) reaches y through the row sums
        # of Q, times w_perp, over the three directions (the oracle's own
        # rounding is of the same size)
        qnorm = 3 * np.abs(Q1).sum(axis=1).max() * w1.max() ** 2
        for e in range(E):
            scale = max(np.abs(orc.physical_flux_euler(u[:, e, 0], m)).max() for m in range(3))
            err = np.abs(y[:, e] - ref[:, e]).max()
            bound = max(TOL64 * np.abs(ref[:, e]).max(), 64 * 2.2e-16 * scale * qnorm)
            print(f"near-equal {nodes} rel={10.0 ** (-12 + e):.0e}: err {err:.2e} bound {bound:.2e} |y| {np.abs(ref[:, e]).max():.2e}")
            assert err <= bound, (nodes, e, err)
        y32 = run_gpu(torch_dev, sf, u, n, 3, "euler", nodes=nodes, precision="fp32_split")
        for e in range(E):
            scale = max(np.abs(orc.physical_flux_euler(u[:, e, 0], m)).max() for m in range(3))
            err = np.abs(y32[:, e] - ref[:, e]).max()
            assert err <= max(TOL32 * np.abs(ref[:, e]).max(), 1e-6 * scale), (nodes, e, err)


def test_empty_and_single_element(torch_dev, sf, orc):
    torch = torch_dev
    u0 = torch.zeros((5, 0, 512), dtype=torch.float64, device="cuda")
    y0 = sf.volume(u0, 8, 3, "euler")
    assert y0.shape == (5, 0, 512)
    u = state("euler", 1, 8, 3, seed=600)
    y = run_gpu(torch, sf, u, 8, 3, "euler")
    ref = orc.dense_volume(u, 8, 3, "euler")
    assert normwise(y, ref)[0].max() <= TOL64


def test_large_ragged_mesh_sampled(torch_dev, sf, orc):
    """A large element count that is not a multiple of anything (1,000,003
    elements at n = 4, 16 elements per block: 2.6 GB in and out, 62,501 blocks
    with a ragged last one): sampled elements, the last ones included,
    against the dense oracle, in FP64 and FP32-split."""
    torch = torch_dev
    n, E = 4, 1_000_003
    rng = np.random.default_rng(17)
    from paper_2306_11665_amd import workloads as W
    ut = torch.empty((5, E, n ** 3), dtype=torch.float64, device="cuda")
    chunk = 200_000
    for e0 in range(0, E, chunk):                      # generate in chunks (host memory)
        k = min(chunk, E - e0)
        ut[:, e0:e0 + k] = torch.from_numpy(W.euler_state(k, n, seed=int(rng.integers(1 << 30)),
                                                          freestream_frac=0.1))
    idx = np.unique(np.concatenate([rng.choice(E, 40, replace=False), np.arange(E - 16, E)]))
    us = ut[:, idx].cpu().numpy()
    ref = orc.dense_volume(us, n, 3, "euler")
    for prec, tol in (("fp64", TOL64), ("fp32_split", TOL32)):
        y = sf.volume(ut, n, 3, "euler", precision=prec)
        torch.cuda.synchronize()
        ys = y[:, idx].cpu().numpy()
        mx, _ = normwise(ys, ref)
        assert mx.max() <= tol, (prec, mx)
        del y


def test_bitwise_deterministic(torch_dev, sf):
    torch = torch_dev
    u = torch.from_numpy(state("euler", 2000, 8, 3, seed=700, fs=0.1)).cuda()
    for prec in ("fp64", "fp32_split"):
        a = sf.volume(u, 8, 3, "euler", precision=prec)
        b = sf.volume(u, 8, 3, "euler", precision=prec)
        torch.cuda.synchronize()
        assert torch.equal(a, b), prec


def test_operator_override_unweighted_product(torch_dev, sf, orc):
    """op_1d_host = D, w_1d_host = 1: the paper's sum_j dl/dxi_j o C with C = c c^T."""
    n, d = 6, 3
    x, w, D, Q = orc.operator_1d(n, "gl")
    u = state("product", 4, n, d, seed=800)
    y = run_gpu(torch_dev, sf, u, n, d, "product", Q=D, w=np.ones(n))
    ref = orc.dense_volume(u, n, d, "product", Q=D, w=np.ones(n))
    assert normwise(y, ref)[0].max() <= TOL64


def test_gamma_override(torch_dev, sf, orc):
    u = state("euler", 5, 4, 3, seed=900)
    y = run_gpu(torch_dev, sf, u, 4, 3, "euler", gamma=5.0 / 3.0)
    ref = orc.dense_volume(u, 4, 3, "euler", gamma=5.0 / 3.0)
    assert normwise(y, ref)[0].max() <= TOL64


def test_side_stream_and_raw_entry(torch_dev, sf):
    torch = torch_dev
    u = torch.from_numpy(state("euler", 300, 5, 3, seed=1000)).cuda()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        a = sf.volume(u, 5, 3, "euler", stream=s)
    s.synchronize()
    b = torch.empty_like(u)
    torch.cuda.synchronize()
    assert sf.volume_raw(u.data_ptr(), 300, 5, 3, 1, b.data_ptr()) == 0
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    c = torch.empty_like(u)
    assert sf.dense_volume_raw(u.data_ptr(), 300, 5, 3, 1, c.data_ptr()) == 0
    torch.cuda.synchronize()
    assert (a - c).abs().max().item() <= TOL64 * a.abs().max().item()


def test_staging_log1p_accuracy(torch_dev, sf):
    """The staging logarithm against mpmath (40 digits): <= 2 ulp of the result
    plus one ulp of the argument, over the ranges the relative logs see."""
    import mpmath as mp
    torch = torch_dev
    mp.mp.dps = 40
    rng = np.random.default_rng(1100)
    x = np.concatenate([rng.uniform(-0.9, 3.0, 3000), rng.uniform(-1e-3, 1e-3, 1000),
                        10.0 ** rng.uniform(-18, -6, 500) * rng.choice([-1, 1], 500),
                        10.0 ** rng.uniform(0, 30, 300), [0.0, -0.5, 1.0, 2.0 ** -30]])
    y = sf.diag_log1p(torch.from_numpy(x).cuda()).cpu().numpy()
    worst = 0.0
    for xi, yi in zip(x, y):
        ref = mp.log1p(mp.mpf(float(xi)))
        err = abs(mp.mpf(float(yi)) - ref)
        tol = 2 * np.spacing(abs(float(ref))) + np.spacing(abs(xi)) / (1 + xi)
        worst = max(worst, float(err / max(tol, 1e-300)))
        assert err <= tol, (xi, float(yi), float(ref))
    assert y[-4] == 0.0
    print("log1p worst error / tolerance", worst)


def test_map_log_exp_accuracy(torch_dev, sf):
    """The logarithm and exponential of the entropy-variable maps against
    mpmath (40 digits): within 2 ulp of the result over the double range,
    subnormal arguments of ln included (1 ulp of the smallest subnormal more
    where e^x is subnormal), and the
    special values: ln 0 = -inf, ln of a negative or NaN = NaN, ln inf = inf,
    e^x = 0 or inf beyond the range, e^(+-inf) = inf, 0, e^NaN = NaN."""
    import mpmath as mp
    torch = torch_dev
    mp.mp.dps = 40
    rng = np.random.default_rng(1200)
    tiny = 2.2250738585072014e-308
    xl = np.concatenate([rng.uniform(1e-3, 10.0, 2000), 10.0 ** rng.uniform(-307, 308, 2000),
                         1.0 + rng.uniform(-1e-6, 1e-6, 500), rng.uniform(0.5, 2.0, 1000),
                         [5e-324, 1e-320, 1e-310, 2.2250738585072009e-308,   # subnormal
                          1.0, 2.0, 0.5, np.nextafter(1.0, 2.0), np.nextafter(1.0, 0.0), tiny,
                          1.7976931348623157e308]])
    yl = sf.diag_log(torch.from_numpy(xl).cuda()).cpu().numpy()
    for xi, yi in zip(xl, yl):
        ref = mp.log(mp.mpf(float(xi)))
        assert abs(mp.mpf(float(yi)) - ref) <= 2 * np.spacing(abs(float(ref))), (xi, yi, float(ref))
    assert yl[-7] == 0.0
    xe = np.concatenate([rng.uniform(-700.0, 700.0, 3000), rng.uniform(-1.0, 1.0, 1000),
                         rng.uniform(-1e-10, 1e-10, 200), rng.uniform(-745.0, -708.5, 200),
                         [0.0, 1.0, -1.0, 709.78, -708.39]])
    ye = sf.diag_exp(torch.from_numpy(xe).cuda()).cpu().numpy()
    for xi, yi in zip(xe, ye):
        ref = mp.exp(mp.mpf(float(xi)))
        tol = 2 * np.spacing(float(ref)) + (5e-324 if float(ref) < tiny else 0.0)
        assert abs(mp.mpf(float(yi)) - ref) <= tol, (xi, yi, float(ref))
    assert ye[-5] == 1.0
    inf, nan = np.inf, np.nan
    sl = sf.diag_log(torch.tensor([0.0, -0.0, -1.0, -inf, inf, nan], dtype=torch.float64).cuda()).cpu().numpy()
    assert sl[0] == -inf and sl[1] == -inf and np.isnan(sl[2]) and np.isnan(sl[3])
    assert sl[4] == inf and np.isnan(sl[5])
    se = sf.diag_exp(torch.tensor([710.0, -746.0, 1e300, -1e300, inf, -inf, nan],
                                  dtype=torch.float64).cuda()).cpu().numpy()
    assert se[0] == inf and se[1] == 0.0 and se[2] == inf and se[3] == 0.0
    assert se[4] == inf and se[5] == 0.0 and np.isnan(se[6])


def test_library_is_the_path(torch_dev, sf):
    """The product path runs the in-tree HIP library, nothing else."""
    import ctypes
    maps = open("/proc/self/maps").read()
    assert os.path.realpath(sf.LIB_PATH) in maps


def test_concurrent_host_threads_on_own_streams(torch_dev, sf):
    """Four host threads call the library at once, each on its own stream and
    with its own shapes (first calls of new (n, node kind) operators race in
    the mutex-protected cache): every result equals the same call made alone."""
    import threading
    torch = torch_dev
    assert sf.lib().sf_init(0, 8) == 0
    cases = [(3, "gll", 0), (5, "gl", 1), (6, "gll", 2), (7, "gl", 3)]
    inputs, alone = [], []
    for n, kind, seed in cases:
        u = torch.from_numpy(state("euler", 300, n, 3, seed=900 + seed, fs=0.1)).cuda()
        inputs.append(u)
    outs = [None] * len(cases)
    errs = []

    def worker(i):
        try:
            n, kind, _ = cases[i]
            s = torch.cuda.Stream()
            res = []
            for _ in range(20):
                res.append(sf.volume(inputs[i], n, 3, "euler", nodes=kind, stream=s))
            s.synchronize()
            outs[i] = res
        except Exception as e:  # surfaced below
            errs.append(e)

    ths = [threading.Thread(target=worker, args=(i,)) for i in range(len(cases))]
    for th in ths:
        th.start()
    for th in ths:
        th.join(timeout=120)
    assert not errs, errs
    torch.cuda.synchronize()
    for i, (n, kind, _) in enumerate(cases):
        ref = sf.volume(inputs[i], n, 3, "euler", nodes=kind)
        torch.cuda.synchronize()
        for r in outs[i]:
            assert torch.equal(r, ref), (n, kind)


def test_binding_rejects_outputs_off_the_device(torch_dev, sf):
    """Caller-provided outputs must be contiguous float64 tensors on the input's
    device: a host tensor is refused before any launch (its pointer would
    reach the kernel)."""
    torch = torch_dev
    from paper_2306_11665_amd import workloads as W
    n, E = 3, 4
    u_np = W.euler_state(E, n, seed=1)
    u = torch.from_numpy(u_np).cuda()
    # facet states: each element's first node state on all of its facet nodes
    uf = torch.from_numpy(np.ascontiguousarray(
        np.repeat(u_np[:, :, :1], 6 * n * n, axis=2).reshape(5, E, 6, n * n))).cuda()
    host = torch.empty((5, E, n ** 3), dtype=torch.float64)
    with pytest.raises(ValueError):
        sf.volume(u, n, 3, "euler", out=host)
    with pytest.raises(ValueError):
        sf.volume(u, n, 3, "euler", out=torch.empty((5, E, n ** 3), dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError):
        sf.entropy_variables(u, out=host)
    with pytest.raises(ValueError):
        sf.entropy_trace(u, n, out=torch.empty((5, E, 6, n * n), dtype=torch.float64))
    with pytest.raises(ValueError):
        sf.surface(u, uf, n, 3, "euler", y_vol=host)
    with pytest.raises(ValueError):
        sf.surface(u, uf, n, 3, "euler", y_face=torch.empty((5, E, 6, n * n), dtype=torch.float64))
    Ja = torch.zeros((3, 3, E, n ** 3), dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        sf.volume_curvilinear(u, Ja, n, out=host)
    with pytest.raises(ValueError):
        sf.tensor_apply(u, n, 3, np.eye(n), out=host)
    # the same calls with device outputs run
    y = sf.volume(u, n, 3, "euler", out=torch.empty_like(u))
    torch.cuda.synchronize()
    assert torch.isfinite(y).all()
