"""GPU tests of the serving loop: served results equal the direct call, and
each request's result is the same alone and inside a Poisson mix of
concurrent requests of mixed n and precision (continuous batching)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    from paper_2306_11665_amd import serving, sfhad, workloads
    sfhad.lib()
    return torch, serving, sfhad, workloads


def test_served_result_equals_direct_call(env, orc):
    torch, serving, sfhad, W = env
    with serving.Server(1 << 30, max_inflight=16) as srv:
        cases = [(n, E, nodes) for n, E in [(2, 129), (3, 37), (4, 65), (5, 101), (6, 23), (7, 11), (8, 40)]
                 for nodes in ("gl", "gll")]
        for n, E, nodes in cases:
            u = W.euler_state(E, n, seed=1200 + n, freestream_frac=0.1)
            m = srv.register(u, n, nodes)
            for prec in ("fp64", "fp32_split"):
                t = srv.submit(m.mesh_id, prec)
                y = srv.result(t)
                srv.release(t)
                ref = sfhad.volume(torch.from_numpy(u).cuda(), n, 3, "euler", nodes=nodes,
                                   precision=prec).cpu().numpy()
                assert np.array_equal(y, ref), (n, prec, np.abs(y - ref).max())
            orc_ref = orc.dense_volume(u[:, :3], n, 3, "euler", nodes_kind=nodes)
            t = srv.submit(m.mesh_id, "fp64")
            y = srv.result(t)[:, :3]
            srv.release(t)
            err = max(np.abs(y[v] - orc_ref[v]).max() / np.abs(orc_ref[v]).max() for v in range(5))
            assert err <= 1e-12, err


def test_alone_equals_mix(env):
    torch, serving, sfhad, W = env
    specs = [W.MeshSpec(k, n, E, 1300 + k) for k, (n, E) in
             enumerate([(3, 700), (4, 513), (5, 1200), (6, 333), (7, 900), (8, 640), (8, 2000), (4, 4000)])]
    with serving.Server(2 << 30, max_inflight=64) as srv:
        meshes = [srv.register(W.serving_mesh_state(s), s.n) for s in specs]
        alone = {}
        for i, m in enumerate(meshes):
            for prec in ("fp64", "fp32_split"):
                t = srv.submit(m.mesh_id, prec)
                alone[(i, prec)] = srv.result(t)
                srv.release(t)
        rng = np.random.default_rng(1301)
        count = 96
        arr, which = W.poisson_arrivals(40000.0, count, len(meshes), seed=1302)   # ~25 us apart: well inside one request's latency
        precs = rng.choice(["fp64", "fp32_split"], size=count)
        # run both precisions in one mix: submit per request with its precision
        tickets = []
        import time
        t0 = time.perf_counter()
        for k in range(count):
            while time.perf_counter() - t0 < arr[k]:
                pass
            tickets.append(srv.submit(meshes[which[k]].mesh_id, str(precs[k])))
        b0, _, _ = srv.batch_stats()
        for k, t in enumerate(tickets):
            y = srv.result(t)
            ref = alone[(int(which[k]), str(precs[k]))]
            assert np.array_equal(y, ref), (k, int(which[k]), str(precs[k]))
            srv.release(t)
        batches, max_reqs, max_busy = srv.batch_stats()
        print(f"mix: {batches - b0} batches for {count} requests, at most {max_reqs} requests in one batch, "
              f"at most {max_busy} batches on the device at once")
        assert max_reqs >= 2      # requests that arrived while others ran were packed into one batch
        assert max_busy >= 2      # a batch started while the previous one was still running


def test_register_from_device_memory(env):
    """sf_mesh_register takes a device pointer as well as a host one: both
    registrations give the same, bitwise equal, results."""
    torch, serving, sfhad, W = env
    n, E = 5, 300
    u = W.euler_state(E, n, seed=1350)
    ud = torch.from_numpy(u).cuda()
    with serving.Server(1 << 30, max_inflight=8) as srv:
        mh = srv.register(u, n)
        md = srv.register(ud, n)
        del ud                                         # the server holds its own copy
        torch.cuda.empty_cache()
        out = []
        for m in (mh, md):
            t = srv.submit(m.mesh_id)
            out.append(srv.result(t))
            srv.release(t)
        assert np.array_equal(out[0], out[1])
        ref = sfhad.volume(torch.from_numpy(u).cuda(), n, 3, "euler").cpu().numpy()
        assert np.array_equal(out[1], ref)


def test_small_budget_forces_queueing(env):
    torch, serving, sfhad, W = env
    n, E = 6, 500
    u = W.euler_state(E, n, seed=1400)
    nbytes = 5 * E * n ** 3 * 8
    with serving.Server(int(2.5 * nbytes) + 1024, max_inflight=64) as srv:
        m = srv.register(u, n)
        ref = sfhad.volume(torch.from_numpy(u).cuda(), n, 3, "euler").cpu().numpy()
        ts = [srv.submit(m.mesh_id) for _ in range(12)]
        q, inflight, used = srv.stats()
        assert inflight <= 2 and used <= 2.5 * nbytes + 1024
        for t in ts:
            y = srv.result(t)
            assert np.array_equal(y, ref)
            srv.release(t)
        assert srv.stats() == (0, 0, 0)
        srv.unregister(m.mesh_id)
