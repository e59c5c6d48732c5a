"""Host tests of the serving runtime with the simulated executor (no GPU).

The scheduler, FIFO admission, HBM-budget accounting, batching into launch
slots, release/unregister rules and argument checks run exactly as on the
device; only the executor is the host simulation (sf_server_create_sim),
which completes a batch a fixed time per element block after it starts.
"""
import time

import numpy as np
import pytest

from paper_2306_11665_amd import sfhad


@pytest.fixture(scope="module")
def serving():
    from paper_2306_11665_amd import serving
    sfhad.lib()
    return serving


def tiny_state(E, n):
    return np.ones((5, E, n ** 3))


def out_bytes(E, n):
    b = 5 * E * n ** 3 * 8
    return (b + 255) // 256 * 256


def test_budget_admission_fifo_and_release(serving):
    E, n = 64, 4                       # 4 elements per block -> 16 blocks
    budget = 3 * out_bytes(E, n)
    with serving.Server(budget, max_inflight=64, sim_us_per_block=2000.0) as srv:   # 32 ms per request
        m = srv.register(tiny_state(E, n), n)
        ts = [srv.submit(m.mesh_id) for _ in range(7)]
        wait_until(lambda: srv.stats()[1] == 3)
        q, inflight, used = srv.stats()
        assert inflight == 3 and q == 4 and used == 3 * out_bytes(E, n)
        # nothing beyond the budget ever holds memory; completion is FIFO
        order = []
        for t in ts:
            srv.wait(t)
            order.append(t)
            _, inflight, used = srv.stats()
            assert inflight <= 3 and used <= budget
            srv.release(t)
        assert order == sorted(order)
        assert srv.stats() == (0, 0, 0)


def wait_until(cond, timeout=5.0):
    """Poll cond() until it holds (the scheduler thread runs on its own
    time, later under a loaded host): the tests wait for the state they
    check instead of sleeping a fixed time."""
    t_end = time.monotonic() + timeout
    while not cond():
        assert time.monotonic() < t_end, "condition not reached"
        time.sleep(0.0005)


def test_requests_arriving_mid_flight_join_the_next_batch(serving):
    E, n = 32, 4                       # 8 blocks
    with serving.Server(1 << 30, max_inflight=64, sim_us_per_block=25000.0) as srv:   # 200 ms per request
        m = srv.register(tiny_state(E, n), n)
        t0 = srv.submit(m.mesh_id)
        wait_until(lambda: srv.batch_stats()[0] == 1)   # t0 is launched in one slot,
        ta = srv.submit(m.mesh_id)
        wait_until(lambda: srv.batch_stats()[0] == 2)   # ta in the other
        t1 = srv.submit(m.mesh_id)         # admitted at once (budget is free) ...
        t2 = srv.submit(m.mesh_id)
        wait_until(lambda: srv.stats()[:2] == (0, 4))
        assert srv.batch_stats()[0] == 2   # ... and wait for a slot
        _, l0 = srv.wait(t0)
        _, la = srv.wait(ta)
        _, l1 = srv.wait(t1)
        _, l2 = srv.wait(t2)
        # when t0's slot frees they go as one batch (16 blocks), finish
        # together, after ta
        assert abs(l1 - l2) < 0.05
        assert l0 < la
        assert l1 > 0.5                    # behind t0's 200 ms, then 400 ms of their own
        # three batches (t0; ta; t1 + t2), two of them on the device at once
        assert srv.batch_stats() == (3, 2, 2)
        for t in (t0, ta, t1, t2):
            srv.release(t)


def test_max_inflight_bound(serving):
    with serving.Server(1 << 30, max_inflight=2, sim_us_per_block=50000.0) as srv:   # 200 ms per request
        m = srv.register(tiny_state(16, 4), 4)
        ts = [srv.submit(m.mesh_id) for _ in range(5)]
        wait_until(lambda: srv.stats()[1] == 2)
        q, inflight, _ = srv.stats()
        assert inflight == 2 and q == 3
        for t in ts:
            srv.wait(t)
            _, inflight, _ = srv.stats()
            assert inflight <= 2
            srv.release(t)


def test_rejections_and_errors(serving):
    E, n = 64, 4
    with serving.Server(out_bytes(E, n) - 256, max_inflight=8, sim_us_per_block=0.0) as srv:
        m = srv.register(tiny_state(E, n), n)
        with pytest.raises(sfhad.SFError) as e:
            srv.submit(m.mesh_id)                         # larger than the whole budget
        assert e.value.status == -5
        with pytest.raises(sfhad.SFError) as e:
            srv.register(tiny_state(4, 9), 9)             # n > 8 not built for serving
        assert e.value.status == -2
        with pytest.raises(sfhad.SFError) as e:
            srv.submit(12345)
        assert e.value.status == -7
        with pytest.raises(sfhad.SFError) as e:
            srv.wait(999)
        assert e.value.status == -7
        with pytest.raises(sfhad.SFError) as e:
            srv.release(4242)
        assert e.value.status == -7
    with serving.Server(1 << 30, max_inflight=8, sim_us_per_block=20000.0) as srv:
        m = srv.register(tiny_state(16, 4), 4)
        t = srv.submit(m.mesh_id)
        with pytest.raises(sfhad.SFError) as e:
            srv.release(t)                                # not complete yet
        assert e.value.status == -6
        with pytest.raises(sfhad.SFError) as e:
            srv.unregister(m.mesh_id)                     # request outstanding
        assert e.value.status == -6
        assert not srv.poll(t)
        srv.wait(t)
        assert srv.poll(t)
        srv.release(t)
        srv.unregister(m.mesh_id)


def test_c_level_argument_checks(serving):
    import ctypes
    L = serving._lib()
    h = ctypes.c_void_p()
    assert L.sf_server_create_sim(1 << 20, 0, 1.0, ctypes.byref(h)) == -1
    assert L.sf_server_create_sim(1 << 20, 2000, 1.0, ctypes.byref(h)) == -1
    assert L.sf_server_create_sim(1 << 20, 8, -1.0, ctypes.byref(h)) == -1
    assert L.sf_server_create_sim(1 << 20, 8, 1.0, None) == -1
    assert L.sf_submit(None, 1, 0, None) == -1
    assert L.sf_server_destroy(None) == -1
    assert L.sf_server_create_sim(1 << 20, 8, 1.0, ctypes.byref(h)) == 0
    t = ctypes.c_int64()
    assert L.sf_submit(h, 1, 7, ctypes.byref(t)) == -1            # bad precision
    u = np.ones((5, 4, 27))
    m = ctypes.c_int64()
    dp = u.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert L.sf_mesh_register(h, dp, 4, 3, 0, 0, ctypes.byref(m)) == -2   # Burgers not served
    assert L.sf_mesh_register(h, dp, 0, 3, 1, 0, ctypes.byref(m)) == -1   # E = 0
    assert L.sf_mesh_register(h, dp, 4, 3, 1, 5, ctypes.byref(m)) == -1   # node kind
    assert L.sf_server_destroy(h) == 0


def test_poisson_load_on_simulated_device(serving):
    from paper_2306_11665_amd import workloads as W
    specs = [W.MeshSpec(k, 3 + k % 6, 64 * (k + 1), 0) for k in range(6)]
    with serving.Server(64 << 20, max_inflight=64, sim_us_per_block=5.0) as srv:
        meshes = [srv.register(tiny_state(s.E, s.n), s.n) for s in specs]
        arr, which = W.poisson_arrivals(2000.0, 300, len(meshes), seed=5)
        res = serving.run_load(srv, meshes, arr, which, skip=20)
        s = res.summary()
        assert s["requests"] == 280
        assert 0 < s["p50_ms"] <= s["p99_ms"] <= s["max_ms"] < 1000
        assert srv.stats() == (0, 0, 0)


def test_concurrent_clients_stress(serving):
    """Four client threads submit, wait and release requests on random meshes
    (registered and unregistered while others run) against a small budget:
    the budget and the in-flight bound hold at every observation, every
    request completes, and the server ends empty."""
    import threading
    budget = 6 * out_bytes(64, 4)
    errors = []
    with serving.Server(budget, max_inflight=5, sim_us_per_block=20.0) as srv:
        base = [srv.register(tiny_state(16 * (k + 1), 4), 4) for k in range(4)]
        lock = threading.Lock()

        def client(seed):
            rng = np.random.default_rng(seed)
            try:
                for it in range(40):
                    m = base[rng.integers(len(base))]
                    ts = [srv.submit(m.mesh_id, "fp64" if rng.random() < 0.5 else "fp32_split")
                          for _ in range(int(rng.integers(1, 4)))]
                    q, inflight, used = srv.stats()
                    assert used <= budget and inflight <= 5, (used, inflight)
                    for t in ts:
                        srv.wait(t)
                        srv.release(t)
                    if it % 10 == 0:                         # a private mesh comes and goes
                        with lock:
                            extra = srv.register(tiny_state(8, 3), 3)
                        t = srv.submit(extra.mesh_id)
                        srv.wait(t)
                        srv.release(t)
                        srv.unregister(extra.mesh_id)
            except Exception as e:                           # surfaced below
                errors.append(e)

        ths = [threading.Thread(target=client, args=(s,)) for s in range(4)]
        for th in ths:
            th.start()
        for th in ths:
            th.join(timeout=120)
        assert not any(th.is_alive() for th in ths)
        assert not errors, errors
        assert srv.stats() == (0, 0, 0)


def test_failed_batch_launch_reports_to_waiters(serving):
    """A batch whose launch fails completes its requests with SF_ERR_HIP; they
    are released normally and later batches run."""
    import ctypes
    L = serving._lib()
    L.sf_server_sim_fail_launches.argtypes = [ctypes.c_void_p, ctypes.c_int]
    with serving.Server(1 << 30, max_inflight=8, sim_us_per_block=50.0) as srv:
        m = srv.register(tiny_state(16, 4), 4)
        assert L.sf_server_sim_fail_launches(srv._h, 1) == 0
        b0 = srv.batch_stats()[0]
        bad = [srv.submit(m.mesh_id) for _ in range(2)]
        failed = []
        for t in bad:
            try:
                srv.wait(t)
                failed.append(False)
            except sfhad.SFError as e:
                assert e.status == -3 and "launched" in str(e)
                failed.append(True)
            srv.release(t)
        # the first request is in the failed batch; the second joined it, or
        # (when the scheduler woke between the two submissions) ran in the next one
        assert failed[0]
        assert failed[1] == (srv.batch_stats()[0] - b0 == 1)
        good = srv.submit(m.mesh_id)
        srv.wait(good)
        srv.release(good)
        assert srv.stats() == (0, 0, 0)
    assert L.sf_server_sim_fail_launches(None, 1) == -1
