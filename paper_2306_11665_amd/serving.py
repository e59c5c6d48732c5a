"""Serving-loop binding (sf_server_* in include/sfhad.h) and a Poisson load driver.

The scheduler, admission, batching and launches all run in the C++ runtime of
libsfhad.so; this module marshals arguments, copies results out of the
server's device buffers for inspection, and drives arrival processes.
"""
from __future__ import annotations

import ctypes
import threading
import time
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from . import sfhad

_i64 = ctypes.c_int64
_vp = ctypes.c_void_p
_hip = None


def _hiplib():
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [_vp, _vp, ctypes.c_size_t, ctypes.c_int]
        _hip.hipMemcpy.restype = ctypes.c_int
    return _hip


def _lib():
    L = sfhad.lib()
    if not getattr(L, "_serving_ready", False):
        L.sf_server_create_sim.argtypes = [ctypes.c_size_t, ctypes.c_int, ctypes.c_double,
                                           ctypes.POINTER(_vp)]
        L.sf_server_create_sim.restype = ctypes.c_int
        L.sf_server_stats.argtypes = [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_i64)]
        L.sf_server_stats.restype = ctypes.c_int
        L.sf_server_batch_stats.argtypes = [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_i64)]
        L.sf_server_batch_stats.restype = ctypes.c_int
        L._serving_ready = True
    return L


@dataclass
class MeshInfo:
    mesh_id: int
    E: int
    n: int

    @property
    def nodes(self) -> int:
        return self.n ** 3

    @property
    def dof(self) -> int:
        return 5 * self.E * self.nodes


class Server:
    """A serving loop on the current device (or a simulated one)."""

    def __init__(self, budget_bytes: int, max_inflight: int = 256, sim_us_per_block: Optional[float] = None):
        L = _lib()
        h = _vp()
        if sim_us_per_block is None:
            st = L.sf_server_create(int(budget_bytes), int(max_inflight), ctypes.byref(h))
        else:
            st = L.sf_server_create_sim(int(budget_bytes), int(max_inflight), float(sim_us_per_block),
                                        ctypes.byref(h))
        sfhad.check(st, "sf_server_create")
        self._h = h
        self.sim = sim_us_per_block is not None
        self.meshes: dict = {}
        self._tickets: dict = {}

    def register(self, u, n: int, nodes: str = "gl") -> MeshInfo:
        """Register a mesh state (5, E, n^3): a host array, or a contiguous
        float64 CUDA tensor (copied device to device)."""
        if hasattr(u, "is_cuda") and u.is_cuda:
            import torch
            if u.dtype != torch.float64 or not u.is_contiguous():
                raise ValueError("a device state must be a contiguous float64 tensor")
            shape, ptr = tuple(u.shape), ctypes.cast(ctypes.c_void_p(u.data_ptr()), ctypes.POINTER(ctypes.c_double))
            torch.cuda.synchronize(u.device)           # the state is complete before the copy
        else:
            u = np.ascontiguousarray(u, dtype=np.float64)
            shape, ptr = u.shape, u.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        if len(shape) != 3 or shape[0] != 5 or shape[2] != n ** 3:
            raise ValueError(f"state must be (5, E, {n ** 3}), got {shape}")
        mid = _i64()
        sfhad.check(_lib().sf_mesh_register(self._h, ptr, shape[1], n, sfhad.FLUX["euler"], sfhad.NODES[nodes],
                                            ctypes.byref(mid)), "sf_mesh_register")
        info = MeshInfo(mid.value, shape[1], n)
        self.meshes[info.mesh_id] = info
        return info

    def submit(self, mesh: int, precision: str = "fp64") -> int:
        t = _i64()
        sfhad.check(_lib().sf_submit(self._h, mesh, sfhad.PRECISION[precision], ctypes.byref(t)), "sf_submit")
        self._tickets[t.value] = mesh
        return t.value

    def poll(self, ticket: int) -> bool:
        return sfhad.check(_lib().sf_poll(self._h, ticket), "sf_poll") == 1

    def wait(self, ticket: int):
        """(device pointer of the result or None, latency in seconds)."""
        y = _vp()
        lat = ctypes.c_double()
        sfhad.check(_lib().sf_wait(self._h, ticket, ctypes.byref(y), ctypes.byref(lat)), "sf_wait")
        return y.value, lat.value

    def result(self, ticket: int) -> np.ndarray:
        """Copy a completed ticket's output (5, E, n^3) to the host."""
        ptr, _ = self.wait(ticket)
        info = self.meshes[self._tickets[ticket]]
        out = np.empty((5, info.E, info.nodes))
        if ptr is None:
            raise RuntimeError("a simulated server has no results")
        st = _hiplib().hipMemcpy(out.ctypes.data, ptr, out.nbytes, 2)  # device to host
        if st != 0:
            raise RuntimeError(f"hipMemcpy failed ({st})")
        return out

    def release(self, ticket: int) -> None:
        sfhad.check(_lib().sf_release(self._h, ticket), "sf_release")
        self._tickets.pop(ticket, None)

    def unregister(self, mesh: int) -> None:
        sfhad.check(_lib().sf_mesh_unregister(self._h, mesh), "sf_mesh_unregister")
        self.meshes.pop(mesh, None)

    def stats(self):
        q, i, u = _i64(), _i64(), _i64()
        sfhad.check(_lib().sf_server_stats(self._h, ctypes.byref(q), ctypes.byref(i), ctypes.byref(u)),
                    "sf_server_stats")
        return q.value, i.value, u.value

    def batch_stats(self):
        """(batches launched, most requests in one batch, most slots busy at once)."""
        b, r, k = _i64(), _i64(), _i64()
        sfhad.check(_lib().sf_server_batch_stats(self._h, ctypes.byref(b), ctypes.byref(r), ctypes.byref(k)),
                    "sf_server_batch_stats")
        return b.value, r.value, k.value

    def close(self) -> None:
        if self._h:
            _lib().sf_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


@dataclass
class LoadResult:
    latencies: np.ndarray
    submitted: int
    wall_s: float
    dof: int
    elements: int
    lateness_s: float
    results: dict = field(default_factory=dict)

    def summary(self) -> dict:
        lat = self.latencies
        return {
            "requests": int(len(lat)),
            "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p90_ms": float(np.percentile(lat, 90) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "max_ms": float(lat.max() * 1e3),
            "dof_per_s": self.dof / self.wall_s,
            "elem_evals_per_s": self.elements / self.wall_s,
            "wall_s": self.wall_s,
            "max_submit_lateness_ms": self.lateness_s * 1e3,
        }


def run_load(srv: Server, meshes: list, arrivals: np.ndarray, which: np.ndarray, precision="fp64",
             collect: bool = False, skip: int = 0) -> LoadResult:
    """Submit request k for mesh meshes[which[k]] at time arrivals[k] (seconds
    from now), with precision `precision` (one name, or one per request); a
    consumer thread waits, records and releases in submission order.  The
    first `skip` requests are excluded from the statistics.  The submitting
    thread only sleeps (no spinning), so the consumer is never starved of the
    interpreter lock."""
    import sys
    count = len(arrivals)
    precs = [precision] * count if isinstance(precision, str) else list(precision)
    tickets = [None] * count
    lat = np.zeros(count)
    done_ev = [threading.Event() for _ in range(count)]
    results = {}
    err = []

    def consumer():
        try:
            for k in range(count):
                done_ev[k].wait()
                t = tickets[k]
                _, latency = srv.wait(t)
                lat[k] = latency
                if collect:
                    results[k] = srv.result(t)
                srv.release(t)
        except Exception as e:  # surfaced after join
            err.append(e)

    old_switch = sys.getswitchinterval()
    sys.setswitchinterval(5e-5)
    th = threading.Thread(target=consumer, daemon=True)
    th.start()
    t0 = time.perf_counter()
    late = 0.0
    try:
        for k in range(count):
            target = t0 + arrivals[k]
            now = time.perf_counter()
            if target > now:
                time.sleep(target - now)
            late = max(late, time.perf_counter() - target)
            tickets[k] = srv.submit(meshes[which[k]].mesh_id, precs[k])
            done_ev[k].set()
        th.join()
    finally:
        sys.setswitchinterval(old_switch)
    wall = time.perf_counter() - t0
    if err:
        raise err[0]
    sel = slice(skip, count)
    dof = sum(meshes[which[k]].dof for k in range(skip, count))
    elements = sum(meshes[which[k]].E for k in range(skip, count))
    t_first = arrivals[skip] if skip < count else 0.0
    return LoadResult(lat[sel], count - skip, wall - t_first, dof, elements, late, results)


def saturation_rate(srv: Server, meshes: list, which: np.ndarray, precision: str = "fp64") -> float:
    """Requests per second when `which` is submitted as one burst (the
    device is never idle): the throughput capacity of the serving loop."""
    t0 = time.perf_counter()
    tickets = [srv.submit(meshes[k].mesh_id, precision) for k in which]
    for t in tickets:
        srv.wait(t)
        srv.release(t)
    return len(which) / (time.perf_counter() - t0)
