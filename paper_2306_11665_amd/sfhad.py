"""Thin ctypes binding of libsfhad.so (C-ABI in include/sfhad.h).

Argument marshalling only: every step of the volume term runs in the HIP
library.  PyTorch provides device memory and the stream; tensors must be
contiguous float64 CUDA tensors in the layout u[v, e, node].  If the library
is not built, every call raises -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsfhad.so")

FLUX = {"burgers": 0, "euler": 1, "product": 2, "euler_pfix": 3}
NODES = {"gl": 0, "gll": 1}
PRECISION = {"fp64": 0, "fp32_split": 1}
NVAR = {"burgers": 1, "euler": 5, "product": 1, "euler_pfix": 5}
STATUS = {0: "SF_OK", -1: "SF_ERR_ARG", -2: "SF_ERR_UNSUPPORTED", -3: "SF_ERR_HIP",
          -4: "SF_ERR_NOMEM", -5: "SF_ERR_BUDGET", -6: "SF_ERR_BUSY", -7: "SF_ERR_NOT_FOUND"}


class SFError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)}" + (f" ({detail})" if detail else ""))


class SfOpts(ctypes.Structure):
    _fields_ = [("node_kind", ctypes.c_int), ("precision", ctypes.c_int), ("gamma", ctypes.c_double),
                ("stream", ctypes.c_void_p), ("op_1d_host", ctypes.POINTER(ctypes.c_double)),
                ("w_1d_host", ctypes.POINTER(ctypes.c_double))]


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)


def lib() -> ctypes.CDLL:
    """Open libsfhad.so once (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2306_11665_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        i64, ci, vp = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
        for name in ("sf_hadamard_volume", "dense_hadamard_volume"):
            f = getattr(L, name)
            f.argtypes = [vp, i64, ci, ci, ci, vp]
            f.restype = ci
        for name in ("sf_hadamard_volume_ex", "dense_hadamard_volume_ex"):
            f = getattr(L, name)
            f.argtypes = [vp, i64, ci, ci, ci, vp, ctypes.POINTER(SfOpts)]
            f.restype = ci
        L.sf_opts_init.argtypes = [ctypes.POINTER(SfOpts)]
        L.sf_opts_init.restype = ci
        L.sf_operator_1d.argtypes = [ci, ci, _dp, _dp, _dp]
        L.sf_operator_1d.restype = ci
        L.sf_init.argtypes = [ci, ci]
        L.sf_init.restype = ci
        L.sf_status_string.argtypes = [ci]
        L.sf_status_string.restype = ctypes.c_char_p
        L.sf_last_error.argtypes = []
        L.sf_last_error.restype = ctypes.c_char_p
        L.sf_version.argtypes = []
        L.sf_version.restype = ctypes.c_char_p
        vpp = ctypes.POINTER(ctypes.c_void_p)
        L.sf_server_create.argtypes = [ctypes.c_size_t, ci, vpp]
        L.sf_server_create.restype = ci
        L.sf_mesh_register.argtypes = [vp, _dp, i64, ci, ci, ci, ctypes.POINTER(i64)]
        L.sf_mesh_register.restype = ci
        L.sf_submit.argtypes = [vp, i64, ci, ctypes.POINTER(i64)]
        L.sf_submit.restype = ci
        L.sf_poll.argtypes = [vp, i64]
        L.sf_poll.restype = ci
        L.sf_wait.argtypes = [vp, i64, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_double)]
        L.sf_wait.restype = ci
        for name in ("sf_release", "sf_mesh_unregister"):
            getattr(L, name).argtypes = [vp, i64]
            getattr(L, name).restype = ci
        for name in ("sf_hadamard_surface", "sf_hadamard_volume_surface"):
            getattr(L, name).argtypes = [vp, vp, i64, ci, ci, ci, vp, vp, ctypes.POINTER(SfOpts)]
            getattr(L, name).restype = ci
        L.sf_hadamard_volume_curvilinear.argtypes = [vp, vp, i64, ci, ci, vp, ctypes.POINTER(SfOpts)]
        L.sf_hadamard_volume_curvilinear.restype = ci
        for name in ("sf_entropy_variables", "sf_conserved_variables"):
            getattr(L, name).argtypes = [vp, i64, vp, ctypes.c_double, vp]
            getattr(L, name).restype = ci
        L.sf_entropy_trace.argtypes = [vp, i64, ci, vp, ctypes.POINTER(SfOpts)]
        L.sf_entropy_trace.restype = ci
        L.sf_surface_operator_1d.argtypes = [ci, ci, _dp, _dp]
        L.sf_surface_operator_1d.restype = ci
        L.sf_basis_1d.argtypes = [ci, ci, _dp, _dp]
        L.sf_basis_1d.restype = ci
        L.sf_tensor_apply.argtypes = [vp, i64, ci, ci, ci, _dp, vp, vp]
        L.sf_tensor_apply.restype = ci
        L.sf_tensor_apply_rect.argtypes = [vp, i64, ci, ci, ci, ci, _dp, vp, vp]
        L.sf_tensor_apply_rect.restype = ci
        L.sf_tensor_apply_rect_map.argtypes = [vp, i64, ci, ci, ci, ctypes.c_double, _dp, vp, vp]
        L.sf_tensor_apply_rect_map.restype = ci
        L.sf_basis_rect.argtypes = [ci, ci, ci, _dp, _dp]
        L.sf_basis_rect.restype = ci
        for name in ("sf_diag_log1p", "sf_diag_log", "sf_diag_exp"):
            getattr(L, name).argtypes = [vp, i64, vp, vp]
            getattr(L, name).restype = ci
        L.sf_server_destroy.argtypes = [vp]
        L.sf_server_destroy.restype = ci
        _lib = L
    return _lib


def last_error() -> str:
    return lib().sf_last_error().decode()


def check(status: int, where: str) -> int:
    if status < 0:
        raise SFError(status, where, last_error())
    return status


def operator_1d(n: int, nodes: str = "gl"):
    """(x, w, Q) of the library's 1D operator, Q = diag(w) D (host, FP64)."""
    x = np.zeros(n); w = np.zeros(n); Q = np.zeros((n, n))
    check(lib().sf_operator_1d(n, NODES[nodes], x.ctypes.data_as(_dp), w.ctypes.data_as(_dp),
                               Q.ctypes.data_as(_dp)), "sf_operator_1d")
    return x, w, Q


def _stream_handle(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


def _record(stream, *tensors) -> None:
    """Mark tensors as used on `stream` when it is not the current stream, so
    that torch's caching allocator does not hand their memory to another
    tensor while the launched kernels may still read or write it."""
    import torch
    if stream is None:
        return
    s = stream if isinstance(stream, torch.cuda.Stream) else torch.cuda.ExternalStream(int(stream))
    if s.cuda_stream == torch.cuda.current_stream().cuda_stream:
        return
    for t in tensors:
        if t is not None:
            t.record_stream(s)


def make_opts(nodes="gl", precision="fp64", gamma=1.4, stream=None, Q=None, w=None):
    o = SfOpts()
    lib().sf_opts_init(ctypes.byref(o))
    o.node_kind = NODES[nodes]
    o.precision = PRECISION[precision]
    o.gamma = float(gamma)
    o.stream = _stream_handle(stream)
    keep = []
    if Q is not None or w is not None:
        Qh = np.ascontiguousarray(Q, dtype=np.float64)
        wh = np.ascontiguousarray(w, dtype=np.float64)
        keep = [Qh, wh]
        o.op_1d_host = Qh.ctypes.data_as(_dp)
        o.w_1d_host = wh.ctypes.data_as(_dp)
    return o, keep


def _check_tensor(u, flux: str, n: int, d: int):
    import torch
    nv = NVAR[flux]
    if not isinstance(u, torch.Tensor) or u.device.type != "cuda" or u.dtype != torch.float64:
        raise TypeError("u must be a float64 CUDA tensor")
    if not u.is_contiguous() or u.dim() != 3 or u.shape[0] != nv or u.shape[2] != n ** d:
        raise ValueError(f"u must be a contiguous ({nv}, E, {n ** d}) tensor, got {tuple(u.shape)}")


def _check_out(out, shape, like, what: str = "out"):
    """A caller-provided output: a contiguous float64 tensor of `shape` on the
    device of `like` (a host tensor's pointer would reach the kernel)."""
    import torch
    if (not isinstance(out, torch.Tensor) or out.device != like.device or out.dtype != torch.float64
            or not out.is_contiguous() or tuple(out.shape) != tuple(shape)):
        raise ValueError(f"{what} must be a contiguous float64 tensor {tuple(shape)} on {like.device}")


def _check_same_device(x, like, what: str):
    if x.device != like.device:
        raise ValueError(f"{what} must be on {like.device}, got {x.device}")


def _call(fn_name: str, u, n: int, d: int, flux: str, *, nodes="gl", precision="fp64", gamma=1.4,
          stream=None, out=None, Q=None, w=None):
    import torch
    _check_tensor(u, flux, n, d)
    if out is None:
        out = torch.empty_like(u)
    else:
        _check_out(out, u.shape, u)
    opts, keep = make_opts(nodes, precision, gamma, stream, Q, w)
    fn = getattr(lib(), fn_name)
    check(fn(u.data_ptr(), u.shape[1], n, d, FLUX[flux], out.data_ptr(), ctypes.byref(opts)), fn_name)
    del keep
    _record(stream, u, out)
    return out


def volume(u, n: int, d: int, flux: str, **kw):
    """y = sum_m (A_m o F_m) 1 by the sum-factorized kernels (sf_hadamard_volume_ex)."""
    return _call("sf_hadamard_volume_ex", u, n, d, flux, **kw)


def dense_volume(u, n: int, d: int, flux: str, **kw):
    """Same term over all n^(2d) pairs (dense_hadamard_volume_ex)."""
    return _call("dense_hadamard_volume_ex", u, n, d, flux, **kw)


def volume_curvilinear(u, Ja, n: int, flux: str = "euler", *, nodes="gl", gamma=1.4, stream=None, out=None):
    """Curvilinear volume term (sf_hadamard_volume_curvilinear): u (5, E, n^3),
    Ja (3, 3, E, n^3) = [m][k][e][node] contravariant metric terms."""
    import torch
    _check_tensor(u, flux, n, 3)
    E = u.shape[1]
    if (not isinstance(Ja, torch.Tensor) or Ja.device.type != "cuda" or Ja.dtype != torch.float64
            or not Ja.is_contiguous() or tuple(Ja.shape) != (3, 3, E, n ** 3)):
        raise ValueError(f"Ja must be a contiguous float64 CUDA tensor (3, 3, {E}, {n ** 3})")
    _check_same_device(Ja, u, "Ja")
    if out is None:
        out = torch.empty_like(u)
    else:
        _check_out(out, u.shape, u)
    opts, keep = make_opts(nodes, "fp64", gamma, stream)
    check(lib().sf_hadamard_volume_curvilinear(u.data_ptr(), Ja.data_ptr(), E, n, FLUX[flux], out.data_ptr(),
                                               ctypes.byref(opts)), "sf_hadamard_volume_curvilinear")
    del keep
    _record(stream, u, Ja, out)
    return out


def _entropy_map(name, x, gamma, stream, out):
    import torch
    if not isinstance(x, torch.Tensor) or x.device.type != "cuda" or x.dtype != torch.float64 \
            or not x.is_contiguous() or x.shape[0] != 5:
        raise ValueError("expected a contiguous float64 CUDA tensor with 5 leading components")
    if out is None:
        out = torch.empty_like(x)
    else:
        _check_out(out, x.shape, x)
    check(getattr(lib(), name)(x.data_ptr(), x.numel() // 5, out.data_ptr(), float(gamma), _stream_handle(stream)),
          name)
    _record(stream, x, out)
    return out


def entropy_variables(u, *, gamma=1.4, stream=None, out=None):
    """Entropy variables of conserved states u (5, ...) (sf_entropy_variables)."""
    return _entropy_map("sf_entropy_variables", u, gamma, stream, out)


def conserved_variables(v, *, gamma=1.4, stream=None, out=None):
    """Conserved states of entropy variables v (5, ...) (sf_conserved_variables)."""
    return _entropy_map("sf_conserved_variables", v, gamma, stream, out)


def entropy_trace(u, n: int, *, nodes="gl", gamma=1.4, stream=None, out=None):
    """Entropy-projected facet states (sf_entropy_trace): u (5, E, n^3) ->
    (5, E, 6, n^2)."""
    import torch
    _check_tensor(u, "euler", n, 3)
    E = u.shape[1]
    if out is None:
        out = torch.empty((5, E, 6, n * n), dtype=u.dtype, device=u.device)
    else:
        _check_out(out, (5, E, 6, n * n), u)
    opts, keep = make_opts(nodes, "fp64", gamma, stream)
    check(lib().sf_entropy_trace(u.data_ptr(), E, n, out.data_ptr(), ctypes.byref(opts)), "sf_entropy_trace")
    del keep
    _record(stream, u, out)
    return out


def surface_operator_1d(n: int, nodes: str = "gl"):
    """(lm, lp): the Lagrange basis of the nodes at -1 and +1 (host, FP64)."""
    lm = np.zeros(n); lp = np.zeros(n)
    check(lib().sf_surface_operator_1d(n, NODES[nodes], lm.ctypes.data_as(_dp), lp.ctypes.data_as(_dp)),
          "sf_surface_operator_1d")
    return lm, lp


def surface(u, uf, n: int, d: int, flux: str, *, with_volume=False, nodes="gl", gamma=1.4, stream=None,
            y_vol=None, y_face=None, w=None):
    """(y_vol, y_face) of the surface term (sf_hadamard_surface), or of the
    volume and surface terms together (sf_hadamard_volume_surface) when
    with_volume.  u: (nvar, E, n^d); uf: (nvar, E, 2d, n^(d-1))."""
    import torch
    _check_tensor(u, flux, n, d)
    nv = NVAR[flux]
    E = u.shape[1]
    if (not isinstance(uf, torch.Tensor) or uf.device.type != "cuda" or uf.dtype != torch.float64
            or not uf.is_contiguous() or tuple(uf.shape) != (nv, E, 2 * d, n ** (d - 1))):
        raise ValueError(f"u_face must be a contiguous float64 CUDA tensor ({nv}, {E}, {2 * d}, {n ** (d - 1)})")
    _check_same_device(uf, u, "u_face")
    if y_vol is None:
        y_vol = torch.empty_like(u)
    else:
        _check_out(y_vol, u.shape, u, "y_vol")
    if y_face is None:
        y_face = torch.empty_like(uf)
    else:
        _check_out(y_face, uf.shape, u, "y_face")
    opts, keep = make_opts(nodes, "fp64", gamma, stream, None if w is None else np.zeros((n, n)), w)
    name = "sf_hadamard_volume_surface" if with_volume else "sf_hadamard_surface"
    check(getattr(lib(), name)(u.data_ptr(), uf.data_ptr(), E, n, d, FLUX[flux], y_vol.data_ptr(),
                               y_face.data_ptr(), ctypes.byref(opts)), name)
    del keep
    _record(stream, u, uf, y_vol, y_face)
    return y_vol, y_face


def basis_1d(n: int, nodes: str = "gl"):
    """(V, P) of the library's modal basis: orthonormal Legendre values
    V[q, k] on the nodes and the projection P = V^{-1} (host, FP64)."""
    V = np.zeros((n, n)); P = np.zeros((n, n))
    check(lib().sf_basis_1d(n, NODES[nodes], V.ctypes.data_as(_dp), P.ctypes.data_as(_dp)), "sf_basis_1d")
    return V, P


def basis_rect(n_modes: int, m_nodes: int, nodes: str = "gl"):
    """(V, P): n_modes orthonormal Legendre modes on m_nodes nodes (m x n) and
    the L2 projection (n x m) (host, FP64)."""
    V = np.zeros((m_nodes, n_modes)); P = np.zeros((n_modes, m_nodes))
    check(lib().sf_basis_rect(n_modes, m_nodes, NODES[nodes], V.ctypes.data_as(_dp), P.ctypes.data_as(_dp)),
          "sf_basis_rect")
    return V, P


def tensor_apply(u, n: int, d: int, M, *, out=None, stream=None):
    """out[v, e] = (M kron ... kron M) u[v, e] (sf_tensor_apply_rect); u is a
    contiguous float64 CUDA tensor (nvar, E, n^d), M is (n_out, n); out is
    (nvar, E, n_out^d) and may be u itself when n_out == n."""
    import torch
    if not isinstance(u, torch.Tensor) or u.device.type != "cuda" or u.dtype != torch.float64:
        raise TypeError("u must be a float64 CUDA tensor")
    if not u.is_contiguous() or u.dim() != 3 or u.shape[2] != n ** d:
        raise ValueError(f"u must be a contiguous (nvar, E, {n ** d}) tensor, got {tuple(u.shape)}")
    Mh = np.ascontiguousarray(M, dtype=np.float64)
    if Mh.ndim != 2 or Mh.shape[1] != n:
        raise ValueError(f"M must be (n_out, {n})")
    n_out = Mh.shape[0]
    shape = (u.shape[0], u.shape[1], n_out ** d)
    if out is None:
        out = torch.empty(shape, dtype=u.dtype, device=u.device)
    elif tuple(out.shape) != shape or out.dtype != u.dtype or not out.is_contiguous() or out.device != u.device:
        raise ValueError(f"out must be a contiguous float64 tensor {shape} on u's device")
    check(lib().sf_tensor_apply_rect(u.data_ptr(), u.shape[1], n, n_out, d, u.shape[0], Mh.ctypes.data_as(_dp),
                                     out.data_ptr(), _stream_handle(stream)), "sf_tensor_apply_rect")
    _record(stream, u, out)
    return out


POST_MAP = {"entropy": 1, "conserved": 2}


def tensor_apply_map(u, n: int, M, post_map: str, *, gamma=1.4, out=None, stream=None):
    """out = map((M kron M kron M) u) in one pass (sf_tensor_apply_rect_map):
    u a contiguous float64 CUDA tensor (5, E, n^3) of 3D Euler states, M
    (n + 2, n), post_map "entropy" (conserved -> entropy variables) or
    "conserved" (the map back); out (5, E, (n + 2)^3), not overlapping u."""
    import torch
    if post_map not in POST_MAP:
        raise ValueError(f"post_map must be one of {sorted(POST_MAP)}")
    if not isinstance(u, torch.Tensor) or u.device.type != "cuda" or u.dtype != torch.float64:
        raise TypeError("u must be a float64 CUDA tensor")
    if not u.is_contiguous() or u.dim() != 3 or u.shape[0] != 5 or u.shape[2] != n ** 3:
        raise ValueError(f"u must be a contiguous (5, E, {n ** 3}) tensor, got {tuple(u.shape)}")
    Mh = np.ascontiguousarray(M, dtype=np.float64)
    if Mh.ndim != 2 or Mh.shape[1] != n:
        raise ValueError(f"M must be (n_out, {n})")
    n_out = Mh.shape[0]
    shape = (5, u.shape[1], n_out ** 3)
    if out is None:
        out = torch.empty(shape, dtype=u.dtype, device=u.device)
    elif tuple(out.shape) != shape or out.dtype != u.dtype or not out.is_contiguous() or out.device != u.device:
        raise ValueError(f"out must be a contiguous float64 tensor {shape} on u's device")
    check(lib().sf_tensor_apply_rect_map(u.data_ptr(), u.shape[1], n, n_out, POST_MAP[post_map], float(gamma),
                                         Mh.ctypes.data_as(_dp), out.data_ptr(), _stream_handle(stream)),
          "sf_tensor_apply_rect_map")
    _record(stream, u, out)
    return out


def _diag(name, x, stream):
    import torch
    if not isinstance(x, torch.Tensor) or x.device.type != "cuda" or x.dtype != torch.float64:
        raise TypeError("x must be a float64 CUDA tensor")
    x = x.contiguous()
    y = torch.empty_like(x)
    check(getattr(lib(), name)(x.data_ptr(), x.numel(), y.data_ptr(), _stream_handle(stream)), name)
    _record(stream, x, y)
    return y


def diag_log1p(x, stream=None):
    """ln(1 + x) by the kernels' staging routine (float64 CUDA tensor in and out)."""
    return _diag("sf_diag_log1p", x, stream)


def diag_log(x, stream=None):
    """ln x by the entropy-variable maps' routine (float64 CUDA tensor in and out)."""
    return _diag("sf_diag_log", x, stream)


def diag_exp(x, stream=None):
    """e^x by the entropy-variable maps' routine (float64 CUDA tensor in and out)."""
    return _diag("sf_diag_exp", x, stream)


def volume_raw(u_ptr: int, E: int, n: int, d: int, flux: int, out_ptr: int) -> int:
    """The short C entry point with raw device pointers (returns the status)."""
    return lib().sf_hadamard_volume(u_ptr, E, n, d, flux, out_ptr)


def dense_volume_raw(u_ptr: int, E: int, n: int, d: int, flux: int, out_ptr: int) -> int:
    return lib().dense_hadamard_volume(u_ptr, E, n, d, flux, out_ptr)
