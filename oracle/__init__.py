"""CPU oracle for the flux-differencing volume term -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the package's ``smoke()`` check and the benchmark's
``cpu_baseline`` leg may import this package.  The product library never does,
and this package never imports the product package: the two share no code.

Python side of ``oracle.c`` (plain FP64 C, see its header for the paper
passages it follows).  Functions take and return numpy arrays in the layout
``u[v, e, node]`` with ``node = ix + n*iy + n*n*iz``.

Parity unpinned by the paper: the Euler flux's logarithmic-mean mass flux and
pressure average (the paper names the flux without printing it); everything
that follows from them is pinned by the tests (see ``oracle.c``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

FLUX = {"burgers": 0, "euler": 1, "product": 2, "euler_pfix": 3}
NODES = {"gl": 0, "gll": 1}
NVAR = {"burgers": 1, "euler": 5, "product": 1, "euler_pfix": 5}

_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.oracle_nodes.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp]
        L.oracle_operator.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, dp]
        L.oracle_diff_matrix.argtypes = [ctypes.c_int, dp, dp]
        L.oracle_diff_matrix.restype = None
        L.oracle_logmean.argtypes = [ctypes.c_double, ctypes.c_double]
        L.oracle_logmean.restype = ctypes.c_double
        L.oracle_flux.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int, ctypes.c_double, dp]
        L.oracle_flux.restype = None
        L.oracle_physical_flux_euler.argtypes = [dp, ctypes.c_int, ctypes.c_double, dp]
        L.oracle_physical_flux_euler.restype = None
        L.oracle_build_A.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp, dp]
        L.oracle_build_A.restype = None
        for f in (L.oracle_dense_volume, L.oracle_sf_volume):
            f.argtypes = [dp, ctypes.c_long, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                          dp, dp, ctypes.c_double, dp]
        L.oracle_sparsity_pattern.argtypes = [ctypes.c_int, ctypes.c_int, ip, ip]
        L.oracle_basis_sparse.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, ip, ip, dp]
        L.oracle_basis_1d.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp]
        L.oracle_tensor_apply.argtypes = [dp, ctypes.c_long, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp]
        L.oracle_tensor_apply_rect.argtypes = [dp, ctypes.c_long, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                               ctypes.c_int, dp, dp]
        L.oracle_basis_rect.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp]
        L.oracle_entropy_vars.argtypes = [dp, ctypes.c_double, dp]
        L.oracle_entropy_vars.restype = None
        L.oracle_conserved_from_entropy.argtypes = [dp, ctypes.c_double, dp]
        L.oracle_conserved_from_entropy.restype = None
        L.oracle_entropy_trace.argtypes = [dp, ctypes.c_long, ctypes.c_int, dp, dp, ctypes.c_double, dp]
        L.oracle_curv_volume.argtypes = [dp, dp, ctypes.c_long, ctypes.c_int, ctypes.c_int, dp, dp,
                                         ctypes.c_double, dp]
        L.oracle_lagrange_endpoints.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp]
        L.oracle_surface.argtypes = [dp, dp, ctypes.c_long, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     dp, dp, dp, ctypes.c_double, dp, dp]
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_set_num_threads.argtypes = [ctypes.c_int]
        L.oracle_set_num_threads.restype = None
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def nodes(n: int, kind: str = "gl"):
    x = np.zeros(n); w = np.zeros(n)
    if lib().oracle_nodes(n, NODES[kind], _dp(x), _dp(w)) != 0:
        raise ValueError(f"bad node request n={n} kind={kind}")
    return x, w


def operator_1d(n: int, kind: str = "gl"):
    """(x, w, D, Q) with Q = diag(w) D, the 1D factor of Eq. (5)."""
    x = np.zeros(n); w = np.zeros(n); D = np.zeros((n, n)); Q = np.zeros((n, n))
    if lib().oracle_operator(n, NODES[kind], _dp(x), _dp(w), _dp(D), _dp(Q)) != 0:
        raise ValueError(f"bad operator request n={n} kind={kind}")
    return x, w, D, Q


def diff_matrix(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    D = np.zeros((len(x), len(x)))
    lib().oracle_diff_matrix(len(x), _dp(x), _dp(D))
    return D


def logmean(a: float, b: float) -> float:
    return lib().oracle_logmean(float(a), float(b))


def flux(kind: str, uL, uR, m: int, gamma: float = 1.4) -> np.ndarray:
    nv = NVAR[kind]
    uL = np.ascontiguousarray(uL, dtype=np.float64).reshape(nv)
    uR = np.ascontiguousarray(uR, dtype=np.float64).reshape(nv)
    F = np.zeros(nv)
    lib().oracle_flux(FLUX[kind], _dp(uL), _dp(uR), m, gamma, _dp(F))
    return F


def physical_flux_euler(u, m: int, gamma: float = 1.4) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(5)
    F = np.zeros(5)
    lib().oracle_physical_flux_euler(_dp(u), m, gamma, _dp(F))
    return F


def build_A(n: int, d: int, m: int, Q: np.ndarray, w: np.ndarray) -> np.ndarray:
    N = n ** d
    Q = np.ascontiguousarray(Q, dtype=np.float64); w = np.ascontiguousarray(w, dtype=np.float64)
    A = np.zeros((N, N))
    lib().oracle_build_A(n, d, m, _dp(Q), _dp(w), _dp(A))
    return A


def _volume(fn, u, n, d, flux_kind, Q, w, gamma):
    u = np.ascontiguousarray(u, dtype=np.float64)
    nv = NVAR[flux_kind]
    N = n ** d
    if u.ndim != 3 or u.shape[0] != nv or u.shape[2] != N:
        raise ValueError(f"u must be ({nv}, E, {N}), got {u.shape}")
    E = u.shape[1]
    Q = np.ascontiguousarray(Q, dtype=np.float64); w = np.ascontiguousarray(w, dtype=np.float64)
    out = np.zeros_like(u)
    rc = fn(_dp(u), E, n, d, FLUX[flux_kind], _dp(Q), _dp(w), gamma, _dp(out))
    if rc != 0:
        raise ValueError("oracle rejected arguments")
    return out


def dense_volume(u, n, d, flux_kind, Q=None, w=None, nodes_kind="gl", gamma=1.4):
    """The definition y = sum_m (A_m o F_m) 1 over all n^(2d) pairs."""
    if Q is None or w is None:
        _, w0, _, Q0 = operator_1d(n, nodes_kind)
        Q = Q0 if Q is None else Q
        w = w0 if w is None else w
    return _volume(lib().oracle_dense_volume, u, n, d, flux_kind, Q, w, gamma)


def sf_volume(u, n, d, flux_kind, Q=None, w=None, nodes_kind="gl", gamma=1.4):
    """The paper's CPU method (Algorithms 1-2, then the Hadamard product)."""
    if Q is None or w is None:
        _, w0, _, Q0 = operator_1d(n, nodes_kind)
        Q = Q0 if Q is None else Q
        w = w0 if w is None else w
    return _volume(lib().oracle_sf_volume, u, n, d, flux_kind, Q, w, gamma)


def sparsity_pattern(n: int, d: int):
    rows = np.zeros((n ** (d + 1), d), dtype=np.int32)
    cols = np.zeros((n ** (d + 1), d), dtype=np.int32)
    if lib().oracle_sparsity_pattern(n, d, _ip(rows), _ip(cols)) != 0:
        raise ValueError("d must be 2 or 3")
    return rows, cols


def basis_sparse(n: int, d: int, Q: np.ndarray, w: np.ndarray):
    rows, cols = sparsity_pattern(n, d)
    Q = np.ascontiguousarray(Q, dtype=np.float64); w = np.ascontiguousarray(w, dtype=np.float64)
    bs = np.zeros((d, n ** d, n))
    lib().oracle_basis_sparse(n, d, _dp(Q), _dp(w), _ip(rows), _ip(cols), _dp(bs))
    return bs


def basis_1d(n: int, kind: str = "gl"):
    """(V, P): orthonormal Legendre values V[q, k] = L_k(x_q) on the nodes,
    and the projection P = V^{-1} (P V = I)."""
    V = np.zeros((n, n)); P = np.zeros((n, n))
    if lib().oracle_basis_1d(n, NODES[kind], _dp(V), _dp(P)) != 0:
        raise ValueError("bad arguments or singular basis")
    return V, P


def tensor_apply(u, n: int, d: int, M) -> np.ndarray:
    """out[v, e] = (M kron ... kron M) u[v, e] (d factors), u of shape
    (nvar, E, n^d); M is (n_out, n) (square or rectangular), out (nvar, E, n_out^d)."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    M = np.ascontiguousarray(M, dtype=np.float64)
    if u.ndim != 3 or u.shape[2] != n ** d or M.ndim != 2 or M.shape[1] != n:
        raise ValueError("shape mismatch")
    n_out = M.shape[0]
    out = np.zeros((u.shape[0], u.shape[1], n_out ** d))
    if lib().oracle_tensor_apply_rect(_dp(u), u.shape[1], n, n_out, d, u.shape[0], _dp(M), _dp(out)) != 0:
        raise ValueError("oracle rejected arguments")
    return out


def basis_rect(n: int, m: int, kind: str = "gl"):
    """(V, P): n orthonormal Legendre modes on m nodes (m x n) and the L2
    projection P = (V^T W V)^{-1} V^T W (n x m)."""
    V = np.zeros((m, n)); P = np.zeros((n, m))
    if lib().oracle_basis_rect(n, m, NODES[kind], _dp(V), _dp(P)) != 0:
        raise ValueError("bad arguments")
    return V, P


def entropy_vars(u, gamma: float = 1.4) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.float64); v = np.zeros(5)
    lib().oracle_entropy_vars(_dp(u), gamma, _dp(v))
    return v


def conserved_from_entropy(v, gamma: float = 1.4) -> np.ndarray:
    v = np.ascontiguousarray(v, dtype=np.float64); u = np.zeros(5)
    lib().oracle_conserved_from_entropy(_dp(v), gamma, _dp(u))
    return u


def entropy_trace(u, n: int, nodes_kind: str = "gl", gamma: float = 1.4, lm=None, lp=None) -> np.ndarray:
    """Entropy-projected facet states u(E_f v(u)), shape (5, E, 6, n^2)."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    E = u.shape[1]
    if u.shape != (5, E, n ** 3):
        raise ValueError("shape mismatch")
    if lm is None or lp is None:
        lm, lp = lagrange_endpoints(n, nodes_kind)
    lm = np.ascontiguousarray(lm, dtype=np.float64); lp = np.ascontiguousarray(lp, dtype=np.float64)
    uf = np.zeros((5, E, 6, n * n))
    if lib().oracle_entropy_trace(_dp(u), E, n, _dp(lm), _dp(lp), gamma, _dp(uf)) != 0:
        raise ValueError("oracle rejected arguments")
    return uf


def curv_volume(u, Ja, n: int, flux_kind: str = "euler", Q=None, w=None, nodes_kind="gl", gamma=1.4):
    """Curvilinear volume term (3D) with the metric-averaged flux; Ja of shape
    (3, 3, E, n^3) = [m][k][e][node], Ja^m_k = J d xi^m / d x_k."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    Ja = np.ascontiguousarray(Ja, dtype=np.float64)
    nv = NVAR[flux_kind]
    E = u.shape[1]
    if u.shape != (nv, E, n ** 3) or Ja.shape != (3, 3, E, n ** 3):
        raise ValueError("shape mismatch")
    if Q is None or w is None:
        _, w0, _, Q0 = operator_1d(n, nodes_kind)
        Q = Q0 if Q is None else Q
        w = w0 if w is None else w
    Q = np.ascontiguousarray(Q, dtype=np.float64); w = np.ascontiguousarray(w, dtype=np.float64)
    out = np.zeros_like(u)
    if lib().oracle_curv_volume(_dp(u), _dp(Ja), E, n, FLUX[flux_kind], _dp(Q), _dp(w), gamma, _dp(out)) != 0:
        raise ValueError("oracle rejected arguments")
    return out


def lagrange_endpoints(n: int, kind: str = "gl"):
    """(lm, lp): the Lagrange basis of the nodes at -1 and +1."""
    lm = np.zeros(n); lp = np.zeros(n)
    if lib().oracle_lagrange_endpoints(n, NODES[kind], _dp(lm), _dp(lp)) != 0:
        raise ValueError("bad arguments")
    return lm, lp


def surface(u, uf, n: int, d: int, flux_kind: str, w=None, lm=None, lp=None, nodes_kind="gl", gamma=1.4):
    """The surface term by its definition: (y_vol, y_face) for volume states
    u (nvar, E, n^d) and facet states uf (nvar, E, 2d, n^(d-1))."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    uf = np.ascontiguousarray(uf, dtype=np.float64)
    nv = NVAR[flux_kind]
    E = u.shape[1]
    if u.shape != (nv, E, n ** d) or uf.shape != (nv, E, 2 * d, n ** (d - 1)):
        raise ValueError("shape mismatch")
    if w is None:
        _, w = nodes(n, nodes_kind)
    if lm is None or lp is None:
        lm0, lp0 = lagrange_endpoints(n, nodes_kind)
        lm = lm0 if lm is None else lm
        lp = lp0 if lp is None else lp
    w = np.ascontiguousarray(w, dtype=np.float64)
    lm = np.ascontiguousarray(lm, dtype=np.float64); lp = np.ascontiguousarray(lp, dtype=np.float64)
    yv = np.zeros_like(u); yf = np.zeros_like(uf)
    if lib().oracle_surface(_dp(u), _dp(uf), E, n, d, FLUX[flux_kind], _dp(w), _dp(lm), _dp(lp), gamma,
                            _dp(yv), _dp(yf)) != 0:
        raise ValueError("oracle rejected arguments")
    return yv, yf


def num_threads() -> int:
    return lib().oracle_num_threads()


def set_num_threads(t: int) -> None:
    lib().oracle_set_num_threads(int(t))
