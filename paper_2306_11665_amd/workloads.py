"""Seeded synthetic workloads for the volume term (inputs only).

This module draws states; it holds none of the volume term's arithmetic.  The
only formula here is the ideal-gas equation of state used to turn drawn
primitive variables into the conserved variables that both the library and
the CPU oracle read:  E = p/(gamma-1) + rho |v|^2 / 2.

Workload recipe (all FP64, layout u[v, e, node], node = ix + n*iy + n*n*iz):

* burgers2d_n4_gll_e64: 2D Burgers, n = 4 Gauss-Lobatto nodes, 64 elements,
  u ~ U[-1, 1], seed 1.
* euler3d_n4_gl_e4096: 3D Euler, n = 4 Gauss-Legendre nodes, 4096 elements,
  rho ~ U[0.5, 1.5], each velocity component ~ U[-0.5, 0.5],
  p ~ U[0.5, 1.5] per node, seed 2.
* euler3d_n8_gl_e32768: as above with n = 8, 32768 elements, seed 3; a
  seeded permutation picks round(0.1 E) elements that are set to one
  constant (free-stream) state drawn from the same distributions, so every
  pair inside them is exactly equal.
* serving mix: meshes with p ~ U{2..7} (n = p + 1), E log-uniform in
  [512, 32768], states as the n = 4 workload, seed 5000 + k for mesh k;
  Poisson arrivals from seed 5.

The random numbers come from numpy's PCG64 (default_rng).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GAMMA = 1.4


@dataclass(frozen=True)
class Workload:
    name: str
    flux: str          # "burgers" | "euler" | "product"
    d: int
    n: int
    nodes: str         # "gl" | "gll"
    E: int
    seed: int
    freestream_frac: float = 0.0
    precision: str = "fp64"

    @property
    def nvar(self) -> int:
        return 5 if self.flux == "euler" else 1

    @property
    def nodes_per_elem(self) -> int:
        return self.n ** self.d

    @property
    def dof(self) -> int:
        return self.E * self.nodes_per_elem * self.nvar

    def state(self) -> np.ndarray:
        return make_state(self)


WORKLOADS = {
    "burgers2d_n4_gll_e64": Workload("burgers2d_n4_gll_e64", "burgers", 2, 4, "gll", 64, 1),
    "euler3d_n4_gl_e4096": Workload("euler3d_n4_gl_e4096", "euler", 3, 4, "gl", 4096, 2),
    "euler3d_n8_gl_e32768": Workload("euler3d_n8_gl_e32768", "euler", 3, 8, "gl", 32768, 3, 0.1),
    "euler3d_n8_gl_e32768_fp32split": Workload("euler3d_n8_gl_e32768_fp32split", "euler", 3, 8, "gl",
                                               32768, 3, 0.1, "fp32_split"),
}


def primitives_to_conserved(rho, vel, p, gamma=GAMMA):
    """(rho, v[3], p) -> (rho, rho v[3], E) with E = p/(gamma-1) + rho |v|^2 / 2."""
    q = vel[0] * vel[0] + vel[1] * vel[1] + vel[2] * vel[2]
    return np.stack([rho, rho * vel[0], rho * vel[1], rho * vel[2], p / (gamma - 1.0) + 0.5 * rho * q])


def euler_state(E: int, n: int, seed: int, freestream_frac: float = 0.0, gamma: float = GAMMA,
                d: int = 3) -> np.ndarray:
    """Conserved Euler states (5, E, n^d) drawn per node; optional free-stream elements."""
    N = n ** d
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.5, 1.5, size=(E, N))
    vel = rng.uniform(-0.5, 0.5, size=(3, E, N))
    p = rng.uniform(0.5, 1.5, size=(E, N))
    if freestream_frac > 0.0 and E > 0:
        k = int(round(freestream_frac * E))
        idx = np.sort(rng.permutation(E)[:k])
        rho_c = rng.uniform(0.5, 1.5, size=k)
        vel_c = rng.uniform(-0.5, 0.5, size=(3, k))
        p_c = rng.uniform(0.5, 1.5, size=k)
        rho[idx, :] = rho_c[:, None]
        vel[:, idx, :] = vel_c[:, :, None]
        p[idx, :] = p_c[:, None]
    return np.ascontiguousarray(primitives_to_conserved(rho, vel, p, gamma))


def wide_ratio_euler_state(E: int, n: int, ratio: float, seed: int, rho_scale: float = 1.0,
                           p_scale: float = 1.0, switch_tau: float = 0.0, vel_scale: float = 1.0,
                           gamma: float = GAMMA) -> np.ndarray:
    """Conserved Euler states (5, E, n^3) whose density and pressure vary
    within each element by factors up to `ratio`: ln(rho / rho_scale) and
    ln(p / p_scale) ~ U[-ln(ratio)/2, ln(ratio)/2] per node, velocity
    components ~ vel_scale U[-0.5, 0.5] (a vel_scale of about
    sqrt(p_scale / rho_scale) keeps the kinetic and internal energies of one
    size, so that the pressure survives the conserved-variable round trip).  With switch_tau > 0, on every x-line the
    second node is moved next to the first so that both |ln rho_1 - ln rho_0|
    and |ln beta_1 - ln beta_0| (beta = rho / (2p)) equal switch_tau (1 + s)
    with s drawn from {-1e-2, -1e-3, 1e-3, 1e-2} (signs random): node pairs
    just either side of a log-difference threshold switch_tau."""
    N = n ** 3
    rng = np.random.default_rng(seed)
    h = 0.5 * math.log(ratio)
    lr = math.log(rho_scale) + rng.uniform(-h, h, size=(E, N))
    lp = math.log(p_scale) + rng.uniform(-h, h, size=(E, N))
    vel = vel_scale * rng.uniform(-0.5, 0.5, size=(3, E, N))
    if switch_tau > 0.0:
        first = np.arange(0, N, n)                     # node 0 of every x-line
        k = first.size
        s = np.array([-1e-2, -1e-3, 1e-3, 1e-2])
        dr = switch_tau * (1 + rng.choice(s, size=(E, k))) * rng.choice([-1.0, 1.0], size=(E, k))
        db = switch_tau * (1 + rng.choice(s, size=(E, k))) * rng.choice([-1.0, 1.0], size=(E, k))
        lr[:, first + 1] = lr[:, first] + dr
        # ln beta = ln rho - ln p - ln 2, so ln p moves by d(ln rho) - d(ln beta)
        lp[:, first + 1] = lp[:, first] + dr - db
    rho, p = np.exp(lr), np.exp(lp)
    return np.ascontiguousarray(primitives_to_conserved(rho, vel, p, gamma))


def _freestream_idx(E: int, n: int, seed: int, freestream_frac: float, d: int = 3) -> np.ndarray:
    N = n ** d
    rng = np.random.default_rng(seed)
    rng.uniform(0.5, 1.5, size=(E, N))
    rng.uniform(-0.5, 0.5, size=(3, E, N))
    rng.uniform(0.5, 1.5, size=(E, N))
    k = int(round(freestream_frac * E))
    return np.sort(rng.permutation(E)[:k])


def freestream_index(w: Workload) -> np.ndarray:
    if w.freestream_frac <= 0.0:
        return np.zeros(0, dtype=np.int64)
    return _freestream_idx(w.E, w.n, w.seed, w.freestream_frac, w.d)


def scalar_state(E: int, n: int, d: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """Scalar nodal states (1, E, n^d) ~ U[lo, hi]."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(1, E, n ** d))


def make_state(w: Workload) -> np.ndarray:
    if w.flux == "euler":
        return euler_state(w.E, w.n, w.seed, w.freestream_frac, d=w.d)
    if w.flux == "product":
        return scalar_state(w.E, w.n, w.d, w.seed, 1e-8, 30.0)
    return scalar_state(w.E, w.n, w.d, w.seed)


def sample_elements(E: int, k: int, seed: int, must_include=()) -> np.ndarray:
    """A seeded sorted sample of k element indices (plus any must_include)."""
    rng = np.random.default_rng(seed)
    k = min(k, E)
    pick = set(rng.choice(E, size=k, replace=False).tolist())
    pick.update(int(i) for i in must_include)
    return np.array(sorted(pick), dtype=np.int64)


@dataclass
class MeshSpec:
    mesh_id: int
    n: int
    E: int
    seed: int


def reference_nodes(n: int, nodes: str = "gl") -> np.ndarray:
    """The n nodes on [-1, 1] from numpy's Legendre routines (input
    generation only: Gauss-Legendre roots, or +-1 and the roots of P'_{n-1})."""
    if nodes == "gl":
        return np.polynomial.legendre.leggauss(n)[0]
    interior = np.polynomial.legendre.Legendre.basis(n - 1).deriv().roots()
    return np.concatenate([[-1.0], np.sort(interior.real), [1.0]])


def smooth_euler_state(E: int, n: int, seed: int, nodes: str = "gl", slope: float = 0.15) -> np.ndarray:
    """Conserved state (5, E, n^3) of primitive fields that are linear in each
    element (rho, p = 1 + g . x, |g_k| <= slope; vel_k = c_k + g . x), so the
    polynomial interpolant of the state stays physical on any node set of the
    element (inputs of the over-integrated and entropy-projected paths)."""
    x = reference_nodes(n, nodes)
    node = np.arange(n ** 3)
    X = np.stack([x[node % n], x[(node // n) % n], x[node // (n * n)]])   # (3, n^3)
    rng = np.random.default_rng(seed)
    g = rng.uniform(-slope, slope, (5, E, 3))
    c = rng.uniform(-0.3, 0.3, (3, E))
    rho = 1.0 + g[0] @ X
    p = 1.0 + g[1] @ X
    vel = np.stack([c[k][:, None] + g[2 + k] @ X for k in range(3)])
    return np.ascontiguousarray(primitives_to_conserved(rho, vel, p))


def warped_mesh_metrics(E: int, n: int, nodes: str = "gl", amp: float = 0.02, length: float = 2 * math.pi):
    """Contravariant metric terms Ja^m_k = J d xi^m / d x_k, shape (3, 3, E, n^3)
    ([m][k][e][node], node = ix + n iy + n^2 iz), of a non-symmetrically
    warped curvilinear mesh: the first E elements (x fastest) of a K^3 mesh of
    the box [0, length]^3, K = ceil(E^(1/3)), mapped by
        x = X + a sin(2 pi Y/L) sin(4 pi Z/L),  y = Y + a sin(4 pi X/L) sin(2 pi Z/L),
        z = Z + a sin(2 pi X/L) sin(6 pi Y/L),  a = amp * L,
    evaluated exactly (analytic Jacobian, cross-product form
    Ja^1 = x_xi2 x x_xi3, Ja^2 = x_xi3 x x_xi1, Ja^3 = x_xi1 x x_xi2)."""
    K = int(round(E ** (1.0 / 3.0)))
    while K ** 3 < E:
        K += 1
    L = length
    h = L / K
    a = amp * L
    xi = reference_nodes(n, nodes)
    e = np.arange(E)
    ex, ey, ez = e % K, (e // K) % K, e // (K * K)
    node = np.arange(n ** 3)
    ix, iy, iz = node % n, (node // n) % n, node // (n * n)
    X = (ex[:, None] + (xi[ix][None, :] + 1) / 2) * h
    Y = (ey[:, None] + (xi[iy][None, :] + 1) / 2) * h
    Z = (ez[:, None] + (xi[iz][None, :] + 1) / 2) * h
    w1, w2, w3 = 2 * math.pi / L, 4 * math.pi / L, 6 * math.pi / L
    one = np.ones_like(X)
    # M[i][j] = d x_i / d X_j
    M = np.empty((3, 3) + X.shape)
    M[0, 0] = one
    M[0, 1] = a * w1 * np.cos(w1 * Y) * np.sin(w2 * Z)
    M[0, 2] = a * w2 * np.sin(w1 * Y) * np.cos(w2 * Z)
    M[1, 0] = a * w2 * np.cos(w2 * X) * np.sin(w1 * Z)
    M[1, 1] = one
    M[1, 2] = a * w1 * np.sin(w2 * X) * np.cos(w1 * Z)
    M[2, 0] = a * w1 * np.cos(w1 * X) * np.sin(w3 * Y)
    M[2, 1] = a * w3 * np.sin(w1 * X) * np.cos(w3 * Y)
    M[2, 2] = one
    cols = [M[:, j] * (h / 2) for j in range(3)]       # d x / d xi_j
    Ja = np.empty((3, 3) + X.shape)
    Ja[0] = np.cross(cols[1], cols[2], axis=0)
    Ja[1] = np.cross(cols[2], cols[0], axis=0)
    Ja[2] = np.cross(cols[0], cols[1], axis=0)
    return np.ascontiguousarray(Ja)


def serving_meshes(count: int = 64, base_seed: int = 5000, e_lo: int = 512, e_hi: int = 32768,
                   p_lo: int = 2, p_hi: int = 7) -> list:
    """Mesh k: p ~ U{p_lo..p_hi}, n = p + 1, E = round(exp(U[ln e_lo, ln e_hi])), seed base+k."""
    out = []
    for k in range(count):
        rng = np.random.default_rng(base_seed + k)
        p = int(rng.integers(p_lo, p_hi + 1))
        E = int(round(math.exp(rng.uniform(math.log(e_lo), math.log(e_hi)))))
        out.append(MeshSpec(k, p + 1, E, base_seed + k))
    return out


def serving_mesh_state(spec: MeshSpec) -> np.ndarray:
    return euler_state(spec.E, spec.n, spec.seed)


def poisson_arrivals(rate_hz: float, count: int, n_meshes: int, seed: int = 5):
    """(arrival times in s, mesh index per request) for a Poisson stream."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, size=count)
    mesh = rng.integers(0, n_meshes, size=count)
    return np.cumsum(gaps), mesh
