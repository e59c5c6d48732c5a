"""Pins of the oracle's volume term y = sum_m (A_m o F_m) 1.

Every check here fixes the oracle against something other than itself:
hand-worked entries of Algorithms 1-2, the structure of Eq. (3) (each stored
pair shares a grid line), closed forms (the rank-one workload of the Results
section, Burgers with linear data), free-stream preservation, the
summation-by-parts line identity, an mpmath brute force at tiny n that builds
A_m entry by entry (no Kronecker routine), and the O(n^(2d)) vs O(n^(d+1))
cost slopes of Figure 1.
"""
import json
import os
import time

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _digits(node, n, d):
    return [(node // n ** k) % n for k in range(d)]


# ---------------------------------------------------------------- Alg. 1 / 2
def test_alg1_alg2_hand_worked_entries(orc):
    n = 3
    rows, cols = orc.sparsity_pattern(n, 3)
    rng = np.random.default_rng(0)
    Q = rng.standard_normal((n, n))
    w = rng.uniform(0.5, 1.5, n)
    bs = orc.basis_sparse(n, 3, Q, w)
    seen = 0
    with open(os.path.join(GOLDEN, "alg1_alg2_entries_n3.txt")) as f:
        for line in f:
            t = line.split()
            if not t or t[0].startswith("#"):
                continue
            if t[0] == "ALG1":
                i, j, k, l, idx, row, cx, cy, cz = map(int, t[1:])
                assert idx == ((i * n + j) * n + k) * n + l
                assert list(rows[idx]) == [row, row, row]
                assert list(cols[idx]) == [cx, cy, cz]
            elif t[0] == "ALG2":
                m, row, l, a, b, p, q = map(int, t[1:])
                assert bs[m, row, l] == pytest.approx(Q[a, b] * w[p] * w[q], rel=1e-15)
            seen += 1
    assert seen == 11


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("n", [2, 3, 5])
def test_sparsity_pairs_share_a_line(orc, n, d):
    """Eq. (3): the n^(d+1) stored pairs of direction m are exactly the pairs
    whose node digits agree in every direction except m."""
    rows, cols = orc.sparsity_pattern(n, d)
    N = n ** d
    for m in range(d):
        got = set()
        for idx in range(N * n):
            r, c = int(rows[idx, m]), int(cols[idx, m])
            dr, dc = _digits(r, n, d), _digits(c, n, d)
            assert all(dr[k] == dc[k] for k in range(d) if k != m)
            assert dc[m] == idx % n       # the column digit along m is the counter
            got.add((r, c))
        want = {(r, c) for r in range(N) for c in range(N)
                if all(_digits(r, n, d)[k] == _digits(c, n, d)[k] for k in range(d) if k != m)}
        assert got == want


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("n,kind", [(3, "gll"), (4, "gl"), (5, "gl")])
def test_basis_sparse_equals_kronecker_nonzeros(orc, n, d, kind):
    """Algorithm 2's stored values are the nonzeros of the explicit Kronecker
    matrix A_m (W in every direction but m, Q = W D in direction m)."""
    x, w, D, Q = orc.operator_1d(n, kind)
    rows, cols = orc.sparsity_pattern(n, d)
    bs = orc.basis_sparse(n, d, Q, w)
    for m in range(d):
        A = orc.build_A(n, d, m, Q, w)
        mask = np.zeros_like(A, dtype=bool)
        for idx in range(n ** (d + 1)):
            r, c = rows[idx, m], cols[idx, m]
            assert bs[m, r, idx % n] == pytest.approx(A[r, c], rel=1e-15, abs=1e-300)
            mask[r, c] = True
        assert np.all(A[~mask] == 0.0)


def test_build_A_entrywise(orc):
    """A_m against a digit-by-digit product (no Kronecker routine)."""
    n, d = 3, 3
    rng = np.random.default_rng(1)
    Q = rng.standard_normal((n, n)); w = rng.uniform(0.5, 2.0, n)
    for m in range(d):
        A = orc.build_A(n, d, m, Q, w)
        for i in range(n ** d):
            for j in range(n ** d):
                di, dj = _digits(i, n, d), _digits(j, n, d)
                v = Q[di[m], dj[m]]
                for k in range(d):
                    if k != m:
                        v *= w[di[k]] if di[k] == dj[k] else 0.0
                assert A[i, j] == pytest.approx(v, rel=1e-15, abs=0)


# ------------------------------------------------------------ closed forms
def _sumfact_apply(Q, w, c, n, d):
    """sum_m A_m c by sum-factorization (einsum along each axis)."""
    cs = c.reshape((n,) * d)            # axes (z, y, x) for d=3, (y, x) for d=2
    tot = np.zeros_like(cs)
    for m in range(d):
        ax = d - 1 - m                   # direction m lives on this numpy axis
        t = np.moveaxis(np.tensordot(Q, cs, axes=([1], [ax])), 0, ax)
        for k in range(d):
            if k != m:
                shape = [1] * d; shape[d - 1 - k] = n
                t = t * w.reshape(shape)
        tot += t
    return tot.reshape(-1)


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("n,kind", [(4, "gl"), (5, "gll"), (7, "gl")])
@pytest.mark.parametrize("unweighted", [False, True])
def test_product_flux_closed_form(orc, n, d, kind, unweighted):
    """Results section workload C_ij = c_i c_j: (A o c c^T) 1 = c o (A c)."""
    x, w, D, Q = orc.operator_1d(n, kind)
    if unweighted:                       # the paper's sum_j dl/dxi_j o C
        Q, w = D, np.ones(n)
    rng = np.random.default_rng(7)
    E = 3
    c = rng.uniform(1e-8, 30.0, size=(1, E, n ** d))
    y = orc.dense_volume(c, n, d, "product", Q=Q, w=w)
    for e in range(E):
        ref = c[0, e] * _sumfact_apply(Q, w, c[0, e], n, d)
        err = np.abs(y[0, e] - ref).max() / np.abs(ref).max()
        assert err < 1e-14, err


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("n,kind", [(3, "gll"), (4, "gl"), (6, "gll"), (8, "gl")])
def test_burgers_linear_closed_form(orc, n, d, kind):
    """u linear: each line gives sum_c Q_ac (u_a^2+u_a u_c+u_c^2)/6 = w_a u_a u'/2,
    so y_i = (prod_k w_ik) u_i (sum of slopes) / 2  (needs n >= 3)."""
    x, w, D, Q = orc.operator_1d(n, kind)
    slopes = np.array([0.7, -1.3, 0.4])[:d]
    grid = np.meshgrid(*([x] * d), indexing="ij")     # grid[k] has axis k = direction k
    u = 0.25 + sum(slopes[k] * grid[k] for k in range(d))
    wprod = np.ones_like(u)
    for k in range(d):
        wprod = wprod * w.reshape([n if a == k else 1 for a in range(d)])
    # flatten with x fastest
    flat = lambda a: np.transpose(a, list(range(d))[::-1]).reshape(-1)
    uu = flat(u)[None, None, :]
    y = orc.dense_volume(uu, n, d, "burgers", Q=Q, w=w)
    ref = flat(wprod * u) * slopes.sum() / 2.0
    assert np.abs(y[0, 0] - ref).max() < 2e-14 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("flux", ["euler", "euler_pfix"])
@pytest.mark.parametrize("n,kind", [(4, "gl"), (5, "gll"), (8, "gl")])
def test_freestream_is_zero(orc, n, kind, flux):
    """Constant state: Q 1 = 0 and f(u,u) = f(u) give y = 0."""
    from paper_2306_11665_amd import workloads as W
    E = 2
    u = W.euler_state(E, n, seed=11, freestream_frac=1.0)
    y = orc.dense_volume(u, n, 3, flux, nodes_kind=kind)
    fmax = max(np.abs(orc.physical_flux_euler(u[:, e, 0], m)).max() for e in range(E) for m in range(3))
    assert np.abs(y).max() <= 1e-13 * fmax


def _line_boundary_sum(orc, flux, ue, n, d, x, w, gamma=1.4):
    """sum over all nodes of y via the SBP line identity:
    each line contributes w_perp * (t_R^T F t_R - t_L^T F t_L) / 2."""
    def lag(t):
        out = np.ones(n)
        for j in range(n):
            for k in range(n):
                if k != j:
                    out[j] *= (t - x[k]) / (x[j] - x[k])
        return out
    tR, tL = lag(1.0), lag(-1.0)
    nv = ue.shape[0]
    total = np.zeros(nv)
    for m in range(d):
        others = [k for k in range(d) if k != m]
        for q in np.ndindex(*([n] * (d - 1))):
            dig = [0] * d
            for k, v in zip(others, q):
                dig[k] = v
            wperp = np.prod([w[v] for v in q])
            nodes = []
            for a in range(n):
                dig[m] = a
                nodes.append(sum(dig[k] * n ** k for k in range(d)))
            acc = np.zeros(nv)
            for a in range(n):
                for c in range(n):
                    F = orc.flux(flux, ue[:, nodes[a]], ue[:, nodes[c]], m, gamma)
                    acc += (tR[a] * tR[c] - tL[a] * tL[c]) * F
            total += wperp * 0.5 * acc
    return total


@pytest.mark.parametrize("n,kind", [(3, "gll"), (4, "gl"), (5, "gll")])
def test_line_conservation_euler(orc, n, kind):
    """Summation by parts: 1^T y equals the boundary sum per line (pins the
    reduction direction, the sign and the w_perp scaling)."""
    from paper_2306_11665_amd import workloads as W
    x, w, D, Q = orc.operator_1d(n, kind)
    u = W.euler_state(1, n, seed=5)
    y = orc.dense_volume(u, n, 3, "euler", Q=Q, w=w)
    ref = _line_boundary_sum(orc, "euler", u[:, 0, :], n, 3, x, w)
    np.testing.assert_allclose(y[:, 0, :].sum(axis=1), ref, rtol=0, atol=2e-14 * max(1, np.abs(ref).max()))


def test_line_conservation_burgers_2d(orc):
    from paper_2306_11665_amd import workloads as W
    n = 4
    x, w, D, Q = orc.operator_1d(n, "gll")
    u = W.scalar_state(1, n, 2, seed=9)
    y = orc.dense_volume(u, n, 2, "burgers", Q=Q, w=w)
    ref = _line_boundary_sum(orc, "burgers", u[:, 0, :], n, 2, x, w)
    assert abs(y[0, 0].sum() - ref[0]) < 1e-14


def test_skew_part_sums_to_zero(orc):
    """1^T ((Q - Q^T) o S) 1 = 0 for symmetric S: the skew part carries no total."""
    for n, kind in [(4, "gl"), (8, "gl"), (8, "gll")]:
        x, w, D, Q = orc.operator_1d(n, kind)
        rng = np.random.default_rng(n)
        S = rng.standard_normal((n, n)); S = S + S.T
        assert abs(np.sum((Q - Q.T) * S)) < 1e-13


# ------------------------------------------------------ dense vs the method
@pytest.mark.parametrize("flux,d,n,kind", [("burgers", 2, 4, "gll"), ("euler", 3, 4, "gl"),
                                          ("euler", 3, 5, "gll"), ("product", 3, 6, "gl"),
                                          ("burgers", 3, 3, "gl"), ("euler", 3, 8, "gl"),
                                          ("euler_pfix", 3, 5, "gl")])
def test_sf_method_equals_dense_definition(orc, flux, d, n, kind):
    from paper_2306_11665_amd import workloads as W
    E = 2 if n >= 8 else 5
    if flux in ("euler", "euler_pfix"):
        u = W.euler_state(E, n, seed=3, d=d)
    else:
        u = W.scalar_state(E, n, d, seed=3)
    yd = orc.dense_volume(u, n, d, flux, nodes_kind=kind)
    ys = orc.sf_volume(u, n, d, flux, nodes_kind=kind)
    scale = np.abs(yd).max(axis=(1, 2), keepdims=True)
    assert (np.abs(yd - ys) / scale).max() < 1e-14


# ------------------------------------------------------ mpmath brute force
def _mp_operator(n, kind, mp):
    """Nodes, weights and D at high precision, by routes unlike the oracle's:
    mpmath root polishing and the direct (non-barycentric) derivative formula."""
    if kind == "gl":
        guess = np.polynomial.legendre.leggauss(n)[0]
        P = lambda t: mp.legendre(n, t)
        x = [mp.findroot(P, mp.mpf(float(g))) for g in guess]
        w = [2 / ((1 - t ** 2) * mp.diff(P, t) ** 2) for t in x]
    else:
        N = n - 1
        dP = lambda t: mp.diff(lambda s: mp.legendre(N, s), t)
        inner = []
        if n > 2:
            from scipy.special import roots_jacobi
            inner = [mp.findroot(dP, mp.mpf(float(g))) for g in np.sort(roots_jacobi(n - 2, 1, 1)[0])]
        x = [mp.mpf(-1)] + inner + [mp.mpf(1)]
        w = [mp.mpf(2) / (N * (N + 1) * mp.legendre(N, t) ** 2) for t in x]
    D = [[mp.mpf(0)] * n for _ in range(n)]
    for i in range(n):
        for j in range(n):
            if i == j:
                D[i][i] = mp.fsum(1 / (x[i] - x[k]) for k in range(n) if k != i)
            else:
                num = mp.fprod([x[i] - x[k] for k in range(n) if k not in (i, j)])
                den = mp.fprod([x[j] - x[k] for k in range(n) if k != j])
                D[i][j] = num / den
    Q = [[w[i] * D[i][j] for j in range(n)] for i in range(n)]
    return x, w, Q


def _mp_flux(flux, uL, uR, m, mp, gamma):
    if flux == "burgers":
        a, b = uL[0], uR[0]
        return [(a * a + a * b + b * b) / 6]
    if flux == "product":
        return [uL[0] * uR[0]]
    g = mp.mpf(gamma)

    def prim(u):
        r = u[0]; v = [u[1] / r, u[2] / r, u[3] / r]
        p = (g - 1) * (u[4] - r * (v[0] ** 2 + v[1] ** 2 + v[2] ** 2) / 2)
        return r, v, p, r / (2 * p)

    rl, vl, pl, bl = prim(uL); rr, vr, pr, br = prim(uR)
    lm = lambda a, b: a if a == b else (a - b) / (mp.log(a) - mp.log(b))
    rho_ln, beta_ln = lm(rl, rr), lm(bl, br)
    vb = [(vl[k] + vr[k]) / 2 for k in range(3)]
    phat = (rl + rr) / 2 / (bl + br)
    Fr = rho_ln * vb[m]
    Fm = [Fr * vb[k] + (phat if k == m else 0) for k in range(3)]
    # equivalent algebraic form of the energy flux (v_L . v_R instead of {{|v|^2}})
    vlvr = vl[0] * vr[0] + vl[1] * vr[1] + vl[2] * vr[2]
    FE = Fr * (1 / (2 * (g - 1) * beta_ln) + vlvr / 2) + phat * vb[m]
    return [Fr] + Fm + [FE]


@pytest.mark.parametrize("flux,d,n,kind", [("burgers", 2, 2, "gl"), ("burgers", 2, 3, "gll"),
                                          ("product", 3, 3, "gl"), ("burgers", 3, 2, "gll"),
                                          ("euler", 3, 2, "gl"), ("euler", 3, 3, "gll"),
                                          ("euler", 3, 3, "gl")])
def test_bruteforce_mpmath(orc, flux, d, n, kind):
    import mpmath as mp
    from paper_2306_11665_amd import workloads as W
    mp.mp.dps = 40
    gamma = 1.4
    if flux == "euler":
        u = W.euler_state(1, n, seed=21, d=d)
    else:
        u = W.scalar_state(1, n, d, seed=21)
    y = orc.dense_volume(u, n, d, flux, nodes_kind=kind)
    x, w, Q = _mp_operator(n, kind, mp)
    N = n ** d
    nv = u.shape[0]
    um = [[mp.mpf(float(u[v, 0, i])) for v in range(nv)] for i in range(N)]
    ref = [[mp.mpf(0)] * nv for _ in range(N)]
    for m in range(d):
        for i in range(N):
            di = _digits(i, n, d)
            for j in range(N):
                dj = _digits(j, n, d)
                if any(di[k] != dj[k] for k in range(d) if k != m):
                    continue     # A_m[i, j] is a structural zero
                a = Q[di[m]][dj[m]]
                for k in range(d):
                    if k != m:
                        a *= w[di[k]]
                F = _mp_flux(flux, um[i], um[j], m, mp, gamma)
                for v in range(nv):
                    ref[i][v] += a * F[v]
    R = np.array([[float(ref[i][v]) for i in range(N)] for v in range(nv)])
    for v in range(nv):
        scale = max(np.abs(R[v]).max(), 1e-300)
        assert np.abs(y[v, 0] - R[v]).max() / scale < 2e-14, (v, np.abs(y[v, 0] - R[v]).max() / scale)


# ------------------------------------------------------ Figure 1 cost slopes
@pytest.mark.slow
def test_cost_slopes_figure1(orc):
    """Figure 1 (Results section): in 3D the direct Hadamard product scales
    with slope 6 on a log-log plot and the sum-factorized one with slope 4.
    Workload: C_ij = c_i c_j, c ~ U[1e-8, 30], unweighted D, one thread."""
    with open(os.path.join(GOLDEN, "fig1_slopes.json")) as f:
        gold = json.load(f)
    def slopes():
        ns = [4, 5, 6, 7, 8]
        td, ts = [], []
        for n in ns:
            x, w, D, Q = orc.operator_1d(n, "gl")
            rng = np.random.default_rng(n)
            Ed = max(1, int(2 * 9 ** 6 / n ** 6))
            Es = max(1, int(400 * 9 ** 4 / n ** 4))
            cd = rng.uniform(1e-8, 30.0, size=(1, Ed, n ** 3))
            cs = rng.uniform(1e-8, 30.0, size=(1, Es, n ** 3))
            best_d = best_s = np.inf
            for _ in range(5):
                t0 = time.perf_counter(); orc.dense_volume(cd, n, 3, "product", Q=D, w=np.ones(n))
                best_d = min(best_d, (time.perf_counter() - t0) / Ed)
                t0 = time.perf_counter(); orc.sf_volume(cs, n, 3, "product", Q=D, w=np.ones(n))
                best_s = min(best_s, (time.perf_counter() - t0) / Es)
            td.append(best_d); ts.append(best_s)
        return np.polyfit(np.log(ns), np.log(td), 1)[0], np.polyfit(np.log(ns), np.log(ts), 1)[0], td, ts

    def ok(sd, ss):
        return abs(sd - gold["dense_slope"]) < 0.6 and abs(ss - gold["sum_factorized_slope"]) < 0.6

    # a wall-clock measurement: a busy host can distort one sweep, so up to
    # three sweeps are taken and the first inside the bound counts
    old = orc.num_threads()
    orc.set_num_threads(1)
    try:
        tries = []
        for _ in range(3):
            sd, ss, td, ts = slopes()
            tries.append((round(sd, 2), round(ss, 2)))
            if ok(sd, ss):
                break
    finally:
        orc.set_num_threads(old)
    assert ok(sd, ss), (tries, td, ts)
