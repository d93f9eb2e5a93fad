"""Pins of the oracle's mass-transfer step, random walk and reaction (CPU only).

Each test fixes a property that the paper or the mathematics determines
independently of the oracle's code: brute-force neighbour sets, closed forms on
two particles and on a lattice, conservation and symmetry, the maximum
principle, the analytic erfc spreading of Sec. 2.1, the exact solution of the
well-mixed reaction, and compensated sums against math.fsum.
"""
import math

import numpy as np
import pytest
from scipy import special

from paper_2204_03756_amd import workloads as W


# ------------------------------------------------------------ neighbours --
@pytest.mark.parametrize("dim,n", [(2, 1), (2, 7), (2, 3000), (2, 20000), (3, 5000), (3, 20000)])
def test_kdtree_equals_brute_force(oracle, dim, n):
    w = W.plain2d(n=n) if dim == 2 else W.rw3d(n=n)
    psi = w.params.psi_eff
    rb, cb = oracle.neighbors(w.x0, psi, "brute")
    rk, ck = oracle.neighbors(w.x0, psi, "kdtree")
    assert np.array_equal(rb, rk) and np.array_equal(cb, ck)
    # self always included, relation symmetric
    rows = np.repeat(np.arange(n), np.diff(rb))
    assert np.all(np.isin(np.arange(n), cb))
    a = set(zip(rows.tolist(), cb.tolist()))
    assert all((j, i) in a for (i, j) in a)


def _lattice(nx, ny, nz=None, h=1.0):
    if nz is None:
        g = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy"), -1).reshape(-1, 2)
    else:
        g = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij"),
                     -1).reshape(-1, 3)
    return g.astype(np.float64) * h


@pytest.mark.parametrize("method", ["brute", "kdtree"])
def test_cutoff_is_inclusive_on_lattice_ties(oracle, method):
    """Unit lattice: r2 = 1 exactly for the 4 (2-d) / 6 (3-d) nearest sites, so
    psi = 1 keeps them (r2 <= psi^2) and the next double below 1 drops them."""
    x = _lattice(9, 7)
    r, _ = oracle.neighbors(x, 1.0, method)
    cnt = np.diff(r).reshape(7, 9)
    assert np.all(cnt[1:-1, 1:-1] == 5) and cnt[0, 0] == 3 and cnt[0, 4] == 4
    r, _ = oracle.neighbors(x, np.nextafter(1.0, 0.0), method)
    assert np.all(np.diff(r) == 1)
    x3 = _lattice(5, 5, 5)
    r, _ = oracle.neighbors(x3, 1.0, method)
    assert np.diff(r).reshape(5, 5, 5)[2, 2, 2] == 7
    # sqrt(2) diagonal is in at psi = 1.5, out at 1.2
    r, _ = oracle.neighbors(x, 1.5, method)
    assert np.diff(r).reshape(7, 9)[3, 4] == 9


# ------------------------------------------------------ weights / update --
@pytest.mark.parametrize("beta", [0.5, 0.25, 1.0])
def test_two_particles_closed_form(oracle, beta):
    d_mt, dt, r = 0.7, 0.1, 0.9
    x = np.array([[10.0, 10.0], [10.0 + r, 10.0]])
    m = np.array([[0.3, 1.7]])
    K = math.exp(-beta * r * r / (4 * d_mt * dt))
    s, _, wv = oracle.mt_weights(x, *oracle.neighbors(x, 2.0), d_mt, dt, beta)
    assert s == pytest.approx([1 + K, 1 + K], rel=1e-15)
    assert wv[1] == pytest.approx(K / (1 + K), rel=1e-15)
    out, pairs = oracle.mt_step(x, m, d_mt, dt, beta, 2.0)
    assert pairs == 2
    expect = 0.3 + beta * K / (1 + K) * (1.7 - 0.3)
    assert out[0, 0] == pytest.approx(expect, rel=1e-15)
    assert out[0, 1] == pytest.approx(2.0 - expect, rel=1e-15)
    # beyond psi nothing moves
    out, pairs = oracle.mt_step(x, m, d_mt, dt, beta, 0.5)
    assert pairs == 0 and np.array_equal(out, m)


def test_lattice_stencil_closed_forms(oracle):
    """Unit lattice with beta = 1/2 and 8 D_MT dt = 1, so K = exp(-r^2):
    interior N(i) = self + 4 sites, s = 1 + 4/e, W = e^-1/(1 + 4/e).  A linear
    field is a fixed point in the interior; m = x^2 gives delta = 2 beta W."""
    beta, d_mt, dt = 0.5, 0.125, 1.0
    nx, ny = 12, 10
    x = _lattice(nx, ny)
    for psi in (1.2, 1.0):
        row, col = oracle.neighbors(x, psi)
        s, _, wv = oracle.mt_weights(x, row, col, d_mt, dt, beta)
        s = s.reshape(ny, nx)
        e1 = math.exp(-1.0)
        assert np.allclose(s[2:-2, 2:-2], 1 + 4 * e1, rtol=1e-15, atol=0)
        Wexp = e1 / (1 + 4 * e1)
        interior = [i for i in range(nx * ny) if 2 <= i % nx < nx - 2 and 2 <= i // nx < ny - 2]
        for i in interior[:10]:
            ws = [wv[e] for e in range(row[i], row[i + 1]) if col[e] != i]
            assert np.allclose(ws, Wexp, rtol=1e-15)
        lin = (3.0 + 2.0 * x[:, 0] - 1.0 * x[:, 1])[None, :]
        out, _ = oracle.mt_step(x, lin, d_mt, dt, beta, psi)
        d = (out - lin)[0].reshape(ny, nx)
        assert np.all(d[2:-2, 2:-2] == 0.0)
        sq = (x[:, 0] ** 2)[None, :]
        out, _ = oracle.mt_step(x, sq, d_mt, dt, beta, psi)
        d = (out - sq)[0].reshape(ny, nx)
        assert np.allclose(d[2:-2, 2:-2], 2 * beta * Wexp, rtol=1e-13, atol=0)


def test_weights_symmetric_and_bounded(oracle):
    for w in (W.plain2d(n=5000), W.rw3d(n=8000)):
        x = w.x0
        row, col = oracle.neighbors(x, w.params.psi_eff)
        s, kv, wv = oracle.mt_weights(x, row, col, w.params.d_mt, w.params.dt, w.params.beta)
        n = x.shape[0]
        rows = np.repeat(np.arange(n), np.diff(row))
        key = rows * n + col
        tkey = col * n + rows
        order = np.argsort(key)
        pos = np.searchsorted(key[order], tkey)
        assert np.array_equal(key[order][pos], tkey)
        assert np.array_equal(wv, wv[order][pos])           # W_ij == W_ji bit for bit
        rs = np.bincount(rows, weights=wv, minlength=n)
        assert np.all(rs > 0) and np.all(rs <= 2.0)
        assert np.all(s >= 1.0)                               # self term K_ii = 1


def test_constant_field_conservation_and_max_principle(oracle):
    w = W.plain2d(n=6000)
    p = w.params
    const = np.full((1, p.n), 0.625)
    out, _ = oracle.mt_step(w.x0, const, p.d_mt, p.dt, p.beta, p.psi_eff)
    assert np.array_equal(out, const)
    rng = np.random.default_rng(3)
    m = rng.random((2, p.n))
    for beta in (0.5, 0.3):
        out, _ = oracle.mt_step(w.x0, m, p.d_mt, p.dt, beta, p.psi_eff)
        for c in range(2):
            assert abs(out[c].sum() - m[c].sum()) <= 1e-12 * m[c].sum()
            assert out[c].min() >= m[c].min() and out[c].max() <= m[c].max()


def test_total_is_compensated(oracle):
    rng = np.random.default_rng(5)
    v = np.concatenate([rng.random(10000) * 1e-8, [1e16, -1e16, 3.0, 1e-3]])
    rng.shuffle(v)
    exact = math.fsum(v)
    eps = 2.0 ** -53
    # Neumaier's bound: |err| <= 2 eps |S| + O(n eps^2) sum|v|
    bound = 2 * eps * abs(exact) + 4 * v.size * eps * eps * np.abs(v).sum()
    assert abs(oracle.total(v) - exact) <= bound
    naive = 0.0
    for t in v:
        naive += t
    assert abs(naive - exact) > 1e3 * bound     # the case really needs compensation


# ----------------------------------------------------------- random walk --
def test_rw_variance_reflection_and_fp32(oracle):
    n, dim = 200_000, 3
    lo, hi = [0.0, 0.0, 0.0], [1000.0, 1000.0, 1000.0]
    x0 = np.full((n, dim), 500.0)
    d_rw, dt = 1.3, 0.1
    x1 = oracle.rw_step(x0, lo, hi, d_rw, dt, 99, 4)
    dx = x1 - x0
    var = 2 * d_rw * dt
    assert np.all(np.abs(dx.mean(0)) < 5 * math.sqrt(var / n))
    assert np.all(np.abs(dx.var(0) / var - 1) < 5 * math.sqrt(2.0 / n))
    # a small box forces repeated reflections: every coordinate stays inside
    xs = np.full((n, 2), 0.5)
    xb = oracle.rw_step(xs, [0.0, 0.0], [1.0, 1.0], 50.0, 0.1, 7, 0)
    assert np.all((xb >= 0.0) & (xb <= 1.0))
    # reflection is the mirror image: the unfolded jump equals the free jump
    free = oracle.rw_step(xs, [-1e9, -1e9], [1e9, 1e9], 50.0, 0.1, 7, 0) - 0.5
    folded = np.abs(((free + 0.5) % 2.0 + 2.0) % 2.0)
    folded = np.where(folded > 1.0, 2.0 - folded, folded)
    assert np.allclose(folded, xb, atol=1e-12)
    # FP32 state stays float-representable
    x32 = oracle.rw_step(x0.astype(np.float32).astype(np.float64), lo, hi, d_rw, dt, 99, 4,
                         fp32=True)
    assert np.array_equal(x32, x32.astype(np.float32).astype(np.float64))
    assert np.max(np.abs(x32 - x1)) < 1e-4


def test_rw_keeps_uniform_density_uniform(oracle):
    """Reflecting walls preserve the uniform distribution: chi^2 over cells."""
    w = W.rw2d(n=40_000)
    p = w.params
    res = oracle.run(p, w.x0, w.m0, 1, method="kdtree")
    x = w.x0
    for t in range(30):
        x = oracle.rw_step(x, p.lo[:2], p.hi[:2], 50.0, 0.1, p.seed, t)
    h, _, _ = np.histogram2d(x[:, 0], x[:, 1], bins=20, range=[[0, p.hi[0]], [0, p.hi[1]]])
    e = p.n / 400
    chi2 = ((h - e) ** 2 / e).sum()
    assert stats_chi2_sf(chi2, 399) > 1e-4
    assert res.pairs[0] > 0


def stats_chi2_sf(x, k):
    return float(special.gammaincc(k / 2.0, x / 2.0))


def test_run_resume_is_bitwise(oracle):
    w = W.rw2d(n=20_000)
    p = w.params
    full = oracle.run(p, w.x0, w.m0, 6)
    a = oracle.run(p, w.x0, w.m0, 3)
    p2 = W.Params(**{**p.as_dict(), "start_step": 3})
    b = oracle.run(p2, a.x, a.m, 3)
    assert np.array_equal(full.x, b.x) and np.array_equal(full.m, b.m)
    assert np.array_equal(full.pairs[3:], b.pairs)


# ------------------------------------------------------------- physics ----
def _d_eff_mean_field(rho, d_mt, dt, beta, psi, dim):
    """Mean-field D_eff of the normalised kernel with the self term in s_i:
    D_MT * rho' P(d/2+1, a) / (1 + rho' P(d/2, a)), rho' = rho (2 pi h^2)^(d/2),
    h^2 = 2 D_MT dt / beta, a = psi^2 / (2 h^2) (for beta = 1/2)."""
    h2 = 2 * d_mt * dt / beta
    rp = rho * (2 * math.pi * h2) ** (dim / 2)
    a = psi * psi / (2 * h2)
    return d_mt * rp * special.gammainc(dim / 2 + 1, a) / (1 + rp * special.gammainc(dim / 2, a))


def _fit_erfc_d(x, m, t, x0c, half):
    """Least-squares D of 1/2 erfc((x - x0c)/sqrt(4 D t)) over |x - x0c| < half."""
    xs = x[:, 0]
    mask = np.abs(xs - x0c) < half
    Ds = np.linspace(0.2, 1.4, 241)
    err = [np.mean((m[mask] - 0.5 * special.erfc((xs[mask] - x0c) / math.sqrt(4 * D * t))) ** 2)
           for D in Ds]
    i = int(np.argmin(err))
    return Ds[i], math.sqrt(err[i])


def test_plain2d_spreads_as_erfc(oracle):
    """Sec. 2.1: a Heaviside initial mass spreads as 1/2 erfc((x-x')/sqrt(4 D t)).

    * The kernel's second moment sum_j W_ij dx^2 * beta/(2 dt) equals the
      mean-field D_eff of the Gaussian integral with the self term in s_i
      (0.68 D_MT at the plain2d density 1).
    * On random points the operator is a random conductance network, whose
      effective D can only be lower than that affine-field value (Dirichlet
      principle) and approaches it as the density grows: at density 10 the
      fitted D must sit within 8 % of the mean-field value, and below it.
    * The RMSE against the fitted profile is at particle-noise level."""
    w = W.plain2d()
    p = w.params
    t = w.steps * p.dt
    d_mf = _d_eff_mean_field(1.0, p.d_mt, p.dt, p.beta, p.psi_eff, 2)
    assert 0.6 < d_mf < 0.75
    row, col = oracle.neighbors(w.x0, p.psi_eff)
    _, _, wv = oracle.mt_weights(w.x0, row, col, p.d_mt, p.dt, p.beta)
    rows = np.repeat(np.arange(p.n), np.diff(row))
    dx = w.x0[col, 0] - w.x0[rows, 0]
    xi = w.x0
    inner = (xi[:, 0] > 4) & (xi[:, 0] < 96) & (xi[:, 1] > 4) & (xi[:, 1] < 96)
    d2 = p.beta / (2 * p.dt) * np.bincount(rows, weights=wv * dx * dx, minlength=p.n)[inner].mean()
    assert abs(d2 / d_mf - 1) < 0.02
    res = oracle.run(p, w.x0, w.m0, w.steps)
    d_fit, rmse = _fit_erfc_d(w.x0, res.m[0], t, 50.0, 15.0)
    assert 0.5 * d_mf < d_fit < d2
    assert rmse < 0.06
    assert abs(res.totals[-1, 0] - w.m0.sum()) <= 1e-12 * w.m0.sum()
    # resolved: density 10 (same sizes otherwise)
    n = 40_000
    L = math.sqrt(n / 10.0)
    wr = W.plain2d(n=n)
    xr = wr.x0 * (L / wr.params.hi[0])
    pr = W.Params(**{**wr.params.as_dict(), "hi": [L, L, 0.0]})
    mr = (xr[:, 0] < L / 2).astype(np.float64)[None, :]
    rr = oracle.run(pr, xr, mr, 50)
    d_fit10, rmse10 = _fit_erfc_d(xr, rr.m[0], t, L / 2, 15.0)
    d_mf10 = _d_eff_mean_field(10.0, pr.d_mt, pr.dt, pr.beta, pr.psi_eff, 2)
    assert 0.92 * d_mf10 < d_fit10 <= d_mf10
    assert rmse10 < 0.02


# ----------------------------------------------------------- advection ----
def test_drift_moves_straight_and_piles_up_at_walls(oracle):
    """D_RW = 0 with a drift v: a particle whose straight path x0 + k v dt
    stays inside the box is there after k steps (to the rounding of k
    additions); one that reaches a wall is mirrored back each step and the
    drift pushes it in again, so it stays within |v| dt of the wall it
    drifts into (zero-flux walls hold the advected particles)."""
    rng = np.random.default_rng(21)
    lo, hi = np.array([0.0, 0.0]), np.array([10.0, 7.0])
    x0 = lo + rng.random((5000, 2)) * (hi - lo)
    vel, dt, k = np.array([1.3, -2.1]), 0.1, 20
    p = W.Params(dim=2, n=len(x0), lo=[0.0, 0.0, 0.0], hi=[10.0, 7.0, 0.0], d_rw=0.0, d_mt=1e-4,
                 dt=dt, vel=[vel[0], vel[1], 0.0])
    for prec, tol in ((W.FP64, 1e-12), (W.FP32W_FP64ACC, 2e-4)):
        p.precision = prec
        res = oracle.run(p, x0, np.ones((1, len(x0))), k)
        free = x0 + k * vel * dt
        for d in range(2):
            inside = (free[:, d] >= lo[d]) & (free[:, d] <= hi[d])
            assert inside.sum() > 100 and (~inside).sum() > 100
            assert np.max(np.abs(res.x[inside, d] - free[inside, d])) < tol
            wall = hi[d] if vel[d] > 0 else lo[d]
            gap = np.abs(res.x[~inside, d] - wall)
            assert np.max(gap) <= abs(vel[d]) * dt * (1 + 1e-6) + tol
    # the drift adds to the random jump: with D_RW > 0 the step is the jump of
    # the same normals plus v dt (away from the walls)
    xc = np.full((1000, 2), 5.0)
    step = oracle.rw_step(xc, [-1e9, -1e9], [1e9, 1e9], 0.7, 0.1, 3, 5, vel=[1.3, -2.1])
    free = oracle.rw_step(xc, [-1e9, -1e9], [1e9, 1e9], 0.7, 0.1, 3, 5)
    assert np.allclose(step - free, vel * dt, atol=1e-12, rtol=0)


def test_drift_translates_the_erfc_profile(oracle):
    """The advection-dispersion equation: with a drift v the Heaviside
    interface of Sec. 2.1 moves to x' + v t and spreads as before
    (1/2 erfc((x - x' - v t)/sqrt(4 D t)) with the same effective D)."""
    w = W.plain2d()
    p = W.Params(**{**w.params.as_dict(), "vel": [2.0, 0.0, 0.0]})
    t = w.steps * p.dt
    res = oracle.run(p, w.x0, w.m0, w.steps)
    x1 = res.x
    d_mf = _d_eff_mean_field(1.0, p.d_mt, p.dt, p.beta, p.psi_eff, 2)
    d_fit, rmse = _fit_erfc_d(x1, res.m[0], t, 50.0 + 2.0 * t, 15.0)
    assert 0.5 * d_mf < d_fit < 1.05 * d_mf
    assert rmse < 0.06
    _, rmse_unshifted = _fit_erfc_d(x1, res.m[0], t, 50.0, 15.0)
    assert rmse_unshifted > 3 * rmse
    assert abs(res.totals[-1, 0] - w.m0.sum()) <= 1e-12 * w.m0.sum()


# ------------------------------------------------- dispersion tensor ----
def _spd(rng, dim, cond=8.0):
    """A random symmetric positive-definite [3][3] tensor (2-d: 2x2 block used)."""
    q, _ = np.linalg.qr(rng.standard_normal((dim, dim)))
    ev = np.exp(rng.uniform(0.0, math.log(cond), dim))
    t = q @ np.diag(ev) @ q.T
    t = 0.5 * (t + t.T)
    t3 = np.eye(3)
    t3[:dim, :dim] = t
    return t3


@pytest.mark.parametrize("dim", [2, 3])
def test_tensor_distance_is_mahalanobis(oracle, dim):
    """The cutoff metric under a shape tensor T is dx^T T^-1 dx (numpy's
    inverse as the reference), and T = I gives the Euclidean r^2 bit for bit."""
    rng = np.random.default_rng(31 + dim)
    for _ in range(20):
        t = _spd(rng, dim)
        ti = np.linalg.inv(t[:dim, :dim])
        for _ in range(20):
            xi = rng.uniform(-5, 5, dim)
            xj = xi + rng.normal(0, 1.5, dim)
            dx = xj - xi
            ref = dx @ ti @ dx
            assert oracle.pair_dist2(xi, xj, t) == pytest.approx(ref, rel=1e-12)
    for _ in range(50):
        xi = rng.uniform(-5, 5, dim)
        xj = xi + rng.normal(0, 1.5, dim)
        assert oracle.pair_dist2(xi, xj, np.eye(3)) == oracle.pair_dist2(xi, xj, None)
    bad = np.eye(3); bad[0, 1] = 0.5   # not symmetric
    with pytest.raises(ValueError):
        oracle.pair_dist2(np.zeros(dim), np.ones(dim), bad)
    neg = np.eye(3); neg[1, 1] = -1.0
    with pytest.raises(ValueError):
        oracle.pair_dist2(np.zeros(dim), np.ones(dim), neg)


@pytest.mark.parametrize("dim,n", [(2, 3000), (3, 4000)])
def test_tensor_neighbors_equal_brute_force(oracle, dim, n):
    """Ellipsoidal cutoff: the K-D tree (pruned by the ellipsoid's reach along
    each axis) and the brute-force search give the set of pairs with
    dx^T T^-1 dx <= psi^2, computed here with numpy's inverse (pairs within
    1e-9 of the cutoff are left out of the comparison)."""
    rng = np.random.default_rng(7 * dim)
    L = n ** (1.0 / dim)
    x = rng.uniform(0, L, (n, dim))
    t = _spd(rng, dim, cond=10.0)
    psi = 1.3
    rb, cb = oracle.neighbors(x, psi, "brute", tens=t)
    rk, ck = oracle.neighbors(x, psi, "kdtree", tens=t)
    assert np.array_equal(rb, rk) and np.array_equal(cb, ck)
    ti = np.linalg.inv(t[:dim, :dim])
    rows = np.repeat(np.arange(n), np.diff(rk))
    got = set(zip(rows.tolist(), ck.tolist()))
    # reference: all pairs (chunked), with numpy's quadratic form
    for i0 in range(0, n, 500):
        dx = x[None, :, :] - x[i0:i0 + 500, None, :]
        q = np.einsum("abk,kl,abl->ab", dx, ti, dx)
        ii, jj = np.nonzero(q <= psi * psi * (1 - 1e-9))
        for i, j in zip((ii + i0).tolist(), jj.tolist()):
            assert (i, j) in got
        ii, jj = np.nonzero(q <= psi * psi * (1 + 1e-9))
        assert sum(1 for i, j in zip((ii + i0).tolist(), jj.tolist()) if (i, j) in got) == \
            sum(1 for r in range(i0, min(n, i0 + 500)) for _ in range(rk[r + 1] - rk[r]))


def test_tensor_pair_closed_form(oracle):
    """A pair at distance r along principal axis e_k (eigenvalue l_k) of a
    rotated tensor exchanges with K = exp(-beta r^2 / (4 l_k D_MT dt)); the
    cutoff r^2 / l_k <= psi^2 keeps it or drops it.  The positions do not
    move without a walk."""
    d_mt, dt, beta = 0.7, 0.1, 0.5
    eig = [4.0, 0.25]
    ang = 0.4
    t = W.rotated_tensor(eig, [ang])
    e = [np.array([math.cos(ang), math.sin(ang)]), np.array([-math.sin(ang), math.cos(ang)])]
    m = np.array([[0.3, 1.7]])
    for k in (0, 1):
        for r in (0.45, 0.9, 1.1, 3.5):
            x = np.array([[10.0, 10.0], [10.0, 10.0]]) + np.array([[0.0, 0.0], r * e[k]])
            p = W.Params(dim=2, n=2, lo=[0.0, 0.0, 0.0], hi=[20.0, 20.0, 0.0], d_rw=0.0, d_mt=d_mt,
                         dt=dt, beta=beta, psi=2.0, disp=t)
            res = oracle.run(p, x, m, 1, method="brute")
            if r * r / eig[k] <= 4.0 * (1 - 1e-9):
                K = math.exp(-beta * r * r / (4 * eig[k] * d_mt * dt))
                expect = 0.3 + beta * K / (1 + K) * (1.7 - 0.3)
                assert res.pairs[0] == 2
                assert res.m[0, 0] == pytest.approx(expect, rel=1e-12)
                assert res.m[0, 1] == pytest.approx(2.0 - expect, rel=1e-12)
            elif r * r / eig[k] > 4.0 * (1 + 1e-9):
                assert res.pairs[0] == 0 and np.array_equal(res.m, m)
            assert np.array_equal(res.x, x)


@pytest.mark.parametrize("dim", [2, 3])
def test_tensor_walk_covariance(oracle, dim):
    """The jumps under a shape tensor T have covariance 2 d_rw dt T (their
    sample covariance within 5 standard errors of every entry), so the walk
    realises D_RW = d_rw T; the walls stay mirrors of the box."""
    rng = np.random.default_rng(5 + dim)
    t = _spd(rng, dim, cond=6.0)
    n = 200_000
    L = 1000.0
    x = np.full((n, dim), L / 2)
    d_rw, dt = 0.8, 0.1
    lo = [0.0] * dim
    hi = [L] * dim
    y = oracle.rw_step(x, lo, hi, d_rw, dt, 77, 3, tens=t)
    d = y - x
    c = np.cov(d.T, bias=True)
    ref = 2 * d_rw * dt * t[:dim, :dim]
    # standard error of a sample covariance entry: sqrt((S_kk S_ll + S_kl^2) / n)
    se = np.sqrt((np.outer(np.diag(ref), np.diag(ref)) + ref * ref) / n)
    assert np.all(np.abs(c - ref) < 5 * se)
    assert np.all(np.abs(d.mean(axis=0)) < 5 * np.sqrt(np.diag(ref) / n))
    # reflection keeps the box: start next to the lower walls
    x0 = np.full((2000, dim), 0.05)
    y0 = oracle.rw_step(x0, lo, hi, 50.0, 1.0, 78, 0, tens=t)
    assert np.all(y0 >= 0.0) and np.all(y0 <= L)
    # the identity tensor is the isotropic walk, bit for bit
    yi = oracle.rw_step(x[:5000], lo, hi, d_rw, dt, 77, 3, tens=np.eye(3))
    yn = oracle.rw_step(x[:5000], lo, hi, d_rw, dt, 77, 3)
    assert np.array_equal(yi, yn)


def test_tensor_spreading_rates(oracle):
    """A Heaviside front whose normal is principal axis e_k of a rotated
    tensor spreads as 1/2 erfc(s / sqrt(4 D t)) along e_k with D = l_k times
    the isotropic mean-field effective D (det T = 1 keeps the density of the
    whitened frame), for both axes (the erfc fit of Sec. 2.1 along each)."""
    n = 40_000
    L = math.sqrt(n / 10.0)
    w = W.plain2d(n=n)
    x0 = w.x0 * (L / w.params.hi[0])
    eig = [2.0, 0.5]
    ang = math.pi / 6
    t = W.rotated_tensor(eig, [ang])
    e = [np.array([math.cos(ang), math.sin(ang)]), np.array([-math.sin(ang), math.cos(ang)])]
    p = W.Params(**{**w.params.as_dict(), "hi": [L, L, 0.0], "disp": t})
    tt = 50 * p.dt
    d_mf = _d_eff_mean_field(10.0, p.d_mt, p.dt, p.beta, p.psi_eff, 2)
    c = np.array([L / 2, L / 2])
    central = np.linalg.norm(x0 - c, axis=1) < L / 3
    fits = []
    for k in (0, 1):
        s = (x0 - c) @ e[k]
        m0 = (s < 0).astype(np.float64)[None, :]
        res = oracle.run(p, x0, m0, 50)
        mask = central & (np.abs(s) < 15.0)
        Ds = np.linspace(0.05, 3.0, 1181)
        err = [np.mean((res.m[0][mask] - 0.5 * special.erfc(s[mask] / math.sqrt(4 * D * tt))) ** 2)
               for D in Ds]
        d_fit = Ds[int(np.argmin(err))]
        assert 0.90 * eig[k] * d_mf < d_fit <= 1.02 * eig[k] * d_mf
        fits.append(d_fit)
    assert fits[0] / fits[1] == pytest.approx(eig[0] / eig[1], rel=0.1)


def test_tensor_reaction_uses_the_box_volume(oracle):
    """With a dispersion tensor of determinant 8 and A+B->C, a well-mixed field
    (equal masses everywhere, so the transfer moves nothing) reacts on the
    concentrations c = N M / V of the simulation's own box volume V (Sec. 3's
    mass-to-concentration map): one step gives a0 / (1 + k a0 dt)."""
    n = 3000
    Lx, Ly, Lz = 30.0, 10.0, 10.0
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 1, (n, 3)) * [Lx, Ly, Lz]
    t = W.rotated_tensor([4.0, 2.0, 1.0], [0.3, 0.2, 0.1])
    m0 = np.zeros((3, n))
    m0[0] = m0[1] = 0.7
    k, dt = 1.3, 0.05
    p = W.Params(dim=3, n=n, lo=[0.0, 0.0, 0.0], hi=[Lx, Ly, Lz], d_rw=0.0, d_mt=0.5, dt=dt,
                 beta=0.5, psi=0.0, k_react=k, n_species=3, disp=t)
    res = oracle.run(p, x, m0, 1)
    V = Lx * Ly * Lz
    a0 = 0.7 * n / V
    a1 = a0 / (1 + k * a0 * dt)
    assert np.allclose(res.m[0] * n / V, a1, rtol=1e-12, atol=0)
    assert np.allclose(res.m[2] * n / V, a0 - a1, rtol=1e-12, atol=0)


# ------------------------------------------------------------ reaction ----
def test_reaction_invariants_and_closed_form(oracle):
    rng = np.random.default_rng(9)
    n = 5000
    m = rng.random((3, n))
    V = 2.0 * n
    k, dt = 1.0, 0.05
    out = oracle.react(m, k, dt, V)
    assert np.allclose(out[0] - out[1], m[0] - m[1], rtol=0, atol=1e-15)
    assert np.allclose(out[0] + out[2], m[0] + m[2], rtol=0, atol=1e-15)
    assert np.all(out[0] <= m[0]) and np.all(out[1] <= m[1]) and np.all(out[2] >= m[2])
    # well mixed, a = b: a(t) = a0 / (1 + k a0 t) composes exactly over steps
    c = n / V
    mm = np.zeros((3, 4)); mm[0] = mm[1] = [0.2, 1.0, 3.0, 0.0]
    a0 = mm[0] * c
    for _ in range(40):
        mm = oracle.react(mm, k, dt, 4 / c)
    assert np.allclose(mm[0] * c, a0 / (1 + k * a0 * 40 * dt), rtol=1e-14, atol=0)
    # unequal: a(t) = D / (1 - (b0/a0) exp(-k D t))
    mm = np.zeros((3, 1)); mm[0, 0] = 2.0; mm[1, 0] = 0.5
    a, b = 2.0 * c, 0.5 * c
    for _ in range(40):
        mm = oracle.react(mm, k, dt, 1 / c)
    D = a - b
    assert mm[0, 0] * c == pytest.approx(D / (1 - (b / a) * math.exp(-k * D * 40 * dt)), rel=1e-13)
    assert mm[1, 0] * c == pytest.approx(mm[0, 0] * c - D, rel=1e-13)
