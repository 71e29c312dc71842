"""Pins of the CPU oracle against facts fixed outside the oracle itself:
published known-answer vectors, an independent library implementation,
closed forms, invariants, special cases and brute force on tiny inputs.
Each pin is chosen so that a plausible slip (a dropped term, a wrong sign or
index, a transposed operand) fails it.  CPU only."""
import math
import os
import sys

import numpy as np
import pytest
from scipy import integrate
from scipy.spatial import cKDTree

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import workloads as W  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


# ------------------------------------------------------------------ Philox
def _read_kat():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            v = [int(t, 16) for t in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers(orc):
    rows = _read_kat()
    assert len(rows) == 3
    for ctr, key, expect in rows:
        assert orc.philox(ctr, key) == expect


def test_philox_matches_torch_header(orc):
    import _torch_philox as T
    try:
        T.load()
    except Exception as e:  # pragma: no cover
        pytest.skip(f"cannot compile torch Philox header: {e}")
    rng = np.random.default_rng(7)
    for _ in range(200):
        ctr = [int(v) for v in rng.integers(0, 2 ** 32, 4)]
        key = [int(v) for v in rng.integers(0, 2 ** 32, 2)]
        assert orc.philox(ctr, key) == T.block(ctr, key)


def test_philox_matches_rocrand_header(orc):
    import _rocrand_philox as R
    try:
        R.load()
    except Exception as e:  # pragma: no cover
        pytest.skip(f"cannot compile rocRAND Philox header: {e}")
    rng = np.random.default_rng(8)
    for _ in range(200):
        ctr = [int(v) for v in rng.integers(0, 2 ** 32, 4)]
        key = [int(v) for v in rng.integers(0, 2 ** 32, 2)]
        assert orc.philox(ctr, key) == R.block(ctr, key)


def test_accept_draws_uniform(orc):
    """The acceptance draws u(seed, step, a, b) of 40 000 pairs are uniform on
    [0, 1): chi-square over 50 equal bins, and the mean and variance."""
    from scipy import stats
    rng = np.random.default_rng(9)
    a = rng.integers(0, 2 ** 24, 40000)
    b = a + 1 + rng.integers(0, 2 ** 20, 40000)
    u = np.array([orc.accept_u(12345, 7, int(x), int(y)) for x, y in zip(a, b)])
    assert np.all((u >= 0.0) & (u < 1.0))
    counts, _ = np.histogram(u, bins=50, range=(0.0, 1.0))
    assert stats.chisquare(counts).pvalue > 1e-3
    assert np.mean(u) == pytest.approx(0.5, abs=4 * math.sqrt(1 / 12 / u.size))
    assert np.var(u) == pytest.approx(1 / 12, rel=0.03)


def test_u53_mapping(orc):
    assert orc.u53(0, 0) == 0.0
    assert orc.u53(0, 2048) == 2.0 ** -53
    assert orc.u53(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0 ** -53
    assert orc.u53(0x80000000, 0) == 0.5


def test_accept_u_counter_layout(orc):
    import _torch_philox as T
    try:
        T.load()
    except Exception as e:  # pragma: no cover
        pytest.skip(str(e))
    seed = (0x12345678 << 32) | 0x9ABCDEF0
    w = T.block([5, 17, 3, 0], [0x9ABCDEF0, 0x12345678])
    assert orc.accept_u(seed, 3, 5, 17) == ((w[0] << 32 | w[1]) >> 11) * 2.0 ** -53


# ------------------------------------------------------------------ kernel
@pytest.mark.parametrize("h", [0.3, 1.0, 2.5])
def test_kernel_normalised(orc, h):
    val, _ = integrate.quad(lambda r: 4 * math.pi * r * r * orc.kernel_W(r, h), 0, h,
                            points=[0.5 * h], epsabs=1e-13, epsrel=1e-13)
    assert abs(val - 1.0) < 1e-11
    # continuity at q = 1/2 and compact support
    assert abs(orc.kernel_W(0.5 * h * (1 - 1e-12), h) - orc.kernel_W(0.5 * h * (1 + 1e-12), h)) \
        < 1e-9 * orc.kernel_W(0, h)
    assert orc.kernel_W(h, h) == 0.0 and orc.kernel_W(1.01 * h, h) == 0.0
    assert orc.kernel_W(0, h) == pytest.approx(8 / (math.pi * h ** 3), rel=1e-15)


def test_lambda_zero_distance_closed_form(orc):
    """Lambda(0; h, h) = int W^2 d^3x, derived symbolically here."""
    import sympy as sp
    r, h = sp.symbols("r h", positive=True)
    q = r / h
    w_in = 8 / (sp.pi * h ** 3) * (1 - 6 * q ** 2 + 6 * q ** 3)
    w_out = 8 / (sp.pi * h ** 3) * 2 * (1 - q) ** 3
    expr = 4 * sp.pi * (sp.integrate(r ** 2 * w_in ** 2, (r, 0, h / 2))
                        + sp.integrate(r ** 2 * w_out ** 2, (r, h / 2, h)))
    expr = sp.simplify(expr)
    assert sp.simplify(expr - sp.Rational(982, 315) / (sp.pi * h ** 3)) == 0
    for hv in (0.5, 1.0, 3.0):
        assert orc.lam(0.0, hv, hv) == pytest.approx(float(expr.subs(h, hv)), rel=1e-14)


def _lambda_cylindrical(orc, d, hi, hj):
    """Independent evaluation: int 2 pi rho W(|(rho, z)|, hi) W(|(rho, z - d)|, hj)
    over the half-plane, by adaptive 2-D quadrature."""
    def inner(z):
        f = lambda rho: 2 * math.pi * rho * orc.kernel_W(math.hypot(rho, z), hi) * \
            orc.kernel_W(math.hypot(rho, z - d), hj)
        rmax = min(math.sqrt(max(hi * hi - z * z, 0.0)), math.sqrt(max(hj * hj - (z - d) ** 2, 0.0)))
        if rmax <= 0:
            return 0.0
        return integrate.quad(f, 0, rmax, epsabs=1e-14, epsrel=1e-12, limit=200)[0]
    zlo, zhi = max(-hi, d - hj), min(hi, d + hj)
    if zlo >= zhi:
        return 0.0
    pts = sorted({p for p in (-hi / 2, hi / 2, d - hj / 2, d + hj / 2, 0.0, d) if zlo < p < zhi})
    return integrate.quad(inner, zlo, zhi, points=pts, epsabs=1e-14, epsrel=1e-11, limit=200)[0]


@pytest.mark.parametrize("d,hi,hj", [(0.25, 1.0, 1.0), (0.9, 1.0, 0.5), (0.3, 0.4, 1.1),
                                     (1.3, 1.0, 0.6), (0.05, 0.7, 0.7)])
def test_lambda_vs_cylindrical_quadrature(orc, d, hi, hj):
    ref = _lambda_cylindrical(orc, d, hi, hj)
    assert orc.lam(d, hi, hj) == pytest.approx(ref, rel=1e-8, abs=1e-12)


def test_lambda_printed_values(orc):
    """Values written out by an independent adaptive quadrature (golden file)."""
    with open(os.path.join(GOLDEN, "lambda_values.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            d, hi, hj, val = (float(t) for t in line.split())
            assert orc.lam(d, hi, hj) == pytest.approx(val, rel=2e-9, abs=1e-13)


@pytest.mark.parametrize("hi,hj", [(1.0, 1.0), (1.0, 0.5), (0.3, 0.8), (2.0, 0.1)])
def test_lambda_normalised_symmetric_supported(orc, hi, hj):
    tot = integrate.quad(lambda d: 4 * math.pi * d * d * orc.lam(d, hi, hj), 0, hi + hj,
                         points=sorted({abs(hi - hj), hi / 2, hj / 2, min(hi, hj),
                                        abs(hi / 2 - hj / 2), hi / 2 + hj / 2}),
                         limit=400, epsabs=1e-13, epsrel=1e-12)[0]
    assert abs(tot - 1.0) < 1e-9
    for d in np.linspace(0, hi + hj, 23):
        assert orc.lam(d, hi, hj) == pytest.approx(orc.lam(d, hj, hi), rel=1e-12, abs=1e-300)
    assert orc.lam(hi + hj, hi, hj) == 0.0
    assert orc.lam(1.5 * (hi + hj), hi, hj) == 0.0


def test_lambda_point_limit(orc):
    """For hj << hi the second kernel acts as a delta: Lambda -> W(d, hi)."""
    hi, hj = 1.0, 1e-3
    for d in (0.1, 0.3, 0.6, 0.8):
        assert orc.lam(d, hi, hj) == pytest.approx(orc.kernel_W(d, hi), rel=1e-5)


def test_lambda_small_distance_continuous(orc):
    for hi, hj in ((1.0, 1.0), (1.0, 0.6)):
        l0 = orc.lam(0.0, hi, hj)
        assert orc.lam(1e-7, hi, hj) == pytest.approx(l0, rel=1e-9)


# ------------------------------------------------------------------ gravity
def test_gravity_two_body_closed_form(orc):
    G, eps = 2.0, 0.3
    x = np.array([0.1, 1.3]); y = np.array([-0.2, 0.4]); z = np.array([0.5, 0.5])
    m = np.array([1.5, 0.25])
    ax, ay, az, pot = orc.gravity(x, y, z, m, G, eps)
    d = np.array([x[1] - x[0], y[1] - y[0], 0.0])
    r2 = d @ d
    s = (r2 + eps * eps) ** -1.5
    assert np.allclose([ax[0], ay[0], az[0]], G * m[1] * s * d, rtol=1e-14, atol=0)
    assert np.allclose([ax[1], ay[1], az[1]], -G * m[0] * s * d, rtol=1e-14, atol=0)
    assert pot[0] == pytest.approx(-G * m[1] / math.sqrt(r2 + eps * eps), rel=1e-14)
    assert pot[1] == pytest.approx(-G * m[0] / math.sqrt(r2 + eps * eps), rel=1e-14)


def test_gravity_momentum_and_virial(orc):
    s = W.clustered(600, seed=3)
    s["m"] = np.random.default_rng(1).uniform(0.5, 2.0, 600)
    ax, ay, az, pot = orc.gravity(s["x"], s["y"], s["z"], s["m"], 1.0, 0.01)
    for a in (ax, ay, az):
        assert abs(np.sum(s["m"] * a)) < 1e-10 * np.sum(s["m"] * np.abs(a))
    # pair-count identity: sum_i m_i phi_i = 2 W with W from an explicit pair loop
    p = np.stack([s["x"], s["y"], s["z"]], 1)
    Wpair = 0.0
    for i in range(600):
        r = np.sqrt(np.sum((p[i + 1:] - p[i]) ** 2, 1) + 1e-4)
        Wpair -= np.sum(s["m"][i] * s["m"][i + 1:] / r)
    assert np.sum(s["m"] * pot) == pytest.approx(2 * Wpair, rel=1e-12)


def test_gravity_query_subset_matches_full(orc):
    s = W.plummer(500, seed=2)
    full = orc.gravity(s["x"], s["y"], s["z"], s["m"], 1.0, 0.05)
    q = np.array([0, 7, 499, 250])
    sub = orc.gravity(s["x"], s["y"], s["z"], s["m"], 1.0, 0.05, query=q)
    for a, b in zip(full, sub):
        assert np.array_equal(a[q], b)


def test_gravity_plummer_potential(orc):
    n = 8192
    s = W.plummer(n, seed=5)
    ax, ay, az, pot = orc.gravity(s["x"], s["y"], s["z"], s["m"], 1.0, 1e-3)
    r = np.sqrt(s["x"] ** 2 + s["y"] ** 2 + s["z"] ** 2)
    # total potential energy of a Plummer sphere: -3 pi G M^2 / (32 a)
    Wtot = 0.5 * np.sum(s["m"] * pot)
    assert Wtot == pytest.approx(-3 * math.pi / 32, rel=0.03)
    # shell means of phi follow -G M / sqrt(r^2 + a^2)
    for lo, hi in ((0.3, 0.5), (0.8, 1.2), (1.5, 2.5)):
        sel = (r > lo) & (r < hi)
        assert np.mean(pot[sel]) == pytest.approx(np.mean(-1 / np.sqrt(r[sel] ** 2 + 1)), rel=0.03)
    # radial acceleration: -G M(<r) r / (r^2 + a^2)^{3/2}
    ar = (ax * s["x"] + ay * s["y"] + az * s["z"]) / r
    sel = (r > 0.8) & (r < 1.2)
    assert np.mean(ar[sel]) == pytest.approx(np.mean(-r[sel] / (r[sel] ** 2 + 1) ** 1.5), rel=0.05)


def test_gravity_truncated_nfw_potential(orc):
    n = 8192
    s = W.nfw_halo(n, seed=1)
    _, _, _, pot = orc.gravity(s["x"], s["y"], s["z"], s["m"], 1.0, 1e-3)
    r = np.sqrt(s["x"] ** 2 + s["y"] ** 2 + s["z"] ** 2)
    c = 10.0
    for lo, hi in ((0.5, 0.8), (1.5, 2.5), (4.0, 6.0)):
        sel = (r > lo) & (r < hi)
        rr = r[sel]
        expect = -4 * math.pi * (np.log1p(rr) / rr - 1 / (1 + c))
        assert np.mean(pot[sel]) == pytest.approx(np.mean(expect), rel=0.03)


# ------------------------------------------------------------------ host
def test_host_force_is_minus_gradient(orc):
    G, rho_s, r_s, c = 1.0, 2.7852, 15.3125, (1.0, -2.0, 0.5)
    rng = np.random.default_rng(0)
    pts = rng.normal(0, 40, (20, 3))
    pts[0] = [c[0] + 1e-6, c[1], c[2]]  # deep inside the series branch
    ax, ay, az, pot = orc.host_nfw(pts[:, 0], pts[:, 1], pts[:, 2], G, rho_s, r_s, c)
    for i in range(1, 20):
        h = 1e-4 * max(1.0, np.linalg.norm(pts[i] - c))
        for comp, a in enumerate((ax, ay, az)):
            e = np.zeros(3); e[comp] = h
            pp = pts[i] + e; pm = pts[i] - e
            _, _, _, fp = orc.host_nfw([pp[0]], [pp[1]], [pp[2]], G, rho_s, r_s, c)
            _, _, _, fm = orc.host_nfw([pm[0]], [pm[1]], [pm[2]], G, rho_s, r_s, c)
            assert a[i] == pytest.approx(-(fp[0] - fm[0]) / (2 * h), rel=1e-6, abs=1e-9)
    # potential matches the paper's formula and is finite at the centre
    K = 4 * math.pi * G * rho_s * r_s ** 3
    r = np.linalg.norm(pts[5] - c)
    assert pot[5] == pytest.approx(-K * math.log1p(r / r_s) / r, rel=1e-14)
    _, _, _, p0 = orc.host_nfw([c[0]], [c[1]], [c[2]], G, rho_s, r_s, c)
    assert p0[0] == pytest.approx(-K / r_s, rel=1e-14)
    # the small-radius series joins the closed form
    for s_ in (0.99e-4, 1.01e-4):
        x = [c[0] + s_ * r_s]
        a1 = orc.host_nfw(x, [c[1]], [c[2]], G, rho_s, r_s, c)[0][0]
        mu = math.log1p(s_) - s_ / (1 + s_)
        assert a1 == pytest.approx(-K * mu / (s_ * r_s) ** 2, rel=1e-9)


def test_host_circular_speed(orc):
    R = W.ORBIT_R
    ax, _, _, _ = orc.host_nfw([R], [0.0], [0.0], 1.0, W.HOST_RHO_S, W.HOST_R_S, (0, 0, 0))
    assert math.sqrt(-ax[0] * R) == pytest.approx(W.circular_speed(R), rel=1e-12)
    assert W.circular_speed(R) == pytest.approx(29.300, abs=2e-3)


# ------------------------------------------------------------------ kNN
def _lex_knn(s, k, i):
    """Brute force with numpy's lexsort on (id, d2)."""
    dx = s["x"] - s["x"][i]; dy = s["y"] - s["y"][i]; dz = s["z"] - s["z"][i]
    d2 = (dx * dx + dy * dy) + dz * dz
    order = np.lexsort((s["id"], d2))
    order = order[order != i][:k]
    return s["id"][order], d2[order]


@pytest.mark.parametrize("kind", ["random", "clustered", "lattice"])
def test_knn_brute_force(orc, kind):
    k = 16
    if kind == "random":
        s = W.maxwell_box(3000, seed=4)
    elif kind == "clustered":
        s = W.clustered(3000, seed=6)
    else:
        s = W.lattice(12, seed=2)  # many exact ties
    h, nbr = orc.knn(s["x"], s["y"], s["z"], s["id"], k, want_list=True)
    for i in range(0, s["x"].size, 97):
        ids, d2 = _lex_knn(s, k, i)
        assert np.array_equal(nbr[i], ids)
        assert h[i] == math.sqrt(d2[-1])
    # distances agree with scipy's k-d tree
    tree = cKDTree(np.stack([s["x"], s["y"], s["z"]], 1))
    dd, _ = tree.query(np.stack([s["x"], s["y"], s["z"]], 1), k=k + 1)
    assert np.allclose(h, dd[:, k], rtol=1e-14, atol=0)


def test_knn_query_subset(orc):
    s = W.clustered(2000, seed=9)
    q = np.array([3, 1999, 0, 1000])
    full = orc.knn(s["x"], s["y"], s["z"], s["id"], 32)
    sub = orc.knn(s["x"], s["y"], s["z"], s["id"], 32, query=q)
    assert np.array_equal(full[q], sub)


# ------------------------------------------------------------------ scatter
def test_events_tiny_brute_force(orc):
    """Six particles: every pair, every draw and every probability recomputed
    here from independent pieces (torch's Philox, 2-D quadrature for Lambda)."""
    import _torch_philox as T
    try:
        T.load()
    except Exception as e:  # pragma: no cover
        pytest.skip(str(e))
    rng = np.random.default_rng(11)
    n = 6
    s = dict(x=rng.uniform(0, 0.3, n), y=rng.uniform(0, 0.3, n), z=rng.uniform(0, 0.3, n),
             vx=rng.normal(0, 1, n), vy=rng.normal(0, 1, n), vz=rng.normal(0, 1, n),
             m=np.full(n, 0.5), id=np.array([9, 2, 40, 7, 13, 5], dtype=np.uint32))
    h = rng.uniform(0.1, 0.25, n)
    sigma_m, dt, seed, step = 800.0, 0.05, 77, 4
    ev, npairs, _ = orc.find_events(s["x"], s["y"], s["z"], s["vx"], s["vy"], s["vz"], s["m"],
                                    s["id"], h, sigma_m, dt, seed, step)
    expect, pairs = [], 0
    for i in range(n):
        for j in range(i + 1, n):
            d = math.dist((s["x"][i], s["y"][i], s["z"][i]), (s["x"][j], s["y"][j], s["z"][j]))
            if d >= h[i] + h[j]:
                continue
            pairs += 1
            a, b = sorted((int(s["id"][i]), int(s["id"][j])))
            w = T.block([a, b, step, 0], [seed & 0xffffffff, seed >> 32])
            u = ((w[0] << 32 | w[1]) >> 11) * 2.0 ** -53
            g = math.dist((s["vx"][i], s["vy"][i], s["vz"][i]), (s["vx"][j], s["vy"][j], s["vz"][j]))
            P = sigma_m * 0.5 * g * _lambda_cylindrical(orc, d, h[i], h[j]) * dt
            assert abs(u - P) > 1e-6 * P  # not a marginal case
            if u < P:
                expect.append((a, b))
    assert npairs == pairs and pairs >= 8
    assert [(int(e["a"]), int(e["b"])) for e in ev] == sorted(expect)
    assert 1 <= len(expect) < pairs


def test_kick_conserves_and_is_isotropic(orc):
    rng = np.random.default_rng(3)
    cos_list = []
    for t in range(4000):
        ma, mb = rng.uniform(0.5, 2, 2)
        va, vb = rng.normal(0, 1, 3), rng.normal(0, 1, 3)
        na, nb = orc.kick_pair(5, t, 1, 2, ma, mb, va, vb)
        p0, p1 = ma * va + mb * vb, ma * na + mb * nb
        assert np.allclose(p0, p1, rtol=0, atol=1e-15 * np.abs(p0).max() + 1e-15)
        e0 = 0.5 * ma * va @ va + 0.5 * mb * vb @ vb
        e1 = 0.5 * ma * na @ na + 0.5 * mb * nb @ nb
        assert abs(e1 - e0) <= 1e-14 * e0
        g = na - nb
        assert np.linalg.norm(g) == pytest.approx(np.linalg.norm(va - vb), rel=1e-13)
        cos_list.append(g / np.linalg.norm(g))
    n = np.array(cos_list)
    assert np.all(np.abs(n.mean(0)) < 4 / math.sqrt(3 * 4000))
    assert np.all(np.abs((n ** 2).mean(0) - 1 / 3) < 4 * math.sqrt(4 / 45 / 4000))


def test_events_applied_in_order(orc):
    """Sequential application in (a, b) order; a particle may scatter twice."""
    ev = np.zeros(3, dtype=orc.EVENT_DTYPE)
    ev[0] = (1, 2, 0, 1, 0.0, 0.0)
    ev[1] = (1, 3, 0, 2, 0.0, 0.0)
    ev[2] = (2, 3, 1, 2, 0.0, 0.0)
    m = np.array([1.0, 2.0, 3.0])
    v = np.random.default_rng(0).normal(0, 1, (3, 3))
    vx, vy, vz = v[:, 0].copy(), v[:, 1].copy(), v[:, 2].copy()
    orc.apply_events(ev, m, vx, vy, vz, 9, 1)
    ref = v.copy()
    for (a, b, ia, ib) in ((1, 2, 0, 1), (1, 3, 0, 2), (2, 3, 1, 2)):
        na, nb = orc.kick_pair(9, 1, a, b, m[ia], m[ib], ref[ia], ref[ib])
        ref[ia], ref[ib] = na, nb
    assert np.array_equal(np.stack([vx, vy, vz], 1), ref)


def test_scattering_rate_maxwell_box(orc):
    """Fixed h in a uniform Maxwellian box: the expected number of events per
    interior particle and step is rho (sigma/m) <|dv|> dt, <|dv|> = 4 sigma_v/sqrt(pi)."""
    n, k = 8192, 64
    s = W.maxwell_box(n, seed=21)
    rho = s["m"][0] * (n - 1)
    h = np.full(n, (k * 3 / (4 * math.pi * n)) ** (1 / 3))
    margin = 2 * h[0]
    inner = ((s["x"] > margin) & (s["x"] < 1 - margin) & (s["y"] > margin) & (s["y"] < 1 - margin)
             & (s["z"] > margin) & (s["z"] < 1 - margin))
    qmask = inner.astype(np.uint8)
    sigma_m, dt, steps = 1.0, 0.04, 8
    count = 0
    for step in range(steps):
        ev, _, _ = orc.find_events(s["x"], s["y"], s["z"], s["vx"], s["vy"], s["vz"], s["m"],
                                   s["id"], h, sigma_m, dt, 3, step, qmask=qmask)
        count += int(np.sum(inner[ev["ia"]])) + int(np.sum(inner[ev["ib"]]))
    expect = inner.sum() * steps * rho * sigma_m * 4 / math.sqrt(math.pi) * dt
    sd = math.sqrt(2 * expect)  # interior-interior events count twice
    assert abs(count - expect) < 4 * sd, (count, expect)


def test_sigma_velocity_dependence(orc):
    """Sec. 3.8 Eq. vel_dep: sigma(0) = sigma_0, sigma(w) = sigma_0 / 4, the
    (w/v)^4 tail, and w = 0 for a constant cross-section."""
    assert orc.sigma(7.0, 2.0, 0.0) == 7.0
    assert orc.sigma(7.0, 2.0, 2.0) == pytest.approx(7.0 / 4.0, rel=1e-15)
    assert orc.sigma(7.0, 2.0, 2e4) == pytest.approx(7.0 * (2.0 / 2e4) ** 4, rel=1e-7)
    assert orc.sigma(7.0, 0.0, 123.0) == 7.0


def test_scattering_rate_maxwell_box_velocity_dependent(orc):
    """As the constant-sigma rate pin, with sigma(v) = sigma_0 [1 + (v/w)^2]^-2:
    the expected number of events per interior particle and step is
    rho dt <v sigma(v)> over the Maxwellian distribution of relative speeds
    (dispersion sqrt(2) sigma_v per component), by quadrature."""
    from scipy.integrate import quad
    n, k = 8192, 64
    s = W.maxwell_box(n, seed=22)
    rho = s["m"][0] * (n - 1)
    h = np.full(n, (k * 3 / (4 * math.pi * n)) ** (1 / 3))
    margin = 2 * h[0]
    inner = ((s["x"] > margin) & (s["x"] < 1 - margin) & (s["y"] > margin) & (s["y"] < 1 - margin)
             & (s["z"] > margin) & (s["z"] < 1 - margin))
    qmask = inner.astype(np.uint8)
    sigma0, w, dt, steps = 12.0, 1.0, 0.04, 8
    sr = math.sqrt(2.0)
    fv = lambda v: math.sqrt(2 / math.pi) * v * v / sr ** 3 * math.exp(-v * v / (2 * sr * sr))
    mean_vs, _ = quad(lambda v: v * sigma0 / (1 + (v / w) ** 2) ** 2 * fv(v), 0, np.inf)
    count = 0
    for step in range(steps):
        ev, _, _ = orc.find_events(s["x"], s["y"], s["z"], s["vx"], s["vy"], s["vz"], s["m"],
                                   s["id"], h, sigma0, dt, 5, step, qmask=qmask, sigma_w=w)
        count += int(np.sum(inner[ev["ia"]])) + int(np.sum(inner[ev["ib"]]))
    expect = inner.sum() * steps * rho * mean_vs * dt
    sd = math.sqrt(2 * expect)
    assert abs(count - expect) < 4 * sd, (count, expect)
    # the constant cross-section gives the 4 sigma_v / sqrt(pi) mean for comparison
    assert mean_vs < sigma0 * 4 / math.sqrt(math.pi) * 0.5


# ------------------------------------------------------------------ step
def _two_body(orc, dt, t_end):
    s = dict(x=np.array([-0.5, 0.5]), y=np.zeros(2), z=np.zeros(2),
             vx=np.zeros(2), vy=np.array([-0.5, 0.5]) * 0.9, vz=np.zeros(2),
             m=np.array([0.5, 0.5]), id=np.array([0, 1], dtype=np.uint32))
    p = orc.make_params(eps=0.0 + 1e-9, sigma_m=0.0, dt=dt, k=1)
    orc.total_accel(s, p)
    def energy():
        return 0.5 * np.sum(s["m"] * (s["vx"] ** 2 + s["vy"] ** 2)) + 0.5 * np.sum(s["m"] * s["pot"])
    e0 = energy()
    for step in range(int(round(t_end / dt))):
        orc.kdk_step(s, p, step)
    return abs(energy() - e0) / abs(e0), s


def test_kdk_energy_error_second_order(orc):
    e1, _ = _two_body(orc, 0.02, 1.0)
    e2, _ = _two_body(orc, 0.01, 1.0)
    assert 3.0 < e1 / e2 < 5.0


def test_kdk_time_reversible(orc):
    s = W.plummer(256, seed=8)
    p = orc.make_params(eps=0.05, sigma_m=0.0, dt=0.01, k=8)
    orc.total_accel(s, p)
    x0 = np.stack([s["x"], s["y"], s["z"]]).copy()
    for step in range(32):
        orc.kdk_step(s, p, step)
    for c in ("vx", "vy", "vz"):
        s[c] = -s[c]
    for step in range(32):
        orc.kdk_step(s, p, step)
    x1 = np.stack([s["x"], s["y"], s["z"]])
    assert np.max(np.abs(x1 - x0)) < 1e-12 * np.max(np.abs(x0)) * 100


def test_kdk_step_with_scattering_conserves_momentum(orc):
    s = W.nfw_halo(2048, seed=3)
    p = orc.make_params(eps=0.01, sigma_m=200.0, dt=1e-3, k=16, seed=1)
    orc.total_accel(s, p)
    p0 = np.array([np.sum(s["m"] * s[c]) for c in ("vx", "vy", "vz")])
    ev = orc.kdk_step(s, p, 0)
    assert ev.size > 10
    p1 = np.array([np.sum(s["m"] * s[c]) for c in ("vx", "vy", "vz")])
    scale = np.sum(s["m"] * np.sqrt(s["vx"] ** 2 + s["vy"] ** 2 + s["vz"] ** 2))
    assert np.all(np.abs(p1 - p0) < 1e-12 * scale)
    # h equals the k-th neighbour distance of the drifted positions
    hk = orc.knn(s["x"], s["y"], s["z"], s["id"], 16)
    assert np.array_equal(hk, s["h"])


def test_step_parts_compose_to_the_step(orc):
    """The parts the full-size GPU tests call (kick + drift, forces, closing
    kick, the k-d tree kNN and pair search, the ordered kicks) make exactly
    orc.kdk_step, bit for bit, for a satellite in the host."""
    s0 = W.place_on_orbit(W.nfw_halo(3000, seed=9))
    p = orc.make_params(eps=0.01, sigma_m=300.0, dt=1e-3, k=24, seed=6, host=W.host_params())
    orc.total_accel(s0, p)
    a = {k: v.copy() for k, v in s0.items()}
    ev = orc.kdk_step(a, p, 4)
    b = {k: v.copy() for k, v in s0.items()}
    orc.kick_drift(b, p)
    orc.total_accel(b, p)
    orc.close_kick(b, p)
    b["h"] = orc.knn_tree(b["x"], b["y"], b["z"], b["id"], 24)
    ev2, _, _ = orc.find_events_tree(b["x"], b["y"], b["z"], b["vx"], b["vy"], b["vz"], b["m"],
                                     b["id"], b["h"], 300.0, 1e-3, 6, 4)
    orc.apply_events(ev2, b["m"], b["vx"], b["vy"], b["vz"], 6, 4)
    assert ev.size > 0 and bytes(ev) == bytes(ev2)
    for k in ("x", "y", "z", "vx", "vy", "vz", "ax", "ay", "az", "pot", "h"):
        assert np.array_equal(a[k], b[k]), k


def test_step_independent_of_thread_count(orc):
    """Every sum of the oracle belongs to one target particle and runs in a
    fixed order, so a step on one thread equals the step on all threads bit
    for bit (the CPU timing's single-thread figure times the same arithmetic)."""
    s0 = W.nfw_halo(1024, seed=4)
    p = orc.make_params(eps=0.01, sigma_m=200.0, dt=1e-3, k=16, seed=2)
    out = []
    cores = orc.num_threads()
    for threads in (1, cores):
        orc.set_threads(threads)
        try:
            s = {k: v.copy() for k, v in s0.items()}
            orc.total_accel(s, p)
            ev = orc.kdk_step(s, p, 0)
        finally:
            orc.set_threads(cores)
        out.append((s, ev))
    (a, ea), (b, eb) = out
    assert ea.size > 0 and np.array_equal(ea, eb)
    for k in ("x", "y", "z", "vx", "vy", "vz", "ax", "ay", "az", "pot", "h"):
        assert np.array_equal(a[k], b[k]), k


def test_diag_two_body(orc):
    vx, vy, vz = np.array([1.0, -1.0]), np.array([0.0, 2.0]), np.zeros(2)
    m = np.array([2.0, 3.0])
    pot = np.array([-3.0, -2.0]) + np.array([0.5, 0.25])
    pext = np.array([0.5, 0.25])
    d = orc.diag(vx, vy, vz, m, pot, pext)
    assert d["K"] == pytest.approx(0.5 * 2 * 1 + 0.5 * 3 * 5)
    assert d["W"] == pytest.approx(0.5 * (2 * -3 + 3 * -2))
    assert d["Eext"] == pytest.approx(2 * 0.5 + 3 * 0.25)
    assert (d["px"], d["py"], d["pz"]) == pytest.approx((2 - 3, 6, 0))
