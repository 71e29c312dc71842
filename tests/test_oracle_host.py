"""Pins of the oracle's Milky-Way host (Sec. 4.1: NFW halo, Hernquist bulge,
four Miyamoto-Nagai discs) and of the reflecting sphere (Sec. 2)."""
import math

import numpy as np
import pytest

import workloads as W


def _fd_grad(f, p, h):
    g = np.zeros(3)
    for c in range(3):
        e = np.zeros(3)
        e[c] = h
        g[c] = (f(p + e) - f(p - e)) / (2 * h)
    return g


def test_mw_field_is_minus_gradient(orc):
    """a = -grad Phi for the total Milky-Way field, by central differences, at
    points near the centre, near the disc plane and far out."""
    p = orc.make_params(host=W.mw_host_params())
    rng = np.random.default_rng(3)
    pts = np.concatenate([rng.normal(0, 3, (10, 3)), rng.normal(0, 60, (10, 3)),
                          np.column_stack([rng.normal(0, 4, (10, 2)), rng.normal(0, 0.02, 10)])])
    ax, ay, az, _ = orc.host_field(pts[:, 0], pts[:, 1], pts[:, 2], p)

    def phi(q):
        return orc.host_field(np.array([q[0]]), np.array([q[1]]), np.array([q[2]]), p)[3][0]
    for i, q in enumerate(pts):
        h = 1e-5 * max(0.05, abs(q[2])) if i >= 20 else 1e-5 * max(1.0, np.linalg.norm(q))
        g = _fd_grad(phi, q, h)
        a = np.array([ax[i], ay[i], az[i]])
        assert np.linalg.norm(a + g) <= 1e-6 * np.linalg.norm(a) + 1e-10, (i, a, -g)


def test_hernquist_enclosed_mass(orc):
    """Radial force of the bulge alone: G M(<r) / r^2 with M(<r) = M r^2/(r+a)^2."""
    G, M, a = 1.3, 99.6, 1.02
    r = np.array([0.01, 0.5, 1.02, 3.0, 40.0])
    u = np.array([0.6, -0.48, 0.64])
    x, y, z = r * u[0], r * u[1], r * u[2]
    ax, ay, az, pot = orc.host_hernquist(x, y, z, G, M, a, (0.0, 0.0, 0.0))
    ar = -(ax * u[0] + ay * u[1] + az * u[2])
    np.testing.assert_allclose(ar * r ** 2 / G, M * r ** 2 / (r + a) ** 2, rtol=1e-14)
    np.testing.assert_allclose(pot, -G * M / (r + a), rtol=1e-15)


def test_disk_closed_forms(orc):
    """Miyamoto-Nagai: a = 0 is the Plummer sphere of scale b; on the axis
    Phi = -GM/(a + sqrt(z^2 + b^2)); far away the potential of a point mass."""
    G, M, b = 1.0, 7.0, 0.4
    rng = np.random.default_rng(5)
    pts = rng.normal(0, 2, (20, 3))
    ax, ay, az, pot = orc.host_disk(pts[:, 0], pts[:, 1], pts[:, 2], G, M, 0.0, b, (0, 0, 0))
    r2 = np.sum(pts ** 2, 1)
    np.testing.assert_allclose(pot, -G * M / np.sqrt(r2 + b * b), rtol=1e-14)
    for c, a in enumerate((ax, ay, az)):
        np.testing.assert_allclose(a, -G * M * pts[:, c] / (r2 + b * b) ** 1.5, rtol=1e-13,
                                   atol=1e-15)
    a_d = 2.5
    zs = np.array([-3.0, -0.1, 0.2, 5.0])
    _, _, azz, pz = orc.host_disk(np.zeros(4), np.zeros(4), zs, G, M, a_d, b, (0, 0, 0))
    np.testing.assert_allclose(pz, -G * M / (a_d + np.sqrt(zs ** 2 + b * b)), rtol=1e-15)
    far = np.array([3e4, -1e4, 2e4])
    _, _, _, pf = orc.host_disk(far[:1], far[1:2], far[2:], G, M, a_d, b, (0, 0, 0))
    assert pf[0] == pytest.approx(-G * M / np.linalg.norm(far), rel=1e-3)


def test_mw_circular_speed_plausible(orc):
    """The model's circular speed in the disc plane at 8 kpc lies between 180
    and 260 km/s (the solar neighbourhood of a Milky-Way model)."""
    p = orc.make_params(host=W.mw_host_params())
    R = 8.0 * W.KPC
    ax, _, _, _ = orc.host_field(np.array([R]), np.zeros(1), np.zeros(1), p)
    vc = math.sqrt(-ax[0] * R) / W.KMS
    assert 180.0 < vc < 260.0, vc


def test_reflecting_sphere(orc):
    """Without forces (G = 0): beyond the radius, outward motion has its radial
    component reversed (|v| and the tangential part kept); inward motion and
    particles inside are untouched."""
    s = dict(x=np.array([5.0, 5.0, 1.0, -0.2]), y=np.array([0.0, 0.1, 0.0, 4.9]),
             z=np.zeros(4), vx=np.array([1.0, -1.0, 1.0, 0.3]), vy=np.array([0.5, 0.0, 0.0, 2.0]),
             vz=np.array([0.0, 0.2, 0.0, -0.4]), m=np.full(4, 1.0),
             id=np.arange(4, dtype=np.uint32))
    p = orc.make_params(G=0.0, eps=0.1, sigma_m=0.0, dt=0.01, k=1,
                        boundary=dict(r=4.0, center=(0.0, 0.0, 0.0)))
    orc.total_accel(s, p)
    v0 = np.stack([s["vx"], s["vy"], s["vz"]], 1).copy()
    orc.kdk_step(s, p, 0)
    x1 = np.stack([s["x"], s["y"], s["z"]], 1)
    v1 = np.stack([s["vx"], s["vy"], s["vz"]], 1)
    n = x1 / np.linalg.norm(x1, axis=1)[:, None]
    # 0: outside, outwards -> reflected
    assert np.dot(v1[0], n[0]) == pytest.approx(-np.dot(v0[0], n[0]), rel=1e-14)
    assert np.linalg.norm(v1[0]) == pytest.approx(np.linalg.norm(v0[0]), rel=1e-15)
    t0 = v0[0] - np.dot(v0[0], n[0]) * n[0]
    t1 = v1[0] - np.dot(v1[0], n[0]) * n[0]
    np.testing.assert_allclose(t1, t0, atol=1e-14)
    # 1: outside, inwards; 2: inside -> unchanged
    assert np.array_equal(v1[1], v0[1]) and np.array_equal(v1[2], v0[2])
    # 3: outside (r = 4.9), outwards -> reflected
    assert np.dot(v1[3], n[3]) < 0 < np.dot(v0[3], n[3])


def _compact_satellite(n, R, D, seed):
    rng = np.random.default_rng(seed)
    u = rng.normal(size=(n, 3))
    u *= (R * rng.uniform(0, 1, n) ** (1 / 3) / np.linalg.norm(u, axis=1))[:, None]
    return dict(x=u[:, 0] + D, y=u[:, 1], z=u[:, 2], m=np.full(n, 1.0 / n))


def test_tidal_radius_compact_satellite(orc):
    """A satellite of unit mass inside R = 0.01 at D = 50 from a Hernquist host
    (M = 1e4, a = 1), with six marker particles of negligible mass at distance 5
    that set the search range: r_t solves
    G/r^2 = G M (1/(D - r + a)^2 - 1/(D + r + a)^2), found independently by root
    bracketing on the closed form."""
    from scipy.optimize import brentq
    M, a, D = 1.0e4, 1.0, 50.0
    s = _compact_satellite(2000, 0.01, D, 7)
    mk = np.array([[5, 0, 0], [-5, 0, 0], [0, 5, 0], [0, -5, 0], [0, 0, 5], [0, 0, -5]], float)
    for c, k in zip("xyz", range(3)):
        s[c] = np.concatenate([s[c], mk[:, k] + (D if c == "x" else 0.0)])
    s["m"] = np.concatenate([s["m"], np.full(6, 1e-300)])
    _, _, _, pot = orc.gravity(s["x"], s["y"], s["z"], s["m"], 1.0, 1e-3)
    host = dict(rho_s=0.0, r_s=1.0, center=(0.0, 0.0, 0.0), hern=(M, a), disks=[])
    p = orc.make_params(host=host)
    r_t, mass, c, st = orc.tidal_radius(s["x"], s["y"], s["z"], s["m"], pot, p)
    xc = np.array([s["x"][c], s["y"][c], s["z"][c]])
    Dc = np.linalg.norm(xc)
    f = lambda r: 1.0 / r ** 2 - M * (1.0 / (Dc - r + a) ** 2 - 1.0 / (Dc + r + a) ** 2)
    ref = brentq(f, 0.05, 20.0, xtol=1e-15, rtol=1e-15)
    assert st == 0
    assert r_t == pytest.approx(ref, rel=1e-10)
    assert mass == pytest.approx(1.0, rel=1e-14)
    assert 1.0 < r_t < 2.0
    assert np.hypot(s["y"][c], s["z"][c]) < 0.01


def test_tidal_radius_no_crossing(orc):
    """A host too light to strip anything within twice the satellite's extent."""
    s = _compact_satellite(500, 0.5, 100.0, 8)
    _, _, _, pot = orc.gravity(s["x"], s["y"], s["z"], s["m"], 1.0, 1e-3)
    host = dict(rho_s=0.0, r_s=1.0, center=(0.0, 0.0, 0.0), hern=(1e-3, 1.0), disks=[])
    r_t, mass, c, st = orc.tidal_radius(s["x"], s["y"], s["z"], s["m"], pot,
                                       orc.make_params(host=host))
    assert st == 1 and mass == pytest.approx(1.0, rel=1e-14)
