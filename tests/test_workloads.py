"""Sanity of the synthetic initial conditions (the NFW satellite of Sec. 2,
truncated sharply at 10 r_s, velocities from the isotropic distribution
function by Eddington's inversion): radii follow the profile's enclosed mass,
the radial dispersion follows the Jeans equation, the virial ratio is the one
these velocities imply, and without scattering the mass profile holds over a
dynamical time.  The profile's formulas are restated here from the definition
rho = rho_s / (x (1 + x)^2), x = r / r_s, in units G = r_s = rho_s = 1.

A sharp edge has no non-negative isotropic distribution function: the density
jump at the edge would need f < 0 near zero binding energy.  Eddington's
inversion without that term, as the generator does it, reproduces
rho - rho(r_cut) instead of rho, in the potential of the whole truncated
halo, so the velocities are those of the Jeans solution for rho - rho(r_cut):
within 2 % of the equilibrium dispersion inside r_s (where rho(r_cut) / rho
< 0.4 %), 5 % low at 2 r_s, 20 % low at 5 r_s, and 2K/|W| = 0.90 overall.
The tests pin that property."""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import workloads as W

C = 10.0   # truncation radius in r_s


def _mass(r):
    """Enclosed mass: 4 pi [ln(1 + r) - r / (1 + r)]."""
    return 4.0 * math.pi * (math.log1p(r) - r / (1.0 + r))


def _rho(r):
    return 1.0 / (r * (1.0 + r) ** 2)


def _radii(s):
    return np.sqrt(s["x"] ** 2 + s["y"] ** 2 + s["z"] ** 2)


def test_nfw_radii_follow_the_enclosed_mass():
    s = W.nfw_halo(20000, seed=3)
    r = _radii(s)
    # radii from the centre of mass, which the generator moves to the origin
    # (a shift of order C / sqrt(n))
    assert r.max() <= C + 0.2
    cdf = np.vectorize(lambda x: _mass(min(max(x, 0.0), C)) / _mass(C))
    res = stats.kstest(r, cdf)
    assert res.pvalue > 1e-3, res
    # total mass is the truncated profile's
    assert np.sum(s["m"]) == pytest.approx(_mass(C), rel=1e-12)


def _pressure(x, edge):
    """int_x^C (rho(r) - edge) M(r) / r^2 dr."""
    return integrate.quad(lambda y: (_rho(y) - edge) * _mass(y) / y ** 2, x, C, limit=200)[0]


def test_nfw_radial_dispersion_follows_jeans():
    """sigma_r^2 = pressure / density of rho - rho(C), averaged over each
    radial bin with the bin's number density rho r^2; inside r_s also the
    equilibrium dispersion of rho itself."""
    s = W.nfw_halo(400000, seed=4)
    r = _radii(s)
    vr = (s["x"] * s["vx"] + s["y"] * s["vy"] + s["z"] * s["vz"]) / r
    edge = _rho(C)
    for r0 in (0.3, 1.0, 2.16, 5.0, 8.0):
        lo, hi = r0 / 1.15, r0 * 1.15
        sel = (r > lo) & (r < hi)
        assert sel.sum() > 3000
        xs = np.linspace(lo, hi, 41)
        w = np.array([_rho(x) * x * x for x in xs])
        dfj = float(np.sum(w * np.array([_pressure(x, edge) / (_rho(x) - edge) for x in xs]))
                    / np.sum(w))
        eqj = float(np.sum(w * np.array([_pressure(x, 0.0) / _rho(x) for x in xs])) / np.sum(w))
        got = float(np.mean(vr[sel] ** 2))
        print(f"r = {r0}: sigma_r^2 {got:.4f}, Jeans of rho - rho(C) {dfj:.4f}, of rho {eqj:.4f} "
              f"({sel.sum()} particles)")
        assert got == pytest.approx(dfj, rel=0.04)
        if r0 <= 1.0:
            assert got == pytest.approx(eqj, rel=0.04)


def test_nfw_virial_ratio(orc):
    """2K/|W| of a sample against the ratio the velocities imply:
    K = 3/2 int rho p~ / rho~ dV with rho~ = rho - rho(C) and p~ its Jeans
    pressure, W = -int rho M / r dV (0.896; an equilibrium would give 1)."""
    edge = _rho(C)
    K = 1.5 * integrate.quad(lambda x: _rho(x) * _pressure(x, edge) / (_rho(x) - edge)
                             * 4.0 * math.pi * x * x, 1e-8, C * (1 - 1e-9), limit=400)[0]
    Wth = -integrate.quad(lambda x: _rho(x) * _mass(x) / x * 4.0 * math.pi * x * x, 0.0, C,
                          limit=200)[0]
    expect = 2.0 * K / abs(Wth)
    s = W.nfw_halo(8192, seed=5)
    _, _, _, pot = orc.gravity(s["x"], s["y"], s["z"], s["m"], 1.0, 1e-3)
    Ks = 0.5 * np.sum(s["m"] * (s["vx"] ** 2 + s["vy"] ** 2 + s["vz"] ** 2))
    Ws = 0.5 * np.sum(s["m"] * pot)
    print(f"2K/|W| = {2 * Ks / abs(Ws):.4f}, implied {expect:.4f}; W {Ws:.4f} against {Wth:.4f}")
    assert Ws == pytest.approx(Wth, rel=0.03)
    assert 2 * Ks / abs(Ws) == pytest.approx(expect, rel=0.03)


def test_nfw_profile_holds_without_scattering(orc):
    """sigma = 0, the C1 set-up (N = 8192, eps = 0.01, dt = 1e-3): over its 32
    steps the enclosed mass at 0.3, 1 and 3 r_s changes by no more than 3 %
    plus twice the Poisson spread of the particles crossing each shell."""
    n = 8192
    s = W.nfw_halo(n, seed=0)
    p = orc.make_params(eps=0.01, sigma_m=0.0, dt=1e-3, k=32, seed=0)
    orc.total_accel(s, p)
    r0 = _radii(s)
    for step in range(32):
        orc.kdk_step(s, p, step)
    r1 = _radii(s)
    for R in (0.3, 1.0, 3.0):
        m0, m1 = int(np.sum(r0 < R)), int(np.sum(r1 < R))
        print(f"M(<{R}): {m0} -> {m1}")
        assert abs(m1 - m0) <= 0.03 * m0 + 2.0 * math.sqrt(m0)
