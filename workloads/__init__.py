"""Seeded synthetic inputs for the SIDM N-body step.

This module only builds initial conditions and run parameters; it holds none
of the step's arithmetic (no forces, neighbour search, overlap integral or
scattering) so that both the GPU library and the CPU oracle can be fed the same
bits without sharing any of the computation they are compared on.

Units: G = r_s = rho_s = 1 for the halo (the paper's NFW satellite of Sec. 2,
rho_0 = 4.42e7 Msun/kpc^3, r_s = 1.28 kpc).  Randomness: numpy PCG64 streams
seeded by the workload seed.

Workloads (the paper's halo at the sizes used for testing and timing):
  C1  isolated NFW, N = 8192, eps 0.01, sigma/m 1, k 32, dt 1e-3, FP64
  C2  NFW N = 2^20 on a circular orbit in a static NFW host, k 64, sigma/m 10
  C3  C2's halo, FP64 vs mixed precision, with an N = 2^16 oracle companion
  C4  64 independent halos, N log-uniform in 2^12..2^17, mixed sigma/m and k
  C5  NFW N = 2^24, eps 0.002, k 64, sigma/m 10, in the host
  BLK isolated NFW N = 2^20 with block time steps (eta 0.025, cycles of 1/16
      in up to 2^6 ticks), sigma/m 1, k 64
"""
import math

import numpy as np

FOUR_PI = 4.0 * math.pi


# ----------------------------------------------------------------- NFW halo
def nfw_mass(r):
    """Enclosed mass of rho = 1/(r (1+r)^2) (G = r_s = rho_s = 1)."""
    r = np.asarray(r, dtype=np.float64)
    return FOUR_PI * (np.log1p(r) - r / (1.0 + r))


def _nfw_rho(r):
    return 1.0 / (r * (1.0 + r) ** 2)


def _nfw_psi(r, c):
    """Relative potential of the NFW profile truncated sharply at c (zero at c)."""
    return FOUR_PI * (np.log1p(r) / r - math.log1p(c) / c)


class _Eddington:
    """Isotropic distribution function of the sharply truncated NFW halo."""

    def __init__(self, c=10.0, n_r=6000, n_e=600):
        self.c = c
        r = np.logspace(-7, math.log10(c), n_r)
        self.r = r
        self.psi = _nfw_psi(r, c)
        self.psi0 = FOUR_PI * (1.0 - math.log1p(c) / c)
        # derivatives of rho with respect to psi through r
        M = nfw_mass(r)
        dpsi = -M / r ** 2
        ddpsi = -FOUR_PI * _nfw_rho(r) + 2.0 * M / r ** 3
        drho = -(1.0 + 3.0 * r) / (r ** 2 * (1.0 + r) ** 3)
        ddrho = (2.0 + 8.0 * r + 12.0 * r ** 2) / (r ** 3 * (1.0 + r) ** 4)
        self.d1 = drho / dpsi
        self.d2 = (ddrho * dpsi - drho * ddpsi) / dpsi ** 3
        # boundary term (d rho / d psi at psi = 0, i.e. r = c)
        self.d1_edge = float(self.d1[-1])
        # f(E) on a log grid of binding energies joined with E = psi(r) on a
        # log grid of radii, which resolves the steep rise of f towards psi0
        # (the cusp) where a log grid in E alone is far too coarse
        E = np.unique(np.concatenate([
            self.psi0 * np.logspace(-10, math.log10(0.999999), n_e),
            _nfw_psi(np.logspace(-6, math.log10(c), 2 * n_e), c)[:-1]]))
        E = E[(E > 0.0) & (E < self.psi0)]
        tg, tw = np.polynomial.legendre.leggauss(400)
        f = np.empty_like(E)
        lr_of_psi_x = self.psi[::-1]
        lr_of_psi_y = np.log(self.r[::-1])
        d2_sorted = self.d2[::-1]
        for k, e in enumerate(E):
            # int_0^E d2 dpsi / sqrt(E - psi) with psi = E - t^2
            tmax = math.sqrt(e)
            t = 0.5 * tmax * (tg + 1.0)
            ps = e - t * t
            val = np.interp(ps, lr_of_psi_x, d2_sorted)
            integral = np.sum(tw * 2.0 * val) * 0.5 * tmax
            f[k] = (integral + self.d1_edge / math.sqrt(e)) / (math.sqrt(8.0) * math.pi ** 2)
        self.E = E
        self.f = np.maximum(f, 0.0)
        self._logE = np.log(E)
        self._logf = np.log(np.maximum(self.f, 1e-300))
        # inverse cumulative distribution of the speed at radius r: with
        # v = q sqrt(2 psi(r)), the density of q is q^2 f(psi (1 - q^2)); rows
        # are tabulated on a log grid of r (fine where psi approaches psi0 in
        # the cusp) and columns on s = u^(1/3) (u uniform), which keeps the
        # q ~ u^(1/3) start of every row resolved
        self._inv_logr = np.linspace(math.log(1e-6), math.log(c), 2048)
        pg = _nfw_psi(np.exp(self._inv_logr), c)
        q = np.linspace(0.0, 1.0, 4097)
        dens = q[None, :] ** 2 * self.df(pg[:, None] * (1.0 - q[None, :] ** 2))
        cdf = np.concatenate([np.zeros((pg.size, 1)),
                              np.cumsum(0.5 * (dens[:, 1:] + dens[:, :-1]), axis=1)], axis=1)
        tot = cdf[:, -1].copy()
        cdf /= np.where(tot > 0.0, tot, 1.0)[:, None]
        sg = np.linspace(0.0, 1.0, 1025)
        self._inv_q = np.empty((pg.size, sg.size))
        for k in range(pg.size):
            if tot[k] > 0.0:
                # cumsum of non-negative terms is non-decreasing, as np.interp needs
                self._inv_q[k] = np.interp(sg ** 3, cdf[k], q)
            else:
                self._inv_q[k] = sg
        self._inv_ns = sg.size - 1

    def df(self, e):
        e = np.asarray(e, dtype=np.float64)
        out = np.exp(np.interp(np.log(np.maximum(e, 1e-300)), self._logE, self._logf,
                               left=-700.0))
        return np.where(e > 0.0, out, 0.0)

    def speed_fraction(self, r, u):
        """q = v / sqrt(2 psi(r)) for uniform u in [0, 1): bilinear lookup of
        the inverse cumulative table in (log r, u^(1/3))."""
        lr = np.log(np.maximum(r, 1e-300))
        t = (lr - self._inv_logr[0]) / (self._inv_logr[1] - self._inv_logr[0])
        t = np.clip(t, 0.0, self._inv_logr.size - 1.000001)
        k = t.astype(np.int64)
        ft = t - k
        sc = np.cbrt(u) * self._inv_ns
        j = np.minimum(sc.astype(np.int64), self._inv_ns - 1)
        fs = sc - j
        Q = self._inv_q
        lo = Q[k, j] * (1.0 - fs) + Q[k, j + 1] * fs
        hi = Q[k + 1, j] * (1.0 - fs) + Q[k + 1, j + 1] * fs
        return lo * (1.0 - ft) + hi * ft


_EDD_CACHE = {}


def _eddington(c):
    if c not in _EDD_CACHE:
        _EDD_CACHE[c] = _Eddington(c)
    return _EDD_CACHE[c]


def _isotropic(rng, n):
    cz = rng.uniform(-1.0, 1.0, n)
    ph = rng.uniform(0.0, 2.0 * math.pi, n)
    s = np.sqrt(np.maximum(0.0, 1.0 - cz * cz))
    return s * np.cos(ph), s * np.sin(ph), cz


def nfw_halo(n, seed=0, r_cut=10.0):
    """Equal-mass NFW halo truncated at r_cut, velocities from Eddington
    inversion, centre of mass and bulk velocity removed.

    Returns a dict with x, y, z, vx, vy, vz, m (float64) and id (uint32)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    edd = _eddington(float(r_cut))
    Mc = float(nfw_mass(r_cut))
    # radii by inverting M(r)/M(c) on a fine table
    rt = np.logspace(-8, math.log10(r_cut), 200001)
    Mt = nfw_mass(rt) / Mc
    r = np.interp(rng.uniform(0.0, 1.0, n), Mt, rt)
    psi = _nfw_psi(r, r_cut)
    # speeds from the inverse cumulative distribution of v^2 f(psi - v^2/2)
    v = np.sqrt(2.0 * np.maximum(psi, 0.0)) * edd.speed_fraction(r, rng.uniform(0.0, 1.0, n))
    ux, uy, uz = _isotropic(rng, n)
    wx, wy, wz = _isotropic(rng, n)
    s = dict(x=r * ux, y=r * uy, z=r * uz, vx=v * wx, vy=v * wy, vz=v * wz)
    for a in ("x", "y", "z", "vx", "vy", "vz"):
        s[a] = s[a] - s[a].mean()
    s["m"] = np.full(n, Mc / n)
    s["id"] = np.arange(n, dtype=np.uint32)
    return s


# ----------------------------------------------------------------- other inputs
def plummer(n, seed=0, a=1.0, M=1.0):
    """Plummer sphere (G = 1) with isotropic velocities (Aarseth, Henon &
    Wielen 1974 sampling); centre of mass removed."""
    rng = np.random.Generator(np.random.PCG64(seed))
    X = rng.uniform(1e-10, 1.0, n)
    r = a / np.sqrt(X ** (-2.0 / 3.0) - 1.0)
    q = np.zeros(n)
    todo = np.arange(n)
    while todo.size:
        x = rng.uniform(0.0, 1.0, todo.size)
        y = rng.uniform(0.0, 0.1, todo.size)
        ok = y < x * x * (1.0 - x * x) ** 3.5
        q[todo[ok]] = x[ok]
        todo = todo[~ok]
    v = q * np.sqrt(2.0 * M) * (r * r + a * a) ** -0.25 / math.sqrt(a)
    ux, uy, uz = _isotropic(rng, n)
    wx, wy, wz = _isotropic(rng, n)
    s = dict(x=r * ux, y=r * uy, z=r * uz, vx=v * wx, vy=v * wy, vz=v * wz)
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        s[k] = s[k] - s[k].mean()
    s["m"] = np.full(n, M / n)
    s["id"] = np.arange(n, dtype=np.uint32)
    return s


def maxwell_box(n, seed=0, L=1.0, sigma_v=1.0, mass=None):
    """Uniform positions in [0, L)^3, Gaussian velocities of dispersion sigma_v
    per component, equal masses summing to 1 unless `mass` is given."""
    rng = np.random.Generator(np.random.PCG64(seed))
    s = dict(x=rng.uniform(0.0, L, n), y=rng.uniform(0.0, L, n), z=rng.uniform(0.0, L, n),
             vx=rng.normal(0.0, sigma_v, n), vy=rng.normal(0.0, sigma_v, n),
             vz=rng.normal(0.0, sigma_v, n))
    s["m"] = np.full(n, (1.0 / n) if mass is None else float(mass))
    s["id"] = np.arange(n, dtype=np.uint32)
    return s


def lattice(nside, spacing=1.0, seed=0, shuffle=True):
    """Cubic lattice of nside^3 points: many exactly equal distances (ties).
    Ids are shuffled so that tie-breaking by id is exercised."""
    g = np.arange(nside, dtype=np.float64) * spacing
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    n = nside ** 3
    rng = np.random.Generator(np.random.PCG64(seed))
    ids = rng.permutation(n).astype(np.uint32) if shuffle else np.arange(n, dtype=np.uint32)
    return dict(x=X.ravel().copy(), y=Y.ravel().copy(), z=Z.ravel().copy(),
                vx=rng.normal(0, 1, n), vy=rng.normal(0, 1, n), vz=rng.normal(0, 1, n),
                m=np.full(n, 1.0 / n), id=ids)


def clustered(n, seed=0, n_clumps=8, width=0.02):
    """Gaussian clumps in a unit box: strong density contrast."""
    rng = np.random.Generator(np.random.PCG64(seed))
    centres = rng.uniform(0.0, 1.0, (n_clumps, 3))
    which = rng.integers(0, n_clumps, n)
    p = centres[which] + rng.normal(0.0, width, (n, 3))
    return dict(x=p[:, 0].copy(), y=p[:, 1].copy(), z=p[:, 2].copy(),
                vx=rng.normal(0, 1, n), vy=rng.normal(0, 1, n), vz=rng.normal(0, 1, n),
                m=np.full(n, 1.0 / n), id=rng.permutation(n).astype(np.uint32))


# ----------------------------------------------------------------- host orbit
# Static NFW host.  Reading of "M_host / M_halo = 1e4": rho_s,h r_s,h^3 = 1e4
# (same-concentration masses), with the paper's host/satellite scale-radius
# ratio r_s,h = 19.6 kpc / 1.28 kpc (Sec. 4.1 and Sec. 2).  The satellite is
# placed on a circular orbit at 20 r_s,h.
HOST_R_S = 19.6 / 1.28
HOST_RHO_S = 1.0e4 / HOST_R_S ** 3
ORBIT_R = 20.0 * HOST_R_S


def host_params():
    return dict(rho_s=HOST_RHO_S, r_s=HOST_R_S, center=(0.0, 0.0, 0.0))


def circular_speed(R, rho_s=HOST_RHO_S, r_s=HOST_R_S, G=1.0):
    """Circular speed in the static host, sqrt(G M_h(<R) / R)."""
    Mh = rho_s * r_s ** 3 * nfw_mass(R / r_s)
    return math.sqrt(G * float(Mh) / R)


def place_on_orbit(s, R=ORBIT_R):
    s = dict(s)
    s["x"] = s["x"] + R
    s["vy"] = s["vy"] + circular_speed(R)
    return s


# ----------------------------------------------------------------- Milky-Way host
# Code units of the satellite (Sec. 2): length r_s = 1.28 kpc, density
# rho_0 = 4.42e7 Msun/kpc^3, G = 1, hence mass rho_0 r_s^3 and velocity
# sqrt(G rho_0 r_s^2) with G = 4.30091e-6 kpc (km/s)^2 / Msun.
KPC = 1.0 / 1.28
MSUN = 1.0 / (4.42e7 * 1.28 ** 3)
KMS = 1.0 / math.sqrt(4.30091e-6 * 4.42e7 * 1.28 ** 2)


def mw_host_params():
    """The Milky-Way host of Sec. 4.1 in code units: NFW halo (rho_s, r_s),
    Hernquist bulge (M, a) and four Miyamoto-Nagai discs (M, a, b): thin and
    thick stellar, thin and thick gas."""
    disks = [(3.52e10, 2.5, 0.3), (1.05e10, 3.02, 0.9), (1.2e9, 1.5, 0.045), (1.1e10, 7.0, 0.085)]
    return dict(rho_s=8.54e6 * MSUN / KPC ** 3, r_s=19.6 * KPC, center=(0.0, 0.0, 0.0),
                hern=(9.23e9 * MSUN, 1.3 * KPC),
                disks=[(M * MSUN, a * KPC, b * KPC) for M, a, b in disks])


def place_on_mw_orbit(s):
    """The satellite's initial position and velocity of Sec. 4.1 relative to
    the Milky-Way host's centre."""
    s = dict(s)
    for c, (x, v) in zip("xyz", zip((58.16, 40.12, 101.41), (45.94, 83.42, 53.12))):
        s[c] = s[c] + x * KPC
        s["v" + c] = s["v" + c] + v * KMS
    return s


def mw_boundary():
    """The reflecting sphere of Sec. 2: 200 kpc about the host centre."""
    return dict(r=200.0 * KPC, center=(0.0, 0.0, 0.0))


# ----------------------------------------------------------------- configs
NFW_MASS_10 = float(nfw_mass(10.0))


def config(name):
    """Run parameters of the named workload (C1..C5, BLK)."""
    base = dict(G=1.0, eps=0.01, dt=1e-3, r_cut=10.0, seed=0)
    if name == "C1":
        return dict(base, name=name, n=8192, sigma_m=1.0, k=32, steps=32, precision="fp64",
                    host=None)
    if name == "C2":
        return dict(base, name=name, n=1 << 20, sigma_m=10.0, k=64, steps=100,
                    precision="mixed", host=host_params())
    if name == "C3":
        return dict(base, name=name, n=1 << 20, sigma_m=10.0, k=64, steps=1000,
                    precision="both", host=host_params(), oracle_n=1 << 16)
    if name == "C5":
        return dict(base, name=name, n=1 << 24, eps=0.002, sigma_m=10.0, k=64, steps=1,
                    precision="mixed", host=host_params())
    if name == "BLK":
        # Table 1's gravitational step parameter eta = 0.025 with a cycle of
        # 1/16 (about 4.4 Myr in the code units of the workloads) whose deepest
        # bin, 1/1024, is about the fixed step of C1..C5
        return dict(base, name=name, n=1 << 20, dt=1.0 / 16, sigma_m=1.0, k=64, steps=4,
                    precision="mixed", host=None, steps_param=dict(eta=0.025, max_bin=6))
    raise KeyError(name)


def batch_c4():
    """64 halos, b = 0..63: N_b = 64 round(2^(12 + 5b/63) / 64), sigma/m from
    {1, 10, 50}[b mod 3], k from {16, 32, 64, 128}[b mod 4], seed b."""
    halos = []
    for b in range(64):
        nb = 64 * int(round(2.0 ** (12.0 + 5.0 * b / 63.0) / 64.0))
        halos.append(dict(n=nb, sigma_m=(1.0, 10.0, 50.0)[b % 3], k=(16, 32, 64, 128)[b % 4],
                          seed=b, G=1.0, eps=0.01, dt=1e-3, host=None))
    return halos


def make_state(cfg, n=None, seed=None):
    """Initial conditions for a config dict (satellite placed on its orbit when
    the config has a host)."""
    n = cfg["n"] if n is None else n
    s = nfw_halo(n, cfg.get("seed", 0) if seed is None else seed, cfg.get("r_cut", 10.0))
    if cfg.get("host") is not None:
        s = place_on_orbit(s)
    return s
