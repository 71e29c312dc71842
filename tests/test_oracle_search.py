"""Pins of the oracle's exact accelerated searches and of its central density.

The grid kNN, the k-d tree kNN, the x-sorted pair sweep and the k-d tree pair
search must return exactly what the brute-force definitions return (h and
neighbour lists bit for bit; the same events, pair count and P > 1 count) on
inputs with ties, duplicates, flat and clustered geometry.
The central density is checked on configurations whose answer is known by
construction (Sec. 3: the centre is the potential minimum)."""
import math

import numpy as np
import pytest

import workloads as W


def _dup(base, copies, seed):
    s = {f: np.concatenate([base[f]] * copies) for f in ("x", "y", "z", "vx", "vy", "vz", "m")}
    s["id"] = np.random.default_rng(seed).permutation(s["x"].size).astype(np.uint32)
    return s


def _flat(n, seed):
    s = W.maxwell_box(n, seed=seed)
    s["z"] = np.zeros(n)
    return s


CASES = [
    ("nfw", lambda: W.nfw_halo(6000, seed=3), (1, 32, 64)),
    ("lattice", lambda: W.lattice(9, seed=1), (1, 6, 18, 26)),
    ("clustered", lambda: W.clustered(3000, seed=2), (16, 64)),
    ("duplicates", lambda: _dup(W.maxwell_box(300, seed=4), 3, 5), (1, 2, 5)),
    ("flat", lambda: _flat(1500, 6), (8, 40)),
    ("pair", lambda: W.maxwell_box(2, seed=7), (1,)),
]


@pytest.mark.parametrize("name,make,ks", CASES, ids=[c[0] for c in CASES])
def test_knn_grid_equals_brute_force(orc, name, make, ks):
    s = make()
    for k in ks:
        hb = orc.knn(s["x"], s["y"], s["z"], s["id"], k)
        hg = orc.knn_grid(s["x"], s["y"], s["z"], s["id"], k)
        assert np.array_equal(hb, hg), (name, k)


@pytest.mark.parametrize("name,make,ks", CASES, ids=[c[0] for c in CASES])
def test_knn_tree_equals_brute_force(orc, name, make, ks):
    s = make()
    for k in ks:
        hb, lb = orc.knn(s["x"], s["y"], s["z"], s["id"], k, want_list=True)
        ht, lt = orc.knn_tree(s["x"], s["y"], s["z"], s["id"], k, want_list=True)
        assert np.array_equal(hb, ht), (name, k)
        assert np.array_equal(lb, lt), (name, k)


@pytest.mark.parametrize("name,make,ks", CASES, ids=[c[0] for c in CASES])
def test_event_tree_equals_brute_force(orc, name, make, ks):
    """Also with a velocity-dependent cross-section, and at sigma/m large
    enough for pairs with P > 1 (where the bound that spares the overlap
    integral exceeds 1 and never applies)."""
    s = make()
    k = max(ks)
    h = orc.knn(s["x"], s["y"], s["z"], s["id"], k)
    for sigma, w, seed, step in ((1.0, 0.0, 0, 0), (300.0, 0.0, 3, 7), (5e4, 0.0, 9, 2),
                                 (2e3, 0.3, 4, 5)):
        ref = orc.find_events(s["x"], s["y"], s["z"], s["vx"], s["vy"], s["vz"], s["m"],
                              s["id"], h, sigma, 1e-3, seed, step, sigma_w=w)
        got = orc.find_events_tree(s["x"], s["y"], s["z"], s["vx"], s["vy"], s["vz"], s["m"],
                                   s["id"], h, sigma, 1e-3, seed, step, sigma_w=w)
        assert got[1] == ref[1] and got[2] == ref[2], (name, sigma)
        assert bytes(got[0]) == bytes(ref[0]), (name, sigma)


def test_event_tree_counts_p_above_one(orc):
    """A case where pairs with P > 1 exist, so the P > 1 count is pinned."""
    s = W.clustered(1500, seed=8)
    h = orc.knn(s["x"], s["y"], s["z"], s["id"], 16)
    ref = orc.find_events(s["x"], s["y"], s["z"], s["vx"], s["vy"], s["vz"], s["m"], s["id"], h,
                          3e6, 1e-2, 2, 3)
    got = orc.find_events_tree(s["x"], s["y"], s["z"], s["vx"], s["vy"], s["vz"], s["m"],
                               s["id"], h, 3e6, 1e-2, 2, 3)
    assert ref[2] > 0
    assert got[1:] == ref[1:] and bytes(got[0]) == bytes(ref[0])


@pytest.mark.parametrize("name,make,ks", CASES, ids=[c[0] for c in CASES])
def test_event_sweep_equals_brute_force(orc, name, make, ks):
    s = make()
    k = max(ks)
    h = orc.knn(s["x"], s["y"], s["z"], s["id"], k)
    for sigma, seed, step in ((1.0, 0, 0), (300.0, 3, 7), (5e4, 9, 2)):
        ref = orc.find_events(s["x"], s["y"], s["z"], s["vx"], s["vy"], s["vz"], s["m"],
                              s["id"], h, sigma, 1e-3, seed, step)
        got = orc.find_events_sweep(s["x"], s["y"], s["z"], s["vx"], s["vy"], s["vz"], s["m"],
                                    s["id"], h, sigma, 1e-3, seed, step)
        assert got[1] == ref[1] and got[2] == ref[2], (name, sigma)
        assert bytes(got[0]) == bytes(ref[0]), (name, sigma)


def test_event_sweep_equal_kernel_sizes(orc):
    """All h equal (the tie rule of the sweep decides which member finds a pair)."""
    s = W.lattice(8, seed=3)
    h = np.full(s["x"].size, 1.01)
    ref = orc.find_events(s["x"], s["y"], s["z"], s["vx"], s["vy"], s["vz"], s["m"], s["id"], h,
                          2e3, 1e-3, 1, 1)
    got = orc.find_events_sweep(s["x"], s["y"], s["z"], s["vx"], s["vy"], s["vz"], s["m"],
                                s["id"], h, 2e3, 1e-3, 1, 1)
    # lattice pairs closer than 2.02: distances 1, sqrt 2, sqrt 3 and 2
    d1, d2, d3, d4 = 3 * 8 * 8 * 7, 6 * 8 * 7 * 7, 4 * 7 * 7 * 7, 3 * 8 * 8 * 6
    assert got[1] == ref[1] == d1 + d2 + d3 + d4
    assert bytes(got[0]) == bytes(ref[0])
    got = orc.find_events_tree(s["x"], s["y"], s["z"], s["vx"], s["vy"], s["vz"], s["m"],
                               s["id"], h, 2e3, 1e-3, 1, 1)
    assert got[1] == ref[1] and bytes(got[0]) == bytes(ref[0])


def test_central_density_lattice(orc):
    """Lattice of spacing 1 with the lowest phi at an interior point: the
    counts within radii 1, 1.5, 1.75 and 2.05 are 7, 19, 27 and 33."""
    s = W.lattice(9, seed=2)
    x, y, z = s["x"], s["y"], s["z"]
    m = np.full(x.size, 0.5)
    c0 = np.array([4.0, 4.0, 4.0])
    phi = (x - c0[0]) ** 2 + (y - c0[1]) ** 2 + (z - c0[2]) ** 2 - 5.0
    for radius, expect in ((1.0, 7), (1.5, 19), (1.75, 27), (2.05, 33)):
        c, cnt, mass = orc.central_density(x, y, z, m, phi, radius)
        assert (x[c], y[c], z[c]) == (4.0, 4.0, 4.0)
        assert cnt == expect
        assert mass == 0.5 * expect


def test_central_density_ties_and_nan(orc):
    """The first index wins a tie; NaN potentials are never the centre."""
    x = np.array([0.0, 1.0, 2.0, 3.0])
    y = z = np.zeros(4)
    m = np.ones(4)
    phi = np.array([np.nan, -2.0, -2.0, -1.0])
    c, cnt, mass = orc.central_density(x, y, z, m, phi, 1.0)
    assert c == 1 and cnt == 3 and mass == 3.0


def test_central_density_plummer(orc):
    """Plummer sphere: the potential minimum lies near the centre and the mean
    density within 0.2 a is 3M/(4 pi a^3) (1 + 0.2^2)^(-3/2) up to Poisson
    noise (about 1 %)."""
    n = 1 << 16
    s = W.plummer(n, seed=11)
    _, _, _, pot = orc.gravity(s["x"], s["y"], s["z"], s["m"], 1.0, 1e-3)
    c, cnt, mass = orc.central_density(s["x"], s["y"], s["z"], s["m"], pot, 0.2)
    assert math.sqrt(s["x"][c] ** 2 + s["y"][c] ** 2 + s["z"][c] ** 2) < 0.1
    rho = mass / (4.0 / 3.0 * math.pi * 0.2 ** 3)
    expect = 3.0 / (4.0 * math.pi) * (1.0 + 0.2 ** 2) ** -1.5
    assert rho == pytest.approx(expect, rel=5.0 / math.sqrt(cnt))
