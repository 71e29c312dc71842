"""Pins of the oracle's tree gravity (Sec. 2: the gravity tree with the
relative opening criterion alpha of Springel 2005; Table 1 and Sec. 2 give
alpha = 5e-4).  The tree, groups and criterion are defined in the oracle's
header; the pins: alpha = 0 opens every node and is the direct sum, with
exactly one term per particle and group; with every disjoint node accepted
and a softening far above the system's size every particle still feels the
whole mass but itself once (complete, non-overlapping cover; node masses);
the error against the direct sum shrinks with alpha and stays within a few
alpha of |a| at the paper's value; a compact cluster far away acts as its
monopole."""
import numpy as np
import pytest

import workloads as W


def _rel_err(t, d):
    num = np.sqrt((t[0] - d[0]) ** 2 + (t[1] - d[1]) ** 2 + (t[2] - d[2]) ** 2)
    return num / np.sqrt(d[0] ** 2 + d[1] ** 2 + d[2] ** 2)


@pytest.mark.parametrize("n", [1, 2, 64, 65, 1000, 3000])
def test_alpha_zero_is_the_direct_sum(orc, n):
    s = W.nfw_halo(max(n, 2), seed=82)
    x, y, z, m = (s[k][:n] for k in ("x", "y", "z", "m"))
    d = orc.gravity(x, y, z, m, 1.3, 0.02, want_norm=True)
    t = orc.tree_gravity(x, y, z, m, (d[0], d[1], d[2]), 1.3, 0.02, 0.0)
    groups = (n + 63) // 64
    assert t[4] == groups * n
    if n > 1:
        err = np.sqrt((t[0] - d[0]) ** 2 + (t[1] - d[1]) ** 2 + (t[2] - d[2]) ** 2) / d[4]
        assert err.max() < 1e-13
        assert np.max(np.abs(t[3] - d[3]) / np.abs(d[3])) < 1e-13
    else:
        assert t[0][0] == t[1][0] == t[2][0] == t[3][0] == 0.0


def test_cover_is_complete_and_disjoint(orc):
    """a_old = 1e30 accepts every node whose box is disjoint from the group's;
    with eps = 1e5 every term is m / eps to 1e-8, so pot_i = -G (M - m_i)/eps:
    each other particle counted exactly once, through a node or itself."""
    n = 5000
    s = W.nfw_halo(n, seed=83)
    m = s["m"] * (1.0 + 0.5 * np.random.default_rng(1).random(n))   # unequal masses
    big = np.full(n, 1e30)
    eps = 1e5
    t = orc.tree_gravity(s["x"], s["y"], s["z"], m, (big, big, big), 1.0, eps, 5e-4)
    want = -(m.sum() - m) / eps
    assert np.max(np.abs(t[3] - want) / np.abs(want)) < 1e-8
    assert t[4] < 0.2 * ((n + 63) // 64) * n        # most of the mass came through nodes


def test_error_shrinks_with_alpha(orc):
    n = 20000
    s = W.nfw_halo(n, seed=84)
    d = orc.gravity(s["x"], s["y"], s["z"], s["m"], 1.0, 0.01)
    med, mx, terms = [], [], []
    for alpha in (2.5e-2, 2.5e-3, 5e-4, 5e-5):
        t = orc.tree_gravity(s["x"], s["y"], s["z"], s["m"], d[:3], 1.0, 0.01, alpha)
        e = _rel_err(t, d)
        med.append(np.median(e))
        mx.append(e.max())
        terms.append(t[4])
        if alpha == 5e-4:
            assert np.median(e) < 2 * alpha and e.max() < 10 * alpha
            ep = np.abs(t[3] - d[3]) / np.abs(d[3])
            assert ep.max() < 10 * alpha
    print("median", med, "max", mx, "terms", terms)
    assert med == sorted(med, reverse=True) and mx == sorted(mx, reverse=True)
    assert terms == sorted(terms)
    assert terms[0] < 0.6 * terms[-1]


def test_distant_cluster_acts_as_its_monopole(orc):
    """Two Plummer clusters 1000 apart: the force of the far cluster on each
    member of the near one is G M_far (c - x)/|c - x|^3 to its quadrupole
    order (a/R)^2 ~ 1e-6, where c is the far cluster's centre of mass."""
    a = W.plummer(2000, seed=85, a=1.0, M=1.0)
    b = W.plummer(3000, seed=86, a=1.0, M=2.0)
    shift = np.array([1000.0, 0.0, 0.0])
    x = np.concatenate([a["x"], b["x"] + shift[0]])
    y = np.concatenate([a["y"], b["y"]])
    z = np.concatenate([a["z"], b["z"]])
    m = np.concatenate([a["m"], b["m"]])
    d = orc.gravity(x, y, z, m, 1.0, 0.01)
    t = orc.tree_gravity(x, y, z, m, d[:3], 1.0, 0.01, 5e-4)
    near = orc.gravity(a["x"], a["y"], a["z"], a["m"], 1.0, 0.01)
    cm = np.array([np.sum(b["m"] * (b[k] + s)) / np.sum(b["m"])
                   for k, s in (("x", shift[0]), ("y", 0.0), ("z", 0.0))])
    dx = cm[0] - a["x"]
    dy = cm[1] - a["y"]
    dz = cm[2] - a["z"]
    r3 = (dx * dx + dy * dy + dz * dz + 1e-4) ** 1.5
    Mb = np.sum(b["m"])
    far = (Mb * dx / r3, Mb * dy / r3, Mb * dz / r3)
    n1 = a["x"].size
    for c in range(3):
        got = t[c][:n1] - near[c]
        assert np.max(np.abs(got - far[c])) < 1e-5 * np.max(np.abs(far[0]))


def test_step_with_a_vanishing_alpha_is_the_direct_step(orc):
    """tree_alpha = 1e-300 runs the step's tree path with every node opened
    (r^8 alpha^2 underflows): the same step as the direct sum to rounding."""
    n = 700
    s = W.nfw_halo(n, seed=87)
    p0 = orc.make_params(eps=0.02, sigma_m=5.0, dt=4e-3, k=16, seed=3)
    p1 = orc.make_params(eps=0.02, sigma_m=5.0, dt=4e-3, k=16, seed=3, tree_alpha=1e-300)
    orc.total_accel(s, p0)
    a = {k: np.array(v, copy=True) for k, v in s.items()}
    b = {k: np.array(v, copy=True) for k, v in s.items()}
    for step in range(2):
        ea = orc.kdk_step(a, p0, step)
        eb = orc.kdk_step(b, p1, step)
        assert ea.size == eb.size
        for k in ("x", "y", "z", "vx", "vy", "vz", "ax", "ay", "az", "pot"):
            assert np.max(np.abs(a[k] - b[k])) <= 1e-13 * np.max(np.abs(a[k])), k


def test_query_form_equals_the_full_form(orc):
    """Forces of a sample of particles (repeats and the last one included)
    equal those of the full evaluation bit for bit; the terms counted are
    those of the groups walked."""
    n = 6000
    s = W.nfw_halo(n, seed=88)
    d = orc.gravity(s["x"], s["y"], s["z"], s["m"], 1.0, 0.01)
    full = orc.tree_gravity(s["x"], s["y"], s["z"], s["m"], d[:3], 1.0, 0.01, 5e-4)
    q = np.array([0, 17, 17, n - 1, 2500, 4097, 1], dtype=np.int64)
    part = orc.tree_gravity(s["x"], s["y"], s["z"], s["m"], d[:3], 1.0, 0.01, 5e-4, query=q)
    for c in range(4):
        assert np.array_equal(part[c], full[c][q])
    assert 0 < part[4] < full[4]


def _rod_and_probes(R, seed=87):
    """An elongated cluster (Gaussian, sigma = (4, 1, 0.5)) of unit mass centred
    at (R, 0, 0), and 50 massless probes within 1 of the origin."""
    rng = np.random.default_rng(seed)
    n = 3000
    rod = np.stack([rng.normal(0, 4.0, n) + R, rng.normal(0, 1.0, n), rng.normal(0, 0.5, n)])
    probes = rng.uniform(-1.0, 1.0, (3, 50))
    x, y, z = (np.concatenate([probes[c], rod[c]]) for c in range(3))
    m = np.concatenate([np.zeros(50), np.full(n, 1.0 / n)])
    return x, y, z, m


def test_far_nodes_carry_their_quadrupole(orc):
    """Every node of the elongated cluster disjoint from the probes' group is
    accepted (a_old huge): with monopoles alone the error of the far field
    would fall as (l/R)^2, with the quadrupole term it falls as (l/R)^3 --
    doubling R divides it by about 8 -- and is far below the monopole's
    (l/R)^2 level.  The direct sum is the reference."""
    errs = []
    for R in (150.0, 300.0):
        x, y, z, m = _rod_and_probes(R)
        d = orc.gravity(x, y, z, m, 1.0, 1e-3)
        big = [np.full(x.size, 1e30)] * 3
        q = np.arange(50)
        t = orc.tree_gravity(x, y, z, m, big, 1.0, 1e-3, 1.0, query=q)
        e = _rel_err([t[c] for c in range(3)], [d[c][:50] for c in range(3)])
        errs.append(e.max())
        assert e.max() < 0.05 * (4.0 / R) ** 2, (R, e.max())
    assert 5.0 < errs[0] / errs[1] < 12.0, errs


@pytest.mark.parametrize("n", [2, 100, 2000])
def test_octree_without_a_old_is_the_direct_sum(orc, n):
    """a_old = 0 opens every cell of the paper-style oct-tree: each particle
    sums every other one (n(n-1) terms), the direct sum to rounding."""
    s = W.nfw_halo(max(n, 2), seed=88)
    x, y, z, m = (s[k][:n] for k in ("x", "y", "z", "m"))
    d = orc.gravity(x, y, z, m, 1.3, 0.02, want_norm=True)
    zero = [np.zeros(n)] * 3
    t = orc.octree_gravity(x, y, z, m, zero, 1.3, 0.02, 5e-4)
    assert t[4] == n * (n - 1)
    e = np.sqrt((t[0] - d[0]) ** 2 + (t[1] - d[1]) ** 2 + (t[2] - d[2]) ** 2) / d[4]
    assert e.max() < 1e-13
    assert np.max(np.abs(t[3] - d[3]) / np.abs(d[3])) < 1e-13


def test_octree_distant_cluster_is_one_monopole(orc):
    """Massless probes near the origin and a Plummer cluster (mass 2, a = 1)
    1000 away: with the per-particle criterion at alpha = 5e-4 the far
    cluster is taken as one cell or a few, so the probes feel
    G M (c - x) / |c - x|^3 (c its centre of mass) to order (a/R)^2."""
    b = W.plummer(3000, seed=86, a=1.0, M=2.0)
    rng = np.random.default_rng(4)
    pr = rng.uniform(-1.0, 1.0, (3, 40))
    x = np.concatenate([pr[0], b["x"] + 1000.0])
    y = np.concatenate([pr[1], b["y"]])
    z = np.concatenate([pr[2], b["z"]])
    m = np.concatenate([np.zeros(40), b["m"]])
    d = orc.gravity(x, y, z, m, 1.0, 0.01)
    q = np.arange(40)
    t = orc.octree_gravity(x, y, z, m, d[:3], 1.0, 0.01, 5e-4, query=q)
    assert t[4] < 40 * 100      # a few cells per probe, not the 3000 particles
    Mb = np.sum(b["m"])
    cm = [np.sum(b["m"] * (b["x"] + 1000.0)) / Mb, np.sum(b["m"] * b["y"]) / Mb,
          np.sum(b["m"] * b["z"]) / Mb]
    dx, dy, dz = cm[0] - pr[0], cm[1] - pr[1], cm[2] - pr[2]
    r3 = (dx * dx + dy * dy + dz * dz + 1e-4) ** 1.5
    far = (Mb * dx / r3, Mb * dy / r3, Mb * dz / r3)
    for c in range(3):
        assert np.max(np.abs(t[c] - far[c])) < 1e-5 * np.max(np.abs(far[0]))


def test_octree_error_and_work_follow_alpha(orc):
    """On an NFW halo with a_old from the direct sum: the terms summed fall and
    the error against the direct sum grows as alpha grows, and at alpha =
    5e-4 the median error stays within a few alpha of |a| (normwise)."""
    s = W.nfw_halo(6000, seed=89)
    d = orc.gravity(s["x"], s["y"], s["z"], s["m"], 1.0, 0.01, want_norm=True)
    q = np.arange(0, 6000, 7)
    meds, terms = [], []
    for alpha in (1e-4, 5e-4, 2.5e-3):
        t = orc.octree_gravity(s["x"], s["y"], s["z"], s["m"], d[:3], 1.0, 0.01, alpha, query=q)
        e = np.sqrt((t[0] - d[0][q]) ** 2 + (t[1] - d[1][q]) ** 2 + (t[2] - d[2][q]) ** 2)
        e /= np.sqrt(d[0][q] ** 2 + d[1][q] ** 2 + d[2][q] ** 2)
        meds.append(np.median(e))
        terms.append(t[4])
    assert terms[0] > terms[1] > terms[2]
    assert meds[0] < meds[1] < meds[2]
    assert meds[1] < 10 * 5e-4
