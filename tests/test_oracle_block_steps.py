"""Pins of the oracle's block time steps (Sec. 2: individual steps from the
gravitational criterion eta, Springel 2005 eq. 34, with a minimum step; the
energy error that changing steps can cause is discussed in Sec. 3.1).

A cycle of length dt holds 2^max_bin ticks; a particle in bin b is kicked and
gets new forces every 2^(max_bin - b) ticks.  The pins: the bin is the
criterion written with logarithms; max_bin = 0 is the fixed step exactly; one
common bin is that many fixed steps exactly; particles in different bins that
do not feel each other follow their own fixed steps; and a spread of bins
keeps the energy error of the short steps at a fraction of the cost."""
import math

import numpy as np
import pytest

import workloads as W

FIELDS = ("x", "y", "z", "vx", "vy", "vz", "ax", "ay", "az", "pot", "h")


def _copy(s):
    return {k: np.array(v, copy=True) for k, v in s.items()}


def _energy(orc, s, p):
    d = orc.diag(s["vx"], s["vy"], s["vz"], s["m"], s["pot"], np.zeros_like(s["pot"]))
    return d["K"] + d["W"]


def test_bin_is_the_criterion(orc):
    """b = ceil(log2(dt / s_max)) clipped to [0, max_bin], s_max = sqrt(2 eta
    eps / |a|), then lowered while dt / 2^b < dt_min; values within 1e-9 of a
    boundary are left out (there the two forms may round apart)."""
    rng = np.random.default_rng(1)
    dt, eta, eps = 0.01, 0.025, 0.02
    for max_bin, dt_min in ((6, 0.0), (6, dt / 16), (0, 0.0), (3, 0.0)):
        p = orc.make_params(eps=eps, dt=dt, steps=dict(eta=eta, max_bin=max_bin, dt_min=dt_min))
        a = rng.normal(size=(4000, 3)) * np.exp(rng.uniform(-4, 12, 4000))[:, None]
        got = orc.time_bin(p, a[:, 0], a[:, 1], a[:, 2])
        amag = np.linalg.norm(a, axis=1)
        smax = np.sqrt(2 * eta * eps / amag)
        x = np.log2(dt / smax)
        want = np.clip(np.ceil(x), 0, max_bin).astype(int)
        if dt_min > 0:
            cap = int(math.floor(math.log2(dt / dt_min) + 1e-12))
            want = np.minimum(want, cap)
        keep = np.abs(x - np.round(x)) > 1e-9
        assert keep.sum() > 3900
        assert np.array_equal(got[keep], want[keep]), max_bin
        if max_bin == 6 and dt_min == 0:
            assert len(set(got.tolist())) == 7       # every bin used
    p = orc.make_params(eps=eps, dt=dt, steps=dict(eta=eta, max_bin=5))
    assert orc.time_bin(p, [0.0], [0.0], [0.0])[0] == 0   # no force: the longest step


@pytest.mark.parametrize("with_host", [False, True])
def test_max_bin_zero_is_the_fixed_step(orc, with_host):
    """eta > 0 with max_bin = 0: bit for bit the fixed KDK step (gravity, host,
    reflecting sphere, kNN and scattering)."""
    n = 500
    s = W.nfw_halo(n, seed=61)
    kw = dict(eps=0.02, sigma_m=30.0, dt=5e-3, k=16, seed=9)
    if with_host:
        s = W.place_on_orbit(s)
        kw.update(host=W.host_params(),
                  boundary=dict(r=2.0, center=(float(np.mean(s["x"])), float(np.mean(s["y"])),
                                               float(np.mean(s["z"])))))
    p0 = orc.make_params(**kw)
    p1 = orc.make_params(steps=dict(eta=0.025, max_bin=0), **kw)
    orc.total_accel(s, p0)
    a, b = _copy(s), _copy(s)
    for step in range(3):
        ea = orc.kdk_step(a, p0, step)
        eb = orc.kdk_step(b, p1, step)
        assert ea.size == eb.size and np.array_equal(ea, eb)
        for k in FIELDS:
            assert np.array_equal(a[k], b[k]), (step, k)
    assert ea.size > 0


def test_one_common_bin_is_that_many_fixed_steps(orc):
    """A criterion that puts every particle in bin 3 all cycle long: one cycle
    equals 8 fixed steps of dt/8 exactly (without scattering, which a cycle
    applies once at its end)."""
    n = 400
    s = W.plummer(n, seed=62)
    dt = 8e-3
    kw = dict(eps=0.02, sigma_m=0.0, k=16)
    p_cycle = orc.make_params(dt=dt, steps=dict(eta=1e-30, max_bin=3), **kw)
    p_fixed = orc.make_params(dt=dt / 8, **kw)
    orc.total_accel(s, p_cycle)
    a, b = _copy(s), _copy(s)
    for cyc in range(2):
        orc.kdk_step(a, p_cycle, cyc)
        for j in range(8):
            orc.kdk_step(b, p_fixed, 8 * cyc + j)
        for k in FIELDS:
            assert np.array_equal(a[k], b[k]), (cyc, k)


def test_independent_particles_follow_their_own_steps(orc):
    """Massless particles in the host feel only the host: a particle that
    stays in bin b through the cycle moves as under 2^b fixed steps of
    dt / 2^b (up to the rounding of its 2^(max_bin - b) partial drifts)."""
    n = 300
    rng = np.random.default_rng(63)
    r = np.exp(rng.uniform(np.log(1.0), np.log(3000.0), n))
    u = rng.normal(size=(n, 3))
    u /= np.linalg.norm(u, axis=1)[:, None]
    host = W.host_params()
    c = np.array(host["center"])
    pos = c + u * r[:, None]
    vel = rng.normal(size=(n, 3)) * 0.3
    s = dict(x=pos[:, 0].copy(), y=pos[:, 1].copy(), z=pos[:, 2].copy(), vx=vel[:, 0].copy(),
             vy=vel[:, 1].copy(), vz=vel[:, 2].copy(), m=np.zeros(n),
             id=np.arange(n, dtype=np.uint32))
    dt, B = 0.02, 5
    kw = dict(eps=0.01, sigma_m=0.0, k=8, host=host)
    pc = orc.make_params(dt=dt, steps=dict(eta=0.01, max_bin=B), **kw)
    orc.total_accel(s, pc)
    bins0 = orc.time_bin(pc, s["ax"], s["ay"], s["az"])
    assert len(set(bins0.tolist())) >= 4
    a = _copy(s)
    orc.kdk_step(a, pc, 0)
    bins1 = orc.time_bin(pc, a["ax"], a["ay"], a["az"])
    checked = 0
    print("bins", np.bincount(bins0))
    for b in sorted(set(bins0.tolist())):
        sel = np.flatnonzero((bins0 == b) & (bins1 == b))
        if sel.size < 2:
            continue
        sub = {k: np.array(s[k][sel], copy=True) for k in s if k != "h"}
        pf = orc.make_params(dt=dt / 2 ** b, **kw)
        for j in range(2 ** b):
            orc.kdk_step(sub, pf, j)
        for k in ("x", "y", "z", "vx", "vy", "vz", "ax", "ay", "az", "pot"):
            scale = np.max(np.abs(sub[k]))
            err = np.max(np.abs(a[k][sel] - sub[k]))
            assert err <= 1e-13 * scale, (b, k, err / scale)
            if b == B:
                assert np.array_equal(a[k][sel], sub[k]), (b, k)
        checked += sel.size
    assert checked > 0.8 * n


def test_block_steps_energy(orc):
    """A Plummer sphere whose bins spread over 0..3: over a time of 8 dt the
    energy error of the block steps is far below that of the fixed step dt and
    within a small factor of the fixed step dt/8, with fewer force
    evaluations than the latter."""
    n = 600
    s = W.plummer(n, seed=64)
    dt, eta, eps, B = 0.04, 0.004, 0.01, 3
    kw = dict(eps=eps, sigma_m=0.0, k=16)
    pc = orc.make_params(dt=dt, steps=dict(eta=eta, max_bin=B), **kw)
    orc.total_accel(s, pc)
    bins = orc.time_bin(pc, s["ax"], s["ay"], s["az"])
    assert bins.min() <= 1 and bins.max() == B
    work = float(np.sum(2.0 ** bins)) / (n * 2 ** B)
    e0 = _energy(orc, s, pc)
    runs = {}
    for name, p, reps in (("big", orc.make_params(dt=dt, **kw), 8),
                          ("small", orc.make_params(dt=dt / 8, **kw), 64),
                          ("block", pc, 8)):
        t = _copy(s)
        for j in range(reps):
            orc.kdk_step(t, p, j)
        runs[name] = abs(_energy(orc, t, p) - e0) / abs(e0)
    print(runs, "work fraction", work)
    assert work < 0.8
    assert runs["block"] < 0.25 * runs["big"]
    assert runs["block"] < 4.0 * runs["small"] + 1e-12


def test_changing_bins_keep_test_particle_energy(orc):
    """Massless particles on eccentric orbits in the host change bins many
    times.  Their specific energies v^2/2 + Phi_host drift no more than under
    fixed steps of about the bins' lengths: the median final error is far
    below that of the fixed step dt and within a small factor of the fixed
    step dt/4 (a kick with the wrong step length at each bin change leaves a
    first-order error that grows with the number of changes instead)."""
    n = 100
    rng = np.random.default_rng(65)
    host = W.host_params()
    c = np.array(host["center"])
    r = np.exp(rng.uniform(np.log(5.0), np.log(200.0), n))
    u = rng.normal(size=(n, 3))
    u /= np.linalg.norm(u, axis=1)[:, None]
    pos = c + u * r[:, None]
    pv = orc.make_params(host=host)
    _, _, _, phi = orc.host_field(pos[:, 0], pos[:, 1], pos[:, 2], pv)
    w = rng.normal(size=(n, 3))
    w -= np.sum(w * u, axis=1)[:, None] * u          # tangential: eccentric orbits
    w /= np.linalg.norm(w, axis=1)[:, None]
    vel = w * (0.3 * np.sqrt(-phi))[:, None]
    s = dict(x=pos[:, 0].copy(), y=pos[:, 1].copy(), z=pos[:, 2].copy(), vx=vel[:, 0].copy(),
             vy=vel[:, 1].copy(), vz=vel[:, 2].copy(), m=np.zeros(n),
             id=np.arange(n, dtype=np.uint32))
    dt, B, cycles = 0.25, 4, 40
    kw = dict(eps=1.0, sigma_m=0.0, k=8, host=host)
    pc = orc.make_params(dt=dt, steps=dict(eta=0.3, max_bin=B), **kw)
    orc.total_accel(s, pc)

    def energy(t):
        return 0.5 * (t["vx"] ** 2 + t["vy"] ** 2 + t["vz"] ** 2) + t["pot"]
    e0 = energy(s)
    final, changes = {}, 0
    for name, p, reps in (("block", pc, cycles), ("big", orc.make_params(dt=dt, **kw), cycles),
                          ("quarter", orc.make_params(dt=dt / 4, **kw), cycles * 4)):
        t = _copy(s)
        prev = orc.time_bin(pc, t["ax"], t["ay"], t["az"])
        for j in range(reps):
            orc.kdk_step(t, p, j)
            if name == "block":
                now = orc.time_bin(pc, t["ax"], t["ay"], t["az"])
                changes += int(np.count_nonzero(now != prev))
                prev = now
        final[name] = float(np.median(np.abs(energy(t) - e0) / np.abs(e0)))
    print("bin changes", changes, "median final |dE/E|", final)
    assert changes > 3 * n
    assert final["block"] < 0.2 * final["big"]
    assert final["block"] < 10.0 * final["quarter"]
