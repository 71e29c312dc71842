"""Symmetric tiles of the mixed direct sum (each unordered pair evaluated once,
the reactions summed in 64-bit fixed point): the oracle's forces and
potentials to the mixed bar (1e-5 normwise) in every launch shape, on uneven
halos with a host, with unequal masses, and for halos smaller than one
i-block; bit-identical results on repeated calls and in a captured graph
replayed between eager work; the one-sided and symmetric sums agree; the
C2 satellite takes them by default."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    import paper_2506_06269_amd as S
    assert torch.cuda.is_available()
    S.lib()
    return S


def _batch(sizes=(6000, 20000, 4096), host_first=True, masses=None):
    parts = []
    for i, n in enumerate(sizes):
        p = W.nfw_halo(n, seed=81 + i)
        if i == 0 and host_first:
            p = W.place_on_orbit(p)
        if masses is not None and masses[i] is not None:
            p["m"] = masses[i](n)
        parts.append(p)
    halos, off = [], 0
    s = {f: np.concatenate([p[f] for p in parts]) for f in ("x", "y", "z", "vx", "vy", "vz",
                                                           "m", "id")}
    for i, p in enumerate(parts):
        n = p["x"].size
        h = dict(n=n, offset=off, eps=0.01, G=1.0, k=32, sigma_m=0.0, dt=1e-3, seed=i)
        if i == 0 and host_first:
            h["host"] = W.host_params()
        halos.append(h)
        off += n
    return s, halos, parts


def _errors(orc, out, halos, parts):
    worst = 0.0
    for h, p in zip(halos, parts):
        o, n = h["offset"], h["n"]
        ax, ay, az, pot, an = orc.gravity(p["x"], p["y"], p["z"], p["m"], 1.0, h["eps"],
                                          want_norm=True)
        if "host" in h:
            q = orc.make_params(host=h["host"])
            hx, hy, hz, hp = orc.host_field(p["x"], p["y"], p["z"], q)
            ax, ay, az, pot = ax + hx, ay + hy, az + hz, pot + hp
            an = an + np.sqrt(hx ** 2 + hy ** 2 + hz ** 2)
        e = np.sqrt((out["ax"][o:o + n] - ax) ** 2 + (out["ay"][o:o + n] - ay) ** 2 +
                    (out["az"][o:o + n] - az) ** 2) / an
        ep = np.abs(out["pot"][o:o + n] - pot) / np.abs(pot)
        worst = max(worst, e.max(), ep.max())
    return worst


def _gravity(S, ctx, halos, dev):
    import torch
    for f in ("ax", "ay", "az", "pot"):
        dev[f].fill_(float("nan"))
    S.sidm_gravity(ctx, halos, dev, S.SIDM_PREC_MIXED)
    torch.cuda.synchronize()
    return S.state_to_host(dev)


def test_every_shape_matches_the_oracle(S, orc):
    s, halos, parts = _batch()
    dev = S.state_to_device(s)
    ctx = S.sidm_create(0, s["x"].size, len(halos))
    S.sidm_set_symmetric(ctx, 1)
    for ireg, nt in S.SHAPES:
        S.sidm_set_launch_shape(ctx, ireg, nt, True)
        out = _gravity(S, ctx, halos, dev)
        w = _errors(orc, out, halos, parts)
        print(f"symmetric {ireg}x{nt}: {w:.2e}", flush=True)
        assert w < 1e-5, (ireg, nt, w)
    S.sidm_destroy(ctx)


def test_unequal_masses_and_small_halos(S, orc):
    """Masses drawn in [0.5, 1.5] m in one halo (the reactions carry m_i), and
    halos of 2, 100 and 1500 particles (inside one i-block: one-sided only)."""
    rng = np.random.default_rng(5)
    masses = [None, lambda n: rng.uniform(0.5, 1.5, n) / n, None]
    s, halos, parts = _batch(sizes=(6000, 20000, 4096), masses=masses)
    small = [W.nfw_halo(n, seed=90 + n) for n in (2, 100, 1500)]
    off = s["x"].size
    for p in small:
        for f in ("x", "y", "z", "vx", "vy", "vz", "m", "id"):
            s[f] = np.concatenate([s[f], p[f]])
        halos.append(dict(n=p["x"].size, offset=off, eps=0.01, G=1.0, k=1, sigma_m=0.0,
                          dt=1e-3, seed=7))
        parts.append(p)
        off += p["x"].size
    dev = S.state_to_device(s)
    ctx = S.sidm_create(0, s["x"].size, len(halos))
    S.sidm_set_symmetric(ctx, 1)
    for ireg, nt in ((2, 512), (4, 256), (8, 128)):
        S.sidm_set_launch_shape(ctx, ireg, nt, True)
        w = _errors(orc, _gravity(S, ctx, halos, dev), halos, parts)
        print(f"unequal masses, {ireg}x{nt}: {w:.2e}", flush=True)
        assert w < 1e-5
    S.sidm_destroy(ctx)


def test_repeatable_and_close_to_one_sided(S, orc):
    """Two calls give the same bits; the one-sided sums (symmetric tiles off)
    agree to 2e-6 normwise; the total sum m a of an isolated halo stays at
    rounding (printed for both)."""
    s, halos, parts = _batch()
    dev = S.state_to_device(s)
    ctx = S.sidm_create(0, s["x"].size, len(halos))
    S.sidm_set_launch_shape(ctx, 2, 512, True)
    S.sidm_set_symmetric(ctx, 1)
    a = _gravity(S, ctx, halos, dev)
    b = _gravity(S, ctx, halos, dev)
    for f in ("ax", "ay", "az", "pot"):
        assert np.array_equal(a[f], b[f]), f
    S.sidm_set_symmetric(ctx, 0)
    c = _gravity(S, ctx, halos, dev)
    for h, p in zip(halos, parts):
        o, n = h["offset"], h["n"]
        _, _, _, _, an = orc.gravity(p["x"], p["y"], p["z"], p["m"], 1.0, h["eps"],
                                     want_norm=True)
        d = np.sqrt(sum((a[f][o:o + n] - c[f][o:o + n]) ** 2 for f in ("ax", "ay", "az"))) / an
        assert d.max() < 2e-6, d.max()
        if "host" in h:
            continue     # the host's field is not a pair force
        m = p["m"]
        mom = lambda r: np.sqrt(sum(np.sum(m * r[f][o:o + n]) ** 2 for f in ("ax", "ay", "az")))
        scale = np.sum(m * an)
        print(f"halo n={n}: |sum m a| symmetric {mom(a) / scale:.2e}, one-sided "
              f"{mom(c) / scale:.2e}", flush=True)
        assert mom(a) < 1e-6 * scale
    S.sidm_destroy(ctx)


def test_captured_graph_replays_bit_identical(S):
    """A mixed gravity call with the symmetric tiles captured into a graph and
    replayed three times, with eager work and synchronisations in between:
    each replay gives the eager call's bits."""
    import torch
    s, halos, parts = _batch()
    dev = S.state_to_device(s)
    ctx = S.sidm_create(0, s["x"].size, len(halos))
    S.sidm_set_launch_shape(ctx, 4, 256, True)
    S.sidm_set_symmetric(ctx, 1)
    ref = _gravity(S, ctx, halos, dev)   # eager: the plan and the fingerprint
    stream = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        graph.capture_begin()
        S.sidm_gravity(ctx, halos, dev, S.SIDM_PREC_MIXED)
        graph.capture_end()
    torch.cuda.synchronize()
    for rep in range(3):
        for f in ("ax", "ay", "az", "pot"):
            dev[f].fill_(0.0)
        _ = torch.ones(16, device="cuda").sum().item()   # eager work between replays
        graph.replay()
        torch.cuda.synchronize()
        out = S.state_to_host(dev)
        for f in ("ax", "ay", "az", "pot"):
            assert np.array_equal(out[f], ref[f]), (rep, f)
    S.sidm_destroy(ctx)


def test_c2_satellite_takes_them_by_default(S, orc):
    """The N = 2^20 satellite in the host (the benchmark's workload) with the
    default threshold: 512 sampled particles against the oracle's sums over
    all N, 1e-5 normwise, and against the one-sided tiles."""
    import torch
    cfg = W.config("C2")
    s = W.make_state(cfg)
    n = cfg["n"]
    halo = dict(n=n, eps=cfg["eps"], G=1.0, k=cfg["k"], sigma_m=0.0, dt=cfg["dt"], seed=0,
                host=cfg["host"])
    dev = S.state_to_device(s)
    ctx = S.sidm_create(0, n, 1)
    S.sidm_set_launch_shape(ctx, 2, 512, True)
    sym = _gravity(S, ctx, [halo], dev)
    S.sidm_set_symmetric(ctx, 0)
    one = _gravity(S, ctx, [halo], dev)
    q = np.random.default_rng(2).choice(n, 512, replace=False)
    ax, ay, az, pot, an = orc.gravity(s["x"], s["y"], s["z"], s["m"], 1.0, cfg["eps"], query=q,
                                      want_norm=True)
    H = halo["host"]
    hx, hy, hz, hp = orc.host_nfw(s["x"][q], s["y"][q], s["z"][q], 1.0, H["rho_s"], H["r_s"],
                                  H["center"])
    ax, ay, az, pot = ax + hx, ay + hy, az + hz, pot + hp
    an = an + np.sqrt(hx ** 2 + hy ** 2 + hz ** 2)
    for out in (sym, one):
        e = np.sqrt((out["ax"][q] - ax) ** 2 + (out["ay"][q] - ay) ** 2 +
                    (out["az"][q] - az) ** 2) / an
        ep = np.abs(out["pot"][q] - pot) / np.abs(pot)
        print(f"C2 sampled: e_a {e.max():.2e} e_phi {ep.max():.2e}", flush=True)
        assert e.max() < 1e-5 and ep.max() < 1e-5
    assert not np.array_equal(sym["ax"], one["ax"])   # the symmetric tiles did run
    S.sidm_destroy(ctx)
