"""The 64-halo batch in one call (uneven N, sigma/m in {1, 10, 50}, k in
{16, 32, 64, 128}, a seed per halo) against the oracle on sampled halos, and
a step captured into a HIP graph replayed against eager steps."""
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


def _batch(halo_list, seed_base=0):
    total = sum(h["n"] for h in halo_list)
    s = {f: np.zeros(total) for f in ("x", "y", "z", "vx", "vy", "vz", "m")}
    s["id"] = np.zeros(total, dtype=np.uint32)
    halos, parts, off = [], [], 0
    for b, h in enumerate(halo_list):
        p = W.nfw_halo(h["n"], seed=seed_base + h["seed"])
        parts.append(p)
        for f in ("x", "y", "z", "vx", "vy", "vz", "m", "id"):
            s[f][off:off + h["n"]] = p[f]
        halos.append(dict(h, offset=off))
        off += h["n"]
    return s, halos, parts


def test_c4_batch_sampled_parity(S, orc):
    """All 64 halos in one sidm_gravity / sidm_knn_h / sidm_scatter call each;
    8 halos (every k and sigma/m) checked against the oracle."""
    import torch
    halo_list = W.batch_c4()
    s, halos, parts = _batch(halo_list)
    total = s["x"].size
    print(f"C4: {len(halos)} halos, {total} particles", flush=True)
    dev = S.state_to_device(s)
    ctx = S.sidm_create(0, total, len(halos))
    S.sidm_gravity(ctx, halos, dev, S.SIDM_PREC_MIXED)
    S.sidm_knn_h(ctx, halos, dev)
    torch.cuda.synchronize()
    g = S.state_to_host(dev)
    ev = S.event_buffer(1 << 18)
    cnt = S.sidm_scatter(ctx, halos, dev, 5, events=ev, want_count=True)
    events = S.read_events(ev, cnt)
    out = S.state_to_host(dev)
    for b in (0, 5, 10, 22, 35, 47, 58, 63):
        h, p, o, n = halos[b], parts[b], halos[b]["offset"], halos[b]["n"]
        ax, ay, az, pot, an = orc.gravity(p["x"], p["y"], p["z"], p["m"], 1.0, h["eps"],
                                          want_norm=True)
        ea = np.sqrt((g["ax"][o:o + n] - ax) ** 2 + (g["ay"][o:o + n] - ay) ** 2 +
                     (g["az"][o:o + n] - az) ** 2) / an
        assert ea.max() < 1e-5, (b, ea.max())
        href = orc.knn(p["x"], p["y"], p["z"], p["id"], h["k"])
        assert np.array_equal(g["h"][o:o + n], href), b
        q = dict(p, h=href)
        ref, _, _ = orc.find_events(q["x"], q["y"], q["z"], q["vx"], q["vy"], q["vz"], q["m"],
                                    q["id"], q["h"], h["sigma_m"], h["dt"], h["seed"], 5)
        mine = events[events["halo"] == b]
        assert sorted(zip(mine["a"].tolist(), mine["b"].tolist())) == \
            sorted(zip(ref["a"].tolist(), ref["b"].tolist())), b
        vx = q["vx"].copy(); vy = q["vy"].copy(); vz = q["vz"].copy()
        orc.apply_events(ref, q["m"], vx, vy, vz, h["seed"], 5)
        assert np.max(np.abs(out["vx"][o:o + n] - vx)) <= 1e-12 * np.abs(vx).max()


@pytest.mark.parametrize("variant", ["fixed", "blocks_and_tree"])
def test_graph_captured_step_matches_eager(S, variant):
    """A captured sidm_kdk_step replayed 3 times (with eager work and
    synchronisations between replays) against 3 eager steps from the same
    state.  The step counter is part of the captured arguments, so both sides
    use the same step number each time.  The second variant captures cycles of
    block time steps (the ticks' work items, a direct-sum halo) with a tree
    halo beside it: some hundreds of launches per captured call."""
    import torch
    halo_list = [dict(n=3000, sigma_m=50.0, k=32, seed=1, G=1.0, eps=0.01, dt=1e-3, host=None),
                 dict(n=5000, sigma_m=10.0, k=64, seed=2, G=1.0, eps=0.01, dt=1e-3, host=None)]
    if variant == "blocks_and_tree":
        halo_list[0].update(dt=1.0 / 32, steps=dict(eta=0.025, max_bin=3))
        halo_list[1].update(tree_alpha=5e-4)
    s, halos, _ = _batch(halo_list, seed_base=40)
    total = s["x"].size

    def fresh():
        dev = S.state_to_device(s)
        ctx = S.sidm_create(0, total, len(halos))
        S.sidm_gravity(ctx, halos, dev, S.SIDM_PREC_MIXED)
        return ctx, dev

    ctx_e, dev_e = fresh()
    diag_e = S.diag_buffer(len(halos))
    for _ in range(3):
        S.sidm_kdk_step(ctx_e, halos, dev_e, 9, S.SIDM_PREC_MIXED, diag=diag_e)
    torch.cuda.synchronize()
    eager = S.state_to_host(dev_e)

    ctx_g, dev_g = fresh()
    diag_g = S.diag_buffer(len(halos))
    # one eager call builds the launch plan outside the capture
    S.sidm_diagnostics(ctx_g, halos, dev_g, diag_g)
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        graph.capture_begin()
        S.sidm_kdk_step(ctx_g, halos, dev_g, 9, S.SIDM_PREC_MIXED, diag=diag_g)
        graph.capture_end()
    torch.cuda.synchronize()
    # capture does not execute: the state is still the initial one
    assert np.array_equal(dev_g["x"].cpu().numpy(), s["x"])
    for r in range(3):
        graph.replay()
        torch.cuda.synchronize()
        _ = torch.ones(16, device="cuda").sum().item()   # eager work between replays
    got = S.state_to_host(dev_g)
    for f in ("x", "y", "z", "vx", "vy", "vz", "ax", "pot", "h"):
        assert np.array_equal(got[f], eager[f]), f
    assert bytes(diag_g.cpu().numpy()) == bytes(diag_e.cpu().numpy())
