"""Step-wise parity of the N = 2^20 satellite in its host (k = 64, sigma/m =
10, mixed precision: the benchmark's workload and launch configuration) at
steps 0, 1, 50 and 99 of a 100-step run.  At a checked step the GPU's state
S_n is copied to the host and the oracle repeats the step from it: kick and
drift (FP64 on both sides, so the positions must agree bit for bit), then
with the GPU's new accelerations (checked on 4096 sampled particles against
the oracle's direct sum over all N) the closing kick, the kernel sizes of all
N particles (bit-exact), the complete event set over all N (mismatches
allowed only for draws within 1e-9 P of P, counted, none expected) and the
ordered kicks (velocities within 1e-12 of the largest).  Energy and momentum
are logged every step."""
import numpy as np
import pytest

import workloads as W
from tests._parity import event_parity

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(900)
def test_c2_stepwise_full_n(orc):
    import torch
    import paper_2506_06269_amd as S
    assert torch.cuda.is_available()
    cfg = W.config("C2")
    n = cfg["n"]
    s = W.make_state(cfg)
    halo = dict(n=n, eps=cfg["eps"], G=1.0, k=cfg["k"], sigma_m=cfg["sigma_m"], dt=cfg["dt"],
                seed=0, host=cfg["host"])
    p = orc.make_params(G=1.0, eps=cfg["eps"], sigma_m=cfg["sigma_m"], dt=cfg["dt"], k=cfg["k"],
                        seed=0, host=cfg["host"])
    dev = S.state_to_device(s)
    ctx = S.sidm_create(0, n, 1)
    S.sidm_gravity(ctx, [halo], dev, S.SIDM_PREC_MIXED)
    diag = S.diag_buffer(1)
    evbuf = S.event_buffer(1 << 16)
    rng = np.random.default_rng(0)
    E0 = None
    checked = 0
    for step in range(100):
        check = step in (0, 1, 50, 99)
        if check:
            torch.cuda.synchronize()
            pre = S.state_to_host(dev)
        S.sidm_kdk_step(ctx, [halo], dev, step, S.SIDM_PREC_MIXED, diag=diag)
        d = S.read_diag(diag)[0]
        assert d["status"] == 0
        E = d["K"] + d["W"] + d["Eext"]
        E0 = E if E0 is None else E0
        if not check:
            continue
        cnt = S.sidm_last_events(ctx, evbuf, want_count=True)
        got = S.read_events(evbuf, cnt)
        out = S.state_to_host(dev)
        ref = {k: v.copy() for k, v in pre.items()}
        orc.kick_drift(ref, p)
        for c in ("x", "y", "z"):
            assert np.array_equal(out[c], ref[c]), c
        # the new forces, sampled, against the oracle's sums over all N
        q = np.concatenate([rng.choice(n, 4096, replace=False), [0, n - 1]])
        ax, ay, az, pot, an = orc.gravity(ref["x"], ref["y"], ref["z"], ref["m"], 1.0,
                                          cfg["eps"], query=q, want_norm=True)
        hx, hy, hz, hp = orc.host_field(ref["x"][q], ref["y"][q], ref["z"][q], p)
        an = an + np.sqrt(hx ** 2 + hy ** 2 + hz ** 2)
        ea = np.sqrt((out["ax"][q] - ax - hx) ** 2 + (out["ay"][q] - ay - hy) ** 2 +
                     (out["az"][q] - az - hz) ** 2) / an
        ep = np.abs(out["pot"][q] - pot - hp) / np.abs(pot + hp)
        assert ea.max() < 1e-5 and ep.max() < 1e-5, (ea.max(), ep.max())
        # the closing kick with the GPU's accelerations, then h over all N
        for c in ("ax", "ay", "az", "pot"):
            ref[c] = out[c].copy()
        orc.close_kick(ref, p)
        ref["h"] = orc.knn_tree(ref["x"], ref["y"], ref["z"], ref["id"], cfg["k"])
        bad = np.flatnonzero(out["h"] != ref["h"])
        assert bad.size == 0, (step, bad.size)
        ev, marginal = event_parity(orc, got, ref, halo, step, 1e-9)
        assert marginal == 0
        orc.apply_events(ev, ref["m"], ref["vx"], ref["vy"], ref["vz"], 0, step)
        for c in ("vx", "vy", "vz"):
            e = np.max(np.abs(out[c] - ref[c])) / np.max(np.abs(ref[c]))
            assert e <= 1e-12, (step, c, e)
        print(f"step {step}: events {cnt} (oracle {ev.size}), forces {ea.max():.2e}, "
              f"|dE/E| {abs(E - E0) / abs(E0):.2e}", flush=True)
        checked += 1
    assert checked == 4
    assert abs(E - E0) / abs(E0) < 1e-6
    S.sidm_destroy(ctx)
