"""GPU parity of block time steps (Sec. 2: individual steps from the
gravitational criterion eta with a minimum step) against the oracle, through
the C ABI, with the step-wise protocol: each checked cycle starts from the
GPU's state (its accelerations included, so both sides start from the same
bins), and the oracle's cycle is compared with the GPU's.  FP64 bars: 1e-12
for positions and velocities relative to their largest magnitude, identical
event counts; the mixed path: 1e-5, where a particle whose bin decision lies
within the FP32 force error of a step boundary may take the other bin (at
most a few such particles are allowed)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

STEPS = dict(eta=0.025, max_bin=6)
XV = ("x", "y", "z", "vx", "vy", "vz")


@pytest.fixture(scope="module")
def S():
    import torch
    import paper_2506_06269_amd as S
    assert torch.cuda.is_available()
    S.lib()
    return S


def _params(orc, halo):
    return orc.make_params(G=halo.get("G", 1.0), eps=halo["eps"], sigma_m=halo["sigma_m"],
                           dt=halo["dt"], k=halo["k"], seed=halo.get("seed", 0),
                           host=halo.get("host"), boundary=halo.get("boundary"),
                           steps=halo.get("steps"))


def _start(S, s, halos, prec):
    import torch
    dev = S.state_to_device(s)
    ctx = S.sidm_create(0, s["x"].size, len(halos))
    S.sidm_gravity(ctx, halos, dev, prec)
    torch.cuda.synchronize()
    return ctx, dev


def _xv_errors(out, ref, sl=slice(None)):
    return {c: np.abs(out[c][sl] - ref[c]) / np.max(np.abs(ref[c])) for c in XV}


@pytest.mark.parametrize("prec", [0, 1])
def test_cycle_parity(S, orc, prec):
    """NFW halo, N = 6000, eps = 0.01, eta = 0.025, a cycle of dt = 1/16 in up
    to 64 ticks: bins 0..3 occupied, so most gravity i-blocks are skipped on
    most ticks."""
    import torch
    n = 6000
    s = W.nfw_halo(n, seed=71)
    halo = dict(n=n, eps=0.01, sigma_m=1.0, dt=1.0 / 16, k=32, seed=5, steps=STEPS)
    p = _params(orc, halo)
    ctx, dev = _start(S, s, [halo], prec)
    diag = S.diag_buffer(1)
    a0 = S.state_to_host(dev)
    bins = orc.time_bin(p, a0["ax"], a0["ay"], a0["az"])
    print("bins", np.bincount(bins), flush=True)
    assert len(set(bins.tolist())) >= 3 and bins.max() < STEPS["max_bin"]
    tol = 1e-12 if prec == 0 else 1e-5
    for cyc in range(2):
        ref = {k: v.copy() for k, v in S.state_to_host(dev).items()}
        ev = orc.kdk_step(ref, p, cyc)
        S.sidm_kdk_step(ctx, [halo], dev, cyc, prec, diag=diag)
        torch.cuda.synchronize()
        out = S.state_to_host(dev)
        d = S.read_diag(diag)[0]
        err = _xv_errors(out, ref)
        worst = max(e.max() for e in err.values())
        off = np.zeros(n, dtype=bool)
        for e in err.values():
            off |= e > tol
        print(f"cycle {cyc}: max err {worst:.3e}, over tol {off.sum()}, events gpu "
              f"{d['n_events']} oracle {ev.size}", flush=True)
        if prec == 0:
            assert not off.any()
            assert d["n_events"] == ev.size
            rel_h = np.abs(out["h"] - ref["h"]) / ref["h"]
            assert rel_h.max() <= 1e-12
        else:
            assert off.sum() <= 3
        assert d["status"] == 0
        assert ev.size > 0


@pytest.mark.parametrize("prec", [0, 1])
def test_max_bin_zero_is_the_fixed_step(S, prec):
    """eta > 0 with max_bin = 0 runs the cycle kernels (opening kick, one tick,
    the bin-aware finalize) and must give the fixed step's state bit for bit."""
    import torch
    n = 3000
    s = W.nfw_halo(n, seed=72)
    fixed = dict(n=n, eps=0.01, sigma_m=2.0, dt=2e-3, k=16, seed=6)
    cyc = dict(fixed, steps=dict(eta=0.025, max_bin=0))
    ctx_a, dev_a = _start(S, s, [fixed], prec)
    ctx_b, dev_b = _start(S, s, [cyc], prec)
    for step in range(3):
        S.sidm_kdk_step(ctx_a, [fixed], dev_a, step, prec)
        S.sidm_kdk_step(ctx_b, [cyc], dev_b, step, prec)
    torch.cuda.synchronize()
    a, b = S.state_to_host(dev_a), S.state_to_host(dev_b)
    for k in XV + ("ax", "ay", "az", "pot", "h"):
        assert np.array_equal(a[k], b[k]), k


def test_batch_with_different_max_bins(S, orc):
    """Three halos in one call: a fixed step (eta = 0), max_bin 2, and max_bin
    4 in the host with dt_min; each against its own oracle cycle (FP64)."""
    import torch
    sizes = [2000, 3000, 2500]
    parts = [W.plummer(sizes[0], seed=73), W.nfw_halo(sizes[1], seed=74),
             W.place_on_orbit(W.nfw_halo(sizes[2], seed=75))]
    s = {f: np.concatenate([q[f] for q in parts]) for f in ("x", "y", "z", "vx", "vy", "vz", "m")}
    s["id"] = np.concatenate([q["id"] for q in parts]).astype(np.uint32)
    offs = np.cumsum([0] + sizes[:-1])
    halos = [dict(offset=int(offs[0]), n=sizes[0], eps=0.02, sigma_m=1.0, dt=4e-3, k=16, seed=1),
             dict(offset=int(offs[1]), n=sizes[1], eps=0.01, sigma_m=1.0, dt=1.0 / 32, k=16,
                  seed=2, steps=dict(eta=0.025, max_bin=2)),
             dict(offset=int(offs[2]), n=sizes[2], eps=0.01, sigma_m=1.0, dt=1.0 / 16, k=32,
                  seed=3, host=W.host_params(), steps=dict(eta=0.025, max_bin=4, dt_min=1.0 / 128))]
    ctx, dev = _start(S, s, halos, 0)
    for cyc in range(2):
        before = S.state_to_host(dev)
        S.sidm_kdk_step(ctx, halos, dev, cyc, 0)
        torch.cuda.synchronize()
        out = S.state_to_host(dev)
        for h, o, n in zip(halos, offs, sizes):
            sl = slice(o, o + n)
            ref = {k: v[sl].copy() for k, v in before.items()}
            orc.kdk_step(ref, _params(orc, h), cyc)
            err = _xv_errors(out, ref, sl)
            for c, e in err.items():
                assert e.max() <= 1e-12, (o, c, e.max())


def test_pass_times_of_a_cycle(S):
    """With timing on, a cycle's pass times are readable; the tile pass holds
    the ticks and dominates."""
    import torch
    n = 4096
    s = W.nfw_halo(n, seed=76)
    halo = dict(n=n, eps=0.01, sigma_m=1.0, dt=1.0 / 16, k=32, seed=7, steps=STEPS)
    ctx, dev = _start(S, s, [halo], 1)
    S.sidm_enable_timing(ctx, True)
    S.sidm_kdk_step(ctx, [halo], dev, 0, 1)
    torch.cuda.synchronize()
    t = S.sidm_pass_times(ctx)
    print(t)
    vals = list(t.values()) if isinstance(t, dict) else list(t)
    assert all(v >= 0.0 for v in vals)


def test_block_step_arguments_rejected(S):
    s = W.nfw_halo(256, seed=77)
    dev = S.state_to_device(s)
    ctx = S.sidm_create(0, 256, 1)
    base = dict(n=256, eps=0.01, k=8, sigma_m=1.0, dt=1e-2)
    bad = [dict(eta=-0.1, max_bin=2), dict(eta=float("nan"), max_bin=2),
           dict(eta=0.025, max_bin=17), dict(eta=0.025, max_bin=-1),
           dict(eta=0.0, max_bin=3), dict(eta=0.025, max_bin=2, dt_min=-1.0),
           dict(eta=0.025, max_bin=2, dt_min=float("inf"))]
    for steps in bad:
        with pytest.raises(S.SidmError):
            S.sidm_kdk_step(ctx, [dict(base, steps=steps)], dev, 0, 0)


def test_full_size_block_workload(S):
    """The block-step benchmark's halo (isolated NFW N = 2^20, eps 0.01, k 64,
    sigma/m 1, mixed precision), properties that hold at any size: eta > 0
    with max_bin = 0 is the fixed step of the same dt bit for bit, and one
    cycle of 1/16 in up to 64 ticks keeps |dE/E| below 1e-5 with a valid
    status."""
    import torch
    cfg = W.config("BLK")
    n = cfg["n"]
    s = W.make_state(cfg)
    base = dict(n=n, eps=cfg["eps"], G=1.0, sigma_m=cfg["sigma_m"], k=cfg["k"], seed=0)
    fixed = dict(base, dt=1.0 / 1024)
    zero = dict(fixed, steps=dict(eta=cfg["steps_param"]["eta"], max_bin=0))
    ctx_a, dev_a = _start(S, s, [fixed], 1)
    ctx_b, dev_b = _start(S, s, [zero], 1)
    S.sidm_kdk_step(ctx_a, [fixed], dev_a, 0, 1)
    S.sidm_kdk_step(ctx_b, [zero], dev_b, 0, 1)
    torch.cuda.synchronize()
    a, b = S.state_to_host(dev_a), S.state_to_host(dev_b)
    for k in XV + ("ax", "ay", "az", "pot", "h"):
        assert np.array_equal(a[k], b[k]), k
    del dev_a, dev_b
    cyc = dict(base, dt=cfg["dt"], steps=cfg["steps_param"])
    ctx, dev = _start(S, s, [cyc], 1)
    diag = S.diag_buffer(1)
    S.sidm_diagnostics(ctx, [cyc], dev, diag)
    d0 = S.read_diag(diag)[0]
    S.sidm_kdk_step(ctx, [cyc], dev, 0, 1, diag=diag)
    torch.cuda.synchronize()
    d1 = S.read_diag(diag)[0]
    e0 = d0["K"] + d0["W"]
    e1 = d1["K"] + d1["W"]
    print(f"one cycle at N=2^20: |dE/E| {abs(e1 - e0) / abs(e0):.2e}, events {d1['n_events']}")
    assert abs(e1 - e0) / abs(e0) < 1e-5
    assert d1["status"] == 0 and d1["n_events"] > 0
