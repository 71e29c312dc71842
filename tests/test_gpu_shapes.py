"""Launch shapes of the direct-sum gravity tiles (i-particles per thread x
threads per block, plain or persistent with a work ticket): every shape gives
the oracle's forces to the usual bars (1e-12 FP64, 1e-5 mixed, normwise) on a
batch of uneven halos with a host; a step in a persistent shape matches the
oracle step-wise; the tuner times the shapes, caches its choice under the
device and size key, and reads it back."""
import json
import os

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


def _batch():
    # the smallest halo has the size of the smallest of the 64-halo batch; in a
    # sparser one (1500 particles) the mixed tiles' FP32 frame rounding
    # reaches 1.2e-5 normwise for a close pair, in every shape alike
    parts = [W.place_on_orbit(W.nfw_halo(6000, seed=71)), W.nfw_halo(20000, seed=72),
             W.nfw_halo(4096, seed=73)]
    halos, off = [], 0
    s = {f: np.concatenate([p[f] for p in parts]) for f in ("x", "y", "z", "vx", "vy", "vz",
                                                           "m", "id")}
    for i, p in enumerate(parts):
        n = p["x"].size
        h = dict(n=n, offset=off, eps=0.01, G=1.0, k=32, sigma_m=10.0, dt=1e-3, seed=i)
        if i == 0:
            h["host"] = W.host_params()
        halos.append(h)
        off += n
    return s, halos, parts


def _check_forces(orc, S, out, halos, parts, tol):
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
    assert worst < tol, worst
    return worst


@pytest.mark.parametrize("prec", [1, 0])
def test_every_shape_matches_the_oracle(S, orc, prec):
    import torch
    s, halos, parts = _batch()
    dev = S.state_to_device(s)
    ctx = S.sidm_create(0, s["x"].size, len(halos))
    tol = 1e-5 if prec == 1 else 1e-12
    for ireg, nt in S.SHAPES:
        for persistent in (False, True):
            S.sidm_set_launch_shape(ctx, ireg, nt, persistent)
            S.sidm_gravity(ctx, halos, dev, prec)
            torch.cuda.synchronize()
            w = _check_forces(orc, S, S.state_to_host(dev), halos, parts, tol)
            print(f"shape {ireg}x{nt} persistent={persistent}: {w:.2e}", flush=True)
    with pytest.raises(S.SidmError) as e:
        S.sidm_set_launch_shape(ctx, 3, 256)
    assert e.value.status == S.SIDM_ERR_UNSUPPORTED
    S.sidm_destroy(ctx)


def test_persistent_shape_step_parity(S, orc):
    """One mixed step of the batch in the persistent 2 x 128 shape from the
    GPU's state, against the oracle's step (events and kernel sizes exact)."""
    import torch
    s, halos, parts = _batch()
    dev = S.state_to_device(s)
    ctx = S.sidm_create(0, s["x"].size, len(halos))
    S.sidm_set_launch_shape(ctx, 2, 128, True)
    S.sidm_gravity(ctx, halos, dev, 1)
    torch.cuda.synchronize()
    before = S.state_to_host(dev)
    diag = S.diag_buffer(len(halos))
    S.sidm_kdk_step(ctx, halos, dev, 3, 1, diag=diag)
    torch.cuda.synchronize()
    out = S.state_to_host(dev)
    for b, h in enumerate(halos):
        o, n = h["offset"], h["n"]
        ref = {k: v[o:o + n].copy() for k, v in before.items()}
        p = orc.make_params(eps=h["eps"], sigma_m=h["sigma_m"], dt=h["dt"], k=h["k"],
                            seed=h["seed"], host=h.get("host"))
        ev = orc.kdk_step(ref, p, 3)
        d = S.read_diag(diag)[b]
        assert d["n_events"] == ev.size
        assert np.array_equal(out["h"][o:o + n], ref["h"])
        for c in ("vx", "vy", "vz"):
            assert np.max(np.abs(out[c][o:o + n] - ref[c])) <= 1e-7 * np.max(np.abs(ref[c]))
    S.sidm_destroy(ctx)


def test_tuner_times_caches_and_reads_back(S, orc, tmp_path):
    import torch
    s, halos, parts = _batch()
    dev = S.state_to_device(s)
    ctx = S.sidm_create(0, s["x"].size, len(halos))
    cache = str(tmp_path / "tiles.json")
    r = S.sidm_autotune(ctx, halos, dev, 1, cache, S.SIDM_TUNE_QUICK)
    torch.cuda.synchronize()
    print("tuned:", r, flush=True)
    assert r["from_cache"] == 0 and r["n_tried"] >= 9
    assert (r["ireg"], r["threads"]) in S.SHAPES
    assert 0 < r["ms"] <= r["ms_default"]
    _check_forces(orc, S, S.state_to_host(dev), halos, parts, 1e-5)
    entries = json.load(open(cache))
    assert entries[r["key"]]["ireg"] == r["ireg"]
    ctx2 = S.sidm_create(0, s["x"].size, len(halos))
    r2 = S.sidm_autotune(ctx2, halos, dev, 1, cache)
    assert r2["from_cache"] == 1 and (r2["ireg"], r2["threads"], r2["persistent"]) == \
        (r["ireg"], r["threads"], r["persistent"])
    # another precision is another key: timed again, added to the same file
    r3 = S.sidm_autotune(ctx2, halos, dev, 0, cache, S.SIDM_TUNE_QUICK)
    assert r3["from_cache"] == 0 and r3["key"] != r["key"]
    assert set(json.load(open(cache))) == {r["key"], r3["key"]}
    S.sidm_destroy(ctx)
    S.sidm_destroy(ctx2)
