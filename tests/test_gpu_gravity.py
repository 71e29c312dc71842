"""GPU parity of sidm_gravity against the FP64 oracle (through the C ABI).

Metric (normwise): e_i = |a_gpu - a_ref| / A_i with A_i = G sum_j m_j r_ij /
(r^2+eps^2)^{3/2} + |a_host|, because rounding errors scale with the sum of
the magnitudes of the pair terms, not with the (cancelling) net force.  The
potential uses |dphi| / |phi_ref|.  Bars: 1e-12 for the FP64 path, 1e-5 for
the mixed path (FP32 pair terms with compensated accumulation)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-5}


@pytest.fixture(scope="module")
def S():
    import torch
    import paper_2506_06269_amd as S
    assert torch.cuda.is_available()
    S.lib()
    return S


def _oracle(orc, s, halo, query=None):
    ax, ay, az, pot, an = orc.gravity(s["x"], s["y"], s["z"], s["m"], halo.get("G", 1.0),
                                      halo["eps"], query=query, want_norm=True)
    if halo.get("host") is not None:
        idx = np.arange(s["x"].size) if query is None else query
        H = halo["host"]
        hx, hy, hz, hp = orc.host_nfw(s["x"][idx], s["y"][idx], s["z"][idx], halo.get("G", 1.0),
                                      H["rho_s"], H["r_s"], H["center"])
        ax, ay, az, pot = ax + hx, ay + hy, az + hz, pot + hp
        an = an + np.sqrt(hx ** 2 + hy ** 2 + hz ** 2)
    return ax, ay, az, pot, an


def _errors(gpu, ref, idx):
    ax, ay, az, pot = (gpu[k][idx] for k in ("ax", "ay", "az", "pot"))
    rx, ry, rz, rp, an = ref
    da = np.sqrt((ax - rx) ** 2 + (ay - ry) ** 2 + (az - rz) ** 2) / an
    dp = np.abs(pot - rp) / np.abs(rp)
    return da, dp


def _run(S, halos, s, prec, ctx=None):
    import torch
    dev = S.state_to_device(s)
    ctx = ctx or S.sidm_create(0, s["x"].size, len(halos))
    S.sidm_gravity(ctx, halos, dev, prec)
    torch.cuda.synchronize()
    return S.state_to_host(dev)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("n", [2, 3, 257, 1000, 8192])
def test_gravity_small_full(S, orc, prec, n):
    s = W.nfw_halo(n, seed=n) if n > 8 else W.plummer(n, seed=1)
    halo = dict(n=n, eps=0.01, G=1.0)
    print(f"gravity n={n} prec={prec}", flush=True)
    out = _run(S, [halo], s, prec)
    ref = _oracle(orc, s, halo)
    da, dp = _errors(out, ref, np.arange(n))
    print(f"  max e_a={da.max():.3e}  p99.9={np.quantile(da, 0.999):.3e}  max e_phi={dp.max():.3e}")
    assert da.max() < TOL[prec]
    assert dp.max() < TOL[prec]


@pytest.mark.parametrize("prec", [0, 1])
def test_gravity_batched_with_host(S, orc, prec):
    """Three halos at scattered offsets (one in the host potential, far from
    the origin), with a gap of unused particles between them."""
    sizes, offs = [3000, 1500, 4100], [0, 3100, 4700]
    total = 8800
    hs = [W.nfw_halo(sizes[0], seed=1), W.place_on_orbit(W.nfw_halo(sizes[1], seed=2)),
          W.plummer(sizes[2], seed=3)]
    halos = [dict(n=sizes[0], offset=offs[0], eps=0.01, G=1.0),
             dict(n=sizes[1], offset=offs[1], eps=0.02, G=1.0, host=W.host_params()),
             dict(n=sizes[2], offset=offs[2], eps=0.05, G=2.0)]
    s = {f: np.zeros(total) for f in ("x", "y", "z", "vx", "vy", "vz")}
    s["m"] = np.ones(total)
    s["id"] = np.arange(total, dtype=np.uint32)
    for h, o, n in zip(hs, offs, sizes):
        for f in ("x", "y", "z", "vx", "vy", "vz", "m"):
            s[f][o:o + n] = h[f]
    out = _run(S, halos, s, prec)
    for h, hp, o, n in zip(hs, halos, offs, sizes):
        ref = _oracle(orc, h, hp)
        da, dp = _errors(out, ref, np.arange(o, o + n))
        print(f"halo n={n} max e_a={da.max():.3e} e_phi={dp.max():.3e}")
        assert da.max() < TOL[prec]
        assert dp.max() < TOL[prec]


def test_gravity_large_sampled(S, orc):
    """N = 2^20 halo in the host at its orbit radius, mixed precision, in the
    launch configuration of the benchmark; 384 sampled particles against the
    oracle's full sums; momentum of the self-gravity part."""
    import torch
    cfg = W.config("C2")
    s = W.make_state(cfg)
    halo = dict(n=cfg["n"], eps=cfg["eps"], G=1.0, host=cfg["host"])
    out = _run(S, [halo], s, 1)
    q = np.random.default_rng(0).choice(cfg["n"], 384, replace=False)
    q = np.concatenate([q, [0, cfg["n"] - 1]])
    ref = _oracle(orc, s, halo, query=q)
    da, dp = _errors(out, ref, q)
    print(f"C2 sampled: max e_a={da.max():.3e} e_phi={dp.max():.3e}")
    assert da.max() < TOL[1]
    assert dp.max() < TOL[1]
    del torch


def test_gravity_deterministic(S):
    s = W.nfw_halo(5000, seed=4)
    halo = dict(n=5000, eps=0.01)
    a = _run(S, [halo], s, 1)
    b = _run(S, [halo], s, 1)
    for f in ("ax", "ay", "az", "pot"):
        assert np.array_equal(a[f], b[f])


def test_gravity_rejects_bad_arguments(S):
    import torch
    s = W.plummer(64, seed=0)
    dev = S.state_to_device(s)
    ctx = S.sidm_create(0, 64, 1)
    with pytest.raises(S.SidmError) as e:
        S.sidm_gravity(ctx, [dict(n=64, eps=0.0)], dev, 1)
    assert e.value.status == S.SIDM_ERR_INVALID
    with pytest.raises(S.SidmError):
        S.sidm_gravity(ctx, [dict(n=128, eps=0.1)], dev, 1)   # beyond max_particles
    with pytest.raises(S.SidmError):
        S.sidm_gravity(ctx, [dict(n=1, eps=0.1)], dev, 1)
    torch.cuda.synchronize()
