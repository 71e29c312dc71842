"""GPU parity of sidm_central_density (Sec. 3: the halo centre is the
potential minimum) against the oracle.  The centre index is an argmin over
floating-point values: where the two sides see identical values (isolated
halos: the self-potential is pot itself) it must be identical; with a host
the device's own host potential enters, so the chosen particle must be a
minimum of the oracle's self-potential to rounding.  Counts are exact (same
distance expression); masses agree to summation rounding."""
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


def _setup(S, halos, s, prec=0):
    import torch
    dev = S.state_to_device(s)
    ctx = S.sidm_create(0, s["x"].size, len(halos))
    S.sidm_gravity(ctx, halos, dev, prec)
    torch.cuda.synchronize()
    return ctx, dev


def _one_hot(n, i):
    phi = np.zeros(n)
    phi[i] = -1.0
    return phi


def test_center_isolated_exact(S, orc):
    n = 8192
    s = W.nfw_halo(n, seed=21)
    halo = dict(n=n, eps=0.01, k=32, sigma_m=1.0, dt=1e-3)
    ctx, dev = _setup(S, [halo], s)
    pot = dev["pot"].cpu().numpy()
    for radius in (0.05, 0.1, 0.5, 3.0):
        got = S.sidm_central_density(ctx, [halo], dev, radius)[0]
        c, cnt, mass = orc.central_density(s["x"], s["y"], s["z"], s["m"], pot, radius)
        assert got["index"] == c
        assert (got["x"], got["y"], got["z"]) == (s["x"][c], s["y"][c], s["z"][c])
        assert got["count"] == cnt
        assert got["mass"] == pytest.approx(mass, rel=1e-12)
        print(f"r={radius}: centre {c}, count {cnt}")


def test_center_with_host_and_batch(S, orc):
    """Three halos in one call (one of them a satellite in the host), one
    radius each."""
    sizes = [3000, 5000, 2048]
    parts = [W.nfw_halo(sizes[0], seed=22), W.place_on_orbit(W.nfw_halo(sizes[1], seed=23)),
             W.plummer(sizes[2], seed=24)]
    s = {f: np.concatenate([p[f] for p in parts]) for f in ("x", "y", "z", "vx", "vy", "vz", "m")}
    s["id"] = np.concatenate([p["id"] for p in parts]).astype(np.uint32)
    offs = np.cumsum([0] + sizes[:-1])
    hosts = [None, W.host_params(), None]
    halos = [dict(offset=int(o), n=n, eps=0.01, k=16, sigma_m=1.0, dt=1e-3, host=h)
             for o, n, h in zip(offs, sizes, hosts)]
    radii = [0.2, 0.3, 0.25]
    ctx, dev = _setup(S, halos, s)
    pot = dev["pot"].cpu().numpy()
    res = S.sidm_central_density(ctx, halos, dev, radii)
    for b, (o, n, h, r, got) in enumerate(zip(offs, sizes, hosts, radii, res)):
        sl = slice(o, o + n)
        x, y, z, m = s["x"][sl], s["y"][sl], s["z"][sl], s["m"][sl]
        phi = pot[sl].copy()
        if h is not None:
            _, _, _, hp = orc.host_nfw(x, y, z, 1.0, h["rho_s"], h["r_s"], h["center"])
            phi -= hp
        li = got["index"] - o
        assert 0 <= li < n
        assert phi[li] <= phi.min() + 1e-12 * abs(phi.min()), b
        if h is None:
            assert li == int(np.argmin(phi))
        _, cnt, mass = orc.central_density(x, y, z, m, _one_hot(n, li), r)
        assert got["count"] == cnt, b
        assert got["mass"] == pytest.approx(mass, rel=1e-12)


def test_center_ties_first_index(S):
    """Equal potentials everywhere: the first particle of each halo."""
    import torch
    s = W.maxwell_box(1000, seed=25)
    halos = [dict(offset=0, n=600, eps=0.01, k=8, sigma_m=0.0, dt=1e-3),
             dict(offset=600, n=400, eps=0.01, k=8, sigma_m=0.0, dt=1e-3)]
    dev = S.state_to_device(s)
    dev["pot"].fill_(-3.0)
    ctx = S.sidm_create(0, 1000, 2)
    res = S.sidm_central_density(ctx, halos, dev, 10.0)
    torch.cuda.synchronize()
    assert [r["index"] for r in res] == [0, 600]
    assert [r["count"] for r in res] == [600, 400]


def test_center_rejects_bad_radius(S):
    s = W.maxwell_box(100, seed=26)
    dev = S.state_to_device(s)
    ctx = S.sidm_create(0, 100, 1)
    halo = dict(n=100, eps=0.01, k=8, sigma_m=0.0, dt=1e-3)
    for bad in (0.0, -1.0, float("nan"), float("inf")):
        with pytest.raises(S.SidmError):
            S.sidm_central_density(ctx, [halo], dev, bad)
