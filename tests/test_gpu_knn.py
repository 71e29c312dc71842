"""GPU parity of sidm_knn_h (kernel sizes from the k nearest neighbours)
against the oracle's brute force: h must match bit for bit (same FP64
distance expression without fused multiply-add, correctly rounded sqrt), and
the optional neighbour lists must equal the oracle's (d2, id)-ordered lists."""
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


def _gpu_knn(S, halos, s, want_list=False, ctx=None):
    import torch
    dev = S.state_to_device(s)
    n = s["x"].size
    ctx = ctx or S.sidm_create(0, n, len(halos))
    kmax = max(h["k"] for h in halos)
    nbr = torch.zeros(n * kmax, dtype=torch.int32, device="cuda") if want_list else None
    S.sidm_knn_h(ctx, halos, dev, nbr=nbr)
    torch.cuda.synchronize()
    h = dev["h"].cpu().numpy()
    lists = nbr.cpu().numpy().view(np.uint32).reshape(n, kmax) if want_list else None
    return h, lists


@pytest.mark.parametrize("kind,n,k", [("nfw", 8192, 32), ("random", 1000, 16), ("random", 33, 32),
                                      ("clustered", 3000, 128), ("lattice", 1000, 16),
                                      ("lattice", 512, 1), ("nfw", 4100, 64)])
def test_knn_bit_exact(S, orc, kind, n, k):
    if kind == "nfw":
        s = W.nfw_halo(n, seed=3)
    elif kind == "random":
        s = W.maxwell_box(n, seed=5)
    elif kind == "clustered":
        s = W.clustered(n, seed=8, width=0.005)
    else:
        s = W.lattice(round(n ** (1 / 3)), seed=4)
        n = s["x"].size
    print(f"knn {kind} n={n} k={k}", flush=True)
    halo = dict(n=n, eps=0.01, k=k)
    h, lists = _gpu_knn(S, [halo], s, want_list=n <= 8192)
    href, lref = orc.knn(s["x"], s["y"], s["z"], s["id"], k, want_list=True)
    bad = np.flatnonzero(h != href)
    assert bad.size == 0, (bad[:5], h[bad[:5]], href[bad[:5]])
    if lists is not None:
        assert np.array_equal(lists[:, :k], lref)


@pytest.mark.parametrize("kind,n,k", [("nfw", 8192, 32), ("clustered", 3000, 128),
                                      ("lattice", 1000, 16), ("lattice", 512, 6),
                                      ("nfw", 4100, 64), ("random", 1000, 16)])
def test_knn_warm_starts_bit_exact(S, orc, kind, n, k):
    """Warm starts from the exact kernel size and from sizes a little off
    (the band around the previous h holds the k-th distance, off its centre,
    or it does not and the general search takes over) give the oracle's h bit
    for bit and its lists; lattices put many equal distances into the band."""
    import torch
    if kind == "nfw":
        s = W.nfw_halo(n, seed=13)
    elif kind == "random":
        s = W.maxwell_box(n, seed=15)
    elif kind == "clustered":
        s = W.clustered(n, seed=18, width=0.005)
    else:
        s = W.lattice(round(n ** (1 / 3)), seed=14)
        n = s["x"].size
    href, lref = orc.knn(s["x"], s["y"], s["z"], s["id"], k, want_list=True)
    halo = dict(n=n, eps=0.01, k=k)
    dev = S.state_to_device(s)
    ctx = S.sidm_create(0, n, 1)
    nbr = torch.zeros(n * k, dtype=torch.int32, device="cuda")
    hr = torch.from_numpy(href).to("cuda")
    for f in (1.0, 0.995, 1.01, 0.97, 1.05, 0.8, 1.3):
        dev["h"].copy_(hr * f)
        S.sidm_knn_h(ctx, [halo], dev, nbr=nbr)
        torch.cuda.synchronize()
        h = dev["h"].cpu().numpy()
        bad = np.flatnonzero(h != href)
        assert bad.size == 0, (f, bad[:5], h[bad[:5]], href[bad[:5]])
        lists = nbr.cpu().numpy().view(np.uint32).reshape(n, k)
        assert np.array_equal(lists, lref), f
    S.sidm_destroy(ctx)


def test_knn_batched_mixed_k(S, orc):
    """Four halos (k = 16, 32, 64, 128) in one call, offsets not in order."""
    sizes = [4096, 5000, 6144, 4500]
    ks = [16, 32, 64, 128]
    offs = [11300, 0, 5100, 15500]
    total = 20000
    s = {f: np.zeros(total) for f in ("x", "y", "z", "vx", "vy", "vz")}
    s["m"] = np.ones(total)
    s["id"] = np.zeros(total, dtype=np.uint32)
    halos, parts = [], []
    for b, (n, k, o) in enumerate(zip(sizes, ks, offs)):
        p = W.nfw_halo(n, seed=20 + b)
        parts.append(p)
        for f in ("x", "y", "z", "vx", "vy", "vz", "m", "id"):
            s[f][o:o + n] = p[f]
        halos.append(dict(n=n, offset=o, eps=0.01, k=k))
    h, lists = _gpu_knn(S, halos, s, want_list=True)
    for p, hh in zip(parts, halos):
        ref, lref = orc.knn(p["x"], p["y"], p["z"], p["id"], hh["k"], want_list=True)
        sl = slice(hh["offset"], hh["offset"] + hh["n"])
        assert np.array_equal(h[sl], ref), hh
        assert np.array_equal(lists[sl, :hh["k"]], lref), hh


def test_knn_large_sampled(S, orc):
    """N = 2^20 halo in the host (the benchmark's workload), k = 64: h and the
    neighbour lists of 512 sampled particles against the oracle's brute force
    over all N."""
    cfg = W.config("C2")
    s = W.make_state(cfg)
    halo = dict(n=cfg["n"], eps=cfg["eps"], k=cfg["k"])
    h, lists = _gpu_knn(S, [halo], s, want_list=True)
    q = np.random.default_rng(1).choice(cfg["n"], 512, replace=False)
    ref, lref = orc.knn(s["x"], s["y"], s["z"], s["id"], cfg["k"], query=q, want_list=True)
    assert np.array_equal(h[q], ref)
    assert np.array_equal(lists[q], lref)
    assert np.all(np.isfinite(h)) and np.all(h > 0)


def test_knn_start_does_not_change_h(S):
    """The starting radius only decides how much work a call does: at the
    benchmark's N = 2^20, a call without a previous h (each sub-range's first
    member resolved from an estimate, the rest from it), a warm call from that
    h, a call from h scaled by 0.5 and by 3 (starts far off, which grow or
    select within a wide sphere) and from unusable values (NaN, negative,
    larger than the halo) all give the same h bit for bit."""
    import torch
    cfg = W.config("C2")
    s = W.make_state(cfg)
    n = cfg["n"]
    halo = dict(n=n, eps=cfg["eps"], k=cfg["k"])
    dev = S.state_to_device(s)
    ctx = S.sidm_create(0, n, 1)
    S.sidm_knn_h(ctx, [halo], dev)
    torch.cuda.synchronize()
    cold = dev["h"].clone()
    assert torch.all(torch.isfinite(cold)) and torch.all(cold > 0)
    starts = [lambda h: h, lambda h: 0.5 * h, lambda h: 3.0 * h,
              lambda h: torch.full_like(h, float("nan")), lambda h: -h,
              lambda h: torch.full_like(h, 1e6)]
    for i, f in enumerate(starts):
        dev["h"].copy_(f(cold))
        S.sidm_knn_h(ctx, [halo], dev)
        torch.cuda.synchronize()
        assert torch.equal(dev["h"], cold), i
    S.sidm_destroy(ctx)


def test_knn_coincident_particles(S, orc):
    """Exact duplicates: zero distances and ties everywhere."""
    base = W.maxwell_box(200, seed=2)
    s = {f: np.concatenate([base[f]] * 3) for f in ("x", "y", "z", "vx", "vy", "vz", "m")}
    s["id"] = np.random.default_rng(0).permutation(600).astype(np.uint32)
    for k in (1, 2, 5):
        halo = dict(n=600, eps=0.01, k=k)
        h, lists = _gpu_knn(S, [halo], s, want_list=True)
        href, lref = orc.knn(s["x"], s["y"], s["z"], s["id"], k, want_list=True)
        assert np.array_equal(h, href)
        assert np.array_equal(lists[:, :k], lref)


def test_knn_rejects_bad_k(S):
    s = W.maxwell_box(64, seed=0)
    dev = S.state_to_device(s)
    ctx = S.sidm_create(0, 64, 1)
    for k in (0, 64, 200):
        with pytest.raises(S.SidmError):
            S.sidm_knn_h(ctx, [dict(n=64, eps=0.1, k=k)], dev)
