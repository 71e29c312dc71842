"""GPU parity of tree gravity (Sec. 2: the gravity tree with the relative
opening criterion; alpha = 5e-4 in the paper's runs) against the oracle's
tree, through the C ABI.  Both sides build the same tree (Morton order,
64-particle buckets, fan-out 8) and take the opening decisions in FP64 from
the same inputs, so the number of source terms must be equal exactly; forces
and potentials within 1e-12 (FP64) or 1e-5 (mixed) of the oracle's tree,
normwise against the direct-sum scale sum m r / (r^2 + eps^2)^(3/2).  A
group's walk runs in four parts that share out the subtrees below a frontier
level; the sizes put that level at the buckets (20 000 particles) and one
level above them (2^17), and leave the small halos in one part."""
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


def _with_old_accel(orc, s, eps, G=1.0):
    """The state with a_old = the direct-sum accelerations (the previous step's
    forces in a run)."""
    ax, ay, az, pot, an = orc.gravity(s["x"], s["y"], s["z"], s["m"], G, eps, want_norm=True)
    s = dict(s, ax=ax, ay=ay, az=az, pot=pot)
    return s, an


def _gravity_terms(S, ctx, halos, dev, prec):
    import torch
    S.sidm_gravity(ctx, halos, dev, prec)
    diag = S.diag_buffer(len(halos))
    S.sidm_diagnostics(ctx, halos, dev, diag)
    torch.cuda.synchronize()
    return [d["n_grav_terms"] for d in S.read_diag(diag)]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("n,alpha", [(20000, 5e-4), (20000, 2.5e-2), (2, 5e-4), (64, 5e-4),
                                     (65, 5e-4), (4097, 5e-3), (1 << 17, 5e-4)])
def test_tree_forces_match_the_oracle_tree(S, orc, prec, n, alpha):
    s0 = W.nfw_halo(max(n, 2), seed=91)
    s, an = _with_old_accel(orc, s0, 0.01)
    halo = dict(n=n, eps=0.01, G=1.0, tree_alpha=alpha)
    dev = S.state_to_device(s)
    ctx = S.sidm_create(0, n, 1)
    terms = _gravity_terms(S, ctx, [halo], dev, prec)[0]
    out = S.state_to_host(dev)
    tx, ty, tz, tp, oterms = orc.tree_gravity(s["x"], s["y"], s["z"], s["m"],
                                              (s["ax"], s["ay"], s["az"]), 1.0, 0.01, alpha)
    err = np.sqrt((out["ax"] - tx) ** 2 + (out["ay"] - ty) ** 2 + (out["az"] - tz) ** 2) / an
    ep = np.abs(out["pot"] - tp) / np.abs(tp)
    tol = 1e-12 if prec == 0 else 1e-5
    print(f"n {n} alpha {alpha} prec {prec}: terms {terms} (oracle {oterms}, direct "
          f"{((n + 63) // 64) * n}), max err {err.max():.2e}, pot {ep.max():.2e}")
    assert terms == oterms
    assert err.max() < tol and ep.max() < tol


def test_vanishing_alpha_is_the_direct_sum(S, orc):
    """alpha = 1e-300 opens every node: the tree walk gives the direct sum."""
    n = 9000
    s, an = _with_old_accel(orc, W.plummer(n, seed=92), 0.02)
    halo = dict(n=n, eps=0.02, G=1.0, tree_alpha=1e-300)
    dev = S.state_to_device(s)
    ctx = S.sidm_create(0, n, 1)
    terms = _gravity_terms(S, ctx, [halo], dev, 0)[0]
    out = S.state_to_host(dev)
    err = np.sqrt((out["ax"] - s["ax"]) ** 2 + (out["ay"] - s["ay"]) ** 2 +
                  (out["az"] - s["az"]) ** 2) / an
    assert terms == ((n + 63) // 64) * n
    assert err.max() < 1e-12
    assert np.max(np.abs(out["pot"] - s["pot"]) / np.abs(s["pot"])) < 1e-12


def test_batch_of_tree_and_direct_halos(S, orc):
    """A tree halo, a direct-sum halo and a tree halo in the host, one call."""
    import torch
    sizes = [5000, 3000, 6000]
    parts = [W.nfw_halo(sizes[0], seed=93), W.plummer(sizes[1], seed=94),
             W.place_on_orbit(W.nfw_halo(sizes[2], seed=95))]
    alphas = [5e-4, 0.0, 2.5e-3]
    hosts = [None, None, W.host_params()]
    st = {f: [] for f in ("x", "y", "z", "vx", "vy", "vz", "m", "id", "ax", "ay", "az", "pot")}
    norms = []
    for q, h in zip(parts, hosts):
        q2, an = _with_old_accel(orc, q, 0.01)
        if h is not None:
            hx, hy, hz, _ = orc.host_field(q["x"], q["y"], q["z"], orc.make_params(host=h))
            q2 = dict(q2, ax=q2["ax"] + hx, ay=q2["ay"] + hy, az=q2["az"] + hz)
        norms.append(an)
        for f in st:
            st[f].append(q2[f])
    s = {f: np.concatenate(v) for f, v in st.items()}
    s["id"] = s["id"].astype(np.uint32)
    offs = np.cumsum([0] + sizes[:-1])
    halos = [dict(offset=int(o), n=n, eps=0.01, G=1.0, tree_alpha=a, host=h)
             for o, n, a, h in zip(offs, sizes, alphas, hosts)]
    dev = S.state_to_device(s)
    ctx = S.sidm_create(0, sum(sizes), 3)
    terms = _gravity_terms(S, ctx, halos, dev, 0)
    torch.cuda.synchronize()
    out = S.state_to_host(dev)
    for b, (o, n, a, h, an) in enumerate(zip(offs, sizes, alphas, hosts, norms)):
        sl = slice(o, o + n)
        x, y, z, m = s["x"][sl], s["y"][sl], s["z"][sl], s["m"][sl]
        if a > 0:
            tx, ty, tz, tp, ot = orc.tree_gravity(x, y, z, m, (s["ax"][sl], s["ay"][sl],
                                                               s["az"][sl]), 1.0, 0.01, a)
            assert terms[b] == ot
        else:
            tx, ty, tz, tp = orc.gravity(x, y, z, m, 1.0, 0.01)
            assert terms[b] == 0
        if h is not None:
            hx, hy, hz, hp = orc.host_field(x, y, z, orc.make_params(host=h))
            tx, ty, tz, tp = tx + hx, ty + hy, tz + hz, tp + hp
            an = an + np.sqrt(hx ** 2 + hy ** 2 + hz ** 2)
        err = np.sqrt((out["ax"][sl] - tx) ** 2 + (out["ay"][sl] - ty) ** 2 +
                      (out["az"][sl] - tz) ** 2) / an
        assert err.max() < 1e-12, b


@pytest.mark.parametrize("steps", [None, dict(eta=0.025, max_bin=3)])
def test_step_with_tree(S, orc, steps):
    """FP64 steps (fixed, then cycles of block steps) with tree gravity:
    step-wise parity with the oracle's step (1e-12, identical events)."""
    import torch
    n = 6000
    s, _ = _with_old_accel(orc, W.nfw_halo(n, seed=96), 0.01)
    dt = 2e-3 if steps is None else 1.0 / 32
    halo = dict(n=n, eps=0.01, sigma_m=2.0, dt=dt, k=32, seed=4, tree_alpha=5e-4)
    if steps is not None:
        halo["steps"] = steps
    p = orc.make_params(eps=0.01, sigma_m=2.0, dt=dt, k=32, seed=4, tree_alpha=5e-4, steps=steps)
    dev = S.state_to_device(s)
    ctx = S.sidm_create(0, n, 1)
    diag = S.diag_buffer(1)
    for step in range(2):
        ref = {k: v.copy() for k, v in S.state_to_host(dev).items()}
        ev = orc.kdk_step(ref, p, step)
        S.sidm_kdk_step(ctx, [halo], dev, step, 0, diag=diag)
        torch.cuda.synchronize()
        out = S.state_to_host(dev)
        d = S.read_diag(diag)[0]
        print(f"step {step}: events {d['n_events']} (oracle {ev.size}), terms {d['n_grav_terms']}")
        assert d["n_events"] == ev.size
        assert d["n_grav_terms"] > 0
        for c in ("x", "y", "z", "vx", "vy", "vz"):
            assert np.max(np.abs(out[c] - ref[c])) <= 1e-12 * np.max(np.abs(ref[c])), (step, c)


def test_tree_alpha_rejected(S):
    s = W.nfw_halo(256, seed=97)
    dev = S.state_to_device(s)
    ctx = S.sidm_create(0, 256, 1)
    for bad in (-1e-3, float("nan"), float("inf")):
        with pytest.raises(S.SidmError):
            S.sidm_gravity(ctx, [dict(n=256, eps=0.01, tree_alpha=bad)], dev, 0)
