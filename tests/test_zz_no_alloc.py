"""sidm_gravity_static (the gravity pass without a context, its scratch in the
library's fixed array) against sidm_gravity on the same halos, through the C
ABI: two calls in a row, the second with a smaller halo, in both precisions;
normwise 1e-12 (FP64) and 1e-5 (mixed) against the context entry point's
output (the same kernels on the same plan: equal bit for bit in practice);
device memory unchanged by repeated calls; the size limit and the tree
option refused."""
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


def _cases():
    big = W.place_on_orbit(W.nfw_halo(40000, seed=51))
    small = W.nfw_halo(5000, seed=52)
    return [(big, dict(n=40000, eps=0.01, G=1.0, host=W.host_params())),
            (small, dict(n=5000, eps=0.02, G=1.0))]


@pytest.mark.parametrize("prec", [0, 1])
def test_static_matches_context_gravity(S, orc, prec):
    import torch
    tol = 1e-12 if prec == 0 else 1e-5
    for s, halo in _cases():
        n = halo["n"]
        ref_dev = S.state_to_device(s)
        ctx = S.sidm_create(0, n, 1)
        S.sidm_gravity(ctx, [halo], ref_dev, prec)
        dev = S.state_to_device(s)
        S.sidm_gravity_static(halo, dev, prec)
        torch.cuda.synchronize()
        ref, got = S.state_to_host(ref_dev), S.state_to_host(dev)
        _, _, _, _, an = orc.gravity(s["x"], s["y"], s["z"], s["m"], 1.0, halo["eps"],
                                     want_norm=True)
        ea = np.sqrt((got["ax"] - ref["ax"]) ** 2 + (got["ay"] - ref["ay"]) ** 2 +
                     (got["az"] - ref["az"]) ** 2) / an
        ep = np.abs(got["pot"] - ref["pot"]) / np.abs(ref["pot"])
        same = all(np.array_equal(got[c], ref[c]) for c in ("ax", "ay", "az", "pot"))
        print(f"n={n} prec={prec}: max e_a {ea.max():.2e} e_phi {ep.max():.2e}, "
              f"identical {same}", flush=True)
        assert ea.max() <= tol and ep.max() <= tol
        for c in ("x", "y", "z", "vx", "m"):
            assert np.array_equal(got[c], s[c]), c
        S.sidm_destroy(ctx)


def test_static_allocates_nothing(S):
    import torch
    s, halo = _cases()[1]
    dev = S.state_to_device(s)
    S.sidm_gravity_static(halo, dev, 1)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for _ in range(3):
        S.sidm_gravity_static(halo, dev, 1)
        S.sidm_gravity_static(halo, dev, 0)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0


def test_static_limits(S):
    import torch
    s = W.nfw_halo(S.SIDM_STATIC_MAX_N + 1, seed=53)
    dev = S.state_to_device(s)
    with pytest.raises(S.SidmError) as e:
        S.sidm_gravity_static(dict(n=S.SIDM_STATIC_MAX_N + 1, eps=0.01), dev, 1)
    assert e.value.status == S.SIDM_ERR_CAPACITY
    assert "exceeds" in S.sidm_last_error(None)
    with pytest.raises(S.SidmError) as e:
        S.sidm_gravity_static(dict(n=1000, eps=0.01, tree_alpha=5e-4), dev, 1)
    assert e.value.status == S.SIDM_ERR_UNSUPPORTED
    with pytest.raises(S.SidmError) as e:
        S.sidm_gravity_static(dict(n=1000, eps=0.0), dev, 1)
    assert e.value.status == S.SIDM_ERR_INVALID
    torch.cuda.synchronize()
