"""Failure detection through the device status word: a non-finite position
or velocity in a halo is reported in that halo's diagnostics (and only
there), forced from the host by writing NaN or infinity into the state; only
the diagnostics pass runs on such a state (every pass is bounded, but no
other result would mean anything)."""
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


@pytest.mark.parametrize("field,value", [("vx", float("nan")), ("z", float("inf")),
                                         ("vy", -float("inf"))])
def test_nonfinite_state_flagged_per_halo(S, field, value):
    import torch
    sizes = [1500, 2500]
    parts = [W.nfw_halo(sizes[0], seed=41), W.nfw_halo(sizes[1], seed=42)]
    s = {f: np.concatenate([q[f] for q in parts]) for f in ("x", "y", "z", "vx", "vy", "vz", "m")}
    s["id"] = np.arange(sum(sizes), dtype=np.uint32)
    halos = [dict(offset=0, n=sizes[0], eps=0.01, sigma_m=1.0, dt=1e-3, k=16),
             dict(offset=sizes[0], n=sizes[1], eps=0.01, sigma_m=1.0, dt=1e-3, k=16,
                  host=W.host_params())]
    dev = S.state_to_device(s)
    ctx = S.sidm_create(0, sum(sizes), 2)
    diag = S.diag_buffer(2)
    S.sidm_diagnostics(ctx, halos, dev, diag)
    torch.cuda.synchronize()
    # a context that has not stepped reports a clean status and no events
    for d in S.read_diag(diag):
        assert d["status"] == 0 and d["n_events"] == 0 and d["n_rounds"] == 0
        assert d["n_pairs"] == 0 and d["n_p_gt1"] == 0 and d["n_grav_terms"] == 0
    dev[field][sizes[0] + 17] = value
    S.sidm_diagnostics(ctx, halos, dev, diag)
    torch.cuda.synchronize()
    d0, d1 = S.read_diag(diag)
    assert d0["status"] == 0
    assert d1["status"] & S.SIDM_DEV_NONFINITE
    S.sidm_destroy(ctx)
