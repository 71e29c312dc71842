"""The boundary's contract, forced from the host: a halo that scatters with
unequal masses or a repeated id is refused (not scattered, flagged, and
reported by the call or by the next one), an overflow of the event buffer is
reported by the next call when no diagnostics were asked for, and a captured
step replayed after a call outside capture with other state pointers is
flagged as stale.  Every kernel runs to its normal end in these tests."""
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


def _halo(n=3000, **kw):
    h = dict(n=n, eps=0.01, G=1.0, sigma_m=50.0, dt=1e-3, k=32, seed=3)
    h.update(kw)
    return h


def _setup(S, s, halo):
    import torch
    dev = S.state_to_device(s)
    ctx = S.sidm_create(0, s["x"].size, 1)
    S.sidm_gravity(ctx, [halo], dev, S.SIDM_PREC_FP64)
    S.sidm_knn_h(ctx, [halo], dev)
    torch.cuda.synchronize()
    return ctx, dev


@pytest.mark.parametrize("case", ["unequal_mass", "duplicate_id"])
def test_refused_halo(S, case):
    import torch
    s = W.nfw_halo(3000, seed=21)
    if case == "unequal_mass":
        s["m"] = s["m"].copy()
        s["m"][17] *= 1.5
        bit, code = S.SIDM_DEV_UNEQUAL_MASS, S.SIDM_ERR_UNSUPPORTED
    else:
        s["id"] = s["id"].copy()
        s["id"][1234] = s["id"][99]
        bit, code = S.SIDM_DEV_DUPLICATE_ID, S.SIDM_ERR_INVALID
    halo = _halo()
    ctx, dev = _setup(S, s, halo)
    v0 = dev["vx"].cpu().numpy().copy()
    # synchronous scatter: refused, no kick
    with pytest.raises(S.SidmError) as e:
        S.sidm_scatter(ctx, [halo], dev, 1, want_count=True)
    assert e.value.status == code
    assert np.array_equal(dev["vx"].cpu().numpy(), v0)
    # a step with diagnostics flags the halo and scatters nothing
    diag = S.diag_buffer(1)
    S.sidm_kdk_step(ctx, [halo], dev, 2, S.SIDM_PREC_FP64, diag=diag)
    torch.cuda.synchronize()
    d = S.read_diag(diag)[0]
    assert d["status"] & bit and d["n_events"] == 0
    # the next call reports it once (and does not run), the one after runs
    with pytest.raises(S.SidmError) as e:
        S.sidm_kdk_step(ctx, [halo], dev, 3, S.SIDM_PREC_FP64)
    assert e.value.status == code
    S.sidm_gravity(ctx, [halo], dev, S.SIDM_PREC_FP64)
    assert S.sidm_take_status(ctx) == 0
    # without scattering the same state is accepted
    quiet = dict(halo, sigma_m=0.0)
    S.sidm_kdk_step(ctx, [quiet], dev, 4, S.SIDM_PREC_FP64, diag=diag)
    torch.cuda.synchronize()
    assert S.read_diag(diag)[0]["status"] == 0
    assert S.sidm_take_status(ctx) == 0
    S.sidm_destroy(ctx)


def test_ids_unique_per_halo_only(S):
    """The same ids in two halos of a batch are allowed (halos are independent
    and each keys its own draws)."""
    import torch
    a, b = W.nfw_halo(2000, seed=22), W.nfw_halo(2000, seed=23)
    s = {f: np.concatenate([a[f], b[f]]) for f in ("x", "y", "z", "vx", "vy", "vz", "m", "id")}
    assert np.array_equal(a["id"], b["id"])
    halos = [_halo(2000, offset=0), _halo(2000, offset=2000, seed=4)]
    dev = S.state_to_device(s)
    ctx = S.sidm_create(0, 4000, 2)
    S.sidm_gravity(ctx, halos, dev, S.SIDM_PREC_FP64)
    S.sidm_knn_h(ctx, halos, dev)
    cnt = S.sidm_scatter(ctx, halos, dev, 1, want_count=True)
    torch.cuda.synchronize()
    assert cnt > 0
    S.sidm_destroy(ctx)


def test_overflow_reported_by_next_call(S):
    """An event buffer too small for the step, no diagnostics: the step
    returns at once; the next call finds the overflow and reports
    SIDM_ERR_CAPACITY without running; after a larger buffer the step runs."""
    import torch
    s = W.nfw_halo(3000, seed=24)
    halo = _halo(sigma_m=2000.0)
    ctx, dev = _setup(S, s, halo)
    S.sidm_set_event_capacity(ctx, 4)
    S.sidm_kdk_step(ctx, [halo], dev, 1, S.SIDM_PREC_FP64)
    torch.cuda.synchronize()
    x1 = dev["x"].cpu().numpy().copy()
    with pytest.raises(S.SidmError) as e:
        S.sidm_kdk_step(ctx, [halo], dev, 2, S.SIDM_PREC_FP64)
    assert e.value.status == S.SIDM_ERR_CAPACITY
    assert "overflow" in S.sidm_last_error(ctx)
    torch.cuda.synchronize()
    assert np.array_equal(dev["x"].cpu().numpy(), x1)   # the refused call did not run
    S.sidm_set_event_capacity(ctx, 1 << 16)
    diag = S.diag_buffer(1)
    S.sidm_kdk_step(ctx, [halo], dev, 2, S.SIDM_PREC_FP64, diag=diag)
    torch.cuda.synchronize()
    d = S.read_diag(diag)[0]
    assert d["status"] == 0 and d["n_events"] > 4
    assert S.sidm_take_status(ctx) == 0
    S.sidm_destroy(ctx)


def test_stale_graph_replay_flagged(S):
    """A step captured on state A replays cleanly; after a call outside
    capture on state B (other tensors) its replay is flagged; a capture whose
    halos and state differ from the last call outside capture is refused."""
    import torch
    s = W.nfw_halo(3000, seed=25)
    halo = _halo(sigma_m=5.0)
    ctx, dev_a = _setup(S, s, halo)
    diag = S.diag_buffer(1)
    stream = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        graph.capture_begin()
        S.sidm_kdk_step(ctx, [halo], dev_a, 7, S.SIDM_PREC_FP64, diag=diag)
        graph.capture_end()
    torch.cuda.synchronize()
    graph.replay()
    torch.cuda.synchronize()
    assert S.read_diag(diag)[0]["status"] == 0
    assert S.sidm_take_status(ctx) == 0
    dev_b = S.state_to_device(s)
    S.sidm_gravity(ctx, [halo], dev_b, S.SIDM_PREC_FP64)
    torch.cuda.synchronize()
    graph.replay()
    torch.cuda.synchronize()
    assert S.read_diag(diag)[0]["status"] & S.SIDM_DEV_STALE_GRAPH
    assert S.sidm_take_status(ctx) & S.SIDM_DEV_STALE_GRAPH
    # capturing with state A now (the last call outside capture used B) is refused
    graph2 = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        graph2.capture_begin()
        with pytest.raises(S.SidmError) as e:
            S.sidm_kdk_step(ctx, [halo], dev_a, 8, S.SIDM_PREC_FP64, diag=diag)
        graph2.capture_end()
    assert e.value.status == S.SIDM_ERR_INVALID
    torch.cuda.synchronize()
    S.sidm_destroy(ctx)
