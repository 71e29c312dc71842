"""Accuracy of the tree gravity option against an independent reference.
The oracle's per-particle oct-tree follows the paper's statement of the
method (Sec. 2: a one-sided oct-tree opened with the relative criterion
G M l^2 <= alpha |a_old| r^4, alpha = 5e-4 for every run of Table 1); the
library's tree is a different design (the cell list's Morton tree of
64-particle buckets walked per bucket, with node quadrupoles).  On the
N = 2^20 benchmark satellite in its host, with the same a_old for both
(the library's pass that accepts every disjoint node, as its benchmark
seeds a run), the library's force errors against the oracle's direct sum
over all N (normwise, 2048 sampled particles) must be no larger than the
reference's at the same alpha in median and 99th percentile, and below
2e-3 everywhere."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec", [1, 0])
def test_tree_no_worse_than_the_papers_tree(orc, prec):
    import torch
    import paper_2506_06269_amd as S
    assert torch.cuda.is_available()
    cfg = W.config("C2")
    n, eps, alpha = cfg["n"], cfg["eps"], 5e-4
    s = W.make_state(cfg)
    halo = dict(n=n, eps=eps, G=1.0, k=cfg["k"], host=cfg["host"], tree_alpha=alpha)
    dev = S.state_to_device(s)
    ctx = S.sidm_create(0, n, 1)
    for f in ("ax", "ay", "az"):
        dev[f].fill_(1e300)
    S.sidm_gravity(ctx, [halo], dev, prec)
    torch.cuda.synchronize()
    a_old = [dev[f].cpu().numpy().copy() for f in ("ax", "ay", "az")]
    S.sidm_gravity(ctx, [halo], dev, prec)
    torch.cuda.synchronize()
    out = S.state_to_host(dev)
    S.sidm_destroy(ctx)
    q = np.random.default_rng(12).choice(n, 2048, replace=False)
    p = orc.make_params(G=1.0, eps=eps, host=cfg["host"])
    dx, dy, dz, dp, an = orc.gravity(s["x"], s["y"], s["z"], s["m"], 1.0, eps, query=q,
                                     want_norm=True)
    hx, hy, hz, hp = orc.host_field(s["x"][q], s["y"][q], s["z"][q], p)
    rx, ry, rz, rp, rterms = orc.octree_gravity(s["x"], s["y"], s["z"], s["m"], a_old, 1.0, eps,
                                                alpha, query=q)
    e_lib = np.sqrt((out["ax"][q] - hx - dx) ** 2 + (out["ay"][q] - hy - dy) ** 2 +
                    (out["az"][q] - hz - dz) ** 2) / an
    e_ref = np.sqrt((rx - dx) ** 2 + (ry - dy) ** 2 + (rz - dz) ** 2) / an
    stats = {k: (np.median(v), np.percentile(v, 99), v.max())
             for k, v in (("library", e_lib), ("paper tree", e_ref))}
    for k, (med, p99, mx) in stats.items():
        print(f"{k}: median {med:.2e} p99 {p99:.2e} max {mx:.2e}", flush=True)
    print(f"reference terms per particle {rterms / q.size:.0f}", flush=True)
    assert stats["library"][0] <= stats["paper tree"][0]
    assert stats["library"][1] <= stats["paper tree"][1]
    assert stats["library"][2] < 2e-3
