"""Shared comparison helpers of the GPU parity tests (no arithmetic of the
method: the oracle computes every reference value)."""
import numpy as np


def event_parity(orc, got, pre, halo, step, marginal_tol, ref=None):
    """GPU events `got` (structured array with fields a, b) against the
    oracle's decisions on the pre-scatter state `pre` (dict of arrays with h):
    the (a, b) sets must be equal, except pairs whose draw u lies within
    marginal_tol * P of the oracle's P.  `ref`: the oracle's events if already
    computed.  Returns (oracle events, number of marginal mismatches)."""
    seed = halo.get("seed", 0)
    if ref is None:
        ref, _, _ = orc.find_events_tree(pre["x"], pre["y"], pre["z"], pre["vx"], pre["vy"],
                                         pre["vz"], pre["m"], pre["id"], pre["h"],
                                         halo["sigma_m"], halo["dt"], seed, step,
                                         sigma_w=halo.get("sigma_w", 0.0))
    rset = {(int(a), int(b)): (u, P) for a, b, u, P in zip(ref["a"], ref["b"], ref["u"], ref["P"])}
    gset = {(int(a), int(b)) for a, b in zip(got["a"], got["b"])}
    assert len(gset) == len(got), "an event appears twice"
    diff = gset ^ set(rset)
    idx_of = None
    marginal = 0
    for pair in diff:
        if pair in rset:
            u, P = rset[pair]
        else:
            if idx_of is None:
                idx_of = np.empty(int(pre["id"].max()) + 1, dtype=np.int64)
                idx_of[pre["id"]] = np.arange(pre["id"].size)
            ia, ib = idx_of[pair[0]], idx_of[pair[1]]
            d = np.sqrt((pre["x"][ia] - pre["x"][ib]) ** 2 + (pre["y"][ia] - pre["y"][ib]) ** 2 +
                        (pre["z"][ia] - pre["z"][ib]) ** 2)
            g = np.sqrt((pre["vx"][ia] - pre["vx"][ib]) ** 2 +
                        (pre["vy"][ia] - pre["vy"][ib]) ** 2 +
                        (pre["vz"][ia] - pre["vz"][ib]) ** 2)
            u = orc.accept_u(seed, step, *pair)
            P = orc.sigma(halo["sigma_m"], halo.get("sigma_w", 0.0), g) * pre["m"][ib] * g * \
                orc.lam(d, pre["h"][ia], pre["h"][ib]) * halo["dt"]
        assert abs(u - P) <= marginal_tol * P, (pair, u, P)
        marginal += 1
    return ref, marginal
