#!/usr/bin/env python3
"""Benchmark of the SIDM N-body step on one MI355X.

Workload: the N = 2^20 NFW halo (r_s = rho_s = G = 1, truncated at 10 r_s,
Eddington velocities) on a circular orbit at 20 host scale radii in a static
NFW host, Plummer softening 0.01, k = 64 neighbours, sigma/m = 10, dt = 1e-3,
mixed precision (FP32 gravity tiles with compensated accumulation, FP64
everything else).  A step is one full kick-drift-kick step with the kNN kernel
sizes and the scattering pass.  Inputs are synthetic and resident in HBM.

Prints one JSON line: gravity interactions per second of whole steps (value),
SIDM particle updates per second, |dE/E| over the run, the same for the
all-FP64 form, per-pass times from HIP events, the roofline of the dominant
kernel (the gravity tiles) and the CPU oracle on a bounded sample.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_PEAK_TFLOPS = 157.3      # MI355X vector FP32 (datasheet)
FP64_PEAK_TFLOPS = 78.6       # MI355X vector FP64 (datasheet)
FLOPS_PER_INTERACTION = 20    # 3 sub, 3 fma (r^2+eps^2), rsqrt, 4 mul/add, 3 fma
# the symmetric tiles evaluate an unordered pair once for both members: 3 sub,
# 3 fma, rsqrt, 2 mul, 3 fma + 1 add for each side = 26 flops, 13 per interaction
SYM_FLOPS_PER_INTERACTION = 13
SYM_MIN_N = 4096              # the library's default threshold of the symmetric tiles


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--fp64-steps", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--tune", action="store_true",
                    help="time every launch shape of the gravity tiles for the workload and "
                         "store the fastest in the tiles cache (default: read the cache only)")
    ap.add_argument("--symmetric-min-n", type=int, default=None, metavar="N",
                    help="halos of at least N particles take the symmetric tiles in mixed "
                         "precision (0: none; default: the library's 4096)")
    ap.add_argument("--shape", default=None, metavar="IxT[p]",
                    help="force a launch shape of the gravity tiles, e.g. 4x256 or 2x128p "
                         "(p: persistent)")
    ap.add_argument("--workload", default="C2",
                    choices=("C1", "C2", "C3", "C4", "C5", "BLK", "TREE"),
                    help="C2 (default, the benchmark line): N=2^20 satellite; C3: the same halo "
                         "for --steps steps in one --precision with |dE/E| and central density; "
                         "C4: 64-halo batch; C5: N=2^24 satellite, one step, per-pass rooflines; "
                         "BLK: N=2^20 isolated halo, --steps cycles of block time steps against "
                         "fixed steps of the deepest bin over the same time; TREE: the satellite "
                         "(N=--tree-n) with tree gravity, alpha=5e-4, against the direct sum")
    ap.add_argument("--tree-n", type=int, default=1 << 20,
                    help="TREE: particles (2^20: the C2 set-up; 2^24: the C5 set-up)")
    ap.add_argument("--precision", default="mixed", choices=("mixed", "fp64"),
                    help="precision of the C3 run")
    ap.add_argument("--set", action="append", default=[], metavar="KEY=VALUE",
                    help="C2 and C3: override a field of the workload (n, eps, dt, sigma_m, k, "
                         "seed, r_cut); the output's config lists the overrides, and no "
                         "counter-based traffic figure is reported for an overridden run")
    ap.add_argument("--log-jsonl", default=None, metavar="PATH",
                    help="append one JSON line per timed step and halo (energies, momentum, "
                         "events, rounds, pairs, P > 1, status, pass times); each line reads "
                         "the diagnostics back, one more wait per step")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="also run one plain device-to-device copy of BYTES bytes (a reference "
                         "dispatch for scaling HBM byte counters)")
    return ap.parse_args()


_OVERRIDABLE = {"n": int, "k": int, "seed": int, "eps": float, "dt": float, "sigma_m": float,
                "r_cut": float}


def _apply_overrides(cfg, sets):
    """Applies --set KEY=VALUE items to a workload config; returns them."""
    ov = {}
    for item in sets:
        key, sep, val = item.partition("=")
        if not sep or key not in _OVERRIDABLE:
            raise SystemExit(f"--set {item!r}: expected KEY=VALUE with KEY one of "
                             f"{', '.join(sorted(_OVERRIDABLE))}")
        ov[key] = _OVERRIDABLE[key](val)
    cfg.update(ov)
    return ov


def _energy(d):
    return d["K"] + d["W"] + d["Eext"]


def _internal_energy(d, mass):
    """K relative to the halo's centre-of-mass motion plus W: the halo's own
    energy, without its orbit in the host (which dominates E for a satellite)."""
    p2 = d["px"] ** 2 + d["py"] ** 2 + d["pz"] ** 2
    return d["K"] - 0.5 * p2 / mass + d["W"]


_TUNE = {"mode": "cache", "shape": None, "sym_min_n": None}   # set from the command line


def _tiles(S, ctx, halos, dev, prec):
    """Launch shape of the gravity tiles for this run: forced, timed (--tune,
    stored in the cache) or read from the cache (default; without an entry the
    default shape).  Computes the initial forces.  Returns the tuner's record."""
    if _TUNE["sym_min_n"] is not None:
        S.sidm_set_symmetric(ctx, _TUNE["sym_min_n"])
    if _TUNE["shape"]:
        spec = _TUNE["shape"]
        i, t = spec.rstrip("p").split("x")
        S.sidm_set_launch_shape(ctx, int(i), int(t), spec.endswith("p"))
        S.sidm_gravity(ctx, halos, dev, prec)
        return {"ireg": int(i), "threads": int(t), "persistent": int(spec.endswith("p")),
                "source": "forced"}
    flags = S.SIDM_TUNE_FORCE if _TUNE["mode"] == "tune" else S.SIDM_TUNE_CACHE_ONLY
    r = S.sidm_autotune(ctx, halos, dev, prec, S.TILES_CACHE, flags)
    r["source"] = "timed" if r["n_tried"] else ("cache" if r["from_cache"] else "default")
    return r


def _halo_of(cfg):
    return dict(n=cfg["n"], eps=cfg["eps"], G=1.0, sigma_m=cfg["sigma_m"], dt=cfg["dt"],
                k=cfg["k"], seed=cfg["seed"], host=cfg["host"])


_LOG = None   # open file of --log-jsonl, or None


def _log_step(S, run_label, step, dl, e0, passes):
    for h, d in enumerate(dl):
        rec = {"run": run_label, "step": step, "halo": h, "E": _energy(d),
               "dE_over_E0": (_energy(d) - e0[h]) / abs(e0[h]) if e0[h] else None}
        rec.update({k: d[k] for k in ("K", "W", "Eext", "px", "py", "pz", "n_events",
                                      "n_rounds", "n_pairs", "n_p_gt1", "n_candidates", "status",
                                      "n_grav_terms")})
        rec["pass_ms"] = passes
        _LOG.write(json.dumps(rec) + "\n")
    _LOG.flush()


def _run(S, torch, halos, s, prec, steps, warmup, timing, progress=False, graph_replays=0):
    n = s["x"].size
    dev = S.state_to_device(s)
    ctx = S.sidm_create(0, n, len(halos))
    diag = S.diag_buffer(len(halos))
    tiles = _tiles(S, ctx, halos, dev, prec)
    _run.tiles = tiles
    S.sidm_diagnostics(ctx, halos, dev, diag)
    d0 = S.read_diag(diag)
    e0_each = [_energy(d) for d in d0]
    e0 = sum(e0_each)
    mass0 = float(s["m"][halos[0].get("offset", 0):halos[0].get("offset", 0) + halos[0]["n"]].sum())
    ei0 = _internal_energy(d0[0], mass0)
    run_label = f"{'fp64' if prec == S.SIDM_PREC_FP64 else 'mixed'} n={n} halos={len(halos)}"
    if progress:
        print("initial forces done", file=sys.stderr, flush=True)
    step = 0
    for _ in range(warmup):
        S.sidm_kdk_step(ctx, halos, dev, step, prec, diag=diag)
        step += 1
    if timing:
        S.sidm_enable_timing(ctx, True)
    passes = {}
    events = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        S.sidm_kdk_step(ctx, halos, dev, step, prec, diag=diag)
        step += 1
        pt = S.sidm_pass_times(ctx) if timing else {}
        for k, v in pt.items():
            passes[k] = passes.get(k, 0.0) + v
        if _LOG is not None:
            _log_step(S, run_label, step - 1, S.read_diag(diag), e0_each, pt)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dl = S.read_diag(diag)
    d = dl[0]
    events = sum(x["n_events"] for x in dl)
    rel_e = abs(sum(_energy(x) for x in dl) - e0) / abs(e0)
    _run.rel_e_internal = abs(_internal_energy(d, mass0) - ei0) / abs(ei0)
    _run.last = {k: sum(x[k] for x in dl) for k in ("n_pairs", "n_candidates", "n_p_gt1")}
    for k in passes:
        passes[k] /= steps
    _run.graph_ms = None
    if graph_replays > 0:
        # the same step captured once in a HIP graph and replayed (the step
        # index, and so the draws, are those of the captured call)
        S.sidm_enable_timing(ctx, False)
        S.sidm_diagnostics(ctx, halos, dev, diag)
        torch.cuda.synchronize()
        stream = torch.cuda.Stream()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.stream(stream):
            graph.capture_begin()
            S.sidm_kdk_step(ctx, halos, dev, step, prec, diag=diag)
            graph.capture_end()
        graph.replay()
        torch.cuda.synchronize()
        g0 = time.perf_counter()
        for _ in range(graph_replays):
            graph.replay()
        torch.cuda.synchronize()
        _run.graph_ms = (time.perf_counter() - g0) / graph_replays * 1e3
        del graph
    S.sidm_destroy(ctx)
    return (t1 - t0) / steps, rel_e, passes, d, events


def _cpu_baseline(cfg, s, budget_s):
    """The oracle as it stands, on a bounded sample of the same workload: the
    full per-particle work (gravity against all N, brute-force kNN, pair tests
    with probabilities) for a random subset of particles, extrapolated to N."""
    import numpy as np
    from oracle import oracle as O
    n = cfg["n"]
    rng = np.random.default_rng(0)

    order = rng.permutation(n)
    used = 0

    def sample_seconds(m):
        nonlocal used
        q = np.sort(order[used:used + m])
        used += m
        t = time.perf_counter()
        O.gravity(s["x"], s["y"], s["z"], s["m"], 1.0, cfg["eps"], query=q)
        tg = time.perf_counter() - t
        t = time.perf_counter()
        h = O.knn(s["x"], s["y"], s["z"], s["id"], cfg["k"], query=q)
        tk = time.perf_counter() - t
        hh = np.full(n, float(np.median(h)))
        hh[q] = h
        qm = np.zeros(n, np.uint8)
        qm[q] = 1
        t = time.perf_counter()
        O.find_events(s["x"], s["y"], s["z"], s["vx"], s["vy"], s["vz"], s["m"], s["id"], hh,
                      cfg["sigma_m"], cfg["dt"], 0, 0, qmask=qm)
        ts = time.perf_counter() - t
        return np.array([tg, tk, ts])

    def sample_until(budget, first=16):
        # batches of doubling size, all counted, until the next batch would
        # pass the budget; every particle is drawn once
        total, m, batch = np.zeros(3), 0, first
        while True:
            dt = sample_seconds(batch)
            total += dt
            m += batch
            if total.sum() + 2.0 * dt.sum() > budget or used + 2 * batch > n:
                return float(total.sum()) / m, total, m
            batch *= 2

    per, parts, m = sample_until(budget_s)
    step_s = per * n
    cores = O.num_threads()
    # the same per-particle work on one thread, on a sample of about a fifth of
    # the budget, for the oracle's parallel speed-up
    O.set_threads(1)
    try:
        per1, _, m1 = sample_until(0.2 * budget_s, first=4)
    finally:
        O.set_threads(cores)
    return {
        "value": n * (n - 1) / step_s,
        "unit": "gravity interactions/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"{m} random particles of the N={n} halo: gravity against all N, brute-force "
                   f"kNN and pair tests with probabilities ({parts[0]:.1f} s, {parts[1]:.1f} s, "
                   f"{parts[2]:.1f} s), extrapolated to a full step of N particles"),
        "step_seconds_extrapolated": step_s,
        "single_thread_value": n * (n - 1) / (per1 * n),
        "single_thread_sample": m1,
        "host_cpu": _host_cpu(),
    }


def _host_cpu():
    """Model name and logical CPU count of the host, from /proc/cpuinfo."""
    try:
        with open("/proc/cpuinfo") as f:
            names = [ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")]
    except OSError:
        names = []
    return {"model": names[0] if names else None, "logical_cpus": len(names) or os.cpu_count(),
            "affinity": len(os.sched_getaffinity(0))}


def _kernel_source_sha():
    """SHA-256 of the gravity kernels' sources: the kernels, the constants they
    are compiled with and the planner that cuts their work items."""
    h = hashlib.sha256()
    for name in ("k_gravity.hip", "sidm_internal.hpp", "sidm_plan.hpp"):
        with open(os.path.join(ROOT, "paper_2506_06269_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _traffic(per_launch_flops):
    """HBM bytes per launch of the gravity tiles from committed rocprofv3
    counter runs, if taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic_grav_mixed_c2.json")
    try:
        with open(path) as f:
            rec = json.load(f)
        h = _kernel_source_sha()
        if rec.get("kernel_source_sha256") != h:
            return None
        return rec.get("bytes_per_launch")
    except (OSError, ValueError):
        return None


def _pass_rooflines(passes, n, inter, k):
    """Per-pass rates for the one-step workloads: the gravity tiles against the
    FP32 vector peak, the searches against HBM with their algorithmic bytes
    (kNN: 24 B of position in + 8 B of h out per particle; pair pass: x, v, h, id
    and m = 60 B per particle)."""
    g = passes["gravity_tiles"] * 1e-3
    return {
        "gravity_tiles": {"bound": "alu", "achieved": FLOPS_PER_INTERACTION * inter / g / 1e12,
                          "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                          "frac": FLOPS_PER_INTERACTION * inter / g / 1e12 / FP32_PEAK_TFLOPS},
        "knn": {"algorithmic_GBps": 32 * n / (passes["knn"] * 1e-3) / 1e9, "peak": 8000.0,
                "unit": "GB/s", "frac": 32 * n / (passes["knn"] * 1e-3) / 1e9 / 8000.0},
        "pairs": {"algorithmic_GBps": 60 * n / (passes["pairs"] * 1e-3) / 1e9, "peak": 8000.0,
                  "unit": "GB/s", "frac": 60 * n / (passes["pairs"] * 1e-3) / 1e9 / 8000.0},
    }


def _bench_c3(a, S, torch, W):
    """The N = 2^20 satellite for --steps steps in one precision: throughput,
    |dE/E| every 100 steps and the central density within 0.1 r_s of the
    potential minimum (Sec. 3) at the start and every 100 steps."""
    cfg = W.config("C3")
    overrides = _apply_overrides(cfg, a.set)
    n, radius = cfg["n"], 0.1
    s = W.make_state(cfg)
    halo = _halo_of(cfg)
    prec = S.SIDM_PREC_FP64 if a.precision == "fp64" else S.SIDM_PREC_MIXED
    dev = S.state_to_device(s)
    ctx = S.sidm_create(0, n, 1)
    diag = S.diag_buffer(1)
    tiles = _tiles(S, ctx, [halo], dev, prec)
    S.sidm_diagnostics(ctx, [halo], dev, diag)
    d0 = S.read_diag(diag)[0]
    e0 = _energy(d0)
    mass = float(s["m"].sum())
    ei0 = _internal_energy(d0, mass)
    vol = 4.0 / 3.0 * math.pi * radius ** 3

    def center(step):
        c = S.sidm_central_density(ctx, [halo], dev, radius)[0]
        return dict(step=step, count=c["count"], rho=c["mass"] / vol, index=c["index"])

    centers, energy = [center(0)], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for step in range(a.steps):
        S.sidm_kdk_step(ctx, [halo], dev, step, prec, diag=diag)
        if _LOG is not None:
            _log_step(S, f"C3 {a.precision}", step, S.read_diag(diag), [e0], {})
        if (step + 1) % 100 == 0 or step + 1 == a.steps:
            d = S.read_diag(diag)[0]
            energy.append(dict(step=step + 1, dE_over_E=abs(_energy(d) - e0) / abs(e0),
                               dEint_over_Eint=abs(_internal_energy(d, mass) - ei0) / abs(ei0),
                               events=d["n_events"], status=d["status"]))
            centers.append(center(step + 1))
            print(f"C3 {a.precision} step {step + 1}: |dE/E| {energy[-1]['dE_over_E']:.3e} "
                  f"internal {energy[-1]['dEint_over_Eint']:.3e} "
                  f"rho(<{radius}) {centers[-1]['rho']:.4g} ({centers[-1]['count']}) "
                  f"{time.perf_counter() - t0:.0f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / a.steps
    S.sidm_destroy(ctx)
    inter = n * (n - 1)
    out = {"metric": f"C3 {a.precision}: gravity interactions/s over {a.steps} steps, |dE/E|, "
                     f"central density", "value": inter / ms, "unit": "gravity interactions/s",
           "n_gpus": 1, "steps": a.steps, "warmup": 0, "ms_per_step": ms * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if a.precision == "fp64" else "f32 gravity tiles (compensated), "
                                                         "f64 elsewhere",
           "data": "synthetic NFW halo",
           "config": {"workload": "C3: NFW N=2^20 satellite in the host, eps=0.01, k=64, "
                                  "sigma/m=10, dt=1e-3", "precision": a.precision,
                      **({"overrides": overrides} if overrides else {})},
           "dE_over_E": energy[-1]["dE_over_E"] if energy else None,
           "dEint_over_Eint": energy[-1]["dEint_over_Eint"] if energy else None,
           "tiles": tiles,
           "max_dE_over_E": max((e["dE_over_E"] for e in energy), default=None),
           "energy": energy, "central_density": centers, "radius": radius}
    print(json.dumps(out), flush=True)


def _bench_c1(a, S, torch, W):
    """C1 (N = 8192, FP64, isolated, k = 32, sigma/m = 1, dt = 1e-3): the
    latency of one step, eager (one call per step) and replayed from a HIP
    graph captured from one call, over its 32 steps."""
    cfg = W.config("C1")
    n = cfg["n"]
    s = W.nfw_halo(n, seed=0)
    halo = dict(n=n, eps=cfg["eps"], G=1.0, sigma_m=cfg["sigma_m"], dt=cfg["dt"], k=cfg["k"],
                seed=0)
    steps = 32
    dev = S.state_to_device(s)
    ctx = S.sidm_create(0, n, 1)
    diag = S.diag_buffer(1)
    tiles = _tiles(S, ctx, [halo], dev, S.SIDM_PREC_FP64)
    for st in range(3):
        S.sidm_kdk_step(ctx, [halo], dev, st, S.SIDM_PREC_FP64, diag=diag)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for st in range(steps):
        S.sidm_kdk_step(ctx, [halo], dev, st, S.SIDM_PREC_FP64, diag=diag)
    torch.cuda.synchronize()
    eager = (time.perf_counter() - t0) / steps
    stream = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    S.sidm_diagnostics(ctx, [halo], dev, diag)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        graph.capture_begin()
        S.sidm_kdk_step(ctx, [halo], dev, 0, S.SIDM_PREC_FP64, diag=diag)
        graph.capture_end()
    for _ in range(3):
        graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        graph.replay()
    torch.cuda.synchronize()
    replay = (time.perf_counter() - t0) / steps
    S.sidm_destroy(ctx)
    inter = n * (n - 1)
    out = {"metric": "per-step latency of the C1 step (FP64)", "value": eager * 1e3,
           "unit": "ms/step", "n_gpus": 1, "steps": steps, "warmup": 3,
           "ms_per_step": eager * 1e3, "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic NFW halo",
           "config": {"workload": "C1: isolated NFW N=8192, eps=0.01, k=32, sigma/m=1, "
                                  "dt=1e-3, FP64", "n": n},
           "graph_replay_ms_per_step": replay * 1e3,
           "interactions_per_s_eager": inter / eager, "tiles": tiles}
    print(json.dumps(out), flush=True)


def _bench_c4(a, S, torch, W):
    """64 independent halos in one call per pass (uneven N, sigma/m, k)."""
    import numpy as np
    hl = W.batch_c4()
    total = sum(h["n"] for h in hl)
    s = {f: np.zeros(total) for f in ("x", "y", "z", "vx", "vy", "vz", "m")}
    s["id"] = np.zeros(total, dtype=np.uint32)
    halos, off = [], 0
    for h in hl:
        p = W.nfw_halo(h["n"], seed=h["seed"])
        for f in ("x", "y", "z", "vx", "vy", "vz", "m", "id"):
            s[f][off:off + h["n"]] = p[f]
        halos.append(dict(h, offset=off))
        off += h["n"]
    inter = sum(h["n"] * (h["n"] - 1) for h in hl)
    ms, de, passes, _, events = _run(S, torch, halos, s, S.SIDM_PREC_MIXED, a.steps, a.warmup,
                                     True, graph_replays=a.steps)
    out = {"metric": "gravity interactions/s + SIDM particle-updates/s (64-halo batch)",
           "value": inter / ms, "unit": "gravity interactions/s", "n_gpus": 1,
           "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32 gravity tiles (compensated), f64 elsewhere",
           "data": "synthetic NFW halos", "config": {"workload": "C4: 64 NFW halos, N 4096..131072, "
                                                                  "sigma/m {1,10,50}, k {16..128}",
                                                     "n_total": total, "halos": 64},
           "sidm_particle_updates_per_s": total / ms, "dE_over_E": de, "events_last_step": events,
           "pass_ms": passes, "tiles": _run.tiles, "graph_replay_ms_per_step": _run.graph_ms}
    print(json.dumps(out), flush=True)


def _bench_c5(a, S, torch, W):
    """N = 2^24 satellite (eps = 0.002), one full step, per-pass rooflines."""
    cfg = W.config("C5")
    n = cfg["n"]
    print(f"C5: generating N={n}", file=sys.stderr, flush=True)
    s = W.make_state(cfg)
    inter = n * (n - 1)
    print("C5: initial forces and one timed step", file=sys.stderr, flush=True)
    ms, de, passes, _, events = _run(S, torch, [_halo_of(cfg)], s, S.SIDM_PREC_MIXED, 1, 0, True,
                                     progress=True)
    out = {"metric": "gravity interactions/s + SIDM particle-updates/s (N=2^24, one step)",
           "value": inter / ms, "unit": "gravity interactions/s", "n_gpus": 1, "steps": 1,
           "warmup": 0, "ms_per_step": ms * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32 gravity tiles (compensated), f64 elsewhere",
           "data": "synthetic NFW halo", "config": {"workload": "C5: NFW N=2^24 satellite, "
                                                                "eps=0.002, k=64, sigma/m=10"},
           "sidm_particle_updates_per_s": n / ms, "dE_over_E": de, "events_last_step": events,
           "pass_ms": passes, "rooflines": _pass_rooflines(passes, n, inter, cfg["k"])}
    print(json.dumps(out), flush=True)


def _bench_blk(a, S, torch, W):
    """Block time steps on the N = 2^20 isolated halo: --steps cycles of 1/16,
    then fixed steps of 1/256 (the deepest bin the criterion fills here) over
    the same simulated time, both in mixed precision from the same state;
    simulated time per second and |dE/E| of each."""
    cfg = W.config("BLK")
    n = cfg["n"]
    s = W.make_state(cfg)
    halo = dict(_halo_of(cfg), steps=cfg["steps_param"])
    ms_c, de_c, passes, d, ev = _run(S, torch, [halo], s, S.SIDM_PREC_MIXED, a.steps, a.warmup,
                                     True, progress=True)
    print(f"BLK: {a.steps} cycles, {ms_c * 1e3:.1f} ms each, |dE/E| {de_c:.3e}", file=sys.stderr,
          flush=True)
    sub = 16
    fixed = dict(_halo_of(cfg), dt=cfg["dt"] / sub)
    ms_f, de_f, p_f, _, _ = _run(S, torch, [fixed], s, S.SIDM_PREC_MIXED, a.steps * sub,
                                 a.warmup * sub, True, progress=True)
    out = {"metric": "simulated time per second, block time steps vs fixed steps (N=2^20)",
           "value": cfg["dt"] / ms_c, "unit": "code time units/s", "n_gpus": 1,
           "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms_c * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32 gravity tiles (compensated), f64 elsewhere",
           "data": "synthetic NFW halo",
           "config": {"workload": "BLK: isolated NFW N=2^20, eps=0.01, k=64, sigma/m=1, block "
                                  "steps eta=0.025, cycle 1/16 in up to 64 ticks",
                      "n": n, "cycle": cfg["dt"], **cfg["steps_param"]},
           "dE_over_E": de_c, "events_last_cycle": ev, "status": d["status"], "pass_ms": passes,
           "fixed_step": {"dt": cfg["dt"] / sub, "steps": a.steps * sub,
                          "ms_per_step": ms_f * 1e3, "time_per_s": cfg["dt"] / sub / ms_f,
                          "dE_over_E": de_f, "pass_ms": p_f},
           "speedup_vs_fixed": (ms_f * sub) / ms_c}
    print(json.dumps(out), flush=True)


def _bench_tree(a, S, torch, W):
    """Tree gravity (relative criterion, alpha = 5e-4, Sec. 2) on the satellite
    in the host: force errors of the first tree evaluation against the GPU's
    direct sum on the same state, then --steps steps with the tree and with the
    direct sum from the same state (mixed precision), time and |dE/E| of each.
    The measured tree evaluation takes a_old from a tree pass whose own a_old
    came from a pass that accepts every node whose box is disjoint from the
    group's (a_old = 1e300)."""
    import numpy as np
    cfg = W.config("C5" if a.tree_n > (1 << 22) else "C2")
    n = a.tree_n
    s = W.make_state(cfg, n=n)
    base = _halo_of(dict(cfg, n=n))
    tree = dict(base, tree_alpha=5e-4)
    prec = S.SIDM_PREC_MIXED
    dev = S.state_to_device(s)
    ctx = S.sidm_create(0, n, 1)
    diag = S.diag_buffer(1)
    for f in ("ax", "ay", "az"):
        dev[f].fill_(1e300)
    S.sidm_gravity(ctx, [tree], dev, prec)      # seed: every disjoint node accepted
    S.sidm_gravity(ctx, [tree], dev, prec)      # a_old from the seed
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.sidm_gravity(ctx, [tree], dev, prec)
    S.sidm_diagnostics(ctx, [tree], dev, diag)
    torch.cuda.synchronize()
    t_tree = time.perf_counter() - t0
    terms = S.read_diag(diag)[0]["n_grav_terms"]
    # every member of a group (a 64-particle bucket) sums its group's list
    per_particle = terms * 64 / n
    at = [dev[f].cpu().numpy().copy() for f in ("ax", "ay", "az")]
    print(f"TREE: first tree forces {t_tree * 1e3:.1f} ms, {per_particle:.0f} source terms per "
          f"particle", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    S.sidm_gravity(ctx, [base], dev, prec)
    torch.cuda.synchronize()
    t_direct = time.perf_counter() - t0
    ad = [dev[f].cpu().numpy() for f in ("ax", "ay", "az")]
    err = np.sqrt(sum((x - y) ** 2 for x, y in zip(at, ad))) / np.sqrt(sum(y * y for y in ad))
    S.sidm_destroy(ctx)
    print(f"TREE: direct forces {t_direct * 1e3:.1f} ms; error median {np.median(err):.2e} "
          f"p99 {np.percentile(err, 99):.2e} max {err.max():.2e}", file=sys.stderr, flush=True)
    s_tree = dict(s, ax=ad[0], ay=ad[1], az=ad[2])
    ms_t, de_t, p_t, d_t, _ = _run(S, torch, [tree], s_tree, prec, a.steps, a.warmup, True)
    print(f"TREE: {a.steps} tree steps {ms_t * 1e3:.1f} ms each, |dE/E| {de_t:.2e}",
          file=sys.stderr, flush=True)
    direct = {"gravity_ms": t_direct * 1e3}
    if n <= (1 << 22):
        # full direct-sum steps from the same state (at N = 2^24 one direct step
        # takes about 80 s; there the direct gravity time above stands for it)
        ms_d, de_d, p_d, _, _ = _run(S, torch, [base], s, prec, a.steps, a.warmup, True)
        direct.update(steps=a.steps, ms_per_step=ms_d * 1e3, dE_over_E=de_d, pass_ms=p_d)
    inter = n * (n - 1)
    out = {"metric": "gravity interactions/s (direct-sum equivalent) with tree gravity, "
                     "alpha=5e-4",
           "value": inter / ms_t, "unit": "direct-equivalent gravity interactions/s",
           "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms_t * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32 tree pair terms (compensated), f64 decisions and elsewhere",
           "data": "synthetic NFW halo",
           "config": {"workload": f"TREE: NFW N={n} satellite in the host, eps={cfg['eps']}, "
                                  f"k=64, sigma/m=10, dt=1e-3, tree alpha=5e-4",
                      "n": n, "tree_alpha": 5e-4},
           "source_terms_per_particle": per_particle,
           "tree_interactions_per_s": per_particle * n / (p_t["gravity_tiles"] * 1e-3),
           "force_error": {
               "median": float(np.median(err)), "p99": float(np.percentile(err, 99)),
               "max": float(err.max())},
           "first_forces_ms": {"tree": t_tree * 1e3, "direct": t_direct * 1e3},
           "dE_over_E": de_t, "pass_ms": p_t, "events_last_step": d_t["n_events"],
           "direct": direct,
           "gravity_speedup_vs_direct": t_direct / t_tree,
           "step_speedup_vs_direct": direct["ms_per_step"] / (ms_t * 1e3)
           if "ms_per_step" in direct else None}
    print(json.dumps(out), flush=True)


def main():
    a = _args()
    if a.gpus != 1:
        print(f"bench.py measures one GPU: the library has no multi-GPU path (asked for "
              f"--gpus {a.gpus}); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    global _LOG
    if a.log_jsonl:
        _LOG = open(a.log_jsonl, "a")
    import torch
    import paper_2506_06269_amd as S
    import workloads as W
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    _TUNE["mode"] = "tune" if a.tune else "cache"
    _TUNE["shape"] = a.shape
    _TUNE["sym_min_n"] = a.symmetric_min_n
    if a.workload == "C1":
        return _bench_c1(a, S, torch, W)
    if a.workload == "C3":
        return _bench_c3(a, S, torch, W)
    if a.workload == "C4":
        return _bench_c4(a, S, torch, W)
    if a.workload == "C5":
        return _bench_c5(a, S, torch, W)
    if a.workload == "BLK":
        return _bench_blk(a, S, torch, W)
    if a.workload == "TREE":
        return _bench_tree(a, S, torch, W)
    cfg = W.config("C2")
    overrides = _apply_overrides(cfg, a.set)
    n = cfg["n"]
    s = W.make_state(cfg)
    inter = n * (n - 1)
    halos = [_halo_of(cfg)]
    if a.calibrate_copy > 0:
        src = torch.ones(a.calibrate_copy // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    ms_mixed, de_mixed, passes, dlast, events = _run(S, torch, halos, s, S.SIDM_PREC_MIXED,
                                                     a.steps, a.warmup, True)
    de_int_mixed, tiles_mixed, last_counts = _run.rel_e_internal, _run.tiles, _run.last
    fp64 = None
    if a.fp64_steps > 0:
        ms64, de64, p64, _, _ = _run(S, torch, halos, s, S.SIDM_PREC_FP64, a.fp64_steps, 1, True)
        fp64 = {"interactions_per_s": inter / ms64, "ms_per_step": ms64 * 1e3, "dE_over_E": de64,
                "dEint_over_Eint": _run.rel_e_internal, "tiles": _run.tiles,
                "gravity_tiles_ms": p64.get("gravity_tiles"),
                "gravity_tiles_frac_fp64_peak":
                    FLOPS_PER_INTERACTION * inter / (p64["gravity_tiles"] * 1e-3) / 1e12
                    / FP64_PEAK_TFLOPS if p64.get("gravity_tiles") else None}

    tiles_s = passes["gravity_tiles"] * 1e-3
    achieved = FLOPS_PER_INTERACTION * inter / tiles_s / 1e12
    shape = tiles_mixed
    sym_min = SYM_MIN_N if _TUNE["sym_min_n"] is None else _TUNE["sym_min_n"]
    sym = sym_min > 0 and n >= sym_min
    if sym:
        # each unordered pair once: 26 flops of which 13 per interaction are executed
        jg = 1 if shape["ireg"] >= 8 else 8 // shape["ireg"]
        kname = f"k_grav_sym<{shape['ireg']},{shape['threads']},{jg}>"
    else:
        kname = f"k_grav_mixed<{shape['ireg']},{shape['threads']},{bool(shape['persistent'])}>"
    executed = (SYM_FLOPS_PER_INTERACTION if sym else FLOPS_PER_INTERACTION) * inter / tiles_s / 1e12
    roof = {"bound": "alu", "kernel": kname, "achieved": achieved,
            "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS,
            "executed_flops_per_interaction": SYM_FLOPS_PER_INTERACTION if sym
            else FLOPS_PER_INTERACTION,
            "executed_frac": executed / FP32_PEAK_TFLOPS,
            "traffic": None if overrides else _traffic(FLOPS_PER_INTERACTION * inter)}

    out = {
        "metric": "gravity interactions/s + SIDM particle-updates/s, mixed vs FP64 at |dE/E|",
        "value": inter / ms_mixed,
        "unit": "gravity interactions/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_mixed * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 gravity tiles (compensated), f64 elsewhere",
        "data": "synthetic NFW halo (Eddington ICs), resident in HBM",
        "config": {"workload": "NFW N=2^20 satellite on a circular orbit in a static NFW host, "
                               "eps=0.01, k=64, sigma/m=10, dt=1e-3, mixed precision",
                   "n": n, "k": cfg["k"], "sigma_m": cfg["sigma_m"], "dt": cfg["dt"],
                   "eps": cfg["eps"], "parallelism": "single GPU",
                   **({"overrides": overrides} if overrides else {})},
        "sidm_particle_updates_per_s": n / ms_mixed,
        "dE_over_E": de_mixed,
        "dEint_over_Eint": de_int_mixed,
        "tiles": tiles_mixed,
        "events_last_step": events,
        "pairs_last_step": last_counts["n_pairs"],
        "candidates_last_step": last_counts["n_candidates"],
        "pass_ms": passes,
        "fp64": fp64,
        "roofline": roof,
        "cpu_baseline": None,
    }
    if not a.no_cpu:
        out["cpu_baseline"] = _cpu_baseline(cfg, s, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
