#!/usr/bin/env python3
"""Writes c3_oracle_2p16.json: the oracle's FP64 run of the N = 2^16 satellite
(the N = 2^20 benchmark halo at lower resolution: host on, eps 0.01, k 64,
sigma/m 10, dt 1e-3) for 1000 steps.  Recorded: |dE/E| and |p| every 10 steps,
and the central density within 0.1 r_s of the potential minimum (Sec. 3) at
the start and every 100 steps.  Calls only oracle/ and workloads/; takes a few
hours on 8 cores.

    python tests/golden/make_c3_oracle.py [--steps 1000] [--n 65536]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import oracle as O  # noqa: E402

RADIUS = 0.1


def _energy_and_center(s, p, host):
    hx, hy, hz, hp = O.host_nfw(s["x"], s["y"], s["z"], p.G, host["rho_s"], host["r_s"],
                                host["center"])
    d = O.diag(s["vx"], s["vy"], s["vz"], s["m"], s["pot"], hp)
    c, cnt, mass = O.central_density(s["x"], s["y"], s["z"], s["m"], s["pot"] - hp, RADIUS)
    rho = mass / (4.0 / 3.0 * math.pi * RADIUS ** 3)
    return d, dict(index=c, count=cnt, mass=mass, rho=rho)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--n", type=int, default=1 << 16)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                  "c3_oracle_2p16.json"))
    a = ap.parse_args()
    cfg = W.config("C3")
    host = cfg["host"]
    s = W.make_state(cfg, n=a.n)
    p = O.make_params(G=1.0, eps=cfg["eps"], sigma_m=cfg["sigma_m"], dt=cfg["dt"], k=cfg["k"],
                      seed=cfg["seed"], host=host)
    O.total_accel(s, p)
    d0, c0 = _energy_and_center(s, p, host)
    e0 = d0["K"] + d0["W"] + d0["Eext"]
    rec = {"workload": f"NFW N={a.n} satellite in the host, eps={cfg['eps']}, k={cfg['k']}, "
                       f"sigma/m={cfg['sigma_m']}, dt={cfg['dt']}, FP64 oracle",
           "n": a.n, "steps": a.steps, "radius": RADIUS, "threads": O.num_threads(),
           "energy": [], "center": [dict(step=0, **c0)], "events": 0}
    t0 = time.time()
    for step in range(a.steps):
        ev = O.kdk_step(s, p, step)
        rec["events"] += int(ev.size)
        if (step + 1) % 10 == 0 or step + 1 == a.steps:
            d, c = _energy_and_center(s, p, host)
            e = d["K"] + d["W"] + d["Eext"]
            rec["energy"].append(dict(step=step + 1, dE_over_E=abs(e - e0) / abs(e0),
                                      p=math.sqrt(d["px"] ** 2 + d["py"] ** 2 + d["pz"] ** 2)))
            if (step + 1) % 100 == 0 or step + 1 == a.steps:
                rec["center"].append(dict(step=step + 1, **c))
            print(f"step {step + 1}: |dE/E| {rec['energy'][-1]['dE_over_E']:.3e} "
                  f"rho(<{RADIUS}) {c['rho']:.4g} ({c['count']}) "
                  f"{time.time() - t0:.0f} s", flush=True)
    rec["seconds"] = time.time() - t0
    with open(a.out, "w") as f:
        json.dump(rec, f, indent=1)
    print("wrote", a.out)


if __name__ == "__main__":
    main()
