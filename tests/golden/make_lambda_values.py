"""Writes lambda_values.txt: the kernel overlap Lambda(d; hi, hj) by adaptive
2-D quadrature in cylindrical coordinates (scipy), a route independent of the
oracle's 1-D bipolar reduction.  Only the oracle's kernel W is called."""
import math
import os
import sys

from scipy import integrate

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
from oracle import oracle as O  # noqa: E402


def lam_cyl(d, hi, hj):
    W = O.kernel_W

    def inner(z):
        rmax = min(math.sqrt(max(hi * hi - z * z, 0.0)), math.sqrt(max(hj * hj - (z - d) ** 2, 0.0)))
        if rmax <= 0:
            return 0.0
        f = lambda rho: 2 * math.pi * rho * W(math.hypot(rho, z), hi) * W(math.hypot(rho, z - d), hj)
        return integrate.quad(f, 0, rmax, epsabs=1e-15, epsrel=1e-13, limit=400)[0]
    zlo, zhi = max(-hi, d - hj), min(hi, d + hj)
    if zlo >= zhi:
        return 0.0
    pts = sorted({p for p in (-hi / 2, hi / 2, d - hj / 2, d + hj / 2, 0.0, d) if zlo < p < zhi})
    return integrate.quad(inner, zlo, zhi, points=pts, epsabs=1e-15, epsrel=1e-12, limit=400)[0]


CASES = [(d, 1.0, 1.0) for d in (0.0, 0.25, 0.5, 1.0, 1.5, 1.9)] + \
        [(d, 1.0, 0.5) for d in (0.0, 0.5, 1.0, 1.25, 1.45)] + \
        [(d, 0.3, 0.7) for d in (0.1, 0.4, 0.6, 0.95)]

if __name__ == "__main__":
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lambda_values.txt")
    with open(out, "w") as f:
        f.write("# d hi hj Lambda -- adaptive cylindrical quadrature, make_lambda_values.py\n")
        for d, hi, hj in CASES:
            f.write(f"{d!r} {hi!r} {hj!r} {lam_cyl(d, hi, hj):.15e}\n")
