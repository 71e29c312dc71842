"""CPU checks of the library's per-pair arithmetic (csrc/sidm_math.hpp, the
same header the HIP kernels include), compiled for the host with g++ and
compared with the oracle, which evaluates the same quantities by a different
route (nested Gauss-Legendre in the other particle's frame)."""
import ctypes as C
import math
import os
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
_SRC = r'''
#include "sidm_math.hpp"
extern "C" double lib_overlap(double d, double a, double b) { return sidm::kernel_overlap(d, a, b); }
extern "C" void lib_philox(const unsigned* c, const unsigned* k, unsigned* o) {
  sidm::Philox4 p = sidm::philox4x32_10(c[0], c[1], c[2], c[3], k[0], k[1]);
  for (int i = 0; i < 4; ++i) o[i] = p.w[i];
}
extern "C" double lib_unit53(unsigned hi, unsigned lo) { return sidm::unit53(hi, lo); }
'''


@pytest.fixture(scope="module")
def L():
    d = tempfile.mkdtemp(prefix="sidm_math_")
    src, so = os.path.join(d, "m.cpp"), os.path.join(d, "m.so")
    with open(src, "w") as f:
        f.write(_SRC)
    subprocess.run(["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-shared", "-fPIC", "-I",
                    os.path.join(ROOT, "paper_2506_06269_amd", "csrc"), src, "-o", so],
                   check=True)
    lib = C.CDLL(so)
    lib.lib_overlap.restype = C.c_double
    lib.lib_overlap.argtypes = [C.c_double] * 3
    lib.lib_unit53.restype = C.c_double
    lib.lib_unit53.argtypes = [C.c_uint32, C.c_uint32]
    return lib


def test_overlap_matches_oracle(L, orc):
    rng = np.random.default_rng(5)
    worst = 0.0
    for _ in range(4000):
        ha, hb = rng.uniform(0.05, 2.0, 2)
        d = rng.uniform(0, 1.05) * (ha + hb)
        ref = orc.lam(d, ha, hb)
        got = L.lib_overlap(d, ha, hb)
        if ref == 0.0:
            assert got == 0.0
            continue
        # both exact up to rounding.  The library's shell moment loses a few
        # digits when d is tiny compared with h (difference of two tail
        # moments), and both lose relative digits at the very edge of the
        # support where Lambda vanishes: the absolute part of the bar is set
        # against the peak value Lambda(0), far below the 2^-53 spacing of the
        # accept draws once multiplied by P's prefactors.
        lam0 = orc.lam(0.0, ha, hb)
        tol = (1e-12 + 4e-16 * (ha + hb) / max(d, 1e-300)) * ref + 1e-15 * lam0
        err = abs(got - ref)
        worst = max(worst, err / ref)
        assert err < tol, (d, ha, hb, got, ref)
    for hv in (0.3, 1.0):
        assert L.lib_overlap(0.0, hv, hv) == pytest.approx(982 / (315 * math.pi * hv ** 3), rel=1e-14)
    print("worst relative difference", worst)


def test_philox_matches_oracle(L, orc):
    rng = np.random.default_rng(9)
    c = (C.c_uint32 * 4)()
    k = (C.c_uint32 * 2)()
    o = (C.c_uint32 * 4)()
    for _ in range(500):
        cv = [int(v) for v in rng.integers(0, 2 ** 32, 4)]
        kv = [int(v) for v in rng.integers(0, 2 ** 32, 2)]
        c[:] = cv
        k[:] = kv
        L.lib_philox(c, k, o)
        assert list(o) == orc.philox(cv, kv)
    for hi, lo in ((0, 0), (0xFFFFFFFF, 0xFFFFFFFF), (123, 456789)):
        assert L.lib_unit53(hi, lo) == orc.u53(hi, lo)
