"""CPU checks of the launch planner (csrc/sidm_plan.hpp, compiled for the host
with g++): the number of j-splits of the gravity sums is the one whose work
items, started largest first on the device's resident blocks, finish
soonest; checked against an independent list-scheduling simulation."""
import ctypes as C
import heapq
import os
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
_SRC = r'''
#include "sidm_plan.hpp"
extern "C" int plan_split(int nh, const long long* n, long long slots, long long partial_rows,
                          int ireg, int nt) {
    std::vector<sidm::HaloDev> hd(nh);
    for (int h = 0; h < nh; ++h) { std::memset(&hd[h], 0, sizeof(hd[h])); hd[h].n = n[h]; }
    sidm::GravShape shape;
    shape.ireg = ireg;
    shape.nt = nt;
    sidm::choose_splits(hd, partial_rows, slots, shape);
    return hd[0].grav_split;
}
'''


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(os.path.join(ROCM, "include", "hip", "hip_runtime.h")):
        pytest.skip("HIP headers not installed")
    d = tempfile.mkdtemp(prefix="sidm_plan_")
    src, so = os.path.join(d, "p.cpp"), os.path.join(d, "p.so")
    with open(src, "w") as f:
        f.write(_SRC)
    subprocess.run(["g++", "-std=c++17", "-O2", "-shared", "-fPIC", "-D__HIP_PLATFORM_AMD__",
                    "-I", os.path.join(ROCM, "include"), "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_2506_06269_amd", "csrc"), src, "-o", so,
                    "-L", os.path.join(ROCM, "lib"), "-lamdhip64"], check=True)
    return C.CDLL(so)


def _split(L, ns, slots, ireg=4, nt=256):
    a = (C.c_longlong * len(ns))(*ns)
    return L.plan_split(len(ns), a, slots, 4 * sum(ns), ireg, nt)


def _makespan(ns, s, slots, ireg=4, nt=256):
    IBLOCK, TILE = ireg * nt, nt
    cost = []
    for n in ns:
        tiles = -(-n // TILE)
        sh = max(1, min(s, tiles))
        ib = -(-n // IBLOCK)
        for q in range(sh):
            c = (tiles * (q + 1) // sh - tiles * q // sh) * TILE + TILE // 4
            cost += [c] * ib
    cost.sort(reverse=True)
    load = [0.0] * min(slots, len(cost))
    end = 0.0
    for c in cost:
        t = heapq.heappop(load) + c
        end = max(end, t)
        heapq.heappush(load, t)
    return end


@pytest.mark.parametrize("ns,slots", [([1 << 20], 768), ([1 << 20], 512), ([1 << 24], 768),
                                      ([1000], 768), ([8192], 768), ([3000, 5000], 768),
                                      ([4096 * (b + 1) for b in range(20)], 1024)])
@pytest.mark.parametrize("ireg,nt", [(4, 256), (2, 128), (8, 512), (2, 256)])
def test_split_minimises_finishing_time(L, ns, slots, ireg, nt):
    """In every launch shape (i-block ireg * nt, j-tiles of nt)."""
    s = _split(L, ns, slots, ireg, nt)
    assert 1 <= s <= 4
    times = {q: _makespan(ns, q, slots, ireg, nt) for q in range(1, 5)}
    best = min(times.values())
    assert times[s] <= best * (1 + 5e-3) + 1e-9, (s, times)


def test_split_known_cases(L):
    # 1024 i-blocks on 768 slots: 3 splits make exactly 4 full rounds
    assert _split(L, [1 << 20], 768) == 3
    # 16384 i-blocks: 3 splits make exactly 64 rounds
    assert _split(L, [1 << 24], 768) == 3
    # 1024 i-blocks on 512 slots: two full rounds already, no split needed
    assert _split(L, [1 << 20], 512) == 1
    # without an occupancy figure: enough items to fill the chip
    assert _split(L, [1 << 20], 0) == 2
