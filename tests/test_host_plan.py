"""CPU checks of the launch planner (csrc/sidm_plan.hpp, compiled for the host
with g++): the number of j-splits of the gravity sums is the one whose work
items, started largest first on the device's resident blocks, finish
soonest; checked against an independent list-scheduling simulation.  The
work items of any plan fit the context's item table, and the searches of a
call with few buckets get enough waves."""
import ctypes as C

import numpy as np
import heapq
import os
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
_SRC = r'''
#include "sidm_plan.hpp"
extern "C" long long plan_items(int nh, const long long* n, long long slots, int ireg, int nt,
                                long long* cap, int* split) {
    std::vector<sidm::HaloDev> hd(nh);
    long long tot = 0;
    for (int h = 0; h < nh; ++h) { std::memset(&hd[h], 0, sizeof(hd[h])); hd[h].n = n[h]; tot += n[h]; }
    sidm::GravShape shape;
    shape.ireg = ireg;
    shape.nt = nt;
    sidm::choose_splits(hd, sidm::gravity_partial_rows(tot), slots, shape);
    long long items = 0;
    const long long ib = (long long)ireg * nt;
    for (int h = 0; h < nh; ++h) items += (n[h] + ib - 1) / ib * hd[h].grav_split;
    *cap = sidm::gravity_items_cap(tot, nh);
    *split = hd[0].grav_split;
    return items;
}
extern "C" int search_split(long long nb, int max_split) { return sidm::search_split(nb, max_split); }
extern "C" long long plan_rows(int nh, const long long* n, const double* alpha,
                               long long partial_rows, int* split) {
    std::vector<sidm::HaloDev> hd(nh);
    for (int h = 0; h < nh; ++h) {
        std::memset(&hd[h], 0, sizeof(hd[h]));
        hd[h].n = n[h]; hd[h].tree_alpha = alpha[h];
        long long m = (n[h] + 63) / 64;   // buckets of 64, then levels of 8 children
        int l = 0;
        hd[h].level_n[0] = m;
        while (m > 1) { m = (m + 7) / 8; hd[h].level_n[++l] = m; }
        hd[h].n_levels = l + 1;
    }
    sidm::GravShape shape;
    shape.ireg = 4;
    shape.nt = 256;
    sidm::choose_splits(hd, partial_rows, 0, shape);
    long long rows = 0;
    for (int h = 0; h < nh; ++h) { split[h] = hd[h].grav_split; rows += n[h] * hd[h].grav_split; }
    return rows;
}
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
extern "C" long long plan_sym(int nh, const long long* n, const long long* off, const double* eps,
                              const double* alpha, long long min_n, long long slots, int ireg,
                              int nt, long long* out, long long cap, int* flags) {
    std::vector<sidm::HaloDev> hd(nh);
    for (int h = 0; h < nh; ++h) {
        std::memset(&hd[h], 0, sizeof(hd[h]));
        hd[h].n = n[h]; hd[h].offset = off[h]; hd[h].eps = eps[h]; hd[h].tree_alpha = alpha[h];
    }
    sidm::GravShape shape;
    shape.ireg = ireg;
    shape.nt = nt;
    std::vector<sidm::SymItem> items;
    sidm::make_sym_items(hd, shape, min_n, slots, items);
    for (int h = 0; h < nh; ++h) flags[h] = hd[h].grav_sym;
    for (size_t k = 0; k < items.size() && (long long)k < cap; ++k) {
        out[4 * k + 0] = items[k].i0; out[4 * k + 1] = items[k].j0;
        out[4 * k + 2] = items[k].j1; out[4 * k + 3] = items[k].halo;
    }
    return (long long)items.size();
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


def _sym(L, ns, offs, eps, alpha, min_n, slots, ireg, nt):
    nh = len(ns)
    A = lambda t, v: (t * nh)(*v)
    cap = 1 << 20
    out = (C.c_longlong * (4 * cap))()
    flags = (C.c_int * nh)()
    L.plan_sym.restype = C.c_longlong
    cnt = L.plan_sym(nh, A(C.c_longlong, ns), A(C.c_longlong, offs), A(C.c_double, eps),
                     A(C.c_double, alpha), min_n, slots, ireg, nt, out, cap, flags)
    items = [tuple(out[4 * k:4 * k + 4]) for k in range(cnt)]
    return items, list(flags)


@pytest.mark.parametrize("ireg,nt", [(2, 128), (4, 256), (8, 512)])
def test_symmetric_items_cover_every_pair_once(L, ireg, nt):
    """Each unordered pair of a halo that takes the symmetric tiles falls in
    exactly one item: a pair of different i-blocks in the item of the lower
    block whose j-range holds the other, a pair inside one i-block in that
    block's own first tiles (summed one-sided there).  Items start at tile
    boundaries, never before their i-block, and come largest first; halos below
    the threshold, with a tree or without softening take none."""
    S = ireg * nt
    ns = [3 * S + 17, 5 * S, S - 3, 7000, 900, 2 * S + 1]
    offs, o = [], 0
    for n in ns:
        offs.append(o)
        o += n + 5
    eps = [0.01, 0.01, 0.01, 0.0, 0.01, 0.01]
    alpha = [0.0, 0.0, 0.0, 0.0, 0.0, 5e-4]
    items, flags = _sym(L, ns, offs, eps, alpha, 1000, 40, ireg, nt)
    expect = [1 if (n >= 1000 and e > 0 and a == 0) else 0 for n, e, a in zip(ns, eps, alpha)]
    assert flags == expect
    lengths = [j1 - j0 for (_, j0, j1, _) in items]
    assert lengths == sorted(lengths, reverse=True)
    for h, (n, off) in enumerate(zip(ns, offs)):
        mine = [it for it in items if it[3] == h]
        if not flags[h]:
            assert not mine
            continue
        nb = -(-n // S)
        cover = np.zeros((nb, n), dtype=np.int32)   # i-block x j
        for i0, j0, j1, _ in mine:
            bi = (i0 - off) // S
            assert (i0 - off) % S == 0 and j0 >= i0 and j1 <= off + n
            assert (j0 - off) % nt == 0 and ((j1 - off) % nt == 0 or j1 == off + n)
            cover[bi, j0 - off:j1 - off] += 1
        for bi in range(nb):
            assert np.all(cover[bi, :bi * S] == 0)       # pairs with earlier blocks: theirs
            assert np.all(cover[bi, bi * S:] == 1)       # own block and every later j, once


def test_symmetric_items_off(L):
    items, flags = _sym(L, [5000, 8000], [0, 5000], [0.01, 0.01], [0.0, 0.0], 0, 64, 4, 256)
    assert items == [] and flags == [0, 0]
    items, flags = _sym(L, [5000, 8000], [0, 5000], [0.01, 0.01], [0.0, 0.0], 6000, 64, 4, 256)
    assert flags == [0, 1] and all(it[3] == 1 for it in items)


SHAPES = [(i, t) for i in (2, 4, 8) for t in (128, 256, 512)]


@pytest.mark.parametrize("ns", [[64], [1000], [4096], [8192], [65536], [100000], [1 << 20],
                                [4096 * (b + 1) for b in range(20)], [300] * 64])
def test_items_fit_the_table(L, ns):
    """For every launch shape and occupancy the planned one-sided items fit
    the item table the context allocates for that many particles and halos,
    and the split stays within what the partial rows hold."""
    a = (C.c_longlong * len(ns))(*ns)
    cap, split = C.c_longlong(0), C.c_int(0)
    L.plan_items.restype = C.c_longlong
    for ireg, nt in SHAPES:
        for slots in (0, 64, 512, 4096):
            items = L.plan_items(len(ns), a, slots, ireg, nt, C.byref(cap), C.byref(split))
            assert items <= cap.value, (ireg, nt, slots, items, cap.value)
            rows = max(4 * sum(ns), 1 << 18)
            assert 1 <= split.value <= min(32, rows // sum(ns))


@pytest.mark.parametrize("ireg,nt", [(2, 128), (2, 256), (4, 256)])
def test_small_call_split_minimises_finishing_time(L, ireg, nt):
    """A call of 8192 particles may take up to 32 j-ranges (2^18 partial
    rows); the chosen number finishes soonest among 1..32."""
    ns, slots = [8192], 1024
    a = (C.c_longlong * 1)(*ns)
    cap, split = C.c_longlong(0), C.c_int(0)
    L.plan_items(1, a, slots, ireg, nt, C.byref(cap), C.byref(split))
    s = split.value
    times = {q: _makespan(ns, q, slots, ireg, nt) for q in range(1, 33)}
    best = min(times.values())
    assert s > 4
    assert times[s] <= best * (1 + 5e-3) + 1e-9, (s, times)


def test_search_split(L):
    """Waves per bucket: 1 from 2048 buckets on, else the smallest power of
    two that reaches 2048 waves, at most the given maximum."""
    assert L.search_split(16384, 16) == 1
    assert L.search_split(2048, 16) == 1
    assert L.search_split(2047, 16) == 2
    assert L.search_split(128, 16) == 16
    assert L.search_split(128, 4) == 4
    assert L.search_split(1, 16) == 16
    for nb in range(1, 3000, 7):
        s = L.search_split(nb, 16)
        assert s in (1, 2, 4, 8, 16)
        assert nb * s >= 2048 or s == 16
        assert s == 1 or nb * (s // 2) < 2048


@pytest.mark.parametrize("ns,alphas", [
    ([1 << 20], [5e-4]),
    ([(1 << 20) - 4096, 4096], [5e-4, 0.0]),
    ([1 << 19, 1 << 19], [5e-4, 0.0]),
    ([8192, 8191, 100, 1 << 16], [5e-4, 5e-4, 5e-4, 0.0]),
    ([1 << 20] + [4096] * 8, [0.0] + [5e-4] * 8),
])
def test_tree_parts_fit_the_partial_rows(L, ns, alphas):
    """A tree halo's walk runs in four parts (a partial row each) when a level
    below the root holds at least 128 nodes, else in one; the rows of all
    halos fit the context's partial rows (the tree halos' rows are set aside
    before the direct halos' j-splits are chosen)."""
    nh = len(ns)
    rows_cap = max(4 * sum(ns), 1 << 18)
    split = (C.c_int * nh)()
    L.plan_rows.restype = C.c_longlong
    used = L.plan_rows(nh, (C.c_longlong * nh)(*ns), (C.c_double * nh)(*alphas), rows_cap, split)
    assert used <= rows_cap
    for n, a, s in zip(ns, alphas, split):
        if a > 0:
            levels = [-(-n // 64)]
            while levels[-1] > 1:
                levels.append(-(-levels[-1] // 8))
            front = [l for l in range(len(levels) - 1) if levels[l] >= 32 * 4]
            assert s == (4 if front else 1), (n, s)
        else:
            assert s >= 1
