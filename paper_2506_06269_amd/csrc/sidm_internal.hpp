// sidm_internal.hpp -- data layout shared by the HIP kernels and the host
// side of libsidm.  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>

#include "sidm.h"

namespace sidm {

constexpr int kBucket = 64;          // particles per leaf bucket of the search tree
constexpr int kFanout = 8;           // children per tree node
constexpr int kMaxLevels = 10;       // tree levels above the buckets
constexpr int kStreamBlock = 256;    // threads per block of the streaming kernels
constexpr int kGravThreads = 256;    // threads per gravity block
constexpr int kGravTileJ = 256;      // j-particles per LDS tile
constexpr int kTickSplit = 16;       // j-splits of a block-step tick
constexpr int kSortBits = 8;         // radix digit width
constexpr int kSortItems = 16;       // keys per thread per sort block
constexpr int kSortBlock = 256;
constexpr int kScanMaxSeg = 1024;   // blocks of the multi-block exclusive scan at most

// Shape of the direct-sum gravity launch: i-particles per thread, threads per
// block (also the j-particles of one LDS tile), and whether the blocks are
// persistent (as many as the device holds, taking work items from a ticket).
// A work item's i-block holds ireg * nt particles; j-ranges are cut at
// multiples of nt.  The tuner chooses among kShapes.
struct GravShape {
    int32_t ireg = 4;
    int32_t nt = 256;
    int32_t persist = 0;
    int32_t pad = 0;
};
constexpr int kNumShapes = 9;
constexpr int kShapeIreg[kNumShapes] = {2, 4, 8, 2, 4, 8, 2, 4, 8};
constexpr int kShapeNt[kNumShapes] = {128, 128, 128, 256, 256, 256, 512, 512, 512};

// Symmetric tiles (the mixed direct sums of large halos, each unordered pair
// evaluated once) run in the launch shape of the one-sided tiles; by default
// halos of at least kSymMinN particles take them.
constexpr int64_t kSymMinN = 4096;
constexpr int kSymFold = 4;           // j-tiles per flush of the i-side sums
constexpr int kSymWaves = 4;          // waves per SIMD the symmetric tiles are compiled for

// Per-halo parameters and derived layout, uploaded once per halo configuration.
struct HaloDev {
    int64_t offset, n;
    double G, eps, eps2, sigma_m, sigma_w, dt;
    int32_t k, host_kind;
    uint64_t seed;
    double host_K, host_r_s, host_c[3];   // host_K = 4 pi G rho_s r_s^3
    double hern_GM, hern_a;               // host_kind 2: Hernquist bulge
    double disk_GM[4], disk_a[4], disk_b[4];   // host_kind 2: Miyamoto-Nagai discs
    double bnd_r, bnd_c[3];               // reflecting sphere (bnd_r = 0: none)
    double eta, dt_min;                   // block time steps (eta = 0: one fixed step)
    int32_t max_bin, pad1;
    double tree_alpha;                    // > 0: gravity through the tree walk
    int64_t tick_part_base;               // block steps: first partial row of a tick
    int32_t tick_split, pad3;             // block steps: j-splits of a tick
    // search tree: level 0 are the buckets, node ranges per level (global index
    // into the box arrays)
    int64_t level_off[kMaxLevels + 1];
    int64_t level_n[kMaxLevels + 1];
    int32_t n_levels;                     // number of levels (>= 1, level 0 = buckets)
    int32_t grav_split;                   // j-splits of the gravity sum
    int64_t part_base;                    // first partial row of this halo
    int64_t stream_block0;                // first streaming block of this halo
    int64_t sbase;                        // first position in the sorted (compact) order
    int32_t rank;                         // halo rank by offset (high bits of the sort key)
    int32_t grav_sym;                     // mixed direct sums run the symmetric tiles
    int32_t win_lo, win_hi;               // kNN bound window, in buckets around b
    int32_t pad;
};

// A block of the streaming kernels never spans two halos.
struct StreamBlock {
    int64_t start;                        // first particle (global index)
    int32_t count;                        // particles in this block (<= kStreamBlock)
    int32_t halo;
};

// One gravity work item: i-block x j-range of one halo.
struct GravItem {
    int64_t i0;                           // first i (global index)
    int64_t j0, j1;                       // j range (global indices), tile aligned
    int32_t halo;
    int32_t slot;                         // which partial row set
};

// One work item of the symmetric tiles: the i-block [i0, i0 + ireg * nt) of one
// halo against the j-range [j0, j1) with j0 >= i0 (global indices, tile
// aligned); its tiles inside the i-block are summed one-sided.
struct SymItem {
    int64_t i0;
    int64_t j0, j1;
    int32_t halo;
    int32_t pad;
};

struct BucketInfo {
    int64_t start;                        // first sorted position
    int32_t count;
    int32_t halo;
};

// Per-halo counters of a scattering pass: events, rounds, pairs tested, pairs
// with P > 1 and candidates of the exact decision.
constexpr int kEvCounts = 5;

// Device-side error bits live in a per-halo status word.
struct DevCounters {
    unsigned long long n_events_total;    // events found (may exceed capacity)
    unsigned long long n_cands;           // pairs whose draw fell below the P bound
    unsigned long long ticket;            // next work item of a persistent gravity launch
};

#ifdef __HIPCC__
// 1/sqrt(r2) for finite r2 > 0: the hardware estimate refined by one Newton
// step, y1 = y0 + y0 (1 - r2 y0^2) / 2, which squares the estimate's relative
// error (the general routine also handles 0, inf, NaN and denormals, which the
// softened r2 >= eps^2 never is).
__device__ inline double rsqrt_pos(double r2)
{
    const double y0 = __builtin_amdgcn_rsq(r2);
    const double e = fma(-r2 * y0, y0, 1.0);
    return fma(0.5 * y0, e, y0);
}

// Work item of workgroup `id` in a launch of n workgroups.  The dispatcher
// hands workgroups to the eight XCDs in turn (id mod 8), and each XCD has an L2
// of its own; this numbering gives XCD x one contiguous run of items instead,
// so that buckets adjacent on the Morton curve, which read the same candidate
// particles, run under one L2.  A bijection on [0, n) for any n.  It suits
// passes whose cost per bucket is even along the curve (the kNN search); the
// pair pass, whose costly buckets crowd into the dense centre, keeps the
// dispatcher's interleaving, which spreads them over all XCDs.
__device__ inline int64_t xcd_contiguous(int64_t id, int64_t n)
{
    const int64_t q = n >> 3, r = n & 7, x = id & 7;
    return x * q + (x < r ? x : r) + (id >> 3);
}

// Between the two: runs of C consecutive items go to the XCDs in turn, so an
// XCD keeps C neighbouring buckets under its L2 while every XCD still samples
// the whole curve (the tree walk, whose lists grow towards the centre).  Items
// past the last whole round of 8 C keep their own number.  A bijection on
// [0, n).
template <int64_t C>
__device__ inline int64_t xcd_chunked(int64_t id, int64_t n)
{
    const int64_t full = n / (8 * C) * (8 * C);
    if (id >= full) return id;
    const int64_t x = id & 7, j = id >> 3;
    return (j / C * 8 + x) * C + j % C;
}
#endif

}  // namespace sidm
