// sidm_plan.hpp -- scratch memory of a context and the launch plan built for
// one halo configuration (tables of streaming blocks, gravity work items,
// search-tree buckets and nodes).  Host side only uses the std containers.
#pragma once

#include <algorithm>
#include <cstdio>
#include <functional>
#include <string>
#include <vector>

#include "sidm_internal.hpp"

namespace sidm {

// Event record kept on the device while the conflict-free rounds run.
struct EventRec {
    unsigned long long key;   // (a << 32) | b
    int64_t ia, ib;           // original particle indices
    int32_t halo;
    uint32_t round;
};

// A pair whose accept draw fell below the cheap upper bound of P: the exact
// probability needs the overlap integral, which a second kernel evaluates.
struct CandRec {
    double sg, mb, g;         // cross-section, mass of b and relative speed
    double d, ha, hb;         // separation and the kernel sizes of a and b
    double u;                 // the accept draw
    uint32_t a, b;            // ids
    uint32_t ia, ib;          // original particle indices
    int32_t halo, pad;
};

// A tree node of level >= 1 and the range of its children (global indices).
struct NodeTask {
    int64_t node;
    int64_t child0;
    int32_t nchild;
    int32_t pad;
};

// Children of every node of the search tree (buckets have none) and the last
// bucket of its subtree (buckets of a subtree are consecutive).
struct NodeChild {
    int64_t child0;
    int64_t last;
    int32_t nchild;
    int32_t pad;
};

// A bucket is cut into at most kSubMax compact sub-ranges at its coarsest
// internal Morton boundaries when that shrinks their boxes: a bucket of 64
// consecutive particles that straddles a coarse cell boundary is otherwise
// spread over a large region.
constexpr int kSubMax = 4;
// At most this many j-ranges per halo for the one-sided gravity tiles.
constexpr int64_t kMaxGravSplit = 32;
// The tree walk of a group is cut into kTreeSplit parts, each with a partial
// row of its own: the nodes of one level of the halo's tree (its frontier)
// are dealt out to the parts in turn, and a part descends only into its own
// frontier nodes (every part tests the nodes above the frontier, and an
// accepted one counts in part 0 only).  Every node is then accepted or opened
// for the group exactly as in one walk, while the few groups that open most
// of the tree (a bucket that straddles the halo's centre, the densest centre
// groups) are shared out over four waves.  The frontier is the highest level
// below the root with at least kTreeFrontPer nodes per part; a halo without
// one walks in one part.
constexpr int kTreeSplit = 4;
constexpr int kTreeFrontPer = 32;
constexpr int tree_front_level(const int64_t* level_n, int n_levels, int parts)
{
    for (int l = n_levels - 2; l >= 0; --l)
        if (level_n[l] >= (int64_t)kTreeFrontPer * parts) return l;
    return -1;
}
inline int32_t tree_parts(const HaloDev& H)
{
    return tree_front_level(H.level_n, H.n_levels, kTreeSplit) >= 0 ? kTreeSplit : 1;
}
// The searches also skip chunks of kChunk consecutive particles of a bucket
// (aligned to the bucket start) that no lane's sphere reaches.
constexpr int kChunk = 16;
constexpr int kChunks = kBucket / kChunk;
struct SubRange {
    int32_t off;                  // first particle, relative to the bucket start
    int32_t cnt;
    double box[6];
};

struct Scratch {
    int64_t max_particles = 0, max_events = 0;
    int32_t max_halos = 0;
    // plan tables
    HaloDev* halos = nullptr;
    StreamBlock* blocks = nullptr;
    int64_t blocks_cap = 0;
    GravItem* items = nullptr;
    int64_t items_cap = 0;
    BucketInfo* buckets = nullptr;
    int64_t buckets_cap = 0;
    NodeTask* node_tasks = nullptr;
    NodeChild* nodes = nullptr;
    int64_t nodes_cap = 0;        // bucket boxes + tree nodes
    // gravity
    double* bsum = nullptr;       // 7 doubles per streaming block
    double* cref = nullptr;       // per halo: the common mass if all are equal, else 0
    double* radius = nullptr;     // per halo: radius of the central density
    sidm_center* center = nullptr;    // per halo: centre of the tidal-radius search
    double* tidal = nullptr;          // per halo: 8 doubles of bisection state
    double* bbox = nullptr;       // 6 per halo (min xyz, max xyz)
    float4* xm32 = nullptr;       // FP32 positions relative to their tile centre, mass
    double4* partial = nullptr;
    int64_t partial_rows = 0;
    // block-step ticks: finer j-splits (allocated with the first plan that needs them)
    GravItem* items_tick = nullptr;
    int64_t items_tick_cap = 0;
    double4* partial_tick = nullptr;
    int64_t partial_tick_rows = 0;
    int64_t grav_slots = 0;       // resident blocks of the gravity tiles on the whole device
    int64_t slots_mixed = 0, slots_fp64 = 0;   // of the plan's shape, per precision
    // symmetric tiles: work items, fixed-point totals (4 per sorted particle),
    // resident blocks
    SymItem* sym_items = nullptr;
    int64_t sym_items_cap = 0;
    unsigned long long* symacc = nullptr;
    int64_t symacc_n = 0;
    int64_t slots_sym = 0;
    // cell list
    unsigned long long* keys[2] = {nullptr, nullptr};
    uint32_t* vals[2] = {nullptr, nullptr};
    uint32_t* hist = nullptr;
    uint32_t* scan_part = nullptr;    // segment sums of the histogram scan
    int64_t hist_cap = 0;
    double *sx = nullptr, *sy = nullptr, *sz = nullptr;
    double4* sp4 = nullptr;       // sorted positions as (x, y, z, 0): one load per candidate
    double *svx = nullptr, *svy = nullptr, *svz = nullptr;
    double *sh = nullptr, *sm = nullptr;
    int8_t* bin = nullptr;        // block time-step bin per particle (caller's order)
    double4* mom = nullptr;       // per node: mass and first moments (tree gravity)
    double* mom2 = nullptr;       // per node: 6 second moments about its centre of mass
    unsigned long long* tree_terms = nullptr;   // per halo: source terms of the tree walk
    uint32_t* sid = nullptr;
    uint32_t* perm = nullptr;
    double* box = nullptr;        // 6 per node (buckets first)
    SubRange* sub = nullptr;      // kSubMax per bucket
    int* sub_n = nullptr;         // sub-ranges per bucket
    double* cbox = nullptr;       // 6 per chunk, kChunks per bucket (searches only)
    double* chmax = nullptr;      // largest h per chunk, kChunks per bucket (pair search)
    unsigned long long* skeys = nullptr;   // sorted keys (one of keys[0..1])
    double* hmax = nullptr;       // 1 per node
    // scattering
    unsigned long long* owner = nullptr;
    EventRec* events = nullptr;
    CandRec* cands = nullptr;         // candidates of the exact decision
    int64_t max_cands = 0;
    DevCounters* counters = nullptr;
    long long* ev_counts = nullptr;   // kEvCounts per halo
    int* status = nullptr;            // per halo
    int* sticky = nullptr;            // OR of the status words not yet read by the host
    unsigned long long* fp_dev = nullptr;   // fingerprint of the last call outside capture
};

struct Plan {
    int n_halos = 0;
    int64_t n_sorted = 0;             // particles in halos
    int64_t n_blocks = 0, n_items = 0, n_buckets = 0, n_nodes = 0;
    int n_levels = 1;                 // max levels over halos
    int key_bits = 48;
    int rank_shift = 48;              // 49 when block steps order active particles first
    bool has_tree = false;            // some halo uses the tree walk
    bool any_scatter = false;         // some halo has sigma_m > 0
    GravShape shape;                  // launch shape of the direct-sum tiles
    int halo_bits = 0;                // bits of a halo index
    int64_t sort_blocks = 0;
    std::vector<HaloDev> halos;
    std::vector<StreamBlock> blocks;
    std::vector<GravItem> items;          // one-sided: the halos without symmetric tiles first
    int64_t n_items_nosym = 0;            // items of the halos without symmetric tiles
    std::vector<SymItem> sym_items;       // symmetric tiles (mixed precision)
    int64_t n_sym_items = 0;
    std::vector<GravItem> items_tick;     // block-step ticks (empty without block steps)
    int64_t tick_rows = 0;                // partial rows the tick items need
    std::vector<BucketInfo> buckets;
    std::vector<NodeTask> node_tasks;
    std::vector<NodeChild> nodes;
    int64_t level_task_off[kMaxLevels + 1] = {};   // tasks of level l: [off[l-1], off[l])
    std::vector<int> rank_of;
};

template <typename T>
inline bool dalloc(T*& p, int64_t count)
{
    p = nullptr;
    if (count <= 0) count = 1;
    return hipMalloc((void**)&p, sizeof(T) * (size_t)count) == hipSuccess;
}

template <typename T>
inline void dfree(T*& p)
{
    if (p) (void)hipFree((void*)p);
    p = nullptr;
}

// Events and the candidates of the exact decision (four per event slot: at the
// benchmark's density a pair's draw falls below the bound some 70 times as
// often as below P, and the default event buffer, N/8, holds about 50 times
// a step's events; an overflow only costs a second pair pass).
inline bool realloc_events(Scratch& w, int64_t max_events, std::string& why)
{
    dfree(w.events);
    dfree(w.cands);
    w.max_events = max_events;
    w.max_cands = 4 * max_events;
    if (!dalloc(w.events, max_events) || !dalloc(w.cands, w.max_cands)) {
        why = "cannot allocate the event buffers";
        w.max_events = w.max_cands = 0;
        return false;
    }
    return true;
}

// Waves per bucket for the searches of a call with few buckets: the smallest
// power of two (at most max_split) that gives kSearchWaves waves in all.
constexpr int64_t kSearchWaves = 2048;
constexpr int kPairSplitMax = 16;
inline int search_split(int64_t n_buckets, int max_split)
{
    int s = 1;
    while (s < max_split && n_buckets * s < kSearchWaves) s *= 2;
    return s;
}

// Partial rows of the one-sided gravity tiles for a context of N particles:
// four per particle, and at least 2^18 (small calls take more j-ranges).
inline int64_t gravity_partial_rows(int64_t N)
{
    return std::max<int64_t>(4 * N, 1 << 18);
}

// Gravity work items a context of N particles in H halos can need: the
// i-blocks of the smallest launch shape (2 x 128) times the j-ranges
// choose_splits may give them (at most kMaxGravSplit, and as many as the
// partial rows hold).
inline int64_t gravity_items_cap(int64_t N, int32_t H)
{
    const int64_t split_cap = std::min<int64_t>(
        kMaxGravSplit, std::max<int64_t>(1, gravity_partial_rows(N) / std::max<int64_t>(N, 1)));
    return std::max<int64_t>((N / (kGravThreads * 4) + H + 1) * 64, (N / 256 + H + 1) * split_cap);
}

inline bool alloc_scratch(Scratch& w, int64_t N, int32_t H, int64_t max_events, std::string& why)
{
    w.max_particles = N;
    w.max_halos = H;
    const int64_t nb = N / kStreamBlock + H + 1;
    w.blocks_cap = nb;
    w.items_cap = gravity_items_cap(N, H);
    w.partial_rows = gravity_partial_rows(N);
    w.buckets_cap = N / kBucket + H + 1;
    w.nodes_cap = w.buckets_cap * 2 + (int64_t)H * (kMaxLevels + 1);
    const int64_t sort_blocks = N / (kSortBlock * kSortItems) + 1;
    w.hist_cap = sort_blocks * (1 << kSortBits) + 1;
    bool ok = dalloc(w.halos, H) && dalloc(w.blocks, nb) && dalloc(w.items, w.items_cap) &&
              dalloc(w.buckets, w.buckets_cap) && dalloc(w.node_tasks, w.nodes_cap) && dalloc(w.nodes, w.nodes_cap) &&
              dalloc(w.bsum, 7 * nb) && dalloc(w.cref, 4 * H) && dalloc(w.radius, H) && dalloc(w.center, H) &&
              dalloc(w.tidal, 8 * H) && dalloc(w.bbox, 6 * H) &&
              dalloc(w.xm32, N) &&  dalloc(w.partial, w.partial_rows) && dalloc(w.keys[0], 2 * N) &&
              dalloc(w.vals[0], N) && dalloc(w.vals[1], N) &&
              dalloc(w.hist, w.hist_cap) && dalloc(w.scan_part, kScanMaxSeg) && dalloc(w.sx, N) && dalloc(w.sy, N) &&
              dalloc(w.sz, N) && dalloc(w.sp4, N) && dalloc(w.svx, N) && dalloc(w.svy, N) && dalloc(w.svz, N) &&
              dalloc(w.sh, N) && dalloc(w.sm, N) && dalloc(w.bin, N) &&
              dalloc(w.mom, w.nodes_cap) && dalloc(w.mom2, 6 * w.nodes_cap) && dalloc(w.tree_terms, H) && dalloc(w.sid, N) && dalloc(w.perm, N) &&
              dalloc(w.box, 6 * w.nodes_cap) && dalloc(w.hmax, w.nodes_cap) &&
              dalloc(w.sub, kSubMax * w.buckets_cap) && dalloc(w.sub_n, w.buckets_cap) &&
              dalloc(w.cbox, 6 * kChunks * w.buckets_cap) && dalloc(w.chmax, kChunks * w.buckets_cap) &&
              dalloc(w.owner, N) && dalloc(w.counters, 1) && dalloc(w.ev_counts, kEvCounts * H) &&
              dalloc(w.status, H) && dalloc(w.sticky, 1) && dalloc(w.fp_dev, 1);
    if (!ok) {
        why = "device allocation failed";
        return false;
    }
    // the two key buffers of the radix sort are one allocation: outside the
    // sort its 2 N words serve as the hash table of the id check
    w.keys[1] = w.keys[0] + N;
    if (!realloc_events(w, max_events, why)) return false;
    // the counters, per-halo event counts, status words and tree term counts
    // read by the diagnostics start at zero (a context that has not stepped
    // yet reports no events and a clean status); the passes reset them later
    if (hipMemset(w.counters, 0, sizeof(DevCounters)) != hipSuccess ||
        hipMemset(w.ev_counts, 0, sizeof(*w.ev_counts) * (size_t)(kEvCounts * H)) != hipSuccess ||
        hipMemset(w.status, 0, sizeof(*w.status) * (size_t)H) != hipSuccess ||
        hipMemset(w.sticky, 0, sizeof(*w.sticky)) != hipSuccess ||
        hipMemset(w.fp_dev, 0, sizeof(*w.fp_dev)) != hipSuccess ||
        hipMemset(w.tree_terms, 0, sizeof(*w.tree_terms) * (size_t)H) != hipSuccess) {
        why = "cannot initialise scratch";
        return false;
    }
    // owner slots start free; the scattering pass restores them after use
    std::vector<unsigned long long> ones((size_t)std::min<int64_t>(N, 1 << 20), ~0ull);
    for (int64_t o = 0; o < N; o += (int64_t)ones.size()) {
        const int64_t c = std::min<int64_t>((int64_t)ones.size(), N - o);
        if (hipMemcpy(w.owner + o, ones.data(), sizeof(unsigned long long) * (size_t)c,
                      hipMemcpyHostToDevice) != hipSuccess) {
            why = "cannot initialise scratch";
            return false;
        }
    }
    return true;
}

inline void free_scratch(Scratch& w)
{
    dfree(w.halos); dfree(w.blocks); dfree(w.items); dfree(w.buckets); dfree(w.node_tasks); dfree(w.nodes);
    dfree(w.bsum); dfree(w.cref); dfree(w.radius); dfree(w.center); dfree(w.tidal); dfree(w.bbox); dfree(w.xm32);  dfree(w.partial);
    dfree(w.keys[0]); w.keys[1] = nullptr; dfree(w.vals[0]); dfree(w.vals[1]); dfree(w.hist); dfree(w.scan_part);
    dfree(w.sx); dfree(w.sy); dfree(w.sz); dfree(w.sp4); dfree(w.svx); dfree(w.svy); dfree(w.svz);
    dfree(w.items_tick); dfree(w.partial_tick);
    w.items_tick_cap = w.partial_tick_rows = 0;
    dfree(w.sh); dfree(w.sm); dfree(w.bin); dfree(w.mom); dfree(w.mom2); dfree(w.tree_terms); dfree(w.sid); dfree(w.perm); dfree(w.box); dfree(w.hmax);
    dfree(w.sub); dfree(w.sub_n); dfree(w.cbox); dfree(w.chmax);
    dfree(w.owner); dfree(w.events); dfree(w.cands); dfree(w.counters); dfree(w.ev_counts); dfree(w.status);
    dfree(w.sticky); dfree(w.fp_dev);
    dfree(w.sym_items); dfree(w.symacc);
    w.sym_items_cap = w.symacc_n = 0;
}

// The physical parameters of a halo (the layout fields stay zero).
inline void fill_halo_params(HaloDev& H, const sidm_halo& S)
{
    std::memset(&H, 0, sizeof H);
    H.offset = S.offset;
    H.n = S.n;
    H.G = S.G;
    H.eps = S.eps;
    H.eps2 = S.eps * S.eps;
    H.sigma_m = S.sigma_m;
    H.sigma_w = S.sigma_w;
    H.dt = S.dt;
    H.k = S.k;
    H.host_kind = S.host_kind;
    H.seed = S.seed;
    H.host_r_s = S.host_r_s > 0 ? S.host_r_s : 1.0;
    H.host_K = 4.0 * M_PI * S.G * S.host_rho_s * H.host_r_s * H.host_r_s * H.host_r_s;
    for (int c = 0; c < 3; ++c) H.host_c[c] = S.host_center[c];
    if (S.host_kind == 2) {
        H.hern_GM = S.G * S.host_hern_M;
        H.hern_a = S.host_hern_a;
        for (int d = 0; d < 4; ++d) {
            H.disk_GM[d] = S.G * S.host_disk[d][0];
            H.disk_a[d] = S.host_disk[d][1];
            H.disk_b[d] = S.host_disk[d][2];
        }
    }
    H.bnd_r = S.boundary_r;
    for (int c = 0; c < 3; ++c) H.bnd_c[c] = S.boundary_center[c];
    H.eta = S.eta;
    H.dt_min = S.dt_min;
    H.max_bin = S.eta > 0.0 ? S.max_bin : 0;
    H.tree_alpha = S.tree_alpha;
}

// Checks of one halo's parameters that do not depend on a context (need: the
// NEED_* bits of the call).  Writes a message into msg and returns a status.
enum Need { NEED_GRAV = 1, NEED_KNN = 2, NEED_SCATTER = 4, NEED_STEP = 8 };
inline sidm_status check_halo(const sidm_halo& H, int need, char* msg, size_t cap)
{
    if (H.offset < 0 || H.n < 2 || H.n > (int64_t(1) << 24)) {
        snprintf(msg, cap, "need offset >= 0 and 2 <= n <= 2^24 (offset=%lld n=%lld)",
                 (long long)H.offset, (long long)H.n);
        return SIDM_ERR_INVALID;
    }
    if (!(H.eps > 0.0) || !std::isfinite(H.eps) || !std::isfinite(H.G)) {
        snprintf(msg, cap, "softening eps must be finite and > 0 (eps=%g)", H.eps);
        return SIDM_ERR_INVALID;
    }
    if ((need & (NEED_SCATTER | NEED_STEP)) && (!(H.dt > 0.0) || !std::isfinite(H.dt))) {
        snprintf(msg, cap, "dt must be finite and > 0 (dt=%g)", H.dt);
        return SIDM_ERR_INVALID;
    }
    if ((need & (NEED_SCATTER | NEED_STEP)) && (!(H.sigma_w >= 0.0) || !std::isfinite(H.sigma_w))) {
        snprintf(msg, cap, "sigma_w must be finite and >= 0");
        return SIDM_ERR_INVALID;
    }
    if ((need & (NEED_SCATTER | NEED_STEP)) && (!(H.sigma_m >= 0.0) || !std::isfinite(H.sigma_m))) {
        snprintf(msg, cap, "sigma_m must be finite and >= 0");
        return SIDM_ERR_INVALID;
    }
    if ((need & (NEED_KNN | NEED_STEP)) &&
        (H.k < 1 || H.k > SIDM_MAX_K || (int64_t)H.k > H.n - 1)) {
        snprintf(msg, cap, "need 1 <= k <= min(n-1, %d) (k=%d n=%lld)", SIDM_MAX_K, H.k,
                 (long long)H.n);
        return SIDM_ERR_INVALID;
    }
    if (H.host_kind < 0 || H.host_kind > 2) {
        snprintf(msg, cap, "host_kind must be 0, 1 or 2");
        return SIDM_ERR_UNSUPPORTED;
    }
    if (H.host_kind != 0 && (!(H.host_r_s > 0.0) || !std::isfinite(H.host_r_s) ||
                             !std::isfinite(H.host_rho_s))) {
        snprintf(msg, cap, "host needs r_s > 0 and finite rho_s");
        return SIDM_ERR_INVALID;
    }
    if (H.host_kind == 2) {
        if (!std::isfinite(H.host_hern_M) ||
            (H.host_hern_M != 0.0 && !(H.host_hern_a > 0.0 && std::isfinite(H.host_hern_a)))) {
            snprintf(msg, cap, "the Hernquist bulge needs a finite mass and a > 0");
            return SIDM_ERR_INVALID;
        }
        for (int d = 0; d < 4; ++d) {
            const double* D = H.host_disk[d];
            if (!std::isfinite(D[0]) ||
                (D[0] != 0.0 && !(D[1] >= 0.0 && D[2] >= 0.0 && D[1] + D[2] > 0.0 &&
                                  std::isfinite(D[1]) && std::isfinite(D[2])))) {
                snprintf(msg, cap, "disc %d needs a finite mass, a, b >= 0, a + b > 0", d);
                return SIDM_ERR_INVALID;
            }
        }
    }
    if (!(H.boundary_r >= 0.0) || !std::isfinite(H.boundary_r)) {
        snprintf(msg, cap, "boundary_r must be finite and >= 0");
        return SIDM_ERR_INVALID;
    }
    if (!(H.tree_alpha >= 0.0) || !std::isfinite(H.tree_alpha)) {
        snprintf(msg, cap, "tree_alpha must be finite and >= 0");
        return SIDM_ERR_INVALID;
    }
    if (!(H.eta >= 0.0) || !std::isfinite(H.eta) || !(H.dt_min >= 0.0) ||
        !std::isfinite(H.dt_min) || H.max_bin < 0 || H.max_bin > SIDM_MAX_BIN ||
        (H.eta == 0.0 && H.max_bin != 0)) {
        snprintf(msg, cap, "block steps need finite eta >= 0, dt_min >= 0 and "
                           "0 <= max_bin <= %d (max_bin = 0 when eta = 0)", SIDM_MAX_BIN);
        return SIDM_ERR_INVALID;
    }
    return SIDM_OK;
}

// Number of j-splits for the gravity sum of each halo.  Work items (one
// block of kGravThreads * 4 i-particles against one j-range) are started
// largest first on `slots` resident blocks; the split whose simulated
// finishing time is smallest wins (ties go to fewer splits, which write fewer
// partial rows).  Without an occupancy figure, enough items to fill the chip.
inline void choose_splits(std::vector<HaloDev>& hd, int64_t partial_rows, int64_t slots,
                          const GravShape& shape)
{
    const int64_t kIBlock = (int64_t)shape.ireg * shape.nt, kGravTileJ = shape.nt;
    int64_t iblocks = 0, ntot = 0, tree_rows = 0;
    for (auto& H : hd) {
        if (H.tree_alpha > 0.0) {
            tree_rows += H.n * tree_parts(H);
            continue;
        }
        iblocks += (H.n + kIBlock - 1) / kIBlock;
        ntot += H.n;
    }
    iblocks = std::max<int64_t>(iblocks, 1);
    // at most kMaxGravSplit j-ranges per halo, and as many as the partial rows
    // left by the tree halos hold (four or more for calls of 2^16 particles
    // and more; small calls get more j-ranges to fill the device)
    const int64_t smax = std::min<int64_t>(
        kMaxGravSplit,
        std::max<int64_t>(1, (partial_rows - tree_rows) / std::max<int64_t>(ntot, 1)));
    int64_t best = 1;
    if (slots <= 0) {
        best = std::min<int64_t>(smax, std::max<int64_t>(1, (2048 + iblocks - 1) / iblocks));
    } else {
        double best_t = 0.0;
        std::vector<int64_t> cost;
        std::vector<double> load;
        for (int64_t sp = 1; sp <= smax; ++sp) {
            cost.clear();
            for (auto& H : hd) {
                if (H.tree_alpha > 0.0) continue;
                const int64_t tiles = (H.n + kGravTileJ - 1) / kGravTileJ;
                const int64_t s_h = std::max<int64_t>(1, std::min<int64_t>(sp, tiles));
                const int64_t ib = (H.n + kIBlock - 1) / kIBlock;
                for (int64_t q = 0; q < s_h; ++q) {
                    const int64_t t0 = tiles * q / s_h, t1 = tiles * (q + 1) / s_h;
                    const int64_t c = (t1 - t0) * kGravTileJ + kGravTileJ / 4;   // + epilogue
                    for (int64_t i = 0; i < ib; ++i) cost.push_back(c);
                }
            }
            std::sort(cost.begin(), cost.end(), std::greater<int64_t>());
            // list scheduling: each item goes to the slot that frees first
            load.assign((size_t)std::min<int64_t>(slots, (int64_t)cost.size()), 0.0);
            std::make_heap(load.begin(), load.end(), std::greater<double>());
            double t_end = 0.0;
            for (int64_t c : cost) {
                std::pop_heap(load.begin(), load.end(), std::greater<double>());
                load.back() += (double)c;
                t_end = std::max(t_end, load.back());
                std::push_heap(load.begin(), load.end(), std::greater<double>());
            }
            if (sp == 1 || t_end < best_t * (1.0 - 5e-3)) {
                best_t = t_end;
                best = sp;
            }
        }
    }
    for (auto& H : hd) {
        const int64_t tiles = (H.n + kGravTileJ - 1) / kGravTileJ;
        if (H.tree_alpha > 0.0)
            H.grav_split = tree_parts(H);
        else
            H.grav_split = (int32_t)std::max<int64_t>(1, std::min<int64_t>(best, tiles));
    }
}

// Symmetric tiles: marks the halos large enough for them (softened, direct
// sum, at least sym_min_n particles; none for sym_min_n = 0) and cuts their
// work: each i-block of ireg * nt against the j from its own start to the
// halo's end, in ranges of L (a multiple of nt, at least four i-blocks),
// about 32 items per resident block over all such halos, largest first.
inline void make_sym_items(std::vector<HaloDev>& halos, const GravShape& shape,
                           int64_t sym_min_n, int64_t sym_slots, std::vector<SymItem>& items)
{
    items.clear();
    if (sym_min_n <= 0 || sym_slots <= 0) return;
    const int64_t sym_i = (int64_t)shape.ireg * shape.nt;
    double pairs = 0.0;
    for (auto& H : halos)
        if (!(H.tree_alpha > 0.0) && H.n >= std::max<int64_t>(sym_min_n, 2) && H.eps > 0.0) {
            H.grav_sym = 1;
            pairs += 0.5 * (double)H.n * (double)H.n;
        }
    const double target = pairs / (32.0 * (double)sym_slots * (double)sym_i);
    for (int h = 0; h < (int)halos.size(); ++h) {
        const HaloDev& H = halos[h];
        if (!H.grav_sym) continue;
        int64_t L = (int64_t)std::min<double>(target, (double)H.n);
        L = std::max<int64_t>(L, 4 * sym_i);
        L = (L + shape.nt - 1) / shape.nt * shape.nt;
        for (int64_t i0 = 0; i0 < H.n; i0 += sym_i)
            for (int64_t j0 = i0; j0 < H.n; j0 += L)
                items.push_back({H.offset + i0, H.offset + j0,
                                 H.offset + std::min<int64_t>(H.n, j0 + L), h, 0});
    }
    std::stable_sort(items.begin(), items.end(), [](const SymItem& a, const SymItem& b) {
        return (a.j1 - a.j0) > (b.j1 - b.j0);
    });
}

// sym_min_n: direct-sum halos of at least that many particles take the
// symmetric tiles in mixed precision (0: none); sym_slots: resident blocks of
// those tiles, which sets how finely their j-ranges are cut.
inline bool build_plan(Plan& P, const Scratch& w, const sidm_halo* halos, int32_t n_halos,
                       const GravShape& shape, int64_t slots, std::string& why,
                       int64_t sym_min_n = 0, int64_t sym_slots = 0)
{
    P = Plan();
    P.shape = shape;
    P.n_halos = n_halos;
    P.halos.resize(n_halos);
    // halos ordered by offset define the sorted (compact) index space
    std::vector<int> order(n_halos);
    for (int h = 0; h < n_halos; ++h) order[h] = h;
    std::sort(order.begin(), order.end(),
              [&](int a, int b) { return halos[a].offset < halos[b].offset; });
    std::vector<int64_t> sbase(n_halos);
    int64_t acc = 0;
    for (int r = 0; r < n_halos; ++r) {
        sbase[order[r]] = acc;
        P.rank_of.resize(n_halos);
        P.rank_of[order[r]] = r;
        acc += halos[order[r]].n;
    }
    P.n_sorted = acc;
    int64_t node_count = 0;
    for (int h = 0; h < n_halos; ++h) {
        const sidm_halo& S = halos[h];
        HaloDev& H = P.halos[h];
        fill_halo_params(H, S);
        if (S.tree_alpha > 0.0) P.has_tree = true;
        if (S.sigma_m > 0.0) P.any_scatter = true;
        H.sbase = sbase[h];
        H.rank = P.rank_of[h];
        // streaming blocks
        H.stream_block0 = (int64_t)P.blocks.size();
        for (int64_t s0 = 0; s0 < S.n; s0 += kStreamBlock)
            P.blocks.push_back(
                {S.offset + s0, (int32_t)std::min<int64_t>(kStreamBlock, S.n - s0), h});
        // buckets over the sorted range
        const int64_t nbk = (S.n + kBucket - 1) / kBucket;
        H.level_off[0] = (int64_t)P.buckets.size();
        H.level_n[0] = nbk;
        for (int64_t b = 0; b < nbk; ++b)
            P.buckets.push_back({H.sbase + b * kBucket,
                                 (int32_t)std::min<int64_t>(kBucket, S.n - b * kBucket), h});
        // kNN bound window: buckets around b holding at least 2(k+1) particles
        const int64_t want = 2 * ((int64_t)std::max(S.k, 1) + 1);
        const int64_t wb = std::min<int64_t>(nbk, (want + kBucket - 1) / kBucket + 1);
        H.win_lo = (int32_t)(wb / 2);
        H.win_hi = (int32_t)(wb - 1 - wb / 2);
    }
    // tree levels (nodes after all buckets)
    P.n_buckets = (int64_t)P.buckets.size();
    node_count = P.n_buckets;
    P.n_levels = 1;
    std::vector<std::vector<NodeTask>> per_level(kMaxLevels + 1);
    for (int h = 0; h < n_halos; ++h) {
        HaloDev& H = P.halos[h];
        int l = 0;
        while (H.level_n[l] > 1) {
            if (l + 1 > kMaxLevels) {
                why = "search tree too deep";
                return false;
            }
            const int64_t nn = (H.level_n[l] + kFanout - 1) / kFanout;
            H.level_off[l + 1] = node_count;
            H.level_n[l + 1] = nn;
            for (int64_t j = 0; j < nn; ++j) {
                const int64_t c0 = H.level_off[l] + j * kFanout;
                const int32_t nc = (int32_t)std::min<int64_t>(kFanout, H.level_n[l] - j * kFanout);
                per_level[l + 1].push_back({node_count + j, c0, nc, 0});
            }
            node_count += nn;
            ++l;
        }
        H.n_levels = l + 1;
        P.n_levels = std::max(P.n_levels, H.n_levels);
    }
    P.n_nodes = node_count;
    P.nodes.assign((size_t)node_count, NodeChild{0, 0, 0, 0});
    for (int64_t b = 0; b < P.n_buckets; ++b) P.nodes[(size_t)b].last = b;
    for (int l = 1; l <= kMaxLevels; ++l)
        for (auto& t : per_level[l])
            P.nodes[(size_t)t.node] =
                NodeChild{t.child0, P.nodes[(size_t)(t.child0 + t.nchild - 1)].last, t.nchild, 0};
    P.level_task_off[0] = 0;
    for (int l = 1; l < P.n_levels; ++l) {
        for (auto& t : per_level[l]) P.node_tasks.push_back(t);
        P.level_task_off[l] = (int64_t)P.node_tasks.size();
    }
    // gravity work items (i-blocks and tiles of the launch shape)
    choose_splits(P.halos, w.partial_rows, slots, shape);
    int64_t prow = 0;
    {
    const int64_t kIBlock = (int64_t)shape.ireg * shape.nt, kGravTileJ = shape.nt;
    for (int h = 0; h < n_halos; ++h) {
        HaloDev& H = P.halos[h];
        H.part_base = prow;
        prow += H.n * H.grav_split;
        if (H.tree_alpha > 0.0) continue;   // the tree walk covers this halo
        const int64_t tiles = (H.n + kGravTileJ - 1) / kGravTileJ;
        for (int s = 0; s < H.grav_split; ++s) {
            const int64_t t0 = tiles * s / H.grav_split, t1 = tiles * (s + 1) / H.grav_split;
            const int64_t j0 = H.offset + t0 * kGravTileJ;
            const int64_t j1 = std::min<int64_t>(H.offset + H.n, H.offset + t1 * kGravTileJ);
            for (int64_t i0 = 0; i0 < H.n; i0 += kIBlock)
                P.items.push_back({H.offset + i0, j0, j1, h, s});
        }
    }
    }
    // Block-step ticks (the default launch shape): a tick may hold only a few active i-blocks (they come
    // first in the tick's order), so its items cut j finer, into up to
    // kTickSplit ranges, to keep the device busy; their partial rows are their own.
    bool blocks = false;
    for (const auto& H : P.halos)
        if (H.max_bin > 0 && !(H.tree_alpha > 0.0)) blocks = true;
    if (blocks) {
        const int64_t kIBlock = kGravThreads * 4;
        int64_t trow = 0;
        for (int h = 0; h < n_halos; ++h) {
            HaloDev& H = P.halos[h];
            if (H.tree_alpha > 0.0) continue;
            const int64_t tiles = (H.n + kGravTileJ - 1) / kGravTileJ;
            H.tick_split = (int32_t)std::max<int64_t>(1, std::min<int64_t>(kTickSplit, tiles));
            H.tick_part_base = trow;
            trow += H.n * H.tick_split;
            for (int s = 0; s < H.tick_split; ++s) {
                const int64_t t0 = tiles * s / H.tick_split, t1 = tiles * (s + 1) / H.tick_split;
                const int64_t j0 = H.offset + t0 * kGravTileJ;
                const int64_t j1 = std::min<int64_t>(H.offset + H.n, H.offset + t1 * kGravTileJ);
                for (int64_t i0 = 0; i0 < H.n; i0 += kIBlock)
                    P.items_tick.push_back({H.offset + i0, j0, j1, h, s});
            }
        }
        P.tick_rows = trow;
    }
    make_sym_items(P.halos, shape, sym_min_n, sym_slots, P.sym_items);
    P.n_sym_items = (int64_t)P.sym_items.size();
    // largest items first so that the uneven tail is short, those of the halos
    // without symmetric tiles ahead of the others; a tick's active i-blocks
    // come first, so its items are ordered by i-block within a j size
    std::stable_sort(P.items.begin(), P.items.end(), [&](const GravItem& a, const GravItem& b) {
        const int sa = P.halos[a.halo].grav_sym, sb = P.halos[b.halo].grav_sym;
        if (sa != sb) return sa < sb;
        return (a.j1 - a.j0) > (b.j1 - b.j0);
    });
    P.n_items_nosym = 0;
    for (const auto& it : P.items)
        if (!P.halos[it.halo].grav_sym) ++P.n_items_nosym;
    std::stable_sort(P.items_tick.begin(), P.items_tick.end(),
                     [](const GravItem& a, const GravItem& b) { return a.i0 < b.i0; });
    P.n_items = (int64_t)P.items.size();
    P.n_blocks = (int64_t)P.blocks.size();
    int hb = 0;
    while ((1 << hb) < n_halos) ++hb;
    P.rank_shift = 48;
    for (const auto& H : P.halos)
        if (H.max_bin > 0 && !(H.tree_alpha > 0.0)) P.rank_shift = 49;
    P.key_bits = P.rank_shift + hb;
    P.halo_bits = hb;
    P.sort_blocks = (P.n_sorted + kSortBlock * kSortItems - 1) / (kSortBlock * kSortItems);
    if (prow > w.partial_rows || P.n_items > w.items_cap || P.n_blocks > w.blocks_cap ||
        P.n_buckets > w.buckets_cap || P.n_nodes > w.nodes_cap ||
        (int64_t)P.node_tasks.size() > w.nodes_cap) {
        why = "launch plan exceeds the context's table capacity";
        return false;
    }
    return true;
}

// Tables of block-step ticks, sized on the first plan that needs them.
inline bool ensure_tick_tables(Scratch& w, const Plan& P, std::string& why)
{
    if ((int64_t)P.items_tick.size() > w.items_tick_cap) {
        dfree(w.items_tick);
        w.items_tick_cap = 0;
        if (!dalloc(w.items_tick, (int64_t)P.items_tick.size())) {
            why = "out of device memory for the block-step work items";
            return false;
        }
        w.items_tick_cap = (int64_t)P.items_tick.size();
    }
    if (P.tick_rows > w.partial_tick_rows) {
        dfree(w.partial_tick);
        w.partial_tick_rows = 0;
        if (!dalloc(w.partial_tick, P.tick_rows)) {
            why = "out of device memory for the block-step partial rows";
            return false;
        }
        w.partial_tick_rows = P.tick_rows;
    }
    return true;
}

// Tables of the symmetric tiles, sized on the first plan that needs them.
inline bool ensure_sym_tables(Scratch& w, const Plan& P, std::string& why)
{
    if (P.n_sym_items == 0) return true;
    if (P.n_sym_items > w.sym_items_cap) {
        dfree(w.sym_items);
        w.sym_items_cap = 0;
        if (!dalloc(w.sym_items, P.n_sym_items)) {
            why = "out of device memory for the symmetric work items";
            return false;
        }
        w.sym_items_cap = P.n_sym_items;
    }
    if (P.n_sorted > w.symacc_n) {
        dfree(w.symacc);
        w.symacc_n = 0;
        if (!dalloc(w.symacc, 4 * P.n_sorted)) {
            why = "out of device memory for the symmetric tiles' totals";
            return false;
        }
        w.symacc_n = P.n_sorted;
    }
    return true;
}

inline hipError_t upload_plan(const Plan& P, const Scratch& w)
{
    hipError_t e = hipMemcpy(w.halos, P.halos.data(), sizeof(HaloDev) * P.halos.size(),
                             hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(w.blocks, P.blocks.data(), sizeof(StreamBlock) * P.blocks.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(w.items, P.items.data(), sizeof(GravItem) * P.items.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(w.buckets, P.buckets.data(), sizeof(BucketInfo) * P.buckets.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(w.nodes, P.nodes.data(), sizeof(NodeChild) * P.nodes.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess && !P.sym_items.empty())
        e = hipMemcpy(w.sym_items, P.sym_items.data(), sizeof(SymItem) * P.sym_items.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess && !P.items_tick.empty())
        e = hipMemcpy(w.items_tick, P.items_tick.data(), sizeof(GravItem) * P.items_tick.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess && !P.node_tasks.empty())
        e = hipMemcpy(w.node_tasks, P.node_tasks.data(), sizeof(NodeTask) * P.node_tasks.size(),
                      hipMemcpyHostToDevice);
    return e;
}

}  // namespace sidm
