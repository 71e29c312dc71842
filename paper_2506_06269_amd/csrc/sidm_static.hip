// sidm_static.hip -- sidm_gravity_static: the pass of sidm_gravity (cell list,
// direct-sum tiles, host, finalize) for one halo of at most SIDM_STATIC_MAX_N
// particles, with every scratch buffer placed in one fixed array of the
// library instead of a context's allocations.  For callers that cannot
// allocate device memory.  The kernels are those of sidm_gravity; only the
// launch tables are written by a kernel from the halo's parameters instead of
// being uploaded from the host.
#include <cstdarg>
#include <cstdio>
#include <mutex>

#include "sidm_plan.hpp"

namespace sidm {
hipError_t launch_gravity(bool mixed, const Plan& P, Scratch& w, const sidm_state* s, int kick,
                          hipStream_t st, hipEvent_t tile_begin, hipEvent_t tile_end, int tick = 0,
                          int bmax = 0);
hipError_t launch_cell_list(const Plan& plan, const sidm_state* s, Scratch& w, hipStream_t st,
                            int tick = 0, int bmax = 0);
int64_t gravity_slots(int device);

namespace {

constexpr int64_t kMaxN = SIDM_STATIC_MAX_N;
constexpr int64_t kMaxSplit = 4;
constexpr int64_t kIBlock = kGravThreads * 4;
constexpr int64_t kBlocksMax = kMaxN / kStreamBlock + 1;
constexpr int64_t kBucketsMax = kMaxN / kBucket + 1;
constexpr int64_t kNodesMax = 2 * kBucketsMax + kMaxLevels + 1;
constexpr int64_t kItemsMax = kMaxSplit * (kMaxN / kIBlock + 1);
constexpr int64_t kSortBlocksMax = kMaxN / (kSortBlock * kSortItems) + 1;
constexpr int64_t kHistMax = kSortBlocksMax * (1 << kSortBits) + 1;

// Byte offsets of the buffers inside the array (each aligned to 256 bytes).
struct Layout {
    size_t halos, blocks, items, buckets, node_tasks, nodes, bsum, cref, bbox, xm32, partial;
    size_t keys0, keys1, vals0, vals1, hist, scan_part, sx, sy, sz, sp4, sh, sm, perm, box, sub,
        sub_n, total;
};

constexpr size_t take(size_t& off, size_t bytes)
{
    const size_t o = (off + 255) & ~size_t(255);
    off = o + bytes;
    return o;
}

constexpr Layout make_layout()
{
    Layout L{};
    size_t off = 0;
    L.halos = take(off, sizeof(HaloDev));
    L.blocks = take(off, sizeof(StreamBlock) * kBlocksMax);
    L.items = take(off, sizeof(GravItem) * kItemsMax);
    L.buckets = take(off, sizeof(BucketInfo) * kBucketsMax);
    L.node_tasks = take(off, sizeof(NodeTask) * kNodesMax);
    L.nodes = take(off, sizeof(NodeChild) * kNodesMax);
    L.bsum = take(off, sizeof(double) * 7 * kBlocksMax);
    L.cref = take(off, sizeof(double) * 4);
    L.bbox = take(off, sizeof(double) * 6);
    L.xm32 = take(off, sizeof(float) * 4 * kMaxN);
    L.partial = take(off, sizeof(double) * 4 * kMaxSplit * kMaxN);
    L.keys0 = take(off, sizeof(unsigned long long) * kMaxN);
    L.keys1 = take(off, sizeof(unsigned long long) * kMaxN);
    L.vals0 = take(off, sizeof(uint32_t) * kMaxN);
    L.vals1 = take(off, sizeof(uint32_t) * kMaxN);
    L.hist = take(off, sizeof(uint32_t) * kHistMax);
    L.scan_part = take(off, sizeof(uint32_t) * kScanMaxSeg);
    L.sx = take(off, sizeof(double) * kMaxN);
    L.sy = take(off, sizeof(double) * kMaxN);
    L.sz = take(off, sizeof(double) * kMaxN);
    L.sp4 = take(off, sizeof(double) * 4 * kMaxN);
    L.sh = take(off, sizeof(double) * kMaxN);
    L.sm = take(off, sizeof(double) * kMaxN);
    L.perm = take(off, sizeof(uint32_t) * kMaxN);
    L.box = take(off, sizeof(double) * 6 * kNodesMax);
    L.sub = take(off, sizeof(SubRange) * kSubMax * kBucketsMax);
    L.sub_n = take(off, sizeof(int) * kBucketsMax);
    L.total = (off + 255) & ~size_t(255);
    return L;
}

constexpr Layout kLayout = make_layout();
static_assert(kLayout.total <= SIDM_STATIC_BYTES, "the fixed scratch array is too small");

}  // namespace
}  // namespace sidm

// The fixed scratch array: one copy per GPU, held until the process ends.
// Host code never uses this name as an address (on the host it only stands
// for the symbol); it takes the device address from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[SIDM_STATIC_BYTES];

namespace sidm {
namespace {

constexpr int kMaxDevices = 64;

struct DeviceScratch {
    std::once_flag once;
    unsigned char* ptr = nullptr;   // device address of `scratch` on this device
    hipError_t err = hipSuccess;
    int64_t slots = 0;              // resident blocks of the gravity tiles
};
DeviceScratch g_dev[kMaxDevices];

thread_local char g_err[256];

sidm_status fail(sidm_status r, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return r;
}

// The Scratch view of the array at device address base (host arithmetic only).
void carve(Scratch& w, unsigned char* base)
{
    const Layout& L = kLayout;
    w.halos = (HaloDev*)(base + L.halos);
    w.blocks = (StreamBlock*)(base + L.blocks);
    w.items = (GravItem*)(base + L.items);
    w.buckets = (BucketInfo*)(base + L.buckets);
    w.node_tasks = (NodeTask*)(base + L.node_tasks);
    w.nodes = (NodeChild*)(base + L.nodes);
    w.bsum = (double*)(base + L.bsum);
    w.cref = (double*)(base + L.cref);
    w.bbox = (double*)(base + L.bbox);
    w.xm32 = (float4*)(base + L.xm32);
    w.partial = (double4*)(base + L.partial);
    w.keys[0] = (unsigned long long*)(base + L.keys0);
    w.keys[1] = (unsigned long long*)(base + L.keys1);
    w.vals[0] = (uint32_t*)(base + L.vals0);
    w.vals[1] = (uint32_t*)(base + L.vals1);
    w.hist = (uint32_t*)(base + L.hist);
    w.scan_part = (uint32_t*)(base + L.scan_part);
    w.sx = (double*)(base + L.sx);
    w.sy = (double*)(base + L.sy);
    w.sz = (double*)(base + L.sz);
    w.sp4 = (double4*)(base + L.sp4);
    w.sh = (double*)(base + L.sh);
    w.sm = (double*)(base + L.sm);
    w.perm = (uint32_t*)(base + L.perm);
    w.box = (double*)(base + L.box);
    w.sub = (SubRange*)(base + L.sub);
    w.sub_n = (int*)(base + L.sub_n);
    w.max_particles = kMaxN;
    w.max_halos = 1;
    w.partial_rows = kMaxSplit * kMaxN;
}

// The launch tables of one halo (the same tables the host plan of
// sidm_gravity holds for it), one entry per thread: streaming blocks,
// buckets, tree nodes and their tasks, gravity work items.
__global__ __launch_bounds__(256) void k_static_plan(HaloDev H, int64_t n_blocks, int64_t n_buckets,
                                                     int64_t n_nodes, int64_t n_items,
                                                     int64_t n_plan,
                                                     HaloDev* __restrict__ halos,
                                                     StreamBlock* __restrict__ blocks,
                                                     BucketInfo* __restrict__ buckets,
                                                     NodeChild* __restrict__ nodes,
                                                     NodeTask* __restrict__ tasks,
                                                     GravItem* __restrict__ items)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= n_plan) return;
    const int64_t n = H.n;
    if (t == 0) halos[0] = H;
    if (t < n_blocks) {
        const int64_t s0 = t * kStreamBlock;
        blocks[t] = StreamBlock{H.offset + s0, (int32_t)min((int64_t)kStreamBlock, n - s0), 0};
    }
    if (t < n_buckets) {
        const int64_t b0 = t * kBucket;
        buckets[t] = BucketInfo{b0, (int32_t)min((int64_t)kBucket, n - b0), 0};
        nodes[t] = NodeChild{0, t, 0, 0};
    } else if (t < n_nodes) {
        // internal node: level l, index j within the level
        int l = 1;
        while (l + 1 < H.n_levels && t >= H.level_off[l + 1]) ++l;
        const int64_t j = t - H.level_off[l];
        int64_t span = 1;   // buckets under one node of level l
        for (int q = 0; q < l; ++q) span *= kFanout;
        const int64_t child0 = H.level_off[l - 1] + j * kFanout;
        const int32_t nchild = (int32_t)min((int64_t)kFanout, H.level_n[l - 1] - j * kFanout);
        const int64_t last = min((j + 1) * span, H.level_n[0]) - 1;
        nodes[t] = NodeChild{child0, last, nchild, 0};
        int64_t task = j;   // tasks are grouped by level, in node order
        for (int q = 1; q < l; ++q) task += H.level_n[q];
        tasks[task] = NodeTask{t, child0, nchild, 0};
    }
    if (t < n_items) {
        const int64_t n_ib = (n + kIBlock - 1) / kIBlock;
        const int64_t s = t / n_ib, ib = t % n_ib;
        const int64_t tiles = (n + kGravTileJ - 1) / kGravTileJ;
        const int64_t t0 = tiles * s / H.grav_split, t1 = tiles * (s + 1) / H.grav_split;
        const int64_t j0 = H.offset + t0 * kGravTileJ;
        const int64_t j1 = min(H.offset + n, H.offset + t1 * kGravTileJ);
        items[t] = GravItem{H.offset + ib * kIBlock, j0, j1, 0, (int32_t)s};
    }
}

}  // namespace
}  // namespace sidm

using namespace sidm;

const char* sidm_static_error_text() { return g_err; }

extern "C" sidm_status sidm_gravity_static(const sidm_halo* halo, const sidm_state* s,
                                           sidm_precision prec, void* stream)
{
    g_err[0] = '\0';
    if (!halo || !s) return fail(SIDM_ERR_INVALID, "halo and state are required");
    if (!s->x || !s->y || !s->z || !s->m || !s->ax || !s->ay || !s->az || !s->pot)
        return fail(SIDM_ERR_INVALID, "state x, y, z, m, ax, ay, az and pot are required");
    if (prec != SIDM_PREC_FP64 && prec != SIDM_PREC_MIXED)
        return fail(SIDM_ERR_INVALID, "unknown precision %d", (int)prec);
    char msg[200];
    sidm_status r = check_halo(*halo, NEED_GRAV, msg, sizeof msg);
    if (r != SIDM_OK) return fail(r, "%s", msg);
    if (halo->n > kMaxN)
        return fail(SIDM_ERR_CAPACITY, "n = %lld exceeds the fixed scratch's limit of %lld",
                    (long long)halo->n, (long long)kMaxN);
    if (halo->tree_alpha > 0.0)
        return fail(SIDM_ERR_UNSUPPORTED, "the tree walk is not available here (tree_alpha > 0)");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(SIDM_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(SIDM_ERR_INVALID, "device %d", dev);
    DeviceScratch& D = g_dev[dev];
    std::call_once(D.once, [&] {
        void* p = nullptr;
        D.err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        D.ptr = (unsigned char*)p;
        D.slots = gravity_slots(dev);
    });
    if (D.err != hipSuccess || !D.ptr)
        return fail(SIDM_ERR_HIP, "hipGetSymbolAddress: %s", hipGetErrorString(D.err));

    // the plan of one halo, as build_plan makes it for sidm_gravity
    const int64_t n = halo->n;
    HaloDev H;
    fill_halo_params(H, *halo);
    Plan P;
    P.n_halos = 1;
    P.n_sorted = n;
    P.n_blocks = (n + kStreamBlock - 1) / kStreamBlock;
    P.n_buckets = (n + kBucket - 1) / kBucket;
    H.level_off[0] = 0;
    H.level_n[0] = P.n_buckets;
    int64_t count = P.n_buckets;
    int l = 0;
    P.level_task_off[0] = 0;
    while (H.level_n[l] > 1) {
        H.level_off[l + 1] = count;
        H.level_n[l + 1] = (H.level_n[l] + kFanout - 1) / kFanout;
        count += H.level_n[l + 1];
        P.level_task_off[l + 1] = P.level_task_off[l] + H.level_n[l + 1];
        ++l;
    }
    H.n_levels = l + 1;
    P.n_levels = H.n_levels;
    P.n_nodes = count;
    const int64_t want = 2 * ((int64_t)std::max(halo->k, 1) + 1);
    const int64_t wb = std::min<int64_t>(P.n_buckets, (want + kBucket - 1) / kBucket + 1);
    H.win_lo = (int32_t)(wb / 2);
    H.win_hi = (int32_t)(wb - 1 - wb / 2);
    // j-splits: with all items resident at once (at most 256 items here), the
    // split that choose_splits takes is the smallest with the shortest longest
    // j-range; without an occupancy figure, the largest
    const int64_t tiles = (n + kGravTileJ - 1) / kGravTileJ;
    const int64_t smax = std::min<int64_t>(kMaxSplit, tiles);
    int64_t split = smax;
    if (D.slots > 0) {
        int64_t best = tiles;
        split = 1;
        for (int64_t sp = 2; sp <= smax; ++sp)
            if ((tiles + sp - 1) / sp < best) {
                best = (tiles + sp - 1) / sp;
                split = sp;
            }
    }
    H.grav_split = (int32_t)split;
    const int64_t n_ib = (n + kIBlock - 1) / kIBlock;
    P.n_items = split * n_ib;
    P.key_bits = 48;
    P.rank_shift = 48;
    P.sort_blocks = (n + kSortBlock * kSortItems - 1) / (kSortBlock * kSortItems);

    Scratch w;
    carve(w, D.ptr);
    w.grav_slots = D.slots;
    hipStream_t st = (hipStream_t)stream;
    const int64_t n_plan = std::max(P.n_nodes, P.n_items);
    hipLaunchKernelGGL(k_static_plan, dim3((unsigned)((n_plan + 255) / 256)), dim3(256), 0, st,
                       H, P.n_blocks, P.n_buckets, P.n_nodes, P.n_items, n_plan, w.halos, w.blocks,
                       w.buckets, w.nodes, w.node_tasks, w.items);
    e = hipGetLastError();
    // the passes read positions and masses only
    sidm_state local = *s;
    local.vx = local.vy = local.vz = nullptr;
    local.id = nullptr;
    local.h = nullptr;
    if (e == hipSuccess) e = launch_cell_list(P, &local, w, st);
    if (e == hipSuccess)
        e = launch_gravity(prec == SIDM_PREC_MIXED, P, w, &local, 0, st, nullptr, nullptr);
    if (e != hipSuccess) return fail(SIDM_ERR_HIP, "gravity launch: %s", hipGetErrorString(e));
    return SIDM_OK;
}
