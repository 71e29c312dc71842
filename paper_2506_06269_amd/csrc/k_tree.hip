// k_tree.hip -- cell list for the neighbour and pair searches: particles of
// each halo are ordered along a Morton curve (48-bit keys over the halo's
// bounding box, halo rank in the high bits) by a stable LSD radix sort, cut
// into buckets of kBucket consecutive particles, and the bucket bounding boxes
// are merged kFanout at a time into a search tree per halo.
#include "sidm_plan.hpp"
#include "sidm_steps.hpp"

namespace sidm {

// ---------------------------------------------------------------- bounding boxes
__global__ __launch_bounds__(kStreamBlock) void k_block_bbox(
    const double* __restrict__ x, const double* __restrict__ y, const double* __restrict__ z,
    const StreamBlock* __restrict__ blocks, double* __restrict__ bout)
{
    __shared__ double lo[3][kStreamBlock], hi[3][kStreamBlock];
    const StreamBlock B = blocks[blockIdx.x];
    const int t = threadIdx.x;
    const int64_t i = B.start + (t < B.count ? t : 0);
    const double p[3] = {x[i], y[i], z[i]};
    for (int c = 0; c < 3; ++c) { lo[c][t] = p[c]; hi[c][t] = p[c]; }
    __syncthreads();
    for (int s = kStreamBlock / 2; s > 0; s >>= 1) {
        if (t < s)
            for (int c = 0; c < 3; ++c) {
                lo[c][t] = fmin(lo[c][t], lo[c][t + s]);
                hi[c][t] = fmax(hi[c][t], hi[c][t + s]);
            }
        __syncthreads();
    }
    if (t < 3) {
        bout[7 * (int64_t)blockIdx.x + t] = lo[t][0];
        bout[7 * (int64_t)blockIdx.x + 3 + t] = hi[t][0];
    }
}

__global__ __launch_bounds__(kStreamBlock) void k_halo_bbox(
    const HaloDev* __restrict__ halos, const double* __restrict__ bin, double* __restrict__ bbox)
{
    __shared__ double lo[3][kStreamBlock], hi[3][kStreamBlock];
    const HaloDev& H = halos[blockIdx.x];
    const int t = threadIdx.x;
    const int64_t nb = (H.n + kStreamBlock - 1) / kStreamBlock;
    double l[3] = {INFINITY, INFINITY, INFINITY}, u[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t b = t; b < nb; b += kStreamBlock)
        for (int c = 0; c < 3; ++c) {
            l[c] = fmin(l[c], bin[7 * (H.stream_block0 + b) + c]);
            u[c] = fmax(u[c], bin[7 * (H.stream_block0 + b) + 3 + c]);
        }
    for (int c = 0; c < 3; ++c) { lo[c][t] = l[c]; hi[c][t] = u[c]; }
    __syncthreads();
    for (int s = kStreamBlock / 2; s > 0; s >>= 1) {
        if (t < s)
            for (int c = 0; c < 3; ++c) {
                lo[c][t] = fmin(lo[c][t], lo[c][t + s]);
                hi[c][t] = fmax(hi[c][t], hi[c][t + s]);
            }
        __syncthreads();
    }
    if (t < 3) {
        bbox[6 * blockIdx.x + t] = lo[t][0];
        bbox[6 * blockIdx.x + 3 + t] = hi[t][0];
    }
}

// ---------------------------------------------------------------- Morton keys
__device__ inline unsigned long long spread3(unsigned v)   // bit k -> bit 3k
{
    unsigned long long x = v & 0xFFFFull;
    x = (x | (x << 32)) & 0x001F00000000FFFFull;
    x = (x | (x << 16)) & 0x001F0000FF0000FFull;
    x = (x | (x << 8)) & 0x100F00F00F00F00Full;
    x = (x | (x << 4)) & 0x10C30C30C30C30C3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

__device__ inline unsigned quant16(double v, double lo, double inv)
{
    double q = (v - lo) * inv;
    q = fmin(fmax(q, 0.0), 65535.0);
    return (unsigned)q;
}

__global__ __launch_bounds__(kStreamBlock) void k_morton_keys(
    const double* __restrict__ x, const double* __restrict__ y, const double* __restrict__ z,
    const StreamBlock* __restrict__ blocks, const HaloDev* __restrict__ halos,
    const double* __restrict__ bbox, unsigned long long* __restrict__ keys,
    uint32_t* __restrict__ vals, const int8_t* __restrict__ bin, int tick, int bmax,
    int rank_shift)
{
    const StreamBlock B = blocks[blockIdx.x];
    const int t = threadIdx.x;
    if (t >= B.count) return;
    const HaloDev& H = halos[B.halo];
    const int64_t i = B.start + t;
    const double* bb = bbox + 6 * B.halo;
    double ext = fmax(fmax(bb[3] - bb[0], bb[4] - bb[1]), bb[5] - bb[2]);
    const double inv = ext > 0.0 ? 65535.0 / ext : 0.0;
    const unsigned long long code = spread3(quant16(x[i], bb[0], inv)) |
                                    (spread3(quant16(y[i], bb[1], inv)) << 1) |
                                    (spread3(quant16(z[i], bb[2], inv)) << 2);
    const int64_t pos = H.sbase + (i - H.offset);
    // in a tick of block steps the inactive particles of a direct-sum halo sort
    // after its active ones (bit 48), so the active ones fill whole i-blocks
    unsigned long long later = 0ull;
    if (rank_shift > 48 && tick > 0 && !(H.tree_alpha > 0.0) &&
        !bin_active(H, bin[i], local_tick(H, tick, bmax)))
        later = 1ull << 48;
    keys[pos] = ((unsigned long long)H.rank << rank_shift) | later | code;
    vals[pos] = (uint32_t)i;
}

// ---------------------------------------------------------------- radix sort
constexpr int kTile = kSortBlock * kSortItems;

__global__ __launch_bounds__(kSortBlock) void k_sort_count(
    const unsigned long long* __restrict__ keys, int64_t n, int shift, uint32_t* __restrict__ hist,
    int64_t nblk)
{
    __shared__ uint32_t cnt[1 << kSortBits];
    const int t = threadIdx.x;
    cnt[t] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTile;
    for (int r = 0; r < kSortItems; ++r) {
        const int64_t i = base + (int64_t)r * kSortBlock + t;
        if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 0xFF], 1u);
    }
    __syncthreads();
    hist[(int64_t)t * nblk + blockIdx.x] = cnt[t];
}

// Exclusive scan of len counts, in place, in three launches: each of nseg
// blocks sums its segment of seg entries (a multiple of the tile), one block
// scans the nseg sums, and each block rescans its segment from its offset in
// tiles of kScanTile entries, four consecutive ones per thread (coalesced).
constexpr int kScanThreads = 256;
constexpr int kScanTile = 4 * kScanThreads;

// Exclusive prefix of v over the block's threads (in thread order); total
// receives the block's sum.  Every thread of the block must call it.
__device__ inline uint32_t block_scan_excl(uint32_t v, uint32_t* sw, uint32_t& total)
{
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    uint32_t inc = v;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t u = __shfl_up(inc, o, 64);
        if (lane >= o) inc += u;
    }
    if (lane == 63) sw[wv] = inc;
    __syncthreads();
    uint32_t off = 0;
    total = 0;
    for (int w = 0; w < kScanThreads / 64; ++w) {
        const uint32_t s = sw[w];
        if (w < wv) off += s;
        total += s;
    }
    __syncthreads();   // sw is reused by the next call
    return off + inc - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const uint32_t* __restrict__ a,
                                                              int64_t len, int64_t seg,
                                                              uint32_t* __restrict__ part)
{
    __shared__ uint32_t sw[kScanThreads / 64];
    const int64_t b0 = (int64_t)blockIdx.x * seg;
    const int64_t b1 = b0 + seg < len ? b0 + seg : len;
    uint32_t s = 0;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += kScanThreads) s += a[i];
    uint32_t total;
    (void)block_scan_excl(s, sw, total);
    if (threadIdx.x == 0) part[blockIdx.x] = total;
}

// Exclusive scan of n <= kScanMaxSeg segment sums, in place, by one block.
__global__ __launch_bounds__(kScanMaxSeg) void k_scan_parts(uint32_t* __restrict__ part, int n)
{
    __shared__ uint32_t p[kScanMaxSeg];
    const int t = threadIdx.x;
    const uint32_t v = t < n ? part[t] : 0u;
    p[t] = v;
    __syncthreads();
    for (int off = 1; off < kScanMaxSeg; off <<= 1) {
        const uint32_t u = t >= off ? p[t - off] : 0u;
        __syncthreads();
        p[t] += u;
        __syncthreads();
    }
    if (t < n) part[t] = p[t] - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply(uint32_t* __restrict__ a,
                                                             int64_t len, int64_t seg,
                                                             const uint32_t* __restrict__ part)
{
    __shared__ uint32_t sw[kScanThreads / 64];
    const int64_t b0 = (int64_t)blockIdx.x * seg;
    const int64_t b1 = b0 + seg < len ? b0 + seg : len;
    uint32_t carry = part[blockIdx.x];
    for (int64_t t0 = b0; t0 < b1; t0 += kScanTile) {
        const int64_t i0 = t0 + 4 * (int64_t)threadIdx.x;
        uint32_t v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = i0 + q < b1 ? a[i0 + q] : 0u;
        uint32_t total;
        uint32_t run = carry + block_scan_excl(v[0] + v[1] + v[2] + v[3], sw, total);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (i0 + q < b1) a[i0 + q] = run;
            run += v[q];
        }
        carry += total;
    }
}

// Stable scatter: items of a tile are taken 256 at a time in index order; the
// rank of an item among equal digits is the running count of the digit plus
// the count in earlier waves plus the count in lower lanes of its own wave.
__global__ __launch_bounds__(kSortBlock) void k_sort_scatter(
    const unsigned long long* __restrict__ kin, const uint32_t* __restrict__ vin,
    unsigned long long* __restrict__ kout, uint32_t* __restrict__ vout, int64_t n, int shift,
    const uint32_t* __restrict__ hist, int64_t nblk)
{
    constexpr int kWaves = kSortBlock / 64;
    __shared__ uint32_t run[1 << kSortBits];
    __shared__ uint32_t wcnt[kWaves][1 << kSortBits];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    run[t] = hist[(int64_t)t * nblk + blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * kTile;
    const unsigned long long lt = (1ull << lane) - 1ull;
    for (int r = 0; r < kSortItems; ++r) {
        const int64_t i = base + (int64_t)r * kSortBlock + t;
        const bool valid = i < n;
        const unsigned long long key = valid ? kin[i] : 0ull;
        const uint32_t val = valid ? vin[i] : 0u;
        const uint32_t d = (uint32_t)(key >> shift) & 0xFFu;
#pragma unroll
        for (int q = 0; q < kWaves; ++q) wcnt[q][t] = 0;
        __syncthreads();
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < kSortBits; ++bit) {
            const bool set = (d >> bit) & 1u;
            const unsigned long long m = __ballot(set);
            peers &= set ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lt);
        if (valid && rank == (uint32_t)__popcll(peers) - 1u) wcnt[w][d] = rank + 1u;
        __syncthreads();
        {
            uint32_t acc = run[t];
#pragma unroll
            for (int q = 0; q < kWaves; ++q) {
                const uint32_t c = wcnt[q][t];
                wcnt[q][t] = acc;
                acc += c;
            }
            run[t] = acc;
        }
        __syncthreads();
        if (valid) {
            const uint32_t pos = wcnt[w][d] + rank;
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- permute
__global__ __launch_bounds__(kStreamBlock) void k_permute(
    int64_t n, const uint32_t* __restrict__ order, const double* __restrict__ x,
    const double* __restrict__ y, const double* __restrict__ z, const double* __restrict__ vx,
    const double* __restrict__ vy, const double* __restrict__ vz, const double* __restrict__ m,
    const uint32_t* __restrict__ id, const double* __restrict__ h, double* __restrict__ sx,
    double* __restrict__ sy, double* __restrict__ sz, double4* __restrict__ sp4,
    double* __restrict__ svx,
    double* __restrict__ svy, double* __restrict__ svz, double* __restrict__ sm,
    uint32_t* __restrict__ sid, double* __restrict__ sh, uint32_t* __restrict__ perm)
{
    const int64_t p = (int64_t)blockIdx.x * kStreamBlock + threadIdx.x;
    if (p >= n) return;
    const uint32_t o = order[p];
    const double px = x[o], py = y[o], pz = z[o];
    sx[p] = px; sy[p] = py; sz[p] = pz;
    sp4[p] = make_double4(px, py, pz, 0.0);
    if (vx) { svx[p] = vx[o]; svy[p] = vy[o]; svz[p] = vz[o]; }
    sm[p] = m[o];
    if (id) sid[p] = id[o];
    sh[p] = h ? h[o] : 0.0;
    perm[p] = o;
}

// ---------------------------------------------------------------- boxes
__device__ inline double wave_min(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ inline double wave_max(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ inline void range_box(int lo, int hi, int lane, double px, double py, double pz,
                                 double* o)
{
    const bool in = lane >= lo && lane < hi;
    o[0] = wave_min(in ? px : INFINITY);
    o[1] = wave_min(in ? py : INFINITY);
    o[2] = wave_min(in ? pz : INFINITY);
    o[3] = wave_max(in ? px : -INFINITY);
    o[4] = wave_max(in ? py : -INFINITY);
    o[5] = wave_max(in ? pz : -INFINITY);
}

__device__ inline double box_diag2(const double* b)
{
    const double ex = b[3] - b[0], ey = b[4] - b[1], ez = b[5] - b[2];
    return ex * ex + ey * ey + ez * ez;
}

// Split point of the lanes [lo, hi) at their coarsest internal Morton boundary,
// kept only if it at least halves the count-weighted extent (count x box
// diagonal summed over the pieces): a dense group is then separated from a few
// far members even when the far piece stays large.  -1 if not kept.
__device__ inline int split_range(int lo, int hi, int lane, unsigned long long key, double px,
                                  double py, double pz, double* ba, double* bb)
{
    if (hi - lo < 2) return -1;
    const unsigned long long kf = __shfl(key, lo, 64), kl = __shfl(key, hi - 1, 64);
    if (kf == kl) return -1;
    const int hb = 63 - __clzll((long long)(kf ^ kl));
    const bool low = lane >= lo && lane < hi && !(((key ^ kf) >> hb) & 1ull);
    const int s = lo + __popcll(__ballot(low));
    if (s <= lo || s >= hi) return -1;
    double full[6];
    range_box(lo, hi, lane, px, py, pz, full);
    range_box(lo, s, lane, px, py, pz, ba);
    range_box(s, hi, lane, px, py, pz, bb);
    const double before = (hi - lo) * sqrt(box_diag2(full));
    const double after = (s - lo) * sqrt(box_diag2(ba)) + (hi - s) * sqrt(box_diag2(bb));
    return after < 0.5 * before ? s : -1;
}

// One wave per bucket: the box, up to kSubMax compact sub-ranges, and (when
// cbox is given) the boxes of its chunks of kChunk particles (an empty
// chunk gets the empty box [+inf, -inf], which no distance test passes).
__global__ __launch_bounds__(256) void k_bucket_boxes(
    const BucketInfo* __restrict__ buckets, int64_t nb, const double* __restrict__ sx,
    const double* __restrict__ sy, const double* __restrict__ sz,
    const unsigned long long* __restrict__ skeys, double* __restrict__ box,
    SubRange* __restrict__ sub, int* __restrict__ sub_n, double* __restrict__ cbox)
{
    const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (b >= nb) return;
    const int lane = threadIdx.x & 63;
    const BucketInfo B = buckets[b];
    const int64_t p = B.start + (lane < B.count ? lane : 0);
    const double px = sx[p], py = sy[p], pz = sz[p];
    const unsigned long long key = skeys[p];
    double full[6];
    range_box(0, B.count, lane, px, py, pz, full);
    if (lane == 0)
        for (int q = 0; q < 6; ++q) box[6 * b + q] = full[q];
    if (cbox)
        for (int g = 0; g < kChunks; ++g) {
            double cb[6];
            range_box(g * kChunk, min(B.count, (g + 1) * kChunk), lane, px, py, pz, cb);
            if (lane == 0)
                for (int q = 0; q < 6; ++q) cbox[6 * (kChunks * b + g) + q] = cb[q];
        }
    // up to two levels of splits
    int lo[kSubMax], hi[kSubMax];
    double bx[kSubMax][6];
    int n = 1;
    lo[0] = 0; hi[0] = B.count;
    for (int q = 0; q < 6; ++q) bx[0][q] = full[q];
    for (int level = 0; level < 2; ++level) {
        const int m = n;
        for (int r = 0; r < m; ++r) {
            double ba[6], bb[6];
            const int sp = split_range(lo[r], hi[r], lane, key, px, py, pz, ba, bb);
            if (sp > 0 && n < kSubMax) {
                lo[n] = sp; hi[n] = hi[r];
                hi[r] = sp;
                for (int q = 0; q < 6; ++q) { bx[r][q] = ba[q]; bx[n][q] = bb[q]; }
                ++n;
            }
        }
    }
    if (lane == 0) {
        // sub-ranges in particle order
        for (int a = 1; a < n; ++a)
            for (int c = a; c > 0 && lo[c] < lo[c - 1]; --c) {
                int t = lo[c]; lo[c] = lo[c - 1]; lo[c - 1] = t;
                t = hi[c]; hi[c] = hi[c - 1]; hi[c - 1] = t;
                for (int q = 0; q < 6; ++q) {
                    const double v = bx[c][q]; bx[c][q] = bx[c - 1][q]; bx[c - 1][q] = v;
                }
            }
        for (int r = 0; r < n; ++r) {
            SubRange R;
            R.off = lo[r];
            R.cnt = hi[r] - lo[r];
            for (int q = 0; q < 6; ++q) R.box[q] = bx[r][q];
            sub[kSubMax * b + r] = R;
        }
        sub_n[b] = n;
    }
}

// The largest kernel size of every bucket and (when chmax is given) of each of
// its chunks of kChunk particles (0 for an empty chunk).
__global__ __launch_bounds__(256) void k_bucket_hmax(
    const BucketInfo* __restrict__ buckets, int64_t nb, const double* __restrict__ sh,
    double* __restrict__ hmax, double* __restrict__ chmax)
{
    const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (b >= nb) return;
    const int lane = threadIdx.x & 63;
    const BucketInfo B = buckets[b];
    const double h = sh[B.start + (lane < B.count ? lane : 0)];
    const double v = wave_max(h);
    if (lane == 0) hmax[b] = v;
    if (chmax)
        for (int g = 0; g < kChunks; ++g) {
            const double c = wave_max(lane < B.count && lane / kChunk == g ? h : 0.0);
            if (lane == 0) chmax[kChunks * b + g] = c;
        }
}

__global__ __launch_bounds__(256) void k_node_boxes(const NodeTask* __restrict__ tasks,
                                                     int64_t nt, double* __restrict__ box)
{
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= nt) return;
    const NodeTask T = tasks[k];
    double o[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int c = 0; c < T.nchild; ++c) {
        const double* b = box + 6 * (T.child0 + c);
        for (int q = 0; q < 3; ++q) {
            o[q] = fmin(o[q], b[q]);
            o[3 + q] = fmax(o[3 + q], b[3 + q]);
        }
    }
    for (int q = 0; q < 6; ++q) box[6 * T.node + q] = o[q];
}

__global__ __launch_bounds__(256) void k_node_hmax(const NodeTask* __restrict__ tasks, int64_t nt,
                                                    double* __restrict__ hmax)
{
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= nt) return;
    const NodeTask T = tasks[k];
    double v = 0.0;
    for (int c = 0; c < T.nchild; ++c) v = fmax(v, hmax[T.child0 + c]);
    hmax[T.node] = v;
}

// ---------------------------------------------------------------- launchers
static unsigned grid_of(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

// about four tiles per segment, at most kScanMaxSeg segments
static void launch_scan(uint32_t* a, int64_t len, uint32_t* part, hipStream_t st)
{
    int64_t nseg = (len + 4 * kScanTile - 1) / (4 * kScanTile);
    nseg = nseg < 1 ? 1 : (nseg > kScanMaxSeg ? kScanMaxSeg : nseg);
    int64_t seg = (len + nseg - 1) / nseg;
    seg = (seg + kScanTile - 1) / kScanTile * kScanTile;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nseg), dim3(kScanThreads), 0, st, a, len, seg,
                       part);
    hipLaunchKernelGGL(k_scan_parts, dim3(1), dim3(kScanMaxSeg), 0, st, part, (int)nseg);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nseg), dim3(kScanThreads), 0, st, a, len, seg,
                       part);
}

// Stable LSD radix sort of keys[0] (with vals[0]) over their low key_bits
// bits, n keys; returns the index of the buffer pair that holds the result.
int launch_sort_keys(Scratch& w, int64_t n, int key_bits, hipStream_t st)
{
    int cur = 0;
    const int passes = (key_bits + kSortBits - 1) / kSortBits;
    const int64_t nblk = (n + kTile - 1) / kTile;
    for (int p = 0; p < passes; ++p) {
        const int shift = p * kSortBits;
        hipLaunchKernelGGL(k_sort_count, dim3((unsigned)nblk), dim3(kSortBlock), 0, st,
                           w.keys[cur], n, shift, w.hist, nblk);
        launch_scan(w.hist, nblk * (1 << kSortBits), w.scan_part, st);
        hipLaunchKernelGGL(k_sort_scatter, dim3((unsigned)nblk), dim3(kSortBlock), 0, st,
                           w.keys[cur], w.vals[cur], w.keys[cur ^ 1], w.vals[cur ^ 1], n, shift,
                           w.hist, nblk);
        cur ^= 1;
    }
    return cur;
}

hipError_t launch_cell_list(const Plan& P, const sidm_state* s, Scratch& w, hipStream_t st,
                            int tick, int bmax)
{
    const int64_t n = P.n_sorted;
    hipLaunchKernelGGL(k_block_bbox, dim3((unsigned)P.n_blocks), dim3(kStreamBlock), 0, st, s->x,
                       s->y, s->z, w.blocks, w.bsum);
    hipLaunchKernelGGL(k_halo_bbox, dim3(P.n_halos), dim3(kStreamBlock), 0, st, w.halos, w.bsum,
                       w.bbox);
    hipLaunchKernelGGL(k_morton_keys, dim3((unsigned)P.n_blocks), dim3(kStreamBlock), 0, st, s->x,
                       s->y, s->z, w.blocks, w.halos, w.bbox, w.keys[0], w.vals[0], w.bin,
                       tick, bmax, P.rank_shift);
    const int cur = launch_sort_keys(w, n, P.key_bits, st);
    hipLaunchKernelGGL(k_permute, dim3(grid_of(n, kStreamBlock)), dim3(kStreamBlock), 0, st, n,
                       w.vals[cur], s->x, s->y, s->z, s->vx, s->vy, s->vz, s->m, s->id, s->h,
                       w.sx, w.sy, w.sz, w.sp4, w.svx, w.svy, w.svz, w.sm, w.sid, w.sh, w.perm);
    w.skeys = w.keys[cur];
    hipLaunchKernelGGL(k_bucket_boxes, dim3(grid_of(P.n_buckets, 4)), dim3(256), 0, st, w.buckets,
                       P.n_buckets, w.sx, w.sy, w.sz, w.skeys, w.box, w.sub, w.sub_n, w.cbox);
    for (int l = 1; l < P.n_levels; ++l) {
        const int64_t t0 = P.level_task_off[l - 1], nt = P.level_task_off[l] - t0;
        if (nt > 0)
            hipLaunchKernelGGL(k_node_boxes, dim3(grid_of(nt, 256)), dim3(256), 0, st,
                               w.node_tasks + t0, nt, w.box);
    }
    return hipGetLastError();
}

hipError_t launch_tree_hmax(const Plan& P, Scratch& w, hipStream_t st)
{
    hipLaunchKernelGGL(k_bucket_hmax, dim3(grid_of(P.n_buckets, 4)), dim3(256), 0, st, w.buckets,
                       P.n_buckets, w.sh, w.hmax, w.chmax);
    for (int l = 1; l < P.n_levels; ++l) {
        const int64_t t0 = P.level_task_off[l - 1], nt = P.level_task_off[l] - t0;
        if (nt > 0)
            hipLaunchKernelGGL(k_node_hmax, dim3(grid_of(nt, 256)), dim3(256), 0, st,
                               w.node_tasks + t0, nt, w.hmax);
    }
    return hipGetLastError();
}

}  // namespace sidm
