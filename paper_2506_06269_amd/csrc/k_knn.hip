// k_knn.hip -- the SIDM kernel size h_i = distance to the k-th nearest other
// particle of the halo (Sec. 2: the kernel size is set by the next N_ngb
// neighbours).
//
// One wavefront per bucket of 64 Morton-consecutive particles, one particle
// per lane.  Candidates are staged bucket by bucket in LDS and every lane reads
// the same candidate (broadcast), as in the gravity tiles.  Selection works on
// values only:
//   1. a bound u_i^2 >= d2_(k) from a window of buckets around the bucket
//      (histogram of its distances, smallest bin edge holding k of them);
//   2. all buckets whose box lies within max_i u_i of the bucket's box are
//      visited through the search tree; each lane histograms its distances in
//      [0, u_i^2] into 32 bins (a private LDS column, no atomics) and keeps the
//      bin that holds the k-th;
//   3. a second visit collects that bin's members (at most 16) or, if it holds
//      more, refines the bin by its own min..max range; equal values end the
//      refinement at once.
// Distances d2 = (dx*dx + dy*dy) + dz*dz are evaluated in FP64 without fused
// multiply-add, the same expression the oracle uses, so h matches bit for bit.
#include "sidm_plan.hpp"

namespace sidm {

constexpr int kKnnBins = 32;
constexpr int kKnnSurv = 16;
constexpr int kKnnLevels = 6;
constexpr int kStackMax = 96;

struct KnnLds {
    double cx[kBucket], cy[kBucket], cz[kBucket];
    uint32_t cpos[kBucket];
    uint32_t hist[kKnnBins][kBucket];
    double surv[kKnnSurv][kBucket];
    double lv_lo[kKnnLevels][kBucket];
    double lv_inv[kKnnLevels][kBucket];
    int lv_beta[kKnnLevels][kBucket];
    int64_t stack[kStackMax];
};

__device__ inline double dist2_exact(double ax, double ay, double az, double bx, double by,
                                     double bz)
{
#pragma clang fp contract(off)
    const double dx = bx - ax, dy = by - ay, dz = bz - az;
    return (dx * dx + dy * dy) + dz * dz;
}

__device__ inline double box_dist2(const double* q, const double* __restrict__ b)
{
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double g = fmax(fmax(b[c] - q[3 + c], q[c] - b[3 + c]), 0.0);
        s += g * g;
    }
    return s;
}

__device__ inline double wave_max_d(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Depth-first visit of the buckets whose box passes `test`.  Wave-uniform:
// every lane calls f(bucket) for every bucket visited.
template <class Test, class F>
__device__ inline void tree_visit(const HaloDev& H, const NodeChild* __restrict__ nodes,
                                  int64_t n_buckets, int64_t* stack, Test test, F f)
{
    const int lane = threadIdx.x & 63;
    const int64_t root = H.level_off[H.n_levels - 1];
    if (H.n_levels == 1) {
        f(root);
        return;
    }
    __syncthreads();
    if (lane == 0) stack[0] = root;
    int sp = 1;
    __syncthreads();
    while (sp > 0) {
        const int64_t node = stack[sp - 1];
        --sp;
        const NodeChild N = nodes[node];
        const bool pass = lane < N.nchild && test(N.child0 + lane);
        unsigned long long mask = __ballot(pass);
        __syncthreads();
        if (N.child0 < n_buckets) {
            while (mask) {
                const int l = __ffsll((long long)mask) - 1;
                mask &= mask - 1ull;
                f(N.child0 + l);
            }
        } else {
            const int cnt = __popcll(mask);
            if (pass) {
                const int below = __popcll(mask & ((1ull << lane) - 1ull));
                stack[sp + cnt - 1 - below] = N.child0 + lane;
            }
            sp += cnt;
            __syncthreads();
        }
    }
}

__device__ inline int bin_of(double d2, double lo, double inv)
{
    int b = (int)((d2 - lo) * inv);
    b = b < 0 ? 0 : b;
    return b > kKnnBins - 1 ? kKnnBins - 1 : b;
}

__global__ __launch_bounds__(kBucket) void k_knn(
    const HaloDev* __restrict__ halos, const BucketInfo* __restrict__ buckets,
    const NodeChild* __restrict__ nodes, const double* __restrict__ box, int64_t n_buckets,
    const double* __restrict__ sx, const double* __restrict__ sy, const double* __restrict__ sz,
    const uint32_t* __restrict__ perm, double* __restrict__ sh, double* __restrict__ h_out,
    int* __restrict__ status)
{
    __shared__ KnnLds L;
    const int64_t b = blockIdx.x;
    const int lane = threadIdx.x;
    const BucketInfo B = buckets[b];
    const HaloDev& H = halos[B.halo];
    const int k = H.k;
    const bool act = lane < B.count;
    const uint32_t mypos = (uint32_t)(B.start + (act ? lane : 0));
    const double xi = sx[mypos], yi = sy[mypos], zi = sz[mypos];
    double qb[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) qb[c] = box[6 * b + c];

    auto stage = [&](int64_t c) -> int {
        const BucketInfo C = buckets[c];
        __syncthreads();
        if (lane < C.count) {
            const int64_t p = C.start + lane;
            L.cx[lane] = sx[p]; L.cy[lane] = sy[p]; L.cz[lane] = sz[p];
            L.cpos[lane] = (uint32_t)p;
        }
        __syncthreads();
        return C.count;
    };

    // ---- 1. bound from a window of buckets around b
    const int64_t hb0 = H.level_off[0], hb1 = H.level_off[0] + H.level_n[0] - 1;
    int64_t w0 = b - H.win_lo, w1 = b + H.win_hi;
    if (w0 < hb0) { w1 += hb0 - w0; w0 = hb0; }
    if (w1 > hb1) { w0 -= w1 - hb1; w1 = hb1; }
    if (w0 < hb0) w0 = hb0;
    double mx = 0.0;
    for (int64_t c = w0; c <= w1; ++c) {
        const int cnt = stage(c);
        for (int j = 0; j < cnt; ++j)
            if (L.cpos[j] != mypos) mx = fmax(mx, dist2_exact(xi, yi, zi, L.cx[j], L.cy[j], L.cz[j]));
    }
    for (int q = 0; q < kKnnBins; ++q) L.hist[q][lane] = 0;
    const double winv = mx > 0.0 ? (double)kKnnBins / mx : 0.0;
    for (int64_t c = w0; c <= w1; ++c) {
        const int cnt = stage(c);
        for (int j = 0; j < cnt; ++j)
            if (L.cpos[j] != mypos)
                ++L.hist[bin_of(dist2_exact(xi, yi, zi, L.cx[j], L.cy[j], L.cz[j]), 0.0, winv)][lane];
    }
    int wbeta = kKnnBins - 1;
    {
        int cum = 0;
        for (int q = 0; q < kKnnBins; ++q) {
            cum += L.hist[q][lane];
            if (cum >= k) { wbeta = q; break; }
        }
    }
    double u2 = 0.0;
    for (int64_t c = w0; c <= w1; ++c) {
        const int cnt = stage(c);
        for (int j = 0; j < cnt; ++j)
            if (L.cpos[j] != mypos) {
                const double d2 = dist2_exact(xi, yi, zi, L.cx[j], L.cy[j], L.cz[j]);
                if (bin_of(d2, 0.0, winv) <= wbeta) u2 = fmax(u2, d2);
            }
    }
    if (!act) u2 = 0.0;
    const double R2 = wave_max_d(u2) * (1.0 + 1e-9);
    auto near = [&](int64_t c) { return box_dist2(qb, box + 6 * c) <= R2; };

    // ---- 2./3. histogram refinement over the tree candidates
    bool done = !act;
    int level = 0, below = 0;
    double d2k = 0.0;
    L.lv_lo[0][lane] = 0.0;
    L.lv_inv[0][lane] = u2 > 0.0 ? (double)kKnnBins / u2 : 0.0;
    auto member = [&](double d2, int upto) {
        if (!(d2 <= u2)) return false;
        for (int l = 0; l < upto; ++l)
            if (bin_of(d2, L.lv_lo[l][lane], L.lv_inv[l][lane]) != L.lv_beta[l][lane]) return false;
        return true;
    };
    while (__ballot(!done)) {
        for (int q = 0; q < kKnnBins; ++q) L.hist[q][lane] = 0;
        const double lo_l = L.lv_lo[level][lane], inv_l = L.lv_inv[level][lane];
        tree_visit(H, nodes, n_buckets, L.stack, near, [&](int64_t c) {
            const int cnt = stage(c);
            if (done) return;
            for (int j = 0; j < cnt; ++j) {
                if (L.cpos[j] == mypos) continue;
                const double d2 = dist2_exact(xi, yi, zi, L.cx[j], L.cy[j], L.cz[j]);
                if (member(d2, level)) ++L.hist[bin_of(d2, lo_l, inv_l)][lane];
            }
        });
        int sel = -1, inb = 0, cum = below;
        if (!done) {
            for (int q = 0; q < kKnnBins; ++q) {
                const int hq = (int)L.hist[q][lane];
                if (cum + hq >= k) { sel = q; inb = hq; break; }
                cum += hq;
            }
            if (sel < 0) {  // cannot happen when the bound holds
                d2k = NAN;
                done = true;
                atomicOr(&status[B.halo], SIDM_DEV_KNN_OVERFLOW);
            } else {
                L.lv_beta[level][lane] = sel;
            }
        }
        double mn = INFINITY, mxv = -INFINITY;
        int ns = 0;
        tree_visit(H, nodes, n_buckets, L.stack, near, [&](int64_t c) {
            const int cnt = stage(c);
            if (done) return;
            for (int j = 0; j < cnt; ++j) {
                if (L.cpos[j] == mypos) continue;
                const double d2 = dist2_exact(xi, yi, zi, L.cx[j], L.cy[j], L.cz[j]);
                if (member(d2, level + 1)) {
                    mn = fmin(mn, d2);
                    mxv = fmax(mxv, d2);
                    if (inb <= kKnnSurv && ns < kKnnSurv) L.surv[ns++][lane] = d2;
                }
            }
        });
        if (!done) {
            if (inb <= kKnnSurv) {
                for (int a = 1; a < ns; ++a) {   // insertion sort of the bin's members
                    const double v = L.surv[a][lane];
                    int q = a - 1;
                    while (q >= 0 && L.surv[q][lane] > v) {
                        L.surv[q + 1][lane] = L.surv[q][lane];
                        --q;
                    }
                    L.surv[q + 1][lane] = v;
                }
                const int r = k - cum - 1;
                d2k = (r >= 0 && r < ns) ? L.surv[r][lane] : NAN;
                done = true;
            } else if (mn == mxv) {
                d2k = mn;           // all members tie at the k-th distance
                done = true;
            } else if (level + 1 >= kKnnLevels) {
                d2k = NAN;
                done = true;
                atomicOr(&status[B.halo], SIDM_DEV_KNN_OVERFLOW);
            } else {
                below = cum;
                ++level;
                L.lv_lo[level][lane] = mn;
                L.lv_inv[level][lane] = (double)kKnnBins / (mxv - mn);
            }
        }
    }
    if (act) {
        const double h = sqrt(d2k);
        sh[mypos] = h;
        h_out[perm[mypos]] = h;
    }
}

// Neighbour lists for verification: brute force over the halo, one thread per
// particle, the best k (d2, id) kept in order in a scratch row.
__global__ __launch_bounds__(kStreamBlock) void k_knn_list(
    const StreamBlock* __restrict__ blocks, const HaloDev* __restrict__ halos,
    const double* __restrict__ x, const double* __restrict__ y, const double* __restrict__ z,
    const uint32_t* __restrict__ id, int k_max, double* __restrict__ rowd2,
    uint32_t* __restrict__ nbr)
{
    const StreamBlock B = blocks[blockIdx.x];
    const int t = threadIdx.x;
    if (t >= B.count) return;
    const HaloDev& H = halos[B.halo];
    const int64_t i = B.start + t;
    const int k = H.k;
    double* rd = rowd2 + i * (int64_t)k_max;
    uint32_t* ri = nbr + i * (int64_t)k_max;
    const double xi = x[i], yi = y[i], zi = z[i];
    int cnt = 0;
    for (int64_t j = H.offset; j < H.offset + H.n; ++j) {
        if (j == i) continue;
        const double d2 = dist2_exact(xi, yi, zi, x[j], y[j], z[j]);
        const uint32_t idj = id[j];
        if (cnt == k && !(d2 < rd[k - 1] || (d2 == rd[k - 1] && idj < ri[k - 1]))) continue;
        int pos = cnt < k ? cnt : k - 1;
        while (pos > 0 && (d2 < rd[pos - 1] || (d2 == rd[pos - 1] && idj < ri[pos - 1]))) {
            rd[pos] = rd[pos - 1];
            ri[pos] = ri[pos - 1];
            --pos;
        }
        rd[pos] = d2;
        ri[pos] = idj;
        if (cnt < k) ++cnt;
    }
}

hipError_t launch_knn(const Plan& P, const sidm_state* s, Scratch& w, uint32_t* nbr, int k_max,
                      hipStream_t st)
{
    hipLaunchKernelGGL(k_knn, dim3((unsigned)P.n_buckets), dim3(kBucket), 0, st, w.halos,
                       w.buckets, w.nodes, w.box, P.n_buckets, w.sx, w.sy, w.sz, w.perm, w.sh,
                       s->h, w.status);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !nbr) return e;
    double* rowd2 = nullptr;
    int64_t total = 0;
    for (const auto& H : P.halos) total = std::max(total, H.offset + H.n);
    e = hipMallocAsync((void**)&rowd2, sizeof(double) * (size_t)(total * k_max), st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_knn_list, dim3((unsigned)P.n_blocks), dim3(kStreamBlock), 0, st, w.blocks,
                       w.halos, s->x, s->y, s->z, s->id, k_max, rowd2, nbr);
    e = hipGetLastError();
    hipError_t f = hipFreeAsync(rowd2, st);
    return e != hipSuccess ? e : f;
}

}  // namespace sidm
