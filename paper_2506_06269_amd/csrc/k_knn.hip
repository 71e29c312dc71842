// k_knn.hip -- the SIDM kernel size h_i = distance to the k-th nearest other
// particle of the halo (Sec. 2: the kernel size is set by the next N_ngb
// neighbours).
//
// One wavefront per bucket of 64 Morton-consecutive particles, one particle
// per lane, all lanes resolved together (each with its own search sphere).
// Candidates are read with wave-uniform loads (every lane evaluates the same
// candidate), and a candidate sub-range is visited only if
// it intersects the search sphere of at least one lane.
// Selection works on values only.  When the particle's kernel size before
// the call is a usable value h0 (a warm start: the result does not depend on
// it), one visit of the sphere of radius (1 + d) h0 counts the candidates
// closer than (1 - d) h0 and keeps the distances in between (the band: its
// kKnnBand smallest values, in an LDS column of the lane); if the k-th
// distance lies in the band and among the kept values, it is read off them.
// In a step h changes by a few tenths of a per cent (a few per cent at the
// tail), so almost every lane ends here.  The other lanes, and lanes without
// a usable h0, take the general search, with a private 32-bin histogram per
// lane (an LDS column, written with LDS atomics that return nothing):
//   1. a histogram of the distances within a starting radius: 1.15 times h0
//      when it is usable; otherwise the first member of the particle's
//      compact sub-range is resolved first, from an estimate out of the
//      nearest members of that sub-range, and the particle starts from 1.15
//      times that member's h; the radius grows until the sphere holds k
//      others;
//   2. a visit restricted to the shell of the bin that holds the k-th
//      collects that bin's members (at most 16, kept sorted in registers) or,
//      if it holds more, records their min..max, whose histogram (step 1 over
//      that range) refines the choice; equal values end the refinement.
// Typical cost: one visit of the candidates around the bucket when warm; two
// visits for the general search, restricted to the sub-ranges that its
// lanes' spheres reach.
// Distances d2 = (dx*dx + dy*dy) + dz*dz are evaluated in FP64 without fused
// multiply-add, the same expression the oracle uses, so h matches bit for bit.
#include "sidm_tree.hpp"

namespace sidm {

constexpr int kKnnBins = 32;
constexpr int kKnnSurv = 16;
constexpr int kKnnLevels = 4;
constexpr int kKnnGrow = 80;
constexpr double kKnnWarm = 1.15 * 1.15;   // squared margin on the previous kernel size
constexpr int kKnnBand = 16;               // band distances kept per lane
constexpr int kKnnSplitMax = 16;           // waves per bucket for calls with few buckets

// The band pass and the general search never run at once: the band's values
// live in the histogram columns, value q of a lane in words 2q (low half) and
// 2q + 1 (high half) of its column (a barrier separates the two uses).
static_assert(2 * kKnnBand <= kKnnBins, "band values fit the histogram columns");
struct KnnLds {
    uint32_t hist[kKnnBins][kBucket];
    int64_t stack[kStackMax];
};

__device__ inline double band_get(const KnnLds& L, int q, int lane)
{
    const uint64_t lo = L.hist[2 * q][lane], hi = L.hist[2 * q + 1][lane];
    return __longlong_as_double((long long)((hi << 32) | lo));
}

__device__ inline void band_put(KnnLds& L, int q, int lane, double v)
{
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    L.hist[2 * q][lane] = (uint32_t)u;
    L.hist[2 * q + 1][lane] = (uint32_t)(u >> 32);
}

__device__ inline double dist2_exact(double ax, double ay, double az, double bx, double by,
                                     double bz)
{
#pragma clang fp contract(off)
    const double dx = bx - ax, dy = by - ay, dz = bz - az;
    return (dx * dx + dy * dy) + dz * dz;
}

__device__ inline double box_diag2_k(const double* b)
{
    const double ex = b[3] - b[0], ey = b[4] - b[1], ez = b[5] - b[2];
    return ex * ex + ey * ey + ez * ez;
}

// Bin of d2 among kKnnBins equal bins starting at lo (monotone in d2; NaN
// products, from an infinite inv, fall in bin 0).
__device__ inline int bin_of(double d2, double lo, double inv)
{
    const double t = (d2 - lo) * inv;
    return t >= (double)(kKnnBins - 1) ? kKnnBins - 1 : (t > 0.0 ? (int)t : 0);
}

// Insertion of v into the ascending list best[0..M) (registers).
template <int M>
__device__ inline void insert_sorted(double (&best)[M], double v)
{
#pragma unroll
    for (int q = 0; q < M; ++q) {
        const double lo = fmin(best[q], v);
        v = fmax(best[q], v);
        best[q] = lo;
    }
}

template <bool LIST>
__global__ __launch_bounds__(kBucket) void k_knn(
    const HaloDev* __restrict__ halos, const BucketInfo* __restrict__ buckets,
    const NodeChild* __restrict__ nodes, const double* __restrict__ box,
    const SubRange* __restrict__ sub, const int* __restrict__ sub_n,
    const double* __restrict__ cbox, int64_t n_buckets,
    const double4* __restrict__ sp4, const uint32_t* __restrict__ perm,
    double* __restrict__ sh, double* __restrict__ h_out, int* __restrict__ status,
    const uint32_t* __restrict__ sid, uint32_t* __restrict__ nbr, int k_max, int split)
{
    __shared__ KnnLds L;
    // split waves per bucket: wave `part` resolves the bucket's lanes
    // [part, part + 1) * 64 / split (a call with few buckets still fills the
    // device, and each wave's candidates are those of its own lanes' spheres)
    const int64_t bw = xcd_contiguous(blockIdx.x, gridDim.x);
    const int64_t b = bw / split;
    const int part = (int)(bw % split);
    const int lane = threadIdx.x;
    const BucketInfo B = buckets[b];
    const HaloDev& H = halos[B.halo];
    const int k = H.k;
    const bool in_bucket = lane < B.count && lane / (kBucket / split) == part;
    const int64_t mypos = B.start + (in_bucket ? lane : 0);
    const double4 me = sp4[mypos];
    const double xi = me.x, yi = me.y, zi = me.z;
    const double hint = sh[mypos];   // the kernel size before the call
    const double diag2 = box_diag2_k(box + 6 * H.level_off[H.n_levels - 1]);
    auto all_nodes = [](int64_t) { return true; };

    // every candidate of the sub-ranges within reach of a lane's sphere
    // (radius^2 r2 of the lane, ignored when `off` is true for the lane);
    // body(p, c) runs on every lane for candidate p at c = (x, y, z, .)
    auto visit = [&](double r2, bool off, auto body) __attribute__((always_inline)) {
        tree_visit(H, nodes, n_buckets, L.stack,
                   [&](int64_t c) { return !off && point_box_dist2(xi, yi, zi, box + 6 * c) <= r2; },
                   all_nodes, [&](int64_t c) {
                       const int64_t c0 = buckets[c].start;
                       const int ns = sub_n[c];
                       for (int q = 0; q < ns; ++q) {
                           const SubRange& R = sub[kSubMax * c + q];
                           if (!__ballot(!off && point_box_dist2(xi, yi, zi, R.box) <= r2)) continue;
                           // a long sub-range is taken by chunks, those that
                           // some sphere reaches
                           const int j1 = R.off + R.cnt;
                           const bool chunked = R.cnt > kChunk;
                           for (int a0 = R.off; a0 < j1;) {
                               const int g = a0 / kChunk;
                               const int a1 = chunked ? min(j1, (g + 1) * kChunk) : j1;
                               const bool reach =
                                   !chunked ||
                                   __ballot(!off && point_box_dist2(xi, yi, zi,
                                                                    cbox + 6 * (kChunks * c + g)) <= r2);
                               // candidates [a0, a1), four loads in flight
                               // before the first use
                               int j = reach ? a0 : a1;
                               for (; j + 4 <= a1; j += 4) {
                                   double4 v[4];
#pragma unroll
                                   for (int u = 0; u < 4; ++u) v[u] = sp4[c0 + j + u];
#pragma unroll
                                   for (int u = 0; u < 4; ++u) body(c0 + j + u, v[u]);
                               }
                               for (; j < a1; ++j) body(c0 + j, sp4[c0 + j]);
                               a0 = a1;
                           }
                       }
                   });
    };
    // histogram of the distances in [a, z] over kKnnBins bins from lo
    auto histogram = [&](bool on, double a, double z, double lo, double inv)
        __attribute__((always_inline)) {
        if (on)
            for (int q = 0; q < kKnnBins; ++q) L.hist[q][lane] = 0u;
        visit(z * (1.0 + 1e-9), !on, [&](int64_t p, const double4& c) {
            const double d2 = dist2_exact(xi, yi, zi, c.x, c.y, c.z);
            if (on && p != mypos && d2 >= a && d2 <= z)
                atomicAdd(&L.hist[bin_of(d2, lo, inv)][lane], 1u);
        });
        __syncthreads();
    };

    // h^2 of the lanes with act set, from a starting radius^2 u2 (NaN for the
    // others); a uniform call: every lane of the wave takes part
    auto resolve = [&](bool act, double u2) __attribute__((always_inline)) {
        // ---- 1. histogram of [0, u2]; grow until the sphere holds k others
        bool need = act, failed = false;
        int grow = 0;
        while (__ballot(need)) {
            histogram(need, 0.0, u2, 0.0, (double)kKnnBins / u2);
            if (need) {
                int tot = 0;
                for (int q = 0; q < kKnnBins; ++q) tot += (int)L.hist[q][lane];
                if (tot >= k) {
                    need = false;
                } else if (++grow > kKnnGrow) {
                    need = false;
                    failed = true;
                    atomicOr(&status[B.halo], SIDM_DEV_KNN_OVERFLOW);
                } else {
                    double f = tot > 0 ? 1.44 * pow((double)k / (double)tot, 2.0 / 3.0) : 4.0;
                    u2 *= fmin(fmax(f, 1.44), 4.0);
                }
            }
        }

        // ---- 2. select the bin of the k-th, collect its members or refine.
        // Members of the current set lie in [a, z]; its histogram uses bins
        // (lo, inv); `below` counts the candidates under the selected bin.
        bool done = !act || failed;
        double a = 0.0, z = u2, lo = 0.0, inv = (double)kKnnBins / u2;
        int below = 0, level = 0;
        double d2k = NAN;
        while (__ballot(!done)) {
            int sel = -1, inb = 0;
            double shell2 = 0.0;
            if (!done) {
                int cum = below;
                for (int q = 0; q < kKnnBins; ++q) {
                    const int hq = (int)L.hist[q][lane];
                    if (cum + hq >= k) { sel = q; inb = hq; break; }
                    cum += hq;
                }
                if (sel < 0) {   // cannot happen: the set holds the k-th
                    done = true;
                    atomicOr(&status[B.halo], SIDM_DEV_KNN_OVERFLOW);
                } else {
                    below = cum;
                    shell2 = inv > 0.0 && isfinite(inv) ? fmin(z, lo + (double)(sel + 1) / inv) : z;
                }
            }
            double best[kKnnSurv];
#pragma unroll
            for (int q = 0; q < kKnnSurv; ++q) best[q] = INFINITY;
            double mn = INFINITY, mxv = -INFINITY;
            const bool collect = !done && inb <= kKnnSurv;
            visit(shell2 * (1.0 + 1e-9), done, [&](int64_t p, const double4& c) {
                const double d2 = dist2_exact(xi, yi, zi, c.x, c.y, c.z);
                if (!done && p != mypos && d2 >= a && d2 <= z && bin_of(d2, lo, inv) == sel) {
                    mn = fmin(mn, d2);
                    mxv = fmax(mxv, d2);
                    if (collect) insert_sorted(best, d2);
                }
            });
            bool refine = false;
            if (!done) {
                if (collect) {
                    const int r = k - below - 1;
#pragma unroll
                    for (int q = 0; q < kKnnSurv; ++q)
                        if (q == r) d2k = best[q];
                    done = true;
                } else if (mn == mxv) {
                    d2k = mn;        // all members tie at the k-th distance
                    done = true;
                } else if (++level >= kKnnLevels) {
                    done = true;
                    atomicOr(&status[B.halo], SIDM_DEV_KNN_OVERFLOW);
                } else {
                    a = mn;
                    z = mxv;
                    lo = mn;
                    inv = (double)kKnnBins / (mxv - mn);
                    refine = true;
                }
            }
            if (__ballot(refine)) histogram(refine, a, z, lo, inv);
        }
        return act ? d2k : NAN;
    };

    // h^2 of the lanes with act set from one visit of the band around their
    // previous kernel size h0 (NaN for lanes whose k-th distance is not
    // among the kept band values); a uniform call
    auto band_pass = [&](bool act, double h0) __attribute__((always_inline)) {
        // half-width relative to h0: about 12 band members expected (a
        // spherical shell of relative width 2d holds about 6 d k
        // neighbours), at least 1 %, at most 6 %
        const double d = fmin(fmax(2.0 / (double)k, 0.01), 0.06);
        const double rlo = h0 * (1.0 - d), rhi = h0 * (1.0 + d);
        const double blo = rlo * rlo, bhi = rhi * rhi;
        // below the band; kept band values (the band's smallest when it holds
        // more than kKnnBand); the slot of the largest kept value when full
        int nlo = 0, kept = 0, imax = 0;
        auto find_max = [&]() {
            imax = 0;
            for (int q = 1; q < kKnnBand; ++q)
                if (band_get(L, q, lane) > band_get(L, imax, lane)) imax = q;
        };
        visit(bhi * (1.0 + 1e-9), !act, [&](int64_t p, const double4& c) {
            const double d2 = dist2_exact(xi, yi, zi, c.x, c.y, c.z);
            if (!act || p == mypos || d2 > bhi) return;
            if (d2 < blo) {
                ++nlo;
            } else if (kept < kKnnBand) {
                band_put(L, kept, lane, d2);
                if (++kept == kKnnBand) find_max();
            } else if (d2 < band_get(L, imax, lane)) {
                band_put(L, imax, lane, d2);
                find_max();
            }
        });
        // the k-th distance has rank r (0-based) in the band; it is a kept
        // value iff 0 <= r < kept
        const int r = k - nlo - 1;
        if (!act || r < 0 || r >= kept) kept = 0;
        double d2k = NAN;
        for (int q = 0; q < kept; ++q) {   // the kept value with r below it and r + 1 up to it
            const double v = band_get(L, q, lane);
            int less = 0, upto = 0;
            for (int t = 0; t < kept; ++t) {
                const double w = band_get(L, t, lane);
                less += w < v;
                upto += w <= v;
            }
            if (less <= r && r < upto) d2k = v;
        }
        __syncthreads();   // the band columns are read before the histograms reuse them
        return d2k;
    };

    // ---- starting radius
    const bool warm = isfinite(hint) && hint > 0.0 && hint * hint <= diag2;
    double u2 = kKnnWarm * hint * hint;
    if (__ballot(in_bucket && !warm)) {
        // the lane's own compact sub-range (members of another sub-range of
        // the bucket can be far away)
        int go = 0, gc = B.count;
        for (int g = 0; g < sub_n[b]; ++g) {
            const SubRange R = sub[kSubMax * b + g];
            if (lane >= R.off && lane < R.off + R.cnt) {
                go = R.off;
                gc = R.cnt;
            }
        }
        // an estimate: the m-th nearest member of that sub-range (m <= 8),
        // scaled to k neighbours
        constexpr int kM = 8;
        double best[kM];
#pragma unroll
        for (int q = 0; q < kM; ++q) best[q] = INFINITY;
        const int64_t p0 = B.start;
        for (int j = 0; j < B.count; ++j) {
            const double4 c = sp4[p0 + j];
            if (p0 + j == mypos || j < go || j >= go + gc) continue;
            double v = dist2_exact(xi, yi, zi, c.x, c.y, c.z);
#pragma unroll
            for (int q = 0; q < kM; ++q) {
                const double lo = fmin(best[q], v);
                v = fmax(best[q], v);
                best[q] = lo;
            }
        }
        const int m = min(min(kM, k), gc - 1);
        double rm2 = 0.0;
#pragma unroll
        for (int q = 0; q < kM; ++q)
            if (q == m - 1) rm2 = best[q];
        // With fewer than four members to go by (a sub-range cut off by a
        // jump of the Morton curve) an estimate can exceed the true radius
        // many times, and in the dense centre such a sphere holds a large
        // part of the halo (one wave then streams most of it); those
        // representatives start instead from the halo's diagonal / N, far
        // below any neighbour distance, and grow.
        double e2 = (m >= 4 && rm2 > 0.0 && rm2 < INFINITY)
                        ? 1.44 * rm2 * pow((double)k / (double)m, 2.0 / 3.0)
                        : diag2 / ((double)H.n * (double)H.n);
        if (!(e2 > 0.0)) e2 = 1.0;
        // The first member of each sub-range is resolved from the estimate
        // alone; every other member then starts as if warm, from 1.15 times
        // that representative's h (the kernel size varies slowly across a
        // compact sub-range).  The estimate errs by a factor of a few in
        // volume, and taken by all 64 lanes it cost four times the warm
        // candidate stream; taken by the few representatives it costs one
        // such stream.
        const bool rep = in_bucket && lane == go;
        const double d2r = resolve(rep, warm ? u2 : 0.25 * e2);
        const double c2 = kKnnWarm * __shfl(d2r, go);
        if (!warm) u2 = (isfinite(c2) && c2 > 0.0) ? fmin(c2, e2) : e2;
    }
    double d2k = NAN;
    bool todo = in_bucket;
    if (__ballot(in_bucket && warm)) {
        d2k = band_pass(in_bucket && warm, hint);
        todo = in_bucket && !(d2k >= 0.0);
    }
    const double d2g = resolve(todo, u2);
    if (todo) d2k = d2g;
    if (in_bucket) {
        const double h = sqrt(d2k);
        sh[mypos] = h;
        h_out[perm[mypos]] = h;
    }
    if (!LIST) return;

    // Neighbour lists: the members of the sphere of the k-th distance, as
    // sorted positions in the particle's row (k_knn_list_order puts them in
    // (d2, id) order and turns them into ids): first every candidate strictly
    // closer than the k-th (fewer than k), then the candidates at exactly that
    // distance, keeping the smallest ids when they are more than the rest.
    uint32_t* row = nbr + (int64_t)(in_bucket ? perm[mypos] : 0) * k_max;
    const bool on = in_bucket && isfinite(d2k);
    int cnt = 0;
    visit(d2k * (1.0 + 1e-9), !on, [&](int64_t p, const double4& c) {
        const double d2 = dist2_exact(xi, yi, zi, c.x, c.y, c.z);
        if (on && p != mypos && d2 < d2k && cnt < k) row[cnt++] = (uint32_t)p;
    });
    const int need = k - cnt;
    int nt = 0;
    visit(d2k * (1.0 + 1e-9), !on, [&](int64_t p, const double4& c) {
        const double d2 = dist2_exact(xi, yi, zi, c.x, c.y, c.z);
        if (!(on && p != mypos && d2 == d2k && need > 0)) return;
        if (nt < need) {
            row[cnt + nt++] = (uint32_t)p;
            return;
        }
        int worst = 0;
        uint32_t wid = 0;
        for (int q = 0; q < need; ++q) {
            const uint32_t iq = sid[row[cnt + q]];
            if (iq >= wid) {
                wid = iq;
                worst = q;
            }
        }
        if (sid[p] < wid) row[cnt + worst] = (uint32_t)p;
    });
}

// The rows k_knn collected, in (d2, id) order, as ids: one thread per
// particle, the distances recomputed with the same expression.
__global__ __launch_bounds__(kStreamBlock) void k_knn_list_order(
    const StreamBlock* __restrict__ blocks, const HaloDev* __restrict__ halos,
    const double* __restrict__ x, const double* __restrict__ y, const double* __restrict__ z,
    const double4* __restrict__ sp4, const uint32_t* __restrict__ sid, int k_max,
    uint32_t* __restrict__ nbr)
{
    const StreamBlock B = blocks[blockIdx.x];
    const int t = threadIdx.x;
    if (t >= B.count) return;
    const HaloDev& H = halos[B.halo];
    const int64_t i = B.start + t;
    const int k = H.k;
    uint32_t* row = nbr + i * (int64_t)k_max;
    const double xi = x[i], yi = y[i], zi = z[i];
    double d[SIDM_MAX_K];
    uint32_t id[SIDM_MAX_K];
    for (int q = 0; q < k; ++q) {
        const uint32_t p = row[q];
        const double4 c = sp4[p];
        const double d2 = dist2_exact(xi, yi, zi, c.x, c.y, c.z);
        const uint32_t iq = sid[p];
        int pos = q;
        while (pos > 0 && (d2 < d[pos - 1] || (d2 == d[pos - 1] && iq < id[pos - 1]))) {
            d[pos] = d[pos - 1];
            id[pos] = id[pos - 1];
            --pos;
        }
        d[pos] = d2;
        id[pos] = iq;
    }
    for (int q = 0; q < k; ++q) row[q] = id[q];
}

hipError_t launch_knn(const Plan& P, const sidm_state* s, Scratch& w, uint32_t* nbr, int k_max,
                      hipStream_t st)
{
    const int split = search_split(P.n_buckets, kKnnSplitMax);
    const dim3 grid((unsigned)(P.n_buckets * split));
    if (!nbr) {
        hipLaunchKernelGGL(k_knn<false>, grid, dim3(kBucket), 0, st,
                           w.halos, w.buckets, w.nodes, w.box, w.sub, w.sub_n, w.cbox, P.n_buckets,
                           w.sp4, w.perm, w.sh, s->h, w.status, w.sid, nbr, k_max, split);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_knn<true>, grid, dim3(kBucket), 0, st, w.halos,
                       w.buckets, w.nodes, w.box, w.sub, w.sub_n, w.cbox, P.n_buckets, w.sp4, w.perm,
                       w.sh, s->h, w.status, w.sid, nbr, k_max, split);
    hipLaunchKernelGGL(k_knn_list_order, dim3((unsigned)P.n_blocks), dim3(kStreamBlock), 0,
                           st, w.blocks, w.halos, s->x, s->y, s->z, w.sp4, w.sid, k_max, nbr);
    return hipGetLastError();
}

}  // namespace sidm
