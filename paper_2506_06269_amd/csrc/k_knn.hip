// k_knn.hip -- the SIDM kernel size h_i = distance to the k-th nearest other
// particle of the halo (Sec. 2: the kernel size is set by the next N_ngb
// neighbours).
//
// One wavefront per bucket of 64 Morton-consecutive particles, one particle
// per lane; the lanes of each compact sub-range of the bucket are resolved
// together.  Candidates are staged sub-range by sub-range in LDS and every
// lane reads the same candidate (broadcast), as in the gravity tiles.  A
// candidate sub-range is visited only if it intersects the search sphere of
// at least one lane.
// Selection works on values only, with a private 32-bin histogram per lane
// (an LDS column, no atomics):
//   1. each lane starts below an estimate from its 8th-nearest bucket-mate and
//      grows the radius by 1.5 until the sphere holds k (counts at four radii
//      in registers pick the smallest that does); a histogram of the
//      distances in [0, u_i^2] then names the bin of the k-th;
//   2. a visit restricted to that bin's shell collects its members (at most
//      16) or, if it holds more, refines the bin by its own min..max range
//      (again visiting only the shell); equal values end the refinement.
// Distances d2 = (dx*dx + dy*dy) + dz*dz are evaluated in FP64 without fused
// multiply-add, the same expression the oracle uses, so h matches bit for bit.
#include "sidm_tree.hpp"

namespace sidm {

constexpr int kKnnBins = 32;
constexpr int kKnnSurv = 16;
constexpr int kKnnLevels = 4;
constexpr int kKnnGrow = 80;

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

__device__ inline double box_diag2_k(const double* b)
{
    const double ex = b[3] - b[0], ey = b[4] - b[1], ez = b[5] - b[2];
    return ex * ex + ey * ey + ez * ez;
}

__device__ inline int bin_of(double d2, double lo, double inv)
{
    int b = (int)((d2 - lo) * inv);
    b = b < 0 ? 0 : b;
    return b > kKnnBins - 1 ? kKnnBins - 1 : b;
}

__global__ __launch_bounds__(kBucket) void k_knn(
    const HaloDev* __restrict__ halos, const BucketInfo* __restrict__ buckets,
    const NodeChild* __restrict__ nodes, const double* __restrict__ box,
    const SubRange* __restrict__ sub, const int* __restrict__ sub_n, int64_t n_buckets,
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
    const bool in_bucket = lane < B.count;
    const uint32_t mypos = (uint32_t)(B.start + (in_bucket ? lane : 0));
    const double xi = sx[mypos], yi = sy[mypos], zi = sz[mypos];
    auto all_nodes = [](int64_t) { return true; };

    // stage particles [p0, p0 + cnt) of the sorted order into LDS
    auto stage = [&](int64_t p0, int cnt) {
        __syncthreads();
        if (lane < cnt) {
            const int64_t p = p0 + lane;
            L.cx[lane] = sx[p]; L.cy[lane] = sy[p]; L.cz[lane] = sz[p];
            L.cpos[lane] = (uint32_t)p;
        }
        __syncthreads();
    };
    // visit every candidate sub-range within reach of a lane's sphere
    // (radius^2 r2 of the lane, ignored when `off` is true for the lane)
    auto visit = [&](double r2, bool off, auto body) {
        tree_visit(H, nodes, n_buckets, L.stack,
                   [&](int64_t c) { return !off && point_box_dist2(xi, yi, zi, box + 6 * c) <= r2; },
                   all_nodes, [&](int64_t c) {
                       const int64_t c0 = buckets[c].start;
                       const int ns = sub_n[c];
                       for (int q = 0; q < ns; ++q) {
                           const SubRange R = sub[kSubMax * c + q];
                           if (!__ballot(!off && point_box_dist2(xi, yi, zi, R.box) <= r2)) continue;
                           stage(c0 + R.off, R.cnt);
                           if (!off) body(R.cnt);
                       }
                   });
    };

    // the lanes of each compact sub-range of this bucket are resolved together
    const int ngroups = sub_n[b];
    for (int g = 0; g < ngroups; ++g) {
        const SubRange G = sub[kSubMax * b + g];
        const bool act = in_bucket && lane >= G.off && lane < G.off + G.cnt;

        // ---- 1. starting radius: distance to the m-th nearest member of the
        // lane's own sub-range (m <= 8), scaled to k neighbours, started low
        double u2;
        {
            constexpr int kM = 8;
            double best[kM];
#pragma unroll
            for (int q = 0; q < kM; ++q) best[q] = INFINITY;
            stage(B.start + G.off, G.cnt);
            for (int j = 0; j < G.cnt; ++j) {
                if (L.cpos[j] == mypos) continue;
                double v = dist2_exact(xi, yi, zi, L.cx[j], L.cy[j], L.cz[j]);
#pragma unroll
                for (int q = 0; q < kM; ++q) {   // insertion into the sorted best list
                    const double lo = fmin(best[q], v);
                    v = fmax(best[q], v);
                    best[q] = lo;
                }
            }
            const int m = min(min(kM, k), G.cnt - 1);
            double rm2 = 0.0;
#pragma unroll
            for (int q = 0; q < kM; ++q)
                if (q == m - 1) rm2 = best[q];
            if (m >= 1 && rm2 > 0.0 && rm2 < INFINITY) {
                // start below the estimate: a pass over a small sphere is
                // cheap, one over a sphere far too large is not
                u2 = 0.3 * 1.44 * rm2 * pow((double)k / (double)m, 2.0 / 3.0);
            } else {
                const double* rb = box + 6 * H.level_off[H.n_levels - 1];
                u2 = box_diag2_k(rb) / cbrt((double)H.n * (double)H.n);
            }
        }
        bool done = !act;      // this lane's h is known
        // grow the radius by 1.5 until the sphere holds k others; counts at four
        // radii inside the sphere (registers only) give the smallest that does
        bool found = !act;
        int grow = 0;
        while (__ballot(!found)) {
            int c0 = 0, c1 = 0, c2 = 0, c3 = 0;
            const double t0 = 0.55 * u2, t1 = 0.7 * u2, t2 = 0.85 * u2, t3 = u2;
            visit(u2 * (1.0 + 1e-9), found, [&](int cnt) {
                for (int j = 0; j < cnt; ++j) {
                    const double d2 = dist2_exact(xi, yi, zi, L.cx[j], L.cy[j], L.cz[j]);
                    const int self = L.cpos[j] == mypos;
                    c0 += (d2 <= t0) - self;
                    c1 += (d2 <= t1) - self;
                    c2 += (d2 <= t2) - self;
                    c3 += (d2 <= t3) - self;
                }
            });
            if (!found) {
                if (c3 >= k) {
                    found = true;
                    u2 = c0 >= k ? t0 : c1 >= k ? t1 : c2 >= k ? t2 : t3;
                } else if (++grow > kKnnGrow) {
                    found = done = true;
                    atomicOr(&status[B.halo], SIDM_DEV_KNN_OVERFLOW);
                } else if (u2 > 0.0) {
                    u2 *= 2.25;
                } else {
                    u2 = box_diag2_k(box + 6 * H.level_off[H.n_levels - 1]) /
                         cbrt((double)H.n * (double)H.n);
                    if (!(u2 > 0.0)) u2 = 1.0;
                }
            }
        }
        // ---- 2. level-0 histogram of the distances in [0, u2]
        const double inv0 = u2 > 0.0 ? (double)kKnnBins / u2 : 0.0;
        for (int q = 0; q < kKnnBins; ++q) L.hist[q][lane] = 0;
        L.lv_lo[0][lane] = 0.0;
        L.lv_inv[0][lane] = inv0;
        visit(u2 * (1.0 + 1e-9), done, [&](int cnt) {
            for (int j = 0; j < cnt; ++j) {
                if (L.cpos[j] == mypos) continue;
                const double d2 = dist2_exact(xi, yi, zi, L.cx[j], L.cy[j], L.cz[j]);
                if (d2 <= u2) atomicAdd(&L.hist[bin_of(d2, 0.0, inv0)][lane], 1u);
            }
        });
        __syncthreads();

        // ---- 3. select the bin of the k-th, collect or refine
        bool ready = true;
        int level = 0, below = 0;
        double d2k = NAN;
        auto member = [&](double d2, int upto) {
            if (!(d2 <= u2)) return false;
            for (int l = 0; l < upto; ++l)
                if (bin_of(d2, L.lv_lo[l][lane], L.lv_inv[l][lane]) != L.lv_beta[l][lane])
                    return false;
            return true;
        };
        double cull2 = u2 * (1.0 + 1e-9);   // members of the current bin lie within
        while (__ballot(!done)) {
            if (__ballot(!done && !ready)) {
                const double lo_l = L.lv_lo[level][lane], inv_l = L.lv_inv[level][lane];
                const bool skip = done || ready;
                if (!skip)
                    for (int q = 0; q < kKnnBins; ++q) L.hist[q][lane] = 0;
                visit(cull2, skip, [&](int cnt) {
                    for (int j = 0; j < cnt; ++j) {
                        if (L.cpos[j] == mypos) continue;
                        const double d2 = dist2_exact(xi, yi, zi, L.cx[j], L.cy[j], L.cz[j]);
                        if (member(d2, level))
                            atomicAdd(&L.hist[bin_of(d2, lo_l, inv_l)][lane], 1u);
                    }
                });
                ready = true;
                __syncthreads();
            }
            int sel = -1, inb = 0, cum = below;
            double shell2 = 0.0;   // members of the selected bin lie within this
            if (!done) {
                for (int q = 0; q < kKnnBins; ++q) {
                    const int hq = (int)L.hist[q][lane];
                    if (cum + hq >= k) { sel = q; inb = hq; break; }
                    cum += hq;
                }
                if (sel < 0) {   // cannot happen: the sphere holds at least k
                    done = true;
                    atomicOr(&status[B.halo], SIDM_DEV_KNN_OVERFLOW);
                } else {
                    L.lv_beta[level][lane] = sel;
                    const double inv_l = L.lv_inv[level][lane];
                    shell2 = inv_l > 0.0 ? L.lv_lo[level][lane] + (double)(sel + 1) / inv_l : u2;
                    shell2 = fmin(u2, shell2) * (1.0 + 1e-9);
                }
            }
            double mn = INFINITY, mxv = -INFINITY;
            int ns = 0;
            visit(shell2, done, [&](int cnt) {
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
                    if (r >= 0 && r < ns) d2k = L.surv[r][lane];
                    done = true;
                } else if (mn == mxv) {
                    d2k = mn;        // all members tie at the k-th distance
                    done = true;
                } else if (level + 1 >= kKnnLevels) {
                    done = true;
                    atomicOr(&status[B.halo], SIDM_DEV_KNN_OVERFLOW);
                } else {
                    below = cum;
                    ++level;
                    L.lv_lo[level][lane] = mn;
                    L.lv_inv[level][lane] = (double)kKnnBins / (mxv - mn);
                    ready = false;
                    cull2 = shell2;
                }
            }
        }
        if (act) {
            const double h = sqrt(d2k);
            sh[mypos] = h;
            h_out[perm[mypos]] = h;
        }
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
                       w.buckets, w.nodes, w.box, w.sub, w.sub_n, P.n_buckets, w.sx, w.sy, w.sz,
                       w.perm, w.sh, s->h, w.status);
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
