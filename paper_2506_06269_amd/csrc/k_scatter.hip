// k_scatter.hip -- SIDM scattering pass (Sec. 2: rare pairwise scatterings
// through the spline kernel, explicitly conserving energy and momentum;
// Sec. 3.5: the geometric factor Lambda of the interaction probability).
//
// k_pairs: one wavefront per bucket, one i per lane.  Candidate buckets come
// from the search tree: bucket c is visited when, for some lane i, the
// distance from x_i to c's box is below h_i + hmax(c).
// A bucket visits only candidate buckets of equal or higher index (pairs
// inside a bucket are owned by the smaller id), so each pair is tested once,
// when d2 < (h_i + h_j)^2; accepted pairs are compacted through an LDS queue
// (ballot + prefix count) so that the expensive per-pair work -- Philox4x32-10,
// |dv|, and Lambda when the draw falls below a cheap upper bound of P -- runs
// on full wavefronts.  A pair whose draw falls below the bound is appended to
// a candidate buffer; k_decide evaluates Lambda for those and appends the
// events (u < P) to the event buffer (when the candidate buffer is full, the
// pair pass decides the rest itself).
//
// k_rounds: the events of a step are applied in (a, b) order as elastic,
// isotropic kicks in the pair's centre-of-mass frame.  Events that share no
// particle commute, so the order is realised by rounds: in each round every
// particle elects the smallest pending event key it belongs to (atomicMin),
// and an event fires when it is the elected one for both of its particles.
// This is exactly the dependency order of one-after-the-other application.
#include "sidm_math.hpp"
#include "sidm_tree.hpp"

namespace sidm {

__device__ inline double dist2_pair(double ax, double ay, double az, double bx, double by,
                                    double bz)
{
#pragma clang fp contract(off)
    const double dx = bx - ax, dy = by - ay, dz = bz - az;
    return (dx * dx + dy * dy) + dz * dz;
}

__device__ inline double norm3(double x, double y, double z)
{
#pragma clang fp contract(off)
    return sqrt((x * x + y * y) + z * z);
}

__global__ void k_scatter_reset(DevCounters* __restrict__ counters,
                                unsigned long long* __restrict__ ev_counts, int* __restrict__ status,
                                int n_halos)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0) {
        counters->n_events_total = 0ull;
        counters->n_cands = 0ull;
        counters->ticket = 0ull;
    }
    if (t < kEvCounts * n_halos) ev_counts[t] = 0ull;
    if (t < n_halos) status[t] = 0;
}

// ---------------------------------------------------------------- contract checks
// Ids key the random draws and order the kicks, so they must be unique per
// halo.  Every particle inserts its key (halo << 32 | id) into an open-
// addressing hash table of cap >= 2 n slots (linear probing, the empty slot
// ~0, which no key equals: halo indices stay below 2^31); finding its own key
// already there flags the halo.  A table at most half full always has an
// empty slot, so every probe sequence ends.
constexpr unsigned long long kEmptySlot = ~0ull;

__global__ __launch_bounds__(256) void k_fill_u64(unsigned long long* __restrict__ a, int64_t n,
                                                   unsigned long long v)
{
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n; p += (int64_t)gridDim.x * 256)
        a[p] = v;
}

__device__ inline unsigned long long mix64(unsigned long long z)
{
    // the finaliser of SplitMix64 (Steele, Lea and Flood 2014)
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(kStreamBlock) void k_id_insert(
    const StreamBlock* __restrict__ blocks, const uint32_t* __restrict__ id,
    unsigned long long* __restrict__ table, unsigned long long cap, int* __restrict__ status)
{
    const StreamBlock B = blocks[blockIdx.x];
    const int t = threadIdx.x;
    if (t >= B.count) return;
    const unsigned long long key = ((unsigned long long)(uint32_t)B.halo << 32) | id[B.start + t];
    unsigned long long slot = __umul64hi(mix64(key), cap);
    for (unsigned long long probe = 0; probe < cap; ++probe) {
        const unsigned long long prev = atomicCAS(&table[slot], kEmptySlot, key);
        if (prev == kEmptySlot) return;
        if (prev == key) {
            atomicOr(&status[B.halo], SIDM_DEV_DUPLICATE_ID);
            return;
        }
        slot = slot + 1 == cap ? 0 : slot + 1;
    }
}

// OR of the halos' status words into the context's sticky word, which keeps
// them until the host has read it.
__global__ __launch_bounds__(256) void k_publish_status(const int* __restrict__ status,
                                                         int n_halos, int* __restrict__ sticky)
{
    for (int h = threadIdx.x; h < n_halos; h += 256) {
        const int v = status[h];
        if (v) atomicOr(sticky, v);
    }
}

// The fingerprint (halos, state pointers, scratch generation) of the last call
// made outside stream capture.
__global__ void k_set_fingerprint(unsigned long long* __restrict__ fp_dev,
                                  unsigned long long fp)
{
    if (threadIdx.x == 0) *fp_dev = fp;
}

// First kernel of a captured call: a replay after a call outside capture
// changed the fingerprint is flagged in every halo and in the sticky word.
__global__ __launch_bounds__(256) void k_guard(const unsigned long long* __restrict__ fp_dev,
                                               unsigned long long fp, int* __restrict__ status,
                                               int n_halos, int* __restrict__ sticky)
{
    if (*fp_dev == fp) return;
    for (int h = threadIdx.x; h < n_halos; h += 256) atomicOr(&status[h], SIDM_DEV_STALE_GRAPH);
    if (threadIdx.x == 0) atomicOr(sticky, SIDM_DEV_STALE_GRAPH);
}

// The events of the last scattering pass as sidm_event records (nothing when
// they overflowed the context's buffer; at most cap).
__global__ __launch_bounds__(256) void k_copy_events(const DevCounters* __restrict__ counters,
                                                     const EventRec* __restrict__ ev,
                                                     int64_t max_events, int64_t cap,
                                                     sidm_event* __restrict__ out)
{
    const int64_t total = (int64_t)counters->n_events_total;
    if (total > max_events) return;
    const int64_t n = total < cap ? total : cap;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * 256) {
        sidm_event o;
        o.a = (uint32_t)(ev[e].key >> 32);
        o.b = (uint32_t)ev[e].key;
        o.halo = ev[e].halo;
        o.round = ev[e].round;
        out[e] = o;
    }
}

// The exact decision of a candidate: P = (sigma/m) m_b g Lambda dt with the
// overlap integral, an event iff u < P (and a count of P > 1).  One function
// for both callers, so that a decision never depends on which kernel took it.
__device__ __forceinline__ void decide_pair(const CandRec& r, double dt,
                                         DevCounters* __restrict__ counters,
                                         EventRec* __restrict__ events, int64_t max_events,
                                         unsigned long long* __restrict__ ev_counts)
{
    const double lam = kernel_overlap(r.d, r.ha, r.hb);
    const double P = r.sg * r.mb * r.g * lam * dt;
    if (P > 1.0) atomicAdd(&ev_counts[kEvCounts * r.halo + 3], 1ull);
    if (r.u < P) {
        const unsigned long long slot = atomicAdd(&counters->n_events_total, 1ull);
        if ((int64_t)slot < max_events) {
            EventRec e;
            e.key = ((unsigned long long)r.a << 32) | r.b;
            e.ia = r.ia;
            e.ib = r.ib;
            e.halo = r.halo;
            e.round = 0u;
            events[slot] = e;
        }
    }
}

// LDS copies of the bucket's own particles (I: what the per-pair work reads)
// and of the candidate range (J: also the positions of the pair test).  The
// rest (positions of I, original indices) is read from memory for the rare
// candidates, and the mass is the halo's common one.
struct PairI {
    double vx[kBucket], vy[kBucket], vz[kBucket], h[kBucket];
    uint32_t id[kBucket];
};
struct PairJ {
    double x[kBucket], y[kBucket], z[kBucket], h[kBucket];
    double vx[kBucket], vy[kBucket], vz[kBucket];
    uint32_t id[kBucket];
};

// Cross-section per unit mass at relative speed g: sigma_m, or with a velocity
// scale w > 0 the form of Sec. 3.8 (Eq. vel_dep), sigma_m [1 + (g/w)^2]^-2.
__device__ inline double sigma_at(const HaloDev& H, double g)
{
#pragma clang fp contract(off)
    if (!(H.sigma_w > 0.0)) return H.sigma_m;
    const double t = g / H.sigma_w;
    const double q = 1.0 + t * t;
    return H.sigma_m / (q * q);
}

// INLINE: the pass after an overflow of the candidate buffer.  It runs only
// then (it returns at once otherwise), repeats the search and decides every
// candidate itself; k_decide then decides none, and the counts of pairs and
// candidates are those of the first pass.
template <bool INLINE>
__global__ __launch_bounds__(kBucket) void k_pairs(
    const HaloDev* __restrict__ halos, const BucketInfo* __restrict__ buckets,
    const NodeChild* __restrict__ nodes, const double* __restrict__ box,
    const double* __restrict__ hmax, const SubRange* __restrict__ sub,
    const int* __restrict__ sub_n, const double* __restrict__ cbox,
    const double* __restrict__ chmax, int64_t n_buckets,
    const double* __restrict__ sx,
    const double* __restrict__ sy, const double* __restrict__ sz, const double* __restrict__ svx,
    const double* __restrict__ svy, const double* __restrict__ svz, const double* __restrict__ sh,
    const double* __restrict__ cmass, const uint32_t* __restrict__ sid,
    const uint32_t* __restrict__ perm, uint32_t step, DevCounters* __restrict__ counters,
    CandRec* __restrict__ cands, int64_t max_cands, EventRec* __restrict__ events,
    int64_t max_events, unsigned long long* __restrict__ ev_counts, const int* __restrict__ status,
    int split)
{
    __shared__ PairI I;
    __shared__ PairJ J;
    __shared__ uint16_t queue[2 * kBucket];
    __shared__ int64_t stack[kStackMax];
    // split waves per bucket: wave `part` takes every split-th candidate
    // bucket of the bucket's visit (a call with few buckets still fills the
    // device; every pair is still tested by exactly one wave)
    const int64_t b = blockIdx.x / split;
    const int part = (int)(blockIdx.x % split);
    const int lane = threadIdx.x;
    if (INLINE && (int64_t)counters->n_cands <= max_cands) return;
    const BucketInfo B = buckets[b];
    const HaloDev& H = halos[B.halo];
    if (!(H.sigma_m > 0.0)) return;   // uniform over the block
    // a halo with unequal masses or repeated ids is not scattered (flagged)
    if (status[B.halo] & (SIDM_DEV_UNEQUAL_MASS | SIDM_DEV_DUPLICATE_ID)) return;
    const bool act = lane < B.count;
    const double mb = cmass[B.halo];   // the masses of a halo that scatters are equal
    int64_t jbase = 0;                  // first sorted position of the range in J
    if (act) {
        const int64_t p = B.start + lane;
        I.vx[lane] = svx[p]; I.vy[lane] = svy[p]; I.vz[lane] = svz[p];
        I.h[lane] = sh[p];
        I.id[lane] = sid[p];
    }
    const uint32_t k0 = (uint32_t)(H.seed & 0xffffffffull), k1 = (uint32_t)(H.seed >> 32);
    const double kInvPi8 = 8.0 / 3.14159265358979323846;
    const double cbound = H.sigma_m * mb * kInvPi8 * H.dt;
    const double cbound2 = cbound * cbound * (1.0 + 1e-12);
    const bool sw = H.sigma_w > 0.0;
    const double inv_w2 = sw ? 1.0 / (H.sigma_w * H.sigma_w) : 0.0;
    const unsigned long long lt = (1ull << lane) - 1ull;
    long long my_cands = 0;
    unsigned long long wave_pairs = 0;   // wave-uniform: the ballots' counts
    int qn = 0;

    // per-pair work for queue entries [0, cnt): lane l takes entry l
    auto process = [&](int cnt) {
        __syncthreads();
        if (lane < cnt) {
            const int e = queue[lane];
            const int il = e & 63, jl = e >> 8;
            // canonical order of the pair: a = smaller id, b = larger id
            const bool iswap = I.id[il] > J.id[jl];
            const uint32_t a = iswap ? J.id[jl] : I.id[il], bb = iswap ? I.id[il] : J.id[jl];
            const Philox4 w = philox4x32_10(a, bb, step, 0u, k0, k1);
            const double u = unit53(w.w[0], w.w[1]);
            const double dvx = I.vx[il] - J.vx[jl], dvy = I.vy[il] - J.vy[jl],
                         dvz = I.vz[il] - J.vz[jl];
            const double g2 = (dvx * dvx + dvy * dvy) + dvz * dvz;
            const double ha = I.h[il], hbb = J.h[jl];
            const double hm = fmax(ha, hbb);

            // Lambda <= min(W_a(0), W_b(0)) = 8 / (pi max(h)^3) bounds P by
            // sigma(g) m g 8 / (pi max(h)^3) dt.  The test u < bound, with
            // sigma(g) = sigma_m / q^2, reads u max(h)^3 q^2 < cbound g;
            // both sides are non-negative, so it is taken squared (no square
            // root, no division), with a relative slack of 1e-12 so that the
            // candidates include every pair whose rounded P exceeds u.
            double lhs = u * (hm * hm * hm);
            if (sw) {
                const double q = 1.0 + g2 * inv_w2;
                lhs *= q * q;
            }
            if (lhs * lhs < cbound2 * g2) {
                // the exact decision needs Lambda: k_decide takes it from here
                // (after an overflow of its buffer, the INLINE pass)
                ++my_cands;
                const double g = norm3(dvx, dvy, dvz);
                CandRec r;
                r.sg = sigma_at(H, g);
                r.mb = mb;
                r.g = g;
                const int64_t pi = B.start + il;
                r.d = sqrt(dist2_pair(sx[pi], sy[pi], sz[pi], J.x[jl], J.y[jl], J.z[jl]));
                r.ha = iswap ? hbb : ha;
                r.hb = iswap ? ha : hbb;
                r.u = u;
                r.a = a;
                r.b = bb;
                const uint32_t oi = perm[pi], oj = perm[jbase + jl];
                r.ia = iswap ? oj : oi;
                r.ib = iswap ? oi : oj;
                r.halo = B.halo;
                r.pad = 0;
                if (INLINE) {
                    decide_pair(r, H.dt, counters, events, max_events, ev_counts);
                } else {
                    const unsigned long long slot = atomicAdd(&counters->n_cands, 1ull);
                    if ((int64_t)slot < max_cands) cands[slot] = r;
                }
            }
        }
        __syncthreads();
    };

    // bucket c can hold a partner of lane i only if its box is closer than
    // h_i + max h over c; pairs between two buckets are handled by the lower
    // bucket index, pairs inside a bucket by the smaller id
    const double hi_l = act ? I.h[lane] : 0.0;
    const int64_t pl = B.start + (act ? lane : 0);
    const double xl = sx[pl], yl = sy[pl], zl = sz[pl];
    int visit_no = 0;   // candidate buckets visited so far (wave-uniform)
    tree_visit(H, nodes, n_buckets, stack,
               [&](int64_t c) {
                   const double r = hi_l + hmax[c];
                   return act && point_box_dist2(xl, yl, zl, box + 6 * c) < r * r * (1.0 + 1e-9);
               },
               [&](int64_t c) { return nodes[c].last >= b; },
               [&](int64_t c) {
        if (split > 1 && (visit_no++ % split) != part) return;
        const BucketInfo C = buckets[c];
        const double hc = hmax[c];
        const int nsub = sub_n[c];
        for (int q = 0; q < nsub; ++q) {
            const SubRange R = sub[kSubMax * c + q];
            const double rr = hi_l + hc;
            if (!__ballot(act && point_box_dist2(xl, yl, zl, R.box) < rr * rr * (1.0 + 1e-9)))
                continue;
            __syncthreads();
            jbase = C.start + R.off;
            if (lane < R.cnt) {
                const int64_t p = jbase + lane;
                J.x[lane] = sx[p]; J.y[lane] = sy[p]; J.z[lane] = sz[p];
                J.h[lane] = sh[p];
                J.vx[lane] = svx[p]; J.vy[lane] = svy[p]; J.vz[lane] = svz[p];
                J.id[lane] = sid[p];
            }
            __syncthreads();
            const double xi = xl, yi = yl, zi = zl, hi = hi_l;
            const uint32_t idi = I.id[act ? lane : 0];
            const bool same = c == b;
            // a long sub-range is tested by chunks, those within reach of
            // some lane
            const bool chunked = R.cnt > kChunk;
            for (int jj = 0; jj < R.cnt;) {
            const int g = (R.off + jj) / kChunk;
            const int je = chunked ? min(R.cnt, (g + 1) * kChunk - R.off) : R.cnt;
            const double rc = hi_l + chmax[kChunks * c + g];   // the chunk's own largest h
            if (chunked &&
                !__ballot(act && point_box_dist2(xl, yl, zl, cbox + 6 * (kChunks * c + g)) <
                                     rc * rc * (1.0 + 1e-9))) {
                jj = je;
                continue;
            }
            for (; jj < je; ++jj) {
                // every lane evaluates the test, without a branch per
                // candidate (a lane past the bucket's end tests lane 0's copy)
                const double d2 = dist2_pair(xi, yi, zi, J.x[jj], J.y[jj], J.z[jj]);
                const double hs = hi + J.h[jj];
                const bool ord = !same || idi < J.id[jj];
                const bool pair = act & ord & (d2 < hs * hs);
                const unsigned long long mask = __ballot(pair);
                if (pair) queue[qn + __popcll(mask & lt)] = (uint16_t)(lane | (jj << 8));
                qn += __popcll(mask);
                wave_pairs += (unsigned long long)__popcll(mask);
                if (qn >= kBucket) {
                    process(kBucket);
                    const int rest = qn - kBucket;
                    const uint16_t moved = lane < rest ? queue[kBucket + lane] : 0;
                    __syncthreads();
                    if (lane < rest) queue[lane] = moved;
                    qn = rest;
                    __syncthreads();
                }
            }
            }
            if (qn > 0) {
                process(qn);   // entries refer to this candidate range: flush now
                qn = 0;
            }
        }
    });
    // pairs tested and candidates of the exact decision found by this bucket
    if (INLINE) return;
    long long vc = my_cands;
    for (int o = 32; o > 0; o >>= 1) vc += __shfl_xor(vc, o, 64);
    if (lane == 0 && wave_pairs > 0) atomicAdd(&ev_counts[kEvCounts * B.halo + 2], wave_pairs);
    if (lane == 0 && vc > 0) atomicAdd(&ev_counts[kEvCounts * B.halo + 4], (unsigned long long)vc);
}

// The exact decisions of the candidates the pair pass stored; none after an
// overflow of their buffer (the INLINE pair pass decides them all).
__global__ __launch_bounds__(256) void k_decide(const HaloDev* __restrict__ halos,
                                                const CandRec* __restrict__ cands,
                                                int64_t max_cands,
                                                DevCounters* __restrict__ counters,
                                                EventRec* __restrict__ events, int64_t max_events,
                                                unsigned long long* __restrict__ ev_counts)
{
    const int64_t total = (int64_t)counters->n_cands;
    if (total > max_cands) return;
    for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < total;
         c += (int64_t)gridDim.x * 256) {
        const CandRec r = cands[c];
        decide_pair(r, halos[r.halo].dt, counters, events, max_events, ev_counts);
    }
}

// Elastic isotropic scattering in the centre-of-mass frame: the relative speed
// is kept and its direction redrawn uniformly on the sphere from the draw at
// counter (a, b, step, 1).
__device__ inline void kick_pair(uint64_t seed, uint32_t step, uint32_t a, uint32_t b, double ma,
                                 double mb, double* va, double* vb)
{
#pragma clang fp contract(off)
    const Philox4 w = philox4x32_10(a, b, step, 1u, (uint32_t)(seed & 0xffffffffull),
                                    (uint32_t)(seed >> 32));
    const double uc = unit53(w.w[0], w.w[1]);
    const double uphi = unit53(w.w[2], w.w[3]);
    const double M = ma + mb;
    const double dvx = va[0] - vb[0], dvy = va[1] - vb[1], dvz = va[2] - vb[2];
    const double g = sqrt((dvx * dvx + dvy * dvy) + dvz * dvz);
    const double cth = 1.0 - 2.0 * uc;
    const double s2 = 1.0 - cth * cth;
    const double sth = sqrt(s2 > 0.0 ? s2 : 0.0);
    const double ph = 2.0 * 3.14159265358979323846 * uphi;
    double sp, cp;
    sincos(ph, &sp, &cp);
    const double n[3] = {sth * cp, sth * sp, cth};
    const double fa = mb / M * g, fb = ma / M * g;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double vcm = (ma * va[c] + mb * vb[c]) / M;
        va[c] = vcm + fa * n[c];
        vb[c] = vcm - fb * n[c];
    }
}

__device__ inline unsigned long long owner_load(unsigned long long* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline void owner_free(unsigned long long* p)
{
    __hip_atomic_store(p, ~0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

constexpr int kRoundThreads = 1024;
// Halos are independent: workgroup g of kRoundGroups takes the events of the
// halos h with h % groups == g, listed (as event indices) in its own segment
// of max_events words of the candidate buffer, which holds nothing once the
// pair decisions are taken.
constexpr int kRoundGroups = 64;
static_assert(4 * sizeof(CandRec) >= kRoundGroups * sizeof(uint32_t),
              "the candidate buffer holds every workgroup's event list");

// Each workgroup applies the events of its halos; all of its waves leave the
// loop in the same round (the pending count is reduced through LDS).
__global__ __launch_bounds__(kRoundThreads) void k_rounds(
    const HaloDev* __restrict__ halos, int n_halos, const DevCounters* __restrict__ counters,
    EventRec* __restrict__ ev, int64_t max_events, unsigned long long* __restrict__ owner,
    double* __restrict__ vx, double* __restrict__ vy, double* __restrict__ vz,
    const double* __restrict__ m, unsigned long long* __restrict__ ev_counts,
    int* __restrict__ status, uint32_t step, int64_t out_cap, sidm_event* __restrict__ out,
    uint32_t* __restrict__ lists)
{
    __shared__ int pending, n_mine;
    const int t = threadIdx.x;
    const int groups = (int)gridDim.x, g = (int)blockIdx.x;
    const unsigned long long total = counters->n_events_total;
    if ((int64_t)total > max_events) {
        for (int h = g + groups * t; h < n_halos; h += groups * kRoundThreads)
            atomicOr(&status[h], SIDM_DEV_EVENT_OVERFLOW);
        return;
    }
    const int64_t n_all = (int64_t)total;
    uint32_t* __restrict__ mine_e = lists + (int64_t)g * max_events;
    if (t == 0) n_mine = 0;
    __syncthreads();
    for (int64_t e = t; e < n_all; e += kRoundThreads)
        if (ev[e].halo % groups == g) mine_e[atomicAdd(&n_mine, 1)] = (uint32_t)e;
    __syncthreads();
    const int64_t n = n_mine;
    for (int64_t q = t; q < n; q += kRoundThreads) {
        const int64_t e = mine_e[q];
        ev[e].round = 0u;
        owner_free(&owner[ev[e].ia]);
        owner_free(&owner[ev[e].ib]);
    }
    __syncthreads();
    for (uint32_t r = 1; n > 0; ++r) {
        for (int64_t q = t; q < n; q += kRoundThreads) {
            const int64_t e = mine_e[q];
            if (ev[e].round == 0u) {
                atomicMin(&owner[ev[e].ia], ev[e].key);
                atomicMin(&owner[ev[e].ib], ev[e].key);
            }
        }
        __syncthreads();
        for (int64_t q = t; q < n; q += kRoundThreads) {
            const int64_t e = mine_e[q];
            if (ev[e].round == 0u) {
                const unsigned long long key = ev[e].key;
                if (owner_load(&owner[ev[e].ia]) == key && owner_load(&owner[ev[e].ib]) == key)
                    ev[e].round = r;
            }
        }
        __syncthreads();
        if (t == 0) pending = 0;
        for (int64_t q = t; q < n; q += kRoundThreads) {
            const int64_t e = mine_e[q];
            const uint32_t er = ev[e].round;
            if (er == 0u || er == r) {
                owner_free(&owner[ev[e].ia]);
                owner_free(&owner[ev[e].ib]);
            }
        }
        __syncthreads();
        int mine = 0;
        for (int64_t q = t; q < n; q += kRoundThreads) {
            const int64_t e = mine_e[q];
            const EventRec E = ev[e];
            if (E.round == r) {
                const HaloDev& H = halos[E.halo];
                double va[3] = {vx[E.ia], vy[E.ia], vz[E.ia]};
                double vb[3] = {vx[E.ib], vy[E.ib], vz[E.ib]};
                kick_pair(H.seed, step, (uint32_t)(E.key >> 32), (uint32_t)E.key, m[E.ia], m[E.ib],
                          va, vb);
                vx[E.ia] = va[0]; vy[E.ia] = va[1]; vz[E.ia] = va[2];
                vx[E.ib] = vb[0]; vy[E.ib] = vb[1]; vz[E.ib] = vb[2];
                atomicAdd(&ev_counts[kEvCounts * E.halo + 0], 1ull);
                atomicMax(&ev_counts[kEvCounts * E.halo + 1], (unsigned long long)r);
            } else if (E.round == 0u) {
                ++mine;
            }
        }
        if (mine) atomicAdd(&pending, mine);
        __syncthreads();
        const int left = pending;
        __syncthreads();
        if (left == 0) break;
    }
    if (out) {
        for (int64_t q = t; q < n; q += kRoundThreads) {
            const int64_t e = mine_e[q];
            if (e >= out_cap) continue;
            sidm_event o;
            o.a = (uint32_t)(ev[e].key >> 32);
            o.b = (uint32_t)ev[e].key;
            o.halo = ev[e].halo;
            o.round = ev[e].round;
            out[e] = o;
        }
    }
}

hipError_t launch_reset(const Plan& P, Scratch& w, hipStream_t st)
{
    const int nt = kEvCounts * P.n_halos + 1;
    hipLaunchKernelGGL(k_scatter_reset, dim3((nt + 255) / 256), dim3(256), 0, st, w.counters,
                       (unsigned long long*)w.ev_counts, w.status, P.n_halos);
    return hipGetLastError();
}

int launch_sort_keys(Scratch& w, int64_t n, int key_bits, hipStream_t st);
hipError_t launch_mass_check(const Plan& P, Scratch& w, const double* m, hipStream_t st);

// The scattering pass's checks of its contract: a common mass in every halo
// that scatters, and ids unique within each halo (the id check reuses the
// cell list's sort buffers, which hold nothing the later passes read).
hipError_t launch_contract_checks(const Plan& P, const sidm_state* s, Scratch& w, hipStream_t st)
{
    if (!P.any_scatter) return hipSuccess;
    hipError_t e = launch_mass_check(P, w, s->m, st);
    if (e != hipSuccess) return e;
    // the hash table: the radix sort's two key buffers, 2 max_particles words
    const unsigned long long cap = 2ull * (unsigned long long)w.max_particles;
    if ((int64_t)cap < 2 * P.n_sorted) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_fill_u64, dim3(1024), dim3(256), 0, st, w.keys[0], (int64_t)cap,
                       kEmptySlot);
    hipLaunchKernelGGL(k_id_insert, dim3((unsigned)P.n_blocks), dim3(kStreamBlock), 0, st,
                       w.blocks, s->id, w.keys[0], cap, w.status);
    return hipGetLastError();
}

hipError_t launch_publish_status(const Plan& P, Scratch& w, hipStream_t st)
{
    hipLaunchKernelGGL(k_publish_status, dim3(1), dim3(256), 0, st, w.status, P.n_halos, w.sticky);
    return hipGetLastError();
}

hipError_t launch_fingerprint(const Plan& P, Scratch& w, unsigned long long fp, bool captured,
                              hipStream_t st)
{
    if (captured)
        hipLaunchKernelGGL(k_guard, dim3(1), dim3(256), 0, st, w.fp_dev, fp, w.status, P.n_halos,
                           w.sticky);
    else
        hipLaunchKernelGGL(k_set_fingerprint, dim3(1), dim3(64), 0, st, w.fp_dev, fp);
    return hipGetLastError();
}

__global__ void k_clear_word(int* __restrict__ w)
{
    if (threadIdx.x == 0) *w = 0;
}

hipError_t launch_clear_sticky(Scratch& w, hipStream_t st)
{
    hipLaunchKernelGGL(k_clear_word, dim3(1), dim3(64), 0, st, w.sticky);
    return hipGetLastError();
}

hipError_t launch_copy_events(Scratch& w, sidm_event* out, int64_t cap, hipStream_t st)
{
    hipLaunchKernelGGL(k_copy_events, dim3(64), dim3(256), 0, st, w.counters, w.events,
                       w.max_events, cap, out);
    return hipGetLastError();
}

hipError_t launch_scatter(const Plan& P, const sidm_state* s, Scratch& w, uint32_t step,
                          sidm_event* out_events, int64_t out_cap, hipStream_t st,
                          hipEvent_t after_pairs)
{
    hipError_t e = launch_contract_checks(P, s, w, st);
    if (e != hipSuccess) return e;
    const int split = search_split(P.n_buckets, kPairSplitMax);
    auto pairs = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3((unsigned)(P.n_buckets * split)), dim3(kBucket), 0, st, w.halos,
                           w.buckets, w.nodes, w.box, w.hmax, w.sub, w.sub_n, w.cbox, w.chmax, P.n_buckets, w.sx,
                           w.sy, w.sz, w.svx, w.svy, w.svz, w.sh, w.cref, w.sid, w.perm, step,
                           w.counters, w.cands, w.max_cands, w.events, w.max_events,
                           (unsigned long long*)w.ev_counts, w.status, split);
    };
    pairs(k_pairs<false>);
    hipLaunchKernelGGL(k_decide, dim3(256), dim3(256), 0, st, w.halos, w.cands, w.max_cands,
                       w.counters, w.events, w.max_events, (unsigned long long*)w.ev_counts);
    pairs(k_pairs<true>);
    if (after_pairs) (void)hipEventRecord(after_pairs, st);
    const int groups = P.n_halos < kRoundGroups ? P.n_halos : kRoundGroups;
    hipLaunchKernelGGL(k_rounds, dim3((unsigned)groups), dim3(kRoundThreads), 0, st, w.halos,
                       P.n_halos, w.counters, w.events, w.max_events, w.owner, s->vx, s->vy,
                       s->vz, s->m, (unsigned long long*)w.ev_counts, w.status, step, out_cap,
                       out_events, (uint32_t*)w.cands);
    return hipGetLastError();
}

}  // namespace sidm
