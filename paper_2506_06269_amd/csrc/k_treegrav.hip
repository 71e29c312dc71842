// k_treegrav.hip -- tree gravity (Sec. 2: a gravity tree opened with the
// relative criterion alpha of Springel 2005, eq. 18; Table 1 runs use
// alpha = 5e-4).
//
// The tree is the cell list's: the Morton-sorted particles of a halo cut into
// buckets of kBucket, every kFanout consecutive nodes merged into a parent up
// to one root, each node with its particles' bounding box.  This pass adds the
// mass and first moments of every node (bucket sums in particle order, then
// child sums in child order, no fused multiply-adds, so the centres of mass
// are reproducible to the bit), and the second moments about each node's
// centre of mass (a bucket's from its particles, a node's from its children
// by parallel axes).
//
// A group is a bucket: waves of 64 lanes, one member per lane, walk the tree
// for all members, one wave per part of the walk (the parts share out the
// subtrees below a frontier level; see kTreeSplit).  A node is accepted when
// its box and the group's box are disjoint and (G M l^2)^2 <= alpha^2
// |a_old|^2 r^8, with l the node box's largest side, |a_old| the smallest
// previous acceleration of the members and r the distance between the two
// boxes: the paper's criterion
// G M l^2 <= alpha |a_old| r^4, squared (no square root in the decision) and
// made to hold for every member and every particle of the node.  An accepted
// node contributes its monopole and quadrupole (the second-order term of the
// softened potential about its centre of mass, from its second moments); an
// opened bucket contributes its particles.  Sources are staged in two LDS
// lists, particles and accepted nodes (the children of a popped node are
// tested by lanes 0..7 at once, accepted ones appended by a ballot prefix);
// full lists are summed by all lanes, each for its own member, with the self
// pair skipped in the group's own bucket, and the list sums are folded into
// compensated accumulators.  The result is one partial row per particle and
// part, summed in part order by the gravity finalize pass (G, host, kicks).
//
// FP64 form: positions and arithmetic in FP64.  Mixed form: the list holds
// FP64 positions; each pair's separation is taken in FP64 and rounded to FP32,
// the rest of the pair term is FP32, and the list sums are folded into FP32
// Kahan accumulators.  (FP32 positions relative to the group's centre lose
// close pairs in a sparse group: a bucket can span several length units, and
// the rounding of both positions then reaches 1e-5 of the force.)  The
// decisions are FP64 in both forms, so both sum the same terms.
#include "sidm_plan.hpp"
#include "sidm_steps.hpp"

namespace sidm {

// A walk round pops up to kTreePop pending nodes and tests their children
// (at most kTreePop * kFanout), so the accepted-node list holds one round's
// acceptances; the particle list one opened bucket.  These sizes keep a
// group's LDS at 9.6 KB, 16 groups per compute unit (as many as the
// registers allow): 128 and 64 entries with eight pops per round took
// 308.8 against 281.2 ms at N = 2^24.
constexpr int kTreePop = 4;
constexpr int kTreeList = 64;                     // source list entries per group
constexpr int kTreeNodes = kTreePop * kFanout;    // accepted-node list entries per group
static_assert(kTreeList >= kBucket, "an opened bucket must fit the particle list");
static_assert(kTreePop <= kFanout, "the stack bound below assumes kTreePop <= kFanout");

// An accepted node: centre of mass, mass and second moments about the centre
// (xx, yy, zz, xy, xz, yz).  The mixed sums take the mass, three times the
// moments and their trace in FP32, rounded once when the node is listed
// rather than per term (a third of the entry's bytes, and about 15 of 53
// vector instructions per node term).
struct NodeEntry {
    double x, y, z, m;
    double S[6];
};
struct NodeEntryF {
    double x, y, z;
    float m, S3[6], T;   // S3 = 3 S
};
template <bool MIXED>
struct NodeOf {
    using type = NodeEntry;
};
template <>
struct NodeOf<true> {
    using type = NodeEntryF;
};

__device__ inline void set_node(NodeEntry& e, double x, double y, double z, double m,
                                const double* __restrict__ S)
{
    e.x = x; e.y = y; e.z = z; e.m = m;
    for (int k = 0; k < 6; ++k) e.S[k] = S[k];
}
__device__ inline void set_node(NodeEntryF& e, double x, double y, double z, double m,
                                const double* __restrict__ S)
{
    e.x = x; e.y = y; e.z = z; e.m = (float)m;
    for (int k = 0; k < 6; ++k) e.S3[k] = (float)(3.0 * S[k]);
    e.T = (float)(S[0] + S[1] + S[2]);
}
// Popping up to kTreePop <= kFanout nodes per round and pushing at most
// kFanout children of each, the stack holds at most kFanout^2 - kFanout nodes
// per level plus one round's pushes (624 for ten levels).
constexpr int kTreeStack = (kFanout * kFanout - kFanout) * kMaxLevels + kFanout * kFanout;

// ---------------------------------------------------------------- moments
__global__ __launch_bounds__(256) void k_tree_mom_bucket(
    const BucketInfo* __restrict__ buckets, int64_t nb, const double* __restrict__ sx,
    const double* __restrict__ sy, const double* __restrict__ sz, const double* __restrict__ sm,
    double4* __restrict__ mom, double* __restrict__ mom2)
{
#pragma clang fp contract(off)
    const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (b >= nb) return;
    const BucketInfo B = buckets[b];
    double M = 0.0, X = 0.0, Y = 0.0, Z = 0.0;
    for (int q = 0; q < B.count; ++q) {
        const int64_t p = B.start + q;
        const double m = sm[p];
        M += m;
        X += m * sx[p];
        Y += m * sy[p];
        Z += m * sz[p];
    }
    mom[b] = make_double4(M, X, Y, Z);
    double S[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (M != 0.0) {
        const double cx = X / M, cy = Y / M, cz = Z / M;
        for (int q = 0; q < B.count; ++q) {
            const int64_t p = B.start + q;
            const double m = sm[p];
            const double u = sx[p] - cx, v = sy[p] - cy, w = sz[p] - cz;
            S[0] += m * u * u;
            S[1] += m * v * v;
            S[2] += m * w * w;
            S[3] += m * u * v;
            S[4] += m * u * w;
            S[5] += m * v * w;
        }
    }
    for (int k = 0; k < 6; ++k) mom2[6 * b + k] = S[k];
}

__global__ __launch_bounds__(256) void k_tree_mom_node(const NodeTask* __restrict__ tasks,
                                                       int64_t nt, double4* __restrict__ mom,
                                                       double* __restrict__ mom2)
{
#pragma clang fp contract(off)
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= nt) return;
    const NodeTask T = tasks[t];
    double M = 0.0, X = 0.0, Y = 0.0, Z = 0.0;
    for (int c = 0; c < T.nchild; ++c) {
        const double4 q = mom[T.child0 + c];
        M += q.x;
        X += q.y;
        Y += q.z;
        Z += q.w;
    }
    mom[T.node] = make_double4(M, X, Y, Z);
    double S[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (M != 0.0) {
        const double cx = X / M, cy = Y / M, cz = Z / M;
        for (int c = 0; c < T.nchild; ++c) {
            const int64_t ch = T.child0 + c;
            const double4 q = mom[ch];
            if (q.x == 0.0) continue;
            const double u = q.y / q.x - cx, v = q.z / q.x - cy, w = q.w / q.x - cz;
            const double* Sc = mom2 + 6 * ch;
            S[0] += Sc[0] + q.x * u * u;
            S[1] += Sc[1] + q.x * v * v;
            S[2] += Sc[2] + q.x * w * w;
            S[3] += Sc[3] + q.x * u * v;
            S[4] += Sc[4] + q.x * u * w;
            S[5] += Sc[5] + q.x * v * w;
        }
    }
    for (int k = 0; k < 6; ++k) mom2[6 * T.node + k] = S[k];
}

// Zeroes the per-halo count of source terms.
__global__ void k_tree_terms_reset(unsigned long long* __restrict__ terms, int n)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) terms[t] = 0ull;
}

// ---------------------------------------------------------------- criterion
// Whether node c is accepted for a group with box gb (see the file header).
__device__ inline bool tree_accept(const double* __restrict__ cb, double M, const double* gb,
                                   double G, double alpha2, double a2min)
{
#pragma clang fp contract(off)
    bool disjoint = false;
    double d[3];
    for (int k = 0; k < 3; ++k) {
        if (cb[k] > gb[3 + k] || cb[3 + k] < gb[k]) disjoint = true;
        const double lo = gb[k] - cb[3 + k], hi = cb[k] - gb[3 + k];
        d[k] = fmax(fmax(lo, hi), 0.0);
    }
    if (!disjoint) return false;
    if (M == 0.0) return true;
    const double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
    const double l = fmax(fmax(cb[3] - cb[0], cb[4] - cb[1]), cb[5] - cb[2]);
    const double q = ((G * M) * l) * l;
    const double lhs = q * q;
    const double r4 = r2 * r2;
    const double rhs = ((alpha2 * a2min) * r4) * r4;
    return lhs <= rhs;
}

__device__ inline double wave_min(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

// ---------------------------------------------------------------- list sums
// A list entry: position and mass.  The mixed sums take the mass in FP32,
// so there it is rounded once here and kept in the low half of w, read back
// by reinterpretation (no conversion per term).
template <bool MIXED>
__device__ inline double4 make_entry(double x, double y, double z, double m)
{
    if (MIXED)
        return make_double4(x, y, z, __longlong_as_double((long long)__float_as_uint((float)m)));
    return make_double4(x, y, z, m);
}

__device__ inline float entry_mass_f32(const double4& q)
{
    return __uint_as_float((uint32_t)__double_as_longlong(q.w));
}

// The list lengths and the self range are the same on every lane; taken into
// scalar registers, the sum loops count in scalar instructions (1.3 % of the
// walk at N = 2^24).
__device__ inline void uniform_bounds(int& len, int& self_lo, int& self_n)
{
    len = __builtin_amdgcn_readfirstlane(len);
    self_lo = __builtin_amdgcn_readfirstlane(self_lo);
    self_n = __builtin_amdgcn_readfirstlane(self_n);
}

template <bool MIXED>
struct TreeAcc;

template <>
struct TreeAcc<false> {
    using Entry = double4;
    double xi, yi, zi, eps2;
    double sx = 0, sy = 0, sz = 0, sp = 0, cx = 0, cy = 0, cz = 0, cp = 0;

    template <bool DIAG>
    __device__ inline void run(const Entry* L, int a, int b, int self, double* p)
    {
        for (int jj = a; jj < b; ++jj) {
            const double4 q = L[jj];
            const double dx = q.x - xi, dy = q.y - yi, dz = q.z - zi;
            const double r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, eps2)));
            double rinv = rsqrt_pos(r2);
            if (DIAG && jj == self) rinv = 0.0;
            const double mr = q.w * rinv;
            const double mr3 = mr * (rinv * rinv);
            p[0] = fma(mr3, dx, p[0]);
            p[1] = fma(mr3, dy, p[1]);
            p[2] = fma(mr3, dz, p[2]);
            p[3] += mr;
        }
    }
    __device__ inline void sum(const Entry* L, int len, int self_lo, int self_n, int lane)
    {
        uniform_bounds(len, self_lo, self_n);
        double p[4] = {0.0, 0.0, 0.0, 0.0};
        if (self_lo < 0) {
            run<false>(L, 0, len, -1, p);
        } else {
            run<false>(L, 0, self_lo, -1, p);
            run<true>(L, self_lo, self_lo + self_n, self_lo + lane, p);
            run<false>(L, self_lo + self_n, len, -1, p);
        }
        double y, t;
        y = p[0] - cx; t = sx + y; cx = (t - sx) - y; sx = t;
        y = p[1] - cy; t = sy + y; cy = (t - sy) - y; sy = t;
        y = p[2] - cz; t = sz + y; cz = (t - sz) - y; sz = t;
        y = p[3] - cp; t = sp + y; cp = (t - sp) - y; sp = t;
    }
    // Accepted nodes: monopole plus quadrupole.  With d from the node's centre
    // of mass to the member, rho^2 = |d|^2 + eps^2, S the second moments and T
    // their trace, the second-order term of -G sum m / sqrt(|d - s|^2 + eps^2)
    // is phi_Q = -G (3 d.S.d - rho^2 T) / (2 rho^5); a_Q = -grad phi_Q.
    __device__ inline void sum_nodes(const NodeEntry* L, int len)
    {
        len = __builtin_amdgcn_readfirstlane(len);
        double p[4] = {0.0, 0.0, 0.0, 0.0};
        for (int jj = 0; jj < len; ++jj) {
            const NodeEntry& q = L[jj];
            const double dx = q.x - xi, dy = q.y - yi, dz = q.z - zi;
            const double r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, eps2)));
            const double rinv = rsqrt_pos(r2);
            const double mr = q.m * rinv;
            const double ri2 = rinv * rinv;
            const double mr3 = mr * ri2;
            const double ri5 = rinv * ri2 * ri2, ri7 = ri5 * ri2;
            const double d0 = -dx, d1 = -dy, d2 = -dz;
            const double Sd0 = fma(q.S[0], d0, fma(q.S[3], d1, q.S[4] * d2));
            const double Sd1 = fma(q.S[3], d0, fma(q.S[1], d1, q.S[5] * d2));
            const double Sd2 = fma(q.S[4], d0, fma(q.S[5], d1, q.S[2] * d2));
            const double T = q.S[0] + q.S[1] + q.S[2];
            const double br = 3.0 * fma(d0, Sd0, fma(d1, Sd1, d2 * Sd2)) - r2 * T;
            const double c5 = 2.5 * br * ri7;
            p[0] += fma(mr3, dx, (3.0 * Sd0 - T * d0) * ri5 - c5 * d0);
            p[1] += fma(mr3, dy, (3.0 * Sd1 - T * d1) * ri5 - c5 * d1);
            p[2] += fma(mr3, dz, (3.0 * Sd2 - T * d2) * ri5 - c5 * d2);
            p[3] += mr + 0.5 * br * ri5;
        }
        double y, t;
        y = p[0] - cx; t = sx + y; cx = (t - sx) - y; sx = t;
        y = p[1] - cy; t = sy + y; cy = (t - sy) - y; sy = t;
        y = p[2] - cz; t = sz + y; cz = (t - sz) - y; sz = t;
        y = p[3] - cp; t = sp + y; cp = (t - sp) - y; sp = t;
    }
    __device__ inline double4 result() const
    {
        return make_double4(sx - cx, sy - cy, sz - cz, sp - cp);
    }
};

template <>
struct TreeAcc<true> {
    using Entry = double4;
    double xi, yi, zi;
    float eps2;
    float sx = 0, sy = 0, sz = 0, sp = 0, cx = 0, cy = 0, cz = 0, cp = 0;

    template <bool DIAG>
    __device__ inline void run(const Entry* L, int a, int b, int self, float* p)
    {
#pragma unroll 4
        for (int jj = a; jj < b; ++jj) {
            const double4 q = L[jj];
            const float dx = (float)(q.x - xi), dy = (float)(q.y - yi), dz = (float)(q.z - zi);
            const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2)));
            float rinv = __builtin_amdgcn_rsqf(r2);
            if (DIAG && jj == self) rinv = 0.f;
            const float mr = entry_mass_f32(q) * rinv;
            const float mr3 = mr * (rinv * rinv);
            p[0] = fmaf(mr3, dx, p[0]);
            p[1] = fmaf(mr3, dy, p[1]);
            p[2] = fmaf(mr3, dz, p[2]);
            p[3] += mr;
        }
    }
    __device__ inline void sum(const Entry* L, int len, int self_lo, int self_n, int lane)
    {
        uniform_bounds(len, self_lo, self_n);
        float p[4] = {0.f, 0.f, 0.f, 0.f};
        if (self_lo < 0) {
            run<false>(L, 0, len, -1, p);
        } else {
            run<false>(L, 0, self_lo, -1, p);
            run<true>(L, self_lo, self_lo + self_n, self_lo + lane, p);
            run<false>(L, self_lo + self_n, len, -1, p);
        }
        float y, t;
        y = p[0] - cx; t = sx + y; cx = (t - sx) - y; sx = t;
        y = p[1] - cy; t = sy + y; cy = (t - sy) - y; sy = t;
        y = p[2] - cz; t = sz + y; cz = (t - sz) - y; sz = t;
        y = p[3] - cp; t = sp + y; cp = (t - sp) - y; sp = t;
    }
    // Accepted nodes (see the FP64 form): separations from FP64, the rest FP32.
    __device__ inline void sum_nodes(const NodeEntryF* L, int len)
    {
        len = __builtin_amdgcn_readfirstlane(len);
        float p[4] = {0.f, 0.f, 0.f, 0.f};
        for (int jj = 0; jj < len; ++jj) {
            const NodeEntryF& q = L[jj];
            const float dx = (float)(q.x - xi), dy = (float)(q.y - yi), dz = (float)(q.z - zi);
            const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2)));
            const float rinv = __builtin_amdgcn_rsqf(r2);
            const float mr = q.m * rinv;
            const float ri2 = rinv * rinv;
            const float mr3 = mr * ri2;
            const float ri5 = rinv * ri2 * ri2, ri7 = ri5 * ri2;
            // with d = -(dx, dy, dz) and U = 3 S d: br = d.U - rho^2 T and
            // a_Q = (U - T d) rho^-5 - (5/2) br rho^-7 d = U rho^-5 - k d
            const float d0 = -dx, d1 = -dy, d2 = -dz;
            const float U0 = fmaf(q.S3[0], d0, fmaf(q.S3[3], d1, q.S3[4] * d2));
            const float U1 = fmaf(q.S3[3], d0, fmaf(q.S3[1], d1, q.S3[5] * d2));
            const float U2 = fmaf(q.S3[4], d0, fmaf(q.S3[5], d1, q.S3[2] * d2));
            const float br = fmaf(-r2, q.T, fmaf(d0, U0, fmaf(d1, U1, d2 * U2)));
            const float c5 = 2.5f * br * ri7;
            const float k = fmaf(q.T, ri5, c5);
            p[0] += fmaf(mr3, dx, fmaf(U0, ri5, -k * d0));
            p[1] += fmaf(mr3, dy, fmaf(U1, ri5, -k * d1));
            p[2] += fmaf(mr3, dz, fmaf(U2, ri5, -k * d2));
            p[3] += fmaf(0.5f * br, ri5, mr);
        }
        float y, t;
        y = p[0] - cx; t = sx + y; cx = (t - sx) - y; sx = t;
        y = p[1] - cy; t = sy + y; cy = (t - sy) - y; sy = t;
        y = p[2] - cz; t = sz + y; cz = (t - sz) - y; sz = t;
        y = p[3] - cp; t = sp + y; cp = (t - sp) - y; sp = t;
    }
    __device__ inline double4 result() const
    {
        return make_double4((double)sx - (double)cx, (double)sy - (double)cy,
                            (double)sz - (double)cz, (double)sp - (double)cp);
    }
};


// ---------------------------------------------------------------- walk
// One block = one wave = one part of one group's walk (writing the group's
// partial row of that part).  tick > 0: tick of a cycle of block steps
// (groups without an active member are skipped).
template <bool MIXED>
__global__ __launch_bounds__(64) void k_tree_walk(
    const BucketInfo* __restrict__ buckets, const NodeChild* __restrict__ nodes,
    const double* __restrict__ box, const double4* __restrict__ mom,
    const double* __restrict__ mom2, const HaloDev* __restrict__ halos, const double* __restrict__ sx,
    const double* __restrict__ sy, const double* __restrict__ sz, const double* __restrict__ sm,
    const uint32_t* __restrict__ perm, const double* __restrict__ ax_old,
    const double* __restrict__ ay_old, const double* __restrict__ az_old,
    const int8_t* __restrict__ bin, int tick, int bmax, double4* __restrict__ partial,
    unsigned long long* __restrict__ terms, int parts)
{
    using Acc = TreeAcc<MIXED>;
    using Entry = typename Acc::Entry;
    __shared__ Entry list[kTreeList];
    using Node = typename NodeOf<MIXED>::type;
    __shared__ Node nlist[kTreeNodes];
    // pending inner nodes as (first child, number of children)
    __shared__ int2 stack[kTreeStack];

    // part s of group g, in the dispatcher's order (runs of groups per XCD
    // would put the costly centre groups, neighbours on the Morton curve, on
    // one XCD)
    const int64_t g = blockIdx.x / parts;
    const int s = (int)(blockIdx.x % parts);
    const int lane = threadIdx.x;
    const BucketInfo GB = buckets[g];
    const HaloDev& H = halos[GB.halo];
    if (!(H.tree_alpha > 0.0) || s >= H.grav_split) return;
    const int nparts = H.grav_split;
    const int front = nparts > 1 ? tree_front_level(H.level_n, H.n_levels, nparts) : -1;
    const bool live = lane < GB.count;
    const int64_t p = GB.start + (live ? lane : 0);
    const int64_t o = perm[p];
    if (tick > 0) {
        const int kl = local_tick(H, tick, bmax);
        const bool act = live && kl > 0 && bin_active(H, bin[o], kl);
        if (!__syncthreads_or(act)) return;
    }
    double gb[6];
    for (int q = 0; q < 6; ++q) gb[q] = box[6 * g + q];
    double a2;
    {
#pragma clang fp contract(off)
        const double ux = ax_old[o], uy = ay_old[o], uz = az_old[o];
        a2 = live ? (ux * ux + uy * uy) + uz * uz : INFINITY;
    }
    const double a2min = wave_min(a2);
    const double alpha2 = H.tree_alpha * H.tree_alpha;

    Acc acc;
    {
        acc.xi = sx[p];
        acc.yi = sy[p];
        acc.zi = sz[p];
        acc.eps2 = H.eps2;
    }

    const int64_t root = H.level_off[H.n_levels - 1];
    int sp = 0, len = 0, nlen = 0, self_lo = -1, self_n = 0;
    unsigned long long total = 0;

    auto flush = [&]() {
        __syncthreads();
        if (len > 0) acc.sum(list, len, self_lo, self_n, lane);
        if (nlen > 0) acc.sum_nodes(nlist, nlen);
        total += (unsigned long long)(len + nlen);
        len = 0;
        nlen = 0;
        self_lo = -1;
        __syncthreads();
    };
    // appends the particles of an opened bucket
    auto append_bucket = [&](int64_t start, int cnt, bool self) {
        if (len + cnt > kTreeList) flush();
        if (lane < cnt) {
            const int64_t q = start + lane;
            list[len + lane] = make_entry<MIXED>(sx[q], sy[q], sz[q], sm[q]);
        }
        if (self) {
            self_lo = len;
            self_n = cnt;
        }
        len += cnt;
    };

    // a stack entry: first child and (number of children | their level << 4)
    {
        const NodeChild rc = nodes[root];
        if (rc.nchild > 0) {
            if (lane == 0) stack[0] = make_int2((int)rc.child0, rc.nchild | ((H.n_levels - 2) << 4));
            sp = 1;
        } else {
            append_bucket(GB.start, GB.count, true);   // a halo of one bucket
        }
        __syncthreads();
    }

    // Each round pops up to kTreePop pending nodes; lane 8 s + k tests child k of
    // the s-th popped node, so one round of dependent loads serves 64 children.
    while (sp > 0) {
        const int npop = sp < kTreePop ? sp : kTreePop;
        const int slot = lane / kFanout, ci = lane % kFanout;
        int2 nd = make_int2(0, 0);
        if (slot < npop) nd = stack[sp - 1 - slot];
        sp -= npop;
        bool take = false, open_inner = false, open_bucket = false, self = false;
        Node e{};
        int2 push = make_int2(0, 0);
        int64_t bstart = 0;
        int bcnt = 0;
        const int lvl = nd.y >> 4;
        const int64_t c = (int64_t)nd.x + ci;
        // a frontier node belongs to one part; those above it count in part 0
        const bool own = lvl != front || (int)(c - H.level_off[front]) % nparts == s;
        if (slot < npop && ci < (nd.y & 15) && own) {
            double cb[6];
            for (int q = 0; q < 6; ++q) cb[q] = box[6 * c + q];
            const double4 mm = mom[c];
            const NodeChild cc = nodes[c];
            if (tree_accept(cb, mm.x, gb, H.G, alpha2, a2min)) {
                if (mm.x != 0.0 && (lvl <= front || s == 0)) {
                    take = true;
                    set_node(e, mm.y / mm.x, mm.z / mm.x, mm.w / mm.x, mm.x, mom2 + 6 * c);
                }
            } else if (cc.nchild > 0) {
                open_inner = true;
                push = make_int2((int)cc.child0, cc.nchild | ((lvl - 1) << 4));
            } else {
                open_bucket = true;
                const BucketInfo cbk = buckets[c];
                bstart = cbk.start;
                bcnt = cbk.count;
                self = c == g;
            }
        }
        __syncthreads();   // the popped entries are read before pushes reuse them
        const unsigned long long below = (1ull << lane) - 1ull;
        const unsigned long long tm = __ballot(take);
        const int nt = __popcll(tm);
        if (nlen + nt > kTreeNodes) flush();
        if (take) nlist[nlen + __popcll(tm & below)] = e;
        nlen += nt;
        const unsigned long long om = __ballot(open_inner);
        if (open_inner) stack[sp + __popcll(om & below)] = push;
        sp += __popcll(om);
        unsigned long long bm = __ballot(open_bucket);
        while (bm) {
            const int src = __ffsll((long long)bm) - 1;
            bm &= bm - 1ull;
            const int64_t st = __shfl(bstart, src, 64);
            const int cnt = __shfl(bcnt, src, 64);
            const int sf = __shfl((int)self, src, 64);
            append_bucket(st, cnt, sf != 0);
        }
        __syncthreads();
    }
    flush();
    if (live) partial[H.part_base + (int64_t)s * H.n + (p - H.sbase)] = acc.result();
    if (lane == 0) atomicAdd(&terms[GB.halo], total);
}

// ---------------------------------------------------------------- launcher
static unsigned grid_of(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

// Expects the cell list and its boxes in place; writes partial row 0 of every
// particle of a tree halo and adds each halo's source terms to w.tree_terms.
hipError_t launch_tree_gravity(bool mixed, const Plan& P, Scratch& w, const sidm_state* s,
                               int tick, int bmax, hipStream_t st)
{
    hipLaunchKernelGGL(k_tree_mom_bucket, dim3(grid_of(P.n_buckets, 256)), dim3(256), 0, st,
                       w.buckets, P.n_buckets, w.sx, w.sy, w.sz, w.sm, w.mom, w.mom2);
    for (int l = 1; l < P.n_levels; ++l) {
        const int64_t t0 = P.level_task_off[l - 1], nt = P.level_task_off[l] - t0;
        if (nt > 0)
            hipLaunchKernelGGL(k_tree_mom_node, dim3(grid_of(nt, 256)), dim3(256), 0, st,
                               w.node_tasks + t0, nt, w.mom, w.mom2);
    }
    int parts = 1;
    for (const auto& H : P.halos)
        if (H.tree_alpha > 0.0) parts = std::max(parts, (int)H.grav_split);
    const dim3 grid((unsigned)(P.n_buckets * parts));
    if (mixed)
        hipLaunchKernelGGL(k_tree_walk<true>, grid, dim3(64), 0, st, w.buckets, w.nodes, w.box,
                           w.mom, w.mom2, w.halos, w.sx, w.sy, w.sz, w.sm, w.perm, s->ax, s->ay,
                           s->az, w.bin, tick, bmax, w.partial, w.tree_terms, parts);
    else
        hipLaunchKernelGGL(k_tree_walk<false>, grid, dim3(64), 0, st, w.buckets, w.nodes, w.box,
                           w.mom, w.mom2, w.halos, w.sx, w.sy, w.sz, w.sm, w.perm, s->ax, s->ay,
                           s->az, w.bin, tick, bmax, w.partial, w.tree_terms, parts);
    return hipGetLastError();
}

hipError_t launch_tree_terms_reset(Scratch& w, int n_halos, hipStream_t st)
{
    hipLaunchKernelGGL(k_tree_terms_reset, dim3(grid_of(n_halos, 64)), dim3(64), 0, st,
                       w.tree_terms, n_halos);
    return hipGetLastError();
}

}  // namespace sidm
