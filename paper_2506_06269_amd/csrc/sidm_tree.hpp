// sidm_tree.hpp -- wave-level depth-first visit of a halo's bucket tree.
#pragma once

#include "sidm_plan.hpp"

namespace sidm {

constexpr int kStackMax = 96;

// A value every lane of the wave holds, moved to a scalar register so that the
// loads it addresses are issued once per wave.
__device__ inline int64_t wave_uniform(int64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Squared distance from point p to an axis-aligned box (lo xyz, hi xyz).
__device__ inline double point_box_dist2(double px, double py, double pz,
                                         const double* __restrict__ b)
{
    const double gx = fmax(fmax(b[0] - px, px - b[3]), 0.0);
    const double gy = fmax(fmax(b[1] - py, py - b[4]), 0.0);
    const double gz = fmax(fmax(b[2] - pz, pz - b[5]), 0.0);
    return gx * gx + gy * gy + gz * gz;
}

// Visits, in depth-first order, every bucket of the halo for which some lane
// of the wave answers `lane_test(node)` with true; internal nodes are entered
// on the same condition (the test must be monotone: true for a bucket implies
// true for its ancestors).  `keep(node)` prunes by node index (wave-uniform).
// Every lane calls f(bucket) for every visited bucket.  One wave per block.
template <class LaneTest, class Keep, class F>
__device__ inline void tree_visit(const HaloDev& H, const NodeChild* __restrict__ nodes,
                                  int64_t n_buckets, int64_t* stack, LaneTest lane_test,
                                  Keep keep, F f)
{
    const int lane = threadIdx.x & 63;
    const int64_t root = H.level_off[H.n_levels - 1];
    if (H.n_levels == 1) {
        if (keep(root) && __ballot(lane_test(root))) f(root);
        return;
    }
    __syncthreads();
    if (lane == 0) stack[0] = root;
    int sp = 1;
    __syncthreads();
    while (sp > 0) {
        const int64_t node = wave_uniform(stack[sp - 1]);
        --sp;
        const NodeChild N = nodes[node];
        unsigned hits = 0u;
        for (int c = 0; c < N.nchild; ++c) {
            const int64_t ch = N.child0 + c;
            if (keep(ch) && __ballot(lane_test(ch))) hits |= 1u << c;
        }
        __syncthreads();   // every lane has read stack[sp] before it is reused
        if (N.child0 < n_buckets) {
            for (int c = 0; c < N.nchild; ++c)
                if ((hits >> c) & 1u) f(N.child0 + c);
        } else {
            for (int c = N.nchild - 1; c >= 0; --c)
                if ((hits >> c) & 1u) {
                    if (lane == 0) stack[sp] = N.child0 + c;
                    ++sp;
                }
            __syncthreads();
        }
    }
}

}  // namespace sidm
