// sidm_steps.hpp -- block time steps (Sec. 2: individual steps from the
// gravitational criterion eta of Springel 2005 eq. 34 and a minimum step).
//
// One cycle of length dt is cut into 2^max_bin ticks; a particle in bin b
// steps s = dt / 2^b and is active on every 2^(max_bin - b)-th tick.  Halos
// with different max_bin share the ticks of the deepest one (bmax): a halo
// steps on every 2^(bmax - max_bin)-th of them.
#pragma once
#include "sidm_internal.hpp"

namespace sidm {

// The bin of a particle with acceleration a: the smallest b in [0, max_bin]
// with s^2 |a| <= 2 eta eps for s = dt / 2^b, tested squared, (s^2)^2 |a|^2 <=
// (2 eta eps)^2, so that the integer decision is a fixed sequence of IEEE
// products and sums; then b decreases while s < dt_min.
__device__ inline int time_bin(const HaloDev& H, double ax, double ay, double az)
{
#pragma clang fp contract(off)
    if (H.max_bin == 0) return 0;
    const double a2 = (ax * ax + ay * ay) + az * az;
    const double lim = 2.0 * H.eta * H.eps;
    const double lim2 = lim * lim;
    int b = 0;
    for (;;) {
        const double s = ldexp(H.dt, -b);
        const double s2 = s * s;
        if (b >= H.max_bin || !((s2 * s2) * a2 > lim2)) break;
        ++b;
    }
    while (b > 0 && ldexp(H.dt, -b) < H.dt_min) --b;
    return b;
}

// The halo's own tick (1 .. 2^max_bin) at tick `tick` of the call's cycle of
// 2^bmax ticks, or 0 when the halo does not step then.
__device__ inline int local_tick(const HaloDev& H, int tick, int bmax)
{
    const int sh = bmax - H.max_bin;
    return (tick & ((1 << sh) - 1)) ? 0 : (tick >> sh);
}

// Whether bin b steps at local tick kl (kl = 0: never).
__device__ inline bool bin_active(const HaloDev& H, int b, int kl)
{
    return kl > 0 && (kl & ((1 << (H.max_bin - b)) - 1)) == 0;
}

// Half of the step of bin b.
__device__ inline double half_step(const HaloDev& H, int b)
{
    return 0.5 * ldexp(H.dt, -b);
}

}  // namespace sidm
