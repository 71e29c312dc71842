// sidm_math.hpp -- per-pair arithmetic of the scattering pass, usable on the
// device and (for unit tests) on the host.
//
//   * Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of the
//     4x32 multiply-xor bijection, key advanced by the Weyl increments between
//     rounds.
//   * The spline kernel (Monaghan 1985, compact support h) and its overlap
//     integral Lambda(d; ha, hb) = int W(|x - xa|, ha) W(|x - xb|, hb) d^3x, the
//     geometric factor of the interaction probability (Sec. 3.5).  Evaluated
//     exactly: with s the distance from particle b, the part of a shell of
//     radius s about b that lies inside a's support contributes through the
//     closed-form radial moment T(q) = int_q^1 t w(t) dt of a's kernel, and the
//     remaining 1-D integral over s is a piecewise polynomial of degree 9 that
//     5-point Gauss-Legendre integrates exactly on each piece.
#pragma once

#include <cstdint>

#ifndef SIDM_HD
#if defined(__HIPCC__)
#define SIDM_HD __host__ __device__
#else
#define SIDM_HD
#endif
#endif

#include <cmath>

namespace sidm {

struct Philox4 {
    uint32_t w[4];
};

SIDM_HD inline Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                     uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t m0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t m1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(m1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(m0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)m1;
        c3 = (uint32_t)m0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    Philox4 o;
    o.w[0] = c0; o.w[1] = c1; o.w[2] = c2; o.w[3] = c3;
    return o;
}

// top 53 bits of (hi:lo) as a double in [0, 1)
SIDM_HD inline double unit53(uint32_t hi, uint32_t lo)
{
    const uint64_t b = ((((uint64_t)hi) << 32) | (uint64_t)lo) >> 11;
    return (double)b * 1.1102230246251565404e-16;  // 2^-53
}

// dimensionless spline shape w(q), W(r, h) = 8 / (pi h^3) w(r / h)
SIDM_HD inline double spline_w(double q)
{
    if (q <= 0.5) return 1.0 + q * q * (6.0 * q - 6.0);
    if (q <= 1.0) {
        const double t = 1.0 - q;
        return 2.0 * t * t * t;
    }
    return 0.0;
}

// Tail moment T(q) = int_q^1 t w(t) dt (zero beyond the support):
// with u = 1 - q, T = u^4 (1/2 - 2u/5) on the outer branch, and
// 7/80 - (q^2/2 - 3q^4/2 + 6q^5/5) on the inner branch.  Written in terms of
// the tail so that shells near the edge of the support keep full precision.
SIDM_HD inline double spline_tail(double q)
{
    if (q >= 1.0) return 0.0;
    if (q > 0.5) {
        const double u = 1.0 - q;
        const double u2 = u * u;
        return u2 * u2 * (0.5 - 0.4 * u);
    }
    const double q2 = q * q;
    return 0.0875 - q2 * (0.5 + q2 * (1.2 * q - 1.5));
}

SIDM_HD inline void sort8(double* v, int n)
{
    for (int i = 1; i < n; ++i) {
        const double x = v[i];
        int j = i - 1;
        while (j >= 0 && v[j] > x) {
            v[j + 1] = v[j];
            --j;
        }
        v[j + 1] = x;
    }
}

// Lambda(d; ha, hb), symmetric in (ha, hb); zero for d >= ha + hb.
SIDM_HD inline double kernel_overlap(double d, double ha, double hb)
{
    const double kPi = 3.14159265358979323846;
    const double gx[5] = {-0.90617984593866399280, -0.53846931010568309104, 0.0,
                          0.53846931010568309104, 0.90617984593866399280};
    const double gw[5] = {0.23692688505618908751, 0.47862867049936646804,
                          0.56888888888888888889, 0.47862867049936646804,
                          0.23692688505618908751};
    if (!(d < ha + hb)) return 0.0;
    if (d == 0.0) {
        // 4 pi int r^2 W_a W_b dr over [0, min(ha, hb)]
        const double hmin = ha < hb ? ha : hb;
        double bp[4] = {0.0, 0.5 * ha, 0.5 * hb, hmin};
        sort8(bp, 4);
        double acc = 0.0;
        for (int p = 0; p < 3; ++p) {
            const double r0 = bp[p], r1 = bp[p + 1] < hmin ? bp[p + 1] : hmin;
            if (!(r1 > r0)) continue;
            const double half = 0.5 * (r1 - r0), mid = r0 + half;
            double s = 0.0;
            for (int k = 0; k < 5; ++k) {
                const double r = mid + half * gx[k];
                s += gw[k] * r * r * spline_w(r / ha) * spline_w(r / hb);
            }
            acc += half * s;
        }
        return 4.0 * kPi * acc * 64.0 / (kPi * kPi * ha * ha * ha * hb * hb * hb);
    }
    // outer variable s = distance from b, over [0, hb]
    double bp[8];
    int nb = 0;
    bp[nb++] = 0.0;
    bp[nb++] = hb;
    const double cand[6] = {0.5 * hb, d, fabs(d - 0.5 * ha), d + 0.5 * ha, fabs(d - ha), d + ha};
    for (int c = 0; c < 6; ++c)
        if (cand[c] > 0.0 && cand[c] < hb) bp[nb++] = cand[c];
    sort8(bp, nb);
    const double inv_ha = 1.0 / ha, inv_hb = 1.0 / hb;
    double acc = 0.0;
    for (int p = 0; p + 1 < nb; ++p) {
        const double s0 = bp[p], s1 = bp[p + 1];
        if (!(s1 > s0)) continue;
        const double half = 0.5 * (s1 - s0), mid = s0 + half;
        double sum = 0.0;
        for (int k = 0; k < 5; ++k) {
            const double s = mid + half * gx[k];
            const double shell = spline_tail(fabs(d - s) * inv_ha) - spline_tail((d + s) * inv_ha);
            sum += gw[k] * s * spline_w(s * inv_hb) * shell;
        }
        acc += half * sum;
    }
    // (2 pi / d) * 8/(pi hb^3) * 8/(pi ha) * acc
    return 128.0 * acc / (kPi * d * ha * hb * hb * hb);
}

}  // namespace sidm
