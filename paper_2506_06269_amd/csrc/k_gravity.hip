// k_gravity.hip -- softened direct-sum self-gravity plus the static NFW host
// (Sec. 2: softening length eps; Sec. 4.1 Eq. nfw_potential).
//
// Work decomposition: a work item is (halo, i-block of kGravThreads * IREG
// particles, j-range).  Each thread keeps IREG i-particles in registers; the
// block stages kGravTileJ j-particles at a time in LDS with one coalesced load
// per thread, and every lane of a wave reads the same j (LDS broadcast).  The
// pair terms of one tile are summed plainly, and the tile sums are folded into
// Kahan-compensated accumulators, so the rounding error does not grow with N.
// The self pair j == i is skipped exactly in the few tiles that hold i.
// Each item writes one FP64 partial row per i; a finalize pass adds the rows
// of an i in a fixed order, scales by G, adds the host and (optionally)
// applies the closing half kick.
#include "sidm_internal.hpp"

namespace sidm {

// ---------------------------------------------------------------- recentre
// Mean position of each halo (FP64), deterministic two-level reduction.
__global__ __launch_bounds__(kStreamBlock) void k_block_sum_pos(
    const double* __restrict__ x, const double* __restrict__ y, const double* __restrict__ z,
    const StreamBlock* __restrict__ blocks, double* __restrict__ bsum)
{
    __shared__ double red[3][kStreamBlock];
    const StreamBlock B = blocks[blockIdx.x];
    const int t = threadIdx.x;
    double sx = 0, sy = 0, sz = 0;
    if (t < B.count) {
        const int64_t i = B.start + t;
        sx = x[i]; sy = y[i]; sz = z[i];
    }
    red[0][t] = sx; red[1][t] = sy; red[2][t] = sz;
    __syncthreads();
    for (int s = kStreamBlock / 2; s > 0; s >>= 1) {
        if (t < s) {
            red[0][t] += red[0][t + s];
            red[1][t] += red[1][t + s];
            red[2][t] += red[2][t + s];
        }
        __syncthreads();
    }
    if (t == 0) {
        bsum[3 * (int64_t)blockIdx.x + 0] = red[0][0];
        bsum[3 * (int64_t)blockIdx.x + 1] = red[1][0];
        bsum[3 * (int64_t)blockIdx.x + 2] = red[2][0];
    }
}

// One block per halo: sums its block partials in a fixed order.
__global__ __launch_bounds__(kStreamBlock) void k_halo_mean_pos(
    const HaloDev* __restrict__ halos, const double* __restrict__ bsum,
    double* __restrict__ cref)
{
    __shared__ double red[3][kStreamBlock];
    const HaloDev& H = halos[blockIdx.x];
    const int t = threadIdx.x;
    const int64_t nb = (H.n + kStreamBlock - 1) / kStreamBlock;
    double s[3] = {0, 0, 0};
    for (int64_t b = t; b < nb; b += kStreamBlock)
        for (int c = 0; c < 3; ++c) s[c] += bsum[3 * (H.stream_block0 + b) + c];
    for (int c = 0; c < 3; ++c) red[c][t] = s[c];
    __syncthreads();
    for (int st = kStreamBlock / 2; st > 0; st >>= 1) {
        if (t < st)
            for (int c = 0; c < 3; ++c) red[c][t] += red[c][t + st];
        __syncthreads();
    }
    if (t == 0)
        for (int c = 0; c < 3; ++c) cref[3 * blockIdx.x + c] = red[c][0] / (double)H.n;
}

// x32 = f32(x - c_ref), w = f32(m)
__global__ __launch_bounds__(kStreamBlock) void k_pack32(
    const double* __restrict__ x, const double* __restrict__ y, const double* __restrict__ z,
    const double* __restrict__ m, const StreamBlock* __restrict__ blocks,
    const double* __restrict__ cref, float4* __restrict__ xm32)
{
    const StreamBlock B = blocks[blockIdx.x];
    const int t = threadIdx.x;
    if (t >= B.count) return;
    const int64_t i = B.start + t;
    const double* c = cref + 3 * B.halo;
    xm32[i] = make_float4((float)(x[i] - c[0]), (float)(y[i] - c[1]), (float)(z[i] - c[2]),
                          (float)m[i]);
}

// ---------------------------------------------------------------- FP32 tiles
template <int IREG>
__global__ __launch_bounds__(kGravThreads) void k_grav_mixed(
    const float4* __restrict__ xm32, const GravItem* __restrict__ items,
    const HaloDev* __restrict__ halos, double4* __restrict__ partial)
{
    __shared__ float4 tile[kGravTileJ];
    const GravItem it = items[blockIdx.x];
    const HaloDev& H = halos[it.halo];
    const int64_t hend = H.offset + H.n;
    const int t = threadIdx.x;
    const float eps2 = (float)H.eps2;

    float xi[IREG], yi[IREG], zi[IREG];
    float sx[IREG], sy[IREG], sz[IREG], sp[IREG];     // Kahan sums
    float cx[IREG], cy[IREG], cz[IREG], cp[IREG];     // Kahan compensations
#pragma unroll
    for (int r = 0; r < IREG; ++r) {
        const int64_t i = it.i0 + (int64_t)r * kGravThreads + t;
        float4 p = make_float4(0.f, 0.f, 0.f, 0.f);
        if (i < hend) p = xm32[i];
        xi[r] = p.x; yi[r] = p.y; zi[r] = p.z;
        sx[r] = sy[r] = sz[r] = sp[r] = 0.f;
        cx[r] = cy[r] = cz[r] = cp[r] = 0.f;
    }

    for (int64_t j0 = it.j0; j0 < it.j1; j0 += kGravTileJ) {
        const int64_t j = j0 + t;
        float4 pj = make_float4(0.f, 0.f, 0.f, 0.f);   // m = 0 pads the last tile
        if (j < it.j1) pj = xm32[j];
        __syncthreads();
        tile[t] = pj;
        __syncthreads();
        float px[IREG], py[IREG], pz[IREG], pp[IREG];
#pragma unroll
        for (int r = 0; r < IREG; ++r) px[r] = py[r] = pz[r] = pp[r] = 0.f;
        // the few tiles that hold i itself skip j == i exactly; all others
        // run the branch-free loop
        const bool diag = j0 < it.i0 + (int64_t)IREG * kGravThreads && j0 + kGravTileJ > it.i0;
        if (diag) {
            for (int jj = 0; jj < kGravTileJ; ++jj) {
                const float4 q = tile[jj];
#pragma unroll
                for (int r = 0; r < IREG; ++r) {
                    const float dx = q.x - xi[r];
                    const float dy = q.y - yi[r];
                    const float dz = q.z - zi[r];
                    const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2)));
                    const float rinv = __builtin_amdgcn_rsqf(r2);
                    const bool self = j0 + jj == it.i0 + (int64_t)r * kGravThreads + t;
                    const float mr = self ? 0.f : q.w * rinv;
                    const float mr3 = mr * (rinv * rinv);
                    px[r] = fmaf(mr3, dx, px[r]);
                    py[r] = fmaf(mr3, dy, py[r]);
                    pz[r] = fmaf(mr3, dz, pz[r]);
                    pp[r] += mr;
                }
            }
        } else {
#pragma unroll 4
            for (int jj = 0; jj < kGravTileJ; ++jj) {
                const float4 q = tile[jj];
#pragma unroll
                for (int r = 0; r < IREG; ++r) {
                    const float dx = q.x - xi[r];
                    const float dy = q.y - yi[r];
                    const float dz = q.z - zi[r];
                    const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2)));
                    const float rinv = __builtin_amdgcn_rsqf(r2);
                    const float mr = q.w * rinv;
                    const float mr3 = mr * (rinv * rinv);
                    px[r] = fmaf(mr3, dx, px[r]);
                    py[r] = fmaf(mr3, dy, py[r]);
                    pz[r] = fmaf(mr3, dz, pz[r]);
                    pp[r] += mr;
                }
            }
        }
#pragma unroll
        for (int r = 0; r < IREG; ++r) {
            float yk, tk;
            yk = px[r] - cx[r]; tk = sx[r] + yk; cx[r] = (tk - sx[r]) - yk; sx[r] = tk;
            yk = py[r] - cy[r]; tk = sy[r] + yk; cy[r] = (tk - sy[r]) - yk; sy[r] = tk;
            yk = pz[r] - cz[r]; tk = sz[r] + yk; cz[r] = (tk - sz[r]) - yk; sz[r] = tk;
            yk = pp[r] - cp[r]; tk = sp[r] + yk; cp[r] = (tk - sp[r]) - yk; sp[r] = tk;
        }
    }
#pragma unroll
    for (int r = 0; r < IREG; ++r) {
        const int64_t i = it.i0 + (int64_t)r * kGravThreads + t;
        if (i >= hend) continue;
        const int64_t row = H.part_base + (int64_t)it.slot * H.n + (i - H.offset);
        // the compensation holds the negated lost low part
        partial[row] = make_double4((double)sx[r] - (double)cx[r], (double)sy[r] - (double)cy[r],
                                    (double)sz[r] - (double)cz[r], (double)sp[r] - (double)cp[r]);
    }
}

// ---------------------------------------------------------------- FP64 tiles
template <int IREG>
__global__ __launch_bounds__(kGravThreads) void k_grav_fp64(
    const double* __restrict__ x, const double* __restrict__ y, const double* __restrict__ z,
    const double* __restrict__ m, const GravItem* __restrict__ items,
    const HaloDev* __restrict__ halos, double4* __restrict__ partial)
{
    __shared__ double4 tile[kGravTileJ];
    const GravItem it = items[blockIdx.x];
    const HaloDev& H = halos[it.halo];
    const int64_t hend = H.offset + H.n;
    const int t = threadIdx.x;
    const double eps2 = H.eps2;

    double xi[IREG], yi[IREG], zi[IREG];
    double sx[IREG], sy[IREG], sz[IREG], sp[IREG];
    double cx[IREG], cy[IREG], cz[IREG], cp[IREG];
#pragma unroll
    for (int r = 0; r < IREG; ++r) {
        const int64_t i = it.i0 + (int64_t)r * kGravThreads + t;
        xi[r] = yi[r] = zi[r] = 0.0;
        if (i < hend) { xi[r] = x[i]; yi[r] = y[i]; zi[r] = z[i]; }
        sx[r] = sy[r] = sz[r] = sp[r] = 0.0;
        cx[r] = cy[r] = cz[r] = cp[r] = 0.0;
    }
    for (int64_t j0 = it.j0; j0 < it.j1; j0 += kGravTileJ) {
        const int64_t j = j0 + t;
        double4 pj = make_double4(0.0, 0.0, 0.0, 0.0);
        if (j < it.j1) pj = make_double4(x[j], y[j], z[j], m[j]);
        __syncthreads();
        tile[t] = pj;
        __syncthreads();
        double px[IREG], py[IREG], pz[IREG], pp[IREG];
#pragma unroll
        for (int r = 0; r < IREG; ++r) px[r] = py[r] = pz[r] = pp[r] = 0.0;
        const bool diag = j0 < it.i0 + (int64_t)IREG * kGravThreads && j0 + kGravTileJ > it.i0;
#pragma unroll 2
        for (int jj = 0; jj < kGravTileJ; ++jj) {
            const double4 q = tile[jj];
#pragma unroll
            for (int r = 0; r < IREG; ++r) {
                const double dx = q.x - xi[r];
                const double dy = q.y - yi[r];
                const double dz = q.z - zi[r];
                const double r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, eps2)));
                const double rinv = rsqrt(r2);
                const bool self = diag && j0 + jj == it.i0 + (int64_t)r * kGravThreads + t;
                const double mr = self ? 0.0 : q.w * rinv;
                const double mr3 = mr * (rinv * rinv);
                px[r] = fma(mr3, dx, px[r]);
                py[r] = fma(mr3, dy, py[r]);
                pz[r] = fma(mr3, dz, pz[r]);
                pp[r] += mr;
            }
        }
#pragma unroll
        for (int r = 0; r < IREG; ++r) {
            double yk, tk;
            yk = px[r] - cx[r]; tk = sx[r] + yk; cx[r] = (tk - sx[r]) - yk; sx[r] = tk;
            yk = py[r] - cy[r]; tk = sy[r] + yk; cy[r] = (tk - sy[r]) - yk; sy[r] = tk;
            yk = pz[r] - cz[r]; tk = sz[r] + yk; cz[r] = (tk - sz[r]) - yk; sz[r] = tk;
            yk = pp[r] - cp[r]; tk = sp[r] + yk; cp[r] = (tk - sp[r]) - yk; sp[r] = tk;
        }
    }
#pragma unroll
    for (int r = 0; r < IREG; ++r) {
        const int64_t i = it.i0 + (int64_t)r * kGravThreads + t;
        if (i >= hend) continue;
        const int64_t row = H.part_base + (int64_t)it.slot * H.n + (i - H.offset);
        partial[row] = make_double4(sx[r] - cx[r], sy[r] - cy[r], sz[r] - cz[r], sp[r] - cp[r]);
    }
}

// ---------------------------------------------------------------- host + finalize
// NFW host (Sec. 4.1, Eq. nfw_potential): Phi = -K ln(1 + s)/r with s = r/r_s,
// K = 4 pi G rho_s r_s^3; the force follows from the enclosed mass,
// a = -K [ln(1+s) - s/(1+s)] (x - c) / r^3 (series in s below 1e-4).
__device__ inline void host_nfw(const HaloDev& H, double px, double py, double pz,
                                double& ax, double& ay, double& az, double& phi)
{
    const double dx = px - H.host_c[0], dy = py - H.host_c[1], dz = pz - H.host_c[2];
    const double r2 = dx * dx + dy * dy + dz * dz;
    if (r2 == 0.0) {
        ax = ay = az = 0.0;
        phi = -H.host_K / H.host_r_s;
        return;
    }
    const double r = sqrt(r2);
    const double s = r / H.host_r_s;
    const double l1p = log1p(s);
    double mu;
    if (s < 1e-4) mu = s * s * (0.5 - s * (2.0 / 3.0 - s * (0.75 - 0.8 * s)));
    else mu = l1p - s / (1.0 + s);
    const double f = -H.host_K * mu / (r2 * r);
    ax = f * dx; ay = f * dy; az = f * dz;
    phi = -H.host_K * l1p / r;
}

// Sums the partial rows of each i in slot order, scales by G, adds the host,
// optionally kicks v by a * dt/2.
__global__ __launch_bounds__(kStreamBlock) void k_grav_finalize(
    const StreamBlock* __restrict__ blocks, const HaloDev* __restrict__ halos,
    const double4* __restrict__ partial, const float4* __restrict__ xm32,
    const double* __restrict__ x, const double* __restrict__ y, const double* __restrict__ z,
    const double* __restrict__ m, double* __restrict__ ax, double* __restrict__ ay,
    double* __restrict__ az, double* __restrict__ pot, double* __restrict__ vx,
    double* __restrict__ vy, double* __restrict__ vz, int kick)
{
    const StreamBlock B = blocks[blockIdx.x];
    const int t = threadIdx.x;
    if (t >= B.count) return;
    const HaloDev& H = halos[B.halo];
    const int64_t i = B.start + t;
    const int64_t li = i - H.offset;
    double sx = 0, sy = 0, sz = 0, sp = 0;
    for (int s = 0; s < H.grav_split; ++s) {
        const double4 p = partial[H.part_base + (int64_t)s * H.n + li];
        sx += p.x; sy += p.y; sz += p.z; sp += p.w;
    }
    double gx = H.G * sx, gy = H.G * sy, gz = H.G * sz, gp = -H.G * sp;
    if (H.host_kind == 1) {
        double hx, hy, hz, hp;
        host_nfw(H, x[i], y[i], z[i], hx, hy, hz, hp);
        gx += hx; gy += hy; gz += hz; gp += hp;
    }
    ax[i] = gx; ay[i] = gy; az[i] = gz; pot[i] = gp;
    if (kick) {
        const double hdt = 0.5 * H.dt;
        vx[i] += gx * hdt; vy[i] += gy * hdt; vz[i] += gz * hdt;
    }
}

// ---------------------------------------------------------------- launchers
hipError_t launch_gravity(bool mixed, const double* x, const double* y, const double* z,
                          const double* m, const HaloDev* d_halos, int n_halos,
                          const StreamBlock* d_blocks, int64_t n_blocks, const GravItem* d_items,
                          int64_t n_items, double* bsum, double* cref, float4* xm32,
                          double4* partial, double* ax, double* ay, double* az, double* pot,
                          double* vx, double* vy, double* vz, int kick, hipStream_t st,
                          hipEvent_t tile_begin, hipEvent_t tile_end)
{
    if (mixed) {
        hipLaunchKernelGGL(k_block_sum_pos, dim3((unsigned)n_blocks), dim3(kStreamBlock), 0, st,
                           x, y, z, d_blocks, bsum);
        hipLaunchKernelGGL(k_halo_mean_pos, dim3(n_halos), dim3(kStreamBlock), 0, st, d_halos,
                           bsum, cref);
        hipLaunchKernelGGL(k_pack32, dim3((unsigned)n_blocks), dim3(kStreamBlock), 0, st, x, y, z,
                           m, d_blocks, cref, xm32);
        if (tile_begin) (void)hipEventRecord(tile_begin, st);
        hipLaunchKernelGGL((k_grav_mixed<4>), dim3((unsigned)n_items), dim3(kGravThreads), 0, st,
                           xm32, d_items, d_halos, partial);
        if (tile_end) (void)hipEventRecord(tile_end, st);
        hipLaunchKernelGGL(k_grav_finalize, dim3((unsigned)n_blocks), dim3(kStreamBlock),
                           0, st, d_blocks, d_halos, partial, xm32, x, y, z, m, ax, ay, az, pot,
                           vx, vy, vz, kick);
    } else {
        if (tile_begin) (void)hipEventRecord(tile_begin, st);
        hipLaunchKernelGGL((k_grav_fp64<4>), dim3((unsigned)n_items), dim3(kGravThreads), 0, st,
                           x, y, z, m, d_items, d_halos, partial);
        if (tile_end) (void)hipEventRecord(tile_end, st);
        hipLaunchKernelGGL(k_grav_finalize, dim3((unsigned)n_blocks), dim3(kStreamBlock),
                           0, st, d_blocks, d_halos, partial, xm32, x, y, z, m, ax, ay, az, pot,
                           vx, vy, vz, kick);
    }
    return hipGetLastError();
}

}  // namespace sidm
