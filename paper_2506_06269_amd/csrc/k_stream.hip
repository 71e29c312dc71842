// k_stream.hip -- streaming FP64 passes of the leapfrog and the energy and
// momentum reductions (kick-drift-kick with a fixed step or block steps; the
// paper's energy error is measured relative to the absolute initial energy,
// App. B).
#include "sidm_host.hpp"
#include "sidm_steps.hpp"

namespace sidm {

// Reflecting sphere (Sec. 2): at the drifted position p, outward motion beyond
// the radius is turned inward, v -> v - 2 (v.d) d / |d|^2 (|v| kept).
__device__ inline void reflect(const HaloDev& H, double px, double py, double pz, double& ux,
                               double& uy, double& uz)
{
#pragma clang fp contract(off)
    if (!(H.bnd_r > 0.0)) return;
    const double dx = px - H.bnd_c[0], dy = py - H.bnd_c[1], dz = pz - H.bnd_c[2];
    const double d2 = (dx * dx + dy * dy) + dz * dz;
    const double vd = (ux * dx + uy * dy) + uz * dz;
    if (d2 > H.bnd_r * H.bnd_r && vd > 0.0) {
        const double f = 2.0 * vd / d2;
        ux = ux - f * dx; uy = uy - f * dy; uz = uz - f * dz;
    }
}

// v += a dt/2 ; x += v dt   (opening half kick fused with the drift)
__global__ __launch_bounds__(kStreamBlock) void k_kick_drift(
    const StreamBlock* __restrict__ blocks, const HaloDev* __restrict__ halos,
    double* __restrict__ x, double* __restrict__ y, double* __restrict__ z,
    double* __restrict__ vx, double* __restrict__ vy, double* __restrict__ vz,
    const double* __restrict__ ax, const double* __restrict__ ay, const double* __restrict__ az)
{
#pragma clang fp contract(off)
    const StreamBlock B = blocks[blockIdx.x];
    const int t = threadIdx.x;
    if (t >= B.count) return;
    const HaloDev& H = halos[B.halo];
    const int64_t i = B.start + t;
    const double hdt = 0.5 * H.dt;
    double ux = vx[i] + ax[i] * hdt;
    double uy = vy[i] + ay[i] * hdt;
    double uz = vz[i] + az[i] * hdt;
    const double px = x[i] + ux * H.dt, py = y[i] + uy * H.dt, pz = z[i] + uz * H.dt;
    x[i] = px; y[i] = py; z[i] = pz;
    reflect(H, px, py, pz, ux, uy, uz);
    vx[i] = ux; vy[i] = uy; vz[i] = uz;
}

// Start of a cycle of block steps: the bin of every particle from its
// acceleration, and its opening half kick v += a s/2.
__global__ __launch_bounds__(kStreamBlock) void k_open_kick(
    const StreamBlock* __restrict__ blocks, const HaloDev* __restrict__ halos,
    double* __restrict__ vx, double* __restrict__ vy, double* __restrict__ vz,
    const double* __restrict__ ax, const double* __restrict__ ay, const double* __restrict__ az,
    int8_t* __restrict__ bin)
{
#pragma clang fp contract(off)
    const StreamBlock B = blocks[blockIdx.x];
    const int t = threadIdx.x;
    if (t >= B.count) return;
    const HaloDev& H = halos[B.halo];
    const int64_t i = B.start + t;
    const double gx = ax[i], gy = ay[i], gz = az[i];
    const int b = time_bin(H, gx, gy, gz);
    bin[i] = (int8_t)b;
    const double h = half_step(H, b);
    vx[i] = vx[i] + gx * h;
    vy[i] = vy[i] + gy * h;
    vz[i] = vz[i] + gz * h;
}

// One tick of a cycle: x += v dt / 2^max_bin for every particle of the halos
// that step at this tick, then the reflecting sphere.
__global__ __launch_bounds__(kStreamBlock) void k_tick_drift(
    const StreamBlock* __restrict__ blocks, const HaloDev* __restrict__ halos,
    double* __restrict__ x, double* __restrict__ y, double* __restrict__ z,
    double* __restrict__ vx, double* __restrict__ vy, double* __restrict__ vz, int tick, int bmax)
{
#pragma clang fp contract(off)
    const StreamBlock B = blocks[blockIdx.x];
    const int t = threadIdx.x;
    if (t >= B.count) return;
    const HaloDev& H = halos[B.halo];
    if (local_tick(H, tick, bmax) == 0) return;
    const int64_t i = B.start + t;
    const double tau = ldexp(H.dt, -H.max_bin);
    double ux = vx[i], uy = vy[i], uz = vz[i];
    const double px = x[i] + ux * tau, py = y[i] + uy * tau, pz = z[i] + uz * tau;
    x[i] = px; y[i] = py; z[i] = pz;
    if (H.bnd_r > 0.0) {
        reflect(H, px, py, pz, ux, uy, uz);
        vx[i] = ux; vy[i] = uy; vz[i] = uz;
    }
}

// Per-block partial sums of K, W, Eext, px, py, pz and a non-finite flag.
__global__ __launch_bounds__(kStreamBlock) void k_diag_block(
    const StreamBlock* __restrict__ blocks, const HaloDev* __restrict__ halos,
    const double* __restrict__ x, const double* __restrict__ y, const double* __restrict__ z,
    const double* __restrict__ vx, const double* __restrict__ vy, const double* __restrict__ vz,
    const double* __restrict__ m, const double* __restrict__ pot, double* __restrict__ bsum)
{
    __shared__ double red[7][kStreamBlock];
    const StreamBlock B = blocks[blockIdx.x];
    const HaloDev& H = halos[B.halo];
    const int t = threadIdx.x;
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    if (t < B.count) {
        const int64_t i = B.start + t;
        const double mi = m[i];
        const double ux = vx[i], uy = vy[i], uz = vz[i];
        double pe = 0.0;
        if (H.host_kind != 0) pe = host_potential(H, x[i], y[i], z[i]);
        v[0] = 0.5 * mi * ((ux * ux + uy * uy) + uz * uz);
        v[1] = 0.5 * mi * (pot[i] - pe);
        v[2] = mi * pe;
        v[3] = mi * ux; v[4] = mi * uy; v[5] = mi * uz;
        const double chk = x[i] + y[i] + z[i] + ux + uy + uz;
        v[6] = isfinite(chk) ? 0.0 : 1.0;
    }
    for (int c = 0; c < 7; ++c) red[c][t] = v[c];
    __syncthreads();
    for (int s = kStreamBlock / 2; s > 0; s >>= 1) {
        if (t < s)
            for (int c = 0; c < 7; ++c) red[c][t] += red[c][t + s];
        __syncthreads();
    }
    if (t < 7) bsum[7 * (int64_t)blockIdx.x + t] = red[t][0];
}

// One block per halo: fixed-order sum of the block partials into sidm_diag.
__global__ __launch_bounds__(kStreamBlock) void k_diag_halo(
    const HaloDev* __restrict__ halos, const double* __restrict__ bsum,
    const long long* __restrict__ ev_counts, const unsigned long long* __restrict__ tree_terms,
    const int* __restrict__ status, sidm_diag* __restrict__ diag)
{
    __shared__ double red[7][kStreamBlock];
    const HaloDev& H = halos[blockIdx.x];
    const int t = threadIdx.x;
    const int64_t nb = (H.n + kStreamBlock - 1) / kStreamBlock;
    double s[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int64_t b = t; b < nb; b += kStreamBlock)
        for (int c = 0; c < 7; ++c) s[c] += bsum[7 * (H.stream_block0 + b) + c];
    for (int c = 0; c < 7; ++c) red[c][t] = s[c];
    __syncthreads();
    for (int st = kStreamBlock / 2; st > 0; st >>= 1) {
        if (t < st)
            for (int c = 0; c < 7; ++c) red[c][t] += red[c][t + st];
        __syncthreads();
    }
    if (t == 0) {
        sidm_diag d;
        d.K = red[0][0]; d.W = red[1][0]; d.Eext = red[2][0];
        d.px = red[3][0]; d.py = red[4][0]; d.pz = red[5][0];
        const int h = blockIdx.x;
        d.n_events = ev_counts ? ev_counts[kEvCounts * h + 0] : 0;
        d.n_rounds = ev_counts ? ev_counts[kEvCounts * h + 1] : 0;
        d.n_pairs = ev_counts ? ev_counts[kEvCounts * h + 2] : 0;
        d.n_p_gt1 = ev_counts ? ev_counts[kEvCounts * h + 3] : 0;
        d.n_candidates = ev_counts ? ev_counts[kEvCounts * h + 4] : 0;
        d.status = (status ? status[h] : 0) | (red[6][0] > 0.0 ? SIDM_DEV_NONFINITE : 0);
        d.reserved = 0;
        d.n_grav_terms = tree_terms ? (int64_t)tree_terms[h] : 0;
        diag[h] = d;
    }
}

hipError_t launch_kick_drift(const StreamBlock* d_blocks, int64_t n_blocks, const HaloDev* d_halos,
                             double* x, double* y, double* z, double* vx, double* vy, double* vz,
                             const double* ax, const double* ay, const double* az, hipStream_t st)
{
    hipLaunchKernelGGL(k_kick_drift, dim3((unsigned)n_blocks), dim3(kStreamBlock), 0, st, d_blocks,
                       d_halos, x, y, z, vx, vy, vz, ax, ay, az);
    return hipGetLastError();
}

hipError_t launch_open_kick(const StreamBlock* d_blocks, int64_t n_blocks, const HaloDev* d_halos,
                            double* vx, double* vy, double* vz, const double* ax, const double* ay,
                            const double* az, int8_t* bin, hipStream_t st)
{
    hipLaunchKernelGGL(k_open_kick, dim3((unsigned)n_blocks), dim3(kStreamBlock), 0, st, d_blocks,
                       d_halos, vx, vy, vz, ax, ay, az, bin);
    return hipGetLastError();
}

hipError_t launch_tick_drift(const StreamBlock* d_blocks, int64_t n_blocks, const HaloDev* d_halos,
                             double* x, double* y, double* z, double* vx, double* vy, double* vz,
                             int tick, int bmax, hipStream_t st)
{
    hipLaunchKernelGGL(k_tick_drift, dim3((unsigned)n_blocks), dim3(kStreamBlock), 0, st, d_blocks,
                       d_halos, x, y, z, vx, vy, vz, tick, bmax);
    return hipGetLastError();
}

hipError_t launch_diag(const StreamBlock* d_blocks, int64_t n_blocks, const HaloDev* d_halos,
                       int n_halos, const double* x, const double* y, const double* z,
                       const double* vx, const double* vy, const double* vz, const double* m,
                       const double* pot, double* bsum, const long long* ev_counts,
                       const unsigned long long* tree_terms, const int* status, sidm_diag* diag,
                       hipStream_t st)
{
    hipLaunchKernelGGL(k_diag_block, dim3((unsigned)n_blocks), dim3(kStreamBlock), 0, st, d_blocks,
                       d_halos, x, y, z, vx, vy, vz, m, pot, bsum);
    hipLaunchKernelGGL(k_diag_halo, dim3(n_halos), dim3(kStreamBlock), 0, st, d_halos, bsum,
                       ev_counts, tree_terms, status, diag);
    return hipGetLastError();
}

// ---------------------------------------------------------------- central density
// Sec. 3 takes the minimum of the gravitational potential as the halo centre:
// the centre is the particle with the lowest self-potential pot - Phi_host
// (first index on ties, NaN never), and the central density counts the
// particles of the halo within a radius of it.

// Per streaming block: lowest self-potential and its index (as a double).
__global__ __launch_bounds__(kStreamBlock) void k_center_block(
    const StreamBlock* __restrict__ blocks, const HaloDev* __restrict__ halos,
    const double* __restrict__ x, const double* __restrict__ y, const double* __restrict__ z,
    const double* __restrict__ pot, double* __restrict__ bsum)
{
    __shared__ double val[kStreamBlock];
    __shared__ int64_t idx[kStreamBlock];
    const StreamBlock B = blocks[blockIdx.x];
    const HaloDev& H = halos[B.halo];
    const int t = threadIdx.x;
    double v = INFINITY;
    int64_t i = -1;
    if (t < B.count) {
        const int64_t p = B.start + t;
        double pe = 0.0;
        if (H.host_kind != 0) pe = host_potential(H, x[p], y[p], z[p]);
        const double ps = pot[p] - pe;
        if (ps == ps) { v = ps; i = p; }
    }
    val[t] = v;
    idx[t] = i;
    __syncthreads();
    for (int s = kStreamBlock / 2; s > 0; s >>= 1) {
        if (t < s) {
            const double vo = val[t + s];
            const int64_t io = idx[t + s];
            if (io >= 0 && (idx[t] < 0 || vo < val[t] || (vo == val[t] && io < idx[t]))) {
                val[t] = vo;
                idx[t] = io;
            }
        }
        __syncthreads();
    }
    if (t == 0) {
        bsum[7 * blockIdx.x + 0] = val[0];
        bsum[7 * blockIdx.x + 1] = (double)idx[0];
    }
}

// Per halo: the centre over its blocks; writes index and position.
__global__ __launch_bounds__(kStreamBlock) void k_center_halo(
    const HaloDev* __restrict__ halos, const double* __restrict__ bsum,
    const double* __restrict__ x, const double* __restrict__ y, const double* __restrict__ z,
    sidm_center* __restrict__ out)
{
    __shared__ double val[kStreamBlock];
    __shared__ int64_t idx[kStreamBlock];
    const HaloDev& H = halos[blockIdx.x];
    const int t = threadIdx.x;
    const int64_t nb = (H.n + kStreamBlock - 1) / kStreamBlock;
    double v = INFINITY;
    int64_t i = -1;
    for (int64_t b = t; b < nb; b += kStreamBlock) {
        const double vo = bsum[7 * (H.stream_block0 + b) + 0];
        const int64_t io = (int64_t)bsum[7 * (H.stream_block0 + b) + 1];
        if (io >= 0 && (i < 0 || vo < v || (vo == v && io < i))) { v = vo; i = io; }
    }
    val[t] = v;
    idx[t] = i;
    __syncthreads();
    for (int s = kStreamBlock / 2; s > 0; s >>= 1) {
        if (t < s) {
            const double vo = val[t + s];
            const int64_t io = idx[t + s];
            if (io >= 0 && (idx[t] < 0 || vo < val[t] || (vo == val[t] && io < idx[t]))) {
                val[t] = vo;
                idx[t] = io;
            }
        }
        __syncthreads();
    }
    if (t == 0) {
        sidm_center c;
        c.index = idx[0];
        c.x = c.index >= 0 ? x[c.index] : NAN;
        c.y = c.index >= 0 ? y[c.index] : NAN;
        c.z = c.index >= 0 ? z[c.index] : NAN;
        c.mass = 0.0;
        c.count = 0;
        out[blockIdx.x] = c;
    }
}

// Per streaming block: number and mass of the particles within the radius.
__global__ __launch_bounds__(kStreamBlock) void k_center_count_block(
    const StreamBlock* __restrict__ blocks, const double* __restrict__ radius,
    const double* __restrict__ x, const double* __restrict__ y, const double* __restrict__ z,
    const double* __restrict__ m, const sidm_center* __restrict__ out, double* __restrict__ bsum)
{
    __shared__ double cnt[kStreamBlock], mass[kStreamBlock];
    const StreamBlock B = blocks[blockIdx.x];
    const sidm_center C = out[B.halo];
    const int t = threadIdx.x;
    double c = 0.0, w = 0.0;
    if (t < B.count && C.index >= 0) {
#pragma clang fp contract(off)
        const int64_t p = B.start + t;
        const double r = radius[B.halo];
        const double dx = x[p] - C.x, dy = y[p] - C.y, dz = z[p] - C.z;
        const double d2 = (dx * dx + dy * dy) + dz * dz;
        if (d2 <= r * r) { c = 1.0; w = m[p]; }
    }
    cnt[t] = c;
    mass[t] = w;
    __syncthreads();
    for (int s = kStreamBlock / 2; s > 0; s >>= 1) {
        if (t < s) { cnt[t] += cnt[t + s]; mass[t] += mass[t + s]; }
        __syncthreads();
    }
    if (t == 0) {
        bsum[7 * blockIdx.x + 2] = cnt[0];
        bsum[7 * blockIdx.x + 3] = mass[0];
    }
}

__global__ __launch_bounds__(kStreamBlock) void k_center_count_halo(
    const HaloDev* __restrict__ halos, const double* __restrict__ bsum,
    sidm_center* __restrict__ out)
{
    __shared__ double cnt[kStreamBlock], mass[kStreamBlock];
    const HaloDev& H = halos[blockIdx.x];
    const int t = threadIdx.x;
    const int64_t nb = (H.n + kStreamBlock - 1) / kStreamBlock;
    double c = 0.0, w = 0.0;
    for (int64_t b = t; b < nb; b += kStreamBlock) {
        c += bsum[7 * (H.stream_block0 + b) + 2];
        w += bsum[7 * (H.stream_block0 + b) + 3];
    }
    cnt[t] = c;
    mass[t] = w;
    __syncthreads();
    for (int s = kStreamBlock / 2; s > 0; s >>= 1) {
        if (t < s) { cnt[t] += cnt[t + s]; mass[t] += mass[t + s]; }
        __syncthreads();
    }
    if (t == 0) {
        out[blockIdx.x].count = (int64_t)cnt[0];
        out[blockIdx.x].mass = mass[0];
    }
}

hipError_t launch_center(const StreamBlock* d_blocks, int64_t n_blocks, const HaloDev* d_halos,
                         int n_halos, const double* radius, const double* x, const double* y,
                         const double* z, const double* m, const double* pot, double* bsum,
                         sidm_center* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_center_block, dim3((unsigned)n_blocks), dim3(kStreamBlock), 0, st,
                       d_blocks, d_halos, x, y, z, pot, bsum);
    hipLaunchKernelGGL(k_center_halo, dim3(n_halos), dim3(kStreamBlock), 0, st, d_halos, bsum, x,
                       y, z, out);
    hipLaunchKernelGGL(k_center_count_block, dim3((unsigned)n_blocks), dim3(kStreamBlock), 0, st,
                       d_blocks, radius, x, y, z, m, out, bsum);
    hipLaunchKernelGGL(k_center_count_halo, dim3(n_halos), dim3(kStreamBlock), 0, st, d_halos,
                       bsum, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------- tidal radius
// Eq. tidal_radius: G M(<= r) / r^2 = |grad Phi_host(c + r n) - grad Phi_host(c - r n)|,
// bisection in log r.  Per-halo state in `tid` (8 doubles): n (3), lo, hi,
// the initial hi, mid.

// Per streaming block: the largest squared distance from the halo's centre.
__global__ __launch_bounds__(kStreamBlock) void k_tidal_extent(
    const StreamBlock* __restrict__ blocks, const double* __restrict__ x,
    const double* __restrict__ y, const double* __restrict__ z,
    const sidm_center* __restrict__ cen, double* __restrict__ bsum)
{
    __shared__ double red[kStreamBlock];
    const StreamBlock B = blocks[blockIdx.x];
    const sidm_center C = cen[B.halo];
    const int t = threadIdx.x;
    double v = 0.0;
    if (t < B.count && C.index >= 0) {
#pragma clang fp contract(off)
        const int64_t p = B.start + t;
        const double dx = x[p] - C.x, dy = y[p] - C.y, dz = z[p] - C.z;
        v = (dx * dx + dy * dy) + dz * dz;
    }
    red[t] = v;
    __syncthreads();
    for (int s = kStreamBlock / 2; s > 0; s >>= 1) {
        if (t < s) red[t] = fmax(red[t], red[t + s]);
        __syncthreads();
    }
    if (t == 0) bsum[7 * blockIdx.x + 4] = red[0];
}

// Per halo: the direction from the host centre and the initial bracket.
__global__ __launch_bounds__(kStreamBlock) void k_tidal_init(
    const HaloDev* __restrict__ halos, const double* __restrict__ bsum,
    const sidm_center* __restrict__ cen, double* __restrict__ tid)
{
    __shared__ double red[kStreamBlock];
    const HaloDev& H = halos[blockIdx.x];
    const int t = threadIdx.x;
    const int64_t nb = (H.n + kStreamBlock - 1) / kStreamBlock;
    double v = 0.0;
    for (int64_t b = t; b < nb; b += kStreamBlock) v = fmax(v, bsum[7 * (H.stream_block0 + b) + 4]);
    red[t] = v;
    __syncthreads();
    for (int s = kStreamBlock / 2; s > 0; s >>= 1) {
        if (t < s) red[t] = fmax(red[t], red[t + s]);
        __syncthreads();
    }
    if (t == 0) {
#pragma clang fp contract(off)
        const sidm_center C = cen[blockIdx.x];
        double* T = tid + 8 * blockIdx.x;
        const double ux = C.x - H.host_c[0], uy = C.y - H.host_c[1], uz = C.z - H.host_c[2];
        const double u = sqrt((ux * ux + uy * uy) + uz * uz);
        T[0] = u > 0.0 ? ux / u : 1.0;
        T[1] = u > 0.0 ? uy / u : 0.0;
        T[2] = u > 0.0 ? uz / u : 0.0;
        const double hi = 2.0 * sqrt(red[0]);
        T[4] = hi;
        T[3] = ldexp(hi, -40);
        T[5] = hi;
        T[6] = sqrt(T[3] * T[4]);
    }
}

// Per streaming block: mass within the radius r of the halo's centre, with
// r the current midpoint (tid[6]) or, with `final_pass`, the upper bracket.
__global__ __launch_bounds__(kStreamBlock) void k_tidal_mass(
    const StreamBlock* __restrict__ blocks, const double* __restrict__ x,
    const double* __restrict__ y, const double* __restrict__ z, const double* __restrict__ m,
    const sidm_center* __restrict__ cen, const double* __restrict__ tid, int final_pass,
    double* __restrict__ bsum)
{
    __shared__ double red[kStreamBlock];
    const StreamBlock B = blocks[blockIdx.x];
    const sidm_center C = cen[B.halo];
    const double r = tid[8 * B.halo + (final_pass ? 4 : 6)];
    const int t = threadIdx.x;
    double w = 0.0;
    if (t < B.count && C.index >= 0) {
#pragma clang fp contract(off)
        const int64_t p = B.start + t;
        const double dx = x[p] - C.x, dy = y[p] - C.y, dz = z[p] - C.z;
        if ((dx * dx + dy * dy) + dz * dz <= r * r) w = m[p];
    }
    red[t] = w;
    __syncthreads();
    for (int s = kStreamBlock / 2; s > 0; s >>= 1) {
        if (t < s) red[t] += red[t + s];
        __syncthreads();
    }
    if (t == 0) bsum[7 * blockIdx.x + 5] = red[0];
}

__device__ inline double halo_block_sum(const HaloDev& H, const double* bsum, int slot,
                                        double* red)
{
    const int t = threadIdx.x;
    const int64_t nb = (H.n + kStreamBlock - 1) / kStreamBlock;
    double v = 0.0;
    for (int64_t b = t; b < nb; b += kStreamBlock) v += bsum[7 * (H.stream_block0 + b) + slot];
    red[t] = v;
    __syncthreads();
    for (int s = kStreamBlock / 2; s > 0; s >>= 1) {
        if (t < s) red[t] += red[t + s];
        __syncthreads();
    }
    return red[0];
}

// One bisection step or the final record (thread 0 of the halo's block).
__device__ inline void tidal_update(const HaloDev& H, double M, const sidm_center C, double* T,
                                    int final_pass, sidm_tidal* o_ptr)
{
#pragma clang fp contract(off)
    if (final_pass) {
        sidm_tidal o;
        o.r_tidal = T[4];
        o.mass = M;
        o.x = C.x; o.y = C.y; o.z = C.z;
        o.index = C.index;
        o.status = T[4] == T[5] ? 1 : 0;
        o.reserved = 0;
        *o_ptr = o;
        return;
    }
    const double r = T[6];
    double ax1, ay1, az1, p1, ax2, ay2, az2, p2;
    host_field(H, C.x + r * T[0], C.y + r * T[1], C.z + r * T[2], ax1, ay1, az1, p1);
    host_field(H, C.x - r * T[0], C.y - r * T[1], C.z - r * T[2], ax2, ay2, az2, p2);
    const double gx = ax1 - ax2, gy = ay1 - ay2, gz = az1 - az2;
    const double tide = sqrt((gx * gx + gy * gy) + gz * gz);
    if (H.G * M / (r * r) > tide) T[3] = r;
    else T[4] = r;
    T[6] = sqrt(T[3] * T[4]);
}

// Per halo: one bisection step (self gravity at the midpoint against the
// host's tidal acceleration there), or the final record.
__global__ __launch_bounds__(kStreamBlock) void k_tidal_step(
    const HaloDev* __restrict__ halos, const double* __restrict__ bsum,
    const sidm_center* __restrict__ cen, double* __restrict__ tid, int final_pass,
    sidm_tidal* __restrict__ out)
{
    __shared__ double red[kStreamBlock];
    const HaloDev& H = halos[blockIdx.x];
    const double M = halo_block_sum(H, bsum, 5, red);
    if (threadIdx.x != 0) return;
    tidal_update(H, M, cen[blockIdx.x], tid + 8 * blockIdx.x, final_pass, out + blockIdx.x);
}

hipError_t launch_tidal(const StreamBlock* d_blocks, int64_t n_blocks, const HaloDev* d_halos,
                        int n_halos, const double* x, const double* y, const double* z,
                        const double* m, const double* pot, double* bsum, sidm_center* cen,
                        double* tid, sidm_tidal* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_center_block, dim3((unsigned)n_blocks), dim3(kStreamBlock), 0, st,
                       d_blocks, d_halos, x, y, z, pot, bsum);
    hipLaunchKernelGGL(k_center_halo, dim3(n_halos), dim3(kStreamBlock), 0, st, d_halos, bsum, x,
                       y, z, cen);
    hipLaunchKernelGGL(k_tidal_extent, dim3((unsigned)n_blocks), dim3(kStreamBlock), 0, st,
                       d_blocks, x, y, z, cen, bsum);
    hipLaunchKernelGGL(k_tidal_init, dim3(n_halos), dim3(kStreamBlock), 0, st, d_halos, bsum, cen,
                       tid);
    for (int it = 0; it <= 60; ++it) {
        const int fin = it == 60 ? 1 : 0;
        hipLaunchKernelGGL(k_tidal_mass, dim3((unsigned)n_blocks), dim3(kStreamBlock), 0, st,
                           d_blocks, x, y, z, m, cen, tid, fin, bsum);
        hipLaunchKernelGGL(k_tidal_step, dim3(n_halos), dim3(kStreamBlock), 0, st, d_halos, bsum,
                           cen, tid, fin, out);
    }
    return hipGetLastError();
}

}  // namespace sidm
