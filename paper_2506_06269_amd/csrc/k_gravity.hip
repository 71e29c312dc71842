// k_gravity.hip -- softened direct-sum self-gravity plus the static NFW host
// (Sec. 2: softening length eps; Sec. 4.1 Eq. nfw_potential).
//
// The sums run over the Morton-sorted order of the cell list, in tiles of
// kGravTileJ consecutive particles.  In the mixed form the frames are the
// compact sub-ranges of the cell list's 64-particle buckets; FP32 positions
// are stored relative to the FP64 centre of their frame, and an i-particle is
// moved into the frame of the j-particles once per frame (x_i - c_j computed as
// (x_i - c_i) - (c_j - c_i)),
// so close pairs subtract small local coordinates: FP32 position rounding is
// relative to the pair separation, not to the size of the halo.
//
// Work decomposition: a work item is (halo, i-block of kGravThreads * IREG
// particles, j-range).  Each thread keeps IREG i-particles in registers; the
// block stages a j-tile in LDS with one coalesced load per thread, and every
// lane of a wave reads the same j (LDS broadcast).  The pair terms of one tile
// are summed plainly and the tile sums are folded into Kahan-compensated
// accumulators, so the rounding error does not grow with N.  The self pair is
// skipped exactly in the few tiles that hold i.  Each item writes one FP64
// partial row per i; a finalize pass adds the rows of an i in a fixed order,
// scales by G, adds the host, optionally applies the closing half kick, and
// scatters to the caller's (unsorted) arrays.
#include "sidm_host.hpp"
#include "sidm_steps.hpp"
#include "sidm_plan.hpp"

namespace sidm {

// ---------------------------------------------------------------- masses, tiles
// Smallest and largest mass per streaming block, then per halo: cmass[h] is
// the common mass when all masses of the halo are equal (else 0), and
// cmass[n_halos + h] the largest mass.  With a
// status array, a halo that scatters (sigma_m > 0) without a common mass is
// flagged: the probability of a pair takes the mass of one member, which is
// only symmetric when the masses are equal (each run of the paper's Table 1
// has one particle mass), so such a halo is not scattered.
__global__ __launch_bounds__(kStreamBlock) void k_block_mass_range(
    const double* __restrict__ m, const StreamBlock* __restrict__ blocks, double* __restrict__ bsum)
{
    __shared__ double lo[kStreamBlock], hi[kStreamBlock];
    const StreamBlock B = blocks[blockIdx.x];
    const int t = threadIdx.x;
    const double mi = m[B.start + (t < B.count ? t : 0)];
    lo[t] = mi;
    hi[t] = mi;
    __syncthreads();
    for (int s = kStreamBlock / 2; s > 0; s >>= 1) {
        if (t < s) {
            lo[t] = fmin(lo[t], lo[t + s]);
            hi[t] = fmax(hi[t], hi[t + s]);
        }
        __syncthreads();
    }
    if (t == 0) {
        bsum[7 * (int64_t)blockIdx.x + 0] = lo[0];
        bsum[7 * (int64_t)blockIdx.x + 1] = hi[0];
    }
}

__global__ __launch_bounds__(kStreamBlock) void k_halo_mass(
    const HaloDev* __restrict__ halos, const double* __restrict__ bsum, double* __restrict__ cmass,
    int* __restrict__ status)
{
    __shared__ double lo[kStreamBlock], hi[kStreamBlock];
    const HaloDev& H = halos[blockIdx.x];
    const int t = threadIdx.x;
    const int64_t nb = (H.n + kStreamBlock - 1) / kStreamBlock;
    double l = INFINITY, u = -INFINITY;
    for (int64_t b = t; b < nb; b += kStreamBlock) {
        l = fmin(l, bsum[7 * (H.stream_block0 + b) + 0]);
        u = fmax(u, bsum[7 * (H.stream_block0 + b) + 1]);
    }
    lo[t] = l;
    hi[t] = u;
    __syncthreads();
    for (int s = kStreamBlock / 2; s > 0; s >>= 1) {
        if (t < s) {
            lo[t] = fmin(lo[t], lo[t + s]);
            hi[t] = fmax(hi[t], hi[t + s]);
        }
        __syncthreads();
    }
    if (t == 0) {
        const bool equal = lo[0] == hi[0];
        cmass[blockIdx.x] = equal ? lo[0] : 0.0;
        cmass[gridDim.x + blockIdx.x] = hi[0];   // the largest mass
        if (status && !equal && H.sigma_m > 0.0)
            atomicOr(&status[blockIdx.x], SIDM_DEV_UNEQUAL_MASS);
    }
}

// Frame of a sorted position: the compact sub-range of its bucket that holds
// it; its centre is the midpoint of the sub-range's box.
__device__ inline void frame_of(const HaloDev& H, const SubRange* __restrict__ sub,
                                const int* __restrict__ sub_n, int64_t local, double* c)
{
    const int64_t b = H.level_off[0] + local / kBucket;
    const int o = (int)(local % kBucket);
    const int ns = sub_n[b];
    int f = 0;
    while (f + 1 < ns && o >= sub[kSubMax * b + f + 1].off) ++f;
    const double* bx = sub[kSubMax * b + f].box;
    c[0] = 0.5 * (bx[0] + bx[3]);
    c[1] = 0.5 * (bx[1] + bx[4]);
    c[2] = 0.5 * (bx[2] + bx[5]);
}

// FP32 positions relative to the centre of their frame, and the mass.
__global__ __launch_bounds__(kStreamBlock) void k_pack_frames(
    const double* __restrict__ sx, const double* __restrict__ sy, const double* __restrict__ sz,
    const double* __restrict__ sm, const StreamBlock* __restrict__ blocks,
    const HaloDev* __restrict__ halos, const SubRange* __restrict__ sub,
    const int* __restrict__ sub_n, float4* __restrict__ xm32)
{
    const StreamBlock B = blocks[blockIdx.x];
    const int t = threadIdx.x;
    if (t >= B.count) return;
    const HaloDev& H = halos[B.halo];
    const int64_t local = (B.start - H.offset) + t;
    const int64_t p = H.sbase + local;
    double c[3];
    frame_of(H, sub, sub_n, local, c);
    xm32[p] = make_float4((float)(sx[p] - c[0]), (float)(sy[p] - c[1]), (float)(sz[p] - c[2]),
                          (float)sm[p]);
}

// ---------------------------------------------------------------- FP32 tiles
// Sums of the pair terms of one LDS tile for IREG i-particles.  With EQM (all
// masses of the halo equal) the mass is factored out of the sums and applied
// once per partial row: one multiply fewer per interaction.  DIAG tiles hold
// some of the block's own i and skip j == i exactly.
template <int IREG, int NT, bool EQM, bool DIAG, int UNROLL = 4>
__device__ inline void tile_f32(const float4* __restrict__ tile, int ja, int jb, const float* xi,
                                const float* yi, const float* zi, float eps2, int64_t j0, int64_t i0,
                                int t, float* px, float* py, float* pz, float* pp)
{
#pragma unroll UNROLL
    for (int jj = ja; jj < jb; ++jj) {
        const float4 q = tile[jj];
#pragma unroll
        for (int r = 0; r < IREG; ++r) {
            const float dx = q.x - xi[r];
            const float dy = q.y - yi[r];
            const float dz = q.z - zi[r];
            const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2)));
            float rinv = __builtin_amdgcn_rsqf(r2);
            if (DIAG && j0 + jj == i0 + (int64_t)r * NT + t) rinv = 0.f;
            if (EQM) {
                const float rinv3 = rinv * (rinv * rinv);
                px[r] = fmaf(rinv3, dx, px[r]);
                py[r] = fmaf(rinv3, dy, py[r]);
                pz[r] = fmaf(rinv3, dz, pz[r]);
                pp[r] += rinv;
            } else {
                const float mr = q.w * rinv;
                const float mr3 = mr * (rinv * rinv);
                px[r] = fmaf(mr3, dx, px[r]);
                py[r] = fmaf(mr3, dy, py[r]);
                pz[r] = fmaf(mr3, dz, pz[r]);
                pp[r] += mr;
            }
        }
    }
}

template <int IREG, int NT, bool EQM>
__device__ inline void grav_mixed_body(const float4* __restrict__ xm32,
                                       const SubRange* __restrict__ sub,
                                       const int* __restrict__ sub_n, const GravItem& it,
                                       const HaloDev& H, double mscale,
                                       double4* __restrict__ partial, float4* tile, int64_t pbase)
{
    const int t = threadIdx.x;
    const float eps2 = (float)H.eps2;
    const int64_t il0 = it.i0 - H.offset;   // local (sorted) index of the i-block

    float xi[IREG], yi[IREG], zi[IREG];
    double cix[IREG], ciy[IREG], ciz[IREG];          // centre of each i's frame
    float sx[IREG], sy[IREG], sz[IREG], sp[IREG];     // Kahan sums
    float cx[IREG], cy[IREG], cz[IREG], cp[IREG];     // Kahan compensations
#pragma unroll
    for (int r = 0; r < IREG; ++r) {
        const int64_t li = il0 + (int64_t)r * NT + t;
        float4 p = make_float4(0.f, 0.f, 0.f, 0.f);
        cix[r] = ciy[r] = ciz[r] = 0.0;
        if (li < H.n) {
            p = xm32[H.sbase + li];
            double c[3];
            frame_of(H, sub, sub_n, li, c);
            cix[r] = c[0]; ciy[r] = c[1]; ciz[r] = c[2];
        }
        xi[r] = p.x; yi[r] = p.y; zi[r] = p.z;
        sx[r] = sy[r] = sz[r] = sp[r] = 0.f;
        cx[r] = cy[r] = cz[r] = cp[r] = 0.f;
    }
    const int64_t last_bucket = H.level_off[0] + H.level_n[0] - 1;
    for (int64_t j0 = it.j0; j0 < it.j1; j0 += NT) {
        const int64_t lj0 = j0 - H.offset;
        float4 pj = make_float4(0.f, 0.f, 0.f, 0.f);
        if (j0 + t < it.j1) pj = xm32[H.sbase + lj0 + t];
        __syncthreads();
        tile[t] = pj;
        __syncthreads();
        float px[IREG], py[IREG], pz[IREG], pp[IREG];
#pragma unroll
        for (int r = 0; r < IREG; ++r) px[r] = py[r] = pz[r] = pp[r] = 0.f;
        const bool diag = j0 < it.i0 + (int64_t)IREG * NT && j0 + NT > it.i0;
        // the tile's buckets and their compact sub-ranges are the frames
        const int64_t b0 = H.level_off[0] + lj0 / kBucket;
        for (int64_t b = b0; b < b0 + NT / kBucket && b <= last_bucket; ++b) {
            const int ns = sub_n[b];
            const int base = (int)((b - b0) * kBucket);
            for (int f = 0; f < ns; ++f) {
                const SubRange& R = sub[kSubMax * b + f];
                const double fx = 0.5 * (R.box[0] + R.box[3]);
                const double fy = 0.5 * (R.box[1] + R.box[4]);
                const double fz = 0.5 * (R.box[2] + R.box[5]);
                // i-positions in the frame of these j
                float qx[IREG], qy[IREG], qz[IREG];
#pragma unroll
                for (int r = 0; r < IREG; ++r) {
                    qx[r] = xi[r] - (float)(fx - cix[r]);
                    qy[r] = yi[r] - (float)(fy - ciy[r]);
                    qz[r] = zi[r] - (float)(fz - ciz[r]);
                }
                const int ja = base + R.off, jb = base + R.off + R.cnt;
                if (diag)
                    tile_f32<IREG, NT, EQM, true>(tile, ja, jb, qx, qy, qz, eps2, j0, it.i0, t, px, py,
                                              pz, pp);
                else
                    tile_f32<IREG, NT, EQM, false>(tile, ja, jb, qx, qy, qz, eps2, j0, it.i0, t, px,
                                               py, pz, pp);
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
        const int64_t li = il0 + (int64_t)r * NT + t;
        if (li >= H.n) continue;
        const int64_t row = pbase + (int64_t)it.slot * H.n + li;
        // the compensation holds the negated lost low part
        partial[row] = make_double4(mscale * ((double)sx[r] - (double)cx[r]),
                                    mscale * ((double)sy[r] - (double)cy[r]),
                                    mscale * ((double)sz[r] - (double)cz[r]),
                                    mscale * ((double)sp[r] - (double)cp[r]));
    }
}

// Block time steps: whether any i-particle of the item is active at this tick
// (tick 0: not a cycle, every item runs).  Uniform over the block.
template <int IREG, int NT>
__device__ inline bool item_active(const GravItem& it, const HaloDev& H,
                                   const int8_t* __restrict__ bin,
                                   const uint32_t* __restrict__ perm, int tick, int bmax)
{
    if (tick == 0) return true;
    const int kl = local_tick(H, tick, bmax);
    int any = 0;
    if (kl > 0) {
        const int64_t il0 = it.i0 - H.offset;
#pragma unroll
        for (int r = 0; r < IREG; ++r) {
            const int64_t li = il0 + (int64_t)r * NT + threadIdx.x;
            if (li < H.n && bin_active(H, bin[perm[H.sbase + li]], kl)) any = 1;
        }
    }
    return __syncthreads_or(any) != 0;
}

// Work items in a plain launch take item blockIdx.x; a persistent launch
// (PERSIST) runs as many blocks as the device holds at once, and each takes
// items from a ticket counter until none is left (every block leaves the loop
// when the counter passes n_items; no block waits on another).
template <int IREG, int NT, bool PERSIST>
__global__ __launch_bounds__(NT) void k_grav_mixed(
    const float4* __restrict__ xm32, const SubRange* __restrict__ sub,
    const int* __restrict__ sub_n, const GravItem* __restrict__ items, int64_t n_items,
    unsigned long long* __restrict__ ticket, const HaloDev* __restrict__ halos,
    const double* __restrict__ cmass, double4* __restrict__ partial,
    const int8_t* __restrict__ bin, const uint32_t* __restrict__ perm, int tick, int bmax,
    int tick_rows)
{
    __shared__ float4 tile[NT];
    __shared__ int64_t next;
    int64_t k = blockIdx.x;
    for (;;) {
        if (PERSIST) {
            __syncthreads();   // every thread has read the previous `next`
            if (threadIdx.x == 0) next = (int64_t)atomicAdd(ticket, 1ull);
            __syncthreads();
            k = next;
            if (k >= n_items) return;
        }
        const GravItem it = items[k];
        const HaloDev& H = halos[it.halo];
        if (item_active<IREG, NT>(it, H, bin, perm, tick, bmax)) {
            // the items of a block-step tick (tick_rows) write their own partial rows
            const int64_t pbase = tick_rows ? H.tick_part_base : H.part_base;
            const double meq = cmass[it.halo];
            if (meq > 0.0)
                grav_mixed_body<IREG, NT, true>(xm32, sub, sub_n, it, H, meq, partial, tile,
                                                pbase);
            else
                grav_mixed_body<IREG, NT, false>(xm32, sub, sub_n, it, H, 1.0, partial, tile,
                                                 pbase);
        }
        if (!PERSIST) return;
    }
}

// ---------------------------------------------------------------- symmetric tiles
// Mixed precision with each unordered pair evaluated once (the force on j is
// minus the force on i): the i-side sums as in the one-sided tiles, and the
// reaction on each j of a tile summed over the 64 lanes of a wave in
// registers, over the block's waves through LDS in a fixed order, and over
// work items in 64-bit fixed point with integer atomics, whose total does not
// depend on the order in which they land (the result is deterministic).  A
// work item is an i-block of IREG * NT particles against a j-range at or
// after it; the tiles inside the i-block itself are summed one-sided.  The
// launch shapes are those of the one-sided tiles (always persistent).

// Fixed-point scales of a halo's sums: a pair's acceleration term is at most
// 2/(3 sqrt 3) / eps^2 and its potential term 1/eps (times the largest mass
// unless the masses are factored out), so no partial sum of n terms exceeds
// 2^61 after scaling.
__device__ inline void sym_scales(const HaloDev& H, double mref, double& sa, double& sp)
{
    const double n = (double)H.n * mref;
    const double ba = n * (0.38490017945975050 * 1.01) / H.eps2;
    const double bp = n * 1.01 / H.eps;
    sa = ldexp(1.0, 60 - ilogb(ba));
    sp = ldexp(1.0, 60 - ilogb(bp));
}

// Lanes 0-31 return a[l] + a[l + 32], lanes 32-63 b[l - 32] + b[l].
__device__ inline float swap32_add(float a, float b)
{
    const auto r =
        __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// In each half of the wave: rows 0 and 2 of the result are a's rows (0 + 1)
// and (2 + 3), rows 1 and 3 are b's (rows of 16 lanes).
__device__ inline float swap16_add(float a, float b)
{
    const auto r =
        __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// a plus a rotated by CTRL within each row of 16 lanes (DPP row_ror)
template <int CTRL>
__device__ inline float row_ror_add(float a)
{
    return a + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(a), CTRL, 0xF, 0xF,
                                                          false));
}

// Component whose wave total row q holds after wave_sum: x, z, y, phi.
__device__ inline int sym_row_comp(int row) { return ((row & 1) << 1) | (row >> 1); }

// v[4 g + c] (slot g < JG; c = x, y, z, phi) summed over the wave's 64 lanes:
// on return x[g] holds, on every lane of row q (lanes 16q .. 16q + 15), the
// total of component sym_row_comp(q) of slot g.  Two halving exchanges leave
// each row one value per slot; rotations sum each row.
template <int JG>
__device__ inline void wave_sum(const float (&v)[4 * JG], float (&x)[JG])
{
    float w[2 * JG];
#pragma unroll
    for (int p = 0; p < 2 * JG; ++p) w[p] = swap32_add(v[2 * p], v[2 * p + 1]);
#pragma unroll
    for (int g = 0; g < JG; ++g) {
        float u = swap16_add(w[2 * g], w[2 * g + 1]);
        u = row_ror_add<0x128>(u);   // row_ror:8
        u = row_ror_add<0x124>(u);   // row_ror:4
        u = row_ror_add<0x122>(u);   // row_ror:2
        x[g] = row_ror_add<0x121>(u);   // row_ror:1
    }
}

// The pairs of the i-particles (in the frame of these j) with the j in
// [ja, jb) of the tile: i-side sums into px..pp, and each j's reaction (the
// sums with the sign of the i-side; the caller negates the acceleration)
// summed over the wave into jp[j][c].  EQM: masses factored out; else mi are
// the i masses and the tile's w the j masses.
template <int IREG, int JG, bool EQM>
__device__ inline void tile_sym(const float4* __restrict__ tile, int ja, int jb, const float* qx,
                                const float* qy, const float* qz, const float* mi, float eps2,
                                float* px, float* py, float* pz, float* pp, float (*jp)[4],
                                int lane)
{
    const int rl = lane & 15, comp = sym_row_comp(lane >> 4);
    for (int g = ja; g < jb; g += JG) {
        float v[4 * JG];
#pragma unroll
        for (int q = 0; q < JG; ++q) {
            float rx = 0.f, ry = 0.f, rz = 0.f, rp = 0.f;
            if (g + q < jb) {   // uniform over the wave
                const float4 p = tile[g + q];
#pragma unroll
                for (int r = 0; r < IREG; ++r) {
                    const float dx = p.x - qx[r];
                    const float dy = p.y - qy[r];
                    const float dz = p.z - qz[r];
                    const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2)));
                    const float rinv = __builtin_amdgcn_rsqf(r2);
                    const float w = rinv * (rinv * rinv);
                    if (EQM) {
                        px[r] = fmaf(w, dx, px[r]);
                        py[r] = fmaf(w, dy, py[r]);
                        pz[r] = fmaf(w, dz, pz[r]);
                        pp[r] += rinv;
                        rx = fmaf(w, dx, rx);
                        ry = fmaf(w, dy, ry);
                        rz = fmaf(w, dz, rz);
                        rp += rinv;
                    } else {
                        const float wj = p.w * w, wi = mi[r] * w;
                        px[r] = fmaf(wj, dx, px[r]);
                        py[r] = fmaf(wj, dy, py[r]);
                        pz[r] = fmaf(wj, dz, pz[r]);
                        pp[r] = fmaf(p.w, rinv, pp[r]);
                        rx = fmaf(wi, dx, rx);
                        ry = fmaf(wi, dy, ry);
                        rz = fmaf(wi, dz, rz);
                        rp = fmaf(mi[r], rinv, rp);
                    }
                }
            }
            v[4 * q + 0] = rx;
            v[4 * q + 1] = ry;
            v[4 * q + 2] = rz;
            v[4 * q + 3] = rp;
        }
        float x[JG];
        wave_sum<JG>(v, x);
        if (rl < JG && g + rl < jb) {
            float val = x[0];
#pragma unroll
            for (int q = 1; q < JG; ++q)
                if (rl == q) val = x[q];
            jp[g + rl][comp] = val;
        }
    }
}

// The same with one j per wave sum, software-pipelined: the wave sum of the
// previous j's reaction is formed while the pairs of the next j are evaluated
// (the two are independent, so their instructions interleave).
template <int IREG, bool EQM>
__device__ inline void tile_sym1(const float4* __restrict__ tile, int ja, int jb, const float* qx,
                                 const float* qy, const float* qz, const float* mi, float eps2,
                                 float* px, float* py, float* pz, float* pp, float (*jp)[4],
                                 int lane)
{
    if (ja >= jb) return;
    const int rl = lane & 15, comp = sym_row_comp(lane >> 4);
    auto pairs = [&](int j, float (&v)[4]) {
        const float4 p = tile[j];
        float rx = 0.f, ry = 0.f, rz = 0.f, rp = 0.f;
#pragma unroll
        for (int r = 0; r < IREG; ++r) {
            const float dx = p.x - qx[r];
            const float dy = p.y - qy[r];
            const float dz = p.z - qz[r];
            const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2)));
            const float rinv = __builtin_amdgcn_rsqf(r2);
            const float w = rinv * (rinv * rinv);
            if (EQM) {
                px[r] = fmaf(w, dx, px[r]);
                py[r] = fmaf(w, dy, py[r]);
                pz[r] = fmaf(w, dz, pz[r]);
                pp[r] += rinv;
                rx = fmaf(w, dx, rx);
                ry = fmaf(w, dy, ry);
                rz = fmaf(w, dz, rz);
                rp += rinv;
            } else {
                const float wj = p.w * w, wi = mi[r] * w;
                px[r] = fmaf(wj, dx, px[r]);
                py[r] = fmaf(wj, dy, py[r]);
                pz[r] = fmaf(wj, dz, pz[r]);
                pp[r] = fmaf(p.w, rinv, pp[r]);
                rx = fmaf(wi, dx, rx);
                ry = fmaf(wi, dy, ry);
                rz = fmaf(wi, dz, rz);
                rp = fmaf(mi[r], rinv, rp);
            }
        }
        v[0] = rx;
        v[1] = ry;
        v[2] = rz;
        v[3] = rp;
    };
    auto finish = [&](int j, const float (&v)[4]) {
        float x[1];
        wave_sum<1>(v, x);
        if (rl == 0) jp[j][comp] = x[0];
    };
    float prev[4];
    pairs(ja, prev);
    for (int j = ja + 1; j < jb; ++j) {
        float cur[4];
        pairs(j, cur);
        finish(j - 1, prev);
#pragma unroll
        for (int c = 0; c < 4; ++c) prev[c] = cur[c];
    }
    finish(jb - 1, prev);
}

template <int IREG, int NT>
struct SymLds {
    float4 tile[NT];
    float jpart[NT / 64][NT][4];
    double ctab[(IREG * NT / kBucket) * kSubMax][3];   // frame centres of the i-block
    int64_t next;
};

template <int IREG, int NT, int JG, bool EQM>
__device__ inline void grav_sym_body(const float4* __restrict__ xm32,
                                     const SubRange* __restrict__ sub,
                                     const int* __restrict__ sub_n, const SymItem& it,
                                     const HaloDev& H, double mref,
                                     unsigned long long* __restrict__ acc, SymLds<IREG, NT>& L)
{
    constexpr int NW = NT / 64;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const float eps2 = (float)H.eps2;
    const int64_t il0 = it.i0 - H.offset;        // local (sorted) index of the i-block
    const int64_t ib0 = H.level_off[0] + il0 / kBucket;   // its first bucket
    const int64_t last_bucket = H.level_off[0] + H.level_n[0] - 1;
    double sa, sp;
    sym_scales(H, mref, sa, sp);

    // frame centres of the i-block's buckets
    __syncthreads();   // the previous item's readers of ctab are done
    for (int e = t; e < (IREG * NT / kBucket) * kSubMax; e += NT) {
        const int64_t b = ib0 + e / kSubMax;
        const int f = e % kSubMax;
        if (b <= last_bucket && f < sub_n[b]) {
            const double* bx = sub[kSubMax * b + f].box;
            L.ctab[e][0] = 0.5 * (bx[0] + bx[3]);
            L.ctab[e][1] = 0.5 * (bx[1] + bx[4]);
            L.ctab[e][2] = 0.5 * (bx[2] + bx[5]);
        }
    }
    float xi[IREG], yi[IREG], zi[IREG], mi[IREG];
    int fid[IREG];
#pragma unroll
    for (int r = 0; r < IREG; ++r) {
        const int64_t li = il0 + (int64_t)r * NT + t;
        float4 p = make_float4(0.f, 0.f, 0.f, 0.f);
        fid[r] = 0;
        if (li < H.n) {
            p = xm32[H.sbase + li];
            const int64_t b = H.level_off[0] + li / kBucket;
            const int o = (int)(li % kBucket);
            const int ns = sub_n[b];
            int f = 0;
            while (f + 1 < ns && o >= sub[kSubMax * b + f + 1].off) ++f;
            fid[r] = (int)(b - ib0) * kSubMax + f;
        }
        xi[r] = p.x; yi[r] = p.y; zi[r] = p.z; mi[r] = p.w;
    }
    __syncthreads();
    float px[IREG], py[IREG], pz[IREG], pp[IREG];
#pragma unroll
    for (int r = 0; r < IREG; ++r) px[r] = py[r] = pz[r] = pp[r] = 0.f;
    int tiles = 0;
    for (int64_t j0 = it.j0; j0 < it.j1; j0 += NT) {
        const int64_t lj0 = j0 - H.offset;
        float4 pj = make_float4(0.f, 0.f, 0.f, 0.f);
        if (j0 + t < it.j1) pj = xm32[H.sbase + lj0 + t];
        __syncthreads();
        L.tile[t] = pj;
        __syncthreads();
        const bool diag = j0 < it.i0 + (int64_t)IREG * NT;   // inside the i-block
        const int64_t b0 = H.level_off[0] + lj0 / kBucket;
        for (int64_t b = b0; b < b0 + NT / kBucket && b <= last_bucket; ++b) {
            const int ns = sub_n[b];
            const int base = (int)((b - b0) * kBucket);
            for (int f = 0; f < ns; ++f) {
                const SubRange& R = sub[kSubMax * b + f];
                const double fx = 0.5 * (R.box[0] + R.box[3]);
                const double fy = 0.5 * (R.box[1] + R.box[4]);
                const double fz = 0.5 * (R.box[2] + R.box[5]);
                float qx[IREG], qy[IREG], qz[IREG];
#pragma unroll
                for (int r = 0; r < IREG; ++r) {
                    const double* c = L.ctab[fid[r]];
                    qx[r] = xi[r] - (float)(fx - c[0]);
                    qy[r] = yi[r] - (float)(fy - c[1]);
                    qz[r] = zi[r] - (float)(fz - c[2]);
                }
                const int ja = base + R.off, jb = base + R.off + R.cnt;
                if (diag)
                    tile_f32<IREG, NT, EQM, true, 1>(L.tile, ja, jb, qx, qy, qz, eps2, j0, it.i0,
                                                     t, px, py, pz, pp);
                else if (JG == 1)
                    tile_sym1<IREG, EQM>(L.tile, ja, jb, qx, qy, qz, mi, eps2, px, py, pz, pp,
                                         L.jpart[wave], lane);
                else
                    tile_sym<IREG, JG, EQM>(L.tile, ja, jb, qx, qy, qz, mi, eps2, px, py, pz, pp,
                                            L.jpart[wave], lane);
            }
        }
        // the i-side sums of kSymFold tiles (and of the item's last) into the
        // fixed-point totals: exact integer sums of FP32 sums over a few
        // hundred j, as the one-sided tiles fold theirs
        if (++tiles == kSymFold || j0 + NT >= it.j1) {
            tiles = 0;
#pragma unroll
            for (int r = 0; r < IREG; ++r) {
                const int64_t li = il0 + (int64_t)r * NT + t;
                if (li < H.n) {
                    unsigned long long* a = acc + 4 * (H.sbase + li);
                    atomicAdd(a + 0, (unsigned long long)llrint((double)px[r] * sa));
                    atomicAdd(a + 1, (unsigned long long)llrint((double)py[r] * sa));
                    atomicAdd(a + 2, (unsigned long long)llrint((double)pz[r] * sa));
                    atomicAdd(a + 3, (unsigned long long)llrint((double)pp[r] * sp));
                }
                px[r] = py[r] = pz[r] = pp[r] = 0.f;
            }
        }
        if (!diag) {
            // the reaction on the tile's j: the waves' sums in a fixed order,
            // negated for the acceleration, into the fixed-point totals
            __syncthreads();
            if (j0 + t < it.j1) {
                double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
                for (int w = 0; w < NW; ++w) {
                    s0 += (double)L.jpart[w][t][0];
                    s1 += (double)L.jpart[w][t][1];
                    s2 += (double)L.jpart[w][t][2];
                    s3 += (double)L.jpart[w][t][3];
                }
                unsigned long long* a = acc + 4 * (H.sbase + lj0 + t);
                atomicAdd(a + 0, (unsigned long long)llrint(-s0 * sa));
                atomicAdd(a + 1, (unsigned long long)llrint(-s1 * sa));
                atomicAdd(a + 2, (unsigned long long)llrint(-s2 * sa));
                atomicAdd(a + 3, (unsigned long long)llrint(s3 * sp));
            }
        }
    }
}

// Persistent: as many blocks as the device holds; each takes items from a
// ticket counter until none is left.  The fixed-point totals (4 per sorted
// particle) start at zero.  EQM: the items of halos with one common mass
// (masses factored out); the other instantiation takes the rest.  Both run,
// each skipping the other's items.  At least kSymWaves waves per SIMD: the
// compiler keeps 128 registers and moves the values used once per frame
// (positions, frame indices) to scratch, which left the pair loop intact and
// was faster than fewer waves with everything in registers.
template <int IREG, int NT, int JG, bool EQM>
__global__ __launch_bounds__(NT, kSymWaves) void k_grav_sym(
    const float4* __restrict__ xm32, const SubRange* __restrict__ sub,
    const int* __restrict__ sub_n, const SymItem* __restrict__ items, int64_t n_items,
    unsigned long long* __restrict__ ticket, const HaloDev* __restrict__ halos,
    const double* __restrict__ cmass, int n_halos, unsigned long long* __restrict__ acc)
{
    __shared__ SymLds<IREG, NT> L;
    for (;;) {
        __syncthreads();   // every thread has read the previous `next`
        if (threadIdx.x == 0) L.next = (int64_t)atomicAdd(ticket, 1ull);
        __syncthreads();
        const int64_t k = L.next;
        if (k >= n_items) return;
        const SymItem it = items[k];
        const HaloDev& H = halos[it.halo];
        const double meq = cmass[it.halo];
        if ((meq > 0.0) != EQM) continue;   // uniform: the other kernel's item
        grav_sym_body<IREG, NT, JG, EQM>(xm32, sub, sub_n, it, H,
                                         EQM ? 1.0 : cmass[n_halos + it.halo], acc, L);
    }
}

// Zero fixed-point totals of the particles of halos that take the symmetric tiles.
__global__ __launch_bounds__(kStreamBlock) void k_sym_zero(const StreamBlock* __restrict__ blocks,
                                                           const HaloDev* __restrict__ halos,
                                                           unsigned long long* __restrict__ acc)
{
    const StreamBlock B = blocks[blockIdx.x];
    const int t = threadIdx.x;
    const HaloDev& H = halos[B.halo];
    if (t >= B.count || !H.grav_sym) return;
    const int64_t p = H.sbase + (B.start - H.offset) + t;
    acc[4 * p + 0] = 0ull;
    acc[4 * p + 1] = 0ull;
    acc[4 * p + 2] = 0ull;
    acc[4 * p + 3] = 0ull;
}

// ---------------------------------------------------------------- FP64 tiles
// Pair terms of one LDS tile for IREG i-particles in FP64 (see tile_f32).
template <int IREG, int NT, bool EQM, bool DIAG>
__device__ inline void tile_f64(const double4* __restrict__ tile, const double* xi,
                                const double* yi, const double* zi, double eps2, int64_t j0,
                                int64_t i0, int t, double* px, double* py, double* pz, double* pp)
{
#pragma unroll 2
    for (int jj = 0; jj < NT; ++jj) {
        const double4 q = tile[jj];
#pragma unroll
        for (int r = 0; r < IREG; ++r) {
            const double dx = q.x - xi[r];
            const double dy = q.y - yi[r];
            const double dz = q.z - zi[r];
            const double r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, eps2)));
            double rinv = rsqrt_pos(r2);
            if (DIAG && j0 + jj == i0 + (int64_t)r * NT + t) rinv = 0.0;
            if (EQM) {
                const double rinv3 = rinv * (rinv * rinv);
                px[r] = fma(rinv3, dx, px[r]);
                py[r] = fma(rinv3, dy, py[r]);
                pz[r] = fma(rinv3, dz, pz[r]);
                pp[r] += rinv;
            } else {
                const double mr = q.w * rinv;
                const double mr3 = mr * (rinv * rinv);
                px[r] = fma(mr3, dx, px[r]);
                py[r] = fma(mr3, dy, py[r]);
                pz[r] = fma(mr3, dz, pz[r]);
                pp[r] += mr;
            }
        }
    }
}

template <int IREG, int NT, bool EQM>
__device__ inline void grav_fp64_body(const double* __restrict__ x, const double* __restrict__ y,
                                      const double* __restrict__ z, const double* __restrict__ m,
                                      const GravItem& it, const HaloDev& H, double mscale,
                                      double4* __restrict__ partial, double4* tile, int64_t pbase)
{
    const int t = threadIdx.x;
    const double eps2 = H.eps2;
    const int64_t il0 = it.i0 - H.offset;

    double xi[IREG], yi[IREG], zi[IREG];
    double sx[IREG], sy[IREG], sz[IREG], sp[IREG];
    double cx[IREG], cy[IREG], cz[IREG], cp[IREG];
#pragma unroll
    for (int r = 0; r < IREG; ++r) {
        const int64_t li = il0 + (int64_t)r * NT + t;
        xi[r] = yi[r] = zi[r] = 0.0;
        if (li < H.n) {
            const int64_t p = H.sbase + li;
            xi[r] = x[p]; yi[r] = y[p]; zi[r] = z[p];
        }
        sx[r] = sy[r] = sz[r] = sp[r] = 0.0;
        cx[r] = cy[r] = cz[r] = cp[r] = 0.0;
    }
    for (int64_t j0 = it.j0; j0 < it.j1; j0 += NT) {
        // padding: r2 ~ 1e300 stays finite, r^-3 underflows to 0 and r^-1 ~ 1e-150
        // cannot change a potential sum
        double4 pj = make_double4(1.0e150, 1.0e150, 1.0e150, 0.0);
        if (j0 + t < it.j1) {
            const int64_t p = H.sbase + (j0 - H.offset) + t;
            pj = make_double4(x[p], y[p], z[p], m[p]);
        }
        __syncthreads();
        tile[t] = pj;
        __syncthreads();
        double px[IREG], py[IREG], pz[IREG], pp[IREG];
#pragma unroll
        for (int r = 0; r < IREG; ++r) px[r] = py[r] = pz[r] = pp[r] = 0.0;
        const bool diag = j0 < it.i0 + (int64_t)IREG * NT && j0 + NT > it.i0;
        if (diag)
            tile_f64<IREG, NT, EQM, true>(tile, xi, yi, zi, eps2, j0, it.i0, t, px, py, pz, pp);
        else
            tile_f64<IREG, NT, EQM, false>(tile, xi, yi, zi, eps2, j0, it.i0, t, px, py, pz, pp);
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
        const int64_t li = il0 + (int64_t)r * NT + t;
        if (li >= H.n) continue;
        const int64_t row = pbase + (int64_t)it.slot * H.n + li;
        partial[row] = make_double4(mscale * (sx[r] - cx[r]), mscale * (sy[r] - cy[r]),
                                    mscale * (sz[r] - cz[r]), mscale * (sp[r] - cp[r]));
    }
}

template <int IREG, int NT, bool PERSIST>
__global__ __launch_bounds__(NT) void k_grav_fp64(
    const double* __restrict__ x, const double* __restrict__ y, const double* __restrict__ z,
    const double* __restrict__ m, const GravItem* __restrict__ items, int64_t n_items,
    unsigned long long* __restrict__ ticket, const HaloDev* __restrict__ halos,
    const double* __restrict__ cmass, double4* __restrict__ partial,
    const int8_t* __restrict__ bin, const uint32_t* __restrict__ perm, int tick, int bmax,
    int tick_rows)
{
    __shared__ double4 tile[NT];
    __shared__ int64_t next;
    int64_t k = blockIdx.x;
    for (;;) {
        if (PERSIST) {
            __syncthreads();
            if (threadIdx.x == 0) next = (int64_t)atomicAdd(ticket, 1ull);
            __syncthreads();
            k = next;
            if (k >= n_items) return;
        }
        const GravItem it = items[k];
        const HaloDev& H = halos[it.halo];
        if (item_active<IREG, NT>(it, H, bin, perm, tick, bmax)) {
            const int64_t pbase = tick_rows ? H.tick_part_base : H.part_base;
            const double meq = cmass[it.halo];
            if (meq > 0.0)
                grav_fp64_body<IREG, NT, true>(x, y, z, m, it, H, meq, partial, tile, pbase);
            else
                grav_fp64_body<IREG, NT, false>(x, y, z, m, it, H, 1.0, partial, tile, pbase);
        }
        if (!PERSIST) return;
    }
}

// ---------------------------------------------------------------- host + finalize
// Sums the partial rows of each i in slot order (or takes the fixed-point
// totals of the symmetric tiles, symacc given), scales by G, adds the host,
// optionally kicks v by a * dt/2 (and refreshes the sorted copy of v that the
// scattering pass reads), and writes to the caller's particle order.  In a
// cycle of block steps (tick > 0) only the particles active at the tick are
// written: closing half kick with the old step, then (before the cycle's
// end) the new bin, lengthened only to a step the tick is a multiple of, and
// the opening half kick with it.
__global__ __launch_bounds__(kStreamBlock) void k_grav_finalize(
    const StreamBlock* __restrict__ blocks, const HaloDev* __restrict__ halos,
    const double4* __restrict__ partial, const uint32_t* __restrict__ perm,
    const double* __restrict__ x, const double* __restrict__ y, const double* __restrict__ z,
    double* __restrict__ ax, double* __restrict__ ay, double* __restrict__ az,
    double* __restrict__ pot, double* __restrict__ vx, double* __restrict__ vy,
    double* __restrict__ vz, double* __restrict__ svx, double* __restrict__ svy,
    double* __restrict__ svz, int kick, int8_t* __restrict__ bin, int tick, int bmax,
    const double4* __restrict__ partial_tick, const unsigned long long* __restrict__ symacc,
    const double* __restrict__ cmass, int n_halos)
{
#pragma clang fp contract(off)
    const StreamBlock B = blocks[blockIdx.x];
    const int t = threadIdx.x;
    if (t >= B.count) return;
    const HaloDev& H = halos[B.halo];
    const int64_t li = (B.start - H.offset) + t;
    const int64_t p = H.sbase + li;
    const int64_t o = perm[p];
    int kl = 0, b = 0;
    if (tick > 0) {
        kl = local_tick(H, tick, bmax);
        b = bin[o];
        if (!bin_active(H, b, kl)) return;
    }
    // a tick of block steps (partial_tick given) keeps the rows of direct-sum
    // halos apart
    const bool trow = partial_tick != nullptr && !(H.tree_alpha > 0.0);
    const double4* __restrict__ rows = trow ? partial_tick : partial;
    const int64_t rbase = trow ? H.tick_part_base : H.part_base;
    const int nrow = trow ? H.tick_split : H.grav_split;
    double sx = 0, sy = 0, sz = 0, sp = 0;
    if (symacc && H.grav_sym) {
        // the fixed-point totals of the symmetric tiles
        const double meq = cmass[B.halo];
        double sa, spp;
        sym_scales(H, meq > 0.0 ? 1.0 : cmass[n_halos + B.halo], sa, spp);
        const long long* q = (const long long*)symacc + 4 * p;
        const double ms = meq > 0.0 ? meq : 1.0;
        sx = ms * ((double)q[0] / sa);
        sy = ms * ((double)q[1] / sa);
        sz = ms * ((double)q[2] / sa);
        sp = ms * ((double)q[3] / spp);
    } else {
        for (int s = 0; s < nrow; ++s) {
            const double4 q = rows[rbase + (int64_t)s * H.n + li];
            sx += q.x; sy += q.y; sz += q.z; sp += q.w;
        }
    }
    double gx = H.G * sx, gy = H.G * sy, gz = H.G * sz, gp = -H.G * sp;
    if (H.host_kind != 0) {
        double hx, hy, hz, hp;
        host_field(H, x[o], y[o], z[o], hx, hy, hz, hp);
        gx += hx; gy += hy; gz += hz; gp += hp;
    }
    ax[o] = gx; ay[o] = gy; az[o] = gz; pot[o] = gp;
    if (tick > 0) {
        double h = half_step(H, b);
        double ux = vx[o] + gx * h, uy = vy[o] + gy * h, uz = vz[o] + gz * h;
        if (kl < (1 << H.max_bin)) {
            int nb = time_bin(H, gx, gy, gz);
            while (nb < b && (kl & ((1 << (H.max_bin - nb)) - 1)) != 0) ++nb;
            bin[o] = (int8_t)nb;
            h = half_step(H, nb);
            ux = ux + gx * h; uy = uy + gy * h; uz = uz + gz * h;
        }
        vx[o] = ux; vy[o] = uy; vz[o] = uz;
        svx[p] = ux; svy[p] = uy; svz[p] = uz;
    } else if (kick) {
        const double hdt = 0.5 * H.dt;
        const double ux = vx[o] + gx * hdt, uy = vy[o] + gy * hdt, uz = vz[o] + gz * hdt;
        vx[o] = ux; vy[o] = uy; vz[o] = uz;
        svx[p] = ux; svy[p] = uy; svz[p] = uz;
    }
}

// ---------------------------------------------------------------- launchers
// The kernel instantiation of a launch shape: f(kernel pointer, threads) for
// the mixed (MIXED) or the FP64 tiles of shape (ireg, nt), plain or
// persistent.  False for a shape without an instantiation.
template <bool MIXED, bool PERSIST, class F>
static bool with_shape(int ireg, int nt, F f)
{
#define SIDM_SHAPE(I, T)                                                                      \
    if (ireg == I && nt == T) {                                                               \
        if constexpr (MIXED) f(k_grav_mixed<I, T, PERSIST>, T);                               \
        else f(k_grav_fp64<I, T, PERSIST>, T);                                                \
        return true;                                                                          \
    }
    SIDM_SHAPE(2, 128) SIDM_SHAPE(4, 128) SIDM_SHAPE(8, 128)
    SIDM_SHAPE(2, 256) SIDM_SHAPE(4, 256) SIDM_SHAPE(8, 256)
    SIDM_SHAPE(2, 512) SIDM_SHAPE(4, 512) SIDM_SHAPE(8, 512)
#undef SIDM_SHAPE
    return false;
}

// Blocks of the tiles of a launch shape that the device holds at once
// (compute units times resident blocks per unit), or 0 if unknown.
int64_t gravity_slots(int device, const GravShape& shape, bool mixed)
{
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
        return 0;
    hipError_t e = hipErrorInvalidValue;
    auto query = [&](auto kern, int threads) {
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, 0);
    };
    if (mixed) with_shape<true, true>(shape.ireg, shape.nt, query);
    else with_shape<false, true>(shape.ireg, shape.nt, query);
    return e == hipSuccess ? (int64_t)cus * per_cu : 0;
}

int64_t gravity_slots(int device) { return gravity_slots(device, GravShape{}, true); }

// The symmetric kernels of a launch shape, the common-mass one first:
// f(kernel pointer, threads) for each.  About
// eight pairs per cross-lane reduction: j-slots per reduction 1, 2 or 4 for
// 8, 4 or 2 i-particles per thread.
template <class F>
static bool with_sym_shape(int ireg, int nt, F f)
{
#define SIDM_SYM(I, T)                                                                        \
    if (ireg == I && nt == T) {                                                               \
        f(k_grav_sym<I, T, (I >= 8 ? 1 : 8 / I), true>, T);                                   \
        f(k_grav_sym<I, T, (I >= 8 ? 1 : 8 / I), false>, T);                                  \
        return true;                                                                          \
    }
    SIDM_SYM(2, 128) SIDM_SYM(4, 128) SIDM_SYM(8, 128)
    SIDM_SYM(2, 256) SIDM_SYM(4, 256) SIDM_SYM(8, 256)
    SIDM_SYM(2, 512) SIDM_SYM(4, 512) SIDM_SYM(8, 512)
#undef SIDM_SYM
    return false;
}

// Blocks of the symmetric tiles of a launch shape the device holds at once,
// or 0 if unknown.
int64_t gravity_sym_slots(int device, const GravShape& shape)
{
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
        return 0;
    hipError_t e = hipErrorInvalidValue;
    bool first = true;   // the common-mass kernel: the one that runs the benchmark halos
    with_sym_shape(shape.ireg, shape.nt, [&](auto kern, int threads) {
        if (first) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, 0);
        first = false;
    });
    return e == hipSuccess ? (int64_t)cus * per_cu : 0;
}

__global__ void k_ticket_reset(DevCounters* __restrict__ c)
{
    if (threadIdx.x == 0) c->ticket = 0ull;
}

// The common mass of each halo (w.cref) and the unequal-mass flag of the
// halos that scatter (w.status).
hipError_t launch_mass_check(const Plan& P, Scratch& w, const double* m, hipStream_t st)
{
    hipLaunchKernelGGL(k_block_mass_range, dim3((unsigned)P.n_blocks), dim3(kStreamBlock), 0, st,
                       m, w.blocks, w.bsum);
    hipLaunchKernelGGL(k_halo_mass, dim3(P.n_halos), dim3(kStreamBlock), 0, st, w.halos, w.bsum,
                       w.cref, w.status);
    return hipGetLastError();
}

// Expects the cell list of the current positions (sorted copies sx, sy, sz, sm
// and perm) to be in place.  tick > 0: tick of a cycle of 2^bmax block steps
// (bins in w.bin).
hipError_t launch_tree_gravity(bool mixed, const Plan& P, Scratch& w, const sidm_state* s,
                               int tick, int bmax, hipStream_t st);

hipError_t launch_gravity(bool mixed, const Plan& P, Scratch& w, const sidm_state* s, int kick,
                          hipStream_t st, hipEvent_t tile_begin, hipEvent_t tile_end, int tick,
                          int bmax)
{
    const unsigned nb = (unsigned)P.n_blocks;
    hipLaunchKernelGGL(k_block_mass_range, dim3(nb), dim3(kStreamBlock), 0, st, s->m, w.blocks,
                       w.bsum);
    hipLaunchKernelGGL(k_halo_mass, dim3(P.n_halos), dim3(kStreamBlock), 0, st, w.halos, w.bsum,
                       w.cref, (int*)nullptr);
    if (P.has_tree) {
        // tree halos: one partial row per particle from the walk
        if (tile_begin) (void)hipEventRecord(tile_begin, st);
        const hipError_t e = launch_tree_gravity(mixed, P, w, s, tick, bmax, st);
        if (e != hipSuccess) return e;
        tile_begin = nullptr;
        if (tick == 0 && P.n_items == 0 && tile_end) (void)hipEventRecord(tile_end, st);
    }
    // a tick of block steps runs the finer tick items into their own rows; any
    // other mixed evaluation runs the symmetric tiles for the halos that take
    // them and the one-sided tiles for the rest (their items come first in the
    // item table).  Without tick items no direct-sum halo has block steps, so
    // all of their particles are active at every tick.
    // The last tick of a cycle steps every particle of every halo: it runs the
    // whole evaluation (the symmetric tiles where they apply) instead of the
    // tick items.
    const bool full_tick = tick > 0 && tick == (1 << bmax);
    const bool tk = tick > 0 && !full_tick && !P.items_tick.empty();
    const bool sym = mixed && !tk && P.n_sym_items > 0;
    const GravItem* items = tk ? w.items_tick : w.items;
    const int64_t n_items =
        tk ? (int64_t)P.items_tick.size() : (sym ? P.n_items_nosym : P.n_items);
    double4* rows = tk ? w.partial_tick : w.partial;
    unsigned long long* ticket = &w.counters->ticket;
    if (mixed && (n_items > 0 || sym))
        hipLaunchKernelGGL(k_pack_frames, dim3(nb), dim3(kStreamBlock), 0, st, w.sx, w.sy, w.sz,
                           w.sm, w.blocks, w.halos, w.sub, w.sub_n, w.xm32);
    if (sym) {
        if (w.slots_sym <= 0 || !w.symacc || !w.sym_items) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_sym_zero, dim3(nb), dim3(kStreamBlock), 0, st, w.blocks, w.halos,
                           w.symacc);
        if (tile_begin) (void)hipEventRecord(tile_begin, st);
        tile_begin = nullptr;
        const unsigned grid = (unsigned)std::min<int64_t>(w.slots_sym, P.n_sym_items);
        const bool ok = with_sym_shape(P.shape.ireg, P.shape.nt, [&](auto kern, int threads) {
            hipLaunchKernelGGL(k_ticket_reset, dim3(1), dim3(64), 0, st, w.counters);
            hipLaunchKernelGGL(kern, dim3(grid), dim3(threads), 0, st, w.xm32, w.sub, w.sub_n,
                               w.sym_items, P.n_sym_items, ticket, w.halos, w.cref, P.n_halos,
                               w.symacc);
        });
        if (!ok) return hipErrorInvalidValue;
        if (n_items == 0 && tile_end) (void)hipEventRecord(tile_end, st);
    }
    if (n_items == 0) {
        // no direct-sum halo (left)
    } else {
        // ticks of block steps use the default shape their items were cut for
        const GravShape shape = tk ? GravShape{} : P.shape;
        const bool persist = shape.persist != 0;
        const int64_t slots = persist ? (mixed ? w.slots_mixed : w.slots_fp64) : 0;
        if (persist && slots <= 0) return hipErrorInvalidValue;
        const unsigned grid = (unsigned)(persist ? std::min<int64_t>(slots, n_items) : n_items);
        if (persist) hipLaunchKernelGGL(k_ticket_reset, dim3(1), dim3(64), 0, st, w.counters);
        if (tile_begin) (void)hipEventRecord(tile_begin, st);
        auto launch_mixed = [&](auto kern, int threads) {
            hipLaunchKernelGGL(kern, dim3(grid), dim3(threads), 0, st, w.xm32, w.sub, w.sub_n,
                               items, n_items, ticket, w.halos, w.cref, rows, w.bin, w.perm,
                               tick, bmax, tk ? 1 : 0);
        };
        auto launch_fp64 = [&](auto kern, int threads) {
            hipLaunchKernelGGL(kern, dim3(grid), dim3(threads), 0, st, w.sx, w.sy, w.sz, w.sm,
                               items, n_items, ticket, w.halos, w.cref, rows, w.bin, w.perm,
                               tick, bmax, tk ? 1 : 0);
        };
        bool ok;
        if (mixed)
            ok = persist ? with_shape<true, true>(shape.ireg, shape.nt, launch_mixed)
                         : with_shape<true, false>(shape.ireg, shape.nt, launch_mixed);
        else
            ok = persist ? with_shape<false, true>(shape.ireg, shape.nt, launch_fp64)
                         : with_shape<false, false>(shape.ireg, shape.nt, launch_fp64);
        if (!ok) return hipErrorInvalidValue;
        if (tile_end) (void)hipEventRecord(tile_end, st);
    }
    hipLaunchKernelGGL(k_grav_finalize, dim3(nb), dim3(kStreamBlock), 0, st, w.blocks, w.halos,
                       w.partial, w.perm, s->x, s->y, s->z, s->ax, s->ay, s->az, s->pot, s->vx,
                       s->vy, s->vz, w.svx, w.svy, w.svz, kick, w.bin, tick, bmax,
                       tk ? w.partial_tick : nullptr, sym ? w.symacc : nullptr, w.cref,
                       P.n_halos);
    return hipGetLastError();
}

}  // namespace sidm
