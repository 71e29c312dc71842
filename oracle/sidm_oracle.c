/*
 * sidm_oracle.c -- plain FP64 CPU reference for the SIDM N-body step.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline leg of the benchmark.  The product library never links or calls it.
 *
 * Written from the paper (Fischer, Yu & Dolag, arXiv 2506.06269) and the
 * published definitions it relies on.  Build with -ffp-contract=off so that
 * every expression is evaluated exactly as written (no fused multiply-add).
 * Readings where the paper is silent are marked "reading:".
 */
#include "sidm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11).  Each round multiplies
 * words 0 and 2 by the two Philox multipliers, and the new block is
 * (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0)).  Between
 * rounds the key is advanced by the two Weyl constants (golden ratio and
 * sqrt(3) - 1, scaled to 32 bits). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t mult0 = 0xD2511F53u, mult1 = 0xCD9E8D57u;
    const uint32_t weyl0 = 0x9E3779B9u, weyl1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += weyl0;
            k1 += weyl1;
        }
        uint64_t p0 = (uint64_t)mult0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)mult1 * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

double orc_u53(uint32_t hi, uint32_t lo)
{
    uint64_t bits = (((uint64_t)hi << 32) | (uint64_t)lo) >> 11;
    return (double)bits * (1.0 / 9007199254740992.0); /* 2^-53 */
}

static void philox_pair(uint64_t seed, uint32_t step, uint32_t a, uint32_t b,
                        uint32_t stream, uint32_t w[4])
{
    uint32_t ctr[4] = {a, b, step, stream};
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, w);
}

double orc_accept_u(uint64_t seed, uint32_t step, uint32_t a, uint32_t b)
{
    uint32_t w[4];
    philox_pair(seed, step, a, b, 0u, w);
    return orc_u53(w[0], w[1]);
}

/* ------------------------------------------------------------------------ */
/* Spline kernel (Monaghan 1985) in the compact-support-h form:
 * W = 8/(pi h^3) (1 - 6q^2 + 6q^3) for q <= 1/2, 8/(pi h^3) 2(1-q)^3 for
 * 1/2 < q <= 1, zero beyond; q = r/h.  Reading: h is the radius that holds the
 * N_ngb neighbours, which is what the h/l relation of Sec. 3.5 implies. */
double orc_kernel_W(double r, double h)
{
    double q = r / h;
    double norm = 8.0 / (M_PI * h * h * h);
    if (q <= 0.5) return norm * (1.0 - 6.0 * q * q + 6.0 * q * q * q);
    if (q <= 1.0) {
        double t = 1.0 - q;
        return norm * 2.0 * t * t * t;
    }
    return 0.0;
}

/* Gauss-Legendre nodes and weights on [-1, 1] from their closed forms. */
static void gauss_legendre5(double xk[5], double wk[5])
{
    double s = 2.0 * sqrt(10.0 / 7.0);
    double x1 = sqrt(5.0 - s) / 3.0, x2 = sqrt(5.0 + s) / 3.0;
    double w1 = (322.0 + 13.0 * sqrt(70.0)) / 900.0;
    double w2 = (322.0 - 13.0 * sqrt(70.0)) / 900.0;
    xk[0] = -x2; xk[1] = -x1; xk[2] = 0.0; xk[3] = x1; xk[4] = x2;
    wk[0] = w2;  wk[1] = w1;  wk[2] = 128.0 / 225.0; wk[3] = w1; wk[4] = w2;
}

static void gauss_legendre3(double xk[3], double wk[3])
{
    double x = sqrt(3.0 / 5.0);
    xk[0] = -x; xk[1] = 0.0; xk[2] = x;
    wk[0] = 5.0 / 9.0; wk[1] = 8.0 / 9.0; wk[2] = 5.0 / 9.0;
}

/* integral of s W(s, h) over [s0, s0 + w]; 3-point Gauss-Legendre is exact
 * because s W(s) is a polynomial of degree 4 on the segment (which must not
 * straddle h/2 or h). */
static double seg_sW(double s0, double w, double h)
{
    double xk[3], wk[3], sum = 0.0;
    gauss_legendre3(xk, wk);
    for (int k = 0; k < 3; ++k) {
        double s = s0 + 0.5 * w * (1.0 + xk[k]);
        sum += wk[k] * s * orc_kernel_W(s, h);
    }
    return 0.5 * w * sum;
}

/* G(r, d) = integral of s W(s, hj) ds over s in [|d - r|, min(d + r, hj)]:
 * the part of the spherical shell of radius r about particle i that lies inside
 * the support of particle j, reduced to one dimension (bipolar coordinates). */
static double shell_overlap(double r, double d, double hj)
{
    double lo = fabs(d - r);
    double up, width;
    if (d + r <= hj) {
        up = d + r;
        width = 2.0 * (d < r ? d : r); /* (d + r) - |d - r| without cancellation */
    } else {
        up = hj;
        width = hj - lo;
    }
    if (!(width > 0.0)) return 0.0;
    double half = 0.5 * hj;
    if (up <= half || lo >= half) return seg_sW(lo, width, hj);
    return seg_sW(lo, half - lo, hj) + seg_sW(half, up - half, hj);
}

static int cmp_double(const void *pa, const void *pb)
{
    double a = *(const double *)pa, b = *(const double *)pb;
    return (a > b) - (a < b);
}

/* Lambda(d; hi, hj) = integral of W(|x - xi|, hi) W(|x - xj|, hj) d^3x.
 * With r = |x - xi| and s = |x - xj| the volume element of a shell of radius r
 * about xi at distance s from xj is (2 pi r s / d) ds dr, so
 *   Lambda = (2 pi / d) int_0^hi r W(r, hi) G(r, d) dr,
 * and at d = 0 simply 4 pi int r^2 W(r, hi) W(r, hj) dr.  On each interval
 * between the breakpoints {hi/2, d, |d -+ hj/2|, d + hj/2, |d - hj|, d + hj}
 * the integrand is a polynomial of degree <= 9, so 5-point Gauss-Legendre per
 * interval is exact up to rounding.  Reading: the paper cites the geometric
 * factor of its SIDM scheme without printing it; it is taken here as the
 * overlap integral of the two particles' kernels. */
double orc_lambda(double d, double hi, double hj)
{
    double xk[5], wk[5];
    gauss_legendre5(xk, wk);
    if (!(d < hi + hj)) return 0.0;
    if (d == 0.0) {
        double hmin = hi < hj ? hi : hj;
        double bp[4] = {0.0, 0.5 * hi, 0.5 * hj, hmin};
        qsort(bp, 4, sizeof(double), cmp_double);
        double total = 0.0;
        for (int p = 0; p < 3; ++p) {
            double r0 = bp[p], r1 = bp[p + 1];
            if (r1 > hmin) r1 = hmin;
            if (!(r1 > r0)) continue;
            double w = r1 - r0, sum = 0.0;
            for (int k = 0; k < 5; ++k) {
                double r = r0 + 0.5 * w * (1.0 + xk[k]);
                sum += wk[k] * r * r * orc_kernel_W(r, hi) * orc_kernel_W(r, hj);
            }
            total += 0.5 * w * sum;
        }
        return 4.0 * M_PI * total;
    }
    double cand[8] = {0.5 * hi, d, fabs(d - 0.5 * hj), d + 0.5 * hj,
                      fabs(d - hj), d + hj, 0.0, hi};
    double bp[8];
    int nb = 0;
    bp[nb++] = 0.0;
    bp[nb++] = hi;
    for (int c = 0; c < 6; ++c)
        if (cand[c] > 0.0 && cand[c] < hi) bp[nb++] = cand[c];
    qsort(bp, (size_t)nb, sizeof(double), cmp_double);
    double total = 0.0;
    for (int p = 0; p + 1 < nb; ++p) {
        double r0 = bp[p], r1 = bp[p + 1];
        if (!(r1 > r0)) continue;
        double w = r1 - r0, sum = 0.0;
        for (int k = 0; k < 5; ++k) {
            double r = r0 + 0.5 * w * (1.0 + xk[k]);
            sum += wk[k] * r * orc_kernel_W(r, hi) * shell_overlap(r, d, hj);
        }
        total += 0.5 * w * sum;
    }
    return 2.0 * M_PI / d * total;
}

/* ------------------------------------------------------------------------ */
/* Neumaier's compensated summation. */
typedef struct { double s, c; } neum;

static void neum_add(neum *acc, double v)
{
    double t = acc->s + v;
    if (fabs(acc->s) >= fabs(v)) acc->c += (acc->s - t) + v;
    else acc->c += (v - t) + acc->s;
    acc->s = t;
}

static double neum_get(const neum *acc) { return acc->s + acc->c; }

/* Softened self-gravity (Sec. 2: softening length eps; reading: Plummer form,
 * self term excluded from both a and phi). */
void orc_gravity(int64_t n, const double *x, const double *y, const double *z,
                 const double *m, double G, double eps,
                 int64_t nq, const int64_t *q,
                 double *ax, double *ay, double *az, double *pot, double *anorm)
{
    if (q == NULL) nq = n;
    double eps2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nq; ++k) {
        int64_t i = q ? q[k] : k;
        neum sx = {0, 0}, sy = {0, 0}, sz = {0, 0}, sp = {0, 0}, sa = {0, 0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = x[j] - x[i], dy = y[j] - y[i], dz = z[j] - z[i];
            double d2 = dx * dx + dy * dy + dz * dz;
            double r2 = d2 + eps2;
            double rinv = 1.0 / sqrt(r2);
            double rinv3 = rinv * rinv * rinv;
            double w = m[j] * rinv3;
            neum_add(&sx, w * dx);
            neum_add(&sy, w * dy);
            neum_add(&sz, w * dz);
            neum_add(&sp, -m[j] * rinv);
            if (anorm) neum_add(&sa, w * sqrt(d2));
        }
        ax[k] = G * neum_get(&sx);
        ay[k] = G * neum_get(&sy);
        az[k] = G * neum_get(&sz);
        pot[k] = G * neum_get(&sp);
        if (anorm) anorm[k] = G * neum_get(&sa);
    }
}

/* ---- tree gravity ---- */
typedef struct {
    int64_t first, count;       /* sorted particle range                       */
    int64_t child0;             /* first child (node index), -1 for a bucket   */
    int32_t nchild, pad;
    double box[6];              /* lo xyz, hi xyz                              */
    double M, Mx, My, Mz;       /* mass and first moments                      */
    double S[6];                /* second moments about the centre of mass:
                                   xx, yy, zz, xy, xz, yz                      */
} tree_node;

typedef struct {
    uint64_t key;
    int64_t idx;
} key_idx;

static int cmp_key_idx(const void *a, const void *b)
{
    const key_idx *p = (const key_idx *)a, *q = (const key_idx *)b;
    if (p->key != q->key) return p->key < q->key ? -1 : 1;
    return (p->idx > q->idx) - (p->idx < q->idx);
}

static uint64_t spread_bits3(unsigned v)
{
    uint64_t r = 0;
    for (int b = 0; b < 16; ++b)
        if (v & (1u << b)) r |= (uint64_t)1 << (3 * b);
    return r;
}

static unsigned quantise16(double v, double lo, double inv)
{
    double q = (v - lo) * inv;
    q = fmin(fmax(q, 0.0), 65535.0);
    return (unsigned)q;
}

typedef struct {
    const double *sx, *sy, *sz, *sm;    /* sorted copies                     */
    const int64_t *sidx;                /* sorted -> caller index            */
    tree_node *nodes;
    double G, eps2, alpha2, a2min;
    const double *gbox;
    /* the source list of one group */
    double *lx, *ly, *lz, *lm;
    int64_t *lidx;
    int64_t len;
} tree_walk;

static int boxes_disjoint(const double *a, const double *b)
{
    for (int c = 0; c < 3; ++c)
        if (a[c] > b[3 + c] || a[3 + c] < b[c]) return 1;
    return 0;
}

static int tree_accept(const tree_walk *W, const tree_node *nd)
{
    if (!boxes_disjoint(nd->box, W->gbox)) return 0;
    if (nd->M == 0.0) return 1;
    double d[3];
    for (int k = 0; k < 3; ++k) {
        double lo = W->gbox[k] - nd->box[3 + k], hi = nd->box[k] - W->gbox[3 + k];
        d[k] = fmax(fmax(lo, hi), 0.0);
    }
    double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
    double l = fmax(fmax(nd->box[3] - nd->box[0], nd->box[4] - nd->box[1]),
                    nd->box[5] - nd->box[2]);
    double q = ((W->G * nd->M) * l) * l;
    double lhs = q * q;
    double r4 = r2 * r2;
    double rhs = ((W->alpha2 * W->a2min) * r4) * r4;
    return lhs <= rhs;
}

static void tree_visit(tree_walk *W, int64_t node)
{
    tree_node *nd = &W->nodes[node];
    if (tree_accept(W, nd)) {
        if (nd->M == 0.0) return;
        W->lx[W->len] = nd->Mx / nd->M;
        W->ly[W->len] = nd->My / nd->M;
        W->lz[W->len] = nd->Mz / nd->M;
        W->lm[W->len] = nd->M;
        W->lidx[W->len] = -2 - node;    /* an accepted node */
        W->len++;
        return;
    }
    if (nd->child0 < 0) {
        for (int64_t p = nd->first; p < nd->first + nd->count; ++p) {
            W->lx[W->len] = W->sx[p];
            W->ly[W->len] = W->sy[p];
            W->lz[W->len] = W->sz[p];
            W->lm[W->len] = W->sm[p];
            W->lidx[W->len] = p;
            W->len++;
        }
        return;
    }
    for (int32_t k = 0; k < nd->nchild; ++k) tree_visit(W, nd->child0 + k);
}

void orc_tree_gravity(int64_t n, const double *x, const double *y, const double *z,
                      const double *m, const double *ax_old, const double *ay_old,
                      const double *az_old, double G, double eps, double alpha, int64_t nq,
                      const int64_t *q, double *ax, double *ay, double *az, double *pot,
                      int64_t *terms)
{
    const int64_t B = 64, F = 8;
    if (terms) *terms = 0;
    if (n <= 0) return;
    /* Morton order over the bounding box */
    double lo[3] = {x[0], y[0], z[0]}, hi[3] = {x[0], y[0], z[0]};
    for (int64_t i = 0; i < n; ++i) {
        const double p[3] = {x[i], y[i], z[i]};
        for (int c = 0; c < 3; ++c) {
            lo[c] = fmin(lo[c], p[c]);
            hi[c] = fmax(hi[c], p[c]);
        }
    }
    double ext = fmax(fmax(hi[0] - lo[0], hi[1] - lo[1]), hi[2] - lo[2]);
    double inv = ext > 0.0 ? 65535.0 / ext : 0.0;
    key_idx *ki = (key_idx *)malloc(sizeof(key_idx) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        ki[i].key = spread_bits3(quantise16(x[i], lo[0], inv)) |
                    (spread_bits3(quantise16(y[i], lo[1], inv)) << 1) |
                    (spread_bits3(quantise16(z[i], lo[2], inv)) << 2);
        ki[i].idx = i;
    }
    qsort(ki, (size_t)n, sizeof(key_idx), cmp_key_idx);
    double *sorted = (double *)malloc(sizeof(double) * (size_t)n * 4);
    double *sx = sorted, *sy = sx + n, *sz = sy + n, *sm = sz + n;
    int64_t *sidx = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t p = 0; p < n; ++p) {
        const int64_t i = ki[p].idx;
        sx[p] = x[i];
        sy[p] = y[i];
        sz[p] = z[i];
        sm[p] = m[i];
        sidx[p] = i;
    }
    free(ki);
    /* buckets, then levels of F consecutive nodes up to one root */
    const int64_t nb = (n + B - 1) / B;
    int64_t cap = nb, level_n = nb;
    while (level_n > 1) {
        level_n = (level_n + F - 1) / F;
        cap += level_n;
    }
    tree_node *nodes = (tree_node *)calloc((size_t)cap, sizeof(tree_node));
    for (int64_t b = 0; b < nb; ++b) {
        tree_node *nd = &nodes[b];
        nd->first = b * B;
        nd->count = (b + 1) * B <= n ? B : n - b * B;
        nd->child0 = -1;
        for (int c = 0; c < 3; ++c) {
            nd->box[c] = INFINITY;
            nd->box[3 + c] = -INFINITY;
        }
        for (int64_t p = nd->first; p < nd->first + nd->count; ++p) {
            const double q[3] = {sx[p], sy[p], sz[p]};
            for (int c = 0; c < 3; ++c) {
                nd->box[c] = fmin(nd->box[c], q[c]);
                nd->box[3 + c] = fmax(nd->box[3 + c], q[c]);
            }
            nd->M += sm[p];
            nd->Mx += sm[p] * sx[p];
            nd->My += sm[p] * sy[p];
            nd->Mz += sm[p] * sz[p];
        }
    }
    int64_t off = 0, cnt = nb, top = nb;
    while (cnt > 1) {
        const int64_t nn = (cnt + F - 1) / F;
        for (int64_t j = 0; j < nn; ++j) {
            tree_node *nd = &nodes[top + j];
            nd->child0 = off + j * F;
            nd->nchild = (int32_t)((j + 1) * F <= cnt ? F : cnt - j * F);
            const tree_node *c0 = &nodes[nd->child0];
            const tree_node *cl = &nodes[nd->child0 + nd->nchild - 1];
            nd->first = c0->first;
            nd->count = cl->first + cl->count - c0->first;
            for (int c = 0; c < 3; ++c) {
                nd->box[c] = INFINITY;
                nd->box[3 + c] = -INFINITY;
            }
            for (int32_t k = 0; k < nd->nchild; ++k) {
                const tree_node *ch = &nodes[nd->child0 + k];
                for (int c = 0; c < 3; ++c) {
                    nd->box[c] = fmin(nd->box[c], ch->box[c]);
                    nd->box[3 + c] = fmax(nd->box[3 + c], ch->box[3 + c]);
                }
                nd->M += ch->M;
                nd->Mx += ch->Mx;
                nd->My += ch->My;
                nd->Mz += ch->Mz;
            }
        }
        off = top;
        top += nn;
        cnt = nn;
    }
    const int64_t root = top - 1;
    /* second moments about each node's centre of mass: a bucket's from its
     * particles in order, a node's from its children (parallel axes) */
    for (int64_t t = 0; t < top; ++t) {
        tree_node *nd = &nodes[t];
        for (int k = 0; k < 6; ++k) nd->S[k] = 0.0;
        if (nd->M == 0.0) continue;
        const double cx = nd->Mx / nd->M, cy = nd->My / nd->M, cz = nd->Mz / nd->M;
        if (nd->child0 < 0) {
            for (int64_t p = nd->first; p < nd->first + nd->count; ++p) {
                const double u = sx[p] - cx, v = sy[p] - cy, w = sz[p] - cz;
                nd->S[0] += sm[p] * u * u;
                nd->S[1] += sm[p] * v * v;
                nd->S[2] += sm[p] * w * w;
                nd->S[3] += sm[p] * u * v;
                nd->S[4] += sm[p] * u * w;
                nd->S[5] += sm[p] * v * w;
            }
            continue;
        }
        for (int32_t k = 0; k < nd->nchild; ++k) {
            const tree_node *ch = &nodes[nd->child0 + k];
            if (ch->M == 0.0) continue;
            const double u = ch->Mx / ch->M - cx, v = ch->My / ch->M - cy,
                         w = ch->Mz / ch->M - cz;
            nd->S[0] += ch->S[0] + ch->M * u * u;
            nd->S[1] += ch->S[1] + ch->M * v * v;
            nd->S[2] += ch->S[2] + ch->M * w * w;
            nd->S[3] += ch->S[3] + ch->M * u * v;
            nd->S[4] += ch->S[4] + ch->M * u * w;
            nd->S[5] += ch->S[5] + ch->M * v * w;
        }
    }
    /* the groups that hold a queried particle (all of them without q) */
    const int64_t nqq = q ? nq : n;
    int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t p = 0; p < n; ++p) pos[sidx[p]] = p;
    key_idx *qe = (key_idx *)malloc(sizeof(key_idx) * (size_t)(nqq > 0 ? nqq : 1));
    for (int64_t k = 0; k < nqq; ++k) {
        const int64_t p = pos[q ? q[k] : k];
        qe[k].key = (uint64_t)(p / B);
        qe[k].idx = k;
    }
    qsort(qe, (size_t)nqq, sizeof(key_idx), cmp_key_idx);
    int64_t *gstart = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nqq + 1));
    int64_t ng = 0;
    for (int64_t k = 0; k < nqq; ++k)
        if (k == 0 || qe[k].key != qe[k - 1].key) gstart[ng++] = k;
    gstart[ng] = nqq;
    /* one walk per group (bucket), then the queried members' sums over its list */
    int64_t total = 0;
#pragma omp parallel reduction(+ : total)
    {
        tree_walk W;
        W.sx = sx; W.sy = sy; W.sz = sz; W.sm = sm; W.sidx = sidx;
        W.nodes = nodes;
        W.G = G;
        W.eps2 = eps * eps;
        W.alpha2 = alpha * alpha;
        const size_t lc = (size_t)(n + cap);
        double *lbuf = (double *)malloc(sizeof(double) * lc * 4);
        W.lx = lbuf; W.ly = lbuf + lc; W.lz = W.ly + lc; W.lm = W.lz + lc;
        W.lidx = (int64_t *)malloc(sizeof(int64_t) * lc);
#pragma omp for schedule(dynamic, 1)
        for (int64_t gi = 0; gi < ng; ++gi) {
            const tree_node *g = &nodes[qe[gstart[gi]].key];
            double a2min = INFINITY;
            for (int64_t p = g->first; p < g->first + g->count; ++p) {
                const int64_t i = sidx[p];
                const double a2 = (ax_old[i] * ax_old[i] + ay_old[i] * ay_old[i]) +
                                  az_old[i] * az_old[i];
                a2min = fmin(a2min, a2);
            }
            W.a2min = a2min;
            W.gbox = g->box;
            W.len = 0;
            tree_visit(&W, root);
            total += W.len;
            for (int64_t k = gstart[gi]; k < gstart[gi + 1]; ++k) {
                const int64_t out = qe[k].idx;
                const int64_t p = pos[q ? q[out] : out];
                neum gx = {0, 0}, gy = {0, 0}, gz = {0, 0}, gp = {0, 0};
                for (int64_t t = 0; t < W.len; ++t) {
                    if (W.lidx[t] == p) continue;
                    const double dx = W.lx[t] - sx[p], dy = W.ly[t] - sy[p],
                                 dz = W.lz[t] - sz[p];
                    const double r2 = dx * dx + dy * dy + dz * dz + W.eps2;
                    const double rinv = 1.0 / sqrt(r2);
                    const double w = W.lm[t] * rinv * rinv * rinv;
                    neum_add(&gx, w * dx);
                    neum_add(&gy, w * dy);
                    neum_add(&gz, w * dz);
                    neum_add(&gp, -W.lm[t] * rinv);
                    if (W.lidx[t] <= -2) {
                        /* an accepted node's quadrupole: the second-order term
                         * of the softened potential -G sum m / sqrt(|d - s|^2
                         * + eps^2) expanded about its centre of mass (s: a
                         * particle's offset from it, d: from it to the member,
                         * rho^2 = |d|^2 + eps^2, S the second moments, T
                         * their trace): phi_Q = -G (3 d.S.d - rho^2 T) /
                         * (2 rho^5), a_Q = -grad phi_Q */
                        const double *S = nodes[-2 - W.lidx[t]].S;
                        const double d0 = -dx, d1 = -dy, d2 = -dz;
                        const double ri2 = rinv * rinv, ri5 = rinv * ri2 * ri2, ri7 = ri5 * ri2;
                        const double Sd0 = (S[0] * d0 + S[3] * d1) + S[4] * d2;
                        const double Sd1 = (S[3] * d0 + S[1] * d1) + S[5] * d2;
                        const double Sd2 = (S[4] * d0 + S[5] * d1) + S[2] * d2;
                        const double T = (S[0] + S[1]) + S[2];
                        const double br = 3.0 * ((d0 * Sd0 + d1 * Sd1) + d2 * Sd2) - r2 * T;
                        neum_add(&gx, (3.0 * Sd0 - T * d0) * ri5 - 2.5 * br * d0 * ri7);
                        neum_add(&gy, (3.0 * Sd1 - T * d1) * ri5 - 2.5 * br * d1 * ri7);
                        neum_add(&gz, (3.0 * Sd2 - T * d2) * ri5 - 2.5 * br * d2 * ri7);
                        neum_add(&gp, -0.5 * br * ri5);
                    }
                }
                ax[out] = G * neum_get(&gx);
                ay[out] = G * neum_get(&gy);
                az[out] = G * neum_get(&gz);
                pot[out] = G * neum_get(&gp);
            }
        }
        free(lbuf);
        free(W.lidx);
    }
    if (terms) *terms = total;
    free(pos);
    free(qe);
    free(gstart);
    free(nodes);
    free(sorted);
    free(sidx);
}

/* NFW host (Sec. 4.1, Eq. nfw_potential).  With s = r/r_s and
 * K = 4 pi G rho_s r_s^3:  Phi = -K ln(1+s)/r, and the enclosed mass gives
 * a = -K [ln(1+s) - s/(1+s)] (x - c)/r^3.  For s < 1e-4 the bracket uses its
 * series s^2/2 - 2s^3/3 + 3s^4/4 - 4s^5/5 to avoid cancellation. */
void orc_host_nfw(int64_t n, const double *x, const double *y, const double *z,
                  double G, double rho_s, double r_s, const double c[3],
                  double *ax, double *ay, double *az, double *pot)
{
    double K = 4.0 * M_PI * G * rho_s * r_s * r_s * r_s;
    for (int64_t i = 0; i < n; ++i) {
        double dx = x[i] - c[0], dy = y[i] - c[1], dz = z[i] - c[2];
        double r = sqrt(dx * dx + dy * dy + dz * dz);
        if (r == 0.0) {
            ax[i] = ay[i] = az[i] = 0.0;
            pot[i] = -K / r_s;
            continue;
        }
        double s = r / r_s;
        double mu;
        if (s < 1e-4) mu = s * s * (0.5 - s * (2.0 / 3.0 - s * (0.75 - s * 0.8)));
        else mu = log1p(s) - s / (1.0 + s);
        double f = -K * mu / (r * r * r);
        ax[i] = f * dx;
        ay[i] = f * dy;
        az[i] = f * dz;
        pot[i] = -K * log1p(s) / r;
    }
}

/* ------------------------------------------------------------------------ */
/* k nearest neighbours by brute force (Sec. 2: kernel size set by the next
 * N_ngb neighbours).  Reading: h_i is the exact distance of the k-th nearest
 * other particle, ties broken by id. */
/* Hernquist bulge (Sec. 4.1, Eq. hernquist_potential): Phi = -G M / (r + a);
 * a = -dPhi/dr r_hat = -G M d / (r (r + a)^2). */
void orc_host_hernquist(int64_t n, const double *x, const double *y, const double *z,
                        double G, double M, double a, const double c[3],
                        double *ax, double *ay, double *az, double *pot)
{
    for (int64_t i = 0; i < n; ++i) {
        double dx = x[i] - c[0], dy = y[i] - c[1], dz = z[i] - c[2];
        double r = sqrt((dx * dx + dy * dy) + dz * dz);
        pot[i] = -G * M / (r + a);
        if (r == 0.0) {
            ax[i] = ay[i] = az[i] = 0.0;
            continue;
        }
        double f = -G * M / (r * (r + a) * (r + a));
        ax[i] = f * dx;
        ay[i] = f * dy;
        az[i] = f * dz;
    }
}

/* Miyamoto-Nagai disc (Sec. 4.1, Eq. disk_potential) in the z = 0 plane of c:
 * with zeta = sqrt(z^2 + b^2) and D^2 = R^2 + (a + zeta)^2, Phi = -G M / D and
 * a = -grad Phi = -G M (x, y, z (a + zeta) / zeta) / D^3. */
void orc_host_disk(int64_t n, const double *x, const double *y, const double *z,
                   double G, double M, double a, double b, const double c[3],
                   double *ax, double *ay, double *az, double *pot)
{
    for (int64_t i = 0; i < n; ++i) {
        double dx = x[i] - c[0], dy = y[i] - c[1], dz = z[i] - c[2];
        double zeta = sqrt(dz * dz + b * b);
        double D2 = (dx * dx + dy * dy) + (a + zeta) * (a + zeta);
        double D = sqrt(D2);
        pot[i] = -G * M / D;
        double f = -G * M / (D2 * D);
        ax[i] = f * dx;
        ay[i] = f * dy;
        az[i] = zeta > 0.0 ? f * dz * (a + zeta) / zeta : 0.0;
    }
}

void orc_host_field(int64_t n, const double *x, const double *y, const double *z,
                    const orc_params *p, double *ax, double *ay, double *az, double *pot)
{
    for (int64_t i = 0; i < n; ++i) ax[i] = ay[i] = az[i] = pot[i] = 0.0;
    if (p->host_kind == 0 || n == 0) return;
    double *t = (double *)malloc(sizeof(double) * (size_t)n * 4);
    double *tx = t, *ty = t + n, *tz = t + 2 * n, *tp = t + 3 * n;
    for (int comp = 0; comp < 6; ++comp) {
        if (comp == 0) {
            if (p->host_rho_s == 0.0) continue;
            orc_host_nfw(n, x, y, z, p->G, p->host_rho_s, p->host_r_s, p->host_c, tx, ty, tz, tp);
        } else if (p->host_kind != 2) {
            break;
        } else if (comp == 1) {
            if (p->host_hern_M == 0.0) continue;
            orc_host_hernquist(n, x, y, z, p->G, p->host_hern_M, p->host_hern_a, p->host_c,
                               tx, ty, tz, tp);
        } else {
            const double *d = p->host_disk[comp - 2];
            if (d[0] == 0.0) continue;
            orc_host_disk(n, x, y, z, p->G, d[0], d[1], d[2], p->host_c, tx, ty, tz, tp);
        }
        for (int64_t i = 0; i < n; ++i) {
            ax[i] += tx[i];
            ay[i] += ty[i];
            az[i] += tz[i];
            pot[i] += tp[i];
        }
    }
    free(t);
}

static int key_less(double d2a, uint32_t ida, double d2b, uint32_t idb)
{
    return d2a < d2b || (d2a == d2b && ida < idb);
}

void orc_knn(int64_t n, const double *x, const double *y, const double *z,
             const uint32_t *id, int32_t k, int64_t nq, const int64_t *q,
             double *h, uint32_t *nbr)
{
    if (q == NULL) nq = n;
#pragma omp parallel
    {
        double *bd = (double *)malloc(sizeof(double) * (size_t)k);
        uint32_t *bi = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)k);
#pragma omp for schedule(dynamic, 16)
        for (int64_t t = 0; t < nq; ++t) {
            int64_t i = q ? q[t] : t;
            int32_t cnt = 0;
            for (int64_t j = 0; j < n; ++j) {
                if (j == i) continue;
                double dx = x[j] - x[i], dy = y[j] - y[i], dz = z[j] - z[i];
                double d2 = (dx * dx + dy * dy) + dz * dz;
                if (cnt == k && !key_less(d2, id[j], bd[k - 1], bi[k - 1])) continue;
                /* insertion into the sorted list of the best k */
                int32_t pos = cnt < k ? cnt : k - 1;
                while (pos > 0 && key_less(d2, id[j], bd[pos - 1], bi[pos - 1])) {
                    bd[pos] = bd[pos - 1];
                    bi[pos] = bi[pos - 1];
                    --pos;
                }
                bd[pos] = d2;
                bi[pos] = id[j];
                if (cnt < k) ++cnt;
            }
            h[t] = sqrt(bd[k - 1]);
            if (nbr) memcpy(nbr + (size_t)t * (size_t)k, bi, sizeof(uint32_t) * (size_t)k);
        }
        free(bd);
        free(bi);
    }
}

/* ------------------------------------------------------------------------ */
/* Scattering decisions (Sec. 2: pairwise interactions through the spline
 * kernel; Sec. 3.5: the geometric factor Lambda).  Readings: every unordered
 * pair whose supports overlap is tested once; the probability uses the
 * velocities at the start of the pass, so the event set does not depend on the
 * order of evaluation. */
static int cmp_event(const void *pa, const void *pb)
{
    const orc_event *a = (const orc_event *)pa, *b = (const orc_event *)pb;
    if (a->a != b->a) return a->a < b->a ? -1 : 1;
    if (a->b != b->b) return a->b < b->b ? -1 : 1;
    return 0;
}

/* Cross-section per unit mass at the pair's relative speed g (Sec. 3.8,
 * Eq. vel_dep): sigma_m [1 + (g/w)^2]^-2, the viscosity cross-section, which the
 * paper normalises to equal the total cross-section for isotropic scattering.
 * Reading: g = |v_a - v_b| with the velocities at the start of the pass; w <= 0
 * means velocity independent. */
double orc_sigma(double sigma_m, double w, double g)
{
    if (!(w > 0.0)) return sigma_m;
    double t = g / w;
    double q = 1.0 + t * t;
    return sigma_m / (q * q);
}

int64_t orc_find_events(int64_t n, const double *x, const double *y, const double *z,
                        const double *vx, const double *vy, const double *vz,
                        const double *m, const uint32_t *id, const double *h,
                        double sigma_m, double sigma_w, double dt, uint64_t seed, uint32_t step,
                        const uint8_t *qmask, orc_event *ev, int64_t cap,
                        int64_t *n_pairs, int64_t *n_p_gt1)
{
    int64_t found = 0, pairs = 0, pgt1 = 0;
    int64_t stored = 0;
    orc_event *all = NULL;
    int64_t all_cap = 0;
#pragma omp parallel
    {
        int64_t my_pairs = 0, my_pgt1 = 0, my_n = 0, my_cap = 64;
        orc_event *mine = (orc_event *)malloc(sizeof(orc_event) * (size_t)my_cap);
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < n; ++i) {
            if (qmask && !qmask[i]) continue;
            for (int64_t j = 0; j < n; ++j) {
                if (j == i) continue;
                if (qmask) {
                    if (qmask[j] && j < i) continue; /* pair already seen from j */
                } else if (j < i) {
                    continue;
                }
                double dx = x[j] - x[i], dy = y[j] - y[i], dz = z[j] - z[i];
                double d2 = (dx * dx + dy * dy) + dz * dz;
                double hs = h[i] + h[j];
                if (!(d2 < hs * hs)) continue;
                ++my_pairs;
                int64_t ia = id[i] < id[j] ? i : j;
                int64_t ib = id[i] < id[j] ? j : i;
                uint32_t a = id[ia], b = id[ib];
                double u = orc_accept_u(seed, step, a, b);
                double gx = vx[ia] - vx[ib], gy = vy[ia] - vy[ib], gz = vz[ia] - vz[ib];
                double g = sqrt((gx * gx + gy * gy) + gz * gz);
                double lam = orc_lambda(sqrt(d2), h[ia], h[ib]);
                double P = orc_sigma(sigma_m, sigma_w, g) * m[ib] * g * lam * dt;
                if (P > 1.0) ++my_pgt1;
                if (u < P) {
                    if (my_n == my_cap) {
                        my_cap *= 2;
                        mine = (orc_event *)realloc(mine, sizeof(orc_event) * (size_t)my_cap);
                    }
                    orc_event e = {a, b, ia, ib, u, P};
                    mine[my_n++] = e;
                }
            }
        }
#pragma omp critical
        {
            if (found + my_n > all_cap) {
                all_cap = 2 * (found + my_n) + 64;
                all = (orc_event *)realloc(all, sizeof(orc_event) * (size_t)all_cap);
            }
            memcpy(all + found, mine, sizeof(orc_event) * (size_t)my_n);
            found += my_n;
            pairs += my_pairs;
            pgt1 += my_pgt1;
        }
        free(mine);
    }
    if (found > 0) qsort(all, (size_t)found, sizeof(orc_event), cmp_event);
    stored = found < cap ? found : cap;
    if (stored > 0 && ev) memcpy(ev, all, sizeof(orc_event) * (size_t)stored);
    free(all);
    if (n_pairs) *n_pairs = pairs;
    if (n_p_gt1) *n_p_gt1 = pgt1;
    return found;
}

/* Elastic isotropic scattering in the pair's centre-of-mass frame (Sec. 2:
 * explicit conservation of energy and linear momentum).  The relative speed g
 * is kept, the direction of the relative velocity is redrawn uniformly on the
 * sphere: cos(theta) = 1 - 2 u_c, phi = 2 pi u_phi, from the direction draw at
 * counter (a, b, step, 1). */
void orc_kick_pair(uint64_t seed, uint32_t step, uint32_t a, uint32_t b,
                   double ma, double mb, double va[3], double vb[3])
{
    uint32_t w[4];
    philox_pair(seed, step, a, b, 1u, w);
    double uc = orc_u53(w[0], w[1]);
    double uphi = orc_u53(w[2], w[3]);
    double M = ma + mb;
    double dvx = va[0] - vb[0], dvy = va[1] - vb[1], dvz = va[2] - vb[2];
    double g = sqrt((dvx * dvx + dvy * dvy) + dvz * dvz);
    double cth = 1.0 - 2.0 * uc;
    double s2 = 1.0 - cth * cth;
    double sth = sqrt(s2 > 0.0 ? s2 : 0.0);
    double ph = 2.0 * M_PI * uphi;
    double nvec[3] = {sth * cos(ph), sth * sin(ph), cth};
    double fa = mb / M * g, fb = ma / M * g;
    for (int c = 0; c < 3; ++c) {
        double vcm = (ma * va[c] + mb * vb[c]) / M;
        va[c] = vcm + fa * nvec[c];
        vb[c] = vcm - fb * nvec[c];
    }
}

void orc_apply_events(int64_t n_ev, const orc_event *ev, const double *m,
                      double *vx, double *vy, double *vz, uint64_t seed, uint32_t step)
{
    for (int64_t e = 0; e < n_ev; ++e) {
        int64_t ia = ev[e].ia, ib = ev[e].ib;
        double va[3] = {vx[ia], vy[ia], vz[ia]};
        double vb[3] = {vx[ib], vy[ib], vz[ib]};
        orc_kick_pair(seed, step, ev[e].a, ev[e].b, m[ia], m[ib], va, vb);
        vx[ia] = va[0]; vy[ia] = va[1]; vz[ia] = va[2];
        vx[ib] = vb[0]; vy[ib] = vb[1]; vz[ib] = vb[2];
    }
}

/* ------------------------------------------------------------------------ */
void orc_diag(int64_t n, const double *vx, const double *vy, const double *vz,
              const double *m, const double *pot, const double *pext, double out[6])
{
    neum K = {0, 0}, W = {0, 0}, E = {0, 0}, px = {0, 0}, py = {0, 0}, pz = {0, 0};
    for (int64_t i = 0; i < n; ++i) {
        double v2 = (vx[i] * vx[i] + vy[i] * vy[i]) + vz[i] * vz[i];
        double pe = pext ? pext[i] : 0.0;
        neum_add(&K, 0.5 * m[i] * v2);
        neum_add(&W, 0.5 * m[i] * (pot[i] - pe));
        neum_add(&E, m[i] * pe);
        neum_add(&px, m[i] * vx[i]);
        neum_add(&py, m[i] * vy[i]);
        neum_add(&pz, m[i] * vz[i]);
    }
    out[0] = neum_get(&K);
    out[1] = neum_get(&W);
    out[2] = neum_get(&E);
    out[3] = neum_get(&px);
    out[4] = neum_get(&py);
    out[5] = neum_get(&pz);
}

/* ------------------------------------------------------------------------ */
/* Exact searches for long runs.  They return exactly what the brute-force
 * definitions above return (the tests require equality): only the order in
 * which candidates are examined changes, never the expression of a distance,
 * the (d2, id) order or the pair test. */

typedef struct {
    double lo[3], c;        /* origin and cell size                               */
    int64_t nc[3];          /* cells per axis                                      */
    int64_t *start;         /* particles of cell q: item[start[q] .. start[q + 1]) */
    int64_t *item;
} orc_grid;

static int64_t grid_axis(const orc_grid *g, double v, int a)
{
    double t = floor((v - g->lo[a]) / g->c);
    if (!(t >= 0.0)) return 0;
    if (t > (double)(g->nc[a] - 1)) return g->nc[a] - 1;
    return (int64_t)t;
}

static int64_t grid_cell(const orc_grid *g, int64_t cx, int64_t cy, int64_t cz)
{
    return (cz * g->nc[1] + cy) * g->nc[0] + cx;
}

/* Uniform grid over the bounding box with about `per_cell` particles per cell
 * on average (at most about 8 cells per particle). */
static void grid_build(orc_grid *g, int64_t n, const double *x, const double *y,
                       const double *z, double per_cell)
{
    const double *p[3] = {x, y, z};
    double hi[3], ext = 0.0, vol = 1.0;
    for (int a = 0; a < 3; ++a) {
        g->lo[a] = INFINITY;
        hi[a] = -INFINITY;
        for (int64_t i = 0; i < n; ++i) {
            if (p[a][i] < g->lo[a]) g->lo[a] = p[a][i];
            if (p[a][i] > hi[a]) hi[a] = p[a][i];
        }
        if (hi[a] - g->lo[a] > ext) ext = hi[a] - g->lo[a];
    }
    if (!(ext > 0.0)) ext = 1.0;
    for (int a = 0; a < 3; ++a) {
        double e = hi[a] - g->lo[a];
        vol *= e > 1e-6 * ext ? e : 1e-6 * ext;
    }
    g->c = cbrt(vol * per_cell / (double)n);
    for (;;) {
        double cells = 1.0;
        for (int a = 0; a < 3; ++a) {
            g->nc[a] = (int64_t)floor((hi[a] - g->lo[a]) / g->c) + 1;
            cells *= (double)g->nc[a];
        }
        if (cells <= 8.0 * (double)n + 64.0) break;
        g->c *= 1.25;
    }
    int64_t ncell = g->nc[0] * g->nc[1] * g->nc[2];
    int64_t *cell = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    g->start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    g->item = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        cell[i] = grid_cell(g, grid_axis(g, x[i], 0), grid_axis(g, y[i], 1), grid_axis(g, z[i], 2));
        ++g->start[cell[i] + 1];
    }
    for (int64_t q = 0; q < ncell; ++q) g->start[q + 1] += g->start[q];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)ncell);
    memcpy(fill, g->start, sizeof(int64_t) * (size_t)ncell);
    for (int64_t i = 0; i < n; ++i) g->item[fill[cell[i]]++] = i;
    free(fill);
    free(cell);
}

static void grid_free(orc_grid *g)
{
    free(g->start);
    free(g->item);
}

/* The k nearest neighbours by (d2, id) as orc_knn, searching cubic shells of
 * cells around the particle's cell: after shell s every unvisited particle is
 * at least s cell sizes away, so the search stops once the k-th distance is
 * below that. */
void orc_knn_grid(int64_t n, const double *x, const double *y, const double *z,
                  const uint32_t *id, int32_t k, double *h)
{
    orc_grid g;
    grid_build(&g, n, x, y, z, k > 8 ? (double)k / 8.0 : 1.0);
#pragma omp parallel
    {
        double *bd = (double *)malloc(sizeof(double) * (size_t)k);
        uint32_t *bi = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)k);
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < n; ++i) {
            const int64_t hx = grid_axis(&g, x[i], 0), hy = grid_axis(&g, y[i], 1),
                          hz = grid_axis(&g, z[i], 2);
            int32_t cnt = 0;
            for (int64_t s = 0;; ++s) {
                for (int64_t cx = hx - s; cx <= hx + s; ++cx) {
                    if (cx < 0 || cx >= g.nc[0]) continue;
                    for (int64_t cy = hy - s; cy <= hy + s; ++cy) {
                        if (cy < 0 || cy >= g.nc[1]) continue;
                        const int face = (cx == hx - s || cx == hx + s || cy == hy - s || cy == hy + s);
                        for (int64_t cz = hz - s; cz <= hz + s; cz += face ? 1 : 2 * s) {
                            if (cz >= 0 && cz < g.nc[2]) {
                                const int64_t q = grid_cell(&g, cx, cy, cz);
                                for (int64_t t = g.start[q]; t < g.start[q + 1]; ++t) {
                                    const int64_t j = g.item[t];
                                    if (j == i) continue;
                                    double dx = x[j] - x[i], dy = y[j] - y[i], dz = z[j] - z[i];
                                    double d2 = (dx * dx + dy * dy) + dz * dz;
                                    if (cnt == k && !key_less(d2, id[j], bd[k - 1], bi[k - 1])) continue;
                                    int32_t pos = cnt < k ? cnt : k - 1;
                                    while (pos > 0 && key_less(d2, id[j], bd[pos - 1], bi[pos - 1])) {
                                        bd[pos] = bd[pos - 1];
                                        bi[pos] = bi[pos - 1];
                                        --pos;
                                    }
                                    bd[pos] = d2;
                                    bi[pos] = id[j];
                                    if (cnt < k) ++cnt;
                                }
                            }
                            if (s == 0) break;
                        }
                    }
                }
                const double reach = (double)s * g.c;
                if (cnt == k && bd[k - 1] < reach * reach * (1.0 - 1e-9)) break;
                if (hx - s <= 0 && hx + s >= g.nc[0] - 1 && hy - s <= 0 && hy + s >= g.nc[1] - 1 &&
                    hz - s <= 0 && hz + s >= g.nc[2] - 1)
                    break;
            }
            h[i] = sqrt(bd[k - 1]);
        }
        free(bd);
        free(bi);
    }
    grid_free(&g);
}

typedef struct {
    double v;
    int64_t i;
} orc_key;

static int cmp_key(const void *pa, const void *pb)
{
    const orc_key *a = (const orc_key *)pa, *b = (const orc_key *)pb;
    if (a->v != b->v) return a->v < b->v ? -1 : 1;
    return a->i < b->i ? -1 : (a->i > b->i);
}

/* The events of orc_find_events (all pairs, no query set) with the same pair
 * test and arithmetic.  A pair with d < h_i + h_j has d < 2 max(h_i, h_j), so
 * it is found from its member with the larger h (the larger index on ties)
 * among the particles whose x lies within twice that h: a sweep over the
 * particles sorted by x. */
int64_t orc_find_events_sweep(int64_t n, const double *x, const double *y, const double *z,
                              const double *vx, const double *vy, const double *vz,
                              const double *m, const uint32_t *id, const double *h,
                              double sigma_m, double sigma_w, double dt, uint64_t seed,
                              uint32_t step, orc_event *ev, int64_t cap, int64_t *n_pairs,
                              int64_t *n_p_gt1)
{
    orc_key *ord = (orc_key *)malloc(sizeof(orc_key) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        ord[i].v = x[i];
        ord[i].i = i;
    }
    qsort(ord, (size_t)n, sizeof(orc_key), cmp_key);
    int64_t found = 0, pairs = 0, pgt1 = 0;
    orc_event *all = NULL;
    int64_t all_cap = 0;
#pragma omp parallel
    {
        int64_t my_pairs = 0, my_pgt1 = 0, my_n = 0, my_cap = 64;
        orc_event *mine = (orc_event *)malloc(sizeof(orc_event) * (size_t)my_cap);
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < n; ++i) {
            const double R = 2.0 * h[i] * (1.0 + 1e-9);
            /* first position with x >= x_i - R */
            int64_t lo = 0, hi = n;
            while (lo < hi) {
                int64_t mid = lo + (hi - lo) / 2;
                if (ord[mid].v < x[i] - R) lo = mid + 1;
                else hi = mid;
            }
            for (int64_t t = lo; t < n && ord[t].v <= x[i] + R; ++t) {
                const int64_t j = ord[t].i;
                if (j == i) continue;
                if (!(h[j] < h[i] || (h[j] == h[i] && j < i))) continue;
                const int64_t lo_i = i < j ? i : j, hi_i = i < j ? j : i;
                double dx = x[hi_i] - x[lo_i], dy = y[hi_i] - y[lo_i], dz = z[hi_i] - z[lo_i];
                double d2 = (dx * dx + dy * dy) + dz * dz;
                double hs = h[lo_i] + h[hi_i];
                if (!(d2 < hs * hs)) continue;
                ++my_pairs;
                int64_t ia = id[lo_i] < id[hi_i] ? lo_i : hi_i;
                int64_t ib = id[lo_i] < id[hi_i] ? hi_i : lo_i;
                uint32_t a = id[ia], b = id[ib];
                double u = orc_accept_u(seed, step, a, b);
                double gx = vx[ia] - vx[ib], gy = vy[ia] - vy[ib], gz = vz[ia] - vz[ib];
                double gg = sqrt((gx * gx + gy * gy) + gz * gz);
                double lam = orc_lambda(sqrt(d2), h[ia], h[ib]);
                double P = orc_sigma(sigma_m, sigma_w, gg) * m[ib] * gg * lam * dt;
                if (P > 1.0) ++my_pgt1;
                if (u < P) {
                    if (my_n == my_cap) {
                        my_cap *= 2;
                        mine = (orc_event *)realloc(mine, sizeof(orc_event) * (size_t)my_cap);
                    }
                    orc_event e = {a, b, ia, ib, u, P};
                    mine[my_n++] = e;
                }
            }
        }
#pragma omp critical
        {
            if (found + my_n > all_cap) {
                all_cap = 2 * (found + my_n) + 64;
                all = (orc_event *)realloc(all, sizeof(orc_event) * (size_t)all_cap);
            }
            memcpy(all + found, mine, sizeof(orc_event) * (size_t)my_n);
            found += my_n;
            pairs += my_pairs;
            pgt1 += my_pgt1;
        }
        free(mine);
    }
    free(ord);
    if (found > 0) qsort(all, (size_t)found, sizeof(orc_event), cmp_event);
    int64_t stored = found < cap ? found : cap;
    if (stored > 0 && ev) memcpy(ev, all, sizeof(orc_event) * (size_t)stored);
    free(all);
    if (n_pairs) *n_pairs = pairs;
    if (n_p_gt1) *n_p_gt1 = pgt1;
    return found;
}

/* ------------------------------------------------------------------------ */
/* The paper's tree (Sec. 2): a one-sided oct-tree with the relative opening
 * criterion, walked per particle (see the header). */

typedef struct {
    double c[3], half;      /* cube centre and half side                        */
    double M, cm[3];        /* mass and centre of mass                          */
    int64_t begin, end;     /* the cell's particles: idx[begin .. end)          */
    int64_t child[8];       /* -1: no particle in that octant                    */
    int leaf;
} oct_cell;

typedef struct {
    const double *x, *y, *z, *m;
    int64_t *idx;
    oct_cell *cell;
    int64_t n_cell, cap;
} oct_tree;

enum { OCT_MAX_DEPTH = 60 };

static int64_t oct_build(oct_tree *T, int64_t begin, int64_t end, const double c[3], double half,
                         int depth)
{
    if (T->n_cell == T->cap) {
        T->cap = T->cap ? 2 * T->cap : 1024;
        T->cell = (oct_cell *)realloc(T->cell, sizeof(oct_cell) * (size_t)T->cap);
    }
    const int64_t id = T->n_cell++;
    oct_cell C;
    for (int a = 0; a < 3; ++a) C.c[a] = c[a];
    C.half = half;
    C.begin = begin;
    C.end = end;
    C.M = 0.0;
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int64_t q = begin; q < end; ++q) {
        const int64_t i = T->idx[q];
        C.M += T->m[i];
        sx += T->m[i] * T->x[i];
        sy += T->m[i] * T->y[i];
        sz += T->m[i] * T->z[i];
    }
    C.cm[0] = sx / C.M;
    C.cm[1] = sy / C.M;
    C.cm[2] = sz / C.M;
    for (int o = 0; o < 8; ++o) C.child[o] = -1;
    C.leaf = (end - begin <= 1 || depth >= OCT_MAX_DEPTH);
    if (!C.leaf) {
        /* counting sort of the particles into the octants, in index order */
        int64_t cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        int *oct = (int *)malloc(sizeof(int) * (size_t)(end - begin));
        for (int64_t q = begin; q < end; ++q) {
            const int64_t i = T->idx[q];
            const int o = (T->x[i] >= c[0] ? 1 : 0) | (T->y[i] >= c[1] ? 2 : 0) |
                          (T->z[i] >= c[2] ? 4 : 0);
            oct[q - begin] = o;
            ++cnt[o];
        }
        int64_t start[8], fill[8], acc = begin;
        for (int o = 0; o < 8; ++o) {
            start[o] = fill[o] = acc;
            acc += cnt[o];
        }
        int64_t *tmp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(end - begin));
        for (int64_t q = begin; q < end; ++q) tmp[fill[oct[q - begin]]++ - begin] = T->idx[q];
        memcpy(T->idx + begin, tmp, sizeof(int64_t) * (size_t)(end - begin));
        free(tmp);
        free(oct);
        for (int o = 0; o < 8; ++o) {
            if (cnt[o] == 0) continue;
            const double h2 = 0.5 * half;
            const double cc[3] = {c[0] + ((o & 1) ? h2 : -h2), c[1] + ((o & 2) ? h2 : -h2),
                                  c[2] + ((o & 4) ? h2 : -h2)};
            C.child[o] = oct_build(T, start[o], start[o] + cnt[o], cc, h2, depth + 1);
        }
    }
    T->cell[id] = C;
    return id;
}

typedef struct {
    double ax, ay, az, pot;
    int64_t terms;
} oct_acc;

static void oct_term(oct_acc *A, double dx, double dy, double dz, double mj, double eps2)
{
    const double r2 = ((dx * dx + dy * dy) + dz * dz) + eps2;
    const double rinv = 1.0 / sqrt(r2);
    const double f = mj * rinv * rinv * rinv;
    A->ax += f * dx;
    A->ay += f * dy;
    A->az += f * dz;
    A->pot -= mj * rinv;
    ++A->terms;
}

static void oct_walk(const oct_tree *T, int64_t id, int64_t i, double GMcrit, double eps2,
                     oct_acc *A)
{
    const oct_cell *C = &T->cell[id];
    const double xi = T->x[i], yi = T->y[i], zi = T->z[i];
    if (C->leaf) {
        for (int64_t q = C->begin; q < C->end; ++q) {
            const int64_t j = T->idx[q];
            if (j == i) continue;
            oct_term(A, T->x[j] - xi, T->y[j] - yi, T->z[j] - zi, T->m[j], eps2);
        }
        return;
    }
    const int inside = fabs(xi - C->c[0]) <= C->half && fabs(yi - C->c[1]) <= C->half &&
                       fabs(zi - C->c[2]) <= C->half;
    if (!inside) {
        const double dx = C->cm[0] - xi, dy = C->cm[1] - yi, dz = C->cm[2] - zi;
        const double r2 = (dx * dx + dy * dy) + dz * dz;
        const double l = 2.0 * C->half;
        /* G M l^2 <= alpha |a_old| r^4; GMcrit = alpha |a_old| / G */
        if (C->M * l * l <= GMcrit * r2 * r2) {
            oct_term(A, dx, dy, dz, C->M, eps2);
            return;
        }
    }
    for (int o = 0; o < 8; ++o)
        if (C->child[o] >= 0) oct_walk(T, C->child[o], i, GMcrit, eps2, A);
}

void orc_octree_gravity(int64_t n, const double *x, const double *y, const double *z,
                        const double *m, const double *ax_old, const double *ay_old,
                        const double *az_old, double G, double eps, double alpha, int64_t nq,
                        const int64_t *q, double *ax, double *ay, double *az, double *pot,
                        int64_t *terms)
{
    if (q == NULL) nq = n;
    oct_tree T = {x, y, z, m, NULL, NULL, 0, 0};
    T.idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    const double *p[3] = {x, y, z};
    for (int64_t i = 0; i < n; ++i) {
        T.idx[i] = i;
        for (int a = 0; a < 3; ++a) {
            if (p[a][i] < lo[a]) lo[a] = p[a][i];
            if (p[a][i] > hi[a]) hi[a] = p[a][i];
        }
    }
    double c[3], half = 0.0;
    for (int a = 0; a < 3; ++a) {
        c[a] = 0.5 * (lo[a] + hi[a]);
        if (0.5 * (hi[a] - lo[a]) > half) half = 0.5 * (hi[a] - lo[a]);
    }
    half = half > 0.0 ? half * (1.0 + 1e-9) : 1.0;
    if (n > 0) oct_build(&T, 0, n, c, half, 0);
    const double eps2 = eps * eps;
    int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : total)
    for (int64_t t = 0; t < nq; ++t) {
        const int64_t i = q ? q[t] : t;
        const double a2 = (ax_old[i] * ax_old[i] + ay_old[i] * ay_old[i]) + az_old[i] * az_old[i];
        const double GMcrit = G != 0.0 ? alpha * sqrt(a2) / G : 0.0;
        oct_acc A = {0.0, 0.0, 0.0, 0.0, 0};
        oct_walk(&T, 0, i, GMcrit, eps2, &A);
        ax[t] = G * A.ax;
        ay[t] = G * A.ay;
        az[t] = G * A.az;
        pot[t] = G * A.pot;
        total += A.terms;
    }
    if (terms) *terms = total;
    free(T.idx);
    free(T.cell);
}

/* ------------------------------------------------------------------------ */
/* Exact searches over a k-d tree (for full-size runs).  Like the grid and the
 * sweep they change only the order in which candidates are examined: every
 * distance, the (d2, id) order and the pair test are the expressions of the
 * brute-force definitions.  A subtree is skipped only when the squared
 * distance from the particle to its box (the same expression on the box's
 * gaps, which rounding cannot make larger than any member's d2) already rules
 * out every member. */

typedef struct {
    double lo[3], hi[3];    /* bounding box of the node's particles            */
    double hmin;            /* smallest h among them (event search; else 0)     */
    int64_t begin, end;     /* the node's particles: idx[begin .. end)          */
    int64_t left, right;    /* children, -1 for a leaf                           */
} kd_node;

typedef struct {
    const double *p[3];
    const double *h;
    int64_t *idx;
    double *q[3];           /* the positions in tree order: q[a][s] = p[a][idx[s]] */
    double *qh;             /* h in tree order (event search)                      */
    kd_node *node;
    int64_t n_node, cap;
} kd_tree;

enum { KD_LEAF = 16 };

/* i before j along axis a (ties by index, so every key is distinct) */
static int kd_before(const kd_tree *t, int a, int64_t i, int64_t j)
{
    const double u = t->p[a][i], v = t->p[a][j];
    return u < v || (u == v && i < j);
}

/* Rearranges idx[lo, hi) so that position k holds the element of rank k - lo
 * along axis a, smaller ones before it and larger ones after it. */
static void kd_select(kd_tree *t, int a, int64_t lo, int64_t hi, int64_t k)
{
    int64_t *v = t->idx;
    while (hi - lo > 1) {
        const int64_t mid = lo + (hi - lo) / 2;
        int64_t tmp = v[mid]; v[mid] = v[hi - 1]; v[hi - 1] = tmp;
        const int64_t pv = v[hi - 1];
        int64_t s = lo;
        for (int64_t i = lo; i < hi - 1; ++i)
            if (kd_before(t, a, v[i], pv)) {
                tmp = v[i]; v[i] = v[s]; v[s] = tmp;
                ++s;
            }
        tmp = v[s]; v[s] = v[hi - 1]; v[hi - 1] = tmp;
        if (k == s) return;
        if (k < s) hi = s;
        else lo = s + 1;
    }
}

static int64_t kd_new(kd_tree *t)
{
    if (t->n_node == t->cap) {
        t->cap = t->cap ? 2 * t->cap : 64;
        t->node = (kd_node *)realloc(t->node, sizeof(kd_node) * (size_t)t->cap);
    }
    return t->n_node++;
}

/* Node over idx[begin, end): its box, then a split at the median of the
 * longest side while it holds more than KD_LEAF particles. */
static int64_t kd_build_node(kd_tree *t, int64_t begin, int64_t end)
{
    const int64_t nd = kd_new(t);
    kd_node N;
    for (int a = 0; a < 3; ++a) {
        N.lo[a] = INFINITY;
        N.hi[a] = -INFINITY;
    }
    N.hmin = INFINITY;
    for (int64_t q = begin; q < end; ++q) {
        const int64_t i = t->idx[q];
        for (int a = 0; a < 3; ++a) {
            if (t->p[a][i] < N.lo[a]) N.lo[a] = t->p[a][i];
            if (t->p[a][i] > N.hi[a]) N.hi[a] = t->p[a][i];
        }
        if (t->h && t->h[i] < N.hmin) N.hmin = t->h[i];
    }
    if (!t->h) N.hmin = 0.0;
    N.begin = begin;
    N.end = end;
    N.left = N.right = -1;
    if (end - begin > KD_LEAF) {
        int a = 0;
        for (int c = 1; c < 3; ++c)
            if (N.hi[c] - N.lo[c] > N.hi[a] - N.lo[a]) a = c;
        const int64_t mid = begin + (end - begin) / 2;
        kd_select(t, a, begin, end, mid);
        N.left = kd_build_node(t, begin, mid);
        N.right = kd_build_node(t, mid, end);
    }
    t->node[nd] = N;
    return nd;
}

static void kd_build(kd_tree *t, int64_t n, const double *x, const double *y, const double *z,
                     const double *h)
{
    t->p[0] = x;
    t->p[1] = y;
    t->p[2] = z;
    t->h = h;
    t->idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) t->idx[i] = i;
    t->node = NULL;
    t->n_node = t->cap = 0;
    kd_build_node(t, 0, n);
    /* copies in tree order, so that a leaf is read from consecutive memory */
    const size_t nn = (size_t)(n > 0 ? n : 1);
    for (int a = 0; a < 3; ++a) t->q[a] = (double *)malloc(sizeof(double) * nn);
    t->qh = h ? (double *)malloc(sizeof(double) * nn) : NULL;
    for (int64_t q = 0; q < n; ++q) {
        const int64_t i = t->idx[q];
        for (int a = 0; a < 3; ++a) t->q[a][q] = t->p[a][i];
        if (h) t->qh[q] = h[i];
    }
}

static void kd_free(kd_tree *t)
{
    free(t->idx);
    free(t->node);
    for (int a = 0; a < 3; ++a) free(t->q[a]);
    free(t->qh);
}

/* Squared distance from (x, y, z) to the node's box: the gaps per axis
 * combined as a candidate's d2 is.  For a member q, |fl(q - x)| is at least
 * the gap on each axis (rounding is monotone), so this is at most its d2. */
static double kd_box_d2(const kd_node *N, double x, double y, double z)
{
    const double p[3] = {x, y, z};
    double g[3];
    for (int a = 0; a < 3; ++a) {
        const double u = N->lo[a] - p[a], v = p[a] - N->hi[a];
        const double w = u > v ? u : v;
        g[a] = w > 0.0 ? w : 0.0;
    }
    return (g[0] * g[0] + g[1] * g[1]) + g[2] * g[2];
}

typedef struct {
    const uint32_t *id;
    double *bd;
    uint32_t *bi;
    int32_t k, cnt;
} kd_best;

/* The k best (d2, id) of particle i over the subtree, nearer child first. */
static void kd_knn_visit(const kd_tree *t, int64_t nd, int64_t i, kd_best *B)
{
    const kd_node *N = &t->node[nd];
    const double *x = t->p[0], *y = t->p[1], *z = t->p[2];
    const int32_t k = B->k;
    if (B->cnt == k && kd_box_d2(N, x[i], y[i], z[i]) > B->bd[k - 1]) return;
    if (N->left < 0) {
        const double *qx = t->q[0], *qy = t->q[1], *qz = t->q[2];
        for (int64_t q = N->begin; q < N->end; ++q) {
            const int64_t j = t->idx[q];
            if (j == i) continue;
            double dx = qx[q] - x[i], dy = qy[q] - y[i], dz = qz[q] - z[i];
            double d2 = (dx * dx + dy * dy) + dz * dz;
            if (B->cnt == k && !key_less(d2, B->id[j], B->bd[k - 1], B->bi[k - 1])) continue;
            int32_t pos = B->cnt < k ? B->cnt : k - 1;
            while (pos > 0 && key_less(d2, B->id[j], B->bd[pos - 1], B->bi[pos - 1])) {
                B->bd[pos] = B->bd[pos - 1];
                B->bi[pos] = B->bi[pos - 1];
                --pos;
            }
            B->bd[pos] = d2;
            B->bi[pos] = B->id[j];
            if (B->cnt < k) ++B->cnt;
        }
        return;
    }
    const double dl = kd_box_d2(&t->node[N->left], x[i], y[i], z[i]);
    const double dr = kd_box_d2(&t->node[N->right], x[i], y[i], z[i]);
    if (dl <= dr) {
        kd_knn_visit(t, N->left, i, B);
        kd_knn_visit(t, N->right, i, B);
    } else {
        kd_knn_visit(t, N->right, i, B);
        kd_knn_visit(t, N->left, i, B);
    }
}

void orc_knn_tree(int64_t n, const double *x, const double *y, const double *z,
                  const uint32_t *id, int32_t k, double *h, uint32_t *nbr)
{
    kd_tree t;
    kd_build(&t, n, x, y, z, NULL);
#pragma omp parallel
    {
        kd_best B;
        B.id = id;
        B.k = k;
        B.bd = (double *)malloc(sizeof(double) * (size_t)k);
        B.bi = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)k);
#pragma omp for schedule(dynamic, 256)
        for (int64_t s = 0; s < n; ++s) {
            const int64_t i = t.idx[s];   /* in tree order: neighbours share the walk */
            B.cnt = 0;
            kd_knn_visit(&t, 0, i, &B);
            h[i] = sqrt(B.bd[k - 1]);
            if (nbr) memcpy(nbr + (size_t)i * (size_t)k, B.bi, sizeof(uint32_t) * (size_t)k);
        }
        free(B.bd);
        free(B.bi);
    }
    kd_free(&t);
}

/* Per-thread event collection of the tree search. */
typedef struct {
    const double *x, *y, *z, *vx, *vy, *vz, *m, *h;
    const uint32_t *id;
    double sigma_m, sigma_w, dt;
    uint64_t seed;
    uint32_t step;
    int64_t pairs, pgt1, n, cap;
    orc_event *ev;
} kd_pairs;

/* The pair {i, j} as orc_find_events tests and decides it (indices ordered
 * for the differences, ids for the roles a and b).  The overlap integral is
 * evaluated only when the draw lies below an upper bound of P: Lambda is at
 * most the smaller of the two kernels' central values, 8 / (pi max(h)^3), so
 * a draw at or above that bound (with a margin far beyond rounding) can be
 * neither an event nor a pair with P > 1 (the bound is then below 1). */
static void kd_pair(kd_pairs *C, int64_t i, int64_t j)
{
    const int64_t lo_i = i < j ? i : j, hi_i = i < j ? j : i;
    const double *x = C->x, *y = C->y, *z = C->z, *h = C->h;
    double dx = x[hi_i] - x[lo_i], dy = y[hi_i] - y[lo_i], dz = z[hi_i] - z[lo_i];
    double d2 = (dx * dx + dy * dy) + dz * dz;
    double hs = h[lo_i] + h[hi_i];
    if (!(d2 < hs * hs)) return;
    ++C->pairs;
    const int64_t ia = C->id[lo_i] < C->id[hi_i] ? lo_i : hi_i;
    const int64_t ib = C->id[lo_i] < C->id[hi_i] ? hi_i : lo_i;
    const uint32_t a = C->id[ia], b = C->id[ib];
    const double u = orc_accept_u(C->seed, C->step, a, b);
    double gx = C->vx[ia] - C->vx[ib], gy = C->vy[ia] - C->vy[ib], gz = C->vz[ia] - C->vz[ib];
    double gg = sqrt((gx * gx + gy * gy) + gz * gz);
    const double sg = orc_sigma(C->sigma_m, C->sigma_w, gg);
    const double hm = h[ia] > h[ib] ? h[ia] : h[ib];
    const double bound = sg * C->m[ib] * gg * (8.0 / (M_PI * hm * hm * hm)) * C->dt * (1.0 + 1e-6);
    if (!(u < bound)) return;
    double lam = orc_lambda(sqrt(d2), h[ia], h[ib]);
    double P = sg * C->m[ib] * gg * lam * C->dt;
    if (P > 1.0) ++C->pgt1;
    if (u < P) {
        if (C->n == C->cap) {
            C->cap = C->cap ? 2 * C->cap : 64;
            C->ev = (orc_event *)realloc(C->ev, sizeof(orc_event) * (size_t)C->cap);
        }
        orc_event e = {a, b, ia, ib, u, P};
        C->ev[C->n++] = e;
    }
}

/* A pair with d < h_i + h_j has d < 2 max(h_i, h_j): it is found from its
 * member with the larger h (the larger index on ties), among the particles
 * within twice that h. */
static void kd_pairs_visit(const kd_tree *t, int64_t nd, int64_t i, double R2, kd_pairs *C)
{
    const kd_node *N = &t->node[nd];
    const double *h = C->h;
    if (N->hmin > h[i] || kd_box_d2(N, C->x[i], C->y[i], C->z[i]) > R2) return;
    if (N->left < 0) {
        const double hi = h[i];
        for (int64_t q = N->begin; q < N->end; ++q) {
            const double hj = t->qh[q];
            if (!(hj <= hi)) continue;
            const int64_t j = t->idx[q];
            if (j == i || (hj == hi && j > i)) continue;
            kd_pair(C, i, j);
        }
        return;
    }
    kd_pairs_visit(t, N->left, i, R2, C);
    kd_pairs_visit(t, N->right, i, R2, C);
}

int64_t orc_find_events_tree(int64_t n, const double *x, const double *y, const double *z,
                             const double *vx, const double *vy, const double *vz,
                             const double *m, const uint32_t *id, const double *h,
                             double sigma_m, double sigma_w, double dt, uint64_t seed,
                             uint32_t step, orc_event *ev, int64_t cap, int64_t *n_pairs,
                             int64_t *n_p_gt1)
{
    kd_tree t;
    kd_build(&t, n, x, y, z, h);
    int64_t found = 0, pairs = 0, pgt1 = 0;
    orc_event *all = NULL;
    int64_t all_cap = 0;
#pragma omp parallel
    {
        kd_pairs C = {x, y, z, vx, vy, vz, m, h, id, sigma_m, sigma_w, dt, seed, step,
                      0, 0, 0, 0, NULL};
#pragma omp for schedule(dynamic, 256)
        for (int64_t s = 0; s < n; ++s) {
            const int64_t i = t.idx[s];
            const double R = 2.0 * h[i] * (1.0 + 1e-9);
            kd_pairs_visit(&t, 0, i, R * R, &C);
        }
#pragma omp critical
        {
            if (found + C.n > all_cap) {
                all_cap = 2 * (found + C.n) + 64;
                all = (orc_event *)realloc(all, sizeof(orc_event) * (size_t)all_cap);
            }
            if (C.n > 0) memcpy(all + found, C.ev, sizeof(orc_event) * (size_t)C.n);
            found += C.n;
            pairs += C.pairs;
            pgt1 += C.pgt1;
        }
        free(C.ev);
    }
    kd_free(&t);
    if (found > 0) qsort(all, (size_t)found, sizeof(orc_event), cmp_event);
    int64_t stored = found < cap ? found : cap;
    if (stored > 0 && ev) memcpy(ev, all, sizeof(orc_event) * (size_t)stored);
    free(all);
    if (n_pairs) *n_pairs = pairs;
    if (n_p_gt1) *n_p_gt1 = pgt1;
    return found;
}

/* ------------------------------------------------------------------------ */
/* Central density (Sec. 3: the halo centre is the minimum of the
 * gravitational potential).  Reading: the centre is the particle with the
 * lowest self-potential phi (first index on ties); the density is the mass
 * within `radius` of it (that particle included, d2 as in the kNN) over the
 * sphere's volume. */
void orc_central_density(int64_t n, const double *x, const double *y, const double *z,
                         const double *m, const double *phi, double radius,
                         int64_t *center, int64_t *count, double *mass)
{
    int64_t c = -1;
    for (int64_t i = 0; i < n; ++i)
        if (phi[i] == phi[i] && (c < 0 || phi[i] < phi[c])) c = i;
    *center = c;
    *count = 0;
    *mass = 0.0;
    if (c < 0) return;
    const double r2 = radius * radius;
    neum acc = {0.0, 0.0};
    int64_t cnt = 0;
    for (int64_t j = 0; j < n; ++j) {
        double dx = x[j] - x[c], dy = y[j] - y[c], dz = z[j] - z[c];
        double d2 = (dx * dx + dy * dy) + dz * dz;
        if (d2 <= r2) {
            ++cnt;
            neum_add(&acc, m[j]);
        }
    }
    *count = cnt;
    *mass = neum_get(&acc);
}

/* ------------------------------------------------------------------------ */
/* Tidal radius (Eq. tidal_radius): G M(<= r) / r^2 equals the difference of
 * the host's acceleration across the satellite, |grad Phi(c + r n) -
 * grad Phi(c - r n)|.  Readings: c is the particle with the lowest self-
 * potential (as the central density), n the unit vector from the host centre
 * to c, M(<= r) the mass with d2 <= r^2; the equation is solved by 60
 * bisection steps in log r between 2^-40 (2 r_max) and 2 r_max (r_max the
 * farthest particle), r_tidal being the final upper bracket.  Returns 1 if the
 * tides do not win even at 2 r_max, else 0. */
static double mass_within(int64_t n, const double *x, const double *y, const double *z,
                          const double *m, int64_t c, double r)
{
    neum acc = {0.0, 0.0};
    for (int64_t j = 0; j < n; ++j) {
        double dx = x[j] - x[c], dy = y[j] - y[c], dz = z[j] - z[c];
        if ((dx * dx + dy * dy) + dz * dz <= r * r) neum_add(&acc, m[j]);
    }
    return neum_get(&acc);
}

int orc_tidal_radius(int64_t n, const double *x, const double *y, const double *z,
                     const double *m, const double *phi, const orc_params *p,
                     double *r_tidal, double *mass, int64_t *center)
{
    int64_t c = -1;
    for (int64_t i = 0; i < n; ++i)
        if (phi[i] == phi[i] && (c < 0 || phi[i] < phi[c])) c = i;
    *center = c;
    *r_tidal = 0.0;
    *mass = 0.0;
    if (c < 0) return 1;
    double ux = x[c] - p->host_c[0], uy = y[c] - p->host_c[1], uz = z[c] - p->host_c[2];
    double u = sqrt((ux * ux + uy * uy) + uz * uz);
    double nx = u > 0.0 ? ux / u : 1.0, ny = u > 0.0 ? uy / u : 0.0, nz = u > 0.0 ? uz / u : 0.0;
    double rmax2 = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        double dx = x[j] - x[c], dy = y[j] - y[c], dz = z[j] - z[c];
        double d2 = (dx * dx + dy * dy) + dz * dz;
        if (d2 > rmax2) rmax2 = d2;
    }
    double hi = 2.0 * sqrt(rmax2), hi0 = hi, lo = ldexp(hi, -40);
    for (int it = 0; it < 60; ++it) {
        double r = sqrt(lo * hi);
        double px[2] = {x[c] + r * nx, x[c] - r * nx}, py[2] = {y[c] + r * ny, y[c] - r * ny};
        double pz[2] = {z[c] + r * nz, z[c] - r * nz};
        double ax[2], ay[2], az[2], pp[2];
        orc_host_field(2, px, py, pz, p, ax, ay, az, pp);
        double gx = ax[0] - ax[1], gy = ay[0] - ay[1], gz = az[0] - az[1];
        double tide = sqrt((gx * gx + gy * gy) + gz * gz);
        if (p->G * mass_within(n, x, y, z, m, c, r) / (r * r) > tide) lo = r;
        else hi = r;
    }
    *r_tidal = hi;
    *mass = mass_within(n, x, y, z, m, c, hi);
    return hi == hi0 ? 1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Total acceleration and potential at the current positions: self-gravity plus
 * the static host. */
/* Self-gravity of all particles: the direct sum, or the tree with the
 * accelerations held in (ax, ay, az) on entry as a_old. */
static void self_gravity(int64_t n, const double *x, const double *y, const double *z,
                         const double *m, const orc_params *p, double *ax, double *ay,
                         double *az, double *pot)
{
    if (p->tree_alpha > 0.0) {
        double *t = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * 4);
        double *tx = t, *ty = t + n, *tz = t + 2 * n, *tp = t + 3 * n;
        orc_tree_gravity(n, x, y, z, m, ax, ay, az, p->G, p->eps, p->tree_alpha, n, NULL, tx,
                         ty, tz, tp, NULL);
        memcpy(ax, tx, sizeof(double) * (size_t)n);
        memcpy(ay, ty, sizeof(double) * (size_t)n);
        memcpy(az, tz, sizeof(double) * (size_t)n);
        memcpy(pot, tp, sizeof(double) * (size_t)n);
        free(t);
        return;
    }
    orc_gravity(n, x, y, z, m, p->G, p->eps, n, NULL, ax, ay, az, pot, NULL);
}

static void accel_total(int64_t n, const double *x, const double *y, const double *z,
                        const double *m, const orc_params *p,
                        double *ax, double *ay, double *az, double *pot)
{
    self_gravity(n, x, y, z, m, p, ax, ay, az, pot);
    if (p->host_kind != 0) {
        double *hx = (double *)malloc(sizeof(double) * (size_t)n * 4);
        double *hy = hx + n, *hz = hy + n, *hp = hz + n;
        orc_host_field(n, x, y, z, p, hx, hy, hz, hp);
        for (int64_t i = 0; i < n; ++i) {
            ax[i] += hx[i];
            ay[i] += hy[i];
            az[i] += hz[i];
            pot[i] += hp[i];
        }
        free(hx);
    }
}

/* Block time steps (Sec. 2: individual time steps with the gravitational
 * criterion eta, Springel 2005 eq. 34, and a minimum step dt_min; the paper
 * traces an energy error to the way steps change, Sec. 3.1).  Readings: a
 * particle's step is s = dt / 2^b, the longest one with s^2 |a| <= 2 eta eps
 * (b <= max_bin), lengthened again while it is shorter than dt_min.  One
 * cycle of length dt starts and ends synchronised and is cut into T = 2^max_bin
 * ticks: every particle drifts each tick; a particle is active at tick k when k
 * is a multiple of its step in ticks; an active particle gets its forces at
 * the current positions, its closing half kick with the old step, a new bin
 * from the criterion (a longer step only when k is a multiple of it) and,
 * before the cycle ends, its opening half kick with the new step. */
int32_t orc_bin(double dt, double eta, double eps, double dt_min, int32_t max_bin,
                double ax, double ay, double az)
{
    /* s^2 |a| <= 2 eta eps, squared on both sides: no square root, so the
     * integer decision is a fixed sequence of IEEE products and sums */
    const double a2 = (ax * ax + ay * ay) + az * az;
    const double lim = 2.0 * eta * eps;
    const double lim2 = lim * lim;
    int32_t b = 0;
    for (;;) {
        const double s = ldexp(dt, -b);
        const double s2 = s * s;
        if (b >= max_bin || !((s2 * s2) * a2 > lim2)) break;
        ++b;
    }
    while (b > 0 && ldexp(dt, -b) < dt_min) --b;
    return b;
}

/* reflecting sphere (Sec. 2): a particle beyond the radius that moves
 * outwards gets its radial velocity reversed, v -> v - 2 (v.d) d / |d|^2 */
static void reflect(int64_t n, const double *x, const double *y, const double *z, double *vx,
                    double *vy, double *vz, const orc_params *p)
{
    if (!(p->boundary_r > 0.0)) return;
    for (int64_t i = 0; i < n; ++i) {
        double dx = x[i] - p->boundary_c[0], dy = y[i] - p->boundary_c[1];
        double dz = z[i] - p->boundary_c[2];
        double d2 = (dx * dx + dy * dy) + dz * dz;
        double vd = (vx[i] * dx + vy[i] * dy) + vz[i] * dz;
        if (d2 > p->boundary_r * p->boundary_r && vd > 0.0) {
            double f = 2.0 * vd / d2;
            vx[i] -= f * dx;
            vy[i] -= f * dy;
            vz[i] -= f * dz;
        }
    }
}

static void half_kick(int64_t i, double *vx, double *vy, double *vz, const double *ax,
                      const double *ay, const double *az, double dt, int32_t b)
{
    double h = 0.5 * ldexp(dt, -b);
    vx[i] += ax[i] * h;
    vy[i] += ay[i] * h;
    vz[i] += az[i] * h;
}

/* One cycle of block time steps; on entry and exit every particle is
 * synchronised and (ax, ay, az, pot) hold the forces at the positions. */
static void block_cycle(int64_t n, double *x, double *y, double *z, double *vx, double *vy,
                        double *vz, const double *m, double *ax, double *ay, double *az,
                        double *pot, const orc_params *p)
{
    const int32_t B = p->max_bin;
    const int64_t T = (int64_t)1 << B;
    const double tau = ldexp(p->dt, -B);
    const size_t nn = (size_t)(n > 0 ? n : 1);
    int32_t *bin = (int32_t *)malloc(sizeof(int32_t) * nn);
    int64_t *act = (int64_t *)malloc(sizeof(int64_t) * nn);
    double *w = (double *)malloc(sizeof(double) * nn * 11);
    double *gx = w, *gy = gx + n, *gz = gy + n, *gp = gz + n;
    double *qx = gp + n, *qy = qx + n, *qz = qy + n;
    double *hx = qz + n, *hy = hx + n, *hz = hy + n, *hp = hz + n;
    for (int64_t i = 0; i < n; ++i) {
        bin[i] = orc_bin(p->dt, p->eta, p->eps, p->dt_min, B, ax[i], ay[i], az[i]);
        half_kick(i, vx, vy, vz, ax, ay, az, p->dt, bin[i]);
    }
    for (int64_t k = 1; k <= T; ++k) {
        for (int64_t i = 0; i < n; ++i) {
            x[i] += vx[i] * tau;
            y[i] += vy[i] * tau;
            z[i] += vz[i] * tau;
        }
        reflect(n, x, y, z, vx, vy, vz, p);
        int64_t na = 0;
        for (int64_t i = 0; i < n; ++i)
            if ((k & (((int64_t)1 << (B - bin[i])) - 1)) == 0) act[na++] = i;
        if (na == 0) continue;
        if (p->tree_alpha > 0.0) {
            /* the tree for everyone (a_old: the last accelerations of each
             * particle), kept for the active ones */
            double *t = (double *)malloc(sizeof(double) * nn * 8);
            double *tx = t, *ty = t + n, *tz = t + 2 * n, *tp = t + 3 * n;
            double *ox = t + 4 * n, *oy = t + 5 * n, *oz = t + 6 * n;
            memcpy(ox, ax, sizeof(double) * (size_t)n);
            memcpy(oy, ay, sizeof(double) * (size_t)n);
            memcpy(oz, az, sizeof(double) * (size_t)n);
            orc_tree_gravity(n, x, y, z, m, ox, oy, oz, p->G, p->eps, p->tree_alpha, n, NULL, tx,
                             ty, tz, tp, NULL);
            for (int64_t t2 = 0; t2 < na; ++t2) {
                gx[t2] = tx[act[t2]];
                gy[t2] = ty[act[t2]];
                gz[t2] = tz[act[t2]];
                gp[t2] = tp[act[t2]];
            }
            free(t);
        } else {
            orc_gravity(n, x, y, z, m, p->G, p->eps, na, act, gx, gy, gz, gp, NULL);
        }
        if (p->host_kind != 0) {
            for (int64_t t = 0; t < na; ++t) {
                qx[t] = x[act[t]];
                qy[t] = y[act[t]];
                qz[t] = z[act[t]];
            }
            orc_host_field(na, qx, qy, qz, p, hx, hy, hz, hp);
            for (int64_t t = 0; t < na; ++t) {
                gx[t] += hx[t];
                gy[t] += hy[t];
                gz[t] += hz[t];
                gp[t] += hp[t];
            }
        }
        for (int64_t t = 0; t < na; ++t) {
            const int64_t i = act[t];
            ax[i] = gx[t];
            ay[i] = gy[t];
            az[i] = gz[t];
            pot[i] = gp[t];
            half_kick(i, vx, vy, vz, ax, ay, az, p->dt, bin[i]);
            if (k == T) continue;
            int32_t nb = orc_bin(p->dt, p->eta, p->eps, p->dt_min, B, ax[i], ay[i], az[i]);
            while (nb < bin[i] && (k & (((int64_t)1 << (B - nb)) - 1)) != 0) ++nb;
            bin[i] = nb;
            half_kick(i, vx, vy, vz, ax, ay, az, p->dt, bin[i]);
        }
    }
    free(bin);
    free(act);
    free(w);
}

/* Opening half kick and drift of a fixed step: v += a dt/2, x += v dt, then
 * the reflecting sphere. */
void orc_kick_drift(int64_t n, double *x, double *y, double *z, double *vx, double *vy,
                    double *vz, const double *ax, const double *ay, const double *az,
                    const orc_params *p)
{
    const double hdt = 0.5 * p->dt;
    for (int64_t i = 0; i < n; ++i) {
        vx[i] += ax[i] * hdt;
        vy[i] += ay[i] * hdt;
        vz[i] += az[i] * hdt;
    }
    for (int64_t i = 0; i < n; ++i) {
        x[i] += vx[i] * p->dt;
        y[i] += vy[i] * p->dt;
        z[i] += vz[i] * p->dt;
    }
    reflect(n, x, y, z, vx, vy, vz, p);
}

/* Closing half kick of a fixed step: v += a dt/2. */
void orc_close_kick(int64_t n, double *vx, double *vy, double *vz, const double *ax,
                    const double *ay, const double *az, const orc_params *p)
{
    const double hdt = 0.5 * p->dt;
    for (int64_t i = 0; i < n; ++i) {
        vx[i] += ax[i] * hdt;
        vy[i] += ay[i] * hdt;
        vz[i] += az[i] * hdt;
    }
}

/* One step: K(dt/2) D(dt) [forces] K(dt/2), then the SIDM pass at the
 * synchronised point (reading: the paper does not state where scattering sits
 * inside the step; placing it after the closing kick keeps x fixed during the
 * pass, so the pass conserves energy exactly and sigma = 0 is plain KDK). */
int64_t orc_kdk_step(int64_t n, double *x, double *y, double *z,
                     double *vx, double *vy, double *vz, const double *m,
                     const uint32_t *id, double *ax, double *ay, double *az,
                     double *pot, double *h, const orc_params *p, uint32_t step,
                     orc_event *ev, int64_t ev_cap)
{
    if (p->eta > 0.0) {
        block_cycle(n, x, y, z, vx, vy, vz, m, ax, ay, az, pot, p);
        goto synchronised;
    }
    orc_kick_drift(n, x, y, z, vx, vy, vz, ax, ay, az, p);
    accel_total(n, x, y, z, m, p, ax, ay, az, pot);
    orc_close_kick(n, vx, vy, vz, ax, ay, az, p);
synchronised:
    orc_knn_tree(n, x, y, z, id, p->k, h, NULL);
    if (p->sigma_m == 0.0) return 0;
    int64_t cap = ev_cap > 0 ? ev_cap : 0;
    orc_event *buf = ev;
    int64_t found = orc_find_events_tree(n, x, y, z, vx, vy, vz, m, id, h, p->sigma_m,
                                         p->sigma_w, p->dt, p->seed, step, buf, cap, NULL,
                                         NULL);
    if (found > cap) {
        /* not enough room to hold the ordered list: collect it privately */
        buf = (orc_event *)malloc(sizeof(orc_event) * (size_t)found);
        orc_find_events_tree(n, x, y, z, vx, vy, vz, m, id, h, p->sigma_m, p->sigma_w, p->dt,
                             p->seed, step, buf, found, NULL, NULL);
    }
    orc_apply_events(found, buf, m, vx, vy, vz, p->seed, step);
    if (buf != ev) {
        free(buf);
        return -1;
    }
    return found;
}
