/*
 * sidm_oracle.h -- plain, slow, FP64 CPU reference for the SIDM N-body step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path links, loads or calls
 * this library: it exists so that tests, the smoke check and the CPU baseline
 * leg of the benchmark can compare the GPU library against a reading of the
 * paper (Fischer, Yu & Dolag, "Accurately simulating core-collapse
 * self-interacting dark matter halos") that a reader can check by eye.  It
 * shares no code, header, table or constant with the HIP library.
 *
 * Every array is host memory, halo-local (indices 0..n-1), structure of arrays,
 * double precision unless stated.  Particle identities `id` are unsigned 32-bit
 * and unique within a halo.
 */
#ifndef SIDM_ORACLE_H
#define SIDM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- counter-based random numbers (Philox4x32-10, Salmon et al. 2011) ---- */

/* One Philox4x32-10 block: 10 rounds of the 4x32 bijection keyed by `key`,
 * with the Weyl key schedule between rounds. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Uniform double in [0,1) from two 32-bit words: the top 53 bits of (hi:lo). */
double orc_u53(uint32_t hi, uint32_t lo);

/* The accept draw u for pair (a, b) with a < b at step `step`:
 * counter (a, b, step, 0), key (lo32(seed), hi32(seed)), u = u53(w0, w1). */
double orc_accept_u(uint64_t seed, uint32_t step, uint32_t a, uint32_t b);

/* ---- SIDM kernel and overlap (paper Sec. 2: spline kernel of Monaghan 1985;
 *      Sec. 3.5: geometric factor Lambda of the interaction probability) ---- */

/* Cubic spline with compact support h (Gadget convention), normalised to 1. */
double orc_kernel_W(double r, double h);

/* Kernel overlap Lambda(d; hi, hj) = integral of W(|x - xi|, hi) W(|x - xj|, hj) d^3x
 * for two particles at distance d. */
double orc_lambda(double d, double hi, double hj);

/* ---- gravity (paper Sec. 2: softened self-gravity, softening length eps) ---- */

/* Plummer-softened direct sum, self term excluded, j ascending, Neumaier
 * compensated.  For the `nq` particles listed in `q` (or all n when q == NULL,
 * in which case nq is ignored) writes
 *   a_i   =  G sum_{j != i} m_j (x_j - x_i) / (r_ij^2 + eps^2)^{3/2}
 *   phi_i = -G sum_{j != i} m_j / (r_ij^2 + eps^2)^{1/2}
 * into ax/ay/az/pot at position k of the query list (or i).  Also writes the
 * normwise scale A_i = G sum_j m_j r_ij / (r^2+eps^2)^{3/2} into `anorm`
 * (nullable).  Uses OpenMP over the query particles. */
void orc_gravity(int64_t n, const double *x, const double *y, const double *z,
                 const double *m, double G, double eps,
                 int64_t nq, const int64_t *q,
                 double *ax, double *ay, double *az, double *pot, double *anorm);

/* Tree gravity (Sec. 2: the gravity tree with the relative opening criterion
 * alpha of Springel 2005, eq. 18; reading of the tree and of the criterion
 * for groups below).  The tree: particles ordered by their 48-bit Morton key
 * over the bounding box (16 bits per axis, q = (v - lo) * (65535 / ext)
 * clamped to [0, 65535] and truncated; ext the box's largest side), ties in
 * index order; leaves are buckets of 64 consecutive particles, a node of the
 * next level holds 8 consecutive nodes of the level below, up to one root.
 * Each node has its particles' bounding box, mass M and first moments
 * (sums in particle order for a bucket, in child order above).  A group is a
 * bucket: a node is accepted for all of its members when its box and the
 * group's box are disjoint and (G M l^2)^2 <= alpha^2 |a_old|^2 r^8, with l the
 * node box's largest side, |a_old|^2 the smallest (ax^2 + ay^2) + az^2 of the
 * group's previous accelerations and r^2 the squared distance between the
 * group's box and the node's box (the criterion G M l^2 <= alpha |a_old| r^4,
 * squared, for every member and every particle of the node: a node's centre
 * of mass can lie far from some of its particles).  Otherwise the
 * node is opened; an opened bucket contributes its particles.  Forces and
 * potentials: Plummer-softened pair terms with the contributed particles (self
 * excluded) and, for an accepted node, its monopole plus its quadrupole (the
 * second-order term of the softened potential about the node's centre of
 * mass, from the node's second moments), Neumaier sums.  alpha = 0
 * opens every node: the direct sum.  q == NULL: writes ax, ay, az, pot of all
 * n particles in the caller's order; otherwise of the nq particles q[k] at
 * index k (the whole tree is built, only the groups holding them walk).
 * `terms` (nullable) receives the number of source terms summed over the
 * groups walked (accepted nodes plus contributed particles per group).  Uses
 * OpenMP over the groups. */
void orc_tree_gravity(int64_t n, const double *x, const double *y, const double *z,
                      const double *m, const double *ax_old, const double *ay_old,
                      const double *az_old, double G, double eps, double alpha, int64_t nq,
                      const int64_t *q, double *ax, double *ay, double *az, double *pot,
                      int64_t *terms);

/* Tree gravity as the paper states it (Sec. 2: a one-sided oct-tree opened
 * with the relative criterion of Springel 2005, eq. 18), the accuracy
 * reference for the tree option.  The tree: a cube around all particles,
 * split into eight octants (a particle on a midplane goes to the upper side)
 * until a cell holds one particle (or at depth 60, where the rest stay
 * together); each cell holds its particles' mass M and centre of mass.  Each
 * particle i walks it from the root on its own: a cell is accepted as one
 * Plummer-softened monopole at its centre of mass when G M l^2 <= alpha
 * |a_old,i| r^4 (l the cube's side, r the distance from x_i to the centre of
 * mass) and x_i lies outside the cube (reading: a cell that holds the
 * particle is always opened, as the criterion assumes a distant cell);
 * otherwise it is opened, and a leaf contributes its particles (self
 * excluded).  a_old = 0 opens every cell: the direct sum.  Plain double sums
 * in walk order.  q == NULL: all n particles; otherwise the nq particles q[k]
 * at index k.  `terms` (nullable): source terms summed over the queried
 * particles.  OpenMP over the queried particles. */
void orc_octree_gravity(int64_t n, const double *x, const double *y, const double *z,
                        const double *m, const double *ax_old, const double *ay_old,
                        const double *az_old, double G, double eps, double alpha, int64_t nq,
                        const int64_t *q, double *ax, double *ay, double *az, double *pot,
                        int64_t *terms);

/* Static NFW host (paper Sec. 4.1, Eq. nfw_potential) centred at c:
 * Phi(r) = -4 pi G rho_s r_s^3 ln(1 + r/r_s) / r and a = -grad Phi.
 * Writes (not adds) the host acceleration and potential for n particles. */
void orc_host_nfw(int64_t n, const double *x, const double *y, const double *z,
                  double G, double rho_s, double r_s, const double c[3],
                  double *ax, double *ay, double *az, double *pot);

struct orc_params_s;   /* the step parameters, defined below */

/* Hernquist bulge (Sec. 4.1, Eq. hernquist_potential): Phi = -G M / (r + a). */
void orc_host_hernquist(int64_t n, const double *x, const double *y, const double *z,
                        double G, double M, double a, const double c[3],
                        double *ax, double *ay, double *az, double *pot);

/* Miyamoto-Nagai disc in the z = 0 plane of centre c (Sec. 4.1, Eq. disk_potential):
 * Phi = -G M / sqrt(R^2 + (a + sqrt(z^2 + b^2))^2). */
void orc_host_disk(int64_t n, const double *x, const double *y, const double *z,
                   double G, double M, double a, double b, const double c[3],
                   double *ax, double *ay, double *az, double *pot);

/* The host field of a parameter set: nothing (host_kind 0), the NFW halo (1),
 * or the Milky-Way host of Sec. 4.1 (2: NFW + Hernquist + four discs).
 * Writes (not adds) a and the potential. */
void orc_host_field(int64_t n, const double *x, const double *y, const double *z,
                    const struct orc_params_s *p, double *ax, double *ay, double *az,
                    double *pot);

/* ---- kernel size from the N_ngb nearest neighbours (paper Sec. 2) ---- */

/* Brute force: for each queried i, order j != i by (d2_ij, id_j) with
 * d2 = (dx*dx + dy*dy) + dz*dz, dx = x_j - x_i; h_i = sqrt of the k-th d2.
 * Writes h for the query list; nbr (nullable) receives the k ids in order,
 * row-major [nq][k]. */
void orc_knn(int64_t n, const double *x, const double *y, const double *z,
             const uint32_t *id, int32_t k, int64_t nq, const int64_t *q,
             double *h, uint32_t *nbr);

/* The same h as orc_knn for every particle (all queried), bit for bit, from a
 * search over cubic shells of a uniform grid. */
void orc_knn_grid(int64_t n, const double *x, const double *y, const double *z,
                  const uint32_t *id, int32_t k, double *h);

/* The same h as orc_knn for every particle, bit for bit, and (nbr nullable)
 * the same neighbour lists, from a search over a k-d tree. */
void orc_knn_tree(int64_t n, const double *x, const double *y, const double *z,
                  const uint32_t *id, int32_t k, double *h, uint32_t *nbr);

/* ---- pairwise scattering (paper Sec. 2 and Sec. 3.5) ---- */

/* Cross-section per unit mass at relative speed g (Sec. 3.8, Eq. vel_dep):
 * sigma_m [1 + (g/w)^2]^-2 for w > 0, else sigma_m. */
double orc_sigma(double sigma_m, double w, double g);

typedef struct {
    uint32_t a, b;     /* ids, a < b                                 */
    int64_t ia, ib;    /* halo-local indices of the particles a, b  */
    double u, P;       /* accept draw and probability                */
} orc_event;

/* Tests every unordered pair {i, j} with d2_ij < (h_i + h_j)^2 once, with
 * a = min id, b = max id, P_ab = (sigma(g)/m) m_b g Lambda_ab dt with g = |v_a - v_b|
 * and sigma(g)/m = orc_sigma(sigma_m, sigma_w, g), and the
 * accept draw u of orc_accept_u; an event is u < P.  When `q` is non-NULL only
 * pairs with at least one endpoint in the query set (flag array `qmask` of
 * length n) are tested.  Writes up to `cap` events in (a, b) order and returns
 * the number found.  n_pairs / n_p_gt1 (nullable) receive the pair count and
 * the number of pairs with P > 1. */
int64_t orc_find_events(int64_t n, const double *x, const double *y, const double *z,
                        const double *vx, const double *vy, const double *vz,
                        const double *m, const uint32_t *id, const double *h,
                        double sigma_m, double sigma_w, double dt, uint64_t seed, uint32_t step,
                        const uint8_t *qmask, orc_event *ev, int64_t cap,
                        int64_t *n_pairs, int64_t *n_p_gt1);

/* The same events, pair count and P > 1 count as orc_find_events without a
 * query set, from a sweep over the particles sorted by x. */
int64_t orc_find_events_sweep(int64_t n, const double *x, const double *y, const double *z,
                              const double *vx, const double *vy, const double *vz,
                              const double *m, const uint32_t *id, const double *h,
                              double sigma_m, double sigma_w, double dt, uint64_t seed,
                              uint32_t step, orc_event *ev, int64_t cap, int64_t *n_pairs,
                              int64_t *n_p_gt1);

/* The same events, pair count and P > 1 count as orc_find_events without a
 * query set, from a range search over a k-d tree (the overlap integral only
 * where the draw falls below an upper bound of P; see the source). */
int64_t orc_find_events_tree(int64_t n, const double *x, const double *y, const double *z,
                             const double *vx, const double *vy, const double *vz,
                             const double *m, const uint32_t *id, const double *h,
                             double sigma_m, double sigma_w, double dt, uint64_t seed,
                             uint32_t step, orc_event *ev, int64_t cap, int64_t *n_pairs,
                             int64_t *n_p_gt1);

/* Elastic isotropic scattering of one pair in its centre-of-mass frame, using
 * the direction draw at counter (a, b, step, 1).  Updates the two velocities. */
void orc_kick_pair(uint64_t seed, uint32_t step, uint32_t a, uint32_t b,
                   double ma, double mb, double va[3], double vb[3]);

/* Applies events (already in (a, b) order) one after the other. */
void orc_apply_events(int64_t n_ev, const orc_event *ev, const double *m,
                      double *vx, double *vy, double *vz, uint64_t seed, uint32_t step);

/* ---- diagnostics ---- */

/* K = 1/2 sum m v^2, W = 1/2 sum m phi_self, Eext = sum m Phi_ext, p = sum m v.
 * pot holds phi_self + Phi_ext and pext holds Phi_ext (nullable: zero). */
void orc_diag(int64_t n, const double *vx, const double *vy, const double *vz,
              const double *m, const double *pot, const double *pext, double out[6]);

/* Central density (Sec. 3: the centre is the potential minimum): the
 * particle c with the lowest phi (self-potential; first index on ties), and
 * the number and total mass of the particles with d2 <= radius^2 from it. */
void orc_central_density(int64_t n, const double *x, const double *y, const double *z,
                         const double *m, const double *phi, double radius,
                         int64_t *center, int64_t *count, double *mass);

/* Tidal radius (Eq. tidal_radius) of a satellite in the host of p: the centre
 * c is the lowest phi (self-potential), n the unit vector from the host centre
 * to c; G M(<= r) / r^2 = |grad Phi(c + r n) - grad Phi(c - r n)| solved by 60
 * bisection steps in log r on [2^-40, 1] x 2 r_max.  Returns 1 if the host's
 * tides do not win even at 2 r_max. */
int orc_tidal_radius(int64_t n, const double *x, const double *y, const double *z,
                     const double *m, const double *phi, const struct orc_params_s *p,
                     double *r_tidal, double *mass, int64_t *center);

/* ---- one kick-drift-kick step with SIDM at the synchronised point ---- */

typedef struct orc_params_s {
    double G, eps, sigma_m, dt;
    int32_t k;
    uint64_t seed;
    int32_t host_kind;          /* 0 none, 1 NFW                             */
    double host_rho_s, host_r_s, host_c[3];
    double sigma_w;             /* velocity scale of sigma(v); 0: constant   */
    double host_hern_M, host_hern_a;      /* host_kind 2: Hernquist bulge */
    double host_disk[4][3];     /* host_kind 2: Miyamoto-Nagai discs (M, a, b) */
    double boundary_r, boundary_c[3];     /* reflecting sphere; r = 0: none */
    double eta;                 /* > 0: block time steps with this criterion  */
    double dt_min;              /* smallest allowed step (0: none)            */
    int32_t max_bin;            /* steps dt / 2^b, 0 <= b <= max_bin          */
    double tree_alpha;          /* > 0: self-gravity by orc_tree_gravity with the
                                   accelerations held on entry as a_old        */
} orc_params;

/* Time-step bin of one particle (Sec. 2: the gravitational criterion of
 * Springel 2005, eq. 34, s <= sqrt(2 eta eps / |a|)): the smallest b in
 * [0, max_bin] with (s^2)^2 |a|^2 <= (2 eta eps)^2 for s = dt / 2^b (else
 * max_bin), then decreased while dt / 2^b < dt_min. */
int32_t orc_bin(double dt, double eta, double eps, double dt_min, int32_t max_bin,
                double ax, double ay, double az);

/* The parts of a fixed step around the forces: K(dt/2) D(dt) with the
 * reflecting sphere, and the closing K(dt/2) (orc_kdk_step calls both). */
void orc_kick_drift(int64_t n, double *x, double *y, double *z, double *vx, double *vy,
                    double *vz, const double *ax, const double *ay, const double *az,
                    const orc_params *p);
void orc_close_kick(int64_t n, double *vx, double *vy, double *vz, const double *ax,
                    const double *ay, const double *az, const orc_params *p);

/* Full-N step for one halo (exact searches: orc_knn_tree, orc_find_events_tree).
 * With eta > 0 the step is one cycle of block time steps (see the source).  On entry a/pot hold the acceleration
 * and potential at x (self + host).  Performs K(dt/2), D(dt), gravity + host,
 * K(dt/2), h from kNN, events, ordered kicks.  Writes h; returns the number of
 * events (or -1 if more than `ev_cap` events were found; ev may be NULL when
 * ev_cap is 0).  `ev` receives the applied events in (a, b) order. */
int64_t orc_kdk_step(int64_t n, double *x, double *y, double *z,
                     double *vx, double *vy, double *vz, const double *m,
                     const uint32_t *id, double *ax, double *ay, double *az,
                     double *pot, double *h, const orc_params *p, uint32_t step,
                     orc_event *ev, int64_t ev_cap);

/* Number of OpenMP threads the oracle uses. */
int orc_num_threads(void);
/* Threads of the OpenMP loops that follow (n > 0; timing of the oracle). */
void orc_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
