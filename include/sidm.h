/*
 * sidm.h -- C ABI of libsidm, an MI355X (gfx950) implementation of the
 * data-parallel hot path of a self-interacting dark matter (SIDM) N-body step
 * as studied by Fischer, Yu & Dolag (arXiv 2506.06269):
 *
 *   - softened self-gravity for every particle plus a static analytic NFW host
 *     (Sec. 2 "softening length"; Sec. 4.1 Eq. nfw_potential),
 *   - the SIDM kernel size h_i from the N_ngb nearest neighbours (Sec. 2),
 *   - rare pairwise scattering through the spline-kernel overlap Lambda_ij
 *     (Sec. 2; Sec. 3.5 geometric factor), with explicit energy and momentum
 *     conservation (Sec. 2),
 *   - all inside a fixed-step kick-drift-kick leapfrog (Sec. 3.1: constant
 *     time steps remove the integrator's energy error).
 *
 * Conventions shared by every entry point
 *   - Every particle array is DEVICE memory owned by the caller, structure of
 *     arrays, length n_total (the largest offset + n over the halos passed).
 *     The library owns only the scratch memory inside its context.
 *   - Work is enqueued on `stream` (a hipStream_t passed as void*, NULL = the
 *     null stream) and the call returns without waiting, unless a host
 *     out-parameter is requested (documented per call).
 *   - Argument errors are detected on the host before anything is enqueued and
 *     return SIDM_ERR_INVALID (or SIDM_ERR_UNSUPPORTED) with a message in
 *     sidm_last_error().  HIP launch errors return SIDM_ERR_HIP.  Conditions the
 *     device detects (the SIDM_DEV_* bits: event buffer overflow, kNN search
 *     overflow, unequal masses or repeated ids in a halo that scatters, a stale
 *     graph replay) are reported in sidm_diag.status, by a synchronous call
 *     itself, and otherwise by the next call on the context that finds the
 *     earlier call's kernels finished: that call returns SIDM_ERR_CAPACITY
 *     (overflows), SIDM_ERR_UNSUPPORTED (unequal masses) or SIDM_ERR_INVALID
 *     (repeated ids, stale replay) without running, with the conditions in
 *     sidm_last_error(); they are reported once.  sidm_take_status() waits and
 *     returns them instead.
 *   - Graphs: calls may be captured into a HIP graph once a call outside
 *     capture has used the same halos and the same state pointers (that call
 *     builds the launch plan).  A replay uses the pointers of the capture.  A
 *     call outside capture with other halos or state pointers, or a change of
 *     the context's scratch (sidm_set_event_capacity, the first call with block
 *     time steps), makes earlier captures stale: their replays set
 *     SIDM_DEV_STALE_GRAPH (the kernels still run with the captured pointers,
 *     so free nothing a graph may still use).  Reallocating state buffers
 *     without any call outside capture in between is not detected.
 *   - Halos are independent systems: particles of different halos neither
 *     attract nor scatter.  Halo ranges must not overlap.
 *   - A context is thread-compatible (one thread at a time), not thread-safe.
 *     Calls on one context must be issued to one stream or be ordered by the
 *     caller: they share the context's scratch memory.
 *   - Units are whatever the caller uses consistently (the tests use
 *     G = r_s = rho_s = 1).
 */
#ifndef SIDM_H
#define SIDM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SIDM_ABI_VERSION 1
#define SIDM_MAX_K 128          /* largest supported neighbour number N_ngb */
#define SIDM_MAX_BIN 16         /* deepest block time-step bin             */

typedef struct sidm_ctx sidm_ctx;

typedef enum {
    SIDM_OK = 0,
    SIDM_ERR_INVALID = -1,      /* bad argument, see sidm_last_error()              */
    SIDM_ERR_NOMEM = -2,        /* device allocation failed                         */
    SIDM_ERR_HIP = -3,          /* a HIP runtime call or launch failed              */
    SIDM_ERR_CAPACITY = -4,     /* a device-side capacity was exceeded             */
    SIDM_ERR_UNSUPPORTED = -5   /* valid request this version does not implement    */
} sidm_status;

typedef enum {
    SIDM_PREC_FP64 = 0,         /* all arithmetic in FP64                           */
    SIDM_PREC_MIXED = 1         /* gravity tiles in FP32 with compensated (Kahan)
                                   accumulation; kicks, drift, SIDM and reductions
                                   in FP64                                          */
} sidm_precision;

/* One halo (host memory; an array of these is a batch). */
typedef struct {
    int64_t offset;             /* particles [offset, offset + n) of the arrays    */
    int64_t n;                  /* number of particles, 2 <= n <= 2^24             */
    double G;                   /* gravitational constant                           */
    double eps;                 /* Plummer softening length, > 0 (Sec. 2)           */
    double sigma_m;             /* cross-section per unit mass, >= 0 (isotropic,
                                   velocity independent: Sec. 2)                    */
    double dt;                  /* fixed time step, > 0                             */
    int32_t k;                  /* N_ngb, 1 <= k <= min(n - 1, SIDM_MAX_K)          */
    int32_t host_kind;          /* 0: isolated; 1: static NFW host; 2: the Milky-Way
                                   host of Sec. 4.1 (NFW + Hernquist bulge + four
                                   Miyamoto-Nagai discs)                            */
    uint64_t seed;              /* Philox key of the scattering draws               */
    double host_rho_s;          /* host NFW density parameter (Eq. nfw_potential)   */
    double host_r_s;            /* host NFW scale radius, > 0 when rho_s != 0       */
    double host_center[3];      /* host centre; the discs lie in its z = 0 plane    */
    double sigma_w;             /* velocity scale w of the cross-section: sigma(v) =
                                   sigma_m [1 + (v/w)^2]^-2 with v the pair's relative
                                   speed (Sec. 3.8 Eq. vel_dep); 0: independent of v  */
    double host_hern_M;         /* host_kind 2: Hernquist bulge mass and scale length */
    double host_hern_a;         /*   (Eq. hernquist_potential); M = 0: none          */
    double host_disk[4][3];     /* host_kind 2: Miyamoto-Nagai discs (M, a, b)
                                   (Eq. disk_potential); M = 0: unused slot         */
    double boundary_r;          /* reflecting sphere (Sec. 2): after the drift, a
                                   particle farther than boundary_r from
                                   boundary_center that moves outwards has its
                                   radial velocity reversed; 0: none                */
    double boundary_center[3];
    double eta;                 /* > 0: sidm_kdk_step runs one cycle of block time
                                   steps of total length dt (see there); 0: one
                                   fixed step                                       */
    double dt_min;              /* smallest allowed block step, >= 0 (Sec. 2)     */
    int32_t max_bin;            /* block steps dt / 2^b, 0 <= b <= max_bin <=
                                   SIDM_MAX_BIN; must be 0 when eta = 0             */
    int32_t reserved;           /* set to 0                                        */
    double tree_alpha;          /* > 0: self-gravity through the tree with this
                                   relative opening parameter (Sec. 2, Table 1:
                                   5e-4; see sidm_gravity); 0: direct sum          */
} sidm_halo;

/* Particle state (device pointers, length n_total each). */
typedef struct {
    double *x, *y, *z;          /* positions (FP64: Sec. 2 stores them in double)  */
    double *vx, *vy, *vz;       /* velocities                                       */
    const double *m;            /* masses; equal within a halo when sigma_m > 0    */
    const uint32_t *id;         /* identities, unique within a halo: they key the
                                   random draws and fix the order of the kicks     */
    double *ax, *ay, *az;       /* total acceleration (self + host) at x            */
    double *pot;                /* total potential (self + host) at x               */
    double *h;                  /* SIDM kernel size                                 */
} sidm_state;

/* One scattering event: ids a < b, the halo index in the call's halo array and
 * the conflict-free round in which it was applied (1-based). */
typedef struct {
    uint32_t a, b;
    int32_t halo;
    uint32_t round;
} sidm_event;

/* Per-halo diagnostics after a step (device memory, one per halo). */
typedef struct {
    double K;                   /* 1/2 sum m v^2                                    */
    double W;                   /* 1/2 sum m phi_self                               */
    double Eext;                /* sum m Phi_host                                   */
    double px, py, pz;          /* sum m v                                          */
    int64_t n_events;           /* scatterings applied this step                    */
    int64_t n_rounds;           /* conflict-free rounds used                        */
    int64_t n_pairs;            /* pairs with overlapping kernels that were tested  */
    int64_t n_p_gt1;            /* pairs with P > 1 (accepted with certainty)       */
    int32_t status;             /* SIDM_DEV_* bits                                  */
    int32_t reserved;
    int64_t n_grav_terms;       /* tree halos: source terms (accepted nodes plus
                                   particles of opened buckets) summed over the
                                   groups by the tree walks since the step (or the
                                   sidm_gravity call) began; 0 for direct sums      */
    int64_t n_candidates;       /* tested pairs whose draw fell below the cheap
                                   bound 8 (sigma/m) m g dt / (pi max(h)^3) of P,
                                   so that the overlap integral was evaluated    */
} sidm_diag;

#define SIDM_DEV_EVENT_OVERFLOW 1   /* more events than the context can hold: no
                                       kicks were applied this step              */
#define SIDM_DEV_KNN_OVERFLOW   2   /* a neighbour search needed more refinement
                                       levels than supported (h is NaN there)   */
#define SIDM_DEV_NONFINITE      4   /* a position or velocity is not finite     */
#define SIDM_DEV_UNEQUAL_MASS   8   /* sigma_m > 0 but the masses of the halo are
                                       not all equal: the halo was not scattered */
#define SIDM_DEV_DUPLICATE_ID  16   /* two particles of the halo share an id: the
                                       halo was not scattered                    */
#define SIDM_DEV_STALE_GRAPH   32   /* a captured sequence was replayed after a
                                       call outside capture changed the halos,
                                       the state pointers or the context's
                                       scratch (see Graphs above)                */

/* ---- context ---------------------------------------------------------------
 * Creates a context on HIP device `device` with scratch memory for up to
 * `max_particles` particles in total and `max_halos` halos per call, and room
 * for max(4096, max_particles / 8) scattering events per call (and four times
 * as many candidates: pairs whose draw falls below the cheap bound of P and
 * whose decision needs the overlap integral; when they are more, a second
 * pair pass decides them all, with the same result).  Allocates
 * device memory (SIDM_ERR_NOMEM on failure).  *out is NULL on error. */
sidm_status sidm_create(sidm_ctx **out, int device, int64_t max_particles, int32_t max_halos);

/* Sets the per-call event capacity, and the candidate capacity to four times
 * it (reallocates; call outside graph capture). */
sidm_status sidm_set_event_capacity(sidm_ctx *ctx, int64_t max_events);

/* Releases the context and its scratch memory (waits for the device). */
void sidm_destroy(sidm_ctx *ctx);

/* Static text for a status code. */
const char *sidm_status_string(sidm_status s);

/* Detail text of the last error on this context ("" if none).  The pointer is
 * valid until the next call on the context.  With ctx = NULL: the text of the
 * last sidm_gravity_static call on the calling thread. */
const char *sidm_last_error(const sidm_ctx *ctx);

/* ---- gravity -----------------------------------------------------------------
 * a_i   = G sum_{j != i} m_j (x_j - x_i) / (|x_j - x_i|^2 + eps^2)^{3/2} + a_host(x_i)
 * pot_i = -G sum_{j != i} m_j / (|x_j - x_i|^2 + eps^2)^{1/2} + Phi_host(x_i)
 * over the particles of the same halo (Sec. 2: softened gravity, here in the
 * Plummer form; Sec. 4.1 Eq. nfw_potential for the host, a = -grad Phi).
 * Writes state->ax/ay/az/pot; reads x, y, z, m.  SIDM_PREC_MIXED evaluates the
 * pair terms in FP32 on positions taken, in FP64, relative to the centre of
 * each compact group of at most 64 spatially sorted particles (the i-particle
 * is moved into the frame of each j group once), sums each tile of 256 terms
 * plainly and the tile sums with compensation, and returns FP64.
 *
 * Halos with tree_alpha > 0 take the self-gravity from a tree walk instead
 * (Sec. 2: the relative opening criterion of Springel 2005, eq. 18): the tree
 * is the Morton-ordered cell list (buckets of 64 particles, 8 children per
 * node, bounding boxes, monopoles at the centres of mass); each bucket walks
 * it once for its members and accepts a node when the two boxes are disjoint
 * and G M l^2 <= tree_alpha |a_old| r^4 (l: the node box's largest side, r:
 * the distance between the boxes, |a_old|: the smallest of the members'
 * accelerations), else opens it; opened buckets contribute their particles.
 * a_old is read from state->ax/ay/az as they are on entry (the previous step's
 * accelerations in a run; zeros open every node and give the direct sum).
 * The decisions are FP64 in both precisions; SIDM_PREC_MIXED forms each pair
 * separation in FP64 and the rest of the pair term in FP32.  The number of
 * source terms summed is reported in sidm_diag.n_grav_terms. */
sidm_status sidm_gravity(sidm_ctx *ctx, const sidm_halo *halos, int32_t n_halos,
                         const sidm_state *state, sidm_precision prec, void *stream);

/* ---- gravity without allocation ---------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the pass of
 * sidm_gravity (direct sum, either precision, host included) for ONE halo of
 * at most SIDM_STATIC_MAX_N particles, without a context.  Every scratch
 * buffer of the pass (cell list, sort keys, FP32 frames, partial rows, launch
 * tables) lies in one fixed array of SIDM_STATIC_BYTES in the library, one per
 * GPU, held until the process ends; the launch tables are written there by a
 * kernel from the halo's parameters.  The call allocates nothing and enqueues
 * on `stream` of the current device.  Every call on a GPU uses that GPU's
 * array, which keeps the last call's contents: calls that overlap on one GPU
 * (other streams, other threads) race and must be ordered by the caller.
 * Results equal sidm_gravity's for the same halo and state.  Errors:
 * SIDM_ERR_CAPACITY when n > SIDM_STATIC_MAX_N, SIDM_ERR_UNSUPPORTED when
 * tree_alpha > 0, SIDM_ERR_INVALID for the argument errors of sidm_gravity;
 * the text is sidm_last_error(NULL) on the calling thread. */
#define SIDM_STATIC_MAX_N 65536
#define SIDM_STATIC_BYTES (17u << 20)
sidm_status sidm_gravity_static(const sidm_halo *halo, const sidm_state *state,
                                sidm_precision prec, void *stream);

/* ---- kernel size -----------------------------------------------------------
 * h_i = distance to the k-th nearest other particle of the same halo (Sec. 2:
 * the kernel size is set by the next N_ngb neighbours), with distances
 * d2 = (dx*dx + dy*dy) + dz*dz evaluated in FP64 without fused multiply-add,
 * ties ordered by id, h = correctly rounded sqrt(d2).  Writes state->h.
 * The value of state->h on entry, where finite, positive and below the halo's
 * extent, only sets the starting search radius (the result does not depend on
 * it): a call after a step, with h a few per cent off, costs about half of a
 * call without usable values.
 * nbr (nullable, device) receives the k neighbour ids of each particle in
 * (d2, id) order, row-major [n_total][k_max] where k_max is the largest k
 * of the halos (rows of halos with smaller k are filled up to their k). */
sidm_status sidm_knn_h(sidm_ctx *ctx, const sidm_halo *halos, int32_t n_halos,
                       const sidm_state *state, uint32_t *nbr, void *stream);

/* ---- scattering ----------------------------------------------------------------
 * Tests every unordered pair {i, j} of a halo with d2_ij < (h_i + h_j)^2 once:
 * a = min id, b = max id,
 *   P_ab = (sigma(g)/m) m_b g Lambda(|x_a - x_b|; h_a, h_b) dt,  g = |v_a - v_b|,
 * with sigma(g)/m = sigma_m, or sigma_m [1 + (g/w)^2]^-2 when sigma_w = w > 0 (the
 * velocity-dependent viscosity cross-section of Sec. 3.8, which for isotropic
 * scattering equals the total cross-section),
 * Lambda = integral of W(|x - x_a|, h_a) W(|x - x_b|, h_b) d^3x with W the
 * cubic spline of compact support h (Sec. 2, Monaghan 1985; Sec. 3.5).  The
 * accept draw is u = top 53 bits of Philox4x32-10 words (w0, w1) at counter
 * (a, b, step, 0) and key (lo32(seed), hi32(seed)); the pair scatters iff
 * u < P.  Probabilities use the velocities at the start of the call.  The
 * events are then applied as elastic isotropic kicks in the pair's
 * centre-of-mass frame (direction cos(theta) = 1 - 2 u_c, phi = 2 pi u_phi from
 * words (w0,w1), (w2,w3) at counter (a, b, step, 1)), in (a, b) order: events
 * sharing no particle are applied concurrently in conflict-free rounds, which
 * gives the same result as applying them one after the other.  Reads x, v, m,
 * id, h; updates vx, vy, vz.
 * events (nullable, device, capacity `cap`) receives the applied events in
 * unspecified order (sort by (halo, a, b) for the application order).
 * n_events_host (nullable): if given, the call waits for the device and stores
 * the number of events; it returns SIDM_ERR_CAPACITY if the context's event
 * capacity or `cap` was exceeded (then no kick was applied; the decisions are a
 * pure function of the state, so a retry with more capacity reproduces them),
 * SIDM_ERR_UNSUPPORTED if a halo with sigma_m > 0 has unequal masses, and
 * SIDM_ERR_INVALID if a halo repeats an id (such halos are not scattered: the
 * probability takes the mass of the member with the larger id, which is only
 * symmetric for equal masses -- every run of the paper's Table 1 has one
 * particle mass -- and ids key the draws and order the kicks). */
sidm_status sidm_scatter(sidm_ctx *ctx, const sidm_halo *halos, int32_t n_halos,
                         const sidm_state *state, uint32_t step, sidm_event *events,
                         int64_t cap, int64_t *n_events_host, void *stream);

/* Copies the events of the last scattering pass run on the context
 * (sidm_scatter or sidm_kdk_step) into out (device, cap records), in
 * unspecified order; nothing when they overflowed the context's buffer.
 * n_events_host (nullable): if given, the call waits for the device, stores the
 * number of events found and returns SIDM_ERR_CAPACITY when they exceed the
 * context's capacity or cap.  For tests and for callers that record events. */
sidm_status sidm_last_events(sidm_ctx *ctx, sidm_event *out, int64_t cap,
                             int64_t *n_events_host, void *stream);

/* ---- one step ------------------------------------------------------------------
 * Pre-condition: state a/pot hold the values at the current x (call
 * sidm_gravity once after loading the initial conditions).
 * K(dt/2) D(dt) gravity+host K(dt/2), then h from the k nearest neighbours,
 * then the scattering pass of sidm_scatter with this `step`.  diag (nullable,
 * device, n_halos entries) receives the energy and momentum after the step.
 *
 * Block time steps (Sec. 2: individual steps from the gravitational criterion
 * eta of Springel 2005 eq. 34 and a minimum step dt_min; Sec. 3.1 on the
 * energy error of changing steps).  When any halo has eta > 0 the call runs
 * one cycle of length dt for every halo; a halo with eta = 0 takes one fixed
 * step in it.  A particle's step is s = dt / 2^b with b the smallest value in
 * [0, max_bin] for which (s^2)^2 |a|^2 <= (2 eta eps)^2 (s^2 |a| <= 2 eta eps
 * without a square root), else max_bin, then decreased while s < dt_min.  The
 * cycle is 2^max_bin ticks of dt / 2^max_bin: every particle drifts each tick
 * (reflecting sphere included); a particle is active at tick k when k is a
 * multiple of its step in ticks, and then gets new forces, its closing half
 * kick with the old step, a new bin (a longer step only when k is a multiple
 * of it) and, before the end, its opening half kick with the new step.  The
 * cycle starts and ends synchronised; h and the scattering pass (probabilities
 * over dt) follow at its end.  Gravity tiles whose i-particles are all
 * inactive are skipped.  Halos with different max_bin share the call's ticks
 * (a halo with max_bin B steps on every 2^(Bmax - B)-th).  With timing on, the
 * pass of the gravity tiles covers all ticks (drift, cell list, tiles, kicks)
 * and the kick+drift pass the opening kick. */
sidm_status sidm_kdk_step(sidm_ctx *ctx, const sidm_halo *halos, int32_t n_halos,
                          const sidm_state *state, uint32_t step, sidm_precision prec,
                          sidm_diag *diag, void *stream);

/* Energies and momentum of the current state (diag: device, n_halos entries).
 * pot must hold the total potential at x.  The event, pair and status fields
 * are those of the last kNN / scattering pass run on this context with the
 * same halos (zero on a context that has run none); the non-finite bit is
 * also set from the state given here. */
sidm_status sidm_diagnostics(sidm_ctx *ctx, const sidm_halo *halos, int32_t n_halos,
                             const sidm_state *state, sidm_diag *diag, void *stream);

/* ---- central density -------------------------------------------------------
 * Sec. 3 takes the minimum of the gravitational potential as the halo centre.
 * For each halo: the centre is the particle with the lowest self-potential
 * pot - Phi_host(x) (first array index on ties; NaN values never), and the
 * central density is counted around it: the particles of the halo with
 * d2 <= radius^2 from the centre (d2 as in sidm_knn_h; the centre included),
 * their number and total mass.  pot must hold the total potential at x (after
 * sidm_gravity or a step).  radius: HOST array, one radius > 0 per halo.
 * out: DEVICE, n_halos entries; index = -1 if no potential is finite.  Copies
 * the radii to the device (not for use inside graph capture). */
typedef struct {
    double x, y, z;             /* position of the centre particle                  */
    double mass;                /* mass within the radius                           */
    int64_t index;              /* array index of the centre particle               */
    int64_t count;              /* particles within the radius                      */
} sidm_center;
sidm_status sidm_central_density(sidm_ctx *ctx, const sidm_halo *halos, int32_t n_halos,
                                 const sidm_state *state, const double *radius,
                                 sidm_center *out, void *stream);

/* ---- tidal radius -----------------------------------------------------------
 * The tidal radius of each halo in its static host (Eq. tidal_radius), with the
 * centre of sidm_central_density and n the unit vector from the host centre to
 * it:  G M(<= r) / r^2 = |grad Phi_host(c + r n) - grad Phi_host(c - r n)|,
 * M(<= r) the mass of the halo's particles with d2 <= r^2 (d2 as in sidm_knn_h).
 * Solved by 60 bisection steps in log r between 2^-40 (2 r_max) and 2 r_max
 * (r_max: the farthest particle from the centre): r_tidal is the final upper
 * bracket, where the host's tides win.  status 1: they do not win even at
 * 2 r_max (r_tidal = 2 r_max).  Needs host_kind != 0.  out: DEVICE, n_halos. */
typedef struct {
    double r_tidal;             /* tidal radius                                      */
    double mass;                /* M(<= r_tidal)                                     */
    double x, y, z;             /* the centre                                        */
    int64_t index;              /* array index of the centre particle                */
    int32_t status;             /* 0, or 1 (no crossing below 2 r_max)              */
    int32_t reserved;
} sidm_tidal;
sidm_status sidm_tidal_radius(sidm_ctx *ctx, const sidm_halo *halos, int32_t n_halos,
                              const sidm_state *state, sidm_tidal *out, void *stream);

/* Waits for the device and returns in *bits the SIDM_DEV_* conditions found
 * by the context's calls and not yet reported, then clears them. */
sidm_status sidm_take_status(sidm_ctx *ctx, int32_t *bits);

/* ---- launch shape of the gravity tiles ------------------------------------
 * The direct-sum tiles run in one of several launch shapes: ireg i-particles
 * per thread (2, 4 or 8) and threads per block, which is also the j-tile
 * staged in LDS (128, 256 or 512), in a plain launch (one block per work
 * item) or a persistent one (as many blocks as the device holds, each taking
 * work items from an atomic ticket until none is left).  The j-splits follow
 * from the shape (a simulation of the items on the resident blocks).  The
 * results of the shapes agree to rounding; the default is 4 x 256, plain.
 * Cycles of block time steps run their ticks in the default shape.  The
 * symmetric tiles (sidm_set_symmetric) run in the same shape, always
 * persistent. */
sidm_status sidm_set_launch_shape(sidm_ctx *ctx, int32_t ireg, int32_t threads,
                                  int32_t persistent);

/* Symmetric tiles.  The softened pair force of the direct sum (Sec. 2) is
 * antisymmetric: the force of j on i is minus that of i on j.  In mixed precision
 * the direct sum of a halo of at least min_n particles evaluates each
 * unordered pair once and applies it to both members; the reactions are
 * summed in 64-bit fixed point with integer atomics, so the result is
 * deterministic: it does not depend on the order in which the work items
 * finish.  The results agree with the one-sided tiles to FP32 rounding.
 * Halos need a softening eps > 0.  min_n = 0 turns them off; the default is
 * 4096.  FP64, tree halos and the ticks of a cycle of block time steps
 * (when some direct-sum halo has max_bin > 0) use the one-sided sums.
 * Changing it invalidates graphs captured before.  SIDM_ERR_INVALID for
 * min_n < 0. */
sidm_status sidm_set_symmetric(sidm_ctx *ctx, int64_t min_n);

/* Chooses the shape for these halos and precision on this device: when
 * cache_path names a file that holds an entry for the key (device
 * architecture, compute units, precision, and the call's direct-sum size
 * class: log2 of its direct-sum particles and of its halos, rounded; a mixed
 * call with a halo that takes the symmetric tiles is keyed apart), that
 * entry; otherwise every shape is timed on the caller's state (the gravity
 * pass, best of a few runs; about 2 x 9 x 4 gravity passes) and the fastest is
 * kept and written to the cache (a JSON object, one entry per key; the file
 * is created or rewritten).  Then runs sidm_gravity with the chosen shape, so
 * a and pot are those of the shape (the timing runs also write them).  The
 * shape stays on the context.  Waits for the device; not during capture. */
#define SIDM_TUNE_FORCE 1       /* time the shapes even if the cache has the key   */
#define SIDM_TUNE_QUICK 2       /* one timed run per shape instead of three        */
#define SIDM_TUNE_CACHE_ONLY 4  /* without a cache entry keep the current shape     */
typedef struct {
    int32_t ireg, threads, persistent;   /* the chosen shape                         */
    int32_t from_cache;                  /* 1: read from the cache, not timed        */
    int32_t n_tried;                     /* shapes timed                             */
    int32_t reserved;
    double ms;                           /* the chosen shape's gravity pass (timed)  */
    double ms_default;                   /* the default shape's                      */
    char key[96];                        /* the cache key                            */
} sidm_tune_result;
sidm_status sidm_autotune(sidm_ctx *ctx, const sidm_halo *halos, int32_t n_halos,
                          const sidm_state *state, sidm_precision prec, const char *cache_path,
                          int32_t flags, sidm_tune_result *out, void *stream);

/* ---- pass timing ---------------------------------------------------------
 * When enabled, sidm_kdk_step records HIP events on its stream around each
 * pass (not usable while the stream is being captured into a graph).
 * sidm_pass_times waits for the last timed step and writes SIDM_N_PASSES
 * durations in milliseconds: kick+drift, gravity (all kernels), gravity tiles
 * (the pair-sum kernel alone), cell list, kNN, pair search, ordered kicks,
 * diagnostics. */
#define SIDM_N_PASSES 8
sidm_status sidm_enable_timing(sidm_ctx *ctx, int on);
sidm_status sidm_pass_times(sidm_ctx *ctx, double ms[SIDM_N_PASSES]);

#ifdef __cplusplus
}
#endif
#endif
