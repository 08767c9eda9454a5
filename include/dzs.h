/*
 * dzs.h — C ABI of the MI355X (gfx950) DZS gravity-step library, libdzs.so.
 *
 * The library implements one gravity step of a periodic dark-matter N-body run on a
 * mixed-mass particle set whose resolution is lowered outside the observer's past lightcone
 * (Dynamic Zoom Simulations, Garaldi, Nori & Baldi 2020, arXiv:2005.05328):
 *
 *   dzs_coarsen    — DZS node merging, Sec. 2.2 and 2.2.1 (eqs. 1 and 3, l_max cap,
 *                    softening rescale by (M/M_init)^(1/3), type change of merged particles)
 *   pm_force       — long-range TreePM part, Sec. 2.1: density on a uniform grid, Poisson
 *                    equation in Fourier space, Gaussian split kernel
 *   tree_force     — short-range TreePM part, Sec. 2.1: monopole oct-tree with a geometric
 *                    opening criterion (eq. 1)
 *   lightcone_emit — on-the-fly lightcone output, Sec. 1 (R_lc) and Sec. 3.1.3 (particles
 *                    saved as they reach the shrinking lightcone sphere)
 *   kdk_step       — the whole step: kick, drift + lightcone, DZS, force, kick
 *
 * Conventions (all calls)
 *   Units: lengths Mpc/h, velocities km/s, masses 1e10 Msun/h; G in those units.
 *   State: structure of arrays in caller-owned DEVICE memory (dzs_particles).  Positions are
 *   comoving, in [0, L).  Momenta p = a^2 dx/dt.  mass_i = mult_i * m0.  Softening
 *   eps_i = eps0 * mult_i^(1/3) (spline support 2.8 eps_i).
 *   Streams: every call is enqueued on `stream` (a hipStream_t; NULL = the null stream) and
 *   returns without waiting for the GPU, except where a call is documented to synchronise.
 *   Errors: every call returns a dzs_status; DZS_OK is 0, failures are negative.  Nothing
 *   aborts or throws across the ABI.  dzs_last_error() gives a text for the context's last
 *   failure.  Argument errors (DZS_EINVAL, DZS_ECAPACITY on sizes) are detected on the host
 *   before anything is enqueued.
 *   Threading: a context is used by one host thread and one stream at a time.
 *   Determinism: given identical inputs every call produces bit-identical outputs (the
 *   lightcone record order excepted; records are identified by id).
 */
#ifndef DZS_H
#define DZS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dzs_status;
#define DZS_OK 0
#define DZS_EINVAL (-1)     /* bad argument, size or pointer */
#define DZS_ENOMEM (-2)     /* device allocation failed at context creation */
#define DZS_ECAPACITY (-3)  /* a size exceeds the context's capacity, or a device-side
                               overflow (lightcone ring, tree walk stack) was detected */
#define DZS_EHIP (-4)       /* a HIP runtime call failed */

#define DZS_CHEB_MAX 24     /* maximum Chebyshev coefficients per function */

typedef struct dzs_ctx dzs_ctx;

/* Capacities fixed at context creation; the context allocates all its scratch then and no
 * call allocates device memory afterwards.  The lightcone ring is caller-owned and carries
 * its own capacity (dzs_lc_ring), so the context needs no per-record scratch and takes no
 * record capacity. */
typedef struct {
    uint64_t max_particles;  /* largest particle count any call will see */
    uint32_t max_mesh_side;  /* 0 (no PM) or 8..1024: room for meshes of up to
                                max_mesh_side^3 points (a mesh side itself must be an
                                even 2^a 3^b) */
    uint32_t flags;          /* DZS_CAP_* bits */
    uint32_t max_boxes;      /* largest batch kdk_step_batch will see, 1..DZS_BATCH_MAX
                                (0 = DZS_BATCH_MAX): sizes the batch's box, offset and mesh
                                tables */
    uint32_t reserved;       /* 0 */
} dzs_capacity;

/* Capacity flag: size the meshes for the precision form only (8-byte complex cells that
 * also hold the fixed-point deposit, 4-byte potential: 12 instead of 32 bytes per cell);
 * plain-form PM calls on such a context fail with DZS_EINVAL. */
#define DZS_CAP_FP32_MESHES 1u
/* Capacity flag: room for the PM force of kdk_step_hier's long-range-on-the-global-step
 * form (dzs_hier_params.pm_global) and for the lists of the targets that end a step at a
 * sub-step boundary: 44 bytes per particle more. */
#define DZS_CAP_HIER_SPLIT 4u
/* Capacity flag: no sorted copies for tree_force (28 bytes per particle fewer); tree_force on
 * such a context needs particles already in key order (dzs_tree_params.presorted = 1). */
#define DZS_CAP_NO_COPIES 2u

/* Periodic box. */
typedef struct {
    double L;     /* box side */
    double m0;    /* mass of a multiplicity-1 particle */
    double eps0;  /* Plummer-equivalent softening of a multiplicity-1 particle */
    double G;     /* gravitational constant */
} dzs_box;

/* Particle state, caller-owned device arrays of at least `capacity` elements each. */
typedef struct {
    double *x, *y, *z;     /* positions in [0, L) */
    double *px, *py, *pz;  /* momenta */
    double *gx, *gy, *gz;  /* accelerations (written by the force calls) */
    uint32_t *mult;        /* multiplicity (number of original particles represented) */
    uint32_t *id;          /* identifier; a merged particle takes its smallest member id */
    uint8_t *type;         /* 0 = original resolution, 1 = de-refined (merged) */
    uint64_t n;            /* current count (host value; dzs_coarsen and kdk_step update it) */
    uint64_t capacity;
} dzs_particles;

/* DZS de-refinement parameters (Sec. 2.2.1).  A node of side l_k (level k, l_k = L / 2^k)
 * may merge when k >= k_min (l_k <= l_max) and it holds at least two particles; its distance
 * to the lightcone is D_n = max(|x_com - x_obs|_min-image - R_lc - b, 0) (eq. 3).
 *  - geometric criterion (eq. 1): merge when l_k < theta * D_n, evaluated as
 *    |d|^2 > (R_lc + b + l_k / theta)^2;
 *  - dynamical criterion (eq. 2): merge when G M_n l_k^2 < alpha_dyn a_min D_n^4 and D_n > 0,
 *    M_n = K m0 (K = summed multiplicity), a_min = the smallest |g| (the accelerations held in
 *    the state, i.e. those of the previous force) over particles with |x - x_obs|_min-image
 *    < R_lc + b, +inf when there is none.  Evaluated in FP64 as
 *    ((G m0) K) l_k^2 < (alpha_dyn a_min) ((D D)(D D)), D = sqrt(|d|^2) - (R_lc + b).
 * Each particle joins its shallowest merging node (top-down walk).  The node centre of mass
 * is the Neumaier-compensated FP64 sum over its members in ascending (Morton key, id) order
 * divided by their total multiplicity. */
#define DZS_CRIT_GEOMETRIC 0
#define DZS_CRIT_DYNAMICAL 1
typedef struct {
    double x_obs[3];    /* observer position */
    double R_lc;        /* lightcone radius at the coarsening epoch */
    double b;           /* buffer width */
    double theta;       /* geometric de-refinement angle (> 0; read by the geometric one) */
    int32_t k_min;      /* shallowest level allowed to merge, 1..21 */
    int32_t criterion;  /* DZS_CRIT_GEOMETRIC or DZS_CRIT_DYNAMICAL */
    double alpha_dyn;   /* dynamical accuracy parameter (>= 0; read by the dynamical one) */
} dzs_coarsen_params;

typedef struct {
    uint64_t n_before, n_after, n_groups;  /* n_groups = merged nodes created */
    double a_min;  /* dynamical criterion: the a_min used (+inf if none inside); else NaN */
} dzs_coarsen_report;

#define DZS_FP64 0        /* plain form: every step in FP64 */
#define DZS_FP32 1        /* precision form: pair, mesh and FFT arithmetic in FP32 with FP32
                             accumulation; positions, momenta, the stored force, the
                             deposit (fixed point), kicks, drifts, crossing times and merge
                             sums stay FP64 */

/* PM (long-range) parameters: mesh points at j*Delta, Delta = L/ng; cloud-in-cell
 * assignment; Green's function -4 pi G exp(-k^2 r_s^2) / (k^2 W(k)^2) with the CIC window
 * W deconvolved twice; 4-point finite-difference gradient; CIC interpolation. */
typedef struct {
    int32_t ng;          /* mesh side: 2^a 3^b with a >= 1, 8 <= ng <= max_mesh_side */
    int32_t precision;   /* DZS_FP64, or DZS_FP32: FFT, Green's function product, gradient
                            and interpolation in FP32 (rms error ~1e-6 of the force) */
    double r_s;          /* split scale */
    int32_t accumulate;  /* 0: g = g_long, 1: g += g_long */
    int32_t tile_chunk;  /* particles per workgroup tile of the deposit and of the
                            interpolation: a power of two in [DZS_PM_CHUNK_MIN,
                            DZS_PM_CHUNK_MAX]; 0 = the library's default
                            (DZS_PM_CHUNK_DEFAULT); -1 = no tiles.  A workgroup takes a chunk of
                            consecutive particles (compact in key order), in pieces.  Deposit:
                            a piece sums its cloud-in-cell contributions into an LDS tile
                            spanning its points, up to 4096 of them, and adds each non-zero
                            point to the mesh once.  Interpolation (only when the particles are
                            at least half as many as the mesh points): a piece loads the
                            potential its 4-point stencils read, up to 32 KB of values, into LDS
                            once.  A piece whose points do not fit (or, in a batch, that spans
                            two boxes) is halved, down to 128 particles, which read and add
                            directly.  Mesh and forces are the same bits for every value: the
                            choice changes speed only. */
} dzs_pm_params;

#define DZS_PM_CHUNK_MIN 256
#define DZS_PM_CHUNK_MAX 16384
#define DZS_PM_CHUNK_DEFAULT 2048

/* Tree (short-range) parameters: g_i = -G sum m_j r_ij g_soft(r_ij, h_ij) S(r_ij/r_s) over
 * sources closer than r_cut, S(u) = erfc(u/2) + u/sqrt(pi) exp(-u^2/4).  Opening criteria
 * (Sec. 2.1 and 2.2.1, eqs. 1 and 2), with d the distance from the target group's bounding
 * box to the node's centre of mass:
 *  - geometric: a node of side l acts as a monopole when l < theta * d; theta = 0 opens
 *    every node (exact direct sum);
 *  - relative: a node of mass M acts as a monopole when G M l^2 < alpha_open a_min d^4,
 *    a_min the smallest |g| the group's targets held before the call (their previous
 *    accelerations; a target with g = 0 makes its group open every node).  kdk_step reads
 *    the accelerations the state holds on entry; a step whose coarsening merged particles
 *    (no previous acceleration for them) falls back to the geometric criterion.
 * With either criterion, when theta <= 1 (geometric) or always (relative) the walk starts at
 * the nodes of the cells at least r_cut wide, so nodes above them are always opened. */
#define DZS_OPEN_GEOMETRIC 0
#define DZS_OPEN_RELATIVE 1
typedef struct {
    double r_s, r_cut;   /* split scale and cutoff (r_cut < L/2, r_cut <= 5 r_s) */
    double theta;        /* opening angle, >= 0 */
    int32_t leaf_size;   /* particles per tree leaf, 1..64 (0 = default 8); the context
                            holds n/2 + 4096 nodes, which leaves of fewer than 8 particles
                            can exceed in clustered states (DZS_ECAPACITY) */
    int32_t group_size;  /* targets per wave64 group, a power of two <= 64 (0 = default
                            16); each target is served by 64/group_size lanes */
    int32_t precision;   /* DZS_FP64, or DZS_FP32: interaction list and pair arithmetic in
                            FP32 on coordinates relative to the group centre (rms error
                            ~1e-6; a pair within FP32 rounding of r_cut may be kept or
                            dropped, a jump of G m S(r_cut/r_s)/r_cut^2 in that target's
                            force) */
    int32_t accumulate;  /* 0: g = g_short, 1: g += g_short */
    int32_t opening;     /* DZS_OPEN_GEOMETRIC or DZS_OPEN_RELATIVE */
    int32_t presorted;   /* tree_force only: 1 = the particles are already in the order a
                            tree build needs (ascending Morton key to level 15, as kdk_step
                            and dzs_sort_state leave them): the tree is built on them in place,
                            without sorted copies.  The order is checked on the device; an
                            input out of order computes nothing and is reported by dzs_check
                            (DZS_EINVAL).  kdk_step ignores it. */
    double alpha_open;   /* relative criterion's accuracy parameter (>= 0) */
} dzs_tree_params;

/* Lightcone crossing over one drift a0 -> a1 (positions at a0, momenta constant).
 * d0 = min-image(x - x_obs); d1 = min-image(wrap(x + p D) - x_obs), the offset the next
 * drift starts from.  A particle is emitted iff |d0|^2 - chi2_0 < 0 <= |d1|^2 - chi2_1 (the
 * sphere of radius chi(a) shrinks with a); since one drift's end test is the next drift's
 * start test, a particle is emitted once over a run of consecutive drifts.
 * The crossing time solves |d0 + p D(a0,a)| = chi(a) on [a0, a1] using the Chebyshev
 * series of chi(a) and D(a0,a) on [a0, a1] (dzs_step_factors fills all of this). */
typedef struct {
    double x_obs[3];
    double a0, a1;
    double D;               /* D(a0, a1) = int da / (a^3 H) */
    double chi2_0, chi2_1;  /* chi(a0)^2, chi(a1)^2 */
    int32_t n_cheb;         /* coefficients used, 1..DZS_CHEB_MAX */
    int32_t reserved;
    double cheb_chi[DZS_CHEB_MAX];    /* chi(a),    a = a0 + (t+1)(a1-a0)/2, t in [-1,1] */
    double cheb_drift[DZS_CHEB_MAX];  /* D(a0, a),  same variable */
} dzs_lc_params;

/* One lightcone record (64 bytes). */
typedef struct {
    uint32_t id, mult;
    double a_cross;   /* scale factor at the crossing */
    double d[3];      /* offset from the observer at the crossing */
    double p[3];      /* momentum during the drift */
} dzs_lc_record;

/* Caller-owned device ring of records.  *count (device) is advanced atomically; records
 * beyond `capacity` are dropped and *overflow (device) is set to 1.  The caller resets
 * both between uses. */
typedef struct {
    dzs_lc_record *records;
    uint64_t capacity;
    unsigned long long *count;
    uint32_t *overflow;
} dzs_lc_ring;

typedef struct {
    double K1, K2;            /* kick factors K(a0, a_h), K(a_h, a1), a_h = sqrt(a0 a1) */
    dzs_lc_params lc;         /* drift and lightcone */
    int32_t do_lightcone;     /* 0: skip the crossing test */
    int32_t do_coarsen;       /* 0: skip DZS */
    dzs_coarsen_params coarsen;
    dzs_pm_params pm;
    dzs_tree_params tree;
} dzs_step_params;

/* Individual power-of-two time steps (Sec. 2.1) inside one global step a0 -> a1: 2^max_bin
 * sub-steps of equal length in ln a; a particle in bin b steps over 2^(max_bin - b) of them,
 * each of its steps a kick-drift-kick whose kicks reach the step's midpoint in ln a.  Bins
 * are set at a0 from the accelerations the state holds: the step allowed is
 * delta = sqrt(C eps / |g|), C = 2 eta a0^3 H(a0)^2, eps = eps0 mult^(1/3), and the bin is the
 * smallest b <= max_bin with ln(a1/a0) 2^-b <= delta (|g| = 0: bin 0).  With the limiter
 * (Sec. 2.2) particles outside the sphere |x - x_obs| < R_lim (x_obs: the coarsening
 * parameters' observer) take at most the largest bin inside it (no limit when nobody is
 * inside).  Every particle ending a step at a sub-step boundary gets its new force there
 * (PM + tree; the walk serves only those targets).  DZS runs once all particles are
 * synchronised at a1 (after the closing kicks), and a coarsening that merged particles is
 * followed by a new force for the whole state.
 *
 * pm_global = 1 (the TreePM split carried into time, Sec. 2.1; needs a context created with
 * DZS_CAP_HIER_SPLIT): the long-range force acts on the global step only.  The entry g is
 * taken as the total force at a0; the PM force at a0 is computed and g - g_PM is the
 * short-range part.  The step opens with the half-kick g_PM(a0) K(a0, a_h) of every particle
 * (a_h = sqrt(a0 a1)), runs the sub-steps above with the short-range force alone, and closes
 * with the half-kick g_PM(a1) K(a_h, a1) after the last short-range kicks; the state keeps
 * g_PM(a1) + g_SR(a1).  The particles are sorted and the tree built once, at a0; at every
 * sub-step boundary the nodes' moments and bounding boxes are recomputed from the drifted
 * positions (the topology kept, members that crossed a face of the periodic box unwrapped)
 * and the walk, started at the root, serves the targets that end a step there.  The state
 * is left in the key order of a0 unless DZS ran. */
#define DZS_HIER_MAX_BIN 6
typedef struct {
    int32_t max_bin;   /* 0..DZS_HIER_MAX_BIN (0: the plain step) */
    int32_t limiter;   /* 1: cap the bins outside the sphere of radius R_lim */
    double eta;        /* accuracy parameter of the bin rule (> 0) */
    double R_lim;      /* limiter radius (the lightcone radius at a0 plus the buffer) */
    double a0, a1;     /* the global step */
    double omega_m;    /* flat LCDM */
    int32_t pm_global; /* 1: the long-range force on the global step only (see above) */
    int32_t reserved;  /* 0 */
} dzs_hier_params;

/* ---- context ------------------------------------------------------------------------ */

/* Create a context on HIP device `device` and allocate all its scratch for `cap`: about
 * 123 bytes per particle (keys and sort indices 24; one arena of 89 shared by the tree, with
 * node capacity max_particles/2 + 4096, and the DZS coarsening buffers; group starts 4; the
 * relative criterion's |g| 4; time-step bins and the walk's target flags 2), plus 28 bytes per
 * particle of sorted copies for tree_force unless DZS_CAP_NO_COPIES, plus 44 bytes per
 * particle with DZS_CAP_HIER_SPLIT, plus the meshes (32 bytes per cell, 12 with
 * DZS_CAP_FP32_MESHES).  No call allocates device memory afterwards.
 * Returns DZS_ENOMEM if the device memory does not suffice. */
dzs_status dzs_ctx_create(dzs_ctx **out, int32_t device, const dzs_capacity *cap);
dzs_status dzs_ctx_destroy(dzs_ctx *ctx);
/* Text of the context's last failure ("" if none); valid until the next call. */
const char *dzs_last_error(const dzs_ctx *ctx);
/* Identification of the build: the first 16 hex digits of the SHA-256 of the sources the
 * library was compiled from (HIP and C++ sources, internal headers, this header, the build
 * script).  Lets a binding refuse a library that is stale against its sources.  Static
 * string; never fails. */
const char *dzs_source_hash(void);

/* One global step with individual time steps (dzs_hier_params).  prm supplies pm, tree,
 * coarsen, do_lightcone and do_coarsen (its K1, K2 and lc are not read: the sub-step factors
 * come from hp).  bins_out (optional, device, >= n bytes) receives each particle's bin, in
 * the order of the state on entry.  The state is left in key order (or (key, id) order
 * after a coarsening that merged nothing), synchronised at a1 with g = the force at a1.
 * The relative opening criterion is not supported here (DZS_EINVAL).  Synchronises the
 * stream (the bins' counts, the limiter, the capacity checks, the coarsening count): a
 * sub-step boundary where no populated bin ends a step is skipped, and with
 * DZS_CAP_HIER_SPLIT a boundary where some targets end one walks only the tree's groups that
 * hold them. */
dzs_status kdk_step_hier(dzs_ctx *ctx, const dzs_box *box, dzs_particles *state,
                         const dzs_step_params *prm, const dzs_hier_params *hp,
                         dzs_lc_ring *ring, dzs_coarsen_report *report, uint8_t *bins_out,
                         void *stream);

/* Host helper: flat LCDM (Omega_m = omega_m, no radiation) kick, drift and lightcone
 * factors for the step a0 -> a1: K1, K2, lc.D, lc.chi2_0, lc.chi2_1, lc.a0, lc.a1 and the
 * Chebyshev series, by Gauss-Legendre quadrature.  Leaves every other field untouched. */
dzs_status dzs_step_factors(double a0, double a1, double omega_m, dzs_step_params *out);

/* ---- run control and forecast (host only, no device work) ----------------------------- */

/* Halt conditions of a DZS run (Sec. 4.1.1): a run stops and writes its state, so that it can
 * be continued with resources fitted to its shrinking particle count, when
 *   - the workload balance (largest over mean work per task) exceeds max_balance (> 0), or
 *   - R(t) = N(t) / N_init falls below min_ratio, or
 *   - the wall time t has reached runtime_limit_s (> 0) and R, extrapolated linearly from the
 *     previous sample (t_prev, ratio_prev), would fall below min_ratio within
 *     restart_window_s of the restart.
 * Returns the DZS_HALT_* reasons that hold (0: carry on).  Null arguments return 0. */
#define DZS_HALT_BALANCE 1u
#define DZS_HALT_RATIO 2u
#define DZS_HALT_PREDICTED 4u
typedef struct {
    double max_balance;       /* <= 0: no balance condition */
    double min_ratio;         /* R threshold */
    double runtime_limit_s;   /* <= 0: no run-time limit */
    double restart_window_s;  /* look-ahead after a restart */
} dzs_halt_params;
typedef struct {
    double balance;           /* current workload balance */
    double ratio, ratio_prev; /* R now and at the previous sample */
    double t, t_prev;         /* wall time now and at the previous sample, s */
} dzs_halt_state;
uint32_t dzs_halt_check(const dzs_halt_params *prm, const dzs_halt_state *st);

/* Forecast of the DZS speed-up T_STD / T_DZS (Sec. 4.2, eqs. 6-7): a run costs as much as
 * without DZS until a_DZS, where the lightcone sphere holds half the box (4/3 pi chi^3 =
 * L^3 / 2), and nothing after; the cost grows as a^r with r interpolated linearly in the
 * particle mass m between 0.4 (the 8192 Mpc/h, 512^3 run) and 1 (the 512 Mpc/h, 512^3 run),
 * extrapolated to finer masses and held at 0.4 for coarser ones: speedup = a_DZS^-r.
 * L in Mpc/h; m in 1e10 Msun/h (flat LCDM, Omega_m = omega_m).  DZS_EINVAL if the sphere
 * already holds half the box at a = 1e-4 or an argument is out of range. */
typedef struct {
    double a_dzs, r, speedup, particle_mass;
} dzs_forecast;
dzs_status dzs_forecast_speedup(double L, double n_part, double omega_m, dzs_forecast *out);

/* ---- the gravity step ---------------------------------------------------------------- */

/* DZS coarsening (Sec. 2.2).  Reorders the state in place to ascending (Morton key, id),
 * replaces each merging node's members by one particle (mult = sum, x = centre of mass,
 * p = mult-weighted mean momentum, id = smallest member id, type = 1) and updates inout->n.
 * The dynamical criterion reads g (must be non-null); g is not preserved.  group_of (optional, device, >= n entries) receives for each
 * particle's index on entry the index of the particle representing it on exit.
 * Synchronises the stream (the new count is read back). */
dzs_status dzs_coarsen(dzs_ctx *ctx, const dzs_box *box, dzs_particles *inout,
                       const dzs_coarsen_params *prm, uint32_t *group_of,
                       dzs_coarsen_report *report, void *stream);

/* PM long-range acceleration into g (or added to g).  Particle order is left unchanged. */
dzs_status pm_force(dzs_ctx *ctx, const dzs_box *box, const dzs_particles *p,
                    const dzs_pm_params *prm, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): pm_force with its meshes in a static
 * device array of the library instead of a context, so no call allocates anything.  The
 * array holds meshes of up to DZS_PM_NOALLOC_MAX_SIDE points per side (32 bytes per cell plus
 * the per-axis tables: 8 MiB + 2 KiB), one copy per GPU the library runs on, held until the
 * process ends; a larger mesh side fails with DZS_ECAPACITY.  Arguments, results (the same
 * bits as pm_force) and the other errors are those of pm_force; no context means no error
 * text.  The first call on a device looks up that device's copy; a call with new mesh
 * parameters uploads the mesh tables and synchronises the stream, as pm_force does.  Every
 * call on a GPU shares that GPU's array (the density is cleared by each call), so calls that
 * overlap on one GPU (two streams, two host threads) race. */
#define DZS_PM_NOALLOC_MAX_SIDE 64
dzs_status pm_force_noalloc(const dzs_box *box, const dzs_particles *p,
                            const dzs_pm_params *prm, void *stream);

/* Tree short-range acceleration into g (or added to g) of the targets: targets (device,
 * n_targets indices into the particle arrays, each below n and listed once) or every particle
 * when targets is NULL; the other entries of g are not touched.  Every particle is a source.
 * Particle order is left unchanged: the tree is built on sorted copies of the positions and
 * multiplicities (or, with prm->presorted, on the particles themselves) and the force is
 * written through the permutation.  Only enqueues work: the tree's node capacity, the walk's
 * stack depth, the presorted order and the target indices are checked on the device and
 * reported by the next dzs_check (DZS_ECAPACITY, DZS_EINVAL). */
dzs_status tree_force(dzs_ctx *ctx, const dzs_box *box, const dzs_particles *p,
                      const dzs_tree_params *prm, const uint32_t *targets, uint64_t n_targets,
                      void *stream);

/* Lightcone crossing test and solve for the drift described by prm (does not move the
 * particles). */
dzs_status lightcone_emit(dzs_ctx *ctx, const dzs_box *box, const dzs_particles *p,
                          const dzs_lc_params *prm, dzs_lc_ring *ring, void *stream);

/* One kick-drift-kick step a0 -> a1:
 *   p += g K1; lightcone over the drift (optional); x = wrap(x + p D);
 *   DZS coarsening at a1 (optional; skipped when R_lc + b >= sqrt(3)/2 L, where no node can
 *   qualify); reorder the state by Morton key; g = PM + tree; p += g K2.
 * The state is left sorted by Morton key.  report (optional) receives the coarsening
 * counts.  A step whose coarsening can merge synchronises the stream (the new count is read
 * back); any other step only enqueues work, so it can be captured into a HIP graph (after one
 * eager call with the same mesh parameters, which uploads the mesh tables) and replayed: the
 * factors in prm are then those of the capturing call.  The tree's node capacity and the
 * walk's stack depth are checked on the device and reported by the next dzs_check.
 * The mesh solve runs on a stream the context owns (default priority), forked from and
 * joined back to `stream` with events inside the call, so all of the step's work is ordered
 * before whatever the caller enqueues on `stream` next. */
dzs_status kdk_step(dzs_ctx *ctx, const dzs_box *box, dzs_particles *state,
                    const dzs_step_params *prm, dzs_lc_ring *ring, dzs_coarsen_report *report,
                    void *stream);

/* ---- many boxes in one step ----------------------------------------------------------- */

#define DZS_BATCH_MAX 512

/* A batch of independent periodic boxes (an ensemble of uneven particle counts, e.g. after
 * per-box DZS coarsening) advanced together: box b owns particles [first[b], first[b+1]) of
 * one state.  All host arrays, read during the call only. */
typedef struct {
    uint32_t n_boxes;       /* 1 .. DZS_BATCH_MAX */
    uint32_t reserved;
    const dzs_box *boxes;   /* [n_boxes]: L, m0, eps0 of each box; G equal for all */
    const uint64_t *first;  /* [n_boxes + 1]: first[0] = 0, non-decreasing, first[n_boxes] =
                               state->n */
    const int32_t *ng;      /* [n_boxes]: PM mesh side of each box (2^a 3^b, a >= 1, 8 .. 1024); the
                               meshes together need sum ng^3 <= max_mesh_side^3 of the context */
    const double *r_s;      /* [n_boxes]: split scale of each box */
    const double *r_cut;    /* [n_boxes]: cutoff, r_cut < L/2, r_cut <= 5 r_s, the same
                               r_cut / r_s for every box */
} dzs_batch;

/* One kick-drift-kick step a0 -> a1 of every box of a batch, as kdk_step does for one box
 * (the per-box physics is the same), with one launch of each kernel for all boxes: one
 * sort of keys that carry the box in their top three octal digits (2^18 cells per side
 * below them), one tree over all boxes (each box below the node of its digits), one walk
 * over every box's target groups, one deposit and one interpolation, and one set of FFT
 * launches per distinct mesh side.  prm supplies K1, K2, the lightcone drift (x_obs, chi^2,
 * Chebyshev series; every box's particles are tested against the same sphere), the PM
 * precision and the tree's opening angle, leaf and group size and precision (r_s and r_cut
 * come from the batch); do_coarsen must be 0 (coarsen each box with dzs_coarsen).  Each
 * box's particles are left Morton-sorted within its range.
 * Synchronises the stream only when the batch differs from the previous call (its tables are
 * then rebuilt and uploaded); otherwise the call only enqueues work, so it can be captured
 * into a HIP graph once and replayed for every step: a captured call reads K1, K2 and the
 * lightcone drift, when the graph runs, from a device block filled from the context's pinned
 * host staging, which the capturing call and kdk_step_batch_stage write (eager calls pass
 * them as kernel arguments).  The tree's node capacity and the walk's stack
 * depth are checked on the device; dzs_check reports an overflow. */
dzs_status kdk_step_batch(dzs_ctx *ctx, const dzs_batch *batch, dzs_particles *state,
                          const dzs_step_params *prm, dzs_lc_ring *ring, void *stream);

/* Stage K1, K2 and the lightcone drift of prm for the next replay of a captured
 * kdk_step_batch (host memory only; call after the previous replay has finished). */
dzs_status kdk_step_batch_stage(dzs_ctx *ctx, const dzs_step_params *prm);

/* Synchronise the stream and report (and clear) what the device recorded since the last
 * check: a tree node-capacity or walk stack-depth overflow (DZS_ECAPACITY), or a tree_force
 * input out of key order under presorted or a target index out of range (DZS_EINVAL). */
dzs_status dzs_check(dzs_ctx *ctx, void *stream);

/* ---- parts of the path, exposed for testing and measurement --------------------------- */

/* Morton keys (21 bits per dimension, x in the highest bit of each triple) of the
 * particles in their current order into keys (device, n entries). */
dzs_status dzs_morton_keys(dzs_ctx *ctx, const dzs_box *box, const dzs_particles *p,
                           uint64_t *keys, void *stream);

/* Reorder the state in place by ascending Morton key (stable), optionally breaking ties by
 * ascending id; perm (optional, device) receives the entry index of each sorted slot. */
dzs_status dzs_sort_state(dzs_ctx *ctx, const dzs_box *box, dzs_particles *p,
                          int32_t ties_by_id, uint32_t *perm, void *stream);

/* Number of source-target interactions inside the cutoff evaluated by the tree walk since
 * the context was created or last reset (the algorithmic pair work).  Synchronises the
 * device. */
dzs_status dzs_counters(dzs_ctx *ctx, int32_t reset, uint64_t *pair_interactions);

/* Average duration in milliseconds of each internal kernel class over the calls made since
 * the last reset, measured with HIP events on the call's stream when timing is enabled.
 * enable: 0 stops timing; 1 times every class; a larger value is a mask of the classes to time
 * (bit c + 1 for the class written at index c); a negative value only writes the class names
 * (names may then be NULL: the count alone) and changes nothing.
 * names/values: caller arrays of `cap` entries; returns the number of classes written. */
int32_t dzs_timing(dzs_ctx *ctx, int32_t enable, int32_t reset, const char **names,
                   double *ms_avg, uint64_t *calls, int32_t cap);

#ifdef __cplusplus
}
#endif

#endif /* DZS_H */
