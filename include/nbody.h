/*
 * nbody.h -- C ABI of the MI355X direct-summation N-body library.
 *
 * What the library computes (paper: Portegies Zwart & Bedorf,
 * "Computational Gravitational Dynamics with Modern Numerical Accelerators",
 * section "Optimizations for the GPU"): the particles are split into
 * j-particles, which exert a force, and i-particles, which receive it; the
 * i-forces are independent sums over the j-set, so they are computed in
 * parallel, and when the i-set is small the j-set is also split into subsets
 * whose partial forces are summed by a second kernel.  The forces drive the
 * 4th-order Hermite predictor-corrector with block time steps that the paper
 * names for its direct code (sections "Simulating Collisional systems with
 * direct force evaluation methods" and "Simulating galaxy mergers with
 * supermassive black holes").  The paper writes none of the formulas; the
 * library uses G = 1, Plummer softening and the Makino-Aarseth Hermite form:
 *
 *   r = x_j - x_i,  u = v_j - v_i,  s = |r|^2 + eps2,
 *   a_i    =  sum_{j != i} m_j r s^{-3/2}
 *   jdot_i =  sum_{j != i} m_j [u s^{-3/2} - 3 (r.u) r s^{-5/2}]
 *   phi_i  = -sum_{j != i} m_j s^{-1/2}
 *
 * The self pair is excluded by index.  With eps2 == 0 a pair at s == 0
 * (coincident distinct particles) contributes nothing.
 *
 * Conventions for every entry point
 *  - Return value: NB_OK (0) or a negative nb_status; nb_last_error(ctx)
 *    then describes the failure.  Argument errors are detected on the host
 *    before anything is launched, so no output is written.  No exception or
 *    abort crosses the ABI.
 *  - Every array pointer is a DEVICE pointer (e.g. a torch tensor's
 *    data_ptr() on the context's GPU) owned by the caller; the library keeps
 *    no reference to it after the call returns.  Arrays of 3-vectors are
 *    row-major [n][3] doubles (torch shape (n, 3), contiguous).
 *  - Calls are asynchronous on the context's stream (nb_set_stream); outputs
 *    are valid once that stream has been synchronised.  A context is used
 *    by one host thread at a time, and its calls must not overlap on the
 *    device: they share the context's work-queue counters and workspace, so
 *    every call -- and every replay of a graph that captured calls -- goes to
 *    one stream, or to streams ordered with events.  Overlapping calls give
 *    wrong results; nb_sync detects the counters they leave behind.
 *  - Index arrays are int32; an index outside [0, N) is an error only where
 *    stated (device-resident indices cannot be checked without a copy).
 *  - The context owns only its launch table, a workspace for j-split
 *    partial sums (grown on demand with hipMalloc outside any stream capture)
 *    and a few bytes of device scratch.  If the environment variable
 *    NB_MAX_WORKSPACE_BYTES holds a decimal byte count, a call whose j-split
 *    (or scalar-path mirror) workspace would exceed it fails with NB_ENOMEM
 *    before anything is launched, leaving every output untouched.  The tree
 *    code keeps its own buffers (about 200 bytes per particle plus its
 *    interaction lists), which the cap does not cover.
 *  - NB_LOG, read by nb_create: 1 prints every error a call on the context
 *    returns (the nb_last_error text with its code) to stderr; 2 also prints
 *    each launch shape the host chooses (K, L, S, T, WG, work items, and the
 *    regimes of a count-on-device launch).  Lines start with "nbody:".
 *    Unset, empty or 0: silent.
 */
#ifndef NBODY_H
#define NBODY_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nb_ctx nb_ctx;

enum nb_status {
    NB_OK = 0,
    NB_EINVAL = -1,    /* bad argument (size, null pointer, range, NaN eps2 ...) */
    NB_ENOMEM = -2,    /* device allocation failed or over NB_MAX_WORKSPACE_BYTES */
    NB_EDEVICE = -3,   /* HIP runtime error (launch, stream, device) */
    NB_ENOTSUP = -6    /* combination the library does not provide */
};

enum nb_precision {
    NB_PREC_FP64 = 0,  /* every pair in IEEE double */
    NB_PREC_MIXED = 1, /* r formed in double and rounded to float; the pair
                          arithmetic in float; per-tile float sums folded
                          into a double-precision accumulator */
    NB_PREC_MIXED_DS = 2 /* as NB_PREC_MIXED, but r formed in emulated double
                          precision on float hardware: positions split into
                          hi + lo floats, r = (hi_j - hi_i) + (lo_j - lo_i)
                          (the paper's remedy for single-precision devices) */
};

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device `device` (>= 0) computing in `precision`.
 * Fails with NB_EINVAL for a bad device or precision, NB_EDEVICE when the
 * device cannot be initialised (no GPU, missing gfx950 code object). */
int nb_create(nb_ctx **out, int device, int precision);
int nb_destroy(nb_ctx *ctx);
/* Stream for all later launches (a hipStream_t; NULL = the null stream). */
int nb_set_stream(nb_ctx *ctx, void *hip_stream);

/* Wait for the context's stream and report errors the kernels found on the
 * device since the last nb_sync: an active_idx entry outside its valid range
 * ([0, N) for nbody_forces, nbody_forces_devcount, nbody_forces6,
 * hermite_correct, hermite6_correct and the block steps; [0, N_i) for
 * nbody_forces_ij; the system's own rows for nbody_forces_batch) is skipped
 * by every kernel that reads it -- no output row, no particle update is
 * written for it and nothing is read through it -- and sets a bit in device
 * memory, so no call has to copy active_idx to the host.  Returns
 * NB_EINVAL (message in nb_last_error) once for any such entries and clears
 * the bit; NB_OK otherwise; NB_EDEVICE on a failed synchronisation.
 * It also checks the context's work-queue counters, which every force
 * launch leaves at zero: non-zero counters mean that calls overlapped on the
 * device (see the conventions above).  They are then cleared, so later calls
 * are correct again, and NB_EINVAL reports that results since the last
 * nb_sync cannot be trusted. */
int nb_sync(nb_ctx *ctx);

/* The same range test on a host array: NB_OK when every active[k], k <
 * n_active, lies in [lo, hi), else NB_EINVAL with the first offending k in
 * *first_bad (-1 when all pass; first_bad may be NULL).  Needs no device. */
int nb_check_active_host(const int32_t *active, int64_t n_active, int64_t lo, int64_t hi, int64_t *first_bad);

/* Device memory held by the context's growable buffers -- the j-split
 * workspace and the scalar j-path's record mirror, the two that
 * NB_MAX_WORKSPACE_BYTES bounds -- in *bytes.  NB_EINVAL for null arguments. */
int nb_workspace_bytes(const nb_ctx *ctx, int64_t *bytes);
int nb_set_precision(nb_ctx *ctx, int precision);
int nb_get_precision(const nb_ctx *ctx);
const char *nb_last_error(const nb_ctx *ctx);
/* Library version string (static storage). */
const char *nb_version(void);

/* ---- launch configuration (the j-split of the paper) --------------------
 * K = i-particles per lane (1, 2, 4; 3 for L <= 0); L = lanes sharing one
 * i-particle, each taking every L-th j of a tile staged in LDS, combined by
 * cross-lane and cross-wave reduction (1, 2, 4, ..., 256); L = 0 selects the
 * scalar j-path (one lane per i-particle, j-records converted once per call
 * into a mirror and read with a wave-uniform index through the scalar
 * cache); L = -1 the hybrid path (mixed precision only, else as L = 0:
 * positions through the scalar cache, velocities and masses through LDS).
 * S = j-subsets, one work item each per i-block, whose partial sums a second
 * kernel adds in fixed order (>= 1).  The paper's rule is that the device is
 * saturated once N_i times the number of j-subsets exceeds the number of
 * threads.  T = j-particles per LDS tile, also the length a j-subset is
 * rounded up to (S <= ceil(N / T)); WG = threads per workgroup, so an
 * i-block holds (WG / L) K i-particles (L = 0: WG K).  T and WG = 0 mean
 * 256, the size every shape is built for; besides that the library builds
 * (T, WG) = (128, 256), (128, 128) and (64, 64) for (K, L) in {(1, 1),
 * (1, 4), (1, 16), (2, 1), (2, 4)}, and WG = 128 (T = 256) for the scalar
 * j-path with K = 1, 2.  eps2 = 0 runs K = 1 with T = WG = 256.
 * nb_set_launch forces one configuration for every later force call
 * (K = 0 returns to automatic choice); nb_get_launch reports the
 * configuration the context would use for (N, n_active) (T and WG may be
 * NULL).  Errors: NB_EINVAL for values outside the ranges above,
 * NB_ENOTSUP for a combination the library does not build. */
int nb_set_launch(nb_ctx *ctx, int K, int L, int S, int T, int WG);
int nb_get_launch(nb_ctx *ctx, int64_t N, int64_t n_active, int *K, int *L, int *S, int *T, int *WG);
/* Install one entry of the automatic table: for this precision, N >= n_min
 * and n_active in [act_min, act_max], use the shape (K, L, T, WG), and
 * choose S by the saturation rule aiming at `items` work items (i-blocks x
 * j-subsets; 0 = 4 per compute unit).  The same entry drives host-count and
 * device-count launches, so both split the work identically.  Later
 * entries take precedence on their range.  Used by the autotuner front end
 * to load its cache. */
int nb_tune_add(nb_ctx *ctx, int precision, int64_t n_min, int64_t act_min, int64_t act_max,
                int K, int L, int items, int T, int WG);
/* One entry of the batched kernel's table (nbody_forces_batch and
 * nb_block_step_batch use one shape for the whole batch): for this
 * precision, use K and L (L = 0: the scalar j-path, K in {1, 2}; L in
 * {1, 4, 16, 64}: the LDS layout, K = 1, or K = 2 with L <= 16) when the key
 * lies in [key_min, key_max].  kind 1 keys nbody_forces_batch by the mean
 * active rows per system, ceil(total active / C); kind 2 keys
 * nb_block_step_batch by the mean system size, ceil(N / C).  Later entries
 * take precedence.  Without an entry the batch takes K = 1 and the LDS
 * layout nearest the single-system table's L for the mean size.  A batch
 * with any unsoftened system (eps2[c] = 0) runs the entry's L with K = 1
 * (the masked kernels hold one i-particle per lane).
 * nb_get_batch_launch reports the shape for a key (N = total rows).
 * Errors: NB_EINVAL for a bad kind, range or K, NB_ENOTSUP for a shape the
 * library does not build.  nb_tune_clear empties both tables. */
int nb_tune_add_batch(nb_ctx *ctx, int precision, int kind, int64_t key_min, int64_t key_max, int K, int L);
int nb_get_batch_launch(nb_ctx *ctx, int kind, int64_t key, int64_t N, int *K, int *L);
int nb_tune_clear(nb_ctx *ctx);
/* How nbody_forces and nbody_forces_ij add the S partial sums of a j-split
 * (S > 1).  mode 0 (the default): each subset writes its partials and a
 * second kernel adds them in a fixed order -- the results do not depend on
 * the launch.  mode 1: the paper's alternative, where every subset's work
 * item adds its part into the outputs with device-scope atomic adds (after
 * a kernel that seeds them); no workspace and no second kernel, but the
 * order of the additions, and so the last bits, vary from run to run.
 * Mode 1 runs the LDS shapes with K <= 2 and T = WG = 256 (a call whose
 * shape is another gets NB_ENOTSUP, as does eps2 = 0); device-count calls,
 * block steps and nbody_forces_noalloc always use mode 0.  Errors:
 * NB_EINVAL for another mode. */
int nb_set_split_sum(nb_ctx *ctx, int mode);
/* Time the force kernel for one configuration on the caller's arrays:
 * `reps` launches after one warm-up, on the context stream, with HIP
 * events; returns the mean milliseconds per launch in *ms.  Synchronises
 * the stream.  This is the measurement primitive of the autotuner. */
int nb_time_forces(nb_ctx *ctx, int K, int L, int S, int T, int WG,
                   const double *pos, const double *vel, const double *mass, int64_t N,
                   const int32_t *active_idx, int64_t n_active, double eps2,
                   double *acc, double *jerk, double *pot, int reps, double *ms);

/* ---- forces --------------------------------------------------------------
 * nbody_forces: acceleration, jerk and potential of the i-set
 * active_idx[0..n_active) in the field of all N particles.
 *   pos, vel  [N][3]  positions and velocities of the j-set (the i-particles
 *                     use their own rows of the same arrays)
 *   mass      [N]     masses (zero allowed: such a particle receives forces
 *                     but exerts none -- the way to express an i-set that is
 *                     not part of the j-set)
 *   active_idx[n_active] rows receiving forces; duplicates allowed
 *   eps2      Plummer softening squared, finite and >= 0
 *   acc, jerk [n_active][3], pot [n_active]: compact outputs, row k for
 *             particle active_idx[k]
 * Errors: NB_EINVAL for N < 1 or N >= 2^31, n_active < 0, negative or
 * non-finite eps2, a null pointer when n_active > 0.  n_active == 0 does
 * nothing.  active_idx is device memory and is checked on the device: an
 * entry outside [0, N) gets no output row (its rows of acc/jerk/pot are left
 * as they were) and is reported by the next nb_sync as NB_EINVAL. */
int nbody_forces(nb_ctx *ctx, const double *pos, const double *vel, const double *mass, int64_t N,
                 const int32_t *active_idx, int64_t n_active, double eps2,
                 double *acc, double *jerk, double *pot);

/* nbody_forces for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments, launch choice and kernels, but the j-split partials
 * and the j-record mirror live in a fixed scratch array of
 * NB_NOALLOC_SCRATCH_BYTES (256 MiB) compiled into the library, one per
 * device, held until the process ends.  The call allocates nothing.
 * Scratch needed: S*7*n_active*8 bytes of partials when the j-split S > 1
 * (rounded up to 256), plus (N+1) j-records (40 B mixed, 56 B FP64) when the
 * scalar j-path is chosen.  The launch is the one nb_get_launch reports, and
 * the results equal nbody_forces' bit for bit, unless its partials do not
 * fit: then the automatic choice takes the largest S that fits (the sums
 * differ only in their order).  Errors: as nbody_forces, plus NB_ENOMEM
 * (nothing launched, message with the bytes needed) when a launch forced by
 * nb_set_launch does not fit, or when the mirror alone does not (N above
 * about 4.7 million in FP64) -- use nbody_forces then -- and NB_EDEVICE when
 * the scratch's device address could not be resolved.  Every call on one
 * device shares that device's scratch, which keeps the last call's contents
 * (the kernels write every element they read, nothing needs clearing): calls
 * that overlap on one device -- other streams, other contexts, other host
 * threads -- race and must be ordered by the caller. */
#define NB_NOALLOC_SCRATCH_BYTES (256u << 20)
int nbody_forces_noalloc(nb_ctx *ctx, const double *pos, const double *vel, const double *mass, int64_t N,
                         const int32_t *active_idx, int64_t n_active, double eps2,
                         double *acc, double *jerk, double *pot);

/* Forces on particles that are not part of the j-set (the paper's section
 * on GPU optimisations lets the i-set be a different set of particles from
 * the j-set; the coupling kicks of a Hamiltonian split need exactly this):
 * acceleration, jerk and potential of the rows active_idx[0..n_active) of
 * pos_i/vel_i ([N_i][3]) in the field of the N_j particles pos_j/vel_j/mass_j.
 * Every (i, j) pair contributes -- no pair is taken to be a self pair -- and
 * with eps2 == 0 a pair at zero distance contributes nothing.  Outputs as
 * nbody_forces.  Errors as nbody_forces (with N_j for N), plus NB_EINVAL for
 * N_i outside [0, 2^31) or empty or null i arrays when n_active > 0.
 * active_idx entries outside [0, N_i) are skipped and reported by nb_sync. */
int nbody_forces_ij(nb_ctx *ctx, const double *pos_j, const double *vel_j, const double *mass_j, int64_t N_j,
                    const double *pos_i, const double *vel_i, int64_t N_i,
                    const int32_t *active_idx, int64_t n_active, double eps2,
                    double *acc, double *jerk, double *pot);

/* Same, with the active count read from device memory (*n_active_dev) when
 * the kernels run, so a captured graph can replay it for any count.
 * max_active bounds *n_active_dev and sizes the launch; the launch
 * configuration is chosen on the device per call from the count. */
int nbody_forces_devcount(nb_ctx *ctx, const double *pos, const double *vel, const double *mass,
                          int64_t N, const int32_t *active_idx, const int32_t *n_active_dev,
                          int64_t max_active, double eps2, double *acc, double *jerk, double *pot);

/* Batched forces over C independent systems (clusters) stored back to back:
 * system c owns rows offsets[c] .. offsets[c+1]-1 of pos/vel/mass (host
 * array offsets[C+1], offsets[0] = 0, non-decreasing) and has softening
 * eps2[c] (host array).  Its i-set is active_idx[act_offsets[c] ..
 * act_offsets[c+1]) (device array of GLOBAL row numbers inside system c;
 * act_offsets is a host array), outputs are compact in the same order.
 * Pairs across systems never interact.  One launch covers every system:
 * the work list (system, i-block, j-chunk) is built on the host and the
 * persistent kernel walks it.  Errors as nbody_forces, plus NB_EINVAL for
 * decreasing offsets or act_offsets or C < 1; an entry outside its system's
 * rows is skipped and reported by nb_sync. */
int nbody_forces_batch(nb_ctx *ctx, const int64_t *offsets, int64_t C, const double *eps2,
                       const double *pos, const double *vel, const double *mass,
                       const int32_t *active_idx, const int64_t *act_offsets,
                       double *acc, double *jerk, double *pot);

/* ---- sixth-order Hermite ------------------------------------------------
 * A higher-order Hermite scheme (the paper cites Hermite integrators of order
 * above four for its direct method, section "Simulating Collisional systems
 * with direct force evaluation methods", and writes none down).  Every
 * particle carries x, v, a, jdot, snap s and crackle c; time and levels are
 * kept as for the fourth-order calls above.
 *
 * nbody_forces6: acceleration, jerk, snap and potential of the i-set
 * active_idx[0..n_active), every particle moving with its own pos, vel and
 * acceleration acc_j ([N][3], e.g. the predicted ones).  For r = x_j - x_i,
 * u = v_j - v_i, w = a_j - a_i, s = |r|^2 + eps2:
 *   snap_i = sum_{j != i} m_j [w s^-3/2 - 6 (r.u) u s^-5/2 - 3 (u.u + r.w) r s^-5/2
 *                              + 15 (r.u)^2 r s^-7/2]
 * and acc, jerk, pot as nbody_forces.  Double precision throughout (the
 * context's precision does not apply).  Outputs [n_active][3] (pot
 * [n_active]); errors as nbody_forces. */
int nbody_forces6(nb_ctx *ctx, const double *pos, const double *vel, const double *acc_j, const double *mass,
                  int64_t N, const int32_t *active_idx, int64_t n_active, double eps2,
                  double *acc, double *jerk, double *snap, double *pot);

/* Predict every particle to t_next (d = (t_next_tick - t_tick[i]) dt_min):
 *   pos_p = x + v d + a d^2/2 + j d^3/6 + s d^4/24 + c d^5/120
 *   vel_p = v + a d + j d^2/2 + s d^3/6 + c d^4/24
 *   acc_p = a + j d + s d^2/2 + c d^3/6 */
int hermite6_predict(nb_ctx *ctx, const double *pos, const double *vel, const double *acc, const double *jerk,
                     const double *snap, const double *crackle, const int64_t *t_tick, int64_t t_next_tick,
                     double dt_min, int64_t N, double *pos_p, double *vel_p, double *acc_p);

/* Correct the active particles after their new acc1/jerk1/snap1 (compact
 * [n_active][3]).  With h = the particle's step, the quintic a(t) through
 * (a, jdot, snap) at both ends gives crackle c0, pop p0 and the fifth
 * derivative q0 at the start; x and v become the exact integrals of that
 * quintic; a, jdot, snap take the new values, crackle the end-of-step
 * c1 = c0 + p0 h + q0 h^2/2; t_tick advances by the step; the new level
 * comes from dt* = eta ((sqrt(|a1||s1|) + |j1|)/(sqrt(|c1||q0|) + |p1|))^(1/3),
 * p1 = p0 + q0 h (dt_max when the denominator is 0), with the level rules of
 * hermite_correct (clamps counted in *clamp_count_dev, may be NULL).
 * active_idx must not repeat an index; N is the number of particles, and
 * entries outside [0, N) are skipped and reported by nb_sync. */
int hermite6_correct(nb_ctx *ctx, const int32_t *active_idx, int64_t n_active, int64_t N, const double *acc1,
                     const double *jerk1, const double *snap1, double *pos, double *vel, double *acc, double *jerk,
                     double *snap, double *crackle, int64_t *t_tick, int32_t *dt_level, double eta, double dt_max,
                     int32_t max_level, int64_t *clamp_count_dev);

/* Start-up levels: dt* = eta_s min(|a|/|j|, sqrt(|a|/|s|)) over the terms
 * with a non-zero denominator (dt_max if none); level = smallest k >= 0 with
 * dt_max 2^-k <= dt*. */
int hermite6_startup(nb_ctx *ctx, const double *acc, const double *jerk, const double *snap, int64_t N,
                     double eta_s, double dt_max, int32_t max_level, int32_t *dt_level);

/* One sixth-order block step with no host synchronisation: schedule (as
 * nb_block_step), predict all particles, forces6 on the scheduled active
 * set (count read on the device), correct.  Scratch arrays pos_p, vel_p,
 * acc_p [N][3], active [N], acc1, jerk1, snap1 [N][3], pot1 [N]; sched[4]
 * as nb_block_step. */
int nb_block_step6(nb_ctx *ctx, int64_t N, double eps2, double eta, double dt_max, int32_t max_level,
                   const double *mass, double *pos, double *vel, double *acc, double *jerk, double *snap,
                   double *crackle, int64_t *t_tick, int32_t *dt_level, double *pos_p, double *vel_p,
                   double *acc_p, int32_t *active, double *acc1, double *jerk1, double *snap1, double *pot1,
                   int64_t *sched, int64_t t_stop_tick);

/* ---- tree code -------------------------------------------------------------
 * Barnes-Hut forces of every particle (the paper's collisionless method,
 * section "Simulating collisionless systems with hierarchical
 * domain-decomposition methods" and its "Implementation"), entirely on the
 * device:
 *  - box: lo = per-dimension minimum of pos, side = the power of two 2^e
 *    >= (1 + 2^-10) x the largest extent (1 if all positions coincide),
 *    h = side 2^-21, integer coordinates floor((x - lo)/h) clamped to
 *    [0, 2^21 - 1];
 *  - particles sorted along the 63-bit Peano-Hilbert curve (Skilling's
 *    construction), ties by index;
 *  - cells: the particles sharing a key prefix; a cell holding more than
 *    n_crit particles is split into its non-empty children (down to prefix
 *    level 21); each cell's cube, mass, centre of mass X and traceless
 *    quadrupole Q = sum m (3 d d^T - |d|^2 I), d = x - X;
 *  - groups: curve-consecutive runs of 64 particles, halved while a group's
 *    bounding box is wider than g_frac x side in some dimension (g_frac <= 0:
 *    never);
 *  - walk: a cell other than the root is accepted for a group when
 *    theta^2 d^2 > side_cell^2, d the distance between the group's bounding
 *    box and the cell's cube; other leaves are opened;
 *  - forces: an accepted cell gives a = -M y s^-3/2 + Q y s^-5/2 -
 *    (5/2)(y.Qy) y s^-7/2 and phi = -M s^-1/2 - (1/2)(y.Qy) s^-5/2 with
 *    y = x - X, s = |y|^2 + eps2; an opened leaf's particles j != i the
 *    softened pair terms (a pair at zero distance with eps2 = 0 is dropped).
 * Keys, tree, moments, groups and walk are double precision; the force terms
 * are double for an NB_PREC_FP64 context and otherwise float terms from
 * double separations, summed in double per staged chunk of up to 64 cells or
 * 64 leaf particles.  The walk and the force evaluation are one kernel (one
 * wavefront per group); no interaction list is stored.
 * theta = 0 opens every leaf: the direct sum.  pos [N][3], mass [N] in,
 * acc [N][3], pot [N] out, all in the caller's order (device pointers).
 * stats (host array of 5, may be NULL): cells, groups, accepted (group, cell)
 * pairs, opened (group, leaf) pairs, depth.  Nothing is read on the host
 * while the tree is built (the level bounds stay in device memory and the
 * buffers are sized from bounds known up front: at most 22 n / (n_crit + 1)
 * + n + 1 cells), so with stats == NULL the call is asynchronous and can be
 * captured in a graph, once a call outside the capture has sized the
 * buffers for this N and n_crit (else NB_ENOTSUP); with stats it
 * synchronises the stream.  Errors: NB_EINVAL for N outside [1, 2^31),
 * negative or non-finite eps2 or theta, n_crit < 1, non-finite g_frac, null
 * pointers; NB_ENOTSUP for stats under capture; NB_ENOMEM when device
 * memory runs out or a walk's stack would exceed its bound (8 x 64 x 21
 * entries, which an octree of 21 levels cannot reach) -- reported by this
 * call when it synchronises, else by the next nb_sync; the outputs are then
 * undefined. */
int nb_tree_forces(nb_ctx *ctx, const double *pos, const double *mass, int64_t N, double eps2, double theta,
                   int32_t n_crit, double g_frac, double *acc, double *pot, int64_t *stats);
/* The tree code's first stage: keys[k] is the 63-bit Peano-Hilbert index of
 * the k-th particle along the curve and idx[k] its row in pos, i.e. the rows
 * sorted by (key, row) with the library's stable radix sort (device arrays
 * of N; same box and key rules as nb_tree_forces).  Asynchronous; not
 * capturable (NB_ENOTSUP).  Errors: NB_EINVAL for N outside [1, 2^31) or a
 * null pointer. */
int nb_tree_keys(nb_ctx *ctx, const double *pos, int64_t N, uint64_t *keys, int32_t *idx);

/* ---- Hamiltonian split (bridge) ------------------------------------------
 * Section "The multi-scale approach" evolves a collisional subsystem c and a
 * field subsystem g together by splitting H = H_A + H_B with H_A = W_gc (the
 * potential energy between them) and H_B = H_g + H_c, to second order as
 * e^{dt/2 A} e^{dt B} e^{dt/2 A}: a half kick by the cross field
 * (nbody_forces_ij both ways, then nb_kick), each subsystem on its own for
 * dt, another half kick.  These two passes are the element-wise parts.
 *
 * nb_kick:       vel[i] = vel[i] + h acc[i]
 * nb_kick_drift: vel[i] = vel[i] + h_kick acc[i]; pos[i] = pos[i] + h_drift vel[i]
 *                (the new velocity), i.e. the first half of a leapfrog step.
 * Arrays are [N][3] doubles and must not overlap; each update is a rounded
 * multiply followed by a rounded add (no fused multiply-add).  Errors:
 * NB_EINVAL for N outside [0, 2^31), a non-finite step, or a null pointer
 * when N > 0; N == 0 does nothing. */
int nb_kick(nb_ctx *ctx, double *vel, const double *acc, int64_t N, double h);
int nb_kick_drift(nb_ctx *ctx, double *pos, double *vel, const double *acc, int64_t N, double h_kick,
                  double h_drift);

/* ---- Hermite block steps --------------------------------------------------
 * Time is kept in int64 ticks of dt_min = dt_max 2^-max_level; particle i
 * has time t_tick[i] and level dt_level[i] (its step is dt_max 2^-level,
 * i.e. 2^(max_level - level) ticks).  max_level must be in [0, 62]. */

/* Stop tick in device memory: while t_stop_dev is set (non-NULL), every
 * block-step call on this context (nb_block_step, nb_block_step_batch,
 * nb_block_step6) reads its stop tick from *t_stop_dev when its scheduler
 * runs, instead of its t_stop_tick argument, so one captured graph of block
 * steps replays for any stop time the caller writes there.  NULL restores
 * the argument.  The pointer is recorded by each launch (a graph keeps the
 * pointer it was captured with); nb_schedule has no stop tick and ignores
 * it. */
int nb_set_stop_source(nb_ctx *ctx, const int64_t *t_stop_dev);

/* Phase timing of block steps.  While on (on != 0), every block-step call
 * on this context (nb_block_step, nb_block_step_batch, nb_block_step6)
 * that is not being captured into a graph records four HIP events on the
 * context stream: at its start, after the scheduler with the predictor (and
 * the batch plan), after the force launches and after the corrector.  The
 * events cost a few microseconds per step; steps captured into a graph
 * record none.  Switching on creates the events (NB_EDEVICE if that fails);
 * switching on or off forgets the last step's times. */
int nb_set_phase_timing(nb_ctx *ctx, int on);

/* Milliseconds of the three phases of the last timed block step: ms[0] the
 * scheduler with the predictor (and the batch plan), ms[1] the forces,
 * ms[2] the partial-sum reduction with the corrector.  Waits for that
 * step's last event.  NB_EINVAL if timing is off or no eager block step
 * has completed its launches since it was switched on. */
int nb_phase_times(nb_ctx *ctx, float ms[3]);

/* Predict every particle to t_next: d = (t_next_tick - t_tick[i]) dt_min,
 * pos_p = pos + vel d + acc d^2/2 + jerk d^3/6, vel_p = vel + acc d + jerk d^2/2.
 * Inputs [N][3] and t_tick [N]; outputs [N][3] (may not alias the inputs). */
int hermite_predict(nb_ctx *ctx, const double *pos, const double *vel, const double *acc,
                    const double *jerk, const int64_t *t_tick, int64_t t_next_tick,
                    double dt_min, int64_t N, double *pos_p, double *vel_p);

/* Correct the active particles after their new forces acc1/jerk1 (compact
 * [n_active][3], row k for active_idx[k]) were evaluated at the predicted
 * state pos_p/vel_p ([N][3]).  For each active i with dt = its current step:
 *   a2 = [-6(a0-a1) - dt(4 j0 + 2 j1)]/dt^2,  a3 = [12(a0-a1) + 6 dt(j0+j1)]/dt^3
 *   x = x_p + a2 dt^4/24 + a3 dt^5/120,        v = v_p + a2 dt^3/6 + a3 dt^4/24
 * then acc/jerk <- acc1/jerk1, t_tick += 2^(max_level-level), and the new
 * level from Aarseth's criterion
 *   dt* = sqrt(eta (|a1||a2e| + |j1|^2)/(|j1||a3| + |a2e|^2)), a2e = a2 + a3 dt
 * (dt* = dt_max when the denominator is 0): halve while dt > dt*; else
 * double once if dt* >= 2 dt, level > 0 and the new time is a multiple of
 * 2 dt.  Levels beyond max_level are clamped to it and counted in
 * *clamp_count_dev (device int64, may be NULL; not reset by the call).
 * pos, vel, acc, jerk [N][3], t_tick, dt_level [N] are updated in place for
 * the active rows only.  active_idx must not repeat an index; N is the
 * number of particles, and entries outside [0, N) are skipped (nothing of
 * theirs is read or written) and reported by nb_sync.  Errors: NB_EINVAL for
 * n_active outside [0, 2^31), N outside [1, 2^31), bad level parameters or a
 * null pointer when n_active > 0. */
int hermite_correct(nb_ctx *ctx, const int32_t *active_idx, int64_t n_active, int64_t N,
                    const double *pos_p, const double *vel_p, const double *acc1, const double *jerk1,
                    double *pos, double *vel, double *acc, double *jerk,
                    int64_t *t_tick, int32_t *dt_level, double eta, double dt_max, int32_t max_level,
                    int64_t *clamp_count_dev);

/* Start-up levels at a common time: level = smallest k >= 0 with
 * dt_max 2^-k <= eta |acc|/|jerk| (0 when jerk = 0), clamped to max_level.
 * acc, jerk [N][3] -> dt_level [N]. */
int hermite_startup(nb_ctx *ctx, const double *acc, const double *jerk, int64_t N,
                    double eta, double dt_max, int32_t max_level, int32_t *dt_level);

/* Block scheduler: t_next = min_i (t_tick[i] + 2^(max_level - dt_level[i]));
 * active_idx <- every i with t_tick[i] + step == t_next, ascending (a stable
 * compaction); writes sched[0] = t_next, sched[1] = n_active (device int64
 * array of at least 2).  active_idx has room for N entries. */
int nb_schedule(nb_ctx *ctx, const int64_t *t_tick, const int32_t *dt_level, int64_t N,
                int32_t max_level, int32_t *active_idx, int64_t *sched);

/* One whole block step with no host synchronisation (capturable in a HIP
 * graph): schedule -> predict all -> forces on the active set (device
 * count) -> correct.  State arrays as above; work arrays supplied by the
 * caller: pos_p, vel_p [N][3]; active_idx [N]; acc1, jerk1 [N][3]; pot1 [N];
 * sched (device int64 [4]): after the call sched[0] = t_next,
 * sched[1] = n_active, sched[2] += 1 (steps taken), sched[3] += clamps.
 * A step whose t_next exceeds t_stop_tick is empty (n_active = 0, nothing
 * changes), so a graph of several steps can be replayed up to a stop time
 * without the host reading the state in between (INT64_MAX: no stop). */
int nb_block_step(nb_ctx *ctx, int64_t N, double eps2, double eta, double dt_max, int32_t max_level,
                  const double *mass, double *pos, double *vel, double *acc, double *jerk,
                  int64_t *t_tick, int32_t *dt_level,
                  double *pos_p, double *vel_p, int32_t *active_idx,
                  double *acc1, double *jerk1, double *pot1, int64_t *sched, int64_t t_stop_tick);

/* One block step over a batch of C independent systems stored back to back
 * (system s owns rows offsets[s] .. offsets[s+1]-1; host arrays offsets
 * [C+1] and eps2 [C]); pairs across systems never interact.  The block step
 * is global: t_next is the minimum over every system.  The work list
 * (system, i-block, j-chunk) is built on the device from the scheduled
 * active set, so the call makes no host-device transfer once the system
 * table has been uploaded (first call, or when offsets/eps2 change -- not
 * allowed during a stream capture) and a graph can replay it.  State, work
 * arrays and sched as for nb_block_step, over all offsets[C] rows. */
int nb_block_step_batch(nb_ctx *ctx, const int64_t *offsets, int64_t C, const double *eps2, double eta,
                        double dt_max, int32_t max_level, const double *mass, double *pos, double *vel,
                        double *acc, double *jerk, int64_t *t_tick, int32_t *dt_level,
                        double *pos_p, double *vel_p, int32_t *active_idx,
                        double *acc1, double *jerk1, double *pot1, int64_t *sched, int64_t t_stop_tick);

/* Energy and momenta of a synchronised system, summed in double in a fixed
 * order: out (device double [8]) = K, W, Px, Py, Pz, Lx, Ly, Lz with
 * K = sum m v^2/2, W = sum m phi / 2 (phi from a force call over all
 * particles), P = sum m v, L = sum m x cross v. */
int nb_energy(nb_ctx *ctx, const double *pos, const double *vel, const double *mass,
              const double *pot, int64_t N, double *out);

#ifdef __cplusplus
}
#endif
#endif /* NBODY_H */
