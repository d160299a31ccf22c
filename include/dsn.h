/*
 * dsn.h - C ABI of the MI355X discrete-ordinates source-iteration library.
 *
 * The library solves the multigroup discrete-ordinates form of the linear
 * Boltzmann equation for low-energy photons (paper section II.A, eq. 2) on a
 * uniform i,j,k voxel mesh with vacuum boundaries.  One solve per source:
 *   1. uncollided fluence by ray tracing from the point/cone source and its
 *      first-collision source (section II.A, eqs. 4-7);
 *   2. for every energy group, source iteration: assemble the P_L scattering
 *      source from flux moments plus downscatter from higher groups (eq. 2,
 *      right-hand side), sweep all N(N+2) directions of the level-symmetric
 *      S_N set with diamond-difference cells (section II.B, sub-sweeps; the
 *      scheme is named in section IV), reduce the angular fluence to scalar
 *      fluence and Legendre moments (eq. 3);
 *   3. total fluence = uncollided + collided.
 *
 * Conventions (all arrays are dense, C order):
 *   voxel index v = i + nx*(j + ny*k); voxel (i,j,k) has its centre at
 *     ((i+1/2)dx, (j+1/2)dy, (k+1/2)dz) in cm; the mesh spans [0, nx*dx] x ...
 *   group g = 0 is the HIGHEST energy; scattering goes from g' to g >= g'.
 *   sigma_s[m][l][g][g'] = sigma_{s,l}^{g'->g} of material m (cm^-1), the
 *     Legendre coefficient WITHOUT the (2l+1) factor; the angular kernel is
 *     sum_l (2l+1)/(4 pi) sigma_{s,l} P_l(mu0).  Entries with g' > g must be 0.
 *   density (optional) scales sigma_t and every sigma_{s,l} of its voxel.
 *   S_N quadrature: level-symmetric (LQn), weights summing to 4 pi, so eq. 3
 *     returns the scalar fluence.  N in {2, 4, 6, 8, 10, 12, 16}.
 *   Spectrum: photons per source particle in each group; fluence results are
 *     per source particle (photons / cm^2).
 *
 * Memory: every pointer passed to dsn_create and every host pointer listed
 * below is read during the call only (deep copy).  Output arrays marked
 * "device" are caller-owned device memory (e.g. torch tensors on cuda:0) of
 * the stated size; the library writes them on the caller's stream.  The
 * library owns the device state behind a dsn_problem and frees it in
 * dsn_destroy.
 *
 * Errors: no function throws.  Every status other than DSN_OK sets a
 * thread-local message readable with dsn_last_error().  Argument checks run on
 * the host before any device call, so they work without a GPU.
 *
 * Threading: distinct handles may be used from different threads; one handle
 * must not be used by two threads at once.
 */
#ifndef DSN_H
#define DSN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dsn_problem dsn_problem; /* opaque, owned by the library */

typedef enum {
    DSN_OK = 0,
    DSN_ERR_INVALID_ARG = 1,   /* bad size, id, order, upscatter, NaN ...      */
    DSN_ERR_UNSUPPORTED = 2,   /* valid input outside what the library handles */
    DSN_ERR_OUT_OF_MEMORY = 3, /* device allocation failed                    */
    DSN_ERR_DEVICE = 4,        /* HIP runtime error or no usable gfx950 GPU   */
    DSN_ERR_NOT_CONVERGED = 5, /* max_iters reached; outputs hold last iterate */
    DSN_ERR_NUMERICAL = 6      /* residual became NaN or infinite             */
} dsn_status;

typedef enum {
    DSN_FP64 = 0, /* every step in FP64                                          */
    DSN_FP32 = 1  /* scattering source, sweep and angular fluence in FP32; flux
                     moments, their quadrature accumulation and the residual in
                     FP64                                                         */
} dsn_precision;

/* Problem description (section II.C: voxel material map and density,
 * multigroup cross sections with Legendre scattering matrices, quadrature and
 * anisotropy order). */
typedef struct {
    int32_t nx, ny, nz;         /* voxels per axis, each >= 1                    */
    double dx, dy, dz;          /* voxel pitch, cm, > 0                          */
    const uint8_t *material;    /* host [nx*ny*nz], values < n_materials         */
    const double *density;      /* host [nx*ny*nz] >= 0, or NULL (all 1)         */
    int32_t n_materials;        /* 1..16                                         */
    int32_t n_groups;           /* G >= 1                                        */
    const double *sigma_t;      /* host [n_materials][G], >= 0                   */
    int32_t legendre_order;     /* L, 0 <= L <= 5 and L <= N-1                   */
    const double *sigma_s;      /* host [n_materials][L+1][G][G] (to, from)      */
    int32_t sn_order;           /* N                                             */
    int32_t fixup;              /* 0 pure diamond difference; 1 set-to-zero fixup
                                   of negative outflows (cell balance kept)      */
    int32_t precision;          /* dsn_precision                                 */
} dsn_problem_desc;

/* Point, cone-beam or fan-beam source (section II.C, source tab: position,
 * spectrum and the angles subtended by the beam).  The cone holds the voxel centres whose
 * direction from the source makes an angle <= half_angle with axis; inside it
 * the source emits spectrum[g]/(4 pi) photons per steradian.  half_angle >= pi
 * gives an isotropic point source (axis ignored).  A voxel centre closer than
 * 1e-6 of the smallest pitch to the source is an invalid argument. */
typedef struct {
    double position[3]; /* cm, anywhere (inside or outside the mesh)             */
    double axis[3];     /* any non-zero length                                    */
    double half_angle;  /* radians                                                */
    const double *spectrum; /* host [G]                                           */
    /* Fan beam (fan_half_thickness > 0): the beam is collimated to a fan
     * around the plane through the axis with normal fan_normal (its component
     * along the axis is ignored; the rest must be non-zero).  It holds the
     * voxel centres whose direction d from the source has |angle(d, plane)|
     * <= fan_half_thickness and, projected onto the plane, makes an angle <=
     * half_angle with the axis (both inclusive); half_angle < pi/2 and
     * fan_half_thickness < pi/2.  0 = a cone as above. */
    double fan_normal[3];
    double fan_half_thickness; /* radians                                         */
} dsn_source;

/* Iteration controls.  Source iteration in each group starts from zero flux.
 * The paper leaves the convergence criterion open (section II.C); with
 * r = ||phi00_new - phi00_old||_2 / ||phi00_new||_2 (FP64, 0/0 = 0) a group
 * stops
 *   stop_rule 0: when r < tol;
 *   stop_rule 1: when the estimated per-voxel error left in the total
 *     fluence, est = d rho / (1 - rho), is < tol, where d is the largest
 *     |phi00_new - phi00_old| / |phi_u + phi00_new| over the voxels whose
 *     |phi_u + phi00_new| is at least 1e-6 of the previous iterate's largest,
 *     and rho = r / r_prev (the first iterate never stops rule 1 unless
 *     r = 0).  Rule 0 can leave low-fluence voxels far above tol off the
 *     converged solution; rule 1 bounds every voxel the 1e-6 floor keeps;
 * or after fixed_iters[g] sweeps when fixed_iters is given, or - when
 * stagnation_stop is set - after three iterations in a row that do not
 * improve on the smallest value so far of what the rule tests (r, or est
 * for rule 1): the FP32 rounding floor.  Reaching max_iters returns DSN_ERR_NOT_CONVERGED with the
 * last iterate in the outputs; an r that is NaN or infinite returns
 * DSN_ERR_NUMERICAL.  The adjoint iterations of dsn_solve_adjoint always use
 * rule 0 (its forward solve uses stop_rule). */
typedef struct {
    double tol;                 /* > 0 unless fixed_iters is given               */
    int32_t max_iters;          /* >= 1                                          */
    const int32_t *fixed_iters; /* host [G] (values >= 0) or NULL                */
    int32_t stagnation_stop;    /* 0 or 1                                        */
    int32_t profile;            /* 1: time every stage with HIP events on the
                                   stream (fills dsn_solve_info.stage_*)          */
    int32_t wait_limit;         /* polls of an upstream face word before a sweep
                                   gives up; the call then returns
                                   DSN_ERR_DEVICE (results invalid) and the
                                   problem stays usable.  0 = default (2^22);
                                   tiny values exist to exercise that path      */
    int32_t autotune;           /* 1: if this handle has not been tuned, time
                                   the sweep's launch shapes (waves per block
                                   that divide N(N+2)/8, FP32 fixup sweeps also
                                   with per-XCD ticket queues, the column-relay
                                   shapes; full, 3/4 and 1/2 resident grid) at the
                                   first iteration of this call and keep the
                                   fastest for the handle's later calls; results
                                   do not depend on the shape.  0: keep the
                                   handle's shape.  dsn_solve_batch: see
                                   batch_mode. */
    int32_t combine_sources;    /* 1: dsn_solve's n_src sources act together in
                                   one solve (e.g. the cone beams of a CT ring,
                                   paper section II.D): their uncollided
                                   fluences and first-collision sources add up
                                   and one collided solution is iterated;
                                   phi_total (and phi_uncollided) are then
                                   [1][G][V] and info->iters [1][G]; n_src
                                   must be >= 1 (else INVALID_ARG).  Needs
                                   (n_src (G + 3) + G (N_m + 1)) V' x 8 bytes
                                   more (ray traces, summed uncollided
                                   fluence and moments; V' = voxels padded
                                   to 8 x 8 columns, N_m = (L+1)^2).  Equal to
                                   the sum of separate solves when the sweep
                                   is linear (fixup off) and the iteration
                                   counts are the same.
                                   dsn_solve_batch rejects 1; the adjoint
                                   ignores it. */
    void *stream;               /* hipStream_t to run on, NULL = null stream     */
    int32_t stop_rule;          /* 0 or 1, see above                             */
    int32_t batch_mode;         /* 0 or 1 (every call checks it; only
                                   dsn_solve_batch uses it):
                                   0 = a stream and a host thread per problem
                                   (the default: as fast or faster on MI355X
                                   for every mix measured);
                                   1 = fused: all problems iterate the same
                                   group in lockstep on opts->stream, and each
                                   source iteration is ONE sweep launch over
                                   every (problem, source) pair, then one
                                   moments launch and one convergence-test
                                   launch over all of them, replayed as one
                                   HIP graph; autotune = 1 times that
                                   launch's shapes at the first group.  Needs
                                   the same fixup setting in every problem and
                                   all with or all without a per-voxel density
                                   (else DSN_ERR_UNSUPPORTED).
                                   Results are the same in both modes. */
} dsn_solve_opts;

/* Stages timed when dsn_solve_opts.profile is set. */
enum {
    DSN_STAGE_SETUP = 0,  /* ray trace, group source, finalize                    */
    DSN_STAGE_M2D = 1,    /* scattering source + moment -> direction contraction  */
    DSN_STAGE_SWEEP = 2,  /* transport sweep (all directions)                      */
    DSN_STAGE_D2M = 3,    /* direction -> moment quadrature + residual              */
    DSN_NUM_STAGES = 4
};

/* Optional per-call report (all host memory, caller-owned). */
typedef struct {
    int32_t *iters;     /* [n_src][G] source iterations per group, or NULL        */
    double *residual;   /* [n_src][G] final relative change per group, or NULL   */
    double updates;     /* voxel*direction*group updates performed                */
    double seconds;     /* wall time of the call                                  */
    double stage_ms[DSN_NUM_STAGES];       /* GPU time per stage (profile = 1)   */
    int64_t stage_launches[DSN_NUM_STAGES]; /* kernel launches per stage          */
    double sweep_bytes; /* algorithmic bytes of the sweeps performed: angular
                           source read + angular fluence written per update      */
    int32_t sweep_waves_per_block; /* sweep launch shape in use (0 from
                                      dsn_solve_batch)                           */
    int32_t sweep_blocks;
    int32_t sweep_xcd_queues;      /* > 0: the sweep takes tickets from that many
                                      per-XCD queues (faces stay in each XCD's
                                      L2); 0: one global queue                   */
    int32_t sweep_relay;           /* > 0: column-relay sweep (see
                                      dsn_set_sweep_shape) with this many roles  */
} dsn_solve_info;

/* Validates the description, derives the quadrature and the moment tables on
 * the host, and copies everything needed.  Device memory is taken lazily at
 * the first solve.  On success *out is a new handle. */
dsn_status dsn_create(const dsn_problem_desc *desc, dsn_problem **out);

/* Frees the handle and its device memory (synchronises the device). */
void dsn_destroy(dsn_problem *p);

/* Device bytes the handle holds (state kept between calls) once it has run
 * a solve; before its first solve, the bytes a one-source solve will take. */
size_t dsn_workspace_bytes(const dsn_problem *p);

/* Forward solve of n_src independent sources (eqs. 2-7), advanced together
 * in batches as large as the device memory allows (at most 64 at a time).
 *   phi_total       device [n_src][G][V] FP64: uncollided + collided fluence
 *                   ([1][G][V] with opts->combine_sources).
 *   phi_uncollided  device [n_src][G][V] FP64 or NULL (likewise).
 * Returns DSN_OK, DSN_ERR_NOT_CONVERGED (outputs valid, last iterate) or an
 * error (outputs unspecified). */
dsn_status dsn_solve(dsn_problem *p, const dsn_source *src, int32_t n_src, const dsn_solve_opts *opts,
                     double *phi_total, double *phi_uncollided, dsn_solve_info *info);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the forward
 * solve of dsn_solve for one source, computed by the same kernels in the
 * same order (identical results for the same sweep launch shape), that calls
 * no device allocation routine.  Every device array of the solve (problem
 * tables, angular fluence, moments, face words, counters, residual partials)
 * lives in one fixed array of 64 MiB of device memory per GPU that the library
 * holds until the process ends; a problem whose solve needs more - about
 * 8 G (N_m + 1) + 8 N_m + 1.5 N(N+2) b + 50 bytes per voxel (b = 4 in FP32,
 * 8 in FP64; N_m = (L+1)^2; the mesh padded to multiples of 8 in y and z),
 * so 32^3 S8 P3 fits up to G = 8 in FP32 - returns DSN_ERR_UNSUPPORTED
 * before any device work.  Every call on a GPU reuses that GPU's array:
 * calls that overlap on one GPU (other streams, other threads, other
 * handles) race and must be serialised by the caller.  The handle's own
 * device state is neither used nor created; its tuned sweep shape is used
 * when it has one on the global ticket queue.  The problem tables are copied
 * from the handle's host copies at every call.
 *   phi_total       device [G][V] FP64, uncollided + collided fluence.
 *   phi_uncollided  device [G][V] FP64 or NULL.
 * opts as for dsn_solve, except: combine_sources must be 0, autotune and
 * profile are ignored (no stage times).  info->iters and residual, when
 * given, are [G].  Returns as dsn_solve. */
dsn_status dsn_solve_noalloc(dsn_problem *p, const dsn_source *src, const dsn_solve_opts *opts, double *phi_total,
                             double *phi_uncollided, dsn_solve_info *info);

/* Adjoint of the converged discrete forward solve of one source.  With the
 * set-to-zero fixup (fixup = 1) the solve is piecewise linear; it is
 * linearised with every cell's set of fixed axes frozen at the converged
 * solution (recorded by one forward sweep per group from its converged
 * moments; device memory N(N+2) x V' bytes), which gives the exact gradient
 * wherever no outflow sits at a fixup switching point.  For the fluence
 * functional
 *   J = sum_g sum_v W[g][v] * phi_total[g][v]
 * returns J (host scalar) and dJ/d(density[v]) for every voxel (device [V],
 * FP64), the density scaling sigma_t and every sigma_{s,l} of its voxel.  The
 * adjoint angular fluence is swept along the reversed directions, groups from
 * lowest energy to highest; each group's forward angular fluence is recomputed
 * from its converged moments instead of being stored.
 *   W            device [G][V] FP64 detector weights.
 *   phi_total    device [G][V] FP64 forward result, or NULL.
 * info->iters, when given, receives [2][G]: forward then adjoint iterations. */
dsn_status dsn_solve_adjoint(dsn_problem *p, const dsn_source *src, const double *W,
                             const dsn_solve_opts *opts, double *J, double *dJ_ddensity,
                             double *phi_total, dsn_solve_info *info);

/* Replaces the per-voxel density (natural order, [V] FP64, host or device
 * pointer; NULL = all 1) of an existing handle, e.g. the trainable parameter
 * of a gradient loop.  Values must be finite and >= 0 (not checked when the
 * pointer is device memory). */
dsn_status dsn_set_density(dsn_problem *p, const double *density);

/* Batched forward solves (the batching form: many CT source positions on
 * phantoms of uneven size): n_src[b] sources on problem probs[b], for
 * b < n_probs, advanced together (all problems must share G, N, L and
 * precision; meshes and materials may differ).  Each problem's result goes to
 * phi_total[b], device [n_src[b]][G][V_b] FP64.  srcs[b] points to n_src[b]
 * sources.  Results equal those of separate dsn_solve calls.  The handles
 * must be distinct (DSN_ERR_INVALID_ARG otherwise).  opts->batch_mode picks
 * how the problems run: fused (one sweep launch per source iteration over
 * every (problem, source) pair, on opts->stream) or a host thread and a
 * stream per problem (which start after the work already on opts->stream).
 * The call returns once every result is written.  The first failing
 * problem's status is returned (a problem that only missed tol gives
 * DSN_ERR_NOT_CONVERGED after the others finish).  info->iters, when given,
 * receives [sum n_src][G] in the order of the problems and their sources;
 * info->sweep_* the fused launch's shape (zero for a stream per problem). */
dsn_status dsn_solve_batch(dsn_problem *const *probs, int32_t n_probs, const dsn_source *const *srcs,
                           const int32_t *n_src, const dsn_solve_opts *opts, double *const *phi_total,
                           dsn_solve_info *info);

/* Host-only query: the library's level-symmetric S_N set.  omega host
 * [N(N+2)][3], w host [N(N+2)].  Order: n = o*N(N+2)/8 + p, octant o has
 * signs (-1)^(o&1), (-1)^((o>>1)&1), (-1)^((o>>2)&1) on (mu, eta, xi); inside
 * an octant p runs over the mu level ascending, then the eta level ascending. */
dsn_status dsn_quadrature(int32_t sn_order, double *omega, double *w);

/* Absorbed dose from group fluences, the quantity the fluence is computed
 * for (paper sections I and IV):
 *   dose[s][v] = sum_g phi[s][g][v] * k[m(v)][g]
 * with m(v) the voxel's material.  k is the caller's fluence-to-dose factor
 * per material and group, e.g. E_g (mu_en/rho)_{m,g} in Gy cm^2 per photon
 * (mass coefficients, so the per-voxel density does not enter).
 *   phi    device [n][G][V] FP64 (as dsn_solve writes phi_total)
 *   k      host [n_materials][G] FP64, finite (copied)
 *   dose   device [n][V] FP64
 * Runs on `stream` (hipStream_t or NULL) and returns after completion.
 * DSN_ERR_INVALID_ARG for NULL arrays, n < 0 or > 65535, non-finite k. */
dsn_status dsn_dose(dsn_problem *p, const double *phi, int32_t n, const double *k, double *dose, void *stream);

/* Pins the sweep launch shape of the handle, e.g. the fastest one an earlier
 * handle's autotune found for the same mesh and quadrature.
 *   relay = 0: pencil items (one 8 x 8 column of voxels over the x extent,
 *     waves_per_block directions of one octant), waves_per_block a built
 *     choice - 1, 2, 3, 4, 5, 6, 9, 10, 12 in FP32, up to 6 in FP64 - that
 *     divides the N(N+2)/8 directions of an octant; xcd_queues 0 for one
 *     global ticket queue, else the device's XCD count (dsn_xcd_queues) for
 *     the per-XCD queues, which are built for FP32 with the fixup and up to 4
 *     waves per block.
 *   relay = R > 0: column-relay items (a whole row of pencils along y,
 *     waves_per_block directions, R waves per direction taking the pencils in
 *     turn and handing their y faces to each other in LDS, so y faces never
 *     reach memory); built for (waves_per_block, R) = (1, 2), (1, 4), (2, 2),
 *     (2, 4) in FP32 and (1, 2), (1, 4) in FP64, with xcd_queues 0; needs LDS
 *     for one pencil's y faces per wave (nx x 32 bytes in FP32), so large
 *     x extents may not fit.  The adjoint's sweeps of such a handle use
 *     pencil items of waves_per_block directions.
 * blocks per launch: 1..2^20 (the sweep's persistent blocks take work from a
 * ticket queue, so any count is correct and about the resident count is
 * fastest).  Every shape gives the same results bit for bit.  The handle
 * counts as tuned afterwards (autotune = 1 times nothing).  Not to be called
 * while a solve on the handle runs.  DSN_ERR_INVALID_ARG (checked before any
 * device call) for a NULL handle, a shape that is not built, blocks out of
 * range or negative counts; DSN_ERR_UNSUPPORTED for per-XCD queues this
 * handle or device cannot use or a column-relay shape whose LDS does not
 * fit; DSN_ERR_DEVICE without a device. */
dsn_status dsn_set_sweep_shape(dsn_problem *p, int32_t waves_per_block, int32_t blocks, int32_t xcd_queues,
                               int32_t relay);

/* Host-only query: the sweep launch shapes the handle's autotune timed, in
 * the order timed.  Writes up to cap entries of waves per block, blocks per
 * launch, per-XCD queues (0: one global queue), column-relay roles (0:
 * pencil items) and milliseconds per sweep (negative: the shape's angular
 * fluence differed from the default shape's and it was not used); each
 * pointer may be NULL.  Returns the number timed (0 before any autotune;
 * NULL handle: 0). */
int32_t dsn_sweep_tuning(const dsn_problem *p, int32_t *waves_per_block, int32_t *blocks, int32_t *xcd_queues,
                         int32_t *relay, float *ms, int32_t cap);

/* The per-XCD ticket queues the handle's device allows (the xcd_queues
 * value dsn_set_sweep_shape accepts and the autotune tries): the device's
 * XCD count when the probe at the handle's first device use saw consecutive
 * workgroups placed on consecutive XCDs (round robin), else 0 (only the
 * global queue).  Sets up the handle's device state if it has none yet.
 * Returns -1 (message in dsn_last_error) for a NULL handle or without a
 * usable device. */
int32_t dsn_xcd_queues(dsn_problem *p);

/* Thread-local message of the last failed call on this thread ("" if none). */
const char *dsn_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DSN_H */
