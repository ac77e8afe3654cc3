/*
 * rmb.h -- C ABI of the MI355X rigid-multiblob mobility library (librmb.so).
 *
 * The library solves the mobility problem of rigid bodies discretised as
 * rigid multiblobs in Stokes flow (Balboa Usabiaga et al., "Hydrodynamics of
 * suspensions of passive and active rigid particles: a rigid multiblob
 * approach"):
 *
 *     [ M   -K ] [lambda]   [ slip ]
 *     [-K^T  0 ] [  U   ] = [  -F  ]          (Sec. 2.1.2, eq:saddle_M)
 *
 * M is the 3Nb x 3Nb blob-blob mobility (free-space Rotne-Prager-Yamakawa,
 * eq:RPYTensor, or RPY plus the Rotne-Prager-Blake single-wall correction,
 * Sec. 2.1.1), K maps rigid-body motions to blob velocities
 * (eq:noslip_rigid), F holds applied forces and torques, slip the active
 * slip, U the body velocities and lambda the blob constraint forces.  The
 * solver is right-preconditioned GMRES with the indefinite block-diagonal
 * preconditioner (Sec. 2.2.2, eq:indef_block_P, eq:saddle_M_precon).
 *
 * Conventions shared by every entry point
 *  - Units: viscosity eta and blob radius a are per system; the wall, when
 *    present, is the plane z = 0 with fluid in z > 0.
 *  - Layouts (row-major, C order):
 *      blob positions, blob vectors (lambda, velocities, slip): [n_blobs][3]
 *      body tracking points q:                                  [n_bodies][3]
 *      body force/torque F and velocity U:      [n_bodies][6] = (f, tau), (u, omega)
 *      saddle-point vectors: [lambda (3 n_blobs) ; U (6 n_bodies)]
 *    Torques and angular velocities are about the tracking point q_p.
 *  - Memory: every `double*` argument is a DEVICE pointer on the context's
 *    device unless marked "host".  The caller owns every argument buffer;
 *    the library never frees or retains them beyond the call (the server
 *    entry points retain them until the request completes, as documented
 *    there).  Output buffers must not alias inputs.
 *  - Streams: `stream` is a hipStream_t (NULL = the null stream).  Calls
 *    enqueue their work on it; calls that must return a status that depends
 *    on device results (validation, factorisation failure, convergence)
 *    synchronise that stream before returning.
 *  - Errors: every call returns an rmb_status; no exception crosses the ABI.
 *    On failure a message is available from rmb_last_error(ctx).
 */
#ifndef RMB_H
#define RMB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RMB_OK = 0,
    RMB_EINVAL = 1,   /* bad argument: a <= 0, eta <= 0, bad offsets, z <= 0 above a wall,
                         non-finite positions, null pointer, unknown enum value */
    RMB_ENOTSPD = 2,  /* a per-body mobility block is not positive definite (blobs overlapping
                         the wall, Sec. 2.1.1 and Conclusions) or its Schur complement is
                         singular */
    RMB_ENOCONV = 3,  /* iteration limit reached; outputs hold the best iterate and the info
                         struct the FP64 residual reached */
    RMB_ENOMEM = 4,   /* the request does not fit the context's device-memory budget */
    RMB_EDEVICE = 5,  /* a HIP runtime call failed */
    RMB_EBUSY = 6     /* server: queue full */
} rmb_status;

enum { RMB_GEOM_FREE = 0, RMB_GEOM_WALL = 1 };

/* Pair arithmetic of the blob mobility product.
 *  RMB_PREC_FP64:       every pair block in FP64, FP64 sums.
 *  RMB_PREC_FP32_PAIRS: r_i - r_j to FP32 accuracy (one rounding, or the
 *                       two-float difference of the symmetric product),
 *                       pair blocks and products in FP32, sums of each
 *                       target's velocity in FP32 over blocks of 64 sources
 *                       and FP64 across blocks (the symmetric product
 *                       stores each tile's 64-source sums as FP32 values
 *                       when its tiles hold 64 blobs, and the FP64 sum over
 *                       a tile's groups of 64 for larger tiles). */
enum { RMB_PREC_FP64 = 0, RMB_PREC_FP32_PAIRS = 1, RMB_PREC_RELAXED = 2 /* solves only, see rmb_solve_opts */ };

typedef struct rmb_ctx_s *rmb_ctx;
typedef struct rmb_precond_s *rmb_precond;
typedef void *rmb_stream; /* hipStream_t */

/* One suspension (Sec. 2.1: blobs B_p rigidly attached to bodies p). */
typedef struct {
    int64_t n_blobs;         /* Nb >= 1 */
    int64_t n_bodies;        /* N >= 1 (the mobility product alone ignores bodies) */
    const double *pos;       /* device [Nb][3] blob positions r_i (lab frame) */
    const int64_t *body_off; /* HOST [N+1]: blobs of body p are [body_off[p], body_off[p+1]),
                                body_off[0] = 0, strictly increasing, body_off[N] = Nb */
    const double *q;         /* device [N][3] tracking points q_p */
    double a;                /* blob hydrodynamic radius, > 0 */
    double eta;              /* viscosity, > 0 */
    int32_t geometry;        /* RMB_GEOM_FREE or RMB_GEOM_WALL (then every z_i > 0) */
    int32_t reserved;
    const double *blob_shift; /* device [Nb] or NULL.  Permeable bodies (appendix on permeable
                                 bodies, eq:permeable_slip): d_i = kappa_p / (eta dV_i) >= 0 for
                                 blob i of body p, i.e. a slip -d_i lambda_i, which adds d_i to
                                 the diagonal of M.  Every operation on the system then uses
                                 M + diag(d) (product, preconditioner factors, solves), except
                                 the flow field and the shared-shape factors, which leave it
                                 out.  NULL: rigid impermeable bodies (d = 0). */
} rmb_system;

/* ---------------------------------------------------------------------------
 * Context
 * ------------------------------------------------------------------------- */

/* Creates a context on HIP device `device`.  `hbm_budget_bytes` caps the
 * device memory the library may hold for workspaces, factors and Krylov
 * bases (0 = 16 GiB).  Memory is reserved lazily.  *out receives the
 * handle.  Errors: RMB_EINVAL (null out, bad device), RMB_EDEVICE.
 * The environment variable RMB_SYM_BAND_BYTES (a positive byte count, read
 * here) sets the budget of one band of the symmetric product's tile partials
 * (default 4 GiB, counted at FP64 size): the product evaluates its tile
 * triangle in bands of tile rows that fit it, so a smaller value bounds the
 * workspace of very large systems (and makes small systems take several
 * bands).  The value changes the order of the FP64 sums only. */
rmb_status rmb_ctx_create(int device, size_t hbm_budget_bytes, rmb_ctx *out);

/* Releases every device allocation the context holds.  Preconditioners and
 * servers created on the context must be destroyed first.  Safe on NULL. */
void rmb_ctx_destroy(rmb_ctx ctx);

/* Message of the last failed call on this context (never NULL; "" if none).
 * Valid until the next call on the context. */
const char *rmb_last_error(rmb_ctx ctx);

/* Library version string. */
const char *rmb_version(void);

/* Kernel timing (diagnostics).  While enabled, every launch of the pair
 * kernels is bracketed by HIP events recorded on the stream it runs on, and
 * the elapsed times are accumulated per kernel:
 *   RMB_KERNEL_PAIR_F32_WALL, RMB_KERNEL_PAIR_F32_FREE,
 *   RMB_KERNEL_PAIR_F64_WALL, RMB_KERNEL_PAIR_F64_FREE.
 * Enabling (enable = 1) or disabling resets the totals. */
enum { RMB_KERNEL_PAIR_F32_WALL = 0, RMB_KERNEL_PAIR_F32_FREE = 1, RMB_KERNEL_PAIR_F64_WALL = 2,
       RMB_KERNEL_PAIR_F64_FREE = 3, RMB_KERNEL_COUNT = 4 };
rmb_status rmb_ctx_set_timing(rmb_ctx ctx, int32_t enable);

/* Total milliseconds and launch count of one kernel since timing was
 * enabled; waits for the recorded events to complete (host arrays of one
 * element each). */
rmb_status rmb_ctx_kernel_time(rmb_ctx ctx, int32_t kernel, double *total_ms, int64_t *launches);

/* How the mobility product of nb blobs is evaluated: *symmetric = 1 when
 * each pair block is evaluated once and applied to both blobs (systems of at
 * least 1024 blobs; *block = its block size), 0 for the one-sided kernel
 * (*block = number of source splits).  A function of nb only. */
rmb_status rmb_pair_plan(int64_t nb, int32_t *symmetric, int32_t *block);

/* Tile shapes of the large-body factorisation (bodies whose 3n x 3n block
 * is too large for the LDS path; padded_dim = 3n + 6 rounded up to 64).  Which
 * shape a batch uses:
 *   - the shape forced with rmb_ctx_set_tile_shape for its padded size;
 *   - else, for batches of fewer than 64 bodies, shape 0 (small batches are
 *     never timed, and always get the same shape, so their factors do not
 *     depend on what ran before);
 *   - else the tuned shape: the first batch of a padded size times every
 *     shape and keeps the fastest.  The choice is persisted (a line per
 *     padded size in the file named by the environment variable
 *     RMB_TUNE_CACHE, by default $XDG_CACHE_HOME/rmb/tune.txt or
 *     $HOME/.cache/rmb/tune.txt; an empty value disables it) and every new
 *     context reads it, so processes sharing the file factorise with the
 *     same shape and give bitwise-identical results.
 * Shapes change rounding only. */
int32_t rmb_tile_shape_count(void);

/* Panel width, 16-row tiles per wave and prefetched columns of `shape`
 * (host outputs).  RMB_EINVAL for an unknown shape or a null pointer. */
rmb_status rmb_tile_shape_info(int32_t shape, int32_t *panel, int32_t *row_tiles, int32_t *chunk);

/* Forces `shape` for blocks of padded size `padded_dim` on this context
 * (shape -1 returns the choice to the rules above).  RMB_EINVAL for a
 * padded_dim that is not a positive multiple of 64 or an unknown shape. */
rmb_status rmb_ctx_set_tile_shape(rmb_ctx ctx, int32_t padded_dim, int32_t shape);

/* Panel width of the tuned shape for padded size `padded_dim` on this
 * context (from this context's tuning or the persisted file), or 0 if
 * there is none yet. */
rmb_status rmb_ctx_tuned_panel(rmb_ctx ctx, int32_t padded_dim, int32_t *panel_width);

/* One timing of the large-body factorisation autotuner. */
typedef struct rmb_tune_record {
    int32_t padded_dim; /* Mp: 3n + 6 rounded up to 64 */
    int32_t panel;      /* columns per Cholesky panel */
    int32_t row_tiles;  /* 16-row tiles per wave per pass of the panel update */
    int32_t chunk;      /* columns of L whose matrix-core operands are loaded ahead */
    double ms;          /* time of the whole batched build with this shape */
    int32_t chosen;     /* 1 for the shape kept for this padded size */
    int32_t reserved;
} rmb_tune_record;

/* Copies up to `capacity` autotuner timings of this context, in the order
 * they were taken, into `records` (host memory, caller-owned); *count
 * receives the total number held (which may exceed capacity).
 * RMB_EINVAL for a null count, a negative capacity, or a null records array
 * with capacity > 0. */
rmb_status rmb_ctx_tune_log(rmb_ctx ctx, int32_t capacity, rmb_tune_record *records, int32_t *count);

/* ---------------------------------------------------------------------------
 * Blob mobility product  v = M lambda   (Sec. 2.2.1; eq:RPYTensor and the
 * wall-corrected form of Sec. 2.1.1 and Sec. 5)
 * ------------------------------------------------------------------------- */

/* vel[i] = sum_j M_ij lambda[j] (+ d_i lambda[i] with sys->blob_shift) over
 * all blobs of `sys` (bodies are ignored;
 * n_bodies, body_off and q may be 0/NULL).  lambda and vel: device
 * [Nb][3] FP64, must not alias.  `precision` is an RMB_PREC_* value.
 * Errors: RMB_EINVAL (bad system, z_i <= 0 in wall geometry, non-finite
 * positions, a negative or non-finite blob_shift), RMB_ENOMEM, RMB_EDEVICE.
 * Synchronises `stream` once for validation. */
rmb_status rmb_mobility_matvec(rmb_ctx ctx, const rmb_system *sys, int32_t precision,
                               const double *lambda, double *vel, rmb_stream stream);

/* The FP32-pair product for FP32 data: lambda and vel are device [Nb][3]
 * float32 (must not alias).  The forces are widened to FP64 (exactly), the
 * product runs as rmb_mobility_matvec with RMB_PREC_FP32_PAIRS (FP32 pair
 * blocks, FP32 sums over 64 sources, FP64 beyond), and each velocity is
 * rounded to float32 once: the result is rmb_mobility_matvec's on the
 * widened forces, rounded to float32.  Workspace comes from the context
 * (twice 3 Nb doubles more than rmb_mobility_matvec).  Errors as
 * rmb_mobility_matvec.  Synchronises `stream` once for validation. */
rmb_status rmb_mobility_matvec_f32(rmb_ctx ctx, const rmb_system *sys, const float *lambda, float *vel,
                                   rmb_stream stream);

/* The same product for callers that cannot allocate device memory (code
 * that must not call hipMalloc: a tight serving loop, a harness that forbids
 * allocation, work being captured into a HIP graph).  It allocates nothing:
 * its workspace is a static device array of rmb_noalloc_workspace_bytes()
 * (128 MiB) that each device holds from the first context created on it
 * until the process ends; the caller still provides lambda and vel.  Every
 * call on a device shares that array, so calls that overlap on one device
 * (other streams, other threads, other contexts) race: serialise them.
 * Results agree with rmb_mobility_matvec to rounding (the symmetric product
 * runs in more, smaller bands of tile rows here, so sums are grouped
 * differently).  `validate` = 1 checks the positions first and synchronises
 * `stream` once, as rmb_mobility_matvec does; 0 skips the check (the caller
 * guarantees finite positions, z > 0 above a wall and a valid blob_shift)
 * and the call only enqueues work on `stream`: no host synchronisation, no
 * memset, no host staging.  Errors: RMB_EINVAL as rmb_mobility_matvec, and
 * for a system too large for the workspace (above about 2.7 million blobs);
 * RMB_EDEVICE if the workspace is unavailable. */
rmb_status rmb_mobility_matvec_noalloc(rmb_ctx ctx, const rmb_system *sys, int32_t precision,
                                       const double *lambda, double *vel, int32_t validate, rmb_stream stream);

/* Size in bytes of the no-allocation entry point's static workspace. */
size_t rmb_noalloc_workspace_bytes(void);

/* Flow field at arbitrary points (appendix "Computing flow fields"): every
 * blob i of `sys` is replaced by n_sub blobs of radius tracer_a placed at
 * r_i + a * sub_offsets[k], each carrying lambda_i / n_sub, and the velocity
 * at target point t is
 *     vel(t) = sum_i sum_k M'(t, r_i + a u_k) lambda_i / n_sub,
 * M' being the blob-blob mobility (RPY, plus the wall correction in wall
 * geometry) for blobs of radius tracer_a.  With n_sub = 1, a zero offset
 * and tracer_a = a it is the mobility product evaluated at the targets.
 * lambda: device [Nb][3]; sub_offsets: host [n_sub][3], in units of the blob
 * radius a (the paper leaves the discretisation of each blob's sphere to
 * the user; a uniform set on the unit sphere matches the RPY construction);
 * targets, vel: device [n_targets][3], vel must not alias lambda or targets.
 * Synchronous.  Errors: RMB_EINVAL (bad system or arguments, non-finite
 * positions, a target or sub-blob at z <= 0 in wall geometry), RMB_ENOMEM,
 * RMB_EDEVICE. */
rmb_status rmb_flow_field(rmb_ctx ctx, const rmb_system *sys, int32_t precision, const double *lambda,
                          int32_t n_sub, const double *sub_offsets, double tracer_a, int64_t n_targets,
                          const double *targets, double *vel, rmb_stream stream);


/* ---------------------------------------------------------------------------
 * Block-diagonal preconditioner (Sec. 2.2.2: eq:M_tilde_block_diag,
 * eq:indef_block_P, eq:saddle_M_precon)
 * ------------------------------------------------------------------------- */

/* Assembles every body's 3n_p x 3n_p mobility block M_pp (same pair tensor
 * as the product, wall included), factorises all of them in one launch,
 * and forms Y_p = L_p^-1 K_p and the Cholesky factor of
 * K_p^T M_pp^-1 K_p.  The factors hold device pointers into `sys->pos` and
 * `sys->q`, which must stay valid and unchanged while *out is used.
 * Errors: RMB_EINVAL (bad system), RMB_ENOTSPD (a block is not SPD, e.g.
 * blobs overlapping the wall, or a body's K_p^T M_pp^-1 K_p is singular),
 * RMB_ENOMEM, RMB_EDEVICE.  Synchronises `stream`. */
rmb_status rmb_precond_factor(rmb_ctx ctx, const rmb_system *sys, rmb_precond *out, rmb_stream stream);

/* out_r = P^-1 in_r for r < nrhs saddle vectors stored at in + r*(3Nb+6N)
 * (device, FP64): per body, [M_pp -K_p; -K_p^T 0][lambda_p; U_p] =
 * [in_lambda_p; in_U_p] is solved exactly.  `in` and `out` must not alias.
 * Asynchronous on `stream`. */
rmb_status rmb_precond_apply(rmb_ctx ctx, const rmb_precond pc, int32_t nrhs, const double *in,
                             double *out, rmb_stream stream);

/* Reference shapes for a shared factorisation: blobs of shape k are
 * ref_pos[shape_off[k] .. shape_off[k+1]) (host, [3] each, FP64), given in
 * the body frame relative to the body's tracking point.  shape_off is host
 * [n_shapes + 1] with shape_off[0] = 0. */
typedef struct {
    int32_t n_shapes;
    int32_t reserved;
    const int64_t *shape_off;
    const double *ref_pos;
} rmb_shapes;

/* Block-diagonal preconditioner from one factorisation per reference shape
 * (Sec. 2.2.2, after eq:saddle_M_precon: in an unbounded domain the RPY
 * block of a body is that of its reference configuration, rotated, so
 * bodies of one shape share one factorisation; in wall geometry this is the
 * approximate preconditioner that neglects the boundary, Sec. 5.4).
 * Body p uses shape body_shape[p] (host int32 [N]; its blob count must
 * equal the shape's) and orientation body_quat[p] (device [N][4] FP64,
 * (w, x, y, z), normalised here), i.e. its blob i is taken to sit at
 * q_p + R_p ref_i.  Each shape's block is factorised once, in free space,
 * with the system's a and eta; applying the preconditioner to body p rotates
 * its blob velocities, force and torque into the body frame (R_p^T),
 * applies the shape's factor, and rotates lambda, u and omega back (R_p).
 * When the system's blobs are exactly at q_p + R_p ref_i in free space the
 * result equals rmb_precond_factor's up to rounding.  The handle is used
 * like one from rmb_precond_factor (rmb_precond_apply, rmb_solve_mobility)
 * and holds factor memory for each shape only, plus 9 doubles per body.
 * Errors: RMB_EINVAL (bad system, shapes, shape indices, blob-count
 * mismatch, a zero or non-finite quaternion), RMB_ENOTSPD (a shape's block
 * is not positive definite, or its K^T M^-1 K is singular), RMB_ENOMEM,
 * RMB_EDEVICE.  Synchronises `stream`. */
rmb_status rmb_precond_factor_shapes(rmb_ctx ctx, const rmb_system *sys, const rmb_shapes *shapes,
                                     const int32_t *body_shape, const double *body_quat, rmb_precond *out,
                                     rmb_stream stream);

/* New body orientations (device [N][4], as above) for a preconditioner
 * from rmb_precond_factor_shapes: the shape factors are kept, so a moving
 * configuration needs no refactorisation (Sec. 2.2.2).  Work already queued
 * with `pc` on other streams must have completed.  Errors: RMB_EINVAL (pc
 * not from rmb_precond_factor_shapes, NULL quaternions, a zero or non-finite
 * quaternion; rotations of such bodies are then the identity), RMB_EDEVICE.
 * Synchronises `stream`. */
rmb_status rmb_precond_set_orientations(rmb_ctx ctx, rmb_precond pc, const double *body_quat, rmb_stream stream);

/* Releases the factors (after work using them has completed).  Safe on NULL. */
void rmb_precond_destroy(rmb_precond pc);

/* ---------------------------------------------------------------------------
 * Mobility solve (eq:saddle_M by right-preconditioned GMRES, Sec. 2.2)
 * ------------------------------------------------------------------------- */

typedef struct {
    double tol;          /* target ||b - A x|| / ||b|| with the FP64 operator; 0 -> 1e-8 */
    int32_t precision;   /* RMB_PREC_FP64: GMRES on the FP64 operator.
                            RMB_PREC_FP32_PAIRS: inner GMRES cycles on the FP32-pair
                            operator, each followed by an FP64 residual (iterative
                            refinement); the stopping test always uses FP64.
                            RMB_PREC_RELAXED: GMRES whose product accuracy is relaxed
                            as the residual falls (inexact Krylov, the remark in
                            Sec. 2.2.1): FP64 products while the residual estimate
                            is above tol / 1e-7 relative to ||b||, FP32-pair products
                            below it (their error, under 1e-7 relative, is then
                            within tol ||b|| / ||r_k||); each cycle still ends with
                            an FP64 residual, which alone decides convergence. */
    int32_t restart;     /* GMRES cycle length m in 1..255; 0 -> 100 */
    int32_t max_iters;   /* Arnoldi steps over all cycles; 0 -> 1000 */
    int32_t pad;
    double inner_tol;    /* refinement: residual reduction asked of each inner cycle;
                            0 -> 1e-5 */
    double u_tol;        /* mobility solves only: bound on the forward error of the body
                            velocities, ||U - U_exact|| / ||U_exact||, in addition to
                            `tol`; 0 -> off.  A relative residual r leaves a velocity
                            error of about gamma r, with gamma depending on the
                            system's conditioning (3-5 for the wall boomerangs).  The
                            solver measures gamma from its own refinement cycles: a
                            cycle started from the iterate x_c with residual r_c
                            computes the correction d ~ x_exact - x_c, so
                            gamma ~ (||d_U|| / ||x_U||) / r_c.  It then stops only
                            when r <= min(tol, u_tol / (2 gamma)), reported as
                            tol_internal (half the bound absorbs the error of the
                            estimate itself).  A solve whose first cycle already meets
                            `tol` runs one short verification cycle (residual reduced
                            tenfold) to measure gamma.  A gamma measured by a cycle
                            that reduced the residual less than 1000-fold (such as
                            that one) is trusted less: the target is then
                            u_tol / (4 gamma).  RMB_EINVAL for resistance solves. */
} rmb_solve_opts;

typedef struct {
    int32_t status;        /* rmb_status of this solve */
    int32_t iterations;    /* Arnoldi steps */
    int32_t cycles;        /* GMRES cycles (restarts and refinement sweeps) */
    int32_t matvecs_fp64;  /* FP64 pair products, residual checks included */
    int32_t matvecs_fp32;  /* FP32-pair products */
    int32_t pad;
    double rel_residual;   /* final ||b - A x|| / ||b|| with the FP64 operator */
    double seconds;        /* host wall time from admission to completion */
    double tol_internal;   /* residual target the solve ended with: tol, or
                              min(tol, u_tol / (2 gamma)) (u_tol / (4 gamma) after a
                              short cycle) under velocity-error control */
    double u_err_est;      /* estimated ||U - U_exact|| / ||U_exact|| of the result
                              (gamma * rel_residual), or -1 when u_tol is off or no
                              refinement cycle has measured gamma */
    double gamma;          /* measured velocity-error amplification (see u_tol), or -1 */
} rmb_solve_info;

/* Mobility problem: given F (device [N][6], force then torque about q_p) and
 * optional slip (device [Nb][3] or NULL), returns U (device [N][6]) and
 * lambda (device [Nb][3]) with b = [slip; -F], x0 = 0.  `pc` may be a
 * preconditioner built by rmb_precond_factor or rmb_precond_factor_shapes
 * for this same system, or NULL
 * (factorised internally).  opts may be NULL (defaults).  info may be NULL.
 * Errors: RMB_EINVAL, RMB_ENOTSPD, RMB_ENOCONV (outputs hold the last
 * iterate; info->rel_residual its FP64 residual), RMB_ENOMEM, RMB_EDEVICE.
 * Blocks until the solve is complete (one stream synchronisation per
 * Arnoldi step). */
rmb_status rmb_solve_mobility(rmb_ctx ctx, const rmb_system *sys, const rmb_precond pc, const double *FT,
                              const double *slip, double *U, double *lambda, const rmb_solve_opts *opts,
                              rmb_solve_info *info, rmb_stream stream);

/* Resistance problem (eq:resistance_problem): given body velocities U
 * (device [N][6]: u then omega) and optional slip (device [Nb][3] or NULL),
 * solves M lambda = K U + slip (M + diag(d) for permeable bodies) and
 * returns F = K^T lambda (device [N][6]: force, then torque about q_p) and
 * lambda (device [Nb][3]).  Right-preconditioned GMRES from lambda = 0 with
 * the block-diagonal preconditioner M_pp^-1 (the same per-body factors as
 * the mobility solve; `pc` from rmb_precond_factor or
 * rmb_precond_factor_shapes for this system, or NULL); opts as for the
 * mobility solve, the tolerance applying to ||K U + slip - M lambda|| /
 * ||K U + slip||.  Unlike the mobility problem, its iteration count grows
 * with the linear extent of the suspension (Sec. 4.4).  Errors:
 * RMB_EINVAL, RMB_ENOTSPD (a body's M_pp not positive definite),
 * RMB_ENOCONV, RMB_ENOMEM, RMB_EDEVICE.  Blocks until complete. */
rmb_status rmb_solve_resistance(rmb_ctx ctx, const rmb_system *sys, const rmb_precond pc, const double *U,
                                const double *slip, double *F, double *lambda, const rmb_solve_opts *opts,
                                rmb_solve_info *info, rmb_stream stream);

/* `count` independent mobility problems solved together: every active
 * system advances one Arnoldi step per batched launch, and systems are
 * admitted as device memory frees up.  Arrays of length `count` (host
 * arrays of device pointers; slip entries may be NULL).  Each system's
 * result is bitwise identical to solving it alone with the same options.
 * Returns RMB_OK if every solve succeeded, else the first failing status;
 * per-system statuses are in infos[k].status (infos required). */
rmb_status rmb_solve_batch(rmb_ctx ctx, int32_t count, const rmb_system *systems, const double *const *FT,
                           const double *const *slip, double *const *U, double *const *lambda,
                           const rmb_solve_opts *opts, rmb_solve_info *infos, rmb_stream stream);

/* ---------------------------------------------------------------------------
 * Continuous-batching server
 * ------------------------------------------------------------------------- */

typedef struct rmb_server_s *rmb_server;

/* A request loop over one stream.  At most `max_active` systems run at once
 * (0 -> 1024); admission is first-come first-served and by device-memory
 * footprint within the context's budget. */
rmb_status rmb_server_create(rmb_ctx ctx, int32_t max_active, rmb_stream stream, rmb_server *out);

/* Queues one mobility problem.  The server copies `*sys` and its host
 * body_off array; every device buffer it points to (pos, q, FT, slip, U,
 * lambda) must stay valid until the request is returned by
 * rmb_server_poll.  `tag` identifies the request in poll results.
 * Errors: RMB_EINVAL (bad request), RMB_ENOMEM (the request can never fit
 * the budget). */
rmb_status rmb_server_submit(rmb_server srv, const rmb_system *sys, const double *FT, const double *slip,
                             double *U, double *lambda, const rmb_solve_opts *opts, int64_t tag);

/* Admits queued requests that fit, then advances every active request by
 * one step (setup, an Arnoldi step, or a cycle's update and FP64 residual).
 * Reports the number of active and queued requests.  Synchronises the
 * server's stream once. */
rmb_status rmb_server_step(rmb_server srv, int32_t *n_active, int32_t *n_queued);

/* Returns up to max_out completed requests (tags and infos, host arrays)
 * in completion order; *n_out receives the count. */
rmb_status rmb_server_poll(rmb_server srv, int32_t max_out, int64_t *tags, rmb_solve_info *infos,
                           int32_t *n_out);

/* Destroys the server; requests still queued or active are abandoned. */
void rmb_server_destroy(rmb_server srv);

#ifdef __cplusplus
}
#endif

#endif /* RMB_H */
