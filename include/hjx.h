/*
 * hjx.h -- C ABI of libhjx, MI355X (gfx950) explicit time stepping of the
 * Hamilton-Jacobi initial-value problem on dense Cartesian grids, after the
 * level-set toolbox of LevelSetPy (arXiv 2411.03501).
 *
 * The problem (Sec. II, eq. (ivp)): find phi(x, tau) with
 *     phi_tau + H(x, grad phi) = 0,   phi(x, 0) = phi0(x),
 * tau being time to go.  Its zero sublevel set is a backward reachable set;
 * with min-with-target after every step it is a reachable tube (Sec. VI,
 * variational HJ PDE).  One step of the solver:
 *   1. upwind one-sided derivatives p-_d, p+_d along every axis, with ghost
 *      cells (first order, ENO2, ENO3 or WENO5; Sec. IV-A..IV-C);
 *   2. the Lax-Friedrichs numerical Hamiltonian
 *      Hhat = H(x, (p- + p+)/2) - sum_d alpha_d (p+_d - p-_d)/2 with
 *      alpha_d the grid-wide maximum of |dH/dp_d| (Sec. IV-D, Listing 4);
 *   3. dt = cfl / sum_d alpha_d / dx_d (Sec. IV-D CFL condition, Sec. V);
 *   4. TVD Runge-Kutta of order 1, 2 or 3 on L = -Hhat (Sec. V, odeCFL1/2/3),
 *      then phi <- min(phi, target) if a target is given (Sec. VI).
 *
 * Conventions shared by every call
 * --------------------------------
 * Arrays: device memory owned by the caller, contiguous, row-major with the
 *   LAST axis fastest, n[0]*...*n[dim-1] elements of the problem's dtype
 *   (float for HJX_F32, double for HJX_F64).  The library never frees,
 *   keeps or copies to the host any caller array.
 * Streams: every call that touches the device enqueues on `stream`
 *   (a hipStream_t; NULL is the null stream).  Calls that return host values
 *   (hjx_dissipation, hjx_solve) synchronise that stream.
 * Errors: every call returns an hjx_status; on failure hjx_last_error()
 *   describes it.  Arguments are validated before anything is enqueued.
 * Threads: a problem handle may be used by one thread at a time; distinct
 *   handles are independent.
 * Limits: 1 <= dim <= 4; 3 <= n[d]; total nodes < 2^31; in 1-D and 2-D an
 *   array under 4 GiB, in 3-D a plane of the two fastest axes and in 4-D
 *   seven of them under 4 GiB (HJX_ERR_UNSUPPORTED at create otherwise).
 * Environment: HJX_MAX_WORKSPACE (bytes), read at every create call, caps
 *   the device workspace one hjx_problem_create, hjx_tape_create or
 *   hjx_batch_create may allocate (HJX_ERR_OOM beyond it; a tape then keeps
 *   no derivative store if that would pass the cap); HJX_TUNE_VERBOSE makes
 *   the autotuners print each candidate's time to stderr; HJX_TRACE (not
 *   "0") puts a roctx range around every call and every reverse-sweep
 *   segment (rocprofv3 --marker-trace shows them); HJX_SOLVE_GRAPH=0 keeps
 *   hjx_solve from capturing and replaying its launches.
 */
#ifndef HJX_H
#define HJX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HJX_OK = 0,
    HJX_ERR_INVALID_ARG = 1, /* a NULL pointer, a value out of range, an inconsistent descriptor */
    HJX_ERR_UNSUPPORTED = 2, /* a combination the library does not implement */
    HJX_ERR_DEVICE = 3,      /* a HIP runtime call failed */
    HJX_ERR_NONFINITE = 4,   /* NaN or Inf in the data (the output is still written) */
    HJX_ERR_OOM = 5          /* device memory could not be allocated */
} hjx_status;

typedef enum { HJX_F32 = 0, HJX_F64 = 1 } hjx_dtype;

/* Spatial derivative scheme ('CoStateCalc', Listing 4): Sec. IV-A upwindFirstFirst,
 * Sec. IV-B upwindFirstENO2 / upwindFirstENO3, Sec. IV-C upwindFirstWENO5. */
typedef enum {
    HJX_DERIV_FIRST = 1,
    HJX_DERIV_ENO2 = 2,
    HJX_DERIV_ENO3 = 3,
    HJX_DERIV_WENO5 = 5
} hjx_deriv;

/* TVD Runge-Kutta order, Sec. V (odeCFL1, odeCFL2, odeCFL3). */
typedef enum { HJX_RK1 = 1, HJX_RK2 = 2, HJX_RK3 = 3 } hjx_rk;

/* Restricted update (Sec. VI: the variational HJ PDE with min[0, H], and
 * the 'positive' field of the rockets listing, Listing 4, which the paper
 * does not define).  The rate L of every RK stage is clipped before the
 * stage combination:
 *   HJX_RESTRICT_NONE         L unchanged;
 *   HJX_RESTRICT_NONPOSITIVE  L <- min(L, 0): phi never rises in time to go,
 *                             so {phi <= 0} only grows (the tube form);
 *   HJX_RESTRICT_POSITIVE     L <- max(L, 0): phi never falls.
 * hjx_rhs always returns the unclipped L; the CFL step is unchanged. */
typedef enum {
    HJX_RESTRICT_NONE = 0,
    HJX_RESTRICT_NONPOSITIVE = 1,
    HJX_RESTRICT_POSITIVE = 2
} hjx_restrict;

/* Built-in Hamiltonians (device code cannot call back into Python, so the
 * 'hamFunc'/'partialFunc' pair of Listing 4 is a kind plus parameters).
 *   HJX_HAM_NORMAL      any dim, p = {a}: H = a |p|, alpha_d = |a|.
 *   HJX_HAM_DUBINS3_PE  dim 3, axes (x, y, theta), p = {v_e, v_p, wbar_e, wbar_p}:
 *       pursuit-evasion of two unicycles in the evader's frame,
 *       H = -[p1(-v_e + v_p cos th) + p2 v_p sin th
 *             + wbar_e |p1 y - p2 x - p3| - wbar_p |p3|],
 *       alpha = (|-v_e + v_p cos th| + wbar_e|y|, |v_p sin th| + wbar_e|x|,
 *                wbar_e + wbar_p).  Requires wbar_e, wbar_p >= 0.
 *   HJX_HAM_DUBINS4     dim 4, axes (x, y, theta, v), p = {wbar, abar}:
 *       car with speed state, reach: H = -v(p1 cos th + p2 sin th)
 *       + wbar|p3| + abar|p4|, alpha = (|v cos th|, |v sin th|, wbar, abar).
 *       Requires wbar, abar >= 0.
 *   HJX_HAM_ROCKETS     dim 3, axes (x, z, theta), p = {a, g, ubar_e, ubar_p}:
 *       the two-rocket game of Sec. VI with the vector field of the max-min
 *       in eq. (ham_def) (a_e = a_p = a; |u_e| <= ubar_e, |u_p| <= ubar_p):
 *       H = -[a p1 cos th + p2 (a sin th + a - g)
 *             + ubar_e |p1 x - p3| - ubar_p |p2 x + p3|],
 *       alpha = (|a cos th| + ubar_e|x|, |a sin th + a - g| + ubar_p|x|,
 *                ubar_e + ubar_p).  Requires ubar_e, ubar_p >= 0. */
typedef enum {
    HJX_HAM_NORMAL = 0,
    HJX_HAM_DUBINS3_PE = 1,
    HJX_HAM_DUBINS4 = 2,
    HJX_HAM_ROCKETS = 3
} hjx_ham_kind;

#define HJX_MAX_DIM 4

/* Grid (Sec. III-B, Listing 1: gmin, gmax, N, periodic dims).  A
 * non-periodic axis d has n[d] nodes from gmin[d] to gmax[d] inclusive
 * (dx = (gmax-gmin)/(n-1)); a periodic axis covers [gmin, gmax) with
 * dx = (gmax-gmin)/n.  Bit d of periodic_mask makes axis d periodic; the
 * other axes get linearly extrapolated ghost cells. */
typedef struct {
    int32_t dim;
    uint32_t periodic_mask;
    double gmin[HJX_MAX_DIM];
    double gmax[HJX_MAX_DIM];
    int64_t n[HJX_MAX_DIM];
} hjx_grid_desc;

/* Numerical Hamiltonian ('dissFunc', Listing 4):
 *   HJX_DISS_GLOBAL   Lax-Friedrichs, alpha_d = the grid maximum of the
 *                     partial bound (artificialDissipationGLF, Sec. IV-D);
 *   HJX_DISS_LOCAL    Lax-Friedrichs, alpha_d = the partial bound at the node
 *                     itself (the local form, not in the paper);
 *   HJX_DISS_GODUNOV  HJX_HAM_NORMAL only: Godunov's, per axis the extremum
 *                     of a|p| over the interval between p- and p+ (min for
 *                     a >= 0, max for a < 0), Hhat = a sqrt(sum q_d^2), with
 *                     q_d = max(max(p-_d, 0), -min(p+_d, 0)) for a >= 0 and
 *                     max(-min(p-_d, 0), max(p+_d, 0)) for a < 0 (not in the
 *                     paper).
 * The CFL step uses the grid maximum of the partial bound in every case.
 * The adjoint of the local form differentiates each node's bound in the
 * parameters (d|s|/ds = sign(s)); that of Godunov's follows the one-sided
 * values the forward selected (ties as the forward breaks them), with
 * d|q|/dq = 0 at q = 0. */
typedef enum { HJX_DISS_GLOBAL = 0, HJX_DISS_LOCAL = 1, HJX_DISS_GODUNOV = 2 } hjx_dissipation_kind;

typedef struct {
    int32_t kind;        /* hjx_ham_kind */
    int32_t dissipation; /* hjx_dissipation_kind */
    double p[8];
} hjx_ham_desc;

typedef struct {
    int32_t deriv; /* hjx_deriv */
    int32_t rk;    /* hjx_rk */
    double cfl;    /* 0 < cfl <= 1 */
    int32_t dtype; /* hjx_dtype */
    int32_t restrict_update; /* hjx_restrict */
} hjx_scheme_desc;

typedef struct {
    int64_t steps;              /* RK steps taken */
    double dt;                  /* the CFL step */
    double dt_last;             /* the last (clamped) step */
    double t_final;
    double alpha[HJX_MAX_DIM];  /* dissipation coefficients used */
    double elapsed_ms;          /* device time of the stepping loop */
    double alg_bytes;           /* algorithmic HBM bytes of the stepping loop */
} hjx_stats;

typedef struct hjx_problem hjx_problem;

/* Library version, "major.minor.patch". */
const char *hjx_version(void);

/* Description of the last failure on the calling thread ("" if none).  The
 * string stays valid until the next hjx call on that thread. */
const char *hjx_last_error(void);

/* Create a problem: validates the descriptors, builds the per-axis
 * coordinate tables (Sec. III-B) on the device and allocates the stage
 * workspace (two arrays of n[0]*..*n[dim-1] elements).  On success *out owns
 * that memory until hjx_problem_destroy.  Selects the current HIP device. */
hjx_status hjx_problem_create(const hjx_grid_desc *grid, const hjx_ham_desc *ham,
                              const hjx_scheme_desc *scheme, hjx_problem **out);

/* Free a problem and its device memory (NULL is a no-op).  The caller must
 * make sure no enqueued work still uses it. */
hjx_status hjx_problem_destroy(hjx_problem *p);

/* Replace the Hamiltonian's parameters (the p[] of hjx_ham_desc, the
 * dynamics' bounds of Listing 4's schemeData) of an existing problem: params
 * is a host array of the kind's parameter count (1, 4, 2 or 4 doubles),
 * checked as hjx_problem_create checks them.  The dissipation bounds are
 * reduced again at the next call that needs them, and a captured solve is
 * dropped.  A tape or batch made before the change refuses to run
 * (HJX_ERR_INVALID_ARG) until the parameters are set back. */
hjx_status hjx_problem_set_params(hjx_problem *p, const double *params);

/* Dissipation coefficients and CFL step (Sec. IV-D, GLF dissipation of
 * Listing 4): alpha_d = max over all grid nodes of the partial bound,
 * reduced on the device; dt = cfl / sum_d alpha_d/dx_d (+inf when every
 * alpha_d is 0).  alpha_out: host array of at least dim doubles; dt_out:
 * host double.  alpha depends only on the grid and the parameters, fixed at
 * create: the first call that needs it (this one, or any call below that
 * steps) reduces it and synchronises `stream`; later calls reuse it without
 * touching the device. */
hjx_status hjx_dissipation(hjx_problem *p, double *alpha_out, double *dt_out, void *stream);

/* Lax-Friedrichs right-hand side L = -Hhat(phi) at every node (Sec. IV,
 * steps 1-2 above), with the grid-wide alpha.  phi, L_out: device arrays
 * (may not alias).  Asynchronous on `stream`. */
hjx_status hjx_rhs(hjx_problem *p, const void *phi, void *L_out, void *stream);

/* One TVD-RK step of size dt (Sec. V), in place on phi, followed by
 * phi <- min(phi, target) when target != NULL (Sec. VI).  phi: device
 * array, read and written; target: device array or NULL, which must not
 * alias phi.  dt > 0.  Asynchronous on `stream`. */
hjx_status hjx_step(hjx_problem *p, void *phi, const void *target, double dt, void *stream);

/* Launch shape of the stage kernel (no counterpart in the paper, whose
 * stages are whole-array expressions).  The variants compute the same
 * arithmetic, so results are bit-for-bit the same for every shape:
 *   HJX_TILE_PLANE_MARCH: a block covers tx nodes of the fastest axis by ty
 *     nodes of the second-fastest (ty = 1 when dim = 1), stages that plane
 *     tile with its halo in LDS, evaluates each stencil interval once and
 *     marches over `march` nodes of another axis (ignored when dim < 3).
 *     1-D and 2-D: blocks of tx x ty threads, 1 <= tx*ty <= 256.  3-D and
 *     4-D: blocks of 512 threads over 1 <= tx*ty <= 512 nodes, the
 *     intervals of the tile dealt evenly over them, the march along axis 0,
 *     and axis 1 of a 4-D grid gathered node by node;
 *   HJX_TILE_DIRECT: one thread per node, stencils gathered through the
 *     caches (tx, ty, march ignored); arrays must be under 4 GiB, else
 *     HJX_ERR_UNSUPPORTED.
 *   HJX_TILE_STEPS (1-D and 2-D grids under 4 GiB, else
 *     HJX_ERR_UNSUPPORTED): hjx_solve takes `march` whole RK steps per
 *     launch.  A block of 256 threads owns a tx x ty output tile (tx along
 *     the fastest axis, ty along axis 0; ty = 1 in 1-D) and evaluates every
 *     stage of those steps in LDS over the tile and a halo of
 *     H = march * rk * radius nodes (radius 1 first order, 2 ENO2, 3 ENO3 and
 *     WENO5), which the neighbouring blocks evaluate as well.  Needs
 *     H <= n_d on a periodic axis and (2 buffers, 3 for RK3) x (tx + 2H) x
 *     (ty + 2H) values (a region never longer than a non-periodic axis) in
 *     64 KiB, else HJX_ERR_INVALID_ARG.  Everything other than hjx_solve's
 *     stepping (hjx_step, hjx_rhs, the tape) takes the direct variant.
 * hjx_problem_create picks a default (the steps variant for 1-D and 2-D
 * grids of at most 65536 nodes); hjx_tune may replace it. */
#define HJX_TILE_PLANE_MARCH 0
#define HJX_TILE_DIRECT 1
#define HJX_TILE_STEPS 2
hjx_status hjx_problem_set_tile(hjx_problem *p, int32_t variant, int32_t tx, int32_t ty, int32_t march);
hjx_status hjx_problem_get_tile(const hjx_problem *p, int32_t *variant, int32_t *tx, int32_t *ty,
                                int32_t *march);

/* Autotuner: times the stage kernel on this problem for a set of candidate
 * launch shapes (row widths that split the fastest axis evenly, tiles of
 * 64..256 nodes in 1-D and 2-D and of 512 in 3-D and 4-D, march lengths
 * 1..32, the direct variant, and in 1-D and 2-D steps tiles of 64..1024
 * nodes with 1..8 steps per launch) and keeps the fastest with
 * hjx_problem_set_tile.  Each candidate is timed twice on `reps` whole RK
 * steps from phi into a temporary array, without a target, launched as
 * hjx_solve launches them; the faster timing counts.  phi: device
 * array of the problem's size and dtype, read only.  reps: timed steps per
 * candidate (>= 1).  best_us (host, optional): the winner's mean time per
 * stage launch.  Allocates one temporary array of the problem's size for the
 * duration of the call.  Results do not depend on the choice.  Synchronises
 * `stream`.
 * cache_path: a text file of tuned shapes, one line per problem, keyed by the
 * device (architecture and compute units) and by what the shape can depend
 * on (dtype, sizes, periodic axes, scheme, RK order, Hamiltonian kind,
 * dissipation, restricted update).  A line for this problem sets its shape
 * without timing anything (best_us is the recorded time); otherwise the
 * tuner runs and appends its result.  NULL: the environment variable
 * HJX_TUNE_CACHE names the file, if set; "": no cache.  A file that cannot
 * be read or written is treated as empty. */
hjx_status hjx_tune(hjx_problem *p, const void *phi, int32_t reps, const char *cache_path, void *stream,
                    double *best_us);

/* Solve from t0 to t1 (Listing 3 odeCFLx(schemeFunc, tspan, y0, ...)):
 * steps of the CFL size dt, the one that would reach t1 (or come within
 * 1e-12 max(1,|t1|) of it) clamped to land on t1.  phi0: initial data;
 * target: device array for min-with-target, or NULL for none (target may be
 * phi0, but not phi_out); phi_out: result (may be phi0 itself).  t1 >= t0.
 * The call enqueues a NaN/Inf check of phi0, the steps and a check of the
 * result (under HJX_TILE_STEPS the first and the last stepping launch make
 * the two checks themselves), then synchronises `stream` once.  Returns HJX_ERR_NONFINITE if
 * phi0 or the result holds NaN/Inf (phi_out is written either way).
 * stats (optional, host) receives the step record.
 * When the same solve (the same phi0, target, phi_out, t0 and t1) is asked
 * for twice in a row, the second call captures the stepping launches into a
 * hipGraph on a stream of the problem's own and every later identical call
 * replays it (the same kernels and arguments, so the same bits);
 * hjx_problem_set_tile, hjx_tune and any different solve drop it.  The
 * environment variable HJX_SOLVE_GRAPH=0 keeps every solve on direct
 * launches. */
hjx_status hjx_solve(hjx_problem *p, const void *phi0, const void *target, void *phi_out,
                     double t0, double t1, void *stream, hjx_stats *stats);

/* ------------------------------------------------------------------ adjoint
 * Gradients of a loss of phi(t1) through the whole solve (no counterpart in
 * the paper; the discrete adjoint of the scheme above).  A tape fixes the
 * time schedule of one solve (the CFL step count and the clamped last step,
 * as hjx_solve would take them) and holds checkpoints of phi every
 * ckpt_every steps; hjx_adjoint replays each segment from its checkpoint
 * and runs the transposed stages backwards:
 *   dL/dphi0    the adjoint at t0 through phi0 (the initial value only),
 *   dL/dtarget  through the target of min-with-target, when there is one
 *               (when the target is phi0 itself, dL/dphi0 of the whole map
 *               is the sum of the two),
 *   dL/dparams  through the Hamiltonian parameters, including their effect
 *               on the dissipation coefficients and on the CFL step (the
 *               number of steps held fixed).
 * Subgradient conventions at kinks: d|s|/ds = sign(s) with sign(0) = 0; at
 * a tie of min-with-target the evolved value is the one kept; a rate of
 * exactly 0 under a restricted update is not clipped (derivative 1); a
 * maximum of the dissipation bound differentiates at its first maximising
 * node. */
typedef struct hjx_tape hjx_tape;

/* Create a tape for a solve of p from t0 to t1 (t1 >= t0) with a checkpoint
 * every ckpt_every >= 1 steps.  Runs the dissipation reduction (synchronises
 * `stream`) and allocates the checkpoints and the replay workspace: about
 * (steps/ckpt_every + 6 ckpt_every + 4 + 3 dim) arrays of the problem's size, plus
 * the derivative store of hjx_tape_set_mode.
 * Arrays must be under 4 GiB each (else HJX_ERR_UNSUPPORTED).  With a restricted update the replay also keeps, per
 * stage, a byte per node that records where the rate was clipped: a clipped
 * rate is the constant 0 and passes no adjoint (ckpt_every x rk more bytes
 * per node in each of the two replay sets). */
hjx_status hjx_tape_create(hjx_problem *p, double t0, double t1, int32_t ckpt_every, void *stream,
                           hjx_tape **out);
hjx_status hjx_tape_destroy(hjx_tape *tape);

/* What the replay keeps for the reverse sweep.  HJX_TAPE_STORE_DERIVS keeps
 * the derivative approximations p-_d, p+_d of every stage of a segment
 * (2 ckpt_every * rk * 2 dim more arrays of the problem's size), so the
 * reverse sweep reads them instead of evaluating the stencils again;
 * HJX_TAPE_RECOMPUTE keeps none.  hjx_tape_create picks STORE_DERIVS when
 * that memory is at most a quarter of the device's free memory.  Both modes
 * give the same bits.  set_mode allocates or frees the store (HJX_ERR_OOM if
 * it does not fit). */
#define HJX_TAPE_RECOMPUTE 0
#define HJX_TAPE_STORE_DERIVS 1
hjx_status hjx_tape_set_mode(hjx_tape *tape, int32_t mode);
hjx_status hjx_tape_get_mode(const hjx_tape *tape, int32_t *mode);

/* hjx_solve on the tape's schedule, recording the checkpoints.  The target
 * (NULL for none; may be phi0, not phi_out) must stay unchanged until
 * hjx_adjoint has run. */
hjx_status hjx_solve_taped(hjx_problem *p, hjx_tape *tape, const void *phi0, const void *target, void *phi_out,
                           void *stream, hjx_stats *stats);

/* Reverse sweep after hjx_solve_taped.  dL_dphiT: device array, the
 * gradient of the loss with respect to phi(t1).  dL_dphi0: device array
 * (output).  dL_dtarget: device array (output) or NULL; must be NULL when
 * the solve had no target.  dL_dtarget == dL_dphi0 asks for the gradient
 * of the whole map when phi0 is also the target: that array then receives
 * dL/dtarget + dL/dphi0.  dL_dparams: host array of 8 doubles (output, the
 * entries past the kind's parameter count are 0) or NULL.  All work runs on
 * `stream`: each segment's replay shares launches with the reverse sweep of
 * the segment after it.  `stream` is synchronised at the end. */
hjx_status hjx_adjoint(hjx_problem *p, hjx_tape *tape, const void *dL_dphiT, void *dL_dphi0, void *dL_dtarget,
                       double *dL_dparams, void *stream);

/* Smoothed volume of {phi <= 0}: loss = cell volume * sum_i s(-phi_i / eps),
 * s the logistic function, and its gradient dL/dphi (device array, may be
 * NULL).  loss: host double.  eps > 0.  Synchronises `stream`. */
hjx_status hjx_loss_volume(hjx_problem *p, const void *phi, double eps, double *loss, void *dL_dphi,
                           void *stream);

/* ------------------------------------------------------------------ batch
 * Many problems solved together (no counterpart in the paper: for every
 * member the same solve as hjx_solve from t0 = 0, scheduled as one).  The
 * members may differ in grid, sizes, Hamiltonian and parameters but share
 * dtype, derivative scheme and RK order.  Each RK stage of each global step
 * is one launch of persistent blocks over a work list of (member, run of
 * item_nodes nodes) items; members are ordered by decreasing step count, so
 * a step launches only over those still stepping, and every member keeps
 * its own CFL step and clamped last step.  The launches of one set of
 * horizons are captured once in a hipGraph and replayed while the step
 * counts stay the same.  Results are bit-for-bit those of hjx_solve on each
 * member.  The batch borrows each member's stage workspace: members must
 * outlive the batch, appear once in it, and not be stepped otherwise while
 * a batch solve is in flight.  Member arrays must be under 4 GiB. */
typedef struct hjx_batch hjx_batch;

/* Create a batch of n >= 1 problems (host array of handles, each used once).
 * Runs the dissipation reduction of every member and fixes its CFL step
 * (synchronises `stream`).  The launch shape defaults to the resident
 * block count and 1024-node items.  Any Hamiltonian, dissipation form and
 * restricted update may be mixed; a batch with a ROCKETS member or a local
 * or Godunov dissipation runs a kernel that carries those too (and has its
 * own occupancy). */
hjx_status hjx_batch_create(int32_t n, hjx_problem *const *problems, void *stream, hjx_batch **out);
hjx_status hjx_batch_destroy(hjx_batch *b);

/* Launch shape: item_nodes (a multiple of 256, at most 2^20) nodes per work
 * item, `blocks` persistent blocks per launch (1..blocks_max, the count
 * resident on the whole device).  Results do not depend on it. */
hjx_status hjx_batch_set_shape(hjx_batch *b, int32_t item_nodes, int32_t blocks);
hjx_status hjx_batch_get_shape(const hjx_batch *b, int32_t *item_nodes, int32_t *blocks, int32_t *blocks_max);

/* Solve every member i from 0 to t1[i] >= 0 (host array of n doubles; at
 * most 2^20 steps each).  phi0, phi_out: host arrays of n device pointers
 * (phi_out[i] may be phi0[i]); target: NULL, or a host array of n device
 * pointers each NULL or a target that is not phi_out[i].  stats: NULL or a
 * host array of n records (elapsed_ms is the whole batch's).  Synchronises
 * `stream`.  Returns HJX_ERR_NONFINITE without stepping if some phi0 holds
 * NaN/Inf, and after the solve if some result does (the lowest such member
 * is named by hjx_last_error). */
hjx_status hjx_batch_solve(hjx_batch *b, const void *const *phi0, const void *const *target, void *const *phi_out,
                           const double *t1, void *stream, hjx_stats *stats);

/* Autotuner of the batch launch shape: runs hjx_batch_solve with the given
 * arguments, then times `reps` replays of the horizon per candidate shape
 * (items of 256, 1024 and 4096 nodes by 1, 2 and 4 blocks per compute unit
 * and blocks_max) and keeps the fastest.  phi_out is overwritten.
 * best_ms (optional, host): the winner's mean replay time. */
hjx_status hjx_batch_tune(hjx_batch *b, const void *const *phi0, const void *const *target, void *const *phi_out,
                          const double *t1, int32_t reps, void *stream, double *best_ms);

/* ------------------------------------------------------------------
 * Implicit surfaces and shape operations (Sec. III: implicit surface
 * representations, Listing 2, and the calculus on implicit functions), built
 * on the device.  Arrays are device memory of the grid's size (row-major,
 * last axis fastest) in the given dtype.                                   */
typedef enum {
    HJX_SHAPE_BALL = 0,      /* sqrt(sum_{d in mask} (x_d - c_d)^2) - r: the signed distance to a
                                sphere (every axis in mask) or a cylinder (some axes) */
    HJX_SHAPE_ELLIPSOID = 1  /* sum_{d in mask} w_d (x_d - c_d)^2 - r: Listing 2's form (not a distance) */
} hjx_shape_kind;

typedef struct {
    int32_t kind;            /* hjx_shape_kind */
    uint32_t axis_mask;      /* bit d: axis d takes part (at least one axis, none beyond dim) */
    double center[HJX_MAX_DIM];
    double weights[HJX_MAX_DIM]; /* ELLIPSOID only; finite */
    double radius;
} hjx_shape_desc;

/* phi_out[node] = the shape at the node's coordinates (gmin_d + j dx_d, the
 * grid of hjx_grid_desc), evaluated in double and rounded once to dtype.
 * Asynchronous on `stream`. */
hjx_status hjx_shape(const hjx_grid_desc *grid, const hjx_shape_desc *shape, int32_t dtype, void *phi_out,
                     void *stream);

/* The shapes of 1 <= n <= 65535 grids in one launch (initial data of a batch):
 * phi_out[k] = shapes[k] on grids[k], as hjx_shape would write it.  grids,
 * shapes, phi_out: host arrays of n entries; each phi_out[k] a device array
 * of grids[k]'s size.  Copies the n descriptors to a temporary device array
 * and synchronises `stream`. */
hjx_status hjx_shape_batch(int32_t n, const hjx_grid_desc *grids, const hjx_shape_desc *shapes, int32_t dtype,
                           void *const *phi_out, void *stream);

/* hjx_shape_batch for callers that cannot allocate device memory: code
 * under stream capture, tight serving loops, harnesses that forbid hipMalloc.
 * The same construction with the same bits, but the n descriptors are staged
 * in a fixed array of the library (HJX_SHAPE_NOALLOC_MAX members: a
 * file-scope device array, one on every GPU the library runs on, held until
 * the process ends) and in static host storage, so the call allocates
 * nothing.  1 <= n <= HJX_SHAPE_NOALLOC_MAX, else HJX_ERR_INVALID_ARG.
 * Every call on a GPU shares that GPU's array, which keeps the last call's
 * descriptors (they are rewritten before each launch; nothing needs to start
 * at zero).  Calls that overlap on one GPU would race for it, so the library
 * runs one such call at a time per process, each holding the array until its
 * kernel has finished (the call synchronises `stream`). */
#define HJX_SHAPE_NOALLOC_MAX 1024
hjx_status hjx_shape_batch_noalloc(int32_t n, const hjx_grid_desc *grids, const hjx_shape_desc *shapes,
                                   int32_t dtype, void *const *phi_out, void *stream);

typedef enum {
    HJX_OP_UNION = 0,        /* min(a, b) */
    HJX_OP_INTERSECTION = 1, /* max(a, b) */
    HJX_OP_COMPLEMENT = 2,   /* -a (b unused, may be NULL) */
    HJX_OP_SUBTRACTION = 3   /* max(a, -b): the interior of a without that of b */
} hjx_shape_op_kind;

/* out[i] = op(a[i], b[i]) for 0 <= i < n, elementwise; out may alias a or b.
 * Asynchronous on `stream`. */
hjx_status hjx_shape_op(int32_t op, int32_t dtype, const void *a, const void *b, void *out, int64_t n, void *stream);

/* ------------------------------------------------------------------
 * Scalar conservation laws (Sec. IV-D): v_t + sum_d f_d(v)_{x_d} = 0 by the
 * Lax-Friedrichs scheme.  The paper prints it in one dimension,
 *   v_j' = v_j - (lambda/2)(f(v_{j+1}) - f(v_{j-1})) + (v_{j+1} - 2 v_j + v_{j-1})/2,
 * lambda = dt/dx, monotone when lambda max|f'| <= 1.  In N dimensions the new
 * value is the mean of the 2N axis neighbours minus the central flux
 * differences of every axis,
 *   v' = (1/2N) sum_d (v_{+d} + v_{-d}) - sum_d (dt/2dx_d)(f_d(v_{+d}) - f_d(v_{-d})),
 * monotone when (dt/dx_d) max|f_d'| <= 1/N on every axis.  Periodic axes wrap
 * (the grid of hjx_grid_desc); beyond a non-periodic edge the value is the
 * edge value.  Arrays are device memory of n[0]*..*n[dim-1] elements of the
 * handle's dtype, row-major, last axis fastest.                          */
typedef enum {
    HJX_FLUX_LINEAR = 0,  /* f_d(v) = c_d v       (|f_d'| = |c_d|) */
    HJX_FLUX_BURGERS = 1  /* f_d(v) = c_d v^2 / 2 (|f_d'| = |c_d| |v|) */
} hjx_flux_kind;

typedef struct hjx_claw hjx_claw;

/* Create a conservation law on `grid` with flux `flux`, coefficients c[0..dim-1]
 * (host array, finite), dtype HJX_F32 or HJX_F64 and CFL number 0 < cfl <= 1.
 * Allocates one work array of the grid's size.  Selects the current device. */
hjx_status hjx_claw_create(const hjx_grid_desc *grid, int32_t flux, const double *c, int32_t dtype, double cfl,
                           hjx_claw **out);
hjx_status hjx_claw_destroy(hjx_claw *h);

/* The CFL step for data v: cfl min_d dx_d / (N max|f_d'|), the maximum taken
 * over v for Burgers (a device reduction; synchronises `stream`); +inf when
 * nothing moves.  v may be NULL for the linear flux. */
hjx_status hjx_claw_dt(hjx_claw *h, const void *v, double *dt_out, void *stream);

/* One step of size dt >= 0 from v into v_out (must not alias).
 * Asynchronous on `stream`. */
hjx_status hjx_claw_step(hjx_claw *h, const void *v, void *v_out, double dt, void *stream);

/* Solve from 0 to t1 >= 0: checks v0 for NaN/Inf, takes the CFL step of v0
 * for every step (the scheme is monotone, so max|v| never grows) and lands
 * the step that would reach t1 (within 1e-12 relative) on t1.  v0 and v_out
 * must not alias; v0 is not modified.  Synchronises `stream`.  steps_out,
 * dt_out: optional host outputs.  HJX_ERR_NONFINITE if the result holds
 * NaN or Inf (it is still written). */
hjx_status hjx_claw_solve(hjx_claw *h, const void *v0, void *v_out, double t1, void *stream, int64_t *steps_out,
                          double *dt_out);

#ifdef __cplusplus
}
#endif

#endif /* HJX_H */
