/*
 * sird.h -- C ABI of the gfx950 library for batched calibration of the SIRD
 * model (Blaszczyk, Klimczak, Mahdi, Oprocha, "On automatic calibration of
 * the SIRD epidemiological model for COVID-19 data in Poland").
 *
 * What the calls compute
 *   The model is eq. (SIRD) of Sec. 2.2:
 *       S' = -(beta/N) S I,  I' = (beta/N) S I - (gamma + mu) I,
 *       R' = gamma I,        D' = mu I.
 *   A calibration window (Sec. 3.1) is W days with W+1 daily observations
 *   y_0..y_W of cumulative deaths.  The transmission rate is
 *   piecewise constant: beta_k on days [k*seg_days, (k+1)*seg_days), the last
 *   segment extending to the window end (this replaces the two-level ramp of
 *   eq. (beta); the segment of a step is fixed by the step index, so all four
 *   stages of a step use one beta).  The integrator is classical RK4 with a
 *   fixed step h = 1/steps_per_day (the paper's Euler scheme, Sec. 3.1 and
 *   3.3, is replaced by a fourth-order one).  The cost (Sec. 3.1) compares the
 *   model's deceased compartment with y; the optimiser is particle swarm
 *   optimisation with box clamping (Sec. 3.3).
 *
 * Parameter vector of one particle, d = K + 3 values:
 *       theta = (beta_1, ..., beta_K, gamma, mu, I0)
 *   Initial state: S = N - I0 - R0 - D0, I = I0, R = R0, D = D0.
 *   A fixed parameter is a degenerate box dimension (lo == hi).
 *
 * Conventions for every call
 *   - Array arguments are DEVICE pointers owned by the caller; the library
 *     never allocates, frees or retains them.  Host structs are read during
 *     the call only.
 *   - Work is enqueued asynchronously on `stream` (a hipStream_t passed as
 *     void*; NULL = the null stream) and the call does not synchronise.
 *   - Every call returns SIRD_OK or a negative status.  Host-side argument
 *     checks run before any HIP call, so a rejected call has enqueued
 *     nothing.  sird_last_error() gives a thread-local message.
 *   - A batch holds n_prob independent problems ("fits"); a single fit is the
 *     n_prob = 1 case of the same code path.
 *   - Particle-indexed arrays (loss, pbest_f) have total_particles entries;
 *     problem r owns [p_off, p_off + n_part).
 *   - theta-shaped arrays (theta, x, v, pbest_x, grad_theta) hold, per
 *     problem, a structure-of-arrays block [d][n_part] starting at
 *     theta_off: parameter j of local particle p is at
 *     theta_off + j*n_part + p.
 *   - Box-shaped arrays (lo, hi, gbest_x) hold d values per problem starting
 *     at box_off.
 *   - Non-finite losses are not errors; the swarm treats NaN as +inf.
 *   - Calls sharing a batch's scheduler counters, or the same output
 *     buffers, must be ordered on one stream.
 */
#ifndef SIRD_H
#define SIRD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
#define SIRD_OK 0
#define SIRD_EINVAL (-1)   /* bad host-side argument (null, size, descriptor) */
#define SIRD_ENOSPACE (-2) /* workspace or output too small */
#define SIRD_EHIP (-3)     /* HIP runtime error while enqueueing */

/* ------------------------------------------------------ ODE state precision */
#define SIRD_F64 0 /* state and arithmetic in double */
#define SIRD_F32 1 /* state (S, I, R, D) and arithmetic in float, state
                      updates Kahan-compensated; theta, losses and the
                      swarm stay double */

/* ------------------------------------------------ costs of Sec. 3.1 on D */
/* e_i = y_i - Dhat_i over days i = 0..W, n = W + 1, g_i = max(y_i, 1) */
#define SIRD_LOSS_SSRE 0 /* sum_{i=1..W} ((Dhat_i - y_i)/g_i)^2           */
#define SIRD_LOSS_MSE 1  /* (1/n) sum e_i^2                                */
#define SIRD_LOSS_MXSE 2 /* max e_i^2                                      */
#define SIRD_LOSS_MAE 3  /* (1/n) sum |e_i|                                */
#define SIRD_LOSS_MAPE 4 /* (100/n) sum |e_i / g_i|                        */
/* F_IRD of Sec. 3.1: the maximum over Y in {I, R, D} of a low-level cost
 * on min-max normalised errors (y_i - yhat_i)/(max y - min y) (a flat
 * observed series is normalised by 1); MAPE is not normalised.  Needs a
 * batch with obs_series = 3. */
#define SIRD_LOSS_IRD_MXSE 5
#define SIRD_LOSS_IRD_MSE 6
#define SIRD_LOSS_IRD_MAE 7
#define SIRD_LOSS_IRD_MAPE 8

/* ------------------------------------------------------------- models */
#define SIRD_MODEL_RK4_SEGMENTS 0 /* RK4, beta piecewise constant on K
                                     segments; theta = (beta_1..beta_K,
                                     gamma, mu, I0)                      */
#define SIRD_MODEL_EULER_RAMP 1   /* the paper's own scheme (Sec. 3.1, 3.3):
                                     forward Euler with the ramp of
                                     eq. (beta) evaluated at the start of
                                     each step; K = 4 and theta = (beta1,
                                     beta2, t1, t2, gamma, mu, I0), t in
                                     days from the window start; the swarm
                                     keeps t1 <= t2 by swapping after
                                     every move (and at initialisation)  */

/* ------------------------------------------------------------ descriptors */
/* One calibration window (Sec. 3.1).  96 bytes, naturally aligned. */
typedef struct sird_problem {
    int32_t n_days;        /* W >= 1: observations on days 0..W            */
    int32_t steps_per_day; /* RK4 steps per day >= 1, h = 1/steps_per_day  */
    int32_t seg_days;      /* days per beta segment >= 1                   */
    int32_t n_seg;         /* K >= 1 beta segments; d = K + 3              */
    int32_t n_part;        /* particles (parameter vectors) >= 0           */
    int32_t model;         /* SIRD_MODEL_*                                 */
    double N;              /* population > 0                               */
    double R0;             /* removed (recovered) at day 0, >= 0           */
    double D0;             /* deceased at day 0, >= 0                      */
    int64_t p_off;         /* first entry in particle-indexed arrays       */
    int64_t theta_off;     /* first double of the [d][n_part] block        */
    int64_t obs_off;       /* first of the obs_series x (W+1) observations
                              (I, R, D when obs_series = 3; D when 1)     */
    int64_t traj_off;      /* first double of the [4][W+1][n_part] block   */
    int64_t box_off;       /* first of the d values in lo, hi, gbest_x     */
    uint64_t stream;       /* Philox key word 1 of this problem            */
} sird_problem;

/* 64 consecutive particles of one problem: the unit a wavefront integrates. */
typedef struct sird_tile {
    int32_t prob; /* problem index                      */
    int32_t p0;   /* first local particle, multiple of 64 */
} sird_tile;

/* A batch of problems plus its launch plan.  Host struct; the pointers are
 * device memory owned by the caller.  Fill it with sird_batch_plan(). */
typedef struct sird_batch {
    int32_t n_prob;          /* problems >= 1                                  */
    int32_t n_tiles;         /* entries of tiles                               */
    int32_t max_days;        /* max W over problems                            */
    int32_t max_d;           /* max d over problems                            */
    int64_t max_steps;       /* max W*steps_per_day over problems              */
    int64_t total_particles; /* sum of n_part; length of particle arrays       */
    int64_t theta_len;       /* doubles in theta-shaped arrays                 */
    int64_t obs_len;         /* doubles in obs                                 */
    int64_t traj_len;        /* doubles in traj                                */
    int64_t box_len;         /* doubles in box-shaped arrays                   */
    const sird_problem *probs; /* device copy of the problem table            */
    const sird_tile *tiles;    /* device copy of the tile table (LPT order)   */
    int32_t *sched;          /* device, 2 int32 zero-initialised scheduler
                                counters; needed only when persistent > 0      */
    int32_t dtype;           /* SIRD_F64 or SIRD_F32                           */
    int32_t block;           /* threads per block of the integration kernels:
                                64..1024, multiple of 64; 0 = 256               */
    int32_t persistent;      /* 0: one wavefront per tile, tiles dispatched in
                                table order; > 0: this many resident
                                wavefronts pull tiles from a device counter   */
    int32_t obs_series;      /* observed series per problem: 1 (D) or 3
                                (I, R, D); set by sird_batch_plan          */
    int32_t models;          /* bit m set when some problem has model m;
                                set by sird_batch_plan                     */
    int32_t max_part;        /* max n_part over problems; set by
                                sird_batch_plan (picks the global-best
                                kernel's shape and the L-BFGS kernels'
                                wavefronts per tile, min(64, max_part); a
                                value below the true maximum would leave
                                vectors out, 0 means 64)                   */
    int32_t waves_per_simd;  /* 0: as many wavefronts of the integration
                                kernels per SIMD as registers and LDS allow;
                                1..8: at most this many (the launch reserves
                                LDS so that no more blocks fit on a compute
                                unit; SIRD_EINVAL when the reservation would
                                exceed 64 KiB per block)                     */
    int32_t ppl;             /* particles per lane of the loss and swarm
                                integration: 0 or 1, or 2: a wavefront takes
                                two consecutive tiles of one problem (the
                                pairs of pair_tiles), each lane two particles,
                                with the same results bitwise; applies to
                                batches of the RK4 model with a
                                deceased-count cost and persistent = 0, the
                                others run with one                         */
    int32_t n_pairs;         /* entries of pair_tiles                        */
    const int32_t *pair_tiles; /* device, from sird_plan_pairs: the first tile
                                of every tile pair; read only when ppl = 2    */
} sird_batch;

/* Coefficients of the swarm, Sec. 3.3 (inertia, cognitive, social), the
 * Philox key word 0, and the search box (device, box-shaped). */
typedef struct pso_params {
    double w;
    double c1;
    double c2;
    uint64_t seed;
    const double *lo;
    const double *hi;
} pso_params;

/* Swarm state, all device memory owned by the caller. */
typedef struct pso_state {
    double *x;          /* positions, theta-shaped                           */
    double *v;          /* velocities, theta-shaped                          */
    double *pbest_x;    /* personal bests, theta-shaped                      */
    double *pbest_f;    /* personal best losses, particle-indexed            */
    double *gbest_x;    /* global best per problem, box-shaped               */
    double *gbest_f;    /* [n_prob]                                          */
    int64_t *gbest_idx; /* [n_prob], local particle index, -1 before any     */
    uint64_t *iter;     /* [2]: iteration counter and an internal counter;
                           pso_init sets both to 0                           */
    double *f;          /* losses of the current positions, particle-indexed */
    double *hist_f;     /* optional [hist_len][n_prob] gbest_f per iteration */
    int64_t *hist_idx;  /* optional [hist_len][n_prob] gbest_idx             */
    int64_t hist_len;   /* rows of hist_*; iterations >= hist_len are not
                           recorded                                           */
} pso_state;

/* Adam coefficients (Kingma & Ba 2015) for the projected refinement. */
typedef struct adam_params {
    double lr;
    double beta1;
    double beta2;
    double eps;
} adam_params;

/* ------------------------------------------------------------ host helpers */

/* Message for a status code.  Never NULL. */
const char *sird_status_string(int status);

/* Thread-local message of the last failed call on this thread ("" if none). */
const char *sird_last_error(void);

/* Check a host problem table against the array lengths it indexes:
 * W, steps_per_day, seg_days, n_seg >= 1; n_part >= 0; N > 0; R0, D0 >= 0;
 * model is a SIRD_MODEL_* (the ramp model needs n_seg = 4); obs_series is
 * 1 or 3; each problem's blocks lie inside [0, len) of their arrays
 * (obs blocks are obs_series x (W+1) long) and particle ranges inside
 * [0, total_particles).  Pure host code.  Returns SIRD_OK or SIRD_EINVAL. */
int sird_problem_validate(const sird_problem *probs, int n_prob, int64_t total_particles,
                          int64_t theta_len, int64_t obs_len, int64_t traj_len,
                          int64_t box_len, int obs_series);

/* Build the tile table of a problem table: ceil(n_part/64) tiles per
 * problem, ordered by decreasing W*steps_per_day (longest first, so that
 * dispatch order is a longest-processing-time schedule), ties by problem and
 * first particle.  Writes at most max_tiles entries to tiles_out (host) and
 * returns the tile count, or a negative status (SIRD_ENOSPACE if max_tiles is
 * too small, SIRD_EINVAL for a bad table).  Pure host code. */
int sird_plan_tiles(const sird_problem *probs, int n_prob, sird_tile *tiles_out,
                    int max_tiles);

/* Pair the tiles of a tile table (as sird_plan_tiles orders them) for
 * two particles per lane: a problem's tiles 0 and 1, 2 and 3, ... form a
 * pair, an odd last tile stands alone; writes the first tile of each pair,
 * in table order (longest first stays longest first), to pairs_out (host)
 * and returns the pair count, or SIRD_ENOSPACE if max_pairs is too small,
 * SIRD_EINVAL for a bad table.  Pure host code. */
int sird_plan_pairs(const sird_tile *tiles, int n_tiles, int32_t *pairs_out, int max_pairs);

/* Fill the scalar fields of *batch from a host problem table (validated as
 * in sird_problem_validate) and the given device pointers.  traj_len may be
 * 0 if sird_integrate is not used.  block, persistent, waves_per_simd,
 * dtype, ppl, n_pairs and pair_tiles are left as the caller set them.  Pure
 * host code. */
int sird_batch_plan(sird_batch *batch, const sird_problem *probs_host, int n_prob,
                    int64_t total_particles, int64_t theta_len, int64_t obs_len,
                    int64_t traj_len, int64_t box_len, int obs_series, int n_tiles,
                    const sird_problem *probs_dev, const sird_tile *tiles_dev,
                    int32_t *sched_dev);

/* ---------------------------------------------------------- device calls */

/* RK4 trajectories (eq. (SIRD), Sec. 2.2) of every particle of every
 * problem: S, I, R, D at days 0..W.
 *   theta: theta-shaped input.
 *   traj:  output, per problem a block [4][W+1][n_part] at traj_off
 *          (compartment, day, particle); traj_len must cover every block.
 * Errors: SIRD_EINVAL for null pointers or a bad batch, SIRD_EHIP. */
int sird_integrate(const sird_batch *batch, const double *theta, double *traj,
                   void *stream);

/* Cost of Sec. 3.1 of every particle: RK4 over the window, the deceased
 * compartment sampled at every day and compared with the observations.
 *   theta: theta-shaped input.
 *   obs:   per problem obs_series x (W+1) observations at obs_off: cumulative
 *          deaths (obs_series = 1), or I, R and cumulative D (3).
 *   loss_kind: one of SIRD_LOSS_* (the IRD kinds need obs_series = 3).
 *   loss:  output, particle-indexed.
 *   ckpt_interval, workspace, ws_bytes: optional.  With workspace NULL
 *          only the losses are computed (ckpt_interval and ws_bytes are
 *          ignored).  With a workspace (at least
 *          sird_loss_backward_workspace(batch, ckpt_interval) bytes,
 *          256-byte aligned) the losses come from the forward pass of the
 *          discrete adjoint, which also saves in the workspace the state
 *          every ckpt_interval steps, the daily deceased counts and the
 *          loss; sird_loss_backward with from_forward = 1 then starts at
 *          the reverse sweep.  This form needs what sird_loss_backward
 *          needs (SIRD_F64, the RK4 model, a deceased-count cost); its
 *          losses equal that call's loss_out bitwise and the workspace-free
 *          losses to rounding (it carries S beside s = (beta/N) S).
 * Errors: SIRD_EINVAL (null pointer, bad kind or batch, a workspace form the
 * adjoint does not support), SIRD_ENOSPACE (workspace too small),
 * SIRD_EHIP. */
int sird_loss(const sird_batch *batch, const double *theta, const double *obs,
              int loss_kind, double *loss, int ckpt_interval, void *workspace,
              size_t ws_bytes, void *stream);

/* Initialise the swarm (Sec. 3.3): x = lo + u (hi - lo) with u from
 * Philox4x64-10 (Salmon et al. 2011) under key (seed, problem.stream) and
 * counter (0, local particle, j/2, 0), word 2*(j%2); v = 0; pbest_x = x;
 * pbest_f = +inf; gbest_x = lo; gbest_f = +inf; gbest_idx = -1; iter = 0.
 * Errors: SIRD_EINVAL (null pointer, bad batch), SIRD_EHIP. */
int pso_init(const sird_batch *batch, const pso_params *params, const pso_state *state,
             void *stream);

/* One swarm iteration (Sec. 3.3) given state->f = loss(state->x) of
 * iteration it = state->iter[0]:
 *   1. personal bests: NaN f counts as +inf; f < pbest_f replaces (f, x);
 *   2. global best per problem: argmin of pbest_f, lowest index on ties,
 *      replacing gbest only on strict improvement; recorded in hist_* row it;
 *   3. velocity and position; dimension j of the d takes slot
 *      s = (j + 3) mod d (gamma, mu, I0 first), and r1, r2 come from word
 *      s%4 of the Philox block with counter (it, local particle, s/4, 1):
 *      r1 its high and r2 its low 32 bits, times 2^-32:
 *        t = w v; t = t + (c1 r1)(pbest - x); t = t + (c2 r2)(gbest - x);
 *        v = t;   x = min(max(x + v, lo), hi)
 *      each operation a single rounded IEEE multiply or add (no fusion);
 *   4. iter[0] = it + 1.
 * Errors: SIRD_EINVAL (null pointer, bad batch), SIRD_EHIP. */
int pso_step(const sird_batch *batch, const pso_params *params, const pso_state *state,
             void *stream);

/* The two halves of a swarm iteration with the swarm update fused into the
 * integration (Sec. 3.3).  pso_evaluate: if move_first, first complete the
 * previous iteration's velocity/position update (counter iter[0] - 1,
 * operations as in pso_step step 3; for the RK4 model the kernel moves
 * Philox block 0 before integrating and the later blocks of betas as the
 * integration reaches them, with the same result); then integrate every
 * particle and write state->f = loss(state->x) as sird_loss does; then
 * update the personal bests as in pso_step step 1.  pso_gbest: pso_step step 2 for
 * iteration it = iter[0] (global best, history row it), then iter[0] = it+1.
 * The sequence
 *     pso_evaluate(0); pso_gbest; { pso_evaluate(1); pso_gbest; } x (n-1);
 *     pso_complete_move
 * is bitwise n x [sird_loss; pso_step].
 * Errors: SIRD_EINVAL (null pointer, bad kind or batch), SIRD_EHIP. */
int pso_evaluate(const sird_batch *batch, const pso_params *params, const pso_state *state,
                 const double *obs, int loss_kind, int move_first, void *stream);
int pso_gbest(const sird_batch *batch, const pso_params *params, const pso_state *state,
              void *stream);

/* The velocity/position update of the last finished iteration (counter
 * iter[0] - 1), without advancing iter: ends a pso_evaluate/pso_gbest
 * sequence so that the swarm state equals the one pso_step leaves. */
int pso_complete_move(const sird_batch *batch, const pso_params *params,
                      const pso_state *state, void *stream);

/* n_iters iterations of [sird_loss(state->x) -> state->f; pso_step], the
 * whole hot path of one calibration iteration, enqueued as the fused
 * pso_evaluate / pso_gbest sequence above (same result bitwise). */
int sird_pso_iterate(const sird_batch *batch, const pso_params *params,
                     const pso_state *state, const double *obs, int loss_kind,
                     int n_iters, void *stream);

/* ckpt_interval of the segment-parallel reverse sweep (sird_loss,
 * sird_loss_backward, sird_loss_backward_workspace,
 * sird_loss_backward_static).  The forward pass checkpoints every day start;
 * the reverse sweep then runs every beta segment of every parameter vector
 * at once (one wavefront per tile and segment) as an affine map of the
 * adjoint of (S, I) at the segment's end, three adjoints walked through the
 * segment's steps, and chains the segments' maps per vector.  Three times the
 * reverse work of the sequential sweep, in K times as many wavefronts: for
 * batches too small to fill the GPU (a refinement on a few thousand vectors),
 * where it shortens the call's latency.  The gradient equals the sequential
 * sweep's up to rounding (not bitwise); the losses are the same. */
#define SIRD_CKPT_SEGMENTS (-1)

/* Gradient of the cost with respect to theta by the discrete adjoint of the
 * RK4 scheme (reverse mode through every stage).  The forward pass stores
 * the state every ckpt_interval steps in the workspace; the reverse sweep
 * recomputes each interval from its checkpoint.  The result does not depend
 * on ckpt_interval >= 0 (bitwise).
 *   grad_loss: optional particle-indexed upstream gradient (NULL = 1).
 *   grad_theta: output, theta-shaped: grad_loss[p] * dL/dtheta.
 *   loss_out: optional particle-indexed output of the loss itself.
 *   ckpt_interval: steps between checkpoints.  The reverse sweep replays
 *       an interval from its checkpoint into the wavefront's LDS slice,
 *       which holds lc steps (40 KiB per wavefront less the observations
 *       and the lane's betas; 8 <= lc <= 64), and walks it backwards; a
 *       longer interval is split into lc-step pieces whose start states go
 *       to the workspace first.  0 = per problem, the whole days that fit
 *       lc steps (lc steps when one day is longer), so that every interval
 *       is replayed once and its checkpoints fall on day starts.
 *       SIRD_CKPT_SEGMENTS: the segment-parallel reverse sweep above.
 *   from_forward: 0 = run the forward pass here (contents of the workspace
 *       on entry are ignored); 1 = the workspace holds the forward pass of
 *       a sird_loss call with a workspace on the same batch, theta, obs,
 *       loss_kind and ckpt_interval, and only the reverse sweep runs (the
 *       gradient is bitwise that of from_forward = 0; the saved forward
 *       stays valid, so the call may be repeated, e.g. with another
 *       grad_loss).
 *   workspace: device scratch of at least
 *       sird_loss_backward_workspace(batch, ckpt_interval) bytes, 256-byte
 *       aligned.
 * The deceased-count costs are piecewise smooth: MXSE takes the first day
 * attaining the maximum, MAE/MAPE take sign(0) = 0.
 * Errors: SIRD_EINVAL, SIRD_ENOSPACE (workspace too small), SIRD_EHIP.
 * Only SIRD_F64 batches of the RK4 model with a D-only cost are supported
 * (SIRD_EINVAL otherwise). */
int sird_loss_backward(const sird_batch *batch, const double *theta, const double *obs,
                       int loss_kind, const double *grad_loss, double *grad_theta,
                       double *loss_out, int ckpt_interval, int from_forward,
                       void *workspace, size_t ws_bytes, void *stream);

/* Workspace bytes needed by sird_loss_backward (0 on a bad batch). */
size_t sird_loss_backward_workspace(const sird_batch *batch, int ckpt_interval);

/* Bytes of the device scratch behind sird_loss_backward_static (64 MiB per
 * GPU the library runs on, held until the process ends). */
#define SIRD_STATIC_SCRATCH_BYTES (64u << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * self-contained sird_loss_backward (from_forward = 0) with its workspace in
 * a library-owned static device array of SIRD_STATIC_SCRATCH_BYTES, one per
 * GPU.  Same arguments, meaning and result (bitwise) as sird_loss_backward
 * without workspace, ws_bytes and from_forward; the caller still owns theta,
 * obs, grad_loss, grad_theta and loss_out.  The call allocates nothing; its
 * first call on a device, made with that device current, looks up that
 * device's array.  Every call on one GPU shares that GPU's array (its
 * contents on entry are not read), so calls that overlap on one GPU race:
 * order them on one stream.
 * Errors: as sird_loss_backward; SIRD_ENOSPACE when
 * sird_loss_backward_workspace(batch, ckpt_interval) exceeds
 * SIRD_STATIC_SCRATCH_BYTES (nothing is enqueued). */
int sird_loss_backward_static(const sird_batch *batch, const double *theta, const double *obs,
                              int loss_kind, const double *grad_loss, double *grad_theta,
                              double *loss_out, int ckpt_interval, void *stream);

/* Indices (local to each problem) of the k particles with the smallest
 * pbest_f, ordered by (pbest_f, index), NaN last.  idx_out: device [n_prob][k];
 * problems with fewer than k particles pad with -1.  Up to k = 32 the
 * selection takes k rounds over each problem; above it every particle's
 * rank is counted (O(n^2) comparisons per problem of n particles).
 * Errors: SIRD_EINVAL (k < 1 or k > 65536, null pointer), SIRD_EHIP. */
int pso_topk(const sird_batch *batch, const double *pbest_f, int k, int64_t *idx_out,
             void *stream);

/* Gather columns of a theta-shaped source array into the theta-shaped
 * array of another batch: dst problem r, particle q takes source problem r,
 * local particle idx[r*k + q] (q < k, dst n_part == k for every problem,
 * same d); idx -1 copies the source box lower bound lo.
 * Errors: SIRD_EINVAL, SIRD_EHIP. */
int sird_gather(const sird_batch *src, const double *src_theta, const double *src_lo,
                const sird_batch *dst, double *dst_theta, const int64_t *idx, int k,
                void *stream);

/* One projected Adam step (Kingma & Ba 2015) on every particle, in
 * box-normalised coordinates u = (theta - lo)/(hi - lo) (lo, hi box-shaped):
 *   g_u = grad (hi - lo); m = b1 m + (1-b1) g_u; v = b2 v + (1-b2) g_u^2;
 *   u = clamp(u - lr (m/(1-b1^t)) / (sqrt(v/(1-b2^t)) + eps), 0, 1);
 *   theta = lo + u (hi - lo).   Dimensions with hi == lo are left alone.
 * theta, grad, m, v: theta-shaped.  t >= 1 is the step number.
 * Errors: SIRD_EINVAL, SIRD_EHIP. */
int sird_adam_step(const sird_batch *batch, double *theta, const double *grad, double *m,
                   double *v, const double *lo, const double *hi, int64_t t,
                   const adam_params *params, void *stream);

/* State of projected L-BFGS refinement (all device memory, caller-owned).
 * theta-shaped: theta, grad; particle-indexed: f, alpha, gp, count, head;
 * S and Y: m theta-shaped arrays back to back ([m][theta_len]); rho:
 * [m][total_particles].  The trial points: theta_t and grad_t are T
 * theta-shaped arrays back to back ([T][theta_len]), f_t T particle-indexed
 * ones ([T][total_particles]), T = max(n_trials, 1); trial t of every
 * vector is the t-th block (a batch whose problems are the batch's own
 * repeated T times, trial-major, with theta and particle offsets shifted
 * by t theta_len and t total_particles, evaluates all trials in one
 * sird_loss_backward call).  Start with count = head = 0, alpha = 1, f and
 * grad evaluated at theta. */
typedef struct lbfgs_state {
    double *theta;
    double *grad;
    double *f;
    double *theta_t;
    double *grad_t;
    double *f_t;
    double *S;
    double *Y;
    double *rho;
    double *alpha;
    double *gp;
    int32_t *count;
    int32_t *head;
    int32_t m;        /* pairs kept, 1..32 */
    int32_t log_last; /* 1: the last parameter (I0) is optimised as log I0
                         in [log lo, log hi] (requires lo > 0) */
    int32_t n_trials; /* trial points per round, 0..8 (0 means 1) */
} lbfgs_state;

/* Projected L-BFGS (Liu & Nocedal 1989, two-loop recursion of Nocedal 1980)
 * in box-normalised coordinates u = (theta - lo)/(hi - lo) (for the last
 * parameter u = (log theta - log lo)/(log hi - log lo) when log_last: I0
 * spans decades, and linear scaling would make its curvature dwarf the
 * others'), one round in two
 * halves around a caller's evaluation of (f_t, grad_t) at theta_t (e.g. by
 * sird_loss_backward):
 *   propose: r = H g_u from the stored pairs (initial H = (s.y/y.y) I of the
 *     newest pair, I when none); p = -r with fixed dimensions and components
 *     pushing past an active bound zeroed; if g_u.p >= 0 the memory is
 *     dropped and p = -g_u; without stored pairs alpha is capped so that
 *     max |alpha p| <= 0.01; trial t = 0..T-1 at the step a_t = alpha 2^t:
 *     theta_t[t] = lo + clamp(u + a_t p, 0, 1)(hi - lo); gp = g_u.p.
 *   accept: among the trials with finite f_t[t] <= f + c1 a_t gp, keep the
 *     one of lowest f_t (the first on ties): store the pair (u_t - u,
 *     g_u,t - g_u) when s.y > 0, alpha = 1; with none, halve alpha (below
 *     1e-20: drop the memory, alpha = 1).  T = 1 is backtracking by
 *     halving; more trials try longer steps in the same evaluation.
 * Parameter vectors are independent; d <= 64.
 * Errors: SIRD_EINVAL (null pointer, m outside 1..32, c1 outside (0,1),
 * log_last not 0/1, n_trials outside 0..8), SIRD_EHIP. */
int sird_lbfgs_propose(const sird_batch *batch, const lbfgs_state *state, const double *lo,
                       const double *hi, void *stream);
int sird_lbfgs_accept(const sird_batch *batch, const lbfgs_state *state, const double *lo,
                      const double *hi, double c1, void *stream);

/* Capture iters_per_launch iterations of sird_pso_iterate into a HIP graph
 * (captured on an internal stream; no memset nodes).  Every array the
 * iterations touch must stay allocated while the graph exists; the swarm
 * iteration counter lives in device memory so replays continue the run.
 * *graph_out receives an opaque handle.
 * Errors: SIRD_EINVAL, SIRD_EHIP. */
int sird_graph_create(const sird_batch *batch, const pso_params *params,
                      const pso_state *state, const double *obs, int loss_kind,
                      int iters_per_launch, void **graph_out);

/* Launch a captured graph n_launches times on stream. */
int sird_graph_launch(void *graph, int n_launches, void *stream);

/* Release a captured graph (NULL is accepted). */
int sird_graph_destroy(void *graph);

#ifdef __cplusplus
}
#endif

#endif /* SIRD_H */
