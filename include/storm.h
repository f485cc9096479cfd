/*
 * storm.h - C ABI of the MI355X (gfx950) STORM MPPI library.
 *
 * One MPC iteration of STORM (arXiv 2104.13542): sample N control sequences
 * (Sec. 3.3), integrate each over H steps (Sec. 3.1, Eq. 7), evaluate forward
 * kinematics and the Jacobian (Eq. 8), the running cost (Sec. 3.2, Eq. 9-15)
 * and the horizon cost (Eq. 2), then update the Gaussian policy with
 * exponentiated-cost weights (Eq. 4-6), emit the next command and shift the
 * mean (Alg. 1).
 *
 * Conventions for every call:
 *   - Every function returns a storm_status (0 = success, < 0 = error).
 *   - Arguments named h_* or passed inside structs at init are host memory;
 *     the library copies them and never touches them after the call returns.
 *   - Arguments named d_* are device memory owned by the caller.  They must
 *     stay valid until the work enqueued on `stream` has completed.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Calls
 *     that enqueue work (step, update, grad, batch_*) allocate nothing and do
 *     not synchronise, so they can be captured into a HIP graph.
 *   - Validation errors are reported before anything is enqueued.  A HIP
 *     launch failure returns STORM_E_DEVICE and makes that context sticky:
 *     later calls on it return STORM_E_DEVICE.
 *   - One context is used from one stream at a time; contexts are not
 *     thread-safe.  Data are FP32.
 *
 * Layouts (all contiguous, FP32):
 *   x0     [3][7]        q0, v0, a0 (joint position, velocity, acceleration)
 *   goal   [12]          goal rotation R_g (row-major 3x3), then position p_g
 *   mean   [H][7]        Gaussian means of the controls (joint accelerations)
 *   sigma2 [7]           per-joint control variance (shared over the horizon);
 *          [H][7]        per step and joint with storm_params.cov_per_step
 *   noise  [7][N][H]     standard-normal override (joint, particle, step)
 *   u, q, v, a [7][N][H] controls and states (joint, particle, step)
 *   c      [N][H]        running cost; terms [8][N][H] unweighted terms in the
 *                        order pos, rot, joint, vel, stop, manip, self, env
 *   C      [N]           horizon cost per particle
 */
#ifndef STORM_H
#define STORM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define STORM_DOF 7
#define STORM_NFRAMES 8
#define STORM_MAX_HORIZON 64
#define STORM_MAX_SPHERES 64
#define STORM_MAX_OBSTACLES 256
#define STORM_MAX_PARTICLES (1 << 20)
#define STORM_OBSTACLE_STRIDE 16
#define STORM_NTERMS 9
#define STORM_SELF_MLP_SIZE 45057

/* Status codes. */
#define STORM_OK 0
#define STORM_E_NULL (-1)        /* a required pointer is NULL */
#define STORM_E_RANGE (-2)       /* a size is out of range (N, H, K, spheres, obstacles) */
#define STORM_E_PARAM (-3)       /* a parameter is invalid (beta <= 0, dt <= 0, alpha outside [0,1], NaN) */
#define STORM_E_DEVICE (-4)      /* a HIP call failed; the context is unusable */
#define STORM_E_STATE (-5)       /* calls out of order (update without a step, ...) */
#define STORM_E_NOMEM (-6)       /* device allocation failed */
#define STORM_E_UNSUPPORTED (-7) /* valid request the library does not implement */

/* Cost-term switches for the running cost (Sec. 3.2, Eq. 15). */
#define STORM_COST_POSE (1u << 0)  /* Eq. 9 */
#define STORM_COST_JOINT (1u << 1) /* Eq. 11 on positions */
#define STORM_COST_VEL (1u << 2)   /* Eq. 11 form on velocities */
#define STORM_COST_STOP (1u << 3)  /* Eq. 10 */
#define STORM_COST_MANIP (1u << 4) /* Eq. 12 */
#define STORM_COST_SELF (1u << 5)  /* Eq. 13, as sphere-pair penetration */
#define STORM_COST_ENV (1u << 6)   /* Eq. 14, as sphere vs obstacle signed distance */
#define STORM_COST_ALL 0x7Fu       /* the reaching task's terms above */
/* The ball on the tray (appendix on dynamic object balancing): the ball's
 * distance from the tray centre in the tray plane, along its trajectory
 * under in-plane gravity (storm_rollout_set_ball).  Plain contexts only. */
#define STORM_COST_BALL (1u << 7)

/* Asynchronous device status flags (storm_rollout_status). */
#define STORM_FLAG_NONFINITE_COST (1u << 0) /* some C_i was NaN/Inf: update kept mu, sigma2 */
#define STORM_FLAG_ZERO_WEIGHT (1u << 1)    /* weight sum not positive: update kept mu, sigma2 */

/* Obstacle record kinds (first value of each 16-float record). */
#define STORM_OBSTACLE_SPHERE 0 /* [0, cx, cy, cz, r, -, -, ...] */
#define STORM_OBSTACLE_CUBOID 1 /* [1, cx, cy, cz, ex, ey, ez, R00..R22]: half extents, box-to-world R */

/* Parameters of one MPC problem.  Sec. 2-3 name N, H, K, dt, beta, gamma and
 * the step sizes; Sec. 3.2 the cost weights and thresholds; Sec. 3.3 the
 * sampling strategy.  Particles [0, n_halton) use the Halton + cubic
 * B-spline table (drawn once at init), [n_halton, n_particles - n_null) use
 * Philox4x32-10 Gaussian noise, and the last n_null particles are
 * zero-acceleration ("null") sequences. */
typedef struct storm_params {
    int32_t n_particles; /* N, 1 .. STORM_MAX_PARTICLES */
    int32_t horizon;     /* H, 1 .. STORM_MAX_HORIZON */
    int32_t n_halton;    /* 0 .. N - n_null */
    int32_t n_null;      /* 0 .. N */
    int32_t n_knots;     /* B-spline control points K, 4 .. 32 (ignored if n_halton = 0) */
    uint32_t cost_mask;  /* STORM_COST_* */
    uint64_t seed;       /* Philox key */
    const float *dt;     /* host [H], each > 0 */
    float sigma_init[STORM_DOF]; /* initial per-joint standard deviation, > 0 */
    float beta;          /* temperature of Eq. 3/6, > 0 */
    float gamma;         /* discount of Eq. 2, in [0, 1] */
    float alpha_mu;      /* mean step size of Eq. 4, in [0, 1] */
    float alpha_sigma;   /* covariance step size of Eq. 5, in [0, 1] */
    float w_term;        /* terminal-step scale (terminal cost = running cost), >= 0 */
    float sigma2_min;    /* variance floor, >= 0 */
    float acc_stop;      /* maximum acceleration of the stop cost (Eq. 10), >= 0 */
    float k_jl;          /* joint-limit safety ratio (Eq. 11), in [0, 0.5) */
    float k_vl;          /* velocity-limit safety ratio, in [0, 0.5) */
    float k_m;           /* manipulability threshold (Eq. 12) */
    float w_pos, w_rot;  /* pose weights (position, orientation) of alpha_p */
    float alpha_pos[3];  /* goal-frame axis weights of the position error (Eq. 9 alpha_2) */
    float alpha_rot[3];  /* row weights of the rotation error (Eq. 9 alpha_1) */
    float a_stop, a_joint, a_vel, a_manip, a_coll; /* Eq. 15 weights */
    uint32_t grad_mask;  /* terms of the differentiable form (storm_rollout_grad / refine): a subset of
                            POSE | JOINT | VEL | STOP; 0 = cost_mask, which must then be such a subset */
    int32_t comb_filter; /* 1: the comb filter of Sec. 3.3 smooths the noise of the Gaussian (Philox)
                            particles along the horizon, per joint, in step order:
                            e'_h = comb[0] e_h + comb[1] e'_{h-1} + comb[2] e'_{h-2}, e'_{-1} = e'_{-2} = 0,
                            and u = mu + sigma e'.  With n_halton = 0.6 N this is the paper's "mixed"
                            sampling (B-spline and comb particles).  Halton particles, null particles and
                            a noise override are not filtered.  0: no filter */
    float comb[3];       /* comb filter coefficients c1, c2, c3, finite */
    int32_t cov_per_step; /* 1: Eq. 5 as printed, per step: a diagonal variance per (step, joint),
                             sigma2 [H][7], each updated from the weighted deviations at its step; the
                             shift moves it forward one step with sigma_init^2 appended.  0: the
                             per-joint variance shared over the horizon (Sec. 3.3 parameterisation),
                             sigma2 [7], which the shift leaves as it is */
    /* Ball on the tray (STORM_COST_BALL).  The tray plane is the flange
       frame's x-y plane.  The ball's state at the current arm state (world
       frame, storm_rollout_set_ball) is moved into the flange frame of
       FK(q0) (its z velocity set to 0); at step h its acceleration is the
       in-plane part of g in the flange frame of the rolled-out state,
       integrated with the scheme of Eq. 7.  Term = distance of the ball
       from ball_center in the plane, weighted by w_ball. */
    float w_ball;          /* >= 0, finite */
    float ball_gravity[3]; /* world frame, m/s^2, finite */
    float ball_center[2];  /* tray centre (x, y) in the flange frame, finite */
    /* Self-collision model of STORM_COST_SELF (Sec. 3.2, Eq. 13).  0: sphere
       pairs, the term being the largest penetration.  1: the learned network
       (the paper's jointNERF form) whose parameters storm_robot.self_mlp
       holds: the term is max(0, d) for its predicted distance d, evaluated
       by a kernel after the rollout on the matrix cores: FP16 weights, each
       activation carried as a pair of FP16 values (hi, lo) and FP32
       accumulation, which gives d to FP32 rounding.  Plain contexts only. */
    int32_t self_model;
} storm_params;

/* Serial-chain robot: modified (Craig) Denavit-Hartenberg frames 1..8, frame
 * 8 being the end-effector flange (theta = 0).  Row k of dh holds
 * (a_{k-1}, d_k, alpha_{k-1}).  Spheres rows: (body 1..8, x, y, z, r) in the
 * body frame, sorted by body, 0 < r < 1 m; self-collision checks pairs on
 * bodies at least two apart. */
typedef struct storm_robot {
    float dh[STORM_NFRAMES][3];
    float q_min[STORM_DOF], q_max[STORM_DOF]; /* joint position limits */
    float qd_max[STORM_DOF];                  /* joint speed limits */
    int32_t n_spheres;                        /* 0 .. STORM_MAX_SPHERES */
    const float *spheres;                     /* host [n_spheres][5] */
    /* Learned self-collision network (used with storm_params.self_model = 1;
       may be NULL otherwise): host [STORM_SELF_MLP_SIZE] finite floats, copied
       at init; the weight matrices W1, W2 and W3 must hold values that FP16
       represents exactly (else init returns STORM_E_PARAM).  Input [sin q_1..7, cos q_1..7], ReLU layers of 256, 128 and
       64 units, one linear output; in order W1 [256][14], b1 [256],
       W2 [128][256], b2 [128], W3 [64][128], b3 [64], w4 [64], b4 (weight
       matrices [out][in]). */
    const float *self_mlp;
} storm_robot;

/* Static scene: obstacle records of STORM_OBSTACLE_STRIDE floats. */
typedef struct storm_scene {
    int32_t n_obstacles;     /* 0 .. STORM_MAX_OBSTACLES */
    const float *obstacles;  /* host [n_obstacles][16] */
} storm_scene;

/* Optional per-step outputs (each pointer nullable, device memory). */
typedef struct storm_debug {
    float *u, *q, *v, *a; /* [7][N][H] */
    float *c;             /* [N][H] */
    float *terms;         /* [9][N][H]: pos, rot, joint, vel, stop, manip, self, env, ball */
    float *xd, *xdd;      /* [6][N][H]: flange velocity and acceleration in the world frame (Eq. 8),
                             linear x, y, z then angular x, y, z: xd = J(q) qd, xdd = Jdot qd + J qdd */
} storm_debug;

typedef struct storm_ctx_s *storm_ctx;

/* Create a context for one problem (Alg. 1 set-up).  Copies params, robot and
 * scene; allocates all device workspace; builds the dt, stop-velocity,
 * horizon-weight and limit tables and the Halton + B-spline noise table on
 * the device; sets mu = 0, sigma2 = sigma_init^2 and the step counter to 0.
 * Synchronises `stream` before returning.  Not capturable.
 * Errors: E_NULL, E_RANGE, E_PARAM, E_NOMEM, E_DEVICE. */
int32_t storm_rollout_init(storm_ctx *out, const storm_params *params, const storm_robot *robot,
                           const storm_scene *scene, void *stream);

/* Sample + roll out (Alg. 1 sample_controls and generate_rollouts): controls
 * u = mu + sigma * eps (Sec. 3.3), triple integrator (Eq. 7), FK and
 * Jacobian (Eq. 8), running cost (Eq. 9-15) and horizon cost (Eq. 2).
 * d_x0 [3][7] and d_goal [12] are read on the device.  d_noise (nullable)
 * replaces the sampled standard noise of every non-null particle.  d_C
 * (nullable) receives a copy of C [N].  dbg (nullable) selects extra
 * outputs; asking for xd / xdd (or a problem with the ball term or the
 * learned self-collision model) runs the task-space form of the rollout,
 * which carries that extra work.  A second step before the update replaces
 * the first one's controls and costs.  Errors: E_NULL, E_DEVICE. */
int32_t storm_rollout_step(storm_ctx ctx, const float *d_x0, const float *d_goal, const float *d_noise,
                           const storm_debug *dbg, float *d_C, void *stream);

/* Policy update (Alg. 1 update_distribution, Eq. 4-6) from the last step,
 * then next_command: d_cmd [7] = updated mu_0, written by the update kernel
 * to device memory or to pinned host memory (hipHostMalloc; readable on the
 * host once `stream` has synchronised, with no copy).  d_mean [H][7] and d_sigma2
 * ([7], or [H][7] with cov_per_step; nullable) receive the updated
 * (unshifted) mean and variance.  With shift != 0 the stored mean is shifted
 * one step and a zero mean appended (the warm start of the next control
 * step), and a per-step variance likewise with sigma_init^2 appended;
 * otherwise they are stored as they are (for K > 1 iterations).  Non-finite costs or a zero weight sum keep mu and
 * sigma2 and raise a status flag.  Increments the sampling step counter.
 * Errors: E_NULL (d_cmd), E_STATE (no step since the last update), E_DEVICE. */
int32_t storm_rollout_update(storm_ctx ctx, float *d_mean, float *d_sigma2, float *d_cmd, int32_t shift,
                             void *stream);

/* Free everything (synchronises the context's device first).  NULL is a no-op. */
int32_t storm_rollout_destroy(storm_ctx ctx);

/* Read and clear the asynchronous status flags (STORM_FLAG_*).  Synchronises
 * `stream`; not for the hot loop. */
int32_t storm_rollout_status(storm_ctx ctx, uint32_t *h_flags, void *stream);

/* Read the policy state to host memory (mean [H][7], sigma2 [7] or [H][7]
 * with cov_per_step, step counter); any pointer may be NULL.  Synchronises
 * `stream`. */
int32_t storm_rollout_get_state(storm_ctx ctx, float *h_mean, float *h_sigma2, uint32_t *h_step, void *stream);

/* Restore the policy state from host memory (NULL pointers leave that part
 * unchanged; sigma2 as in get_state, finite and >= 0).  Clears a pending
 * step.  Synchronises `stream`. */
int32_t storm_rollout_set_state(storm_ctx ctx, const float *h_mean, const float *h_sigma2, const uint32_t *h_step,
                                void *stream);

/* The ball's state at the current arm state for the ball term (appendix on
 * dynamic object balancing): d_ball [6] = position (m) and velocity (m/s)
 * in the world frame, device memory, copied on `stream` into the context
 * and read by every later storm_rollout_step (and graph launch) until the
 * next call.  A new context holds zeros.  Capturable.  Errors: E_NULL,
 * E_DEVICE. */
int32_t storm_rollout_set_ball(storm_ctx ctx, const float *d_ball, void *stream);

/* Gradient of the expected horizon cost (the differentiable form; not in
 * the paper): J(mu) = (1/N) sum_i C_i(mu + sigma * eps_i) with the standard
 * noise eps of the last storm_rollout_step held fixed (or d_noise [7][N][H]
 * if not NULL), sigma the current per-joint standard deviation, and C_i the
 * horizon cost (Eq. 2) of the terms in params.grad_mask (else cost_mask)
 * among pose (Eq. 9), joint / velocity limit (Eq. 11) and stop (Eq. 10).
 * Null particles add to J but not to the gradient.  Reverse mode through
 * the costs, the kinematics (Eq. 8) and the integrator (Eq. 7), states
 * recomputed.  d_mean [H][7] in, d_grad [H][7] and d_J [1] out (each
 * nullable).  Errors: E_NULL (x0, goal, mean), E_UNSUPPORTED (grad_mask 0
 * and a cost mask with manipulability or collision terms), E_DEVICE. */
int32_t storm_rollout_grad(storm_ctx ctx, const float *d_x0, const float *d_goal, const float *d_mean,
                           const float *d_noise, float *d_grad, float *d_J, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * gradient and expected cost as storm_rollout_grad, same arguments, layout
 * and errors, bitwise equal results, but the adjoint's per-chunk partial
 * sums go to a static scratch array of the library (0.9 MB per device,
 * [512][7][64] + [512] floats, enough for every context; its device address
 * is looked up once per device by storm_rollout_init) instead of the
 * context's buffers.  Allocates nothing.  Every call on one device shares
 * that device's array: calls that may overlap on one device (other streams,
 * other threads, other contexts) race and must be ordered by the caller.
 * E_RANGE if a context's partials would not fit (cannot happen for contexts
 * storm_rollout_init accepts). */
int32_t storm_rollout_grad_noalloc(storm_ctx ctx, const float *d_x0, const float *d_goal, const float *d_mean,
                                   const float *d_noise, float *d_grad, float *d_J, void *stream);

/* Gradient refinement of the stored mean (the differentiable form):
 * `iterations` Adam steps (Kingma and Ba 2015: beta1 0.9, beta2 0.999,
 * eps 1e-8, moments restarted at each call) of learning rate lr on J above,
 * then d_cmd [7] = refined mu_0 and, if shift != 0, the warm-start shift.
 * Meant to follow storm_rollout_update(..., shift = 0).  Allocates nothing.
 * Errors: E_NULL, E_RANGE (iterations < 0), E_PARAM (lr not finite or < 0),
 * E_UNSUPPORTED, E_DEVICE. */
int32_t storm_rollout_refine(storm_ctx ctx, const float *d_x0, const float *d_goal, int32_t iterations, float lr,
                             float *d_cmd, int32_t shift, void *stream);

/* One whole control step of Alg. 1 in a single call, launched eagerly:
 * `iterations` (K >= 1) rounds of storm_rollout_step + storm_rollout_update
 * on `stream`, the shift applied after the last round only, reading d_x0
 * [3][7] and d_goal [12] (device memory) and writing d_cmd [7] (device or
 * pinned host memory, as in storm_rollout_update).  Enqueues
 * exactly the kernels a graph of storm_rollout_graph_create would, with one
 * crossing of the interface per control step instead of 2K, and leaves no
 * step pending.  Allocates nothing.  Errors: E_NULL, E_RANGE
 * (iterations < 1), E_DEVICE. */
int32_t storm_rollout_control(storm_ctx ctx, const float *d_x0, const float *d_goal, float *d_cmd,
                              int32_t iterations, int32_t shift, void *stream);

/* Opaque handle of an instantiated HIP graph of one control step. */
typedef struct storm_graph_s *storm_graph;

/* Capture one whole control step of Alg. 1 into a HIP graph: `iterations`
 * (K >= 1) rounds of storm_rollout_step + storm_rollout_update, the shift
 * applied after the last round only, reading d_x0 [3][7] and d_goal [12]
 * and writing d_cmd [7] (device buffers, d_cmd also pinned host memory as
 * in storm_rollout_update, whose addresses are baked into the
 * graph: refresh their contents before each launch).  `stream` is used for
 * the capture (NULL: a private stream); the context must not be used on
 * any other stream during the call.  Each launch advances the sampling step
 * counter like the eager calls.  Errors: E_NULL, E_RANGE (iterations < 1),
 * E_DEVICE. */
int32_t storm_rollout_graph_create(storm_ctx ctx, const float *d_x0, const float *d_goal, float *d_cmd,
                                   int32_t iterations, int32_t shift, void *stream, storm_graph *out);

/* As storm_rollout_graph_create, followed by `refine_iters` Adam steps of
 * storm_rollout_refine (learning rate lr) before the command and shift. */
int32_t storm_rollout_graph_create_refine(storm_ctx ctx, const float *d_x0, const float *d_goal, float *d_cmd,
                                          int32_t iterations, int32_t shift, int32_t refine_iters, float lr,
                                          void *stream, storm_graph *out);

/* Enqueue one captured control step on `stream`.  Allocates nothing.
 * Errors: E_NULL, E_DEVICE. */
int32_t storm_rollout_graph_launch(storm_graph graph, void *stream);

/* Free a captured graph (NULL is a no-op). */
int32_t storm_rollout_graph_destroy(storm_graph graph);

/* ------------------------------------------------------------------------
 * Batched form: many independent problems (not in the paper).  One
 * persistent rollout launch covers every (problem, tile) work item of all
 * problems through an integer work queue; one update workgroup per problem
 * follows.  Each problem keeps its own parameters, scene, policy state and
 * sampling counter, and computes exactly what a plain context would.
 * ------------------------------------------------------------------------ */
typedef struct storm_batch_s *storm_batch;

/* Launch shape of the persistent rollout. */
typedef struct storm_launch_config {
    int32_t waves;      /* wavefronts per workgroup: 8 or 16 */
    int32_t grid;       /* persistent workgroups, >= 1 */
    int32_t cost_order; /* 1: work queue sorted by estimated tile cost (largest first); 0: problem order */
} storm_launch_config;

/* Create a batch of n_problems problems (params[p], scenes[p]) sharing one
 * robot.  Every per-problem limit and validation rule of storm_rollout_init
 * applies.  Default launch shape: 8 waves, two workgroups per compute unit,
 * cost-ordered queue.  Synchronises `stream`.  Errors: as init, plus E_RANGE
 * for n_problems < 1 and E_UNSUPPORTED for a problem with the ball term or
 * the learned self-collision model. */
int32_t storm_batch_init(storm_batch *out, int32_t n_problems, const storm_params *params,
                         const storm_robot *robot, const storm_scene *scenes, void *stream);

/* Sample + roll out every problem (as storm_rollout_step per problem):
 * d_x0 [P][3][7], d_goal [P][12].  Allocates nothing.  Errors: E_NULL,
 * E_DEVICE. */
int32_t storm_batch_step(storm_batch b, const float *d_x0, const float *d_goal, void *stream);

/* Policy update of every problem (as storm_rollout_update): d_cmd [P][7].
 * Errors: E_NULL, E_STATE (no step since the last update), E_DEVICE. */
int32_t storm_batch_update(storm_batch b, float *d_cmd, int32_t shift, void *stream);

/* Capture one control step of every problem (K rounds of batch step +
 * update, shift after the last) into a HIP graph; launch it with
 * storm_rollout_graph_launch.  Errors as storm_rollout_graph_create. */
int32_t storm_batch_graph_create(storm_batch b, const float *d_x0, const float *d_goal, float *d_cmd,
                                 int32_t iterations, int32_t shift, void *stream, storm_graph *out);

/* As storm_batch_graph_create, followed by `refine_iters` batched Adam steps
 * (storm_batch_refine, learning rate lr) before the commands and the shift.
 * Errors as storm_batch_graph_create, plus E_PARAM (lr) and E_UNSUPPORTED
 * (a problem whose gradient terms are not differentiable). */
int32_t storm_batch_graph_create_refine(storm_batch b, const float *d_x0, const float *d_goal, float *d_cmd,
                                        int32_t iterations, int32_t shift, int32_t refine_iters, float lr,
                                        void *stream, storm_graph *out);

/* Batched gradient refinement (the differentiable form of
 * storm_rollout_refine for every problem at once): `iterations` Adam steps
 * of learning rate lr on each problem's stored mean, with the gradient of its
 * expected horizon cost over the noise of its last step (terms of its
 * grad_mask), computed for all problems by one adjoint launch per step; then
 * d_cmd [P][7] = each refined mu_0 and, if shift != 0, the warm-start shift.
 * Meant to follow storm_batch_update(..., shift = 0).  Allocates nothing.
 * d_x0 [P][3][7], d_goal [P][12].  Errors: E_NULL, E_RANGE (iterations < 0),
 * E_PARAM (lr not finite or < 0), E_UNSUPPORTED, E_DEVICE. */
int32_t storm_batch_refine(storm_batch b, const float *d_x0, const float *d_goal, int32_t iterations, float lr,
                           float *d_cmd, int32_t shift, void *stream);

/* Set / read the persistent launch shape (graphs capture the shape current
 * at their creation).  Errors: E_NULL, E_RANGE (waves not 8/16, grid < 1). */
int32_t storm_batch_set_config(storm_batch b, const storm_launch_config *cfg);
int32_t storm_batch_get_config(storm_batch b, storm_launch_config *cfg);

/* Autotuner: time the rollout of this batch for every candidate shape
 * (waves 8, 16; grid 1-4 workgroups per compute unit; sorted or problem-order
 * queue), `reps` launches each, with HIP events on `stream`, and keep the
 * fastest.  Writes the chosen shape to *best (nullable); if h_times is not
 * NULL it receives the mean time in microseconds of candidate k, k <
 * *n_candidates (capacity in, count out).  The policies are not updated;
 * call storm_batch_step again before the next update.  Synchronises. */
int32_t storm_batch_autotune(storm_batch b, const float *d_x0, const float *d_goal, int32_t reps, void *stream,
                             storm_launch_config *best, float *h_times, int32_t *n_candidates);

/* Per-problem state and costs (host copies, synchronising; not for the hot
 * loop), as the storm_rollout_* calls of a plain context. */
int32_t storm_batch_get_state(storm_batch b, int32_t problem, float *h_mean, float *h_sigma2, uint32_t *h_step,
                              void *stream);
int32_t storm_batch_set_state(storm_batch b, int32_t problem, const float *h_mean, const float *h_sigma2,
                              const uint32_t *h_step, void *stream);
int32_t storm_batch_costs(storm_batch b, int32_t problem, float *h_C, void *stream);

/* Free a batch (NULL is a no-op). */
int32_t storm_batch_destroy(storm_batch b);

/* Closed-loop plant used by the benchmarks: applies command d_cmd [n][7]
 * (device or pinned host memory) to
 * states d_x [n][3][7] for `dt` seconds with the integrator of Eq. 7
 * (v += dt u, q += dt v, a = u).  Errors: E_NULL, E_RANGE (n < 0), E_PARAM
 * (dt <= 0), E_DEVICE. */
int32_t storm_plant_step(float *d_x, const float *d_cmd, int32_t n, float dt, void *stream);

/* Batched forward kinematics of the robot (Sec. 3.1, Eq. 8): for n joint
 * configurations d_q [7][n], writes the flange pose d_pose [12][n] (R
 * row-major, then p) and, if d_manip is not NULL, the manipulability
 * sqrt(det(J J^T)) (Eq. 12) [n].  Errors: E_NULL, E_RANGE (n < 0), E_DEVICE. */
int32_t storm_fk(const storm_robot *robot, const float *d_q, int32_t n, float *d_pose, float *d_manip,
                 void *stream);

/* Human-readable name of a status code (static storage). */
const char *storm_status_str(int32_t status);

#ifdef __cplusplus
}
#endif

#endif /* STORM_H */
