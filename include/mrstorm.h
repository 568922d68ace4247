/* mrstorm.h -- C-ABI of the MI355X (gfx950) MR-STORM control-step library.
 *
 * One call of mpc_step runs one MPC control step for every arm of a scene,
 * as each arm's controller does in the paper's per-arm loop (arXiv
 * 2602.10114, Alg. 1): Sense (current distance to goal and the priority
 * factors of Eq. 10 against every published neighbour plan), Shift, K
 * optimisation iterations of SampleControls -> Rollout (dynamics, forward
 * kinematics over the collision spheres, the stage cost of Eq. 5 extended by
 * the coordination cost of Eqs. 6-9) -> UpdateDistribution (Eqs. 1-4), then
 * ToPlan and PickBest.  mpc_share_plans is the Publish step that makes the
 * plans written by the last mpc_step visible to the other arms.
 *
 * Conventions for every entry point below:
 *  - Arrays passed to mpc_step / mpc_get_plan / mpc_debug_get / mpc_set_plan /
 *    mpc_set_mean / mpc_sim_execute are DEVICE pointers owned by the caller.
 *    They are read or written in stream order on the stream given to
 *    mpc_init; the calls return without waiting for the GPU.
 *  - mpc_init takes HOST descriptors and copies them; the caller may free
 *    them on return.
 *  - The context owns every internal buffer.  One context must not be used
 *    from two threads at the same time.
 *  - All floating-point data is FP32.  Lengths are metres, angles radians.
 *  - Return codes: MPC_OK (0), or a negative MPC_E* code; mpc_last_error
 *    gives the message.  Nothing throws across the ABI, and there is no host
 *    fallback: without a usable gfx950 device mpc_init fails with MPC_EHIP.
 */
#ifndef MRSTORM_H
#define MRSTORM_H

#ifdef __cplusplus
extern "C" {
#endif

#define MPC_OK 0
#define MPC_EINVAL (-1)      /* a size, index or value out of range */
#define MPC_ENOMEM (-2)      /* device allocation failed */
#define MPC_EHIP (-3)        /* HIP runtime error (text in mpc_last_error) */
#define MPC_ESTATE (-4)      /* call not valid in the current state */
#define MPC_EUNSUPPORTED (-5)

#define MPC_MAX_ARMS 8
#define MPC_MAX_DOF 8
#define MPC_MAX_SPHERES 64
#define MPC_MAX_SPHERES_PER_BODY 8
#define MPC_MAX_HORIZON 64
#define MPC_MAX_ROLLOUTS 16384
#define MPC_MAX_OBSTACLES 64

typedef struct mpc_ctx mpc_ctx;

/* One arm (Sec. III: joint state Theta in R^{d x 3}; Sec. IV-A: the sphere
 * matrix S in R^{N_S x 4} at constant transforms from the links).
 * Geometry bounds (MPC_EINVAL otherwise): base within 3 m of the world
 * origin; sum over joints of sqrt(a^2 + d^2), plus |tool|, plus the largest
 * sphere-centre offset, at most 2.6 m; |a|, |d| and each centre coordinate at
 * most 1.5 m; radii in [0, 1] m.  They keep every sphere within 6 m of the
 * origin, the range the FP32 collision filter's slack is sized for. */
typedef struct {
  int dof;                 /* d: revolute joints; this build runs 7-DoF chains only (any other
                              value: MPC_EUNSUPPORTED); MPC_MAX_DOF sizes the tables */
  int n_spheres;           /* N_S: 1..MPC_MAX_SPHERES, at most 8 per body */
  int n_rollouts;          /* N: 1..MPC_MAX_ROLLOUTS (any value; internally padded to 64) */
  int horizon;             /* H: 1..MPC_MAX_HORIZON */
  const float *dh;         /* [dof][4]: a_{k-1}, alpha_{k-1}, d_k, theta offset (modified DH) */
  const float *q_lim;      /* [dof][2]: lower, upper joint limit */
  const float *qd_max;     /* [dof]: joint speed limit used by the stopping cost */
  const float *spheres;    /* [n_spheres][4]: centre in its body frame, radius */
  const int *sphere_link;  /* [n_spheres]: body 0..dof-1 = link frame 1..dof, dof = hand */
  float base[4];           /* base pose in the world: x, y, z, yaw about z */
  float tool[3];           /* end-effector point in the last link frame */
} mpc_arm_desc;

/* Controller parameters shared by all arms (Sec. III-A and Sec. IV; the
 * paper's standard variant uses w_dyn = 5000, buf_dyn = 0.03, tau = 3). */
typedef struct {
  float dt;                /* integration step of the rollout dynamics, s */
  float sigma;             /* sampling standard deviation, Sigma = sigma^2 I */
  float lambda;            /* softmax temperature (Eq. 2) */
  float gamma;             /* discount (Eq. 1) */
  float alpha_mu;          /* mean step size (Eq. 4), in (0, 1] */
  int iters;               /* K optimisation iterations per control step, 1..8 */
  float w_pose, w_rot, w_stop, w_joint, w_coll, w_dyn;  /* cost weights (Eqs. 5, 7, 9) */
  float buf_env, buf_self, buf_dyn;  /* hinge buffers; buf_dyn is B of Sec. IV-A */
  float tau;               /* trust exponent of the priority factor (Eq. 10) */
  float prio_min, prio_max;  /* clamp of the priority factor */
  float dist_floor;        /* floor of the distances in Eq. 10 */
  float joint_margin;      /* soft joint-limit margin */
  unsigned long long seed; /* key of the counter-based noise */
  int max_obstacles;       /* capacity for obstacle spheres per step, <= MPC_MAX_OBSTACLES */
  int collision_mode;      /* 0: exact coordination distances; 1: learned distance with exact fallback */
  float surrogate_margin;  /* mode 1: predictions below this (metres) are checked exactly;
                              0 (= buf_dyn) or >= buf_dyn, else mpc_init fails with MPC_EINVAL */
  float alpha_sigma;       /* covariance step size (Eqs. 3-4), [0, 1]; 0 keeps Sigma = sigma^2 I */
  float sigma_floor;       /* floor of the Cholesky pivots of the adapted Sigma (std. dev. units), > 0 */
  int plan_mode;           /* 0: publish the predicted plan (Sec. IV-A); 1: publish the current
                              spheres at every step, a static obstacle (the paper's S_d ablation) */
  float w_manip;           /* weight of C_manip (Eq. 5), >= 0; 0 leaves the term out */
  float manip_thresh;      /* C_manip = max(0, 1 - sqrt(det(J J^T)) / manip_thresh), > 0 */
  float surrogate_screen;  /* mode 1: an (arm, neighbour, step) whose mean rollout (the means
                              integrated from the sensed state) lies closer than this (metres)
                              to the neighbour's plan at that step is checked exactly for every
                              rollout without running the network (it would keep nearly all of
                              them); >= 0, 0 = off.  Only ever adds exact checks. */
  int surrogate_probe;     /* mode 1: 0 = off, else 2..1000.  An (arm, neighbour, step) group that
                              dropped at most surrogate_min_drop of its 64-rollout checks in the
                              previous control step (at the step one later, which the shift brings
                              to this one) is checked exactly for every rollout without running
                              the network, except on every surrogate_probe-th control step
                              (staggered over the groups), when it runs the network again.
                              History is forgotten when the mode or the network changes.  Only
                              ever adds exact checks. */
  float surrogate_min_drop;  /* share of a group's checks, [0, 1), see surrogate_probe; 0: a group
                              keeps running the network if it dropped any check */
  int pair_cull;           /* 1: the rollout kernel skips sphere pairs that bounding spheres
                              (per body, body half and group of 8 plan spheres, one per wave of
                              64 rollouts) prove farther apart than the hinge buffer; 0: every
                              pair goes through the filter (the all-pairs check, for comparison).
                              Stage costs, controls and plans are bitwise the same either way;
                              any other value is MPC_EINVAL. */
} mpc_params;

/* Create a context for n_arms arms (1..MPC_MAX_ARMS, all with the same dof).
 * hip_stream: a hipStream_t (NULL = the default stream).  Host pointers.
 * The controls' means start at zero (reading of the random initialisation:
 * a deterministic start) and no plan is published. */
int mpc_init(const mpc_arm_desc *arms, int n_arms, const mpc_params *params,
             void *hip_stream, mpc_ctx **out);

/* Publish (Alg. 1): the plans and distances-to-goal that the last mpc_step
 * wrote for the arms in publish_mask (host [n_arms] bytes; NULL = all)
 * become the ones the other arms read at their next Sense.  An arm that never
 * stepped has nothing to publish and stays invisible (Sec. IV-C: neighbours
 * whose plans were never published are ignored). */
int mpc_share_plans(mpc_ctx *c, const unsigned char *publish_mask);

/* One control step for every arm.
 *  state      [n_arms][dof][3] device: theta, theta_dot, theta_ddot per joint
 *  goal       [n_arms][7] device: goal position xyz, goal orientation quaternion w,x,y,z
 *  obstacles  [n_obstacles][4] device: world-frame sphere centre, radius
 *             (radius >= 0: the collision filter's bound assumes it);
 *             held fixed over the horizon (Sec. IV-A); may be NULL if 0
 *  u_out      [n_arms][dof] device: the executed command U* (first step of
 *             the minimum-cost rollout of the last iteration, Sec. III-A Act)
 * Errors: MPC_EINVAL if n_obstacles is outside [0, max_obstacles]. */
int mpc_step(mpc_ctx *c, const float *state, const float *goal, const float *obstacles,
             int n_obstacles, float *u_out);

/* The anticipated plan of one arm as written by the last mpc_step (Sec. IV-A:
 * P in R^{N_S x 4 x H}).
 *  plan    [n_spheres][4][horizon] device (paper layout), or NULL
 *  plan_q  [horizon][dof] device: the planned joint positions, or NULL
 *  mean    [horizon][dof] device: the control means mu after the update, or NULL
 * Errors: MPC_ESTATE before the first mpc_step, MPC_EINVAL for a bad arm. */
int mpc_get_plan(mpc_ctx *c, int arm, float *plan, float *plan_q, float *mean);

/* Release the context (waits for its stream). */
void mpc_destroy(mpc_ctx *c);

/* Message of the last error on c, or of the last failed mpc_init if c is NULL. */
const char *mpc_last_error(const mpc_ctx *c);

/* ---- inspection and test hooks (same conventions) ---- */

/* Block until every call issued on the context's stream has finished. */
int mpc_sync(mpc_ctx *c);

/* Debug capture: when on, every mpc_step also stores the rollout joint
 * states, world-frame spheres, stage costs and the distance-query counter.
 * Allocates the capture buffers on first use. */
int mpc_debug_enable(mpc_ctx *c, int on);

enum {
  MPC_DBG_NOISE = 0,       /* float [horizon][dof][n_rollouts]: eps of the last iteration */
  MPC_DBG_Q = 1,           /* float [n_rollouts][horizon][dof]: rollout joint positions */
  MPC_DBG_QD = 2,          /* float [n_rollouts][horizon][dof]: rollout joint velocities */
  MPC_DBG_SPHERES = 3,     /* float [n_rollouts][horizon][n_spheres][4]: world-frame spheres */
  MPC_DBG_STAGE_COST = 4,  /* float [horizon][n_rollouts]: Eq. 5 + Eq. 9 stage costs */
  MPC_DBG_COST = 5,        /* float [n_rollouts]: discounted totals (Eq. 1) */
  MPC_DBG_WEIGHTS = 6,     /* float [n_rollouts]: softmax weights (Eq. 2) */
  MPC_DBG_MEAN = 7,        /* float [horizon][dof]: mu after the update */
  MPC_DBG_ALPHA = 8,       /* float [n_arms]: priority factors alpha^(arm,i) used at this step (0 = ignored) */
  MPC_DBG_DIST = 9,        /* float [1]: this arm's distance to goal at Sense */
  MPC_DBG_PAIRS = 10,      /* unsigned long long [1]: coordination distance queries evaluated */
  MPC_DBG_ARGMIN = 11,     /* int [1]: index of the executed rollout */
  MPC_DBG_PASSES = 12,     /* unsigned long long [3]: per-wave count of distance filter
                              passes over obstacle/neighbour sets, of exact (FP64) passes
                              over such sets, and of exact self-collision passes */
  MPC_DBG_PRED = 13,       /* float [n_arms][horizon][n_rollouts]: learned-distance
                              prediction against each neighbour (collision mode 1) for the
                              live queries of the last iteration; 0 elsewhere */
  MPC_DBG_SIGMA = 14,      /* float [horizon][28]: sampling covariance Sigma_h (Eqs. 3-4), packed
                              lower triangle, row j holds (j, 0..j); always available */
  MPC_DBG_CHOL = 15,       /* float [horizon][28]: its Cholesky factor L_h (eps = L_h z); always available */
  MPC_DBG_SKIP = 16        /* unsigned char [n_arms][horizon][n_rollouts]: learned-distance decision of the
                              last step against each neighbour (1 = predicted far; collision mode 1).  A
                              neighbour's check is dropped for rollouts 64b..64b+63 at a step when all 64
                              are 1; steps beyond the shorter of the two horizons hold no decision */
};
/* Copy one captured quantity of one arm into dev_out (device). */
int mpc_debug_get(mpc_ctx *c, int what, int arm, void *dev_out);

/* Read-side plan board of one arm (what the other arms see at Sense):
 * plan [horizon][n_spheres][4], plan_q [horizon][dof] device (either may be
 * NULL); *dist and *valid are host outputs. */
int mpc_get_board(mpc_ctx *c, int arm, float *plan, float *plan_q, float *dist, int *valid);

/* Overwrite the read side of one arm's board (fault injection, external or
 * stale plans).  plan [horizon][n_spheres][4] and plan_q [horizon][dof]
 * device (NULL leaves that part); valid = 0 hides the arm. */
int mpc_set_board(mpc_ctx *c, int arm, const float *plan, const float *plan_q, float dist, int valid);

/* Replace the control means of one arm: mean [horizon][dof] device. */
int mpc_set_mean(mpc_ctx *c, int arm, const float *mean);

/* Step counter t used by the noise stream (advanced by every mpc_step). */
int mpc_get_step(const mpc_ctx *c, unsigned int *t);
int mpc_set_step(mpc_ctx *c, unsigned int t);

/* Plant stand-in for Execute (Alg. 1): advance state [n_arms][dof][3]
 * (device, in place) by one step of the rollout dynamics under u [n_arms][dof]. */
int mpc_sim_execute(mpc_ctx *c, float *state, const float *u);

/* Rollout-kernel launch shape picked by the tuner: rollouts per workgroup
 * (64, 128 or 256: 1, 2 or 4 waves sharing one LDS copy of each step's
 * obstacle and neighbour-plan spheres), horizon steps per work item, and
 * workgroups; valid after the first step.  The tuner times the candidates on
 * the first step at which every arm's plan is published (or the fourth step)
 * and keeps its choice per problem shape and device for the process, so a
 * later context of the same shape reuses it without timing. */
int mpc_get_tuning(const mpc_ctx *c, int *rollouts_per_block, int *h_tile, int *grid);
/* Force a launch shape (0 = let the tuner choose); takes effect at the next
 * mpc_step.  rollouts_per_block must be 0, 64, 128 or 256 (else
 * MPC_EUNSUPPORTED) and divide every arm's rollout count padded to a
 * multiple of 64 (else MPC_EINVAL).  Results do not depend on the launch
 * shape: every rollout's stage costs are summed (Eq. 1) in step order
 * whatever the tiling, and each wave scores its own 64 rollouts. */
int mpc_set_tuning(mpc_ctx *c, int rollouts_per_block, int h_tile, int grid);

/* Kernel timing for measurement: while on, mpc_step launches its kernels
 * directly (no graph) and brackets every rollout launch (the fused sampling,
 * dynamics, kinematics and scoring kernel) and, in collision mode 1, every
 * learned-distance inference launch with HIP events on the context's stream. */
int mpc_profile_enable(mpc_ctx *c, int on);
/* Total and count of the bracketed rollout-launch durations since the last
 * read; waits for them and clears the record. */
int mpc_profile_read(mpc_ctx *c, double *total_ms, int *launches);
/* The same for the learned-distance inference launches. */
int mpc_profile_read_surrogate(mpc_ctx *c, double *total_ms, int *launches);

/* ---- learned arm-pair distance (collision_mode 1) ----
 *
 * An MLP 17 -> 256 -> 256 -> 256 -> 1 (ReLU) predicts the signed minimum
 * sphere distance (Eq. 6) between two arms of the same model from their joint
 * positions and base offset.  In collision mode 1 the network scores every
 * (rollout, step, neighbour) query; a query is "far" when its prediction is
 * at least surrogate_margin and its inputs lie inside the training box.  The
 * rollouts are scored in blocks of 64 (rollouts 64b .. 64b+63 of an arm):
 * when all 64 queries of a block against a neighbour at a step are far, that
 * neighbour's coordination term is dropped for them (hinge zero) and its
 * exact sphere-pair check is not run; otherwise all 64 are checked exactly.
 * So every query predicted below the margin is checked exactly, and a far
 * query is checked exactly unless its whole block is far.  The margin must
 * be at least buf_dyn.  Inputs, in the
 * first arm's base frame: its 7 joints normalised to [-1, 1] by the limits,
 * the other arm's first joint plus the yaw difference (wrapped, / pi), the
 * other arm's 6 further normalised joints, and the base offset (metres).
 * Training uses bfloat16 operands with FP32 accumulation, FP32 master
 * weights and Adam, on distances the exact kernel generates. */
typedef struct {
  int samples;             /* training set size (>= 1024) */
  int epochs;
  int batch;               /* 64..65536 */
  float lr, beta1, beta2, adam_eps;
  float over_weight;       /* loss = mean om(t) [(y-t)^2 + over_weight * max(0, y-t)^2] */
  float target_clip;       /* targets max(min(rho, clip), target_floor), metres */
  float val_fraction;      /* held-out share, [0, 0.5) */
  unsigned long long seed;
  float lr_final;          /* step size at the end of the cosine schedule, (0, lr] */
  float near_weight;       /* om(t) = 1 + near_weight if t < near_band, else 1 (>= 0) */
  float near_band;         /* metres */
  float target_floor;      /* below target_clip; use a large negative value for none */
} mpc_train_params;

typedef struct {
  float final_loss;        /* mean training loss of the last epoch */
  float val_mae, val_rmse, val_p99;  /* held-out absolute error statistics, metres */
  float val_max_over;      /* largest over-prediction (prediction - target) */
  float val_min_err;       /* most negative error */
  long long steps;         /* optimiser steps */
  float seconds;           /* device time of sampling + training + validation */
  float val_skip_rate;     /* share of held-out samples predicted >= surrogate_margin */
  float val_miss_rate;     /* share of held-out samples with target < 0 predicted >= the margin */
  float val_max_over_near; /* largest over-prediction among held-out targets below the margin */
} mpc_train_report;

/* Exact signed distance (Eq. 6, min over all sphere pairs) between arm_i at
 * q_i [m][7] and arm_j at q_j [m][7], at their bases; rho [m].  Device. */
int mpc_pair_distance(mpc_ctx *c, int arm_i, int arm_j, const float *q_i, const float *q_j, int m, float *rho);
/* Input features [m][17] of the learned distance for the same queries.  Device. */
int mpc_pair_features(mpc_ctx *c, int arm_i, int arm_j, const float *q_i, const float *q_j, int m,
                      float *features);
/* Draw training samples (every directed arm pair of the context, joints
 * uniform in the limits, counter-based draws keyed by seed, sample indices
 * first..first+m-1): features [m][17] (the bfloat16 values the network sees),
 * targets [m] = max(min(rho, clip), floor), joints [m][14] (q_i, q_j; may be
 * NULL).  Device. */
int mpc_surrogate_samples(mpc_ctx *c, unsigned long long seed, long long first, int m, float clip, float floor,
                          float *features, float *targets, float *joints);
/* Train the network from scratch on freshly drawn samples (weights and biases
 * uniform in +-1/sqrt(fan_in), Adam, step size on a cosine from lr to
 * lr_final); waits for the GPU. */
int mpc_surrogate_train(mpc_ctx *c, const mpc_train_params *tp, mpc_train_report *report);
/* FP32 parameters [136449], packed per layer as W[out][in] then b[out].  Device. */
int mpc_surrogate_get_params(mpc_ctx *c, float *params);
int mpc_surrogate_set_params(mpc_ctx *c, const float *params);
/* Network output for features [m][17]; y [m].  Device; waits for the GPU. */
int mpc_surrogate_predict(mpc_ctx *c, const float *features, int m, float *y);
/* mpc_surrogate_predict for callers that cannot allocate (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same network output, bitwise, for features [m][17] into y [m] (device),
 * enqueued on the context's stream and not waited for; no hipMalloc, hipFree
 * or allocating library call.  Its working memory (the inputs and two
 * activation buffers of up to MPC_PREDICT_NOALLOC_MAX queries, 4.3 MB) is
 * one fixed array per GPU, held until the process ends and shared by every
 * call on that GPU: calls that overlap on one GPU (two streams or threads)
 * race on it.  Nothing in it needs to start at zero.  Errors: MPC_EINVAL for
 * m < 0, m > MPC_PREDICT_NOALLOC_MAX or a NULL array with m > 0. */
#define MPC_PREDICT_NOALLOC_MAX 4096
int mpc_surrogate_predict_noalloc(mpc_ctx *c, const float *features, int m, float *y);
/* One forward + backward pass of the training dataflow on a batch
 * (features [B][17], targets [B]) with the training loss (over_weight,
 * near_weight, near_band as in mpc_train_params): gradient [136449]
 * (device), loss (host). */
int mpc_surrogate_grad(mpc_ctx *c, const float *features, const float *targets, int B, float over_weight,
                       float near_weight, float near_band, float *grad, float *loss);
/* One Adam step (Kingma and Ba, bias-corrected, step counted from 1) on the
 * network's FP32 parameters with a caller's gradient [136449] (device, e.g.
 * from mpc_surrogate_grad), exactly as the training loop applies it:
 * m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * p -= lr (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps); the bfloat16
 * copy the network runs on is refreshed.  step = 1 clears both moment
 * estimates first.  Together with mpc_surrogate_grad it forms a training
 * loop of the caller's own.  Errors: MPC_EINVAL for step < 1, lr <= 0, a
 * beta outside [0, 1) or eps < 0. */
int mpc_surrogate_adam(mpc_ctx *c, const float *grad, float lr, float beta1, float beta2, float eps, int step);
/* Switch between exact (0) and learned (1) coordination distances.
 * Errors: MPC_EINVAL for mode 1 when surrogate_margin is below buf_dyn;
 * MPC_EUNSUPPORTED when the arms are not one model. */
int mpc_set_collision_mode(mpc_ctx *c, int mode);
/* Audit: in mode 1 also run the exact checks of the dropped blocks (the
 * costs stay those of mode 1) and count their queries whose exact distance
 * is below buf_dyn (misses) or below zero (missed collisions). */
int mpc_surrogate_audit(mpc_ctx *c, int on);
/* Counters summed over arms since the last reset: out[6] = queries, far
 * queries, dropped (block, neighbour, step) checks of 64 rollouts, misses,
 * missed collisions (the last two only while auditing), query rows run
 * through the network (32 per descriptor, padded rollouts included; the
 * screen lowers it).  Waits for the GPU. */
int mpc_surrogate_stats(mpc_ctx *c, unsigned long long *out, int reset);

/* Device Philox4x32-10 (the noise generator) on n counters: ctr [n][4],
 * key [n][2], out [n][4], all device uint32.  Runs on hip_stream. */
int mpc_philox(const unsigned int *ctr, const unsigned int *key, unsigned int *out, int n,
               void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif
