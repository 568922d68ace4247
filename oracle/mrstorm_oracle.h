/* CPU ORACLE for one MR-STORM control step (arXiv 2602.10114) -- TEST
 * INFRASTRUCTURE ONLY.
 *
 * Plain FP64 C written from the paper's definitions, in the paper's order,
 * with no blocking, fusion or reordering.  Only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg load it; the HIP library never
 * includes, links or calls anything here, and this file includes nothing of
 * the HIP library.  Inputs arrive as doubles holding the FP32 values the GPU
 * path is given, so both sides start from identical numbers.
 *
 * Parity status of each function is recorded beside it ("pinned by": the
 * independent facts the tests check it against).
 */
#ifndef MRSTORM_ORACLE_H
#define MRSTORM_ORACLE_H
#include <stdint.h>

#define ORC_MAX_DOF 8
#define ORC_MAX_SPHERES 64
#define ORC_MAX_ARMS 16

typedef struct {
  int dof, n_spheres, n_rollouts, horizon;
  double dh[ORC_MAX_DOF][4];      /* a_{k-1}, alpha_{k-1}, d_k, theta offset (modified DH) */
  double qlim[ORC_MAX_DOF][2];    /* lower, upper */
  double qdmax[ORC_MAX_DOF];
  double spheres[ORC_MAX_SPHERES][4]; /* body-frame centre, radius */
  int link[ORC_MAX_SPHERES];      /* body 0..dof-1 = link frame 1..dof; dof = hand */
  double base[4];                 /* x, y, z, yaw */
  double tool[3];                 /* end-effector point in the last link frame */
} orc_arm;

typedef struct {
  double dt, sigma, lambda, gamma, alpha_mu;
  double w_pose, w_rot, w_stop, w_joint, w_coll, w_dyn;
  double buf_env, buf_self, buf_dyn, tau, prio_min, prio_max, dist_floor, joint_margin;
  unsigned long long seed;
  int iters;
  int plan_mode;                  /* 0: predicted plan; 1: current spheres at every step (S_d) */
  double alpha_sigma, sigma_floor;
  double w_manip, manip_thresh;
} orc_params;

/* ---- primitives ---- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void orc_normals(unsigned long long seed, int arm, uint32_t t, int k, int n, int h, int dof, double *z);
void orc_integrate(int dof, int H, double dt, const double *q0, const double *qd0,
                   const double *U, double *q, double *qd);
void orc_fk(const orc_arm *arm, const double *q, double *frames /*[dof+1][4][4]*/);
void orc_spheres(const orc_arm *arm, const double *q, double *out /*[S][4]*/);
void orc_ee_pose(const orc_arm *arm, const double *q, double *T /*[4][4]*/);
void orc_quat_to_rot(const double *wxyz, double *R /*[3][3]*/);
double orc_sphere_rho(const double *a, const double *b);
double orc_rho_sets(const double *A, int na, const double *B, int nb);
double orc_rho_self(const double *c, const int *link, int S);
double orc_hinge(double rho, double B);
double orc_pose_cost(const double *Tee, const double *goal, double w_rot);
double orc_stop_cost(const orc_arm *arm, int H, int h, const double *qd);
double orc_joint_cost(const orc_arm *arm, const double *q, double margin);
double orc_priority(double d_own, double d_other, double tau, double floor_, double pmin, double pmax);
double orc_total_cost(int H, double gamma, const double *stage /*[H]*/);
void orc_weights(int N, double lambda, const double *C, double *w);
void orc_weighted_mean(int N, int H, int dof, const double *w, const double *U /*[N][H][d]*/, double *mu_tilde);
void orc_ema(int H, int dof, double alpha_mu, const double *mu_tilde, double *mu);
/* Eq. 3, second half: Sigma~_h = sum_n w_n (U_{n,h} - mu~_h)(U_{n,h} - mu~_h)^T;
 * U [N][H][d], mt [H][d], out [H][d][d]. */
void orc_weighted_cov(int N, int H, int dof, const double *w, const double *U, const double *mt, double *out);
/* Lower Cholesky factor of a symmetric d x d matrix, pivots floored at floor_var. */
void orc_cholesky_floor(int dof, const double *S, double floor_var, double *L);
int orc_argmin(int N, const double *C);
void orc_shift(int H, int dof, double *mu);
long long orc_pair_count(int H, int N, int S_own, const int *S_nb, int n_nb);

/* ---- stage-level entry points (fed upstream values from elsewhere) ---- */
/* Geometric Jacobian J [6][dof] (linear rows, then angular) of the
 * end-effector point at q, and the manipulability cost of Eq. 5:
 * max(0, 1 - sqrt(det(J J^T)) / thresh). */
void orc_jacobian(const orc_arm *arm, const double *q, double *J);
double orc_manip_cost(const orc_arm *arm, const double *q, double thresh);
/* Stage cost of one rollout step (Eq. 5 with Eqs. 6-10).  nb_plan[i] points
 * at neighbour i's plan spheres for this h ([S_i][4]); nb_active[i] = 0 skips
 * it (unpublished plan, or h beyond its horizon).  terms[8] receives
 * pose, stop, joint, coll, self, dyn-sum(alpha*hinge), total, manip. */
double orc_stage_cost(const orc_arm *arm, const orc_params *p, int H, int h,
                      const double *q, const double *qd, const double *spheres,
                      const double *goal, const double *obs, int n_obs,
                      const double *const *nb_plan, const int *nb_S, const int *nb_active,
                      const double *alpha_row, int n_nb, double *terms);
/* Batched form over all (n, h) of one arm.  q, qd: [N][H][d]; spheres:
 * [N][H][S][4]; plans: [n_nb][H_max][S_max][4] with nb_H[i] steps valid;
 * out: [H][N]; terms_out (optional): [H][N][8]. */
void orc_stage_costs_batch(const orc_arm *arm, const orc_params *p, int N, int H,
                           const double *q, const double *qd, const double *spheres,
                           const double *goal, const double *obs, int n_obs,
                           const double *plans, int n_nb, int H_max, int S_max,
                           const int *nb_S, const int *nb_H, const int *nb_valid,
                           const double *alpha_row, double *out, double *terms_out);

/* ---- full controller (all arms, Alg. 1 per arm, shared plan board) ---- */
typedef struct orc_ctx orc_ctx;
orc_ctx *orc_create(const orc_arm *arms, int n_arms, const orc_params *p);
void orc_destroy(orc_ctx *c);
void orc_share_plans(orc_ctx *c, const unsigned char *mask);
/* state [A][d][3], goal [A][7], obstacles [O][4]; u_out [A][d]. */
void orc_step(orc_ctx *c, const double *state, const double *goal, const double *obs,
              int n_obs, double *u_out);
/* Restrict the next steps' rollouts to n in [n_lo, n_hi) of every arm (a
 * bounded sample for timing; the update then sees only those rollouts). */
void orc_set_rollout_window(orc_ctx *c, int n_lo, int n_hi);
/* Accessors for the last step (arm a). */
void orc_get_mean(const orc_ctx *c, int a, double *mu /*[H][d]*/);
/* Sampling covariances and their factors of arm a, [Hmax][d][d] each (either may be NULL). */
void orc_get_sigma(const orc_ctx *c, int a, double *sig, double *chol);
void orc_set_mean(orc_ctx *c, int a, const double *mu);
void orc_get_plan(const orc_ctx *c, int a, int side, double *plan /*[H][S][4]*/,
                  double *plan_q /*[H][d]*/, double *dist, int *valid);
void orc_set_plan(orc_ctx *c, int a, const double *plan, const double *plan_q, double dist, int valid);
void orc_get_costs(const orc_ctx *c, int a, double *total /*[N]*/, double *stage /*[H][N]*/,
                   double *weights /*[N]*/);
void orc_get_noise(const orc_ctx *c, int a, double *eps /*[N][H][d]*/);
void orc_get_alpha(const orc_ctx *c, double *alpha /*[A][A]*/, double *dist_now /*[A]*/);
uint32_t orc_get_step(const orc_ctx *c);
void orc_set_step(orc_ctx *c, uint32_t t);

/* ---- learned arm-pair distance: exact target and the MLP ---- */
/* Signed minimum sphere distance between arm i at q_i and arm j at q_j
 * (Eq. 6 over all sphere pairs). */
double orc_arm_pair_rho(const orc_arm *ai, const double *qi, const orc_arm *aj, const double *qj);
/* MLP with layer widths w[0..L] (ReLU between layers, linear output).
 * Parameters are packed per layer as W[out][in] then b[out]. */
long long orc_mlp_param_count(int L, const int *w);
void orc_mlp_forward(int L, const int *w, const double *params, int B, const double *x, double *y);
/* Loss = mean over the batch of om(t) [(y - t)^2 + over_w * max(0, y - t)^2]
 * with om(t) = 1 + near_w if t < near_band else 1, and its gradient with
 * respect to every parameter (same packing). */
double orc_mlp_loss_grad(int L, const int *w, const double *params, int B, const double *x,
                         const double *t, double over_w, double near_w, double near_band, double *grad);
void orc_adam(long long n, double *p, double *m, double *v, const double *g, double lr,
              double b1, double b2, double eps, int step);
/* bfloat16 rounding (round to nearest, ties to even) of a double taken as FP32. */
double orc_bf16(double x);
/* The same loss and gradient with the reduced-precision training dataflow
 * written out: every product operand (inputs, weights, hidden activations,
 * back-propagated deltas) rounded to bfloat16, sums and biases exact. */
double orc_mlp_loss_grad_bf16(int L, const int *w, const double *params, int B, const double *x,
                              const double *t, double over_w, double near_w, double near_band, double *grad);
/* The forward pass of that reduced-precision dataflow alone (the network as
 * the inference kernel computes it): inputs, weights and hidden activations
 * rounded to bfloat16 before each product, sums and biases exact, ReLU
 * between layers, linear output. */
void orc_mlp_forward_bf16(int L, const int *w, const double *params, int B, const double *x, double *y);
/* Input features of the learned distance between arm a at q_a (own) and arm
 * i at q_i (neighbour), in arm a's base frame: 7 normalised own joints, the
 * neighbour's first joint plus the yaw difference (wrapped, / pi), its other
 * 6 normalised joints, and the base offset rotated into arm a's frame. */
void orc_pair_features(const orc_arm *a, const double *qa, const orc_arm *i, const double *qi, double *f);
#endif
