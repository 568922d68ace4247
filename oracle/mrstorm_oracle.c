/* CPU ORACLE for one MR-STORM control step -- TEST INFRASTRUCTURE ONLY.
 *
 * FP64 throughout.  Each function follows a passage of the paper (arXiv
 * 2602.10114, "MR-STORM") or, where the paper defers to STORM or is silent,
 * the reading recorded with it.  No blocking, fusion or reordering beyond the
 * definitions.  Shares no code with the HIP library.
 */
#include "mrstorm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------
 * Counter-based noise.  Philox4x32-10 as defined by Salmon, Moraes, Dror and
 * Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11): ten rounds of
 * two 32x32->64 multiplies, the key bumped by the golden-ratio constants
 * between rounds.
 * Pinned by: the published known-answer vectors of that generator.
 * ---------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Standard normals for rollout n, step h (0-based), iteration k of control
 * step t of arm `arm`: Sec. III-A draws eps_{n,h} ~ N(0, Sigma_h); with
 * Sigma = sigma^2 I the d components are independent standard normals times
 * sigma.  Project definition of the stream: counter (n, 2h+c, t,
 * (arm<<8)|k), key (seed low word, seed high word), c = 0,1 the chunk; each
 * 32-bit word x becomes u = (x>>8 + 1/2) * 2^-24 in (0,1); Box-Muller on
 * (u0,u1) and (u2,u3) gives cos, sin, cos, sin; joint j takes chunk j/4,
 * lane j%4.
 * Pinned by: moments of a large sample; Box-Muller identities. */
void orc_normals(unsigned long long seed, int arm, uint32_t t, int k, int n, int h, int dof,
                 double *z) {
  const double two_pi = 6.283185307179586476925286766559;
  uint32_t key[2] = {(uint32_t)(seed & 0xffffffffull), (uint32_t)(seed >> 32)};
  for (int c = 0; c * 4 < dof; ++c) {
    uint32_t ctr[4] = {(uint32_t)n, (uint32_t)(2 * h + c), t, ((uint32_t)arm << 8) | (uint32_t)k};
    uint32_t x[4];
    orc_philox4x32_10(ctr, key, x);
    double u[4];
    for (int i = 0; i < 4; ++i) u[i] = ((double)(x[i] >> 8) + 0.5) * (1.0 / 16777216.0);
    double lane[4];
    double r01 = sqrt(-2.0 * log(u[0])), r23 = sqrt(-2.0 * log(u[2]));
    lane[0] = r01 * cos(two_pi * u[1]);
    lane[1] = r01 * sin(two_pi * u[1]);
    lane[2] = r23 * cos(two_pi * u[3]);
    lane[3] = r23 * sin(two_pi * u[3]);
    for (int i = 0; i < 4 && 4 * c + i < dof; ++i) z[4 * c + i] = lane[i];
  }
}

/* ------------------------------------------------------------------------
 * Dynamics f (Sec. III-A): sampled controls are joint accelerations; the
 * rollout state (theta, theta_dot, theta_ddot) is integrated from the current
 * state.  Reading: semi-implicit Euler, theta_ddot_h = U_h,
 * theta_dot_h = theta_dot_{h-1} + dt*U_h, theta_h = theta_{h-1} + dt*theta_dot_h.
 * U, q, qd: [H][d].
 * Pinned by: the closed form for constant acceleration. */
void orc_integrate(int dof, int H, double dt, const double *q0, const double *qd0,
                   const double *U, double *q, double *qd) {
  double qc[ORC_MAX_DOF], vc[ORC_MAX_DOF];
  for (int j = 0; j < dof; ++j) { qc[j] = q0[j]; vc[j] = qd0[j]; }
  for (int h = 0; h < H; ++h) {
    for (int j = 0; j < dof; ++j) {
      vc[j] = vc[j] + dt * U[h * dof + j];
      qc[j] = qc[j] + dt * vc[j];
      q[h * dof + j] = qc[j];
      qd[h * dof + j] = vc[j];
    }
  }
}

/* ------------------------------------------------------------------------
 * Forward kinematics (Sec. IV-A: link frames by forward kinematics, spheres
 * at constant transforms from the links).  Modified (Craig) DH:
 *   T_k = T_{k-1} RotX(alpha_{k-1}) TransX(a_{k-1}) RotZ(q_k + off_k) TransZ(d_k),
 * T_0 = Trans(base xyz) RotZ(base yaw).  frames[k] = T_{k+1}, k < dof;
 * frames[dof] = T_dof (the hand is rigid with the last link).
 * Pinned by: orthonormal rotations, constant joint-origin spacing, planar
 * chain closed form, base yaw equivalence, a hand-multiplied 2-link pose.
 * ---------------------------------------------------------------------- */
static void mat4_mul(const double *A, const double *B, double *C) {
  double T[16];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      double s = 0.0;
      for (int k = 0; k < 4; ++k) s += A[i * 4 + k] * B[k * 4 + j];
      T[i * 4 + j] = s;
    }
  memcpy(C, T, sizeof(T));
}
static void mat4_identity(double *A) {
  memset(A, 0, 16 * sizeof(double));
  A[0] = A[5] = A[10] = A[15] = 1.0;
}
static void mat4_rotx(double a, double *A) {
  mat4_identity(A);
  A[5] = cos(a); A[6] = -sin(a);
  A[9] = sin(a); A[10] = cos(a);
}
static void mat4_rotz(double a, double *A) {
  mat4_identity(A);
  A[0] = cos(a); A[1] = -sin(a);
  A[4] = sin(a); A[5] = cos(a);
}
static void mat4_trans(double x, double y, double z, double *A) {
  mat4_identity(A);
  A[3] = x; A[7] = y; A[11] = z;
}

void orc_fk(const orc_arm *arm, const double *q, double *frames) {
  double T[16], M[16];
  mat4_trans(arm->base[0], arm->base[1], arm->base[2], T);
  mat4_rotz(arm->base[3], M);
  mat4_mul(T, M, T);
  for (int k = 0; k < arm->dof; ++k) {
    const double *dh = arm->dh[k];
    mat4_rotx(dh[1], M); mat4_mul(T, M, T);
    mat4_trans(dh[0], 0.0, 0.0, M); mat4_mul(T, M, T);
    mat4_rotz(q[k] + dh[3], M); mat4_mul(T, M, T);
    mat4_trans(0.0, 0.0, dh[2], M); mat4_mul(T, M, T);
    memcpy(frames + 16 * k, T, sizeof(T));
  }
  memcpy(frames + 16 * arm->dof, T, sizeof(T));
}

/* World-frame collision spheres S (Sec. IV-A): centre = T_body * p, radius
 * unchanged.  Pinned by: |c - t_body| = |p| per sphere; hand-multiplied
 * centres of offsets off the frame axes on non-symmetric frame rotations
 * (a transposed rotation fails). */
void orc_spheres(const orc_arm *arm, const double *q, double *out) {
  double frames[(ORC_MAX_DOF + 1) * 16];
  orc_fk(arm, q, frames);
  for (int s = 0; s < arm->n_spheres; ++s) {
    const double *T = frames + 16 * arm->link[s];
    const double *p = arm->spheres[s];
    for (int i = 0; i < 3; ++i)
      out[4 * s + i] = T[4 * i + 0] * p[0] + T[4 * i + 1] * p[1] + T[4 * i + 2] * p[2] + T[4 * i + 3];
    out[4 * s + 3] = p[3];
  }
}

/* End-effector frame: the last link frame translated by the tool point
 * given in that frame (the pose term of Eq. 5).  Pinned by: the hand-derived
 * Panda-scale zero pose with its 0.25 m tool, and the two-link tool offset
 * off the frame axes. */
void orc_ee_pose(const orc_arm *arm, const double *q, double *Tee) {
  double frames[(ORC_MAX_DOF + 1) * 16], M[16];
  orc_fk(arm, q, frames);
  mat4_trans(arm->tool[0], arm->tool[1], arm->tool[2], M);
  mat4_mul(frames + 16 * arm->dof, M, Tee);
}

/* Geometric Jacobian of the end-effector point (reading of C_manip's
 * "Jacobian ellipsoid"): column k = (z_k x (p_ee - o_k), z_k), z_k the axis
 * of joint k (z of frame k in modified DH) and o_k a point on it (the origin
 * of frame k).  Pinned by central differences of the forward kinematics. */
void orc_jacobian(const orc_arm *arm, const double *q, double *J) {
  double frames[(ORC_MAX_DOF + 1) * 16], Tee[16];
  orc_fk(arm, q, frames);
  orc_ee_pose(arm, q, Tee);
  int d = arm->dof;
  for (int k = 0; k < d; ++k) {
    const double *T = frames + 16 * k;
    double z[3] = {T[2], T[6], T[10]}, r[3] = {Tee[3] - T[3], Tee[7] - T[7], Tee[11] - T[11]};
    J[0 * d + k] = z[1] * r[2] - z[2] * r[1];
    J[1 * d + k] = z[2] * r[0] - z[0] * r[2];
    J[2 * d + k] = z[0] * r[1] - z[1] * r[0];
    J[3 * d + k] = z[0];
    J[4 * d + k] = z[1];
    J[5 * d + k] = z[2];
  }
}

/* C_manip (Eq. 5; form a reading, following STORM's manipulability score):
 * the volume of the manipulability ellipsoid sqrt(det(J J^T)), penalised
 * linearly below thresh.  det by Gaussian elimination with partial pivoting. */
double orc_manip_cost(const orc_arm *arm, const double *q, double thresh) {
  int d = arm->dof;
  double J[6 * ORC_MAX_DOF], G[36];
  orc_jacobian(arm, q, J);
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) {
      double s = 0.0;
      for (int k = 0; k < d; ++k) s += J[i * d + k] * J[j * d + k];
      G[i * 6 + j] = s;
    }
  double det = 1.0;
  for (int c = 0; c < 6; ++c) {
    int piv = c;
    for (int r = c + 1; r < 6; ++r) if (fabs(G[r * 6 + c]) > fabs(G[piv * 6 + c])) piv = r;
    if (G[piv * 6 + c] == 0.0) { det = 0.0; break; }
    if (piv != c) {
      for (int j = 0; j < 6; ++j) { double t = G[c * 6 + j]; G[c * 6 + j] = G[piv * 6 + j]; G[piv * 6 + j] = t; }
      det = -det;
    }
    det *= G[c * 6 + c];
    for (int r = c + 1; r < 6; ++r) {
      double f = G[r * 6 + c] / G[c * 6 + c];
      for (int j = c; j < 6; ++j) G[r * 6 + j] -= f * G[c * 6 + j];
    }
  }
  double m = sqrt(det > 0.0 ? det : 0.0);
  double v = 1.0 - m / thresh;
  return v > 0.0 ? v : 0.0;
}

/* Rotation of a unit quaternion given as (w, x, y, z); the input is
 * normalised first.  Pinned by: orthonormality and the quaternion-inner-
 * product identity of the orientation term. */
void orc_quat_to_rot(const double *q, double *R) {
  double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  double w = q[0] / n, x = q[1] / n, y = q[2] / n, z = q[3] / n;
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

/* ------------------------------------------------------------------------
 * Distances (Eq. 6): rho_b between two spheres is the Euclidean gap between
 * their surfaces, |c_a - c_b| - r_a - r_b (negative when they overlap); the
 * distance between two sets is the minimum over all pairs.
 * Pinned by: two-sphere closed form, brute force, rigid-motion invariance,
 * symmetry.
 * ---------------------------------------------------------------------- */
double orc_sphere_rho(const double *a, const double *b) {
  double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
  return sqrt(dx * dx + dy * dy + dz * dz) - a[3] - b[3];
}

double orc_rho_sets(const double *A, int na, const double *B, int nb) {
  double best = INFINITY;
  for (int i = 0; i < na; ++i)
    for (int j = 0; j < nb; ++j) {
      double r = orc_sphere_rho(A + 4 * i, B + 4 * j);
      if (r < best) best = r;
    }
  return best;
}

/* Self-collision set (reading): sphere pairs on bodies at least two apart in
 * the chain (adjacent bodies overlap by construction at their joint). */
double orc_rho_self(const double *c, const int *link, int S) {
  double best = INFINITY;
  for (int s = 0; s < S; ++s)
    for (int u = s + 1; u < S; ++u) {
      if (abs(link[s] - link[u]) < 2) continue;
      double r = orc_sphere_rho(c + 4 * s, c + 4 * u);
      if (r < best) best = r;
    }
  return best;
}

/* Hinge of the coordination cost (Sec. IV-A, C_dyn definition):
 * max(0, 1 - rho/B), with rho clamped at 0 from below (reading: overlapping
 * spheres get the full penalty of vanishing distance).
 * Pinned by: rho >= B -> 0, rho <= 0 -> 1, rho = B/2 -> 1/2. */
double orc_hinge(double rho, double B) {
  double r = rho > 0.0 ? rho : 0.0;
  double v = 1.0 - r / B;
  return v > 0.0 ? v : 0.0;
}

/* ------------------------------------------------------------------------
 * STORM stage-cost terms (Eq. 5).  The paper names the terms and defers
 * their forms to STORM; readings:
 *   pose  = |t_ee - g_p| + w_rot * (3 - tr(R_g^T R_ee)) / 4
 *   stop  = sum_j max(0, |qd_j| - qdmax_j * (H - h') / H), h' = h+1 in 1..H
 *   joint = sum_j max(0, lo_j + m - q_j) + max(0, q_j - hi_j + m)
 * C_manip is not part of this path.
 * ---------------------------------------------------------------------- */
double orc_pose_cost(const double *Tee, const double *goal, double w_rot) {
  double dx = Tee[3] - goal[0], dy = Tee[7] - goal[1], dz = Tee[11] - goal[2];
  double pos = sqrt(dx * dx + dy * dy + dz * dz);
  double Rg[9];
  orc_quat_to_rot(goal + 3, Rg);
  double tr = 0.0;  /* tr(Rg^T R) = sum_ij Rg_ij R_ij */
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) tr += Rg[3 * i + j] * Tee[4 * i + j];
  return pos + w_rot * (3.0 - tr) / 4.0;
}

double orc_stop_cost(const orc_arm *arm, int H, int h, const double *qd) {
  double c = 0.0;
  for (int j = 0; j < arm->dof; ++j) {
    double lim = arm->qdmax[j] * (double)(H - (h + 1)) / (double)H;
    double e = fabs(qd[j]) - lim;
    if (e > 0.0) c += e;
  }
  return c;
}

double orc_joint_cost(const orc_arm *arm, const double *q, double m) {
  double c = 0.0;
  for (int j = 0; j < arm->dof; ++j) {
    double lo = arm->qlim[j][0] + m - q[j];
    double hi = q[j] - arm->qlim[j][1] + m;
    if (lo > 0.0) c += lo;
    if (hi > 0.0) c += hi;
  }
  return c;
}

/* Priority factor (Eq. 10): (d_own / d_other)^tau with d = |ee_p - g_p|.
 * Readings: distances floored at dist_floor, result clamped to
 * [pmin, pmax].  Pinned by: tau = 0 -> 1; unclamped product with the
 * reverse factor is 1; the arm nearer its goal gets the smaller factor. */
double orc_priority(double d_own, double d_other, double tau, double floor_, double pmin, double pmax) {
  double a = d_own > floor_ ? d_own : floor_;
  double b = d_other > floor_ ? d_other : floor_;
  double v = pow(a / b, tau);
  if (v < pmin) v = pmin;
  if (v > pmax) v = pmax;
  return v;
}

/* Stage cost with coordination term (Eq. 5 + Eq. 9): STORM terms plus
 * w_d * sum_i alpha^(j,i) * max(0, 1 - rho_b/B) over neighbours i whose plan
 * is active at this step. */
double orc_stage_cost(const orc_arm *arm, const orc_params *p, int H, int h,
                      const double *q, const double *qd, const double *spheres,
                      const double *goal, const double *obs, int n_obs,
                      const double *const *nb_plan, const int *nb_S, const int *nb_active,
                      const double *alpha_row, int n_nb, double *terms) {
  double Tee[16];
  orc_ee_pose(arm, q, Tee);
  double pose = orc_pose_cost(Tee, goal, p->w_rot);
  double stop = orc_stop_cost(arm, H, h, qd);
  double joint = orc_joint_cost(arm, q, p->joint_margin);
  double coll = orc_hinge(orc_rho_sets(spheres, arm->n_spheres, obs, n_obs), p->buf_env);
  double self = orc_hinge(orc_rho_self(spheres, arm->link, arm->n_spheres), p->buf_self);
  double dyn = 0.0;
  for (int i = 0; i < n_nb; ++i) {
    if (!nb_active[i]) continue;
    double rho = orc_rho_sets(spheres, arm->n_spheres, nb_plan[i], nb_S[i]);
    dyn += alpha_row[i] * orc_hinge(rho, p->buf_dyn);
  }
  double manip = p->w_manip > 0.0 ? orc_manip_cost(arm, q, p->manip_thresh) : 0.0;
  double total = p->w_pose * pose + p->w_stop * stop + p->w_joint * joint +
                 p->w_coll * (coll + self) + p->w_dyn * dyn + p->w_manip * manip;
  if (terms) {
    terms[0] = pose; terms[1] = stop; terms[2] = joint; terms[3] = coll;
    terms[4] = self; terms[5] = dyn; terms[6] = total; terms[7] = manip;
  }
  return total;
}

void orc_stage_costs_batch(const orc_arm *arm, const orc_params *p, int N, int H,
                           const double *q, const double *qd, const double *spheres,
                           const double *goal, const double *obs, int n_obs,
                           const double *plans, int n_nb, int H_max, int S_max,
                           const int *nb_S, const int *nb_H, const int *nb_valid,
                           const double *alpha_row, double *out, double *terms_out) {
  const int d = arm->dof, S = arm->n_spheres;
  const double *ptrs[ORC_MAX_ARMS];
  int active[ORC_MAX_ARMS];
  for (int h = 0; h < H; ++h) {
    for (int i = 0; i < n_nb; ++i) {
      ptrs[i] = plans + ((size_t)i * H_max + h) * S_max * 4;
      active[i] = nb_valid[i] && h < nb_H[i];
    }
    for (int n = 0; n < N; ++n) {
      size_t nh = (size_t)n * H + h;
      double terms[8];
      out[(size_t)h * N + n] = orc_stage_cost(arm, p, H, h, q + nh * d, qd + nh * d,
                                              spheres + nh * S * 4, goal, obs, n_obs, ptrs,
                                              nb_S, active, alpha_row, n_nb, terms);
      if (terms_out) memcpy(terms_out + ((size_t)h * N + n) * 8, terms, sizeof(terms));
    }
  }
}

/* ------------------------------------------------------------------------
 * MPPI update (Sec. III-A).
 * ---------------------------------------------------------------------- */
/* Eq. 1 with the terminal cost-to-go read as the stage cost at H:
 * C_n = sum_{h=1..H} gamma^(h-1) C_{n,h}. */
double orc_total_cost(int H, double gamma, const double *stage) {
  double s = 0.0, g = 1.0;
  for (int h = 0; h < H; ++h) {
    s += g * stage[h];
    g *= gamma;
  }
  return s;
}

/* Eq. 2.  exp(-C_n/lambda) underflows for every n at the cost scales of
 * Eq. 5, so the common factor exp(min_m C_m / lambda) is divided out of
 * numerator and denominator (the same weights in exact arithmetic).
 * Pinned by: sum to one, shift invariance, the two temperature limits. */
void orc_weights(int N, double lambda, const double *C, double *w) {
  double m = INFINITY;
  for (int n = 0; n < N; ++n) if (C[n] < m) m = C[n];
  double z = 0.0;
  for (int n = 0; n < N; ++n) { w[n] = exp(-(C[n] - m) / lambda); z += w[n]; }
  for (int n = 0; n < N; ++n) w[n] /= z;
}

/* Eq. 3, first half: mu~_h = sum_n w_n U_{n,h}.  U: [N][H][d]. */
void orc_weighted_mean(int N, int H, int dof, const double *w, const double *U, double *mt) {
  for (int h = 0; h < H; ++h)
    for (int j = 0; j < dof; ++j) {
      double s = 0.0;
      for (int n = 0; n < N; ++n) s += w[n] * U[((size_t)n * H + h) * dof + j];
      mt[h * dof + j] = s;
    }
}

/* Eq. 4, first line. */
void orc_ema(int H, int dof, double a, const double *mt, double *mu) {
  for (int i = 0; i < H * dof; ++i) mu[i] = (1.0 - a) * mu[i] + a * mt[i];
}

/* Eq. 3, second half: Sigma~_h = sum_n w_n (U_{n,h} - mu~_h)(U_{n,h} - mu~_h)^T.
 * U: [N][H][d], mt: [H][d] (the weighted mean), out: [H][d][d]. */
void orc_weighted_cov(int N, int H, int dof, const double *w, const double *U, const double *mt, double *out) {
  for (int h = 0; h < H; ++h)
    for (int i = 0; i < dof; ++i)
      for (int j = 0; j < dof; ++j) {
        double s = 0.0;
        for (int n = 0; n < N; ++n) {
          const double *u = U + ((size_t)n * H + h) * dof;
          s += w[n] * (u[i] - mt[h * dof + i]) * (u[j] - mt[h * dof + j]);
        }
        out[((size_t)h * dof + i) * dof + j] = s;
      }
}

/* Cholesky factor L (lower, row-major d x d) of the symmetric S, each pivot
 * floored at floor_var (reading: keeps the sampling distribution proper when
 * the weights collapse onto one rollout). */
void orc_cholesky_floor(int dof, const double *S, double floor_var, double *L) {
  for (int i = 0; i < dof * dof; ++i) L[i] = 0.0;
  for (int j = 0; j < dof; ++j) {
    double d = S[j * dof + j];
    for (int m = 0; m < j; ++m) d -= L[j * dof + m] * L[j * dof + m];
    if (d < floor_var) d = floor_var;
    L[j * dof + j] = sqrt(d);
    for (int i = j + 1; i < dof; ++i) {
      double v = S[i * dof + j];
      for (int m = 0; m < j; ++m) v -= L[i * dof + m] * L[j * dof + m];
      L[i * dof + j] = v / L[j * dof + j];
    }
  }
}

/* Act: n* = argmin_n C_n, lowest index on ties (reading of the argmin). */
int orc_argmin(int N, const double *C) {
  int best = 0;
  for (int n = 1; n < N; ++n) if (C[n] < C[best]) best = n;
  return best;
}

/* Left shift phi_h <- phi_{h+1} for h <= H-1; the last step keeps its value
 * (reading: the paper does not fill phi_H). */
void orc_shift(int H, int dof, double *mu) {
  for (int h = 0; h + 1 < H; ++h)
    for (int j = 0; j < dof; ++j) mu[h * dof + j] = mu[(h + 1) * dof + j];
}

/* Distance queries of one arm per control step (Sec. IV-A, Complexity):
 * H N N_S^(j) sum_{i != j} N_S^(i). */
long long orc_pair_count(int H, int N, int S_own, const int *S_nb, int n_nb) {
  long long s = 0;
  for (int i = 0; i < n_nb; ++i) s += S_nb[i];
  return (long long)H * N * S_own * s;
}

/* ------------------------------------------------------------------------
 * Full controller: Alg. 1 for every arm, plans exchanged through a board
 * with a write side (ToPlan) and a read side (what Sense sees); Publish
 * copies write -> read (every arm at step t reads the plans of step t-1).
 * ---------------------------------------------------------------------- */
struct orc_ctx {
  int A;
  orc_arm arms[ORC_MAX_ARMS];
  orc_params p;
  int Hmax, Smax, Nmax, dof;
  uint32_t t;
  int n_lo, n_hi;
  double *mu;           /* [A][Hmax][d] */
  double *sig, *chol;   /* [A][Hmax][d][d]: sampling covariance (Eqs. 3-4) and its factor */
  double *plan[2];      /* [A][Hmax][Smax][4]; side 0 = read, 1 = write */
  double *plan_q[2];    /* [A][Hmax][d] */
  double dist[2][ORC_MAX_ARMS];
  int valid[2][ORC_MAX_ARMS];
  int written[ORC_MAX_ARMS];
  double alpha[ORC_MAX_ARMS * ORC_MAX_ARMS], dist_now[ORC_MAX_ARMS];
  double *last_total, *last_stage, *last_w, *last_eps; /* per arm blocks */
};

orc_ctx *orc_create(const orc_arm *arms, int n_arms, const orc_params *p) {
  if (n_arms < 1 || n_arms > ORC_MAX_ARMS) return NULL;
  orc_ctx *c = (orc_ctx *)calloc(1, sizeof(orc_ctx));
  c->A = n_arms;
  c->p = *p;
  c->dof = arms[0].dof;
  for (int a = 0; a < n_arms; ++a) {
    c->arms[a] = arms[a];
    if (arms[a].horizon > c->Hmax) c->Hmax = arms[a].horizon;
    if (arms[a].n_spheres > c->Smax) c->Smax = arms[a].n_spheres;
    if (arms[a].n_rollouts > c->Nmax) c->Nmax = arms[a].n_rollouts;
  }
  c->n_lo = 0; c->n_hi = 1 << 30;
  size_t A = n_arms, H = c->Hmax, S = c->Smax, N = c->Nmax, d = c->dof;
  c->mu = (double *)calloc(A * H * d, sizeof(double));
  c->sig = (double *)calloc(A * H * d * d, sizeof(double));
  c->chol = (double *)calloc(A * H * d * d, sizeof(double));
  for (size_t i = 0; i < A * H; ++i)
    for (size_t j = 0; j < d; ++j) {
      c->sig[(i * d + j) * d + j] = p->sigma * p->sigma;  /* Sigma = sigma^2 I ... */
      c->chol[(i * d + j) * d + j] = p->sigma;            /* ... whose factor is sigma I */
    }
  for (int s = 0; s < 2; ++s) {
    c->plan[s] = (double *)calloc(A * H * S * 4, sizeof(double));
    c->plan_q[s] = (double *)calloc(A * H * d, sizeof(double));
  }
  c->last_total = (double *)calloc(A * N, sizeof(double));
  c->last_w = (double *)calloc(A * N, sizeof(double));
  c->last_stage = (double *)calloc(A * H * N, sizeof(double));
  c->last_eps = (double *)calloc(A * N * H * d, sizeof(double));
  return c;
}

void orc_destroy(orc_ctx *c) {
  if (!c) return;
  free(c->mu); free(c->sig); free(c->chol);
  for (int s = 0; s < 2; ++s) { free(c->plan[s]); free(c->plan_q[s]); }
  free(c->last_total); free(c->last_w); free(c->last_stage); free(c->last_eps);
  free(c);
}

void orc_set_rollout_window(orc_ctx *c, int n_lo, int n_hi) { c->n_lo = n_lo; c->n_hi = n_hi; }

/* Publish (Alg. 1): the masked arms' freshly written plans become visible. */
void orc_share_plans(orc_ctx *c, const unsigned char *mask) {
  size_t H = c->Hmax, S = c->Smax, d = c->dof;
  for (int a = 0; a < c->A; ++a) {
    if (mask && !mask[a]) continue;
    if (!c->written[a]) continue;
    memcpy(c->plan[0] + a * H * S * 4, c->plan[1] + a * H * S * 4, H * S * 4 * sizeof(double));
    memcpy(c->plan_q[0] + a * H * d, c->plan_q[1] + a * H * d, H * d * sizeof(double));
    c->dist[0][a] = c->dist[1][a];
    c->valid[0][a] = 1;
  }
}

/* ToPlan (Sec. IV-A; Alg. 1 Publish phase): integrate the mean controls from
 * the current state, then forward kinematics and spheres at every step. */
static void to_plan(orc_ctx *c, int a, const double *state) {
  const orc_arm *arm = &c->arms[a];
  int d = arm->dof, H = arm->horizon;
  size_t Hm = c->Hmax, Sm = c->Smax;
  double q0[ORC_MAX_DOF], qd0[ORC_MAX_DOF];
  for (int j = 0; j < d; ++j) { q0[j] = state[3 * j]; qd0[j] = state[3 * j + 1]; }
  double *q = (double *)malloc(sizeof(double) * H * d), *qd = (double *)malloc(sizeof(double) * H * d);
  if (c->p.plan_mode == 1) {
    /* S_d ablation: the arm's current configuration at every step (its
     * spheres act as a static obstacle for the others). */
    for (int h = 0; h < H; ++h)
      for (int j = 0; j < d; ++j) q[h * d + j] = q0[j];
  } else {
    orc_integrate(d, H, c->p.dt, q0, qd0, c->mu + a * Hm * d, q, qd);
  }
  double *out = c->plan[1] + a * Hm * Sm * 4;
  double *outq = c->plan_q[1] + a * Hm * d;
  memset(out, 0, Hm * Sm * 4 * sizeof(double));
  memset(outq, 0, Hm * d * sizeof(double));
  for (int h = 0; h < H; ++h) {
    orc_spheres(arm, q + h * d, out + h * Sm * 4);
    for (int j = 0; j < d; ++j) outq[h * d + j] = q[h * d + j];
  }
  c->written[a] = 1;
  free(q); free(qd);
}

void orc_step(orc_ctx *c, const double *state, const double *goal, const double *obs, int n_obs,
              double *u_out) {
  const orc_params *p = &c->p;
  int A = c->A;
  size_t Hm = c->Hmax, Sm = c->Smax, Nm = c->Nmax;
  /* Sense: own distance to goal now, and the priority factors against every
   * neighbour whose plan (and distance) has been published. */
  for (int a = 0; a < A; ++a) {
    double Tee[16];
    double q[ORC_MAX_DOF];
    for (int j = 0; j < c->arms[a].dof; ++j) q[j] = state[(a * c->dof + j) * 3];
    orc_ee_pose(&c->arms[a], q, Tee);
    double dx = Tee[3] - goal[7 * a], dy = Tee[7] - goal[7 * a + 1], dz = Tee[11] - goal[7 * a + 2];
    c->dist_now[a] = sqrt(dx * dx + dy * dy + dz * dz);
  }
  for (int a = 0; a < A; ++a)
    for (int i = 0; i < A; ++i)
      c->alpha[a * A + i] = (i != a && c->valid[0][i])
          ? orc_priority(c->dist_now[a], c->dist[0][i], p->tau, p->dist_floor, p->prio_min, p->prio_max)
          : 0.0;
  for (int a = 0; a < A; ++a) {
    const orc_arm *arm = &c->arms[a];
    int d = arm->dof, H = arm->horizon, S = arm->n_spheres;
    int n0 = c->n_lo < arm->n_rollouts ? c->n_lo : arm->n_rollouts;
    int n1 = c->n_hi < arm->n_rollouts ? c->n_hi : arm->n_rollouts;
    int N = n1 - n0;
    double *mu = c->mu + a * Hm * d;
    const double *st = state + (size_t)a * c->dof * 3;
    double q0[ORC_MAX_DOF], qd0[ORC_MAX_DOF];
    for (int j = 0; j < d; ++j) { q0[j] = st[3 * j]; qd0[j] = st[3 * j + 1]; }
    orc_shift(H, d, mu);
    /* phi = (mu, Sigma): the covariances (and their factors) shift too. */
    double *sig = c->sig + a * Hm * d * d, *chol = c->chol + a * Hm * d * d;
    orc_shift(H, d * d, sig);
    orc_shift(H, d * d, chol);
    double *U = (double *)malloc(sizeof(double) * N * H * d);
    double *q = (double *)malloc(sizeof(double) * H * d);
    double *qd = (double *)malloc(sizeof(double) * H * d);
    double *sph = (double *)malloc(sizeof(double) * S * 4);
    double *stage = (double *)malloc(sizeof(double) * H);
    double *Ctot = (double *)malloc(sizeof(double) * N);
    double *w = (double *)malloc(sizeof(double) * N);
    double *mt = (double *)malloc(sizeof(double) * H * d);
    const double *nb_plan[ORC_MAX_ARMS];
    int nb_S[ORC_MAX_ARMS], nb_active[ORC_MAX_ARMS];
    double alpha_row[ORC_MAX_ARMS];
    for (int k = 0; k < p->iters; ++k) {
      /* SampleControls: U = mu + eps. */
      for (int n = 0; n < N; ++n)
        for (int h = 0; h < H; ++h) {
          double z[ORC_MAX_DOF];
          orc_normals(p->seed, a, c->t, k, n0 + n, h, d, z);
          const double *L = chol + (size_t)h * d * d;
          for (int j = 0; j < d; ++j) {
            /* eps ~ N(0, Sigma_h): eps = L_h z (sigma z while Sigma = sigma^2 I) */
            double e = 0.0;
            for (int m = 0; m <= j; ++m) e += L[j * d + m] * z[m];
            U[((size_t)n * H + h) * d + j] = mu[h * d + j] + e;
            if (k == p->iters - 1) c->last_eps[(((size_t)a * Nm + n) * Hm + h) * d + j] = e;
          }
        }
      /* Rollout: integrate, forward kinematics, stage costs, total. */
      for (int n = 0; n < N; ++n) {
        orc_integrate(d, H, p->dt, q0, qd0, U + (size_t)n * H * d, q, qd);
        for (int h = 0; h < H; ++h) {
          orc_spheres(arm, q + h * d, sph);
          int m = 0;
          for (int i = 0; i < A; ++i) {
            if (i == a) continue;
            nb_plan[m] = c->plan[0] + ((size_t)i * Hm + h) * Sm * 4;
            nb_S[m] = c->arms[i].n_spheres;
            nb_active[m] = c->valid[0][i] && h < c->arms[i].horizon;
            alpha_row[m] = c->alpha[a * A + i];
            ++m;
          }
          stage[h] = orc_stage_cost(arm, p, H, h, q + h * d, qd + h * d, sph, goal + 7 * a, obs,
                                    n_obs, nb_plan, nb_S, nb_active, alpha_row, m, NULL);
          if (k == p->iters - 1) c->last_stage[((size_t)a * Hm + h) * Nm + n] = stage[h];
        }
        Ctot[n] = orc_total_cost(H, p->gamma, stage);
      }
      /* UpdateDistribution. */
      orc_weights(N, p->lambda, Ctot, w);
      orc_weighted_mean(N, H, d, w, U, mt);
      if (k == p->iters - 1) {
        for (int n = 0; n < N; ++n) {
          c->last_total[(size_t)a * Nm + n] = Ctot[n];
          c->last_w[(size_t)a * Nm + n] = w[n];
        }
        /* PickBest uses the samples of the final iteration. */
        int nb = orc_argmin(N, Ctot);
        for (int j = 0; j < d; ++j) u_out[a * c->dof + j] = U[(size_t)nb * H * d + j];
      }
      if (p->alpha_sigma > 0.0) {
        /* Eq. 3 (Sigma~), Eq. 4 (EMA), then the factor used by the next draw. */
        double *st = (double *)malloc(sizeof(double) * H * d * d);
        orc_weighted_cov(N, H, d, w, U, mt, st);
        for (int i = 0; i < H * d * d; ++i) sig[i] = (1.0 - p->alpha_sigma) * sig[i] + p->alpha_sigma * st[i];
        for (int h = 0; h < H; ++h)
          orc_cholesky_floor(d, sig + (size_t)h * d * d, p->sigma_floor * p->sigma_floor, chol + (size_t)h * d * d);
        free(st);
      }
      orc_ema(H, d, p->alpha_mu, mt, mu);
    }
    to_plan(c, a, st);
    c->dist[1][a] = c->dist_now[a];
    free(U); free(q); free(qd); free(sph); free(stage); free(Ctot); free(w); free(mt);
  }
  c->t += 1;
}

void orc_get_sigma(const orc_ctx *c, int a, double *sig, double *chol) {
  size_t n = (size_t)c->Hmax * c->dof * c->dof;
  if (sig) memcpy(sig, c->sig + a * n, sizeof(double) * n);
  if (chol) memcpy(chol, c->chol + a * n, sizeof(double) * n);
}
void orc_get_mean(const orc_ctx *c, int a, double *mu) {
  memcpy(mu, c->mu + (size_t)a * c->Hmax * c->dof, sizeof(double) * c->Hmax * c->dof);
}
void orc_set_mean(orc_ctx *c, int a, const double *mu) {
  memcpy(c->mu + (size_t)a * c->Hmax * c->dof, mu, sizeof(double) * c->Hmax * c->dof);
}
void orc_get_plan(const orc_ctx *c, int a, int side, double *plan, double *plan_q, double *dist,
                  int *valid) {
  size_t Hm = c->Hmax, Sm = c->Smax, d = c->dof;
  if (plan) memcpy(plan, c->plan[side] + a * Hm * Sm * 4, sizeof(double) * Hm * Sm * 4);
  if (plan_q) memcpy(plan_q, c->plan_q[side] + a * Hm * d, sizeof(double) * Hm * d);
  if (dist) *dist = c->dist[side][a];
  if (valid) *valid = side == 0 ? c->valid[0][a] : c->written[a];
}
void orc_set_plan(orc_ctx *c, int a, const double *plan, const double *plan_q, double dist, int valid) {
  size_t Hm = c->Hmax, Sm = c->Smax, d = c->dof;
  if (plan) memcpy(c->plan[0] + a * Hm * Sm * 4, plan, sizeof(double) * Hm * Sm * 4);
  if (plan_q) memcpy(c->plan_q[0] + a * Hm * d, plan_q, sizeof(double) * Hm * d);
  c->dist[0][a] = dist;
  c->valid[0][a] = valid;
}
void orc_get_costs(const orc_ctx *c, int a, double *total, double *stage, double *weights) {
  size_t Hm = c->Hmax, Nm = c->Nmax;
  if (total) memcpy(total, c->last_total + a * Nm, sizeof(double) * Nm);
  if (weights) memcpy(weights, c->last_w + a * Nm, sizeof(double) * Nm);
  if (stage) memcpy(stage, c->last_stage + a * Hm * Nm, sizeof(double) * Hm * Nm);
}
void orc_get_noise(const orc_ctx *c, int a, double *eps) {
  size_t Hm = c->Hmax, Nm = c->Nmax, d = c->dof;
  memcpy(eps, c->last_eps + a * Nm * Hm * d, sizeof(double) * Nm * Hm * d);
}
void orc_get_alpha(const orc_ctx *c, double *alpha, double *dist_now) {
  if (alpha) memcpy(alpha, c->alpha, sizeof(double) * c->A * c->A);
  if (dist_now) memcpy(dist_now, c->dist_now, sizeof(double) * c->A);
}
uint32_t orc_get_step(const orc_ctx *c) { return c->t; }
void orc_set_step(orc_ctx *c, uint32_t t) { c->t = t; }

/* ------------------------------------------------------------------------
 * Learned arm-pair distance.
 * ---------------------------------------------------------------------- */
/* Exact signed distance between two arms (Eq. 6 over all sphere pairs). */
double orc_arm_pair_rho(const orc_arm *ai, const double *qi, const orc_arm *aj, const double *qj) {
  double si[ORC_MAX_SPHERES * 4], sj[ORC_MAX_SPHERES * 4];
  orc_spheres(ai, qi, si);
  orc_spheres(aj, qj, sj);
  return orc_rho_sets(si, ai->n_spheres, sj, aj->n_spheres);
}

long long orc_mlp_param_count(int L, const int *w) {
  long long n = 0;
  for (int l = 0; l < L; ++l) n += (long long)w[l + 1] * w[l] + w[l + 1];
  return n;
}

/* Plain MLP: a_{l+1} = W_l a_l + b_l, ReLU on every layer but the last.
 * Pinned by: finite differences of the loss (gradient), a hand-computed
 * two-layer case (forward). */
void orc_mlp_forward(int L, const int *w, const double *params, int B, const double *x, double *y) {
  int maxw = 0;
  for (int l = 0; l <= L; ++l) if (w[l] > maxw) maxw = w[l];
  double *a = (double *)malloc(sizeof(double) * maxw), *b = (double *)malloc(sizeof(double) * maxw);
  for (int s = 0; s < B; ++s) {
    for (int i = 0; i < w[0]; ++i) a[i] = x[(size_t)s * w[0] + i];
    const double *P = params;
    for (int l = 0; l < L; ++l) {
      const double *W = P, *bb = P + (size_t)w[l + 1] * w[l];
      for (int o = 0; o < w[l + 1]; ++o) {
        double z = bb[o];
        for (int i = 0; i < w[l]; ++i) z += W[(size_t)o * w[l] + i] * a[i];
        b[o] = (l + 1 < L && z < 0.0) ? 0.0 : z;
      }
      P += (size_t)w[l + 1] * w[l] + w[l + 1];
      double *t = a; a = b; b = t;
    }
    for (int o = 0; o < w[L]; ++o) y[(size_t)s * w[L] + o] = a[o];
  }
  free(a); free(b);
}

/* Loss (reading): mean squared error plus an extra penalty on
 * over-prediction (a predicted distance larger than the true one is the
 * unsafe direction), each sample weighted by 1 + near_w when its target lies
 * below near_band (the region where the skip decision is taken).
 * Backpropagation by the chain rule, layer by layer. */
static double sample_weight(double t, double near_w, double near_band) {
  return t < near_band ? 1.0 + near_w : 1.0;
}

double orc_mlp_loss_grad(int L, const int *w, const double *params, int B, const double *x,
                         const double *t, double over_w, double near_w, double near_band, double *grad) {
  long long np = orc_mlp_param_count(L, w);
  memset(grad, 0, sizeof(double) * np);
  size_t acts = 0;
  for (int l = 0; l <= L; ++l) acts += w[l];
  double *A = (double *)malloc(sizeof(double) * acts);   /* post-activation per layer */
  double *Z = (double *)malloc(sizeof(double) * acts);   /* pre-activation per layer */
  double *D = (double *)malloc(sizeof(double) * acts);   /* dLoss/dZ */
  size_t off[ORC_MAX_DOF * 4];
  size_t po[ORC_MAX_DOF * 4];
  off[0] = 0;
  for (int l = 0; l < L; ++l) off[l + 1] = off[l] + w[l];
  po[0] = 0;
  for (int l = 0; l < L; ++l) po[l + 1] = po[l] + (size_t)w[l + 1] * w[l] + w[l + 1];
  double loss = 0.0;
  for (int s = 0; s < B; ++s) {
    for (int i = 0; i < w[0]; ++i) { A[i] = x[(size_t)s * w[0] + i]; Z[i] = A[i]; }
    for (int l = 0; l < L; ++l) {
      const double *W = params + po[l], *bb = W + (size_t)w[l + 1] * w[l];
      for (int o = 0; o < w[l + 1]; ++o) {
        double z = bb[o];
        for (int i = 0; i < w[l]; ++i) z += W[(size_t)o * w[l] + i] * A[off[l] + i];
        Z[off[l + 1] + o] = z;
        A[off[l + 1] + o] = (l + 1 < L && z < 0.0) ? 0.0 : z;
      }
    }
    double yv = A[off[L]], e = yv - t[s];
    double pos = e > 0.0 ? e : 0.0;
    double om = sample_weight(t[s], near_w, near_band);
    loss += om * (e * e + over_w * pos * pos);
    D[off[L]] = om * (2.0 * e + 2.0 * over_w * pos) / B;
    for (int l = L - 1; l >= 0; --l) {
      const double *W = params + po[l];
      double *gW = grad + po[l], *gb = gW + (size_t)w[l + 1] * w[l];
      for (int o = 0; o < w[l + 1]; ++o) {
        double dz = D[off[l + 1] + o];
        gb[o] += dz;
        for (int i = 0; i < w[l]; ++i) gW[(size_t)o * w[l] + i] += dz * A[off[l] + i];
      }
      if (l > 0) {
        for (int i = 0; i < w[l]; ++i) {
          double s2 = 0.0;
          for (int o = 0; o < w[l + 1]; ++o) s2 += W[(size_t)o * w[l] + i] * D[off[l + 1] + o];
          D[off[l] + i] = Z[off[l] + i] > 0.0 ? s2 : 0.0;
        }
      }
    }
  }
  free(A); free(Z); free(D);
  return loss / B;
}

/* Adam (Kingma and Ba, ICLR 2015), bias-corrected, step counted from 1.
 * Pinned by: the first step moves by lr against the gradient's sign; a
 * constant gradient moves by lr at every step (bias correction exact, steps
 * 1-3); two steps of +1, -1 worked by hand. */
void orc_adam(long long n, double *p, double *m, double *v, const double *g, double lr,
              double b1, double b2, double eps, int step) {
  double c1 = 1.0 - pow(b1, step), c2 = 1.0 - pow(b2, step);
  for (long long i = 0; i < n; ++i) {
    m[i] = b1 * m[i] + (1.0 - b1) * g[i];
    v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
    double mh = m[i] / c1, vh = v[i] / c2;
    p[i] -= lr * mh / (sqrt(vh) + eps);
  }
}

/* Round-to-nearest-even to bfloat16 of the FP32 value of x. */
double orc_bf16(double x) {
  float f = (float)x;
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return x; /* inf / nan */
  uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);
  r &= 0xffff0000u;
  memcpy(&f, &r, 4);
  return (double)f;
}

void orc_mlp_forward_bf16(int L, const int *w, const double *params, int B, const double *x, double *y) {
  int maxw = 0;
  for (int l = 0; l <= L; ++l) if (w[l] > maxw) maxw = w[l];
  double *a = (double *)malloc(sizeof(double) * maxw), *b = (double *)malloc(sizeof(double) * maxw);
  for (int s = 0; s < B; ++s) {
    for (int i = 0; i < w[0]; ++i) a[i] = orc_bf16(x[(size_t)s * w[0] + i]);
    const double *P = params;
    for (int l = 0; l < L; ++l) {
      const double *W = P, *bb = P + (size_t)w[l + 1] * w[l];
      for (int o = 0; o < w[l + 1]; ++o) {
        double z = 0.0;
        for (int i = 0; i < w[l]; ++i) z += orc_bf16(W[(size_t)o * w[l] + i]) * a[i];
        z += bb[o];
        /* a hidden activation enters the next product as bfloat16 */
        b[o] = (l + 1 < L) ? orc_bf16(z < 0.0 ? 0.0 : z) : z;
      }
      P += (size_t)w[l + 1] * w[l] + w[l + 1];
      double *t = a; a = b; b = t;
    }
    for (int o = 0; o < w[L]; ++o) y[(size_t)s * w[L] + o] = a[o];
  }
  free(a); free(b);
}

/* Reduced-precision dataflow of the training kernels (definition above):
 * Z_l = bf(A_{l-1}) bf(W_l)^T + b_l, A_l = relu(Z_l), y = Z_L;
 * dZ_L = dy; dW_l = bf(dZ_l)^T bf(A_{l-1}); db_l = sum dZ_l;
 * dA_{l-1} = bf(dZ_l) bf(W_l); dZ_{l-1} = dA_{l-1} * [Z_{l-1} > 0].
 * Pinned by: equality with the FP64 gradient when every operand is
 * bfloat16-exact; closeness to it otherwise; every forward and backward
 * rounding point on a 1-1-1 chain worked by hand. */
double orc_mlp_loss_grad_bf16(int L, const int *w, const double *params, int B, const double *x,
                              const double *t, double over_w, double near_w, double near_band, double *grad) {
  long long np = orc_mlp_param_count(L, w);
  memset(grad, 0, sizeof(double) * np);
  double *pb = (double *)malloc(sizeof(double) * np);
  for (long long k = 0; k < np; ++k) pb[k] = orc_bf16(params[k]);
  size_t acts = 0;
  for (int l = 0; l <= L; ++l) acts += w[l];
  double *A = (double *)malloc(sizeof(double) * acts), *Z = (double *)malloc(sizeof(double) * acts);
  double *D = (double *)malloc(sizeof(double) * acts);
  size_t off[32], po[32];
  off[0] = 0;
  for (int l = 0; l < L; ++l) off[l + 1] = off[l] + w[l];
  po[0] = 0;
  for (int l = 0; l < L; ++l) po[l + 1] = po[l] + (size_t)w[l + 1] * w[l] + w[l + 1];
  double loss = 0.0;
  for (int s = 0; s < B; ++s) {
    for (int i = 0; i < w[0]; ++i) { A[i] = orc_bf16(x[(size_t)s * w[0] + i]); Z[i] = A[i]; }
    for (int l = 0; l < L; ++l) {
      const double *W = pb + po[l], *bb = params + po[l] + (size_t)w[l + 1] * w[l];
      for (int o = 0; o < w[l + 1]; ++o) {
        double z = 0.0;
        for (int i = 0; i < w[l]; ++i) z += W[(size_t)o * w[l] + i] * A[off[l] + i];
        z += bb[o];
        Z[off[l + 1] + o] = z;
        /* hidden activations enter the next product as bfloat16 */
        A[off[l + 1] + o] = (l + 1 < L) ? orc_bf16(z < 0.0 ? 0.0 : z) : z;
      }
    }
    double e = A[off[L]] - t[s], pos = e > 0.0 ? e : 0.0;
    double om = sample_weight(t[s], near_w, near_band);
    loss += om * (e * e + over_w * pos * pos);
    D[off[L]] = om * (2.0 * e + 2.0 * over_w * pos) / B;
    for (int l = L - 1; l >= 0; --l) {
      const double *W = pb + po[l];
      double *gW = grad + po[l], *gb = gW + (size_t)w[l + 1] * w[l];
      for (int o = 0; o < w[l + 1]; ++o) {
        double dz = D[off[l + 1] + o], dzb = orc_bf16(dz);
        gb[o] += dz;
        for (int i = 0; i < w[l]; ++i) gW[(size_t)o * w[l] + i] += dzb * A[off[l] + i];
      }
      if (l > 0) {
        for (int i = 0; i < w[l]; ++i) {
          double s2 = 0.0;
          for (int o = 0; o < w[l + 1]; ++o) s2 += W[(size_t)o * w[l] + i] * orc_bf16(D[off[l + 1] + o]);
          D[off[l] + i] = Z[off[l] + i] > 0.0 ? s2 : 0.0;
        }
      }
    }
  }
  free(pb); free(A); free(Z); free(D);
  return loss / B;
}

/* Canonical frame of arm a: apply the inverse of a's base transform to both
 * arms.  Arm a then stands at the origin with no yaw; arm i stands at
 * Rz(-yaw_a)(b_i - b_a) with yaw yaw_i - yaw_a, and because the first joint
 * turns about the base z axis (a_0 = alpha_0 = 0), that yaw adds to q_i[0]
 * (pinned by the base-yaw test of the kinematics). */
void orc_pair_features(const orc_arm *a, const double *qa, const orc_arm *i, const double *qi, double *f) {
  const double pi = 3.14159265358979323846;
  for (int j = 0; j < 7; ++j) {
    double mid = 0.5 * (a->qlim[j][0] + a->qlim[j][1]), half = 0.5 * (a->qlim[j][1] - a->qlim[j][0]);
    f[j] = (qa[j] - mid) / half;
  }
  double q0 = qi[0] + (i->base[3] - a->base[3]);
  q0 = fmod(q0 + pi, 2.0 * pi);
  if (q0 < 0.0) q0 += 2.0 * pi;
  f[7] = (q0 - pi) / pi;
  for (int j = 1; j < 7; ++j) {
    double mid = 0.5 * (a->qlim[j][0] + a->qlim[j][1]), half = 0.5 * (a->qlim[j][1] - a->qlim[j][0]);
    f[7 + j] = (qi[j] - mid) / half;
  }
  double dx = i->base[0] - a->base[0], dy = i->base[1] - a->base[1], dz = i->base[2] - a->base[2];
  double c = cos(a->base[3]), s = sin(a->base[3]);
  f[14] = c * dx + s * dy;
  f[15] = -s * dx + c * dy;
  f[16] = dz;
}
