// Data layouts shared by the host runtime and the gfx950 kernels of the
// MR-STORM control step.  Everything here is plain old data copied to HBM.
#pragma once
#include <stdint.h>

namespace mrs {

constexpr int kMaxArms = 8;
constexpr int kMaxDof = 8;
constexpr int kMaxSpheres = 64;
constexpr int kBodies = 8;            // 7 links + hand for the 7-DoF tables
constexpr int kMaxPerBody = 8;
constexpr int kMaxH = 64;
constexpr int kMaxObs = 64;
constexpr int kWave = 64;
// Learned-distance counters per arm: live queries, predicted far, dropped
// 64-rollout checks, audited misses (< B), audited missed collisions (< 0),
// query rows run through the network.
constexpr int kSurCounters = 6;

// Sphere layouts compiled into the rollout kernel: spheres sorted by body,
// `count[b]` slots per body.  Layout 0 = the 52-sphere tiling (4,6,6,6,8,6,8,8),
// layout 1 = up to 8 per body (64 slots; unused slots are parked far away).
constexpr int kLayoutCount[2][kBodies] = {{4, 6, 6, 6, 8, 6, 8, 8}, {8, 8, 8, 8, 8, 8, 8, 8}};
constexpr int kLayoutStart[2][kBodies + 1] = {{0, 4, 10, 16, 22, 30, 36, 44, 52},
                                              {0, 8, 16, 24, 32, 40, 48, 56, 64}};
constexpr int kLayoutSlots[2] = {52, 64};

struct DevArm {
  int dof, S, N, H;            // joints, real spheres, rollouts, horizon
  int Npad, layout, pad0, pad1;
  float a[kMaxDof], cal[kMaxDof], sal[kMaxDof], d[kMaxDof], off[kMaxDof];
  float qlo[kMaxDof], qhi[kMaxDof], qdmax[kMaxDof];
  float base[4];               // x, y, z, unused
  float cyaw, syaw, pad2, pad3;
  float tool[4];
  float slot[kMaxSpheres][4];  // body-frame spheres in kernel slot order
  int slot_src[kMaxSpheres];   // user index of each slot, -1 = parked
  int link[kMaxSpheres];       // body of each user-order sphere
  float usph[kMaxSpheres][4];  // body-frame spheres in user order
  // Bounding sphere of each body's spheres: centre in the body frame (xyz)
  // and radius (w) = largest centre offset from it + largest sphere radius,
  // rounded up; w < 0 marks a body without spheres.
  float bnd[kBodies][4];
  // The same for each half of a body's slots (slots [0, (C+1)/2) and the
  // rest of the body's C slots; parked slots left out); w < 0: no spheres.
  float hb[kBodies][2][4];
  long long eps_off;           // float offset of this arm's [H][d][Npad] noise block
};

// One unit of rollout work: 64*waves rollouts of one arm over steps [h0, h1).
struct Item {
  int arm, block, h0, h1;
};

// Neighbour entry of the per-step table built at Sense.
struct Nb {
  int arm, S, H, pad;
  float alpha, pad1, pad2, pad3;
};

struct Params {
  float dt, sigma, lambda, gamma, alpha_mu;
  float w_pose, w_rot, w_stop, w_joint, w_coll, w_dyn;
  float buf_env, buf_self, buf_dyn, tau, prio_min, prio_max, dist_floor, joint_margin;
  float alpha_sigma, sigma_floor;
  float w_manip, manip_thresh;
  uint32_t seed_lo, seed_hi;
  int iters, A, dof, Hmax, Smax, Nmax, max_obs;
  int plan_mode, cov;          // cov: covariance adaptation on (alpha_sigma > 0)
  float gpow[kMaxH];           // gamma^h rounded to FP32
};

// Packed lower triangle of a 7x7 symmetric matrix: entry (j, m), m <= j.
__host__ __device__ constexpr int tri7(int j, int m) { return j * (j + 1) / 2 + m; }
constexpr int kTri = 28;

// Per-step device scalars written at Sense.
struct StepState {
  uint32_t t;                  // control step counter (noise stream)
  int n_obs;
  float* u_out;                // the caller's U* array [A][7] of this step (device)
  float dist_now[kMaxArms];
  int nb_count[kMaxArms];
  Nb nb[kMaxArms][kMaxArms];
  float alpha[kMaxArms][kMaxArms];
};

// Plan board: side 0 = read (what Sense sees), side 1 = write (ToPlan).
struct BoardMeta {
  float dist[2][kMaxArms];
  int valid[2][kMaxArms];      // side 1: "written since init"
};

}  // namespace mrs
