// Kernel argument blocks and launchers of the MR-STORM step (host side view).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace mrs {

struct RolloutArgs {
  const DevArm* arms;
  const Params* P;
  const StepState* ss;
  const Item* items;
  int n_items;
  int k;                       // optimisation iteration
  int pad;
  const float* mu;             // [A][Hmax][7]
  const float* eps;            // the iteration's noise, per-arm [H][7][Npad] blocks (k_noise)
  float* partial;              // stage costs [A][kMaxH][Nmax] (step-major)
  const float* state;          // staged [A][7][3]
  const float* goal;           // staged [A][7]
  const float* goalR;          // [A][9]
  const float* obs;            // staged [O][4]
  const float* plan_read;      // [A][Hmax][Smax][4]
  // debug capture (only read by the capturing instantiation)
  float* dbg_q;                // [A][Nmax][Hmax][7]
  float* dbg_qd;
  float* dbg_sph;              // [A][Nmax][Hmax][Smax][4]
  float* dbg_stage;            // [A][Hmax][Nmax]
  unsigned long long* dbg_pairs;  // [A][4]: queries, set filter passes, set exact passes, self exact passes (per wave)
  // learned distance (collision mode 1, `learned` set): the network's
  // predictions in inference-descriptor order, the first descriptor of each
  // (arm, neighbour, step) group [A][A][Hmax] (-1: no prediction, the group's
  // queries are checked exactly), the own-feature rows (slot 7 = in-box flag)
  // and neighbour records (word 5 bit 0 = neighbour in box), the margin, and
  // the counters [A][kSurCounters]; the debug instantiation also stores each live
  // query's prediction (NaN without one) and decision (1 far, 0 near, 2 no
  // prediction) [A][A][Hmax][Nmax]
  int learned;
  int audit;
  const float* sur_y;
  const int* sur_grp;
  const uint16_t* sur_F;
  const uint32_t* sur_rec;
  float sur_margin;
  int pad2;
  unsigned long long* sur_counts;
  unsigned* sur_hist;          // dropped checks per group, [2][A][A][Hmax] by step parity (NULL: not counted)
  float* dbg_pred;
  uint8_t* dbg_skip;
  // C_manip of every (arm, step, rollout) [A][Hmax][Nmax], or NULL (w_manip = 0)
  const float* manip;
};

struct SenseArgs {
  const DevArm* arms;
  const Params* P;
  StepState* ss;
  const BoardMeta* meta;
  const float* state;          // caller [A][7][3]
  const float* goal;           // caller [A][7]
  const float* obstacles;      // caller [O][4]
  int n_obs;
  uint32_t t;
  float* u_out;                // caller [A][7], written by k_softmax (PickBest / Act)
  float* st_state;
  float* st_goal;
  float* st_obs;
  float* goalR;
  float* mu;
  float* sig;                  // [A][Hmax][28] packed lower triangles (covariance adaptation)
  float* chol;                 // their Cholesky factors
};

struct ReduceArgs {
  const DevArm* arms;
  const Params* P;
  const StepState* ss;
  int pad;
  const float* partial;        // stage costs [A][kMaxH][Nmax]
  float* cost;                 // [A][Nmax]
  float* w;                    // [A][Nmax]
  const float* eps;
  float* mu;
  float* u_out;                // [A][7] staged copy (debug capture); the caller's array is ss->u_out
  int* argmin;                 // [A]
  const float* st_state;
  float* plan_write;
  float* planq_write;
  BoardMeta* meta;
  float* sig;                  // [A][Hmax][28] packed lower triangles (covariance adaptation)
  float* chol;                 // their Cholesky factors
  float* wpart;                // weighted-mean partial sums [A][Hmax][kWmeanMaxChunks][7 + 28]
};

// The weighted mean (Eq. 3) splits every (arm, step) over chunks of
// kWmeanChunk rollouts (256 threads x 4 consecutive rollouts).
constexpr int kWmeanChunk = 1024;
constexpr int kWmeanMaxChunks = 16;   // 16384 rollouts
constexpr int kWmeanSums = 7 + 28;

struct PublishArgs {
  const float* plan_write;
  const float* planq_write;
  float* plan_read;
  float* planq_read;
  BoardMeta* meta;
  uint32_t mask;
  int Hmax, Smax;
};

hipError_t launch_sense(const SenseArgs& A, hipStream_t s);
// waves: 64-rollout waves per workgroup (1, 2 or 4); every arm's padded
// rollout count must be a multiple of 64 * waves.
hipError_t launch_rollout(const RolloutArgs& A, int layout, bool debug, int waves, int grid, hipStream_t s);
// k_total then k_softmax, or for small problems (Nmax x Hmax <= 64 K) k_softmax
// forming the totals itself.
hipError_t launch_softmax(const ReduceArgs& A, int n_arms, int nmax, int hmax, hipStream_t s);
// k_wmean (chunk partials), then with `fin` k_wmean_fin (totals and Eq. 4).
hipError_t launch_wmean(const ReduceArgs& A, int n_arms, int hmax, int nmax, bool fin, hipStream_t s);
// ToPlan; with `fin` it first applies the last iteration's totals and Eq. 4.
hipError_t launch_toplan(const ReduceArgs& A, int n_arms, bool fin, hipStream_t s);
hipError_t launch_publish(const PublishArgs& A, int n_arms, hipStream_t s);
// C_manip (Eq. 5) of every rollout step from the iteration's noise: out [A][Hmax][Nmax].
hipError_t launch_manip(const DevArm* arms, const Params* P, const StepState* ss, const float* mu, const float* state,
                        const float* eps, int n_arms, int npad_max, float* out, hipStream_t s);
// Noise of iteration k for every arm, step and padded rollout: sigma z, or
// L_h z from the adapted covariances' factors when `chol` is non-null.
hipError_t launch_noise(const DevArm* arms, const Params* P, const StepState* ss, const float* chol, float* eps, int k,
                        int n_arms, int hmax, int npad_max, hipStream_t s);
hipError_t launch_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out, int n, hipStream_t s);
hipError_t launch_sim_execute(float* state, const float* u, int n, float dt, hipStream_t s);
hipError_t launch_copy3d(const float* src, long long s0, long long s1, long long s2, float* dst,
                         long long d0, long long d1, long long d2, int n0, int n1, int n2, hipStream_t s);
hipError_t launch_set_meta(BoardMeta* meta, int arm, float dist, int valid, hipStream_t s);

}  // namespace mrs
