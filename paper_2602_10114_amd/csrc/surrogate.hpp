// Learned arm-pair distance: kernel arguments and launchers (host view).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace mrs {

// MLP 17 -> 256 -> 256 -> 256 -> 1, ReLU on the hidden layers.  FP32 master
// parameters packed per layer as W[out][in] then b[out].
constexpr int kFeat = 17;
constexpr int kHid = 256;
constexpr int kMlpLayers = 4;
constexpr int kMlpWidth[kMlpLayers + 1] = {kFeat, kHid, kHid, kHid, 1};
constexpr long long kMlpParams = 17LL * 256 + 256 + 256LL * 256 + 256 + 256LL * 256 + 256 + 256 + 1;

__host__ __device__ constexpr long long mlp_w_off(int l) {
  long long o = 0;
  for (int i = 0; i < l; ++i) o += (long long)kMlpWidth[i + 1] * kMlpWidth[i] + kMlpWidth[i + 1];
  return o;
}
__host__ __device__ constexpr long long mlp_b_off(int l) {
  return mlp_w_off(l) + (long long)kMlpWidth[l + 1] * kMlpWidth[l];
}

// Joint normalisation of the arm model (shared by every arm of a context).
struct SurModel {
  float mid[7], inv_half[7];
  float margin;                // predictions below this are checked exactly
  float screen;                // mean-rollout distance below which a group skips the network (0 = off)
  int probe;                   // drop-history screen: re-probe period in control steps (0 = off)
  float min_drop;              // share of a group's checks dropped at or below which it goes quiet
};
// Drop history of a group with no history yet (never ran the network, or
// screened for another reason); otherwise the count of dropped checks.
constexpr unsigned kHistNone = 0x80000000u;

// GEMM: C[m][n] = sum_k A(m,k) B(k,n) over bfloat16 operands, FP32 sum.
// A(m,k) = transA ? A[k*lda + m] : A[m*lda + k]; B(k,n) = transB ? B[n*ldb + k] : B[k*ldb + n].
// Epilogue: z = acc (+ bias[n]); if mask: z *= (mask[m*ldm+n] > 0);
// C32[m*ldc+n] = z (if C32); C16[m*ldc16+n] = bf16(relu ? max(z,0) : z) (if C16).
struct GemmArgs {
  int M, N, K;
  const uint16_t* A;
  int lda, transA;
  const uint16_t* B;
  int ldb, transB;
  const float* bias;
  const float* mask;
  int ldm;
  int relu;
  float* C32;
  int ldc;
  uint16_t* C16;
  int ldc16;
};

// One inference work item: 32 consecutive rollouts of `arm` at step h against
// the plan of neighbour `nbr`.
struct SurItem {
  int arm, nbr, h, n0;
};

// Neighbour record of the fused inference, kNbrRec words per (arm a,
// neighbour i, step h) of the read-side plans: [0..3] bfloat16 pairs
// (f7,f8) .. (f13,f14), [4] (f15,f16), [5] flags (bit 0: the neighbour's
// joints lie in the training box; bit 1: i != a, its plan is on the read
// side and covers step h), [6] N of arm a, [7] padded N of arm a.
constexpr int kNbrRec = 8;

struct SurInferArgs {
  const Params* P;
  const SurModel* model;
  const uint16_t* W16;         // bfloat16 parameters (same packing as the FP32 master)
  const float* P32;            // FP32 parameters (biases are taken in FP32)
  const uint16_t* F;           // own-joint feature rows [A][Hmax][Nmax][8] (bfloat16, slot 7 = in-box flag)
  const uint32_t* nbrec;       // neighbour records [A][A][Hmax][kNbrRec]
  const SurItem* items;        // this step's descriptors (k_sur_states)
  const int* count;            // their number (device)
  float* y;                    // predictions in descriptor order [descriptors][32]
};

hipError_t launch_gemm_bf16(const GemmArgs& g, hipStream_t s);
hipError_t launch_pair_distance(int layout, const DevArm* arms, int ai, int aj, const float* qi, const float* qj,
                                int M, float* out, hipStream_t s);
// The iteration's noise (as launch_noise) and the screen flag of every
// (arm, neighbour, step) group ([A][A][Hmax], 1: the group needs no
// prediction) in one launch.  hist: the groups' drop history of the last two
// control steps [2][A][A][Hmax] (step parity; 0 = ran the network or stayed
// quiet and dropped nothing); the previous step's is read, the current
// step's started in iteration 0.
hipError_t launch_noise_screen(const DevArm* arms, const Params* P, const StepState* ss, const float* chol,
                               float* eps, int k, int n_arms, int hmax, int npad_max, const SurModel* model,
                               const BoardMeta* meta, const float* mu, const float* state, const float* plan_read,
                               uint8_t* screened, unsigned* hist, hipStream_t s);
// Own-feature rows of every (arm, step, rollout) from the iteration's noise
// `eps`, the neighbour records of every (a, i, h < Hmax) from the read-side
// plans, and this step's inference descriptors from the screen flags (groups
// in (arm, neighbour, step) order) with each group's first descriptor
// [A][A][Hmax] (-1: none) and their number, in one launch.
hipError_t launch_sur_states(const DevArm* arms, const Params* P, const SurModel* model, const float* mu,
                             const float* state, const float* eps, int n_arms, int npad_max, int hmax, uint16_t* F,
                             const BoardMeta* meta, const float* planq, uint32_t* rec, const uint8_t* screened,
                             SurItem* items, int* grp_first, int* count, unsigned long long* counts,
                             hipStream_t s);
hipError_t launch_sur_infer(const SurInferArgs& A, int grid, hipStream_t s);
// Training samples: arm pairs drawn from `pairs` ([n_pairs][2] arm indices),
// joints uniform within the limits (counter-based draws keyed by seed);
// features (bfloat16 [M][17]), FP32 targets max(min(rho, clip), floor), and
// the joints (FP32 [M][14], optional).
hipError_t launch_sur_sample_layout(int layout, const DevArm* arms, const SurModel* model, const int* pairs,
                                    int n_pairs, uint32_t seed_lo, uint32_t seed_hi, long long first, int M,
                                    float clip, float floor_, uint16_t* X16, float* T, float* Q, hipStream_t s);
hipError_t launch_features(const DevArm* arms, const SurModel* model, int ai, int aj, const float* qi,
                           const float* qj, int M, float* F, hipStream_t s);
hipError_t launch_loss(const float* y, const float* t, int B, float over_w, float near_w, float near_band, float* dy,
                       uint16_t* dy16, float* loss_acc, hipStream_t s);
hipError_t launch_colsum(const float* X, int M, int N, float* out, hipStream_t s);
hipError_t launch_adam(float* p, float* m, float* v, const float* g, long long n, float lr, float b1, float b2,
                       float eps, int step, hipStream_t s);
hipError_t launch_params_to_bf16(const float* p, uint16_t* p16, long long n, hipStream_t s);
hipError_t launch_init_params(float* p, uint32_t seed_lo, uint32_t seed_hi, hipStream_t s);
hipError_t launch_f32_to_bf16(const float* x, uint16_t* y, long long n, hipStream_t s);

}  // namespace mrs
