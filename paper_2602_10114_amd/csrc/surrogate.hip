// gfx950 kernels of the learned arm-pair distance:
//   exact signed distance between two arms (Eq. 6 over all sphere pairs),
//   Philox-drawn training samples, a bfloat16 MFMA GEMM with fused epilogues
//   for training, loss / column sums / Adam, and the fused MLP inference that
//   decides, per (rollout, step, neighbour), whether the exact check can be
//   skipped.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "device.hpp"
#include "surrogate.hpp"

namespace mrs {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

__device__ __forceinline__ bf16x8_t load_bf16x8(const uint16_t* p) {  // 16-byte aligned
  const uint4 v = *reinterpret_cast<const uint4*>(p);
  bf16x8_t r;
  __builtin_memcpy(&r, &v, sizeof(r));
  return r;
}

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

// FP32 -> bfloat16 with gfx950's conversion instruction (round to nearest
// even); the pair form packs a (low half) and b (high half) in one instruction.
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ uint32_t f2bf2(float a, float b) {
  const bf16x2_t v = {(__bf16)a, (__bf16)b};
  return __builtin_bit_cast(uint32_t, v);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ---------------------------------------------------------------------------
// Exact signed distance between two arms: min over sphere pairs of
// |c_i - c_j| - r_i - r_j.  One lane per sample; arm j's spheres go to a
// per-lane column of LDS, arm i's are produced body by body.
constexpr float kFar = 1.0e9f;

template <int LAY>
__device__ float pair_rho_lane(const DevArm* __restrict__ ai, const float qi[8], const DevArm* __restrict__ aj,
                               const float qj[8], float4 (*col)[kWave], int lane) {
  {
    Frame W;
    frame_base(W, aj);
#pragma unroll
    for (int b = 0; b < kBodies; ++b) {
      if (b < 7) {
        float s, c;
        sincosf(qj[b] + aj->off[b], &s, &c);
        frame_joint(W, aj->a[b], aj->cal[b], aj->sal[b], aj->d[b], c, s);
      }
      for (int j = kLayoutStart[LAY][b]; j < kLayoutStart[LAY][b + 1]; ++j) {
        const float* p = aj->slot[j];
        float x, y, z;
        frame_point(W, p[0], p[1], p[2], x, y, z);
        col[j][lane] = p[3] < 0.f ? make_float4(kFar, kFar, kFar, 0.f) : make_float4(x, y, z, p[3]);
      }
    }
  }
  float best = 3.0e38f;
  Frame W;
  frame_base(W, ai);
#pragma unroll
  for (int b = 0; b < kBodies; ++b) {
    if (b < 7) {
      float s, c;
      sincosf(qi[b] + ai->off[b], &s, &c);
      frame_joint(W, ai->a[b], ai->cal[b], ai->sal[b], ai->d[b], c, s);
    }
    for (int j = kLayoutStart[LAY][b]; j < kLayoutStart[LAY][b + 1]; ++j) {
      const float* p = ai->slot[j];
      if (p[3] < 0.f) continue;
      float x, y, z;
      frame_point(W, p[0], p[1], p[2], x, y, z);
      float m = 3.0e38f;
      for (int k = 0; k < kLayoutSlots[LAY]; ++k) {
        const float4 o = col[k][lane];
        const float dx = x - o.x, dy = y - o.y, dz = z - o.z;
        const float d = sqrtf(fmaf_(dx, dx, fmaf_(dy, dy, dz * dz))) - o.w;
        m = fminf(m, d);
      }
      best = fminf(best, m - p[3]);
    }
  }
  return best;
}

template <int LAY>
__global__ __launch_bounds__(kWave) void k_pair_distance(const DevArm* __restrict__ arms, int ai, int aj,
                                                         const float* __restrict__ qi,
                                                         const float* __restrict__ qj, int M,
                                                         float* __restrict__ out) {
  __shared__ float4 col[kMaxSpheres][kWave];
  const int lane = threadIdx.x;
  const int m = blockIdx.x * kWave + lane;
  const int mm = m < M ? m : M - 1;
  float a[8], b[8];
#pragma unroll
  for (int j = 0; j < 7; ++j) {
    a[j] = qi[(size_t)mm * 7 + j];
    b[j] = qj[(size_t)mm * 7 + j];
  }
  a[7] = b[7] = 0.f;
  const float r = pair_rho_lane<LAY>(arms + ai, a, arms + aj, b, col, lane);
  if (m < M) out[m] = r;
}

// Features of the learned distance (arm `a` own at qa, neighbour `i` at qi),
// in arm a's base frame: the base yaw difference folds into the neighbour's
// first joint (first joint axis = base z), the base offset is rotated into a.
__device__ __forceinline__ void pair_features(const DevArm* __restrict__ a, const float qa[8],
                                              const DevArm* __restrict__ i, const float qi[8],
                                              const SurModel* __restrict__ sm, float f[kFeat]) {
  const float kPi = 3.14159265358979f;
#pragma unroll
  for (int j = 0; j < 7; ++j) f[j] = (qa[j] - sm->mid[j]) * sm->inv_half[j];
  float q0 = qi[0] + (i->base[3] - a->base[3]);
  q0 = q0 - 6.28318530717959f * floorf((q0 + kPi) * 0.159154943091895f);
  f[7] = q0 * 0.318309886183791f;
#pragma unroll
  for (int j = 1; j < 7; ++j) f[7 + j] = (qi[j] - sm->mid[j]) * sm->inv_half[j];
  const float dx = i->base[0] - a->base[0], dy = i->base[1] - a->base[1], dz = i->base[2] - a->base[2];
  f[14] = fmaf_(a->cyaw, dx, a->syaw * dy);
  f[15] = fmaf_(-a->syaw, dx, a->cyaw * dy);
  f[16] = dz;
}

__global__ void k_features(const DevArm* __restrict__ arms, const SurModel* __restrict__ sm, int ai, int aj,
                           const float* __restrict__ qi, const float* __restrict__ qj, int M,
                           float* __restrict__ F) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  float a[8], b[8], f[kFeat];
  for (int j = 0; j < 7; ++j) {
    a[j] = qi[(size_t)m * 7 + j];
    b[j] = qj[(size_t)m * 7 + j];
  }
  a[7] = b[7] = 0.f;
  pair_features(arms + ai, a, arms + aj, b, sm, f);
  for (int k = 0; k < kFeat; ++k) F[(size_t)m * kFeat + k] = f[k];
}

// Training samples.  Counter (sample low, sample high, draw c, 0x5A000000):
// word 0 of draw 0 picks the pair, the other 15 words give the 14 joints.
template <int LAY>
__global__ __launch_bounds__(kWave) void k_sur_sample(const DevArm* __restrict__ arms,
                                                      const SurModel* __restrict__ sm,
                                                      const int* __restrict__ pairs, int n_pairs,
                                                      uint32_t slo, uint32_t shi, long long first, int M,
                                                      float clip, float floor_, uint16_t* __restrict__ X16,
                                                      float* __restrict__ T, float* __restrict__ Q) {
  __shared__ float4 col[kMaxSpheres][kWave];
  const int lane = threadIdx.x;
  const long long m = (long long)blockIdx.x * kWave + lane;
  const long long s = first + (m < M ? m : M - 1);
  uint32_t w[16];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    uint32_t c0 = (uint32_t)s, c1 = (uint32_t)(s >> 32), c2 = (uint32_t)c, c3 = 0x5A000000u;
    philox4x32_10(c0, c1, c2, c3, slo, shi);
    w[4 * c] = c0;
    w[4 * c + 1] = c1;
    w[4 * c + 2] = c2;
    w[4 * c + 3] = c3;
  }
  const int p = (int)(w[0] % (uint32_t)n_pairs);
  const DevArm* A = arms + pairs[2 * p];
  const DevArm* B = arms + pairs[2 * p + 1];
  float qa[8], qb[8];
#pragma unroll
  for (int j = 0; j < 7; ++j) {
    qa[j] = fmaf_(A->qhi[j] - A->qlo[j], unit_open(w[1 + j]), A->qlo[j]);
    qb[j] = fmaf_(B->qhi[j] - B->qlo[j], unit_open(w[8 + j]), B->qlo[j]);
  }
  qa[7] = qb[7] = 0.f;
  const float r = pair_rho_lane<LAY>(A, qa, B, qb, col, lane);
  float f[kFeat];
  pair_features(A, qa, B, qb, sm, f);
  if (m < M) {
#pragma unroll
    for (int k = 0; k < kFeat; ++k) X16[m * kFeat + k] = f2bf(f[k]);
    T[m] = fmaxf(fminf(r, clip), floor_);
    if (Q) {
#pragma unroll
      for (int j = 0; j < 7; ++j) {
        Q[m * 14 + j] = qa[j];
        Q[m * 14 + 7 + j] = qb[j];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// bfloat16 MFMA GEMM, 64x64 tile per 256-thread block (4 waves, one 32x32
// sub-tile each), K in steps of 32 through LDS, FP32 accumulation.  Both
// operands are staged k-contiguous ([row][k] and [col][k]) so that every MFMA
// operand is one 16-byte LDS read; global reads are 16-byte vectors along
// the contiguous dimension when the tile is in bounds and aligned, element
// reads with zero fill otherwise.
constexpr int kGemmLd = 32 + 8;

__device__ __forceinline__ bool vec_ok(const uint16_t* base, int ld, int lim_row, int lim_col, int row, int col) {
  return ((reinterpret_cast<uintptr_t>(base) & 15) == 0) && (ld & 7) == 0 && row < lim_row && col + 8 <= lim_col;
}

// Stage a 64 (rows r) x 32 (k) tile of X(r, k) into S[r][k].  X(r, k) =
// trans ? X[k*ld + r] : X[r*ld + k]; R, Kd bound r and k.
__device__ __forceinline__ void stage_tile(uint16_t (*S)[kGemmLd], const uint16_t* __restrict__ X, int ld, int trans,
                                           int r0, int k0, int R, int Kd, int tid) {
  if (!trans) {
    // 64 rows x 4 vectors of 8 k
    const int r = tid >> 2, kv = (tid & 3) * 8;
    const int gr = r0 + r, gk = k0 + kv;
    if (vec_ok(X, ld, R, Kd, gr, gk)) {
      *reinterpret_cast<uint4*>(&S[r][kv]) = *reinterpret_cast<const uint4*>(X + (size_t)gr * ld + gk);
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e)
        S[r][kv + e] = (gr < R && gk + e < Kd) ? X[(size_t)gr * ld + gk + e] : (uint16_t)0;
    }
  } else {
    // 32 k x 8 vectors of 8 rows
    const int k = tid >> 3, rv = (tid & 7) * 8;
    const int gk = k0 + k, gr = r0 + rv;
    uint16_t v[8];
    if (vec_ok(X, ld, Kd, R, gk, gr)) {
      const uint4 u = *reinterpret_cast<const uint4*>(X + (size_t)gk * ld + gr);
      const uint32_t w4[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = (uint16_t)(w4[e >> 1] >> ((e & 1) * 16));
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = (gk < Kd && gr + e < R) ? X[(size_t)gk * ld + gr + e] : (uint16_t)0;
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) S[rv + e][k] = v[e];
  }
}

__global__ __launch_bounds__(256) void k_gemm_bf16(GemmArgs g) {
  __shared__ uint16_t As[64][kGemmLd];
  __shared__ uint16_t Bs[64][kGemmLd];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  f32x16_t acc;
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = 0.f;
  // B(k, n): stored [n][k] when transB, so it stages like a non-transposed A.
  for (int k0 = 0; k0 < g.K; k0 += 32) {
    stage_tile(As, g.A, g.lda, g.transA, m0, k0, g.M, g.K, tid);
    stage_tile(Bs, g.B, g.ldb, !g.transB, n0, k0, g.N, g.K, tid);
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 32; kk += 16) {
      const bf16x8_t a = load_bf16x8(&As[wm + (lane & 31)][kk + (lane >> 5) * 8]);
      const bf16x8_t b = load_bf16x8(&Bs[wn + (lane & 31)][kk + (lane >> 5) * 8]);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int m = m0 + wm + (i >> 2) * 8 + (lane >> 5) * 4 + (i & 3);
    const int n = n0 + wn + (lane & 31);
    if (m < g.M && n < g.N) {
      float z = acc[i];
      if (g.bias) z += g.bias[n];
      if (g.mask && !(g.mask[(size_t)m * g.ldm + n] > 0.f)) z = 0.f;
      if (g.C32) g.C32[(size_t)m * g.ldc + n] = z;
      if (g.C16) g.C16[(size_t)m * g.ldc16 + n] = f2bf(g.relu ? fmaxf(z, 0.f) : z);
    }
  }
}

// Loss (mean of om(t) [e^2 + w max(e,0)^2], e = y - t, om = 1 + near_w below
// near_band) and dLoss/dy; one block, fixed reduction order.
__global__ __launch_bounds__(1024) void k_loss(const float* __restrict__ y, const float* __restrict__ t, int B,
                                               float over_w, float near_w, float near_band, float* __restrict__ dy,
                                               uint16_t* __restrict__ dy16, float* __restrict__ loss_acc) {
  __shared__ float red[1024];
  const int tid = threadIdx.x;
  float acc = 0.f;
  const float invB = 1.0f / (float)B;
  for (int i = tid; i < B; i += blockDim.x) {
    const float e = y[i] - t[i], pos = fmaxf(e, 0.f);
    const float om = t[i] < near_band ? 1.f + near_w : 1.f;
    acc = fmaf_(om, fmaf_(e, e, over_w * pos * pos), acc);
    const float d = om * (2.f * e + 2.f * over_w * pos) * invB;
    dy[i] = d;
    dy16[i] = f2bf(d);
  }
  red[tid] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  if (tid == 0) *loss_acc += red[0] * invB;
}

// out[n] = sum over rows of X[m][n] (bias gradients).  A block owns 64
// columns; its 16 row groups each sum every 16th row in order, then the 16
// partial sums are added in group order (fixed reduction order).
constexpr int kColsumCols = 64, kColsumGroups = 16;
__global__ __launch_bounds__(kColsumCols * kColsumGroups) void k_colsum(const float* __restrict__ X, int M, int N,
                                                                         float* __restrict__ out) {
  __shared__ float part[kColsumGroups][kColsumCols];
  const int c = threadIdx.x % kColsumCols, r = threadIdx.x / kColsumCols;
  const int n = blockIdx.x * kColsumCols + c;
  float s = 0.f;
  if (n < N)
    for (int m = r; m < M; m += kColsumGroups) s += X[(size_t)m * N + n];
  part[r][c] = s;
  __syncthreads();
  if (r == 0 && n < N) {
    float t = 0.f;
    for (int g = 0; g < kColsumGroups; ++g) t += part[g][c];
    out[n] = t;
  }
}

// Adam (Kingma and Ba), bias-corrected, step counted from 1.
__global__ void k_adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, long long n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = fmaf_(b1, m[i], (1.f - b1) * gi);
  const float vi = fmaf_(b2, v[i], (1.f - b2) * gi * gi);
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_to_bf16(const float* __restrict__ x, uint16_t* __restrict__ y, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = f2bf(x[i]);
}

// Weights and biases uniform in +-1/sqrt(fan_in) (fan_in = the layer's input
// width); counter (index, 0, 0, 0x5B000000).
__global__ void k_init_params(float* __restrict__ p, uint32_t slo, uint32_t shi) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kMlpParams) return;
  int l = 0;
  while (l + 1 < kMlpLayers && i >= mlp_w_off(l + 1)) ++l;
  uint32_t c0 = (uint32_t)i, c1 = 0, c2 = 0, c3 = 0x5B000000u;
  philox4x32_10(c0, c1, c2, c3, slo, shi);
  const float bound = 1.0f / sqrtf((float)kMlpWidth[l]);
  p[i] = (2.f * unit_open(c0) - 1.f) * bound;
}

// ---------------------------------------------------------------------------
// Own-joint features of every (arm, step, rollout) for the learned distance:
// the same noise and integration as the rollout kernel, then the normalised
// joints as one 16-byte row of bfloat16 [f0..f6, in-box flag] (flag 1.0 when
// all seven lie within the training box, else 0.0).
__global__ __launch_bounds__(kWave) void k_sur_states(const DevArm* __restrict__ arms,
                                                      const Params* __restrict__ Pp,
                                                      const SurModel* __restrict__ sm,
                                                      const StepState* __restrict__ ssp,
                                                      const float* __restrict__ mu_all,
                                                      const float* __restrict__ state,
                                                      const float* __restrict__ eps_in, int k_iter,
                                                      uint16_t* __restrict__ F) {
  const Params& P = *Pp;
  const int a = blockIdx.y;
  const DevArm* arm = arms + a;
  const int n = blockIdx.x * kWave + threadIdx.x;
  if (n >= arm->Npad) return;
  const uint32_t t = ssp->t;
  const float* mu = mu_all + (size_t)a * P.Hmax * 7;
  float q[7], qd[7], mid[7], ih[7];
  for (int j = 0; j < 7; ++j) {
    q[j] = state[(a * 7 + j) * 3 + 0];
    qd[j] = state[(a * 7 + j) * 3 + 1];
    mid[j] = sm->mid[j];
    ih[j] = sm->inv_half[j];
  }
  for (int h = 0; h < arm->H; ++h) {
    float z[8];
    if (eps_in) {
      for (int j = 0; j < 7; ++j) z[j] = eps_in[arm->eps_off + ((size_t)h * 7 + j) * arm->Npad + n];
    } else {
      normals8(P.seed_lo, P.seed_hi, a, t, k_iter, n, h, z);
      for (int j = 0; j < 7; ++j) z[j] *= P.sigma;
    }
    uint16_t f[8];
    bool inbox = true;
#pragma unroll
    for (int j = 0; j < 7; ++j) {
      const float u = z[j] + mu[h * 7 + j];
      qd[j] = fmaf_(P.dt, u, qd[j]);
      q[j] = fmaf_(P.dt, qd[j], q[j]);
      const float x = (q[j] - mid[j]) * ih[j];
      inbox = inbox && fabsf(x) <= 1.0f + 1e-3f;
      f[j] = f2bf(x);
    }
    f[7] = inbox ? (uint16_t)0x3F80u : (uint16_t)0u;
    uint4 v;
    v.x = (uint32_t)f[0] | ((uint32_t)f[1] << 16);
    v.y = (uint32_t)f[2] | ((uint32_t)f[3] << 16);
    v.z = (uint32_t)f[4] | ((uint32_t)f[5] << 16);
    v.w = (uint32_t)f[6] | ((uint32_t)f[7] << 16);
    *reinterpret_cast<uint4*>(F + (((size_t)a * P.Hmax + h) * P.Nmax + n) * 8) = v;
  }
}

// Fused MLP inference, weight-stationary.  A block of 2 x kGroupWaves waves
// (one block per CU) streams blocks of 32 queries (32 rollouts of one arm at
// one step against one neighbour's plan) through a pipeline with one barrier
// per stage:
//   group B (the upper kGroupWaves waves) holds kWaveRows rows each of the
//   third layer's weights (and of the first layer's) in registers; at stage
//   s it runs the features and first layer of query block s and the third
//   layer of block s-2;
//   group A holds kWaveRows rows each of the second layer's weights and runs
//   that layer on block s-1, then the output layer and the skip decision of
//   block s-3 (8 lanes per query, reduced in the wave).
// Activations pass between the groups through LDS as bfloat16 rows
// [query][feature].  The products are gfx950's 32x32x16 bfloat16 MFMAs with
// features along the rows and queries along the columns: A = weight rows,
// B = activation rows of 32 queries; each B operand read from LDS feeds
// kFB = kWaveRows / 32 independent accumulators.  kGroupWaves = 4 (two waves
// per SIMD, 64 rows each) measured faster than 2 (one wave per SIMD with 128
// rows, whose accumulators then live in AGPRs and cost a move per element).
constexpr int kGroupWaves = 4;
constexpr int kWaveRows = kHid / kGroupWaves;
constexpr int kFB = kWaveRows / 32;
constexpr int kInferThreads = 2 * kGroupWaves * kWave;
constexpr int kActLd = kHid + 8;  // bfloat16 per LDS row: +16 bytes so consecutive rows start 4 banks apart

// What the inference loop needs of each arm, copied to LDS once.
struct InferArm {
  int N, Npad, H, valid;         // valid: the arm's plan is on the read side of the board
  float bx, by, bz, byaw, cyaw, syaw;
};

struct alignas(16) InferLds {
  uint16_t act1[2][32][kActLd];  // first-layer outputs, two query blocks in flight
  uint16_t act2[2][32][kActLd];  // second-layer outputs
  uint16_t act3[2][32][kActLd];  // third-layer outputs
  float bias[3][kHid];
  uint16_t w4[kHid];             // output weights, bfloat16
  int ok[4][32];                 // bit 0: query live; bit 1: live and inside the training box
  long long out_row[4];          // skip / prediction offset of the block's first query
  int out_arm[4];                // own arm of the block
  unsigned cnt[kMaxArms][2];     // queries and predicted-far queries of this block, per arm
  int n_rows[4];                 // rows of the block below the arm's padded rollout count
  InferArm arm[kMaxArms];
  float mid[7], inv_half[7];
  float b4;
};

// First-layer K slots: chunk 0 = [own f0..f6, flag slot (zero weight)] for
// lanes 0-31 and [neighbour f7..f13, f14] for lanes 32-63; chunk 1 = [f15,
// f16, zeros] for lanes 0-31 and zeros for lanes 32-63.
__device__ __forceinline__ int first_layer_feature(int c, int half, int e) {
  if (c == 0) return half ? 7 + e : (e < 7 ? e : -1);
  return (half == 0 && e < 2) ? 15 + e : -1;
}

// Neighbour part of the features (identical for the 32 queries of a block):
// f7..f16 as in pair_features, and whether its joints lie in the box.
__device__ __forceinline__ bool neighbour_features(const InferArm& a, const InferArm& i, const float* qi,
                                                   const float* mid, const float* inv_half, float g[10]) {
  const float kPi = 3.14159265358979f;
  float q0 = qi[0] + (i.byaw - a.byaw);
  q0 = q0 - 6.28318530717959f * floorf((q0 + kPi) * 0.159154943091895f);
  g[0] = q0 * 0.318309886183791f;
  bool inbox = fabsf(g[0]) <= 1.0f + 1e-3f;
#pragma unroll
  for (int j = 1; j < 7; ++j) {
    g[j] = (qi[j] - mid[j]) * inv_half[j];
    inbox = inbox && fabsf(g[j]) <= 1.0f + 1e-3f;
  }
  const float dx = i.bx - a.bx, dy = i.by - a.by, dz = i.bz - a.bz;
  g[7] = fmaf_(a.cyaw, dx, a.syaw * dy);
  g[8] = fmaf_(-a.syaw, dx, a.cyaw * dy);
  g[9] = dz;
  return inbox;
}

// Accumulator block starts from the bias of its features: element q4*4 + r
// holds feature base + q4*8 + (lane/32)*4 + r (`bl` = bias + base + (lane/32)*4).
__device__ __forceinline__ void init_block(f32x16_t& acc, const float* bl) {
#pragma unroll
  for (int q4 = 0; q4 < 4; ++q4) {
    const float4 b = *reinterpret_cast<const float4*>(bl + q4 * 8);
    acc[q4 * 4 + 0] = b.x;
    acc[q4 * 4 + 1] = b.y;
    acc[q4 * 4 + 2] = b.z;
    acc[q4 * 4 + 3] = b.w;
  }
}

// 256-wide layer for this wave's kWaveRows output features over 32 queries
// (`bl` = bias + the lane's first feature).
__device__ __forceinline__ void layer256(const bf16x8_t (&w)[kFB][16], const uint16_t (*act)[kActLd],
                                         const float* bl, f32x16_t (&acc)[kFB], int lane) {
#pragma unroll
  for (int fb = 0; fb < kFB; ++fb) init_block(acc[fb], bl + fb * 32);
  const uint16_t* row = act[lane & 31] + (lane >> 5) * 8;
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    const bf16x8_t b = load_bf16x8(row + c * 16);
#pragma unroll
    for (int fb = 0; fb < kFB; ++fb) acc[fb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w[fb][c], b, acc[fb], 0, 0, 0);
  }
}

// Lane exchange by DPP control `ctrl` (all rows and banks enabled).
template <int ctrl>
__device__ __forceinline__ float dpp_f32(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), ctrl, 0xF, 0xF, false));
}

// max(x, 0) as one integer max on the bit pattern (equal to fmaxf(x, 0) for
// every non-NaN x, -0 included up to the sign of zero).
__device__ __forceinline__ float relu_bits(float x) { return __int_as_float(max(__float_as_int(x), 0)); }

// relu, bfloat16, into the LDS rows of this lane's query (`dst` = row +
// base + (lane/32)*4).
__device__ __forceinline__ void store_block(const f32x16_t& acc, uint16_t* dst) {
#pragma unroll
  for (int q4 = 0; q4 < 4; ++q4) {
    uint2 v;
    v.x = f2bf2(relu_bits(acc[q4 * 4 + 0]), relu_bits(acc[q4 * 4 + 1]));
    v.y = f2bf2(relu_bits(acc[q4 * 4 + 2]), relu_bits(acc[q4 * 4 + 3]));
    *reinterpret_cast<uint2*>(dst + q4 * 8) = v;
  }
}

// The global reads of one query block, issued a stage before they are used.
struct BlockIn {
  SurItem item;
  uint4 fown;     // this lane's own-feature row (lanes 0-31 use it)
  float pq[7];    // neighbour's planned joints at the block's step
};

__device__ __forceinline__ void fetch_block(const SurInferArgs& A, const InferLds& L, int Hmax, int Nmax,
                                            const SurItem& it, int q, BlockIn& b) {
  b.item = it;
  const int n = min(it.n0 + q, L.arm[it.arm].Npad - 1);
  b.fown = *reinterpret_cast<const uint4*>(A.F + (((size_t)it.arm * Hmax + it.h) * Nmax + n) * 8);
  const float* pq = A.planq + ((size_t)it.nbr * Hmax + it.h) * 7;
#pragma unroll
  for (int j = 0; j < 7; ++j) b.pq[j] = pq[j];
}

__global__ __launch_bounds__(kInferThreads, 1) void k_sur_infer(SurInferArgs A) {
  __shared__ InferLds L;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int grp = wave / kGroupWaves, wq = wave % kGroupWaves, half = lane >> 5, q = lane & 31;
  // Loop invariants in registers and LDS: the loop's only global reads are
  // the prefetched query blocks.
  const int nA = A.P->A, Hmax = A.P->Hmax, Nmax = A.P->Nmax;
  const float margin = A.model->margin;
  if (tid < nA) {
    const DevArm& d = A.arms[tid];
    InferArm& m = L.arm[tid];
    m.N = d.N;
    m.Npad = d.Npad;
    m.H = d.H;
    m.valid = A.meta->valid[0][tid];
    m.bx = d.base[0];
    m.by = d.base[1];
    m.bz = d.base[2];
    m.byaw = d.base[3];
    m.cyaw = d.cyaw;
    m.syaw = d.syaw;
  }
  if (tid < 7) {
    L.mid[tid] = A.model->mid[tid];
    L.inv_half[tid] = A.model->inv_half[tid];
  }
  if (tid < 2 * kMaxArms) L.cnt[tid >> 1][tid & 1] = 0u;
  for (int e = tid; e < kHid; e += kInferThreads) {
    L.bias[0][e] = A.P32[mlp_b_off(0) + e];
    L.bias[1][e] = A.P32[mlp_b_off(1) + e];
    L.bias[2][e] = A.P32[mlp_b_off(2) + e];
    L.w4[e] = A.W16[mlp_w_off(3) + e];
  }
  if (tid == 0) L.b4 = A.P32[mlp_b_off(3)];
  // Stationary weights: rows wq*kWaveRows + fb*32 + q, K slots c*16 + half*8 + 0..7.
  const int row0 = wq * kWaveRows + q;
  bf16x8_t w[kFB][16];
  {
    const uint16_t* src = A.W16 + mlp_w_off(grp == 0 ? 1 : 2) + (long long)row0 * kHid + half * 8;
#pragma unroll
    for (int fb = 0; fb < kFB; ++fb)
#pragma unroll
      for (int c = 0; c < 16; ++c) w[fb][c] = load_bf16x8(src + fb * 32 * kHid + c * 16);
  }
  bf16x8_t w1[kFB][2];
#pragma unroll
  for (int fb = 0; fb < kFB; ++fb)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = first_layer_feature(c, half, e);
        uint16_t v = 0;
        if (grp == 1 && k >= 0) v = A.W16[mlp_w_off(0) + (long long)(row0 + fb * 32) * kFeat + k];
        w1[fb][c][e] = __builtin_bit_cast(__bf16, v);
      }

  const int G = gridDim.x;
  const int n_my = A.n_items > (int)blockIdx.x ? (A.n_items - 1 - (int)blockIdx.x) / G + 1 : 0;
  const int fcol = wq * kWaveRows + half * 4;  // this lane's first feature within an accumulator block
  // The pipeline body is straight-line code: edge stages (before the first
  // block reaches a layer, after the last one has left it) compute on
  // in-bounds stand-in data (zeroed activations, the last block's inputs) and
  // only their writes are suppressed, so the compiler may interleave each
  // wave's MFMA and VALU work freely.
  for (int e = tid; e < (int)(3 * sizeof(L.act1) / sizeof(uint4)); e += kInferThreads)
    reinterpret_cast<uint4*>(&L.act1[0][0][0])[e] = make_uint4(0u, 0u, 0u, 0u);
  // Group B keeps the reads of the next block and the item after it in flight.
  BlockIn cur, nxt;
  SurItem item2{};
  __syncthreads();
  if (grp == 1 && n_my > 0) {
    fetch_block(A, L, Hmax, Nmax, A.items[blockIdx.x], q, nxt);
    item2 = A.items[blockIdx.x + (long long)min(1, n_my - 1) * G];
  }
  for (int s = 0; s < n_my + 3; ++s) {
    if (grp == 1) {
      // Features and first layer of query block s (the last block again
      // past the end), then the third layer of block s-2; the block's
      // bookkeeping for the decision three stages later is stored last so
      // that both layers form one straight-line sequence.
      cur = nxt;
      fetch_block(A, L, Hmax, Nmax, item2, q, nxt);
      item2 = A.items[blockIdx.x + (long long)min(s + 2, n_my - 1) * G];
      const SurItem it = cur.item;
      const InferArm& arm = L.arm[it.arm];
      const InferArm& nbr = L.arm[it.nbr];
      const bool live = nbr.valid != 0 && it.h < nbr.H && it.n0 + q < arm.N;
      bool inbox;
      {
        float g[10];
        const bool nbr_in = neighbour_features(arm, nbr, cur.pq, L.mid, L.inv_half, g);
        inbox = nbr_in && (cur.fown.w >> 16) != 0u;
        // B operands: lanes 0-31 take their own-feature row (its flag slot
        // meets a zero weight), lanes 32-63 the neighbour features f7..f14;
        // the second chunk holds f15, f16 for lanes 0-31 and zeros.
        const uint4 nbw = make_uint4(f2bf2(g[0], g[1]), f2bf2(g[2], g[3]), f2bf2(g[4], g[5]), f2bf2(g[6], g[7]));
        const uint4 xw0 = half ? nbw : cur.fown;
        const uint4 xw1 = make_uint4(half ? 0u : f2bf2(g[8], g[9]), 0u, 0u, 0u);
        const bf16x8_t x0 = __builtin_bit_cast(bf16x8_t, xw0);
        const bf16x8_t x1 = __builtin_bit_cast(bf16x8_t, xw1);
        f32x16_t acc[kFB];
#pragma unroll
        for (int fb = 0; fb < kFB; ++fb) {
          init_block(acc[fb], &L.bias[0][fcol + fb * 32]);
          acc[fb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w1[fb][0], x0, acc[fb], 0, 0, 0);
          acc[fb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w1[fb][1], x1, acc[fb], 0, 0, 0);
          store_block(acc[fb], &L.act1[s & 1][q][fcol + fb * 32]);
        }
      }
      {
        f32x16_t acc[kFB];
        layer256(w, L.act2[(s - 2) & 1], &L.bias[2][fcol], acc, lane);
#pragma unroll
        for (int fb = 0; fb < kFB; ++fb) store_block(acc[fb], &L.act3[(s - 2) & 1][q][fcol + fb * 32]);
      }
      if (s < n_my && wq == 0 && half == 0) {
        L.ok[s & 3][q] = (live ? 1 : 0) | ((live && inbox) ? 2 : 0);
        if (q == 0) {
          L.out_row[s & 3] = (((long long)it.arm * nA + it.nbr) * Hmax + it.h) * Nmax + it.n0;
          L.n_rows[s & 3] = arm.Npad - it.n0;
          L.out_arm[s & 3] = it.arm;
        }
      }
    } else {
      {
        // Second layer of query block s-1.
        f32x16_t acc[kFB];
        layer256(w, L.act1[(s - 1) & 1], &L.bias[1][fcol], acc, lane);
#pragma unroll
        for (int fb = 0; fb < kFB; ++fb) store_block(acc[fb], &L.act2[(s - 1) & 1][q][fcol + fb * 32]);
      }
      {
        // Output layer and decision of query block s-3: 8 lanes per query
        // (queries wq*32/kGroupWaves + pass*8 + lane/8); the 8 lanes take
        // 16-byte chunks j, j+8, j+16, j+24 (j = lane%8), so each 8-lane group
        // reads 128 contiguous bytes.
        const int r = (s - 3) & 3, j = lane & 7;
#pragma unroll
        for (int pass = 0; pass < 4 / kGroupWaves; ++pass) {
          const int qq = wq * (32 / kGroupWaves) + pass * 8 + (lane >> 3);
          const uint16_t* row = &L.act3[(s - 3) & 1][qq][0];
          float pi[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int k = (j + 8 * i) * 8;
            const uint4 a = *reinterpret_cast<const uint4*>(row + k);
            const uint4 wv = *reinterpret_cast<const uint4*>(&L.w4[k]);
            float t = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, a.x),
                                                      __builtin_bit_cast(bf16x2_t, wv.x), 0.f, false);
            t = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, a.y), __builtin_bit_cast(bf16x2_t, wv.y),
                                                t, false);
            t = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, a.z), __builtin_bit_cast(bf16x2_t, wv.z),
                                                t, false);
            pi[i] = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, a.w),
                                                    __builtin_bit_cast(bf16x2_t, wv.w), t, false);
          }
          // sum over the 8 lanes of the query: swaps within quads, then the
          // mirrored lane of the other quad of the row of 8
          float part = (pi[0] + pi[1]) + (pi[2] + pi[3]);
          part += dpp_f32<0xB1>(part);   // quad_perm [1,0,3,2]
          part += dpp_f32<0x4E>(part);   // quad_perm [2,3,0,1]
          part += dpp_f32<0x141>(part);  // row_half_mirror
          const bool writer = s >= 3 && j == 0 && qq < L.n_rows[r];
          const int okv = L.ok[r][qq];
          const float y = part + L.b4;
          const bool far = (okv & 2) != 0 && y >= margin;
          if (writer) {
            const long long o = L.out_row[r] + qq;
            A.skip[o] = far ? 1 : 0;
            if (A.pred) A.pred[o] = y;
          }
          const unsigned nq = (unsigned)__popcll(__ballot(writer && (okv & 1)));
          const unsigned nf = (unsigned)__popcll(__ballot(writer && far));
          if (lane == 0 && (nq | nf)) {
            atomicAdd(&L.cnt[L.out_arm[r]][0], nq);
            atomicAdd(&L.cnt[L.out_arm[r]][1], nf);
          }
        }
      }
    }
    __syncthreads();
  }
  if (A.counts && tid < 2 * nA) {
    const unsigned v = L.cnt[tid >> 1][tid & 1];
    if (v) atomicAdd(A.counts + 5 * (tid >> 1) + (tid & 1), (unsigned long long)v);
  }
}

// ---------------------------------------------------------------------------
template <int LAY>
static hipError_t pair_distance_t(const DevArm* arms, int ai, int aj, const float* qi, const float* qj, int M,
                                  float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_pair_distance<LAY>, dim3((M + kWave - 1) / kWave), dim3(kWave), 0, s, arms, ai, aj, qi, qj,
                     M, out);
  return hipGetLastError();
}

hipError_t launch_pair_distance(int layout, const DevArm* arms, int ai, int aj, const float* qi, const float* qj,
                                int M, float* out, hipStream_t s) {
  if (M <= 0) return hipSuccess;
  return layout == 0 ? pair_distance_t<0>(arms, ai, aj, qi, qj, M, out, s)
                     : pair_distance_t<1>(arms, ai, aj, qi, qj, M, out, s);
}

hipError_t launch_sur_sample_layout(int layout, const DevArm* arms, const SurModel* model, const int* pairs,
                                    int n_pairs, uint32_t slo, uint32_t shi, long long first, int M, float clip,
                                    float floor_, uint16_t* X16, float* T, float* Q, hipStream_t s) {
  if (M <= 0) return hipSuccess;
  if (layout == 0)
    hipLaunchKernelGGL(k_sur_sample<0>, dim3((M + kWave - 1) / kWave), dim3(kWave), 0, s, arms, model, pairs,
                       n_pairs, slo, shi, first, M, clip, floor_, X16, T, Q);
  else
    hipLaunchKernelGGL(k_sur_sample<1>, dim3((M + kWave - 1) / kWave), dim3(kWave), 0, s, arms, model, pairs,
                       n_pairs, slo, shi, first, M, clip, floor_, X16, T, Q);
  return hipGetLastError();
}

hipError_t launch_features(const DevArm* arms, const SurModel* model, int ai, int aj, const float* qi,
                           const float* qj, int M, float* F, hipStream_t s) {
  if (M <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_features, dim3((M + 255) / 256), dim3(256), 0, s, arms, model, ai, aj, qi, qj, M, F);
  return hipGetLastError();
}

hipError_t launch_gemm_bf16(const GemmArgs& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gemm_bf16, dim3((g.N + 63) / 64, (g.M + 63) / 64), dim3(256), 0, s, g);
  return hipGetLastError();
}

hipError_t launch_loss(const float* y, const float* t, int B, float over_w, float near_w, float near_band, float* dy,
                       uint16_t* dy16,
                       float* loss_acc, hipStream_t s) {
  hipLaunchKernelGGL(k_loss, dim3(1), dim3(1024), 0, s, y, t, B, over_w, near_w, near_band, dy, dy16, loss_acc);
  return hipGetLastError();
}

hipError_t launch_colsum(const float* X, int M, int N, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_colsum, dim3((N + kColsumCols - 1) / kColsumCols), dim3(kColsumCols * kColsumGroups), 0, s, X,
                     M, N, out);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, float* m, float* v, const float* g, long long n, float lr, float b1, float b2,
                       float eps, int step, hipStream_t s) {
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, m, v, g, n, lr, b1, b2, eps, c1,
                     c2);
  return hipGetLastError();
}

hipError_t launch_params_to_bf16(const float* p, uint16_t* p16, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, p16, n);
  return hipGetLastError();
}

hipError_t launch_f32_to_bf16(const float* x, uint16_t* y, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, y, n);
  return hipGetLastError();
}

hipError_t launch_sur_states(const DevArm* arms, const Params* P, const SurModel* model, const StepState* ss,
                             const float* mu, const float* state, const float* eps_in, int k_iter, int n_arms,
                             int npad_max, uint16_t* F, hipStream_t s) {
  hipLaunchKernelGGL(k_sur_states, dim3((npad_max + kWave - 1) / kWave, n_arms), dim3(kWave), 0, s, arms, P, model,
                     ss, mu, state, eps_in, k_iter, F);
  return hipGetLastError();
}

hipError_t launch_sur_infer(const SurInferArgs& A, int grid, hipStream_t s) {
  if (A.n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sur_infer, dim3(grid), dim3(kInferThreads), 0, s, A);
  return hipGetLastError();
}

hipError_t launch_init_params(float* p, uint32_t slo, uint32_t shi, hipStream_t s) {
  hipLaunchKernelGGL(k_init_params, dim3((unsigned)((kMlpParams + 255) / 256)), dim3(256), 0, s, p, slo, shi);
  return hipGetLastError();
}

}  // namespace mrs
