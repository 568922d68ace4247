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

typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

// FP32 -> bfloat16, round to nearest even (NaN stays NaN).
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
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
                                                      float clip, uint16_t* __restrict__ X16,
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
    T[m] = fminf(r, clip);
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
// sub-tile each), K in steps of 32 through LDS, every operand access
// bounds-checked (zero fill), FP32 accumulation.
__global__ __launch_bounds__(256) void k_gemm_bf16(GemmArgs g) {
  __shared__ uint16_t As[64][40];
  __shared__ uint16_t Bs[32][72];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  f32x16_t acc;
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = 0.f;
  for (int k0 = 0; k0 < g.K; k0 += 32) {
    for (int e = tid; e < 64 * 32; e += 256) {
      int r, c;
      if (g.transA) { r = e % 64; c = e / 64; } else { r = e / 32; c = e % 32; }
      const int m = m0 + r, k = k0 + c;
      uint16_t v = 0;
      if (m < g.M && k < g.K) v = g.transA ? g.A[(size_t)k * g.lda + m] : g.A[(size_t)m * g.lda + k];
      As[r][c] = v;
    }
    for (int e = tid; e < 32 * 64; e += 256) {
      int r, c;
      if (g.transB) { r = e % 32; c = e / 32; } else { r = e / 64; c = e % 64; }
      const int k = k0 + r, n = n0 + c;
      uint16_t v = 0;
      if (k < g.K && n < g.N) v = g.transB ? g.B[(size_t)n * g.ldb + k] : g.B[(size_t)k * g.ldb + n];
      Bs[r][c] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 32; kk += 8) {
      bf16x4_t a, b;
      const int kb = kk + (lane >> 5) * 4;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        a[i] = (short)As[wm + (lane & 31)][kb + i];
        b[i] = (short)Bs[kb + i][wn + (lane & 31)];
      }
      acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
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

// Loss (mean of e^2 + w max(e,0)^2, e = y - t) and dLoss/dy; one block,
// fixed reduction order.
__global__ __launch_bounds__(1024) void k_loss(const float* __restrict__ y, const float* __restrict__ t, int B,
                                               float over_w, float* __restrict__ dy, uint16_t* __restrict__ dy16,
                                               float* __restrict__ loss_acc) {
  __shared__ float red[1024];
  const int tid = threadIdx.x;
  float acc = 0.f;
  const float invB = 1.0f / (float)B;
  for (int i = tid; i < B; i += blockDim.x) {
    const float e = y[i] - t[i], pos = fmaxf(e, 0.f);
    acc = fmaf_(e, e, fmaf_(over_w * pos, pos, acc));
    const float d = (2.f * e + 2.f * over_w * pos) * invB;
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

// out[n] = sum over rows of X[m][n] (bias gradients), rows in order.
__global__ void k_colsum(const float* __restrict__ X, int M, int N, float* __restrict__ out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int m = 0; m < M; ++m) s += X[(size_t)m * N + n];
  out[n] = s;
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
// Own rollout joint positions of every (arm, step, rollout) for the learned
// distance: the same noise and integration as the rollout kernel.
__global__ __launch_bounds__(kWave) void k_sur_states(const DevArm* __restrict__ arms,
                                                      const Params* __restrict__ Pp,
                                                      const StepState* __restrict__ ssp,
                                                      const float* __restrict__ mu_all,
                                                      const float* __restrict__ state, int k_iter,
                                                      float* __restrict__ Q) {
  const Params& P = *Pp;
  const int a = blockIdx.y;
  const DevArm* arm = arms + a;
  const int n = blockIdx.x * kWave + threadIdx.x;
  if (n >= arm->Npad) return;
  const uint32_t t = ssp->t;
  const float* mu = mu_all + (size_t)a * P.Hmax * 7;
  float q[7], qd[7];
  for (int j = 0; j < 7; ++j) {
    q[j] = state[(a * 7 + j) * 3 + 0];
    qd[j] = state[(a * 7 + j) * 3 + 1];
  }
  for (int h = 0; h < arm->H; ++h) {
    float z[8];
    normals8(P.seed_lo, P.seed_hi, a, t, k_iter, n, h, z);
    float* out = Q + (((size_t)a * P.Hmax + h) * P.Nmax + n) * 7;
#pragma unroll
    for (int j = 0; j < 7; ++j) {
      const float u = P.sigma * z[j] + mu[h * 7 + j];
      qd[j] = fmaf_(P.dt, u, qd[j]);
      q[j] = fmaf_(P.dt, qd[j], q[j]);
      out[j] = q[j];
    }
  }
}

// Fused MLP inference, transposed so features run along the MFMA rows and
// queries along the columns: a 32x32 accumulator block of layer l holds, for
// lane l, 16 features of query l%32 in exactly the K order the next layer's
// B operand needs, so activations never leave registers.  One wave = 32
// queries (one rollout block of one (arm, neighbour, step)); a 512-thread
// block shares each layer's weights through LDS.
constexpr int kW1Ld = 32 + 4;    // bf16 per staged row (17 inputs padded to 32, +4 against bank conflicts)
constexpr int kWLd = kHid + 4;

struct InferLds {
  uint16_t W1[kHid][kW1Ld];
  uint16_t W[kHid][kWLd];          // layer 2, then layer 3
  float b[3][kHid];
  float w4[kHid];
  float b4;
};

template <int NKB>
__device__ __forceinline__ void mfma_block_row(const uint16_t* wrow, const bf16x4_t* act, f32x16_t& acc, int lane) {
#pragma unroll
  for (int kb = 0; kb < NKB; ++kb) {
    const uint16_t* p = wrow + kb * 8 + (lane >> 5) * 4;
    const uint2 raw = *reinterpret_cast<const uint2*>(p);
    bf16x4_t a;
    a[0] = (short)(raw.x & 0xffffu);
    a[1] = (short)(raw.x >> 16);
    a[2] = (short)(raw.y & 0xffffu);
    a[3] = (short)(raw.y >> 16);
    acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, act[kb], acc, 0, 0, 0);
  }
}

// Accumulator block fb starts from the bias of its features: element
// q4*4 + r holds feature fb*32 + q4*8 + (lane/32)*4 + r.  `bl` points at
// bias[(lane/32)*4], so every read is that lane base plus a constant.
__device__ __forceinline__ void init_block(f32x16_t& acc, const float* bl, int fb) {
#pragma unroll
  for (int q4 = 0; q4 < 4; ++q4) {
    const float4 b = *reinterpret_cast<const float4*>(bl + fb * 32 + q4 * 8);
    acc[q4 * 4 + 0] = b.x;
    acc[q4 * 4 + 1] = b.y;
    acc[q4 * 4 + 2] = b.z;
    acc[q4 * 4 + 3] = b.w;
  }
}

// One accumulator block -> four B operands of the next layer: relu in bfloat16.
__device__ __forceinline__ void block_to_operands(const f32x16_t& acc, bf16x4_t* dst) {
#pragma unroll
  for (int q4 = 0; q4 < 4; ++q4) {
    bf16x4_t v;
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = (short)f2bf(fmaxf(acc[q4 * 4 + r], 0.f));
    dst[q4] = v;
  }
}

// Stage one 256x256 layer into the shared buffer (all waves done with the
// previous contents first).
__device__ __forceinline__ void stage_weights(InferLds& L, const uint16_t* W, int tid, int nthr) {
  __syncthreads();
  for (int e = tid; e < kHid * kHid / 4; e += nthr) {
    const int f2 = e / (kHid / 4), k4 = (e % (kHid / 4)) * 4;
    *reinterpret_cast<uint2*>(&L.W[f2][k4]) = *reinterpret_cast<const uint2*>(W + (long long)f2 * kHid + k4);
  }
  __syncthreads();
}

__global__ __launch_bounds__(512) void k_sur_infer(SurInferArgs A) {
  __shared__ InferLds L;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const Params& P = *A.P;
  const SurModel& sm = *A.model;
  // Resident: layer 1 (inputs padded to 32 with zeros), biases, output layer.
  for (int e = tid; e < kHid * 32; e += blockDim.x) {
    const int f = e / 32, k = e % 32;
    L.W1[f][k] = k < kFeat ? A.W16[mlp_w_off(0) + (long long)f * kFeat + k] : (uint16_t)0;
  }
  for (int e = tid; e < kHid; e += blockDim.x) {
    L.b[0][e] = A.P32[mlp_b_off(0) + e];
    L.b[1][e] = A.P32[mlp_b_off(1) + e];
    L.b[2][e] = A.P32[mlp_b_off(2) + e];
    L.w4[e] = bf2f(A.W16[mlp_w_off(3) + e]);
  }
  if (tid == 0) L.b4 = A.P32[mlp_b_off(3)];
  __syncthreads();
  const int groups = (A.n_items + 7) / 8;
  for (int g = blockIdx.x; g < groups; g += gridDim.x) {
    const int it = g * 8 + wave;
    const bool have = it < A.n_items;
    SurItem item = have ? A.items[it] : A.items[0];
    const DevArm* arm = A.arms + item.arm;
    const DevArm* nbr = A.arms + item.nbr;
    const int q = lane & 31;
    const int n = item.n0 + q;
    const bool valid = A.meta->valid[0][item.nbr] != 0 && item.h < nbr->H;
    const bool live = have && valid && n < arm->N;
    // Features of this lane's query.
    float qa[8], qb[8], f[kFeat];
    const float* src = A.Q + (((size_t)item.arm * P.Hmax + item.h) * P.Nmax + (n < arm->Npad ? n : 0)) * 7;
    const float* pq = A.planq + ((size_t)item.nbr * P.Hmax + item.h) * 7;
#pragma unroll
    for (int j = 0; j < 7; ++j) {
      qa[j] = src[j];
      qb[j] = pq[j];
    }
    qa[7] = qb[7] = 0.f;
    pair_features(arm, qa, nbr, qb, A.model, f);
    bool inbox = true;
#pragma unroll
    for (int k = 0; k < 14; ++k) inbox = inbox && fabsf(f[k]) <= 1.0f + 1e-3f;
    // Layer 1: K = 32 (17 features + zeros): B operand kb holds features
    // kb*8 + (lane/32)*4 + 0..3 of query lane%32.
    bf16x4_t x[4];
#pragma unroll
    for (int kb = 0; kb < 4; ++kb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int k0 = kb * 8 + r, k1 = kb * 8 + 4 + r;
        const float v0 = k0 < kFeat ? f[k0 < kFeat ? k0 : 0] : 0.f;
        const float v1 = k1 < kFeat ? f[k1 < kFeat ? k1 : 0] : 0.f;
        x[kb][r] = (short)f2bf((lane >> 5) ? v1 : v0);
      }
    bf16x4_t act[32], nxt[32];
    const int lb = (lane >> 5) * 4;
#pragma unroll
    for (int fb = 0; fb < 8; ++fb) {
      f32x16_t acc;
      init_block(acc, &L.b[0][lb], fb);
      mfma_block_row<4>(&L.W1[fb * 32 + (lane & 31)][0], x, acc, lane);
      block_to_operands(acc, &act[fb * 4]);
    }
    // Layer 2 (weights staged through the shared buffer).
    stage_weights(L, A.W16 + mlp_w_off(1), tid, blockDim.x);
#pragma unroll
    for (int fb = 0; fb < 8; ++fb) {
      f32x16_t acc;
      init_block(acc, &L.b[1][lb], fb);
      mfma_block_row<32>(&L.W[fb * 32 + (lane & 31)][0], act, acc, lane);
      block_to_operands(acc, &nxt[fb * 4]);
    }
    // Layer 3, folded straight into the output dot product; its activations
    // are rounded to bfloat16 first, as the output layer's operand is in training.
    stage_weights(L, A.W16 + mlp_w_off(2), tid, blockDim.x);
    float part = 0.f;
#pragma unroll
    for (int fb = 0; fb < 8; ++fb) {
      f32x16_t acc;
      init_block(acc, &L.b[2][lb], fb);
      mfma_block_row<32>(&L.W[fb * 32 + (lane & 31)][0], nxt, acc, lane);
      f32x16_t w4;
      init_block(w4, &L.w4[lb], fb);
#pragma unroll
      for (int i = 0; i < 16; ++i) part = fmaf_(w4[i], bf2f(f2bf(fmaxf(acc[i], 0.f))), part);
    }
    const float y = part + __shfl_xor(part, 32) + L.b4;
    if (lane < 32 && have && n < arm->Npad) {
      const bool skip = live && inbox && y >= sm.margin;
      A.skip[(((size_t)item.arm * P.A + item.nbr) * P.Hmax + item.h) * P.Nmax + n] = skip ? 1 : 0;
      if (A.pred) A.pred[(((size_t)item.arm * P.A + item.nbr) * P.Hmax + item.h) * P.Nmax + n] = y;
    }
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
                                    uint16_t* X16, float* T, float* Q, hipStream_t s) {
  if (M <= 0) return hipSuccess;
  if (layout == 0)
    hipLaunchKernelGGL(k_sur_sample<0>, dim3((M + kWave - 1) / kWave), dim3(kWave), 0, s, arms, model, pairs,
                       n_pairs, slo, shi, first, M, clip, X16, T, Q);
  else
    hipLaunchKernelGGL(k_sur_sample<1>, dim3((M + kWave - 1) / kWave), dim3(kWave), 0, s, arms, model, pairs,
                       n_pairs, slo, shi, first, M, clip, X16, T, Q);
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

hipError_t launch_loss(const float* y, const float* t, int B, float over_w, float* dy, uint16_t* dy16,
                       float* loss_acc, hipStream_t s) {
  hipLaunchKernelGGL(k_loss, dim3(1), dim3(1024), 0, s, y, t, B, over_w, dy, dy16, loss_acc);
  return hipGetLastError();
}

hipError_t launch_colsum(const float* X, int M, int N, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_colsum, dim3((N + 255) / 256), dim3(256), 0, s, X, M, N, out);
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

hipError_t launch_sur_states(const DevArm* arms, const Params* P, const StepState* ss, const float* mu,
                             const float* state, int k_iter, int n_arms, int npad_max, float* Q, hipStream_t s) {
  hipLaunchKernelGGL(k_sur_states, dim3((npad_max + kWave - 1) / kWave, n_arms), dim3(kWave), 0, s, arms, P, ss, mu,
                     state, k_iter, Q);
  return hipGetLastError();
}

hipError_t launch_sur_infer(const SurInferArgs& A, int grid, hipStream_t s) {
  if (A.n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sur_infer, dim3(grid), dim3(512), 0, s, A);
  return hipGetLastError();
}

hipError_t launch_init_params(float* p, uint32_t slo, uint32_t shi, hipStream_t s) {
  hipLaunchKernelGGL(k_init_params, dim3((unsigned)((kMlpParams + 255) / 256)), dim3(256), 0, s, p, slo, shi);
  return hipGetLastError();
}

}  // namespace mrs
