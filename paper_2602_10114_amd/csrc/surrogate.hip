// gfx950 kernels of the learned arm-pair distance:
//   exact signed distance between two arms (Eq. 6 over all sphere pairs),
//   Philox-drawn training samples, a bfloat16 MFMA GEMM with fused epilogues
//   for training, loss / column sums / Adam, and the fused MLP inference that
//   decides, per (rollout, step, neighbour), whether the exact check can be
//   skipped.
#include <hip/hip_runtime.h>

#include <algorithm>

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

// Neighbour record of the fused inference for (arm a, neighbour i, step h)
// of the read-side plans: the neighbour half of the features (identical for
// every rollout of a at step h) and what the decision needs.
__device__ __forceinline__ void nb_record(const DevArm* __restrict__ arms, const SurModel* __restrict__ sm,
                                          const BoardMeta* __restrict__ meta, const float* __restrict__ planq,
                                          int n_arms, int Hmax, int a, int i, int h, uint32_t* __restrict__ rec) {
  uint32_t* r = rec + (((size_t)a * n_arms + i) * Hmax + h) * kNbrRec;
  const DevArm* A = arms + a;
  const DevArm* I = arms + i;
  float qa[8], qi[8], f[kFeat];
  for (int j = 0; j < 8; ++j) {
    qa[j] = 0.f;
    qi[j] = j < 7 ? planq[((size_t)i * Hmax + h) * 7 + j] : 0.f;
  }
  pair_features(A, qa, I, qi, sm, f);
  bool inbox = true;
  for (int j = 7; j < 14; ++j) inbox = inbox && fabsf(f[j]) <= 1.0f + 1e-3f;
  const bool live = i != a && meta->valid[0][i] != 0 && h < I->H;
  const uint4 v0 = make_uint4(f2bf2(f[7], f[8]), f2bf2(f[9], f[10]), f2bf2(f[11], f[12]), f2bf2(f[13], f[14]));
  const uint4 v1 = make_uint4(f2bf2(f[15], f[16]), (inbox ? 1u : 0u) | (live ? 2u : 0u), (uint32_t)A->N,
                              (uint32_t)A->Npad);
  reinterpret_cast<uint4*>(r)[0] = v0;
  reinterpret_cast<uint4*>(r)[1] = v1;
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
// Inference descriptors of every group that needs the network, in (arm,
// neighbour, step, 32-rollout block) order: every block of the descriptor
// row scans the groups' descriptor counts (Npad/32 for a live, unscreened
// group of arm a with i != a and h below both horizons, else 0) in LDS and
// writes the descriptors of its kItemsGroups groups at their offsets, the
// group's first descriptor index (-1 when it has none) and, from the block
// holding the last group, the total.
constexpr int kItemsGroups = 8;
constexpr int kMaxGroups = kMaxArms * kMaxArms * kMaxH;
template <int kThreads>
__device__ __forceinline__ void items_block(const DevArm* __restrict__ arms, const Params& P,
                                            const uint8_t* __restrict__ screened, SurItem* __restrict__ items,
                                            int* __restrict__ grp_first, int* __restrict__ count,
                                            unsigned long long* __restrict__ counts, int block) {
  __shared__ int s_off[kMaxGroups + 1];
  __shared__ int s_wave[kThreads / kWave];
  __shared__ int s_H[kMaxArms], s_blk[kMaxArms];
  const int tid = threadIdx.x, ng = P.A * P.A * P.Hmax;
  if (tid < P.A) {
    s_H[tid] = arms[tid].H;
    s_blk[tid] = arms[tid].Npad / 32;
  }
  __syncthreads();
  auto cnt = [&](int g) -> int {
    const int h = g % P.Hmax, ai = g / P.Hmax, a = ai / P.A, i = ai % P.A;
    if (i == a || h >= s_H[a] || h >= s_H[i] || screened[g]) return 0;
    return s_blk[a];
  };
  // Exclusive scan: each thread a contiguous run of groups, then the runs'
  // totals by wave prefix sums (shuffles) and the waves' totals in order.
  const int lane = tid & (kWave - 1), wv = tid / kWave;
  const int per = (ng + kThreads - 1) / kThreads;
  const int g0 = tid * per, g1 = min(ng, g0 + per);
  int run = 0;
  for (int g = g0; g < g1; ++g) {
    s_off[g] = run;
    run += cnt(g);
  }
  int incl = run;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int u = __shfl_up(incl, off);
    if (lane >= off) incl += u;
  }
  if (lane == kWave - 1) s_wave[wv] = incl;
  __syncthreads();
  int base = 0, total = 0;
#pragma unroll
  for (int w = 0; w < kThreads / kWave; ++w) {
    base += w < wv ? s_wave[w] : 0;
    total += s_wave[w];
  }
  const int excl = base + incl - run;
  for (int g = g0; g < g1; ++g) s_off[g] += excl;
  if (tid == 0) s_off[ng] = total;
  __syncthreads();
  const int gb = block * kItemsGroups;
  for (int k = 0; k < kItemsGroups && gb + k < ng; ++k) {
    const int g = gb + k, n = s_off[g + 1] - s_off[g];
    if (tid == 0) grp_first[g] = n > 0 ? s_off[g] : -1;
    if (n == 0) continue;
    // query rows the network will run for this group (counter slot 5)
    if (tid == 0 && counts) atomicAdd(counts + kSurCounters * (g / P.Hmax / P.A) + 5, (unsigned long long)n * 32ull);
    const int h = g % P.Hmax, ai = g / P.Hmax;
    for (int e = tid; e < n; e += kThreads) items[s_off[g] + e] = SurItem{ai / P.A, ai % P.A, h, 32 * e};
  }
  if (tid == 0 && gb <= ng - 1 && ng - 1 < gb + kItemsGroups) *count = s_off[ng];
}

// Screen of one (arm a, neighbour i, step h) group, one wave: 1 when no query
// of the group needs the network -- the neighbour's plan is not published
// (its queries are not live), or the group dropped no check in the previous
// control step and is not being probed (drop history), or the arm's mean
// rollout (the means
// integrated from the sensed state) lies closer than the screen distance to
// the neighbour's plan at step h, so that nearly every rollout would be
// predicted near anyway (its queries are checked exactly).  Lane = own
// sphere slot: each lane integrates the means, walks the chain and places its
// sphere; the wave takes the minimum gap to the plan's spheres.
__device__ __forceinline__ void screen_group(const DevArm* __restrict__ arms, const Params& P,
                                             const SurModel* __restrict__ sm, const BoardMeta* __restrict__ meta,
                                             const float* __restrict__ mu_all, const float* __restrict__ state,
                                             const float* __restrict__ plan_read, uint32_t t,
                                             const unsigned* __restrict__ hist_prev, unsigned* __restrict__ hist_cur,
                                             int g, int lane, uint8_t* __restrict__ flag) {
  const int h = g % P.Hmax, ai = g / P.Hmax, a = ai / P.A, i = ai % P.A;
  const DevArm* arm = arms + a;
  const DevArm* nb = arms + i;
  uint8_t f = 0;
  bool quiet = false;
  const bool inside = i != a && h < arm->H && h < nb->H;
  if (inside) {
    // Drop history: the group at step h + 1 of the previous control step
    // (the shift brings it here) ran the network or was quiet and dropped at
    // most min_drop of its checks, and this is not the group's probe step.
    if (sm->probe > 0 && (t + (uint32_t)g) % (uint32_t)sm->probe != 0u && h + 1 < arm->H && h + 1 < nb->H) {
      const unsigned v = hist_prev[g + 1];
      quiet = v < kHistNone && (float)v <= sm->min_drop * (float)(arm->Npad / kWave);
    }
    if (!meta->valid[0][i] || quiet) {
      f = 1;
    } else if (sm->screen > 0.f) {
      const float* mu = mu_all + (size_t)a * P.Hmax * 7;
      // The mean rollout's joints at step h: lane j < 7 integrates joint j
      // (the loads of eight steps go out together), then every lane takes
      // the seven values.
      const int jj = lane < 7 ? lane : 0;
      float qq = state[(a * 7 + jj) * 3 + 0], qd = state[(a * 7 + jj) * 3 + 1];
      for (int h0 = 0; h0 <= h; h0 += 8) {
        float m[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) m[u] = h0 + u <= h ? mu[(h0 + u) * 7 + jj] : 0.f;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          if (h0 + u > h) break;  // uniform
          qd = fmaf_(P.dt, m[u], qd);
          qq = fmaf_(P.dt, qd, qq);
        }
      }
      float q[8];
#pragma unroll
      for (int j = 0; j < 7; ++j) q[j] = __shfl(qq, j);
      q[7] = 0.f;
      Frame F[7];
      forward_kinematics(F, arm, q);
      float gmin = 3.0e38f;
      const int slots = kLayoutSlots[arm->layout];
      if (lane < slots && arm->slot_src[lane] >= 0) {
        int b = 0;
        while (lane >= kLayoutStart[arm->layout][b + 1]) ++b;
        const float* p = arm->slot[lane];
        // the body's frame picked by selects (no indexed register array)
        const int fb = b < 7 ? b : 6;
        Frame Fb = F[0];
#pragma unroll
        for (int k = 1; k < 7; ++k)
          if (k == fb) Fb = F[k];
        float x, y, z;
        frame_point(Fb, p[0], p[1], p[2], x, y, z);
        const float4* pl = reinterpret_cast<const float4*>(plan_read) + ((size_t)i * P.Hmax + h) * P.Smax;
        // eight plan spheres per batch, loads first (past the end the last
        // sphere repeats, which leaves the minimum unchanged)
        const int S = nb->S;
        for (int k0 = 0; k0 < S; k0 += 8) {
          float4 o[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) o[u] = pl[min(k0 + u, S - 1)];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const float dx = x - o[u].x, dy = y - o[u].y, dz = z - o[u].z;
            gmin = fminf(gmin, sqrtf(fmaf_(dx, dx, fmaf_(dy, dy, dz * dz))) - p[3] - o[u].w);
          }
        }
      }
#pragma unroll
      for (int off = kWave / 2; off > 0; off >>= 1) gmin = fminf(gmin, __shfl_xor(gmin, off));
      f = gmin < sm->screen ? 1 : 0;
    }
  }
  if (lane == 0) {
    flag[g] = f;
    // This step's history (first iteration): 0 for a group that runs the
    // network (the rollout kernel counts its dropped checks) or stays
    // quiet; none for one screened for another reason or outside both
    // horizons.
    if (hist_cur) hist_cur[g] = inside && (f == 0 || quiet) ? 0u : kHistNone;
  }
}

// Rows of blocks blockIdx.y < number of arms: own-joint features of every
// (arm, step, rollout) for the learned distance -- the iteration's noise
// integrated as in the rollout kernel, then the normalised joints as one
// 16-byte row of bfloat16 [f0..f6, in-box flag] (flag 1.0 when all seven lie
// within the training box, else 0.0).  Eight lanes per rollout: lane j < 7
// integrates joint j (the joints are independent) and writes its feature;
// lane 7 writes the flag, the AND of the group's box tests taken with a
// ballot.  The eight 2-byte writes form the row.
// The row blockIdx.y = number of arms writes the neighbour records, one
// thread per (arm, neighbour, step); the next row writes the inference
// descriptors from the screen flags (k_noise_screen), kItemsGroups groups
// per block.
constexpr int kStatesThreads = 256;
__global__ __launch_bounds__(kStatesThreads) void k_sur_states(const DevArm* __restrict__ arms,
                                                               const Params* __restrict__ Pp,
                                                               const SurModel* __restrict__ sm,
                                                               const float* __restrict__ mu_all,
                                                               const float* __restrict__ state,
                                                               const float* __restrict__ eps,
                                                               uint16_t* __restrict__ F,
                                                               const BoardMeta* __restrict__ meta,
                                                               const float* __restrict__ planq,
                                                               uint32_t* __restrict__ rec,
                                                               const uint8_t* __restrict__ screened,
                                                               SurItem* __restrict__ items,
                                                               int* __restrict__ grp_first,
                                                               int* __restrict__ count,
                                                               unsigned long long* __restrict__ counts) {
  const Params& P = *Pp;
  const int a = blockIdx.y;
  if (a == P.A) {
    const int g = blockIdx.x * kStatesThreads + threadIdx.x;
    if (g >= P.A * P.A * P.Hmax) return;
    const int h = g % P.Hmax, ai = g / P.Hmax;
    nb_record(arms, sm, meta, planq, P.A, P.Hmax, ai / P.A, ai % P.A, h, rec);
    return;
  }
  if (a == P.A + 1) {
    if ((int)blockIdx.x * kItemsGroups >= P.A * P.A * P.Hmax) return;  // whole block
    items_block<kStatesThreads>(arms, P, screened, items, grp_first, count, counts, blockIdx.x);
    return;
  }
  const DevArm* arm = arms + a;
  const int j = threadIdx.x & 7, lane = threadIdx.x & 63;
  const int n = blockIdx.x * (kStatesThreads / 8) + (threadIdx.x >> 3);
  // A wave holds 8 rollouts; it leaves only when all of them are past the
  // arm's padded count (Npad is a multiple of 64, so a wave is all in or all
  // out and every lane takes part in the ballots below).
  if (n >= arm->Npad) return;
  const float* mu = mu_all + (size_t)a * P.Hmax * 7;
  const int jj = j < 7 ? j : 0;
  float q = state[(a * 7 + jj) * 3 + 0], qd = state[(a * 7 + jj) * 3 + 1];
  const float mid = sm->mid[jj], ih = sm->inv_half[jj];
  const int group_shift = lane & ~7;
  const int H = arm->H, Npad = arm->Npad;
  const float* zc = eps + arm->eps_off + (size_t)jj * Npad + n;  // the lane's noise column
  // Steps in groups of kStatesAhead: the group's noise loads go out together.
  constexpr int kStatesAhead = 8;
  for (int h0 = 0; h0 < H; h0 += kStatesAhead) {
    float z[kStatesAhead];
#pragma unroll
    for (int u = 0; u < kStatesAhead; ++u) z[u] = h0 + u < H ? zc[(size_t)(h0 + u) * 7 * Npad] : 0.f;
#pragma unroll
    for (int u = 0; u < kStatesAhead; ++u) {
      const int h = h0 + u;
      if (h >= H) break;  // uniform
      const float uu = z[u] + mu[h * 7 + jj];
      qd = fmaf_(P.dt, uu, qd);
      q = fmaf_(P.dt, qd, q);
      const float x = (q - mid) * ih;
      const bool out_of_box = j < 7 && !(fabsf(x) <= 1.0f + 1e-3f);
      const unsigned long long bad = __ballot(out_of_box);
      const bool inbox = ((bad >> group_shift) & 0x7Full) == 0ull;
      const uint16_t v = j < 7 ? f2bf(x) : (inbox ? (uint16_t)0x3F80u : (uint16_t)0u);
      F[(((size_t)a * P.Hmax + h) * P.Nmax + n) * 8 + j] = v;
    }
  }
}

// Fused MLP inference, weight-stationary.  A block of 2 x kGroupWaves waves
// (one block per CU) streams query blocks of 32 queries (32 rollouts of one
// arm at one step against one neighbour's plan), kQB blocks per stage,
// through a pipeline with one barrier per stage:
//   group A (the lower kGroupWaves waves) holds kWaveRows rows each of the
//   second layer's weights in registers; at stage s it runs the first layer
//   of stage s's blocks (small weights in registers; their inputs, the own-
//   feature rows and the neighbour records, were loaded a stage earlier) and
//   then the second layer on stage s-1's blocks, one chain per block;
//   group B holds kWaveRows rows each of the third layer's weights; it runs
//   that layer on stage s-2's blocks as one chain over both (kQB x kFB
//   independent accumulators) with the output layer folded into its epilogue
//   (each lane takes its ReLU'd third-layer features, rounded to bfloat16,
//   times the matching output weights, and leaves one partial sum per query,
//   wave and lane half in LDS); its first wave adds the partial sums of
//   stage s-3 (one query per lane) and stores the predictions.  The skip
//   decision is taken by the rollout kernel from the stored predictions,
//   off the pipeline's critical path.
// Each SIMD holds one wave of each group, so one wave's MFMA chain runs
// while the other does its latency-bound part (LDS round trips, VALU), and
// the roles swap half-way through the stage.
// Activations pass between the groups through LDS as bfloat16 rows
// [query][feature].  The products are gfx950's 32x32x16 bfloat16 MFMAs with
// features along the rows and queries along the columns: A = weight rows,
// B = activation rows of 32 queries; each B operand read from LDS feeds
// kFB = kWaveRows / 32 independent accumulators, and kInflight operand reads
// stay in flight ahead of the MFMAs that use them.
constexpr int kGroupWaves = 4;
constexpr int kWaveRows = kHid / kGroupWaves;
constexpr int kFB = kWaveRows / 32;
constexpr int kInferThreads = 2 * kGroupWaves * kWave;
constexpr int kActLd = kHid + 8;  // bfloat16 per LDS row: +16 bytes so consecutive rows start 4 banks apart
constexpr int kParts = 2 * kGroupWaves;  // output-layer partial sums per query
constexpr int kPartLd = kParts + 4;      // floats per partial-sum row (16-byte aligned rows)
constexpr int kInflight = 4;
constexpr int kItemBatch = 64;           // query-block descriptors staged in LDS per batch
static_assert(kParts % 4 == 0, "partial sums are read as float4");
static_assert(kItemBatch <= kWave && kItemBatch >= 3, "one lane per staged descriptor; staged two stages early");
static_assert(sizeof(SurItem) == 16, "descriptors are staged as 16-byte vectors");

// Two query blocks through one 256-wide layer in one chain: kQB x kFB
// independent accumulators, started from the layer's FP32 bias (`bias16`:
// the lane's 16 output rows of accumulator block fb at bias16[32 fb], in
// LDS), then per K chunk the operand reads of both blocks (kInflight2 chunks
// ahead) and their MFMAs.
constexpr int kInflight2 = 1;
__device__ __forceinline__ void layer256x2(const bf16x8_t (&w)[kFB][16], const float* bias16,
                                           const uint16_t* row0, const uint16_t* row1, f32x16_t (&acc)[2][kFB]) {
  __builtin_amdgcn_sched_barrier(0);
  bf16x8_t b0[16], b1[16];
#pragma unroll
  for (int fb = 0; fb < kFB; ++fb) {
    acc[0][fb] = *reinterpret_cast<const f32x16_t*>(bias16 + fb * 32);
    acc[1][fb] = *reinterpret_cast<const f32x16_t*>(bias16 + fb * 32);
  }
#pragma unroll
  for (int c = 0; c < kInflight2; ++c) {
    b0[c] = load_bf16x8(row0 + c * 16);
    b1[c] = load_bf16x8(row1 + c * 16);
  }
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    if (c + kInflight2 < 16) {
      b0[c + kInflight2] = load_bf16x8(row0 + (c + kInflight2) * 16);
      b1[c + kInflight2] = load_bf16x8(row1 + (c + kInflight2) * 16);
    }
#pragma unroll
    for (int fb = 0; fb < kFB; ++fb) {
      acc[0][fb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w[fb][c], b0[c], acc[0][fb], 0, 0, 0);
      acc[1][fb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w[fb][c], b1[c], acc[1][fb], 0, 0, 0);
    }
  }
  // Issue order: the accumulator starts (four 16-byte reads each) and the
  // first operand reads, then per chunk its MFMAs and the reads ahead.
  __builtin_amdgcn_sched_group_barrier(0x100, 2 * kFB * 4 + 2 * kInflight2, 0);
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    __builtin_amdgcn_sched_group_barrier(0x008, 2 * kFB, 0);
    if (c + kInflight2 < 16) __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
  }
  __builtin_amdgcn_sched_barrier(0);
}

constexpr int kQB = 2;                   // query blocks of 32 per pipeline stage
constexpr int kStageQ = kQB * 32;        // queries per stage
constexpr int kStagesPerBatch = kItemBatch / kQB;
static_assert(kItemBatch % kQB == 0 && kStagesPerBatch >= 3, "a descriptor batch spans whole stages, staged two stages early");

struct alignas(16) InferLds {
  uint16_t act1[2][kStageQ][kActLd];  // first-layer outputs, two stages in flight
  uint16_t act2[2][kStageQ][kActLd];  // second-layer outputs
  float part[2][kStageQ][kPartLd];    // output-layer partial sums [stage][query][wave * 2 + lane half]
  alignas(16) SurItem items[2][kItemBatch];  // this block's query-block descriptors, two batches
  // FP32 biases of layers 2 and 3 in accumulator order: [layer][wave of the
  // group][accumulator block][lane half][register] (register r of a lane
  // holds output row (r / 4) * 8 + half * 4 + r % 4 of the 32-row block)
  alignas(16) float bias[2][kGroupWaves][kFB][2][16];
  float b4;
};

// First-layer K slots: chunk 0 = [own f0..f6, flag slot (zero weight)] for
// lanes 0-31 and [neighbour f7..f13, f14] for lanes 32-63 (the neighbour
// record's first 16 bytes); chunk 1 = [f15, f16, 1, 1, 1, zeros] for lanes
// 0-31 (the three ones meet the bias split into three bfloat16 parts) and
// zeros for lanes 32-63.  Returns the feature index, kFeat for the bias
// slots, -1 for zero slots.
__device__ __forceinline__ int first_layer_feature(int c, int half, int e) {
  if (c == 0) return half ? 7 + e : (e < 7 ? e : -1);
  if (half != 0) return -1;
  return e < 2 ? 15 + e : (e < 5 ? kFeat : -1);
}

// A bias as three bfloat16 parts (high, middle, low) that sum to it exactly:
// each part takes the next 8 significant bits of what remains, and the
// remainders are exact in FP32.  MFMA products with 1.0 are exact and their
// FP32 sum is the bias again, so a folded bias equals an FP32 one.
__device__ __forceinline__ void split_bias(float b, uint16_t& hi, uint16_t& mid, uint16_t& lo) {
  hi = f2bf(b);
  const float r1 = b - bf2f(hi);
  mid = f2bf(r1);
  lo = f2bf(r1 - bf2f(mid));
}


// 256-wide layer for this wave's kWaveRows output features over 32 queries
// (`row` = the input activation row of the lane's query + (lane/32)*8): the
// accumulators start from the layer's FP32 bias (`bias16`, as in layer256x2),
// read from LDS with the first operands.
__device__ __forceinline__ void layer256(const bf16x8_t (&w)[kFB][16], const float* bias16, const uint16_t* row,
                                         f32x16_t (&acc)[kFB]) {
  __builtin_amdgcn_sched_barrier(0);
  bf16x8_t b[16];
#pragma unroll
  for (int fb = 0; fb < kFB; ++fb) acc[fb] = *reinterpret_cast<const f32x16_t*>(bias16 + fb * 32);
#pragma unroll
  for (int c = 0; c < kInflight; ++c) b[c] = load_bf16x8(row + c * 16);
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    if (c + kInflight < 16) b[c + kInflight] = load_bf16x8(row + (c + kInflight) * 16);
#pragma unroll
    for (int fb = 0; fb < kFB; ++fb) acc[fb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w[fb][c], b[c], acc[fb], 0, 0, 0);
  }
  // Issue order: the accumulator starts and the first kInflight operand
  // reads, then per chunk its kFB MFMAs and the read kInflight chunks ahead.
  __builtin_amdgcn_sched_group_barrier(0x100, kFB * 4 + kInflight, 0);
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    __builtin_amdgcn_sched_group_barrier(0x008, kFB, 0);
    if (c + kInflight < 16) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
  }
  __builtin_amdgcn_sched_barrier(0);
}

// ReLU of two packed bfloat16 values: a signed 16-bit max with 0 on each
// half (a set sign bit reads as a negative integer), one VALU instruction.
// ReLU after rounding equals rounding after ReLU, so the stored activations
// are bfloat16(max(x, 0)).
__device__ __forceinline__ uint32_t relu_bf16x2(uint32_t x) {
  uint32_t r;
  asm("v_pk_max_i16 %0, %1, 0" : "=v"(r) : "v"(x));
  return r;
}

// ReLU, bfloat16, into the LDS rows of this lane's query (`dst` = row +
// base + (lane/32)*4).
__device__ __forceinline__ void store_block(const f32x16_t& acc, uint16_t* dst) {
#pragma unroll
  for (int q4 = 0; q4 < 4; ++q4) {
    uint2 v;
    v.x = relu_bf16x2(f2bf2(acc[q4 * 4 + 0], acc[q4 * 4 + 1]));
    v.y = relu_bf16x2(f2bf2(acc[q4 * 4 + 2], acc[q4 * 4 + 3]));
    *reinterpret_cast<uint2*>(dst + q4 * 8) = v;
  }
}

// The lane's share of the output layer for one accumulator block: its 16
// third-layer features, ReLU'd and rounded to bfloat16, dotted with the
// output weights of the same features (`w4v`, four per quarter, in
// registers), FP32 accumulation.
__device__ __forceinline__ float out_partial(const f32x16_t& acc, const uint2 (&w4v)[4]) {
  float t = 0.f;
#pragma unroll
  for (int q4 = 0; q4 < 4; ++q4) {
    const uint2 wv = w4v[q4];
    const uint32_t h01 = relu_bf16x2(f2bf2(acc[q4 * 4 + 0], acc[q4 * 4 + 1]));
    const uint32_t h23 = relu_bf16x2(f2bf2(acc[q4 * 4 + 2], acc[q4 * 4 + 3]));
    t = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, h01), __builtin_bit_cast(bf16x2_t, wv.x), t,
                                        false);
    t = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, h23), __builtin_bit_cast(bf16x2_t, wv.y), t,
                                        false);
  }
  return t;
}

// The lane's B operand of the first layer's first chunk for query block
// `it` (lanes 0-31: the query's own-feature row; lanes 32-63: the neighbour
// record's first 16 bytes) and the record's second 16 bytes.  Every query
// block lies inside its arm's padded rollout range, so the row is in bounds.
__device__ __forceinline__ void fetch_block(const SurInferArgs& A, int nA, int Hmax, int Nmax, const SurItem& it,
                                            int half, int q, uint4& x0, uint4& r1) {
  const uint32_t* rec = A.nbrec + (((size_t)it.arm * nA + it.nbr) * Hmax + it.h) * kNbrRec;
  const uint16_t* own = A.F + (((size_t)it.arm * Hmax + it.h) * Nmax + it.n0 + q) * 8;
  x0 = half ? *reinterpret_cast<const uint4*>(rec) : *reinterpret_cast<const uint4*>(own);
  r1 = *reinterpret_cast<const uint4*>(rec + 4);
}

__global__ __launch_bounds__(kInferThreads, 1) void k_sur_infer(SurInferArgs A) {
  __shared__ InferLds L;
  const int tid = threadIdx.x, lane = tid & 63;
  // Wave roles are wave-uniform: the group branch below is a scalar branch.
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int grp = wave / kGroupWaves, wq = wave % kGroupWaves, half = lane >> 5, q = lane & 31;
  // Loop invariants in registers and LDS: the loop's only global reads are
  // the first-layer inputs (a stage ahead) and the descriptor batches (a
  // batch ahead).
  const int nA = A.P->A, Hmax = A.P->Hmax, Nmax = A.P->Nmax;
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
  // Biases of layers 2 and 3 in accumulator order (read after the first
  // barrier below).
  for (int e = tid; e < (int)(sizeof(L.bias) / sizeof(float)); e += kInferThreads) {
    const int r = e % 16, hf = (e / 16) % 2, fb = (e / 32) % kFB, wv = (e / (32 * kFB)) % kGroupWaves;
    const int l = e / (32 * kFB * kGroupWaves);
    const int feat = wv * kWaveRows + fb * 32 + (r / 4) * 8 + hf * 4 + r % 4;
    (&L.bias[0][0][0][0][0])[e] = A.P32[mlp_b_off(1 + l) + feat];
  }
  const float* bias16 = &L.bias[grp][wq][0][half][0];

  const int G = gridDim.x;
  const int n_items = *A.count;  // descriptors written for this step (uniform)
  const int n_my = n_items > (int)blockIdx.x ? (n_items - 1 - (int)blockIdx.x) / G + 1 : 0;
  // A block without descriptors leaves before its first barrier (the whole
  // block agrees); the pipeline below needs at least one (its stand-in
  // stages reuse the last descriptor).
  if (n_my == 0) return;
  const int n_st = (n_my + kQB - 1) / kQB;  // stages holding query blocks (the last may hold a stand-in)
  const int fcol = wq * kWaveRows + half * 4;  // this lane's first feature within an accumulator block
  // Within a stage each layer's chains are straight-line code (the last
  // stage's second query block, past the end, is a stand-in: the last block's
  // inputs, writes suppressed); the edge stages skip the layers that have no
  // block yet or any more.  The activations start zeroed.
  for (int e = tid; e < (int)(2 * sizeof(L.act1) / sizeof(uint4)); e += kInferThreads)
    reinterpret_cast<uint4*>(&L.act1[0][0][0])[e] = make_uint4(0u, 0u, 0u, 0u);
  for (int e = tid; e < (int)(sizeof(L.part) / sizeof(float)); e += kInferThreads) (&L.part[0][0][0])[e] = 0.f;
  // Descriptors of this block's query blocks (block k at stage k is item
  // blockIdx.x + k*G): the first batch now; later batches are loaded by the
  // third wave of group A at the start of the batch before and written two
  // stages before they are first needed.  The staging and the prediction
  // store sit on waves of different SIMDs (2 of group A, 0 of group B).
  for (int e = tid; e < min(kItemBatch, n_my); e += kInferThreads)
    L.items[0][e] = A.items[blockIdx.x + (long long)e * G];
  auto item_at = [&](int k) -> SurItem {
    const int c = min(k, n_my - 1);
    return L.items[(c / kItemBatch) & 1][c % kItemBatch];
  };
  uint4 batch_next = make_uint4(0u, 0u, 0u, 0u);  // a descriptor, kept as a vector in registers
  // Group A's inputs of the next stage's query blocks, loaded a stage ahead.
  uint4 x0_next[kQB], r1_next[kQB];
#pragma unroll
  for (int qb = 0; qb < kQB; ++qb) x0_next[qb] = r1_next[qb] = make_uint4(0u, 0u, 0u, 0u);
  __syncthreads();
  if (grp == 0 && n_my > 0) {
#pragma unroll
    for (int qb = 0; qb < kQB; ++qb) fetch_block(A, nA, Hmax, Nmax, item_at(qb), half, q, x0_next[qb], r1_next[qb]);
  }
  // Each SIMD holds one wave of each group, and the two alternate between
  // MFMA-bound and latency-bound work within a stage: group B starts its
  // third-layer chain at the barrier while group A runs the first layer of
  // the next block, then group A runs its second-layer chain while group B
  // finishes the output layer.  Each group has a loop of
  // its own (the same number of stages, one barrier per stage) and keeps
  // its small weights in registers.
  if (grp == 0) {
    // First-layer A operands (bias folded into chunk 1).
    bf16x8_t w1[kFB][2];
#pragma unroll
    for (int fb = 0; fb < kFB; ++fb)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        uint16_t v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int k = first_layer_feature(c, half, e);
          const int r = row0 + fb * 32;
          v[e] = 0;
          if (k >= 0 && k < kFeat) v[e] = A.W16[mlp_w_off(0) + (long long)r * kFeat + k];
        }
        if (c == 1 && half == 0) split_bias(A.P32[mlp_b_off(0) + row0 + fb * 32], v[2], v[3], v[4]);
        w1[fb][c] = __builtin_bit_cast(
            bf16x8_t, make_uint4(v[0] | ((uint32_t)v[1] << 16), v[2] | ((uint32_t)v[3] << 16),
                                 v[4] | ((uint32_t)v[5] << 16), v[6] | ((uint32_t)v[7] << 16)));
      }
    for (int s = 0; s < n_st + 3; ++s) {
      // First layer of stage s's query blocks (the last block again past the
      // end), then the second layer of stage s-1's.  Stage s's inputs arrived
      // during the last stage; stage s+1's are requested now.
      uint4 x0s[kQB], r1s[kQB];
#pragma unroll
      for (int qb = 0; qb < kQB; ++qb) {
        x0s[qb] = x0_next[qb];
        r1s[qb] = r1_next[qb];
        fetch_block(A, nA, Hmax, Nmax, item_at(kQB * (s + 1) + qb), half, q, x0_next[qb], r1_next[qb]);
      }
      if (wq == 2 && lane < kItemBatch) {
        const int k = s % kStagesPerBatch, nb = s / kStagesPerBatch + 1, e = nb * kItemBatch + lane;
        if (k == 0 && e < n_my)
          batch_next = *reinterpret_cast<const uint4*>(A.items + blockIdx.x + (long long)e * G);
        if (k == kStagesPerBatch - 2 && e < n_my) *reinterpret_cast<uint4*>(&L.items[nb & 1][lane]) = batch_next;
      }
      // Edge stages (before the first block reaches a layer, after the last
      // has left it) skip that layer's chains: uniform branches around
      // whole chains, every barrier kept.
      if (s < n_st) {
#pragma unroll
      for (int qb = 0; qb < kQB; ++qb) {
        const uint4 x0w = x0s[qb], r1 = r1s[qb];
        // B operands: chunk 0 as loaded; chunk 1 = [f15, f16, 1, 1, 1, 0..]
        // (the record's fifth word, then the bias ones) for lanes 0-31 and
        // zeros.
        const bf16x8_t x0 = __builtin_bit_cast(bf16x8_t, x0w);
        const bf16x8_t x1 = __builtin_bit_cast(
            bf16x8_t, make_uint4(half ? 0u : r1.x, half ? 0u : 0x3F803F80u, half ? 0u : 0x3F80u, 0u));
        const f32x16_t zero = {};
        f32x16_t acc1[kFB];
#pragma unroll
        for (int fb = 0; fb < kFB; ++fb) {
          acc1[fb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w1[fb][0], x0, zero, 0, 0, 0);
          acc1[fb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w1[fb][1], x1, acc1[fb], 0, 0, 0);
        }
#pragma unroll
        for (int fb = 0; fb < kFB; ++fb) store_block(acc1[fb], &L.act1[s & 1][qb * 32 + q][fcol + fb * 32]);
      }
      }
      if (s >= 1 && s <= n_st) {
#pragma nounroll
        for (int qb = 0; qb < kQB; ++qb) {
          f32x16_t acc[kFB];
          layer256(w, bias16, &L.act1[(s - 1) & 1][qb * 32 + q][half * 8], acc);
#pragma unroll
          for (int fb = 0; fb < kFB; ++fb)
            store_block(acc[fb], &L.act2[(s - 1) & 1][qb * 32 + q][fcol + fb * 32]);
        }
      }
      __syncthreads();
    }
  } else {
    // Output weights of this lane's features.
    uint2 w4v[kFB][4];
#pragma unroll
    for (int fb = 0; fb < kFB; ++fb)
#pragma unroll
      for (int q4 = 0; q4 < 4; ++q4)
        w4v[fb][q4] = *reinterpret_cast<const uint2*>(A.W16 + mlp_w_off(3) + fcol + fb * 32 + q4 * 8);
    for (int s = 0; s < n_st + 3; ++s) {
      // First wave: the outputs of stage s-3 (its partial sums are complete
      // at the barrier), before the chains; then the third layer of stage
      // s-2's query blocks with the output layer folded into the epilogue.
      if (wq == 0) {
        // One query per lane (query block = lane half): the partial sums in
        // a fixed order, then the bias; one 128-byte line per block.
        const float* pr = &L.part[(s - 3) & 1][lane][0];
        float4 p[kParts / 4];
#pragma unroll
        for (int i = 0; i < kParts / 4; ++i) p[i] = *reinterpret_cast<const float4*>(pr + 4 * i);
        float y = 0.f;
#pragma unroll
        for (int i = 0; i < kParts / 4; ++i) y += (p[i].x + p[i].y) + (p[i].z + p[i].w);
        y += L.b4;
        const int k = kQB * (s - 3) + half;
        if (s >= 3 && k < n_my) A.y[((long long)blockIdx.x + (long long)k * G) * 32 + q] = y;
      }
      if (s >= 2 && s <= n_st + 1) {
        f32x16_t acc3[2][kFB];
        layer256x2(w, bias16, &L.act2[(s - 2) & 1][q][half * 8], &L.act2[(s - 2) & 1][32 + q][half * 8], acc3);
#pragma unroll
        for (int qb = 0; qb < kQB; ++qb) {
          float t = 0.f;
#pragma unroll
          for (int fb = 0; fb < kFB; ++fb) t += out_partial(acc3[qb][fb], w4v[fb]);
          L.part[(s - 2) & 1][qb * 32 + q][wq * 2 + half] = t;
        }
      }
      __syncthreads();
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

hipError_t launch_sur_states(const DevArm* arms, const Params* P, const SurModel* model, const float* mu,
                             const float* state, const float* eps, int n_arms, int npad_max, int hmax, uint16_t* F,
                             const BoardMeta* meta, const float* planq, uint32_t* rec, const uint8_t* screened,
                             SurItem* items, int* grp_first, int* count, unsigned long long* counts,
                             hipStream_t s) {
  constexpr int per_block = kStatesThreads / 8;
  const int groups = n_arms * n_arms * hmax;
  int gx = (npad_max + per_block - 1) / per_block;
  gx = std::max(gx, (groups + kStatesThreads - 1) / kStatesThreads);
  gx = std::max(gx, (groups + kItemsGroups - 1) / kItemsGroups);
  hipLaunchKernelGGL(k_sur_states, dim3(gx, n_arms + 2), dim3(kStatesThreads), 0, s, arms, P, model, mu, state, eps,
                     F, meta, planq, rec, screened, items, grp_first, count, counts);
  return hipGetLastError();
}

// The screen flag of every (arm, neighbour, step) group, one wave each, in
// the plane blockIdx.z = 0 (dispatched first, so its latency-bound waves
// overlap the noise), and the iteration's noise in the planes blockIdx.z =
// 1 + arm (as k_noise), ahead of the feature launch whose descriptor row
// reads the flags.
__global__ __launch_bounds__(kNoiseThreads) void k_noise_screen(const DevArm* __restrict__ arms,
                                                                const Params* __restrict__ Pp,
                                                                const StepState* __restrict__ ssp,
                                                                const float* __restrict__ chol,
                                                                float* __restrict__ eps, int k,
                                                                const SurModel* __restrict__ sm,
                                                                const BoardMeta* __restrict__ meta,
                                                                const float* __restrict__ mu_all,
                                                                const float* __restrict__ state,
                                                                const float* __restrict__ plan_read,
                                                                uint8_t* __restrict__ screened,
                                                                unsigned* __restrict__ hist) {
  const Params& P = *Pp;
  const uint32_t t = ssp->t;
  if (blockIdx.z > 0) {
    noise_at(arms, P, t, chol, eps, k, blockIdx.z - 1, blockIdx.y, blockIdx.x * kNoiseThreads + threadIdx.x);
    return;
  }
  const int ng = P.A * P.A * P.Hmax;
  const int g = ((int)(blockIdx.y * gridDim.x + blockIdx.x)) * (kNoiseThreads / kWave) + (int)(threadIdx.x / kWave);
  if (g >= ng) return;  // whole waves
  // The previous step's drop history is read; this step's is started in
  // the first iteration.
  screen_group(arms, P, sm, meta, mu_all, state, plan_read, t, hist + (size_t)((t + 1u) & 1u) * ng,
               k == 0 ? hist + (size_t)(t & 1u) * ng : nullptr, g, threadIdx.x & (kWave - 1), screened);
}

hipError_t launch_noise_screen(const DevArm* arms, const Params* P, const StepState* ss, const float* chol,
                               float* eps, int k, int n_arms, int hmax, int npad_max, const SurModel* model,
                               const BoardMeta* meta, const float* mu, const float* state, const float* plan_read,
                               uint8_t* screened, unsigned* hist, hipStream_t s) {
  // the screen plane holds gx * hmax blocks of kNoiseThreads / 64 waves, one per group
  constexpr int waves = kNoiseThreads / kWave;
  const int gx = std::max((npad_max + kNoiseThreads - 1) / kNoiseThreads, (n_arms * n_arms + waves - 1) / waves);
  hipLaunchKernelGGL(k_noise_screen, dim3(gx, hmax, n_arms + 1), dim3(kNoiseThreads), 0, s, arms, P, ss, chol, eps,
                     k, model, meta, mu, state, plan_read, screened, hist);
  return hipGetLastError();
}


hipError_t launch_sur_infer(const SurInferArgs& A, int grid, hipStream_t s) {
  if (!A.items || grid <= 0) return hipSuccess;  // no arm pair: nothing to predict
  hipLaunchKernelGGL(k_sur_infer, dim3(grid), dim3(kInferThreads), 0, s, A);
  return hipGetLastError();
}

hipError_t launch_init_params(float* p, uint32_t slo, uint32_t shi, hipStream_t s) {
  hipLaunchKernelGGL(k_init_params, dim3((unsigned)((kMlpParams + 255) / 256)), dim3(256), 0, s, p, slo, shi);
  return hipGetLastError();
}

}  // namespace mrs
