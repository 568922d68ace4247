// Device building blocks of the MR-STORM step for gfx950 (wave64).
// All FP32 arithmetic is written with explicit fused multiply-adds and the
// library is compiled with contraction off, so every site that evaluates the
// same expression produces the same bits (the debug capture and the scoring
// pass see identical sphere centres).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace mrs {

__device__ __forceinline__ float fmaf_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 products,
// key bumped by (0x9E3779B9, 0xBB67AE85) between rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3,
                                              uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // one 32 x 32 -> 64 product per word pair (a single v_mad_u64_u32)
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
    const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// u in (0,1): top 24 bits plus half an ulp, exact in FP32.
__device__ __forceinline__ float unit_open(uint32_t x) {
  return ((float)(x >> 8) + 0.5f) * 5.9604644775390625e-8f;
}

// Standard normals of rollout n, step h, iteration k, control step t of arm
// `arm`: counter (n, 2h+c, t, arm<<8|k) gives joints 4c..4c+3 by
// Box-Muller on word pairs (0,1) and (2,3), lanes cos, sin, cos, sin.
__device__ __forceinline__ void normals4(uint32_t slo, uint32_t shi, int arm, uint32_t t, int k, int n, int h,
                                         int c, float z[4]) {
  uint32_t c0 = (uint32_t)n, c1 = (uint32_t)(2 * h + c), c2 = t, c3 = ((uint32_t)arm << 8) | (uint32_t)k;
  philox4x32_10(c0, c1, c2, c3, slo, shi);
  const float r01 = sqrtf(-2.0f * logf(unit_open(c0)));
  const float r23 = sqrtf(-2.0f * logf(unit_open(c2)));
  float s1, co1, s3, co3;
  sincospif(2.0f * unit_open(c1), &s1, &co1);
  sincospif(2.0f * unit_open(c3), &s3, &co3);
  z[0] = r01 * co1;
  z[1] = r01 * s1;
  z[2] = r23 * co3;
  z[3] = r23 * s3;
}

// All joints 0..dof-1 (dof <= 8) of one rollout step.
__device__ __forceinline__ void normals8(uint32_t slo, uint32_t shi, int arm, uint32_t t, int k, int n, int h,
                                         float z[8]) {
  normals4(slo, shi, arm, t, k, n, h, 0, z);
  normals4(slo, shi, arm, t, k, n, h, 1, z + 4);
}

// The iteration's exploration noise of rollout n at step h of arm a, padded
// rollouts included, in the [H][7][Npad] per-arm layout that the rollout,
// manipulability, learned-feature and weighted-mean kernels read: sigma z
// (Sec. III-A's Gaussian sampling), or with the adapted covariance (Eqs. 3-4)
// L_h z, L_h the Cholesky factor of Sigma_h (`chol` non-null).
constexpr int kNoiseThreads = 256;
__device__ __forceinline__ void noise_at(const DevArm* __restrict__ arms, const Params& P, uint32_t t,
                                         const float* __restrict__ chol, float* __restrict__ eps, int k, int a,
                                         int h, int n) {
  const DevArm* arm = arms + a;
  if (h >= arm->H || n >= arm->Npad) return;
  const int Npad = arm->Npad;
  float z[8];
  normals8(P.seed_lo, P.seed_hi, a, t, k, n, h, z);
  float* out = eps + arm->eps_off + (size_t)h * 7 * Npad + n;
  if (chol) {
    const float* L = chol + ((size_t)a * P.Hmax + h) * kTri;
#pragma unroll
    for (int j = 0; j < 7; ++j) {
      float e = 0.f;
#pragma unroll
      for (int m = 0; m <= j; ++m) e = fmaf_(L[tri7(j, m)], z[m], e);
      out[(size_t)j * Npad] = e;
    }
  } else {
#pragma unroll
    for (int j = 0; j < 7; ++j) out[(size_t)j * Npad] = z[j] * P.sigma;
  }
}

// ---------------------------------------------------------------------------
// Rigid frame: rotation columns x, y, z and origin t.
struct Frame {
  float x[3], y[3], z[3], t[3];
};

__device__ __forceinline__ void frame_base(Frame& F, const DevArm* __restrict__ arm) {
  const float cy = arm->cyaw, sy = arm->syaw;
  F.x[0] = cy;  F.x[1] = sy; F.x[2] = 0.f;
  F.y[0] = -sy; F.y[1] = cy; F.y[2] = 0.f;
  F.z[0] = 0.f; F.z[1] = 0.f; F.z[2] = 1.f;
  F.t[0] = arm->base[0]; F.t[1] = arm->base[1]; F.t[2] = arm->base[2];
}

// Modified DH joint: F <- F RotX(alpha) TransX(a) RotZ(theta) TransZ(d).
__device__ __forceinline__ void frame_joint(Frame& F, float a, float ca, float sa, float d, float cq,
                                            float sq) {
  float yx[3], zx[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    F.t[i] = fmaf_(a, F.x[i], F.t[i]);
    yx[i] = fmaf_(sa, F.z[i], ca * F.y[i]);
    zx[i] = fmaf_(-sa, F.y[i], ca * F.z[i]);
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const float xi = F.x[i];
    F.x[i] = fmaf_(sq, yx[i], cq * xi);
    F.y[i] = fmaf_(-sq, xi, cq * yx[i]);
    F.z[i] = zx[i];
    F.t[i] = fmaf_(d, zx[i], F.t[i]);
  }
}

// All 7 link frames of a 7-DoF arm at joint positions q.
__device__ __forceinline__ void forward_kinematics(Frame F[7], const DevArm* __restrict__ arm,
                                                   const float q[8]) {
  Frame cur;
  frame_base(cur, arm);
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    float s, c;
    sincosf(q[k] + arm->off[k], &s, &c);
    frame_joint(cur, arm->a[k], arm->cal[k], arm->sal[k], arm->d[k], c, s);
    F[k] = cur;
  }
}

// World-frame point of body-frame point p.
__device__ __forceinline__ void frame_point(const Frame& F, float px, float py, float pz, float& wx,
                                            float& wy, float& wz) {
  wx = fmaf_(pz, F.z[0], fmaf_(py, F.y[0], fmaf_(px, F.x[0], F.t[0])));
  wy = fmaf_(pz, F.z[1], fmaf_(py, F.y[1], fmaf_(px, F.x[1], F.t[1])));
  wz = fmaf_(pz, F.z[2], fmaf_(py, F.y[2], fmaf_(px, F.x[2], F.t[2])));
}

// Signed gap between two spheres, evaluated in FP64 on FP32 inputs:
// |c_a - c_b| - r_a - r_b (Eq. 6 for one sphere pair).
__device__ __forceinline__ double sphere_gap64(float ax, float ay, float az, float ar, float bx,
                                               float by, float bz, float br) {
  const double dx = (double)ax - (double)bx, dy = (double)ay - (double)by,
               dz = (double)az - (double)bz;
  const double dd = dx * dx + dy * dy + dz * dz;
  return __builtin_sqrt(dd) - (double)ar - (double)br;
}

// max(0, 1 - max(0, rho)/B) in FP64.
__device__ __forceinline__ double hinge64(double rho, double B) {
  const double r = rho > 0.0 ? rho : 0.0;
  const double v = 1.0 - r / B;
  return v > 0.0 ? v : 0.0;
}

__device__ __forceinline__ bool wave_any(bool p) { return __ballot(p) != 0ull; }
// Lane permutations within rows of 16 (DPP): swap neighbours, swap pairs,
// mirror each half row, mirror the row.  All lanes must be active.
template <int CTRL>
__device__ __forceinline__ float dpp_f(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(x), __float_as_int(x), CTRL, 0xF, 0xF, false));
}
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;
// min / max over each run of 8 lanes (lanes 8k..8k+7), in all 8 lanes.
__device__ __forceinline__ float oct_min(float x) {
  x = fminf(x, dpp_f<kDppXor1>(x));
  x = fminf(x, dpp_f<kDppXor2>(x));
  return fminf(x, dpp_f<kDppHalfMirror>(x));
}
__device__ __forceinline__ float oct_max(float x) {
  x = fmaxf(x, dpp_f<kDppXor1>(x));
  x = fmaxf(x, dpp_f<kDppXor2>(x));
  return fmaxf(x, dpp_f<kDppHalfMirror>(x));
}
// max over the wave, in every lane: rows of 16 by DPP, then the four rows.
__device__ __forceinline__ float wave_max(float x) {
  x = oct_max(x);
  x = fmaxf(x, dpp_f<kDppMirror>(x));
  const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 0));
  const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 16));
  const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 32));
  const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 48));
  return fmaxf(fmaxf(r0, r1), fmaxf(r2, r3));
}
// Value of the first active lane, in every lane.
__device__ __forceinline__ float first_lane(float x) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}

}  // namespace mrs
