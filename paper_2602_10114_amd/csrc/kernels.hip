// gfx950 kernels of one MR-STORM control step (arXiv 2602.10114, Alg. 1):
//   k_sense      Sense + Shift: stage inputs, own distance to goal, priority
//                factors (Eq. 10), neighbour table, left shift of the means.
//   k_noise      SampleControls: the iteration's Gaussian noise of every
//                (arm, step, rollout), isotropic or from the adapted covariance.
//   k_rollout    Rollout for every arm in one launch: dynamics, forward
//                kinematics over the collision spheres, the stage cost of
//                Eq. 5 with the coordination term of Eqs. 6-9 (sphere pairs
//                culled per wave by bounding spheres, the rest filtered and
//                checked exactly), written per rollout step.
//   k_total      Eq. 1 totals from the per-step stage costs.
//   k_softmax    Eq. 2 weights, PickBest (Act).
//   k_wmean      Eq. 3 weighted sums per chunk of rollouts; k_wmean_fin (or
//                k_toplan after the last iteration) adds them in order and
//                applies Eq. 4.
//   k_toplan     ToPlan: integrate the means, forward kinematics, plan spheres.
//   k_publish    Publish: board write side -> read side.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "device.hpp"
#include "kernels.hpp"
#include "surrogate.hpp"

namespace mrs {

// Sphere sets scored against the own spheres at one rollout step are staged in
// LDS: obstacles (one set) and each published neighbour plan that reaches the
// step (one set each).  The set's hinge buffer B is folded into the staged
// radius, so the squared-gap expansion
//   |c_s - p_k|^2 - (r_s + r_k + B)^2 = E_s + F_k + c_s.w_xyz + r_s w_r,
//   E_s = |c_s|^2 - r_s^2,  w = -2 (p_k, r_k + B),  F_k = |p_k|^2 - (r_k + B)^2,
// is negative exactly when the pair's gap rho is below B, and the own-sphere
// terms do not depend on the set.  The FP64 gap takes p_k = -w_xyz / 2 (exact:
// w_xyz was formed by an exact doubling) and r_k from rr.
constexpr int kLdsSpheres = kMaxObs + (kMaxArms - 1) * kMaxSpheres;
constexpr int kMaxSets = kMaxArms;  // obstacles + up to 7 neighbours
static_assert(kMaxSets * kBodies <= 64, "one near bit per (set, body) in a 64-bit mask");

// Pair cull.  The staged spheres of a set are taken in groups (each obstacle
// alone; a neighbour plan in runs of 8, one body of a table sorted by body),
// each with a bounding sphere whose radius covers every member's centre
// offset, radius and the set's buffer B.  Every own body has a bounding
// sphere about a fixed point of its frame; the wave takes lane 0's centre and
// widens the radius by the largest distance of any lane's centre from it, so
// one sphere covers the body in all 64 rollouts.  A group whose centre is at
// least the two radii from that sphere has a gap of at least B + kCullPad -
// (FP32 rounding, below 0.005 m for coordinates within 6 m) to every own
// sphere of the body in every lane: no pair of it can contribute to the
// hinge, so the filter skips it.  The lanes test 64 (body, group) pairs at a
// time.  Self collision is culled the same way per pair of body halves.  The
// cost is unchanged bit for bit.
constexpr float kCullPad = 0.01f;
constexpr int kNbGroups = kMaxSpheres / 8;
constexpr int kMaxGroups = kMaxObs + (kMaxArms - 1) * kNbGroups;

struct LdsSets {
  float4 w[kLdsSpheres];
  float rr[kLdsSpheres];
  float F[kLdsSpheres];
  float4 slot[kMaxSpheres];    // body-frame spheres of the item's arm (slot order)
  float4 gq[kMaxGroups];       // group bounding spheres: centre, radius (+ B + pad)
  int set_k0[kMaxSets], set_n[kMaxSets];
  float set_buf[kMaxSets], set_wt[kMaxSets];
  // learned-distance counters of the current item (added by each wave's
  // lane 0), in the layout of the per-arm counter rows: live queries,
  // predicted far, waves skipped, audited misses (exact gap < B), audited
  // missed collisions (gap < 0)
  unsigned sur[5];
};

__device__ __forceinline__ void stage_sphere(LdsSets& L, int dst, float4 s, float buf) {
  L.rr[dst] = s.w;
  const float rb = s.w + buf;
  L.w[dst] = make_float4(-2.f * s.x, -2.f * s.y, -2.f * s.z, -2.f * rb);
  L.F[dst] = fmaf_(s.x, s.x, fmaf_(s.y, s.y, fmaf_(s.z, s.z, -rb * rb)));
}

// Filter value given to unused slots of a padded layout: never below the slack.
constexpr float kParked = 1.0e30f;

// Slack of the squared-gap filter, m^2.  FP32 rounding of the expansion is
// below 1e-5 m^2 for coordinates within 6 m of the origin (checked at init);
// a pair with true gap < B therefore always has a filter value < slack.
constexpr float kSlack = 1.0e-4f;

// Cached joint sines and cosines of one rollout step, and the arm constants
// the chain walk needs.
struct Chain {
  float c[7], s[7];
};

__device__ __forceinline__ void chain_angles(Chain& C, const DevArm* __restrict__ arm, const float q[8]) {
#pragma unroll
  for (int k = 0; k < 7; ++k) sincosf(q[k] + arm->off[k], &C.s[k], &C.c[k]);
}

// Advance a walking frame across joint k (frame of link k+1 = body k).
__device__ __forceinline__ void walk(Frame& W, const DevArm* __restrict__ arm, const Chain& C, int k) {
  frame_joint(W, arm->a[k], arm->cal[k], arm->sal[k], arm->d[k], C.c[k], C.s[k]);
}

// Own spheres of one body: u = (c, r + buf), E = |c|^2 - (r + buf)^2.  The
// compiler barrier keeps sphere centres from being hoisted or shared across
// passes (that would hold every centre of the arm live at once).
template <int LAY, int B_>
__device__ __forceinline__ void body_spheres(const Frame& Fb, const LdsSets& L, float buf, float ux[8],
                                             float uy[8], float uz[8], float ur[8], float E[8]) {
  constexpr int C = kLayoutCount[LAY][B_], S0 = kLayoutStart[LAY][B_];
  asm volatile("" ::: "memory");
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const float4 p = L.slot[S0 + j];
    float x, y, z;
    frame_point(Fb, p.x, p.y, p.z, x, y, z);
    const float rb = p.w + buf;
    const bool parked = p.w < 0.f;  // unused slot of a padded layout
    ux[j] = parked ? 0.f : x;
    uy[j] = parked ? 0.f : y;
    uz[j] = parked ? 0.f : z;
    ur[j] = parked ? 0.f : rb;
    E[j] = parked ? kParked : fmaf_(x, x, fmaf_(y, y, fmaf_(z, z, -rb * rb)));
  }
}

// min over the body's spheres and the staged spheres [k0, k0+K) of the
// squared-gap expansion (two staged spheres per iteration), with every own
// sphere of the body given the body's largest radius rmax: E = |c|^2 - rmax^2
// and, per staged sphere, G = F_k + rmax w_r, so a pair costs three FMAs.
// The value is never above the per-sphere one (r_s <= rmax, r_k + B >= 0),
// so every body with a pair whose gap is below B still falls below the slack.
template <int C>
__device__ __forceinline__ float filter_range_rmax(const float ux[8], const float uy[8], const float uz[8],
                                                   const float E[8], float rmax, const LdsSets& L, int k0,
                                                   int K, float g) {
  const int kend = k0 + K;
  int k = k0;
  for (; k + 1 < kend; k += 2) {
    const float4 w0 = L.w[k], w1 = L.w[k + 1];
    const float G0 = fmaf_(rmax, w0.w, L.F[k]), G1 = fmaf_(rmax, w1.w, L.F[k + 1]);
    float m0 = 3.0e38f, m1 = 3.0e38f;
#pragma unroll
    for (int j = 0; j < C; ++j) {
      float t0 = fmaf_(ux[j], w0.x, E[j]);
      float t1 = fmaf_(ux[j], w1.x, E[j]);
      t0 = fmaf_(uy[j], w0.y, t0);
      t1 = fmaf_(uy[j], w1.y, t1);
      t0 = fmaf_(uz[j], w0.z, t0);
      t1 = fmaf_(uz[j], w1.z, t1);
      m0 = fminf(m0, t0);
      m1 = fminf(m1, t1);
    }
    g = fminf(g, fminf(m0 + G0, m1 + G1));
  }
  if (k < kend) {
    const float4 w = L.w[k];
    const float Gk = fmaf_(rmax, w.w, L.F[k]);
    float m = 3.0e38f;
#pragma unroll
    for (int j = 0; j < C; ++j) {
      float t = fmaf_(ux[j], w.x, E[j]);
      t = fmaf_(uy[j], w.y, t);
      t = fmaf_(uz[j], w.z, t);
      m = fminf(m, t);
    }
    g = fminf(g, m + Gk);
  }
  return g;
}

// Own spheres of one body for the body-radius filters: centres,
// E = |c|^2 - (rmax + buf)^2, and rmax + buf with rmax the body's largest
// radius (unused slots: zero centre, E parked).
template <int LAY, int B_>
__device__ __forceinline__ float body_spheres_rmax(const Frame& Fb, const LdsSets& L, float buf, float ux[8],
                                                   float uy[8], float uz[8], float E[8]) {
  constexpr int C = kLayoutCount[LAY][B_], S0 = kLayoutStart[LAY][B_];
  asm volatile("" ::: "memory");
  float rmax = 0.f;
#pragma unroll
  for (int j = 0; j < C; ++j) rmax = fmaxf(rmax, L.slot[S0 + j].w);
  const float rb = rmax + buf, r2 = rb * rb;
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const float4 p = L.slot[S0 + j];
    float x, y, z;
    frame_point(Fb, p.x, p.y, p.z, x, y, z);
    const bool parked = p.w < 0.f;
    ux[j] = parked ? 0.f : x;
    uy[j] = parked ? 0.f : y;
    uz[j] = parked ? 0.f : z;
    E[j] = parked ? kParked : fmaf_(x, x, fmaf_(y, y, fmaf_(z, z, -r2)));
  }
  return rb;
}

// Filter pass over every staged set at once: body by body down the chain
// (one walking frame, each body's spheres built once), the running minimum of
// the squared-gap expansion with the body's largest own radius per set; bit
// 8*si + b of `near` is set when body b has a pair below the slack in set si.
// The exact pass tests the flagged bodies' pairs with their own radii.
// True when the group bounding sphere q may reach the body sphere bb (both
// radii in .w).
__device__ __forceinline__ bool group_near(float4 bb, float4 q) {
  const float dx = bb.x - q.x, dy = bb.y - q.y, dz = bb.z - q.z;
  const float d2 = fmaf_(dx, dx, fmaf_(dy, dy, dz * dz));
  const float R = bb.w + q.w;
  return d2 < R * R;
}

// Filter pass over the groups no cull removed.  Lane l takes neighbour group
// slot kMaxObs + l (nl: staged and scored) and obstacle l (ol);
// per body the two ballots give the groups near the wave's body sphere wb[b],
// and only their pairs are filtered (the body's spheres are built when it has
// any).  Set 0 holds the obstacles when obs_set is 1; neighbour set si holds
// the plan of ballot byte si - obs_set.
template <int LAY, int B_>
__device__ __forceinline__ void sets_filter(Frame& W, const DevArm* __restrict__ arm, const Chain& C,
                                            const LdsSets& L, const float4* wb, bool nl, bool ol, int obs_set,
                                            unsigned long long& near) {
  constexpr int Cb = kLayoutCount[LAY][B_];
  if constexpr (B_ < 7) walk(W, arm, C, B_);
  const float4 bb = wb[B_];
  if (bb.w >= 0.f) {
    const int lane = threadIdx.x & (kWave - 1);
    const float4 qn = L.gq[kMaxObs + min(lane, kMaxGroups - kMaxObs - 1)], qo = L.gq[lane];
    const unsigned long long nbm = __ballot(nl && group_near(bb, qn));
    const unsigned long long obm = __ballot(ol && group_near(bb, qo));
    if ((nbm | obm) != 0ull) {
      float ux[8], uy[8], uz[8], E[8];
      const float rmax = body_spheres_rmax<LAY, B_>(W, L, 0.f, ux, uy, uz, E);
      if (obm != 0ull) {
        float gb = 3.0e38f;
        for (unsigned long long m = obm; m != 0ull; m &= m - 1ull)
          gb = filter_range_rmax<Cb>(ux, uy, uz, E, rmax, L, __builtin_ctzll(m), 1, gb);
        near |= (gb < kSlack ? 1ull : 0ull) << B_;
      }
      for (unsigned long long m = nbm; m != 0ull;) {
        const int ord = __builtin_ctzll(m) >> 3;
        unsigned grp = (unsigned)(m >> (8 * ord)) & 0xFFu;
        m &= ~(0xFFull << (8 * ord));
        const int si = ord + obs_set;
        const int k0 = L.set_k0[si], K = L.set_n[si];
        float gb = 3.0e38f;
        for (; grp != 0u; grp &= grp - 1u) {
          const int ks = k0 + 8 * __builtin_ctz(grp);
          gb = filter_range_rmax<Cb>(ux, uy, uz, E, rmax, L, ks, min(8, k0 + K - ks), gb);
        }
        near |= (gb < kSlack ? 1ull : 0ull) << (8 * si + B_);
      }
    }
  }
  if constexpr (B_ + 1 < kBodies) sets_filter<LAY, B_ + 1>(W, arm, C, L, wb, nl, ol, obs_set, near);
}

// Exact FP64 gaps of the candidate pairs of one own body against one staged
// sphere: `cand` has bit j set for own sphere j, whose centre the caller
// holds in (ux, uy, uz)[j] (built from the body frame and the LDS table).
// One pass forms the candidates' FP32 gaps (no dependent loads) and marks
// each whose gap is below min(best, B, smallest FP32 gap so far) + 1e-4 m;
// then the marked candidates' FP64 gaps, their centres rebuilt with the same
// operations (the same FP32 values).  With the FP32 error of a gap below
// 2e-6 m (coordinates within 6 m), an unmarked candidate's FP64 gap exceeds
// min(best, B) or the FP64 gap of a marked candidate with a smaller FP32
// gap: the hinge and the audit's tests of the minimum against B and 0 are
// those of the full FP64 scan.
template <int S0, int Cb>
__device__ __forceinline__ void exact_candidates(const Frame& W, const LdsSets& L, unsigned cand, const float ux[8],
                                                 const float uy[8], const float uz[8], float px, float py, float pz,
                                                 float pr, float B, double& best) {
  const double lim = fmin(best, (double)B);
  float m32 = 3.0e38f;
  unsigned need = 0u;
#pragma unroll
  for (int j = 0; j < Cb; ++j) {
    if ((cand >> j) & 1u) {
      const float dx = ux[j] - px, dy = uy[j] - py, dz = uz[j] - pz;
      const float g32 = sqrtf(fmaf_(dx, dx, fmaf_(dy, dy, dz * dz))) - L.slot[S0 + j].w - pr;
      m32 = fminf(m32, g32);
      need |= (double)g32 < fmin(lim, (double)m32) + 1.0e-4 ? 1u << j : 0u;
    }
  }
  while (need) {
    const int j = __builtin_ctz(need);
    need &= need - 1u;
    const float4 p = L.slot[S0 + j];
    float x, y, z;
    frame_point(W, p.x, p.y, p.z, x, y, z);
    const double g = sphere_gap64(x, y, z, p.w, px, py, pz, pr);
    best = g < best ? g : best;
  }
}

// Exact pass for one set: the FP64 gap of every pair the filter can flag; the
// minimum over them is the set distance whenever that distance is below B.
// `fb` has bit b set for the bodies some lane flagged; only the groups the
// cull kept for a body can hold such pairs (qslot, ql: the lane's group slot
// of the set's kind; ord < 0: obstacles, group o = staged sphere o; else the
// plan of ballot byte ord, groups of 8 from k0).
template <int LAY, int B_>
__device__ __forceinline__ void set_refine(Frame& W, const DevArm* __restrict__ arm, const Chain& C,
                                           const LdsSets& L, int k0, int K, unsigned fb, const float4* wb,
                                           int qslot, bool ql, int ord, float B, double& best) {
  constexpr int Cb = kLayoutCount[LAY][B_], S0 = kLayoutStart[LAY][B_];
  if ((fb >> B_) == 0u) return;  // no flagged body at or past B_
  if constexpr (B_ < 7) walk(W, arm, C, B_);
  if ((fb >> B_) & 1u) {
    float ux[8], uy[8], uz[8], ur[8], E[8];
    body_spheres<LAY, B_>(W, L, 0.f, ux, uy, uz, ur, E);
    float rmax = 0.f;
#pragma unroll
    for (int j = 0; j < Cb; ++j) rmax = fmaxf(rmax, L.slot[S0 + j].w);
    const unsigned long long kept = __ballot(ql && group_near(wb[B_], L.gq[qslot]));
    for (unsigned long long m = ord < 0 ? kept : (kept >> (8 * ord)) & 0xFFull; m != 0ull; m &= m - 1ull) {
      const int g = __builtin_ctzll(m);
      const int ka = ord < 0 ? g : k0 + 8 * g;
      const int kb = ord < 0 ? g + 1 : min(k0 + K, ka + 8);
      for (int k = ka; k < kb; ++k) {
        const float4 w = L.w[k];
        const float Fk = L.F[k];
        // Lower bound of the body's pair values for staged sphere k (each
        // radius term r_s w_r is at least rmax w_r, w_r <= 0): k holds no
        // candidate when the bound reaches the slack in every lane.
        float mk = 3.0e38f;
#pragma unroll
        for (int j = 0; j < Cb; ++j) mk = fminf(mk, fmaf_(uz[j], w.z, fmaf_(uy[j], w.y, fmaf_(ux[j], w.x, E[j]))));
        if (!wave_any(mk + fmaf_(rmax, w.w, Fk) < kSlack)) continue;
        unsigned cand = 0;
#pragma unroll
        for (int j = 0; j < Cb; ++j) {
          float t = fmaf_(ux[j], w.x, E[j]);
          t = fmaf_(uy[j], w.y, t);
          t = fmaf_(uz[j], w.z, t);
          t = fmaf_(ur[j], w.w, t);
          cand |= (t + Fk < kSlack ? 1u : 0u) << j;
        }
        if (cand)
          exact_candidates<S0, Cb>(W, L, cand, ux, uy, uz, -0.5f * w.x, -0.5f * w.y, -0.5f * w.z, L.rr[k], B, best);
      }
    }
  }
  if constexpr (B_ + 1 < kBodies) set_refine<LAY, B_ + 1>(W, arm, C, L, k0, K, fb, wb, qslot, ql, ord, B, best);
}

// Self collision: sphere pairs on bodies at least two apart in the chain.  A
// second walking frame runs from body B1 down the chain to every B2 > B1.
// The cull keeps half pairs: K.k[h1][h2] has bit 8*B1+B2 set when half h1 of
// body B1 and half h2 of body B2 (slots [0, (C+1)/2) and the rest) may touch
// in some lane; only their sphere pairs are visited.  The filter pass gives
// body B1's spheres its largest radius (rmb = rmax + buffer, three FMAs per
// pair) and sets bit 8*B1+B2 of `near` for a body pair with a value below
// the slack; the exact pass tests the flagged body pairs sphere by sphere and
// visits only pairs some lane flagged.  A walk stops after the last kept pair
// of its body.
struct SelfKeep {
  unsigned long long k[2][2];
};

template <int LAY, int B1, int B2>
__device__ __forceinline__ void self_inner(Frame& W2, const Frame& W1, const DevArm* __restrict__ arm,
                                           const Chain& C, const LdsSets& L, float buf, const float ux[8],
                                           const float uy[8], const float uz[8], const float ur[8],
                                           const float E[8], float rmb, unsigned row, const SelfKeep& K,
                                           float hbuf, bool refine, unsigned long long& near, double& best) {
  constexpr int C1 = kLayoutCount[LAY][B1], S1 = kLayoutStart[LAY][B1], H1 = (C1 + 1) / 2;
  constexpr int C2 = kLayoutCount[LAY][B2], S2 = kLayoutStart[LAY][B2], H2 = (C2 + 1) / 2;
  constexpr int sh = 8 * B1 + B2;
  constexpr unsigned long long bit = 1ull << sh;
  if ((row >> B2) == 0u) return;  // no kept pair at or past B2
  if constexpr (B2 < 7) walk(W2, arm, C, B2);
  if constexpr (B2 >= B1 + 2) {
    if (((row >> B2) & 1u) && (!refine || wave_any((near & bit) != 0ull))) {
      // halves of B1 kept with each half of B2
      const unsigned m1h[2] = {(unsigned)((K.k[0][0] >> sh) & 1ull) | (unsigned)(((K.k[1][0] >> sh) & 1ull) << 1),
                               (unsigned)((K.k[0][1] >> sh) & 1ull) | (unsigned)(((K.k[1][1] >> sh) & 1ull) << 1)};
      float gp = 3.0e38f;
#pragma nounroll
      for (int i = 0; i < C2; ++i) {
        const unsigned m1 = m1h[i >= H2 ? 1 : 0];
        if (m1 == 0u) continue;
        asm volatile("" ::: "memory");
        const float4 p = L.slot[S2 + i];
        float x, y, z;
        frame_point(W2, p.x, p.y, p.z, x, y, z);
        const float r = p.w;
        const float rb = r + buf;
        const bool parked = r < 0.f;
        const float wx = parked ? 0.f : -2.f * x, wy = parked ? 0.f : -2.f * y;
        const float wz = parked ? 0.f : -2.f * z, wr = parked ? 0.f : -2.f * rb;
        const float Fk = parked ? kParked : fmaf_(x, x, fmaf_(y, y, fmaf_(z, z, -rb * rb)));
        if (refine) {
          unsigned cand = 0;
#pragma unroll
          for (int j = 0; j < C1; ++j) {
            if (!((m1 >> (j >= H1 ? 1 : 0)) & 1u)) continue;
            float t = fmaf_(ux[j], wx, E[j]);
            t = fmaf_(uy[j], wy, t);
            t = fmaf_(uz[j], wz, t);
            t = fmaf_(ur[j], wr, t);
            cand |= (t + Fk < kSlack ? 1u : 0u) << j;
          }
          if (cand) exact_candidates<S1, C1>(W1, L, cand, ux, uy, uz, x, y, z, r, hbuf, best);
        } else {
          float m = 3.0e38f;
#pragma unroll
          for (int j = 0; j < C1; ++j) {
            if (!((m1 >> (j >= H1 ? 1 : 0)) & 1u)) continue;
            m = fminf(m, fmaf_(uz[j], wz, fmaf_(uy[j], wy, fmaf_(ux[j], wx, E[j]))));
          }
          gp = fminf(gp, m + fmaf_(rmb, wr, Fk));
        }
      }
      if (!refine) near |= gp < kSlack ? bit : 0ull;
    }
  }
  if constexpr (B2 + 1 < kBodies)
    self_inner<LAY, B1, B2 + 1>(W2, W1, arm, C, L, buf, ux, uy, uz, ur, E, rmb, row, K, hbuf, refine, near, best);
}

template <int LAY, int B1>
__device__ __forceinline__ void self_outer(Frame& W1, const DevArm* __restrict__ arm, const Chain& C,
                                           const LdsSets& L, float buf, unsigned long long pairs,
                                           const SelfKeep& K, bool refine, unsigned long long& near,
                                           double& best) {
  if constexpr (B1 + 2 < kBodies) {
    walk(W1, arm, C, B1);
    const unsigned row = (unsigned)(pairs >> (8 * B1)) & 0xFFu;
    if (row != 0u) {
      float ux[8], uy[8], uz[8], ur[8], E[8];
      float rmb = 0.f;
      if (refine) {
        body_spheres<LAY, B1>(W1, L, buf, ux, uy, uz, ur, E);
      } else {
        rmb = body_spheres_rmax<LAY, B1>(W1, L, buf, ux, uy, uz, E);
#pragma unroll
        for (int j = 0; j < 8; ++j) ur[j] = 0.f;
      }
      Frame W2 = W1;
      self_inner<LAY, B1, B1 + 1>(W2, W1, arm, C, L, 0.f, ux, uy, uz, ur, E, rmb, row, K, buf, refine, near,
                                  best);
    }
    if ((pairs >> (8 * (B1 + 1))) != 0ull) self_outer<LAY, B1 + 1>(W1, arm, C, L, buf, pairs, K, refine, near, best);
  }
}

template <int LAY>
__device__ __forceinline__ float self_hinge(const DevArm* __restrict__ arm, const Chain& C,
                                            const LdsSets& L, float buf, const SelfKeep& K, unsigned& refines) {
  const unsigned long long pairs = K.k[0][0] | K.k[0][1] | K.k[1][0] | K.k[1][1];
  if (pairs == 0ull) return 0.f;
  unsigned long long near = 0ull;
  double best = 1.0e300;
  Frame W;
  frame_base(W, arm);
  self_outer<LAY, 0>(W, arm, C, L, buf, pairs, K, false, near, best);
  const bool any_near = near != 0ull;
  if (!wave_any(any_near)) return 0.f;
  // the exact pass walks only to the body pairs some lane flagged
  unsigned long long flagged = 0ull;
  for (unsigned long long m = pairs; m != 0ull; m &= m - 1ull) {
    const int b = __builtin_ctzll(m);
    if (wave_any(((near >> b) & 1ull) != 0ull)) flagged |= 1ull << b;
  }
  ++refines;
  frame_base(W, arm);
  self_outer<LAY, 0>(W, arm, C, L, buf, flagged, K, true, near, best);
  return any_near ? (float)hinge64(best, (double)buf) : 0.f;
}

// ---------------------------------------------------------------------------
// Work item = (arm, block of WPB x 64 rollouts, horizon tile); one workgroup
// of WPB waves per item, lane = rollout.  The WPB waves share one LDS copy of
// the sets staged at each rollout step (obstacles and neighbour plans), so a
// step's staging is done once per WPB waves; every arm's padded rollout
// count is a multiple of 64 x WPB (the host only picks such WPB), so no wave
// of an item lies past the arm's padded rollouts.  The launch bound asks for
// three waves per SIMD (168 VGPRs, some spilled to scratch): with the pair
// cull the kernel waits on latency more than on the ALU, and a third wave
// measured faster than two waves without spills.
template <int LAY, bool DBG, int SURM, int WPB>
__global__ __launch_bounds__(kWave * WPB, 3) void k_rollout(const DevArm* __restrict__ arms,
                                                         const Params* __restrict__ Pp,
                                                         const StepState* __restrict__ ssp,
                                                         const Item* __restrict__ items,
                                                         const float* __restrict__ mu_all,
                                                         const float* __restrict__ state,
                                                         const float* __restrict__ goal,
                                                         const float* __restrict__ goalR,
                                                         const float* __restrict__ obs,
                                                         const float* __restrict__ plan_read,
                                                         RolloutArgs A) {
  __shared__ LdsSets L;
  // learned distance: the waves' drop masks over the neighbour table at the
  // current step (bit i: every rollout of the wave predicted far from i)
  __shared__ unsigned s_wdrop[WPB];
  // each wave's body and half-body spheres at the current step (pair cull)
  __shared__ float4 s_wb[WPB][kBodies];
  __shared__ float4 s_wh[WPB][kBodies][2];
  // each lane's joints while the self and set checks run (one column per lane)
  __shared__ float s_qq[14][kWave * WPB];
  static_assert(kNbrRec == 8, "neighbour record layout of the learned distance");
  constexpr int kThreads = kWave * WPB;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  const Params& P = *Pp;
  const StepState& SS = *ssp;
  const int n_obs = SS.n_obs;
  // Obstacles are the same for every item of this launch; each is its own
  // cull group (slot o).
  for (int o = tid; o < n_obs; o += kThreads) {
    const float4 s = reinterpret_cast<const float4*>(obs)[o];
    stage_sphere(L, o, s, P.buf_env);
    L.gq[o] = make_float4(s.x, s.y, s.z, s.w + P.buf_env + kCullPad + 1.0e-4f);
  }

  for (int it = blockIdx.x; it < A.n_items; it += gridDim.x) {
    const Item item = items[it];
    const int a = item.arm;
    const DevArm* __restrict__ arm = arms + a;
    const int N = arm->N, H = arm->H;
    const int n = item.block * kThreads + tid;
    const bool live = n < N;
    const float* __restrict__ mu = mu_all + (size_t)a * P.Hmax * 7;
    // The iteration's noise (drawn by k_noise before the launch), column n.
    const float* __restrict__ eps = A.eps + arm->eps_off + n;
    const int Npad = arm->Npad;
    __syncthreads();
    if (tid < kWave) L.slot[tid] = reinterpret_cast<const float4*>(arm->slot)[tid];
    if (SURM && tid == 0)
      for (int c2 = 0; c2 < 5; ++c2) L.sur[c2] = 0u;
    float q[8], qd[8];
#pragma unroll
    for (int j = 0; j < 7; ++j) {
      q[j] = state[(a * 7 + j) * 3 + 0];
      qd[j] = state[(a * 7 + j) * 3 + 1];
    }
    q[7] = qd[7] = 0.f;
    // Integration prefix of this horizon tile; the noise loads of eight
    // steps go out together.
    int hp = 0;
    for (; hp + 8 <= item.h0; hp += 8) {
      float z[8][7];
#pragma unroll
      for (int s2 = 0; s2 < 8; ++s2)
#pragma unroll
        for (int j = 0; j < 7; ++j) z[s2][j] = eps[(size_t)((hp + s2) * 7 + j) * Npad];
#pragma unroll
      for (int s2 = 0; s2 < 8; ++s2)
#pragma unroll
        for (int j = 0; j < 7; ++j) {
          const float u = z[s2][j] + mu[(hp + s2) * 7 + j];
          qd[j] = fmaf_(P.dt, u, qd[j]);
          q[j] = fmaf_(P.dt, qd[j], q[j]);
        }
    }
    for (; hp < item.h0; ++hp) {
      float z[7];
#pragma unroll
      for (int j = 0; j < 7; ++j) z[j] = eps[(size_t)(hp * 7 + j) * Npad];
#pragma unroll
      for (int j = 0; j < 7; ++j) {
        const float u = z[j] + mu[hp * 7 + j];
        qd[j] = fmaf_(P.dt, u, qd[j]);
        q[j] = fmaf_(P.dt, qd[j], q[j]);
      }
    }
    const float* __restrict__ gR = goalR + a * 9;
    const float* __restrict__ g = goal + a * 7;
    const int nnb = SS.nb_count[a];
    unsigned long long pairs = 0;
    unsigned set_passes = 0, set_refines = 0, self_refines = 0;
    for (int h = item.h0; h < item.h1; ++h) {
      // Learned distance: a neighbour is dropped for this wave at step h
      // when every rollout of the wave is far: live, both arms' joints
      // inside the training box, prediction at least the margin.  Taken
      // first, while few values are live.  The masks go to LDS before the
      // staging barrier below (the previous step's staging, their last
      // reader, finished at the barrier after it).
      unsigned wdrop = 0u;
      if (SURM) {
        // Uniform row bases plus the lane's rollout index (32-bit offsets).
        const uint16_t* Frow = A.sur_F + (((size_t)a * P.Hmax + h) * P.Nmax) * 8;
        const bool own_in = Frow[(uint32_t)n * 8u + 7u] != 0;
        unsigned nq = 0u, nf = 0u;
        for (int i = 0; i < nnb; ++i) {
          const Nb nb = SS.nb[a][i];
          if (h >= nb.H) continue;
          const size_t pi = (size_t)a * P.A + nb.arm;
          const int first = A.sur_grp[pi * P.Hmax + h];  // uniform; -1: no prediction
          float y = __builtin_nanf("");
          if (first >= 0) y = (A.sur_y + (size_t)first * 32)[(uint32_t)n];
          const bool nb_in = (A.sur_rec[(pi * P.Hmax + h) * kNbrRec + 5] & 1u) != 0u;
          const bool far = first >= 0 && live && own_in && nb_in && y >= A.sur_margin;
          const unsigned long long mf = __ballot(far);
          nq += (unsigned)__popcll(__ballot(live));
          nf += (unsigned)__popcll(mf);
          if (mf == ~0ull) {
            wdrop |= 1u << i;
            // drop history of the group for the next control step's screen
            if (A.sur_hist && lane == 0)
              atomicAdd(A.sur_hist + ((size_t)(SS.t & 1u) * P.A * P.A + pi) * P.Hmax + h, 1u);
          }
          if (DBG && live) {
            const size_t o = (pi * P.Hmax + h) * P.Nmax + n;
            A.dbg_pred[o] = y;
            A.dbg_skip[o] = first < 0 ? 2 : (far ? 1 : 0);
          }
        }
        if (lane == 0) {
          s_wdrop[wv] = wdrop;
          if (WPB == 1) {
            L.sur[0] += nq;
            L.sur[1] += nf;
          } else {
            atomicAdd(&L.sur[0], nq);
            atomicAdd(&L.sur[1], nf);
          }
        }
      }

      float z[7];
#pragma unroll
      for (int j = 0; j < 7; ++j) z[j] = eps[(size_t)(h * 7 + j) * Npad];
#pragma unroll
      for (int j = 0; j < 7; ++j) {
        const float e = z[j];
        const float u = e + mu[h * 7 + j];
        qd[j] = fmaf_(P.dt, u, qd[j]);
        q[j] = fmaf_(P.dt, qd[j], q[j]);
      }
      Chain C;
      chain_angles(C, arm, q);
      // Stage the sets scored at step h: obstacles (set 0) and every
      // published neighbour plan that reaches this step (Sec. IV-C: the
      // shorter of the two horizons applies).  A neighbour dropped by every
      // wave of the item is not staged in learned mode (SURM 1); the audit
      // (SURM 2) stages it and marks it for the waves that dropped it.
      __syncthreads();
      const int obs_set = n_obs > 0 ? 1 : 0;
      if (n_obs > 0 && tid == 0) {
        L.set_k0[0] = 0;
        L.set_n[0] = n_obs;
        L.set_buf[0] = P.buf_env;
        L.set_wt[0] = P.w_coll;
      }
      // Neighbour i of the arm's table is set obs_set + i, with its spheres
      // at kMaxObs + 64 i and its groups at kMaxObs + 8 i; a set that is not
      // staged at this step has no spheres.  Wave w stages the plans i = w,
      // w + WPB, ...: each lane loads one sphere of every such plan (the
      // loads go out together), then writes it, and each run of 8 lanes
      // forms its group's bounding sphere by lane permutations.
      constexpr int kPer = (kMaxArms - 1 + WPB - 1) / WPB;
      float4 sv[kPer];
      int sS[kPer];
      float sA[kPer];
#pragma unroll
      for (int m = 0; m < kPer; ++m) {
        const int i = wv + m * WPB;
        sS[m] = 0;
        sA[m] = 0.f;
        sv[m] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (i < nnb) {
          const Nb nb = SS.nb[a][i];
          bool st = h < nb.H;
          if (SURM == 1 && st) {
            bool all = true;
#pragma unroll
            for (int w = 0; w < WPB; ++w) all = all && ((s_wdrop[w] >> i) & 1u) != 0u;
            st = !all;
          }
          if (st) {
            sS[m] = nb.S;
            sA[m] = nb.alpha;
            const float4* src = reinterpret_cast<const float4*>(plan_read) + ((size_t)nb.arm * P.Hmax + h) * P.Smax;
            if (lane < nb.S) sv[m] = src[lane];
          }
        }
      }
#pragma unroll
      for (int m = 0; m < kPer; ++m) {
        const int i = wv + m * WPB;
        if (i < nnb) {
          const int S = sS[m];
          if (S > 0) {
            const float4 p = sv[m];
            const bool v = lane < S;
            if (v) stage_sphere(L, kMaxObs + 64 * i + lane, p, P.buf_dyn);
            const float qx = 0.5f * (oct_min(v ? p.x : 3.0e38f) + oct_max(v ? p.x : -3.0e38f));
            const float qy = 0.5f * (oct_min(v ? p.y : 3.0e38f) + oct_max(v ? p.y : -3.0e38f));
            const float qz = 0.5f * (oct_min(v ? p.z : 3.0e38f) + oct_max(v ? p.z : -3.0e38f));
            const float dx = p.x - qx, dy = p.y - qy, dz = p.z - qz;
            const float rad = oct_max(v ? sqrtf(fmaf_(dx, dx, fmaf_(dy, dy, dz * dz))) + p.w : -3.0e38f);
            // slots of runs past the plan's last sphere get a sphere no body reaches
            if ((lane & 7) == 0)
              L.gq[kMaxObs + 8 * i + (lane >> 3)] =
                  v ? make_float4(qx, qy, qz, rad + P.buf_dyn + kCullPad + 1.0e-4f)
                    : make_float4(1.0e18f, 1.0e18f, 1.0e18f, 0.f);
          }
          if (lane == 0) {
            L.set_k0[obs_set + i] = kMaxObs + 64 * i;
            L.set_n[obs_set + i] = S;
            L.set_buf[obs_set + i] = P.buf_dyn;
            L.set_wt[obs_set + i] = P.w_dyn * sA[m];
          }
        }
      }
      const int nsets = obs_set + nnb;
      unsigned wskip = 0u;  // bit si: set si dropped for this wave
      if (SURM || DBG) {
        for (int i = 0; i < nnb; ++i) {
          const Nb nb = SS.nb[a][i];
          if (h >= nb.H) continue;
          bool wd = false;
          if (SURM) {
            wd = ((wdrop >> i) & 1u) != 0u;
            bool all = true;
#pragma unroll
            for (int w = 0; w < WPB; ++w) all = all && ((s_wdrop[w] >> i) & 1u) != 0u;
            if (wd && lane == 0) {
              if (WPB == 1) L.sur[2] += 1u;
              else atomicAdd(&L.sur[2], 1u);
            }
            if (SURM == 1 && all) continue;
          }
          if (wd) wskip |= 1u << (obs_set + i);
          if (DBG && !(SURM == 1 && wd)) pairs += (unsigned long long)arm->S * (unsigned long long)nb.S;
        }
      }
      __syncthreads();
      // Sets the wave scores: in learned mode the ones it did not drop; the
      // audit scores every set and zeroes the dropped ones' hinge.
      const unsigned wscored = SURM == 1 ? ~wskip : ~0u;

      // Pair cull (see kCullPad).  One walk down the chain gives the
      // centres of each body and of its two halves; lane 0 of the wave
      // stores their spheres for the wave (lane 0's centres, the radii
      // widened by the largest distance of a lane's point from lane 0's) in
      // s_wb and s_wh.  The same walk ends at the last link frame, where the
      // goal pose is scored.
      Frame W;
      frame_base(W, arm);
      float4* wb = s_wb[wv];
      float4(*wh)[2] = s_wh[wv];
#pragma unroll
      for (int b = 0; b < kBodies; ++b) {
        if (b < 7) walk(W, arm, C, b);
        // the body's centre and its two half centres, their lane-0 values
        // and the largest distance of any lane's point from them
        float4 c3[3];
        float dev = 0.f;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const float* o = k == 0 ? arm->bnd[b] : arm->hb[b][k - 1];
          float x, y, z;
          frame_point(W, o[0], o[1], o[2], x, y, z);
          c3[k] = make_float4(first_lane(x), first_lane(y), first_lane(z), o[3]);
          const float dx = x - c3[k].x, dy = y - c3[k].y, dz = z - c3[k].z;
          dev = fmaxf(dev, sqrtf(fmaf_(dx, dx, fmaf_(dy, dy, dz * dz))));
        }
        const float spread = wave_max(dev) + 1.0e-4f;
        if (lane == 0) {
          wb[b] = make_float4(c3[0].x, c3[0].y, c3[0].z, c3[0].w >= 0.f ? c3[0].w + spread : -1.f);
          wh[b][0] = make_float4(c3[1].x, c3[1].y, c3[1].z, c3[1].w >= 0.f ? c3[1].w + spread : -1.f);
          wh[b][1] = make_float4(c3[2].x, c3[2].y, c3[2].z, c3[2].w >= 0.f ? c3[2].w + spread : -1.f);
        }
      }
      // Lane l: neighbour group slot kMaxObs + l, obstacle l, and the self
      // body pair (l / 8, l % 8).  A half pair is kept when the two half
      // spheres (widened by the self buffer and kCullPad) may touch.
      const int qn_slot = kMaxObs + min(lane, kMaxGroups - kMaxObs - 1);
      const int lsi = min(obs_set + (lane >> 3), kMaxSets - 1);
      const bool nl = (lane >> 3) < nnb && L.set_n[lsi] > 0 && ((wscored >> lsi) & 1u);
      const bool ol = lane < n_obs && (wscored & 1u);
      SelfKeep skeep;
#pragma unroll
      for (int h1 = 0; h1 < 2; ++h1)
#pragma unroll
        for (int h2 = 0; h2 < 2; ++h2) {
          const float4 p1 = wh[lane >> 3][h1], p2 = wh[lane & 7][h2];
          const float4 pb = make_float4(p1.x, p1.y, p1.z, p1.w + P.buf_self + kCullPad);
          skeep.k[h1][h2] =
              __ballot((lane & 7) >= (lane >> 3) + 2 && p1.w >= 0.f && p2.w >= 0.f && group_near(pb, p2));
        }
      bool sets_kept = false;
      const float4 qn = L.gq[qn_slot], qo = L.gq[lane];
#pragma unroll
      for (int b = 0; b < kBodies; ++b) {
        const float4 bb = wb[b];
        sets_kept = sets_kept || wave_any(bb.w >= 0.f && ((nl && group_near(bb, qn)) || (ol && group_near(bb, qo))));
      }

      // Goal pose (Eq. 5, C_pose) at the end-effector point of the last link.
      float c;
      {
        float ex, ey, ez;
        frame_point(W, arm->tool[0], arm->tool[1], arm->tool[2], ex, ey, ez);
        const float dx = ex - g[0], dy = ey - g[1], dz = ez - g[2];
        const float pos = sqrtf(fmaf_(dx, dx, fmaf_(dy, dy, dz * dz)));
        float tr = 0.f;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          tr = fmaf_(gR[i * 3 + 0], W.x[i], tr);
          tr = fmaf_(gR[i * 3 + 1], W.y[i], tr);
          tr = fmaf_(gR[i * 3 + 2], W.z[i], tr);
        }
        const float pose = fmaf_(P.w_rot, (3.f - tr) * 0.25f, pos);
        // Safe stopping and joint limits.
        float stop = 0.f, joint = 0.f;
        const float frac = (float)(H - 1 - h) / (float)H;
#pragma unroll
        for (int j = 0; j < 7; ++j) {
          stop += fmaxf(0.f, fabsf(qd[j]) - arm->qdmax[j] * frac);
          joint += fmaxf(0.f, arm->qlo[j] + P.joint_margin - q[j]);
          joint += fmaxf(0.f, q[j] - arm->qhi[j] + P.joint_margin);
        }
        c = P.w_pose * pose;
        c = fmaf_(P.w_stop, stop, c);
        c = fmaf_(P.w_joint, joint, c);
        if (A.manip) c = fmaf_(P.w_manip, A.manip[((size_t)a * P.Hmax + h) * P.Nmax + n], c);
      }
      // The joints wait in LDS while the self and set checks run (fewer
      // registers live through them).
#pragma unroll
      for (int j = 0; j < 7; ++j) {
        s_qq[j][tid] = q[j];
        s_qq[7 + j][tid] = qd[j];
      }
      // Self collision.
      c = fmaf_(P.w_coll, self_hinge<LAY>(arm, C, L, P.buf_self, skeep, self_refines), c);
      // Obstacles and neighbours' plans (Eqs. 6, 8, 9): one filter pass over
      // the groups the cull kept, then per set the exact pass if some lane of
      // the wave may be within B.
      unsigned long long near_all = 0ull;
      if (sets_kept) {
        frame_base(W, arm);
        sets_filter<LAY, 0>(W, arm, C, L, wb, nl, ol, obs_set, near_all);
      }
#pragma nounroll
      for (int si = 0; si < nsets; ++si) {
        if (!((wscored >> si) & 1u)) continue;
        const int k0 = L.set_k0[si], K = L.set_n[si];
        if (K == 0) continue;
        const unsigned nearb = (unsigned)(near_all >> (8 * si)) & 0xFFu;
        const bool near = nearb != 0;
        ++set_passes;
        if (wave_any(near)) {
          ++set_refines;
          double best = 1.0e300;
          Frame W;
          frame_base(W, arm);
          unsigned fb = 0u;
#pragma unroll
          for (int b = 0; b < kBodies; ++b) fb |= wave_any((nearb >> b) & 1u) ? 1u << b : 0u;
          const bool obs = si < obs_set;
          set_refine<LAY, 0>(W, arm, C, L, k0, K, fb, wb, obs ? lane : qn_slot, obs ? ol : nl,
                             obs ? -1 : si - obs_set, L.set_buf[si], best);
          float hv = near ? (float)hinge64(best, (double)L.set_buf[si]) : 0.f;
          if (SURM == 2 && ((wskip >> si) & 1u)) {
            const bool hit = live && near;
            const unsigned m1 = (unsigned)__popcll(__ballot(hit && best < (double)L.set_buf[si]));
            const unsigned m2 = (unsigned)__popcll(__ballot(hit && best < 0.0));
            if (lane == 0) {
              if (WPB == 1) {
                L.sur[3] += m1;
                L.sur[4] += m2;
              } else {
                atomicAdd(&L.sur[3], m1);
                atomicAdd(&L.sur[4], m2);
              }
            }
            hv = 0.f;
          }
          c = fmaf_(L.set_wt[si], hv, c);
        }
      }
      // The stage cost goes out per step; Eq. 1's discounted sum is formed in
      // k_total over h in a fixed order, so it does not depend on the tiling.
      if (live) A.partial[((size_t)a * kMaxH + h) * P.Nmax + n] = c;
#pragma unroll
      for (int j = 0; j < 7; ++j) {
        asm volatile("" ::: "memory");
        q[j] = s_qq[j][tid];
        qd[j] = s_qq[7 + j][tid];
      }

      if (DBG && live) {
        const size_t row = ((size_t)a * P.Nmax + n) * P.Hmax + h;
#pragma unroll
        for (int j = 0; j < 7; ++j) {
          A.dbg_q[row * 7 + j] = q[j];
          A.dbg_qd[row * 7 + j] = qd[j];
        }
        float4* sp = reinterpret_cast<float4*>(A.dbg_sph) + row * P.Smax;
        Frame W;
        frame_base(W, arm);
#pragma unroll
        for (int b = 0; b < kBodies; ++b) {
          if (b < 7) walk(W, arm, C, b);
          for (int j = kLayoutStart[LAY][b]; j < kLayoutStart[LAY][b + 1]; ++j) {
            const int u = arm->slot_src[j];
            if (u < 0) continue;
            const float4 p = L.slot[j];
            float x, y, zz;
            frame_point(W, p.x, p.y, p.z, x, y, zz);
            sp[u] = make_float4(x, y, zz, p.w);
          }
        }
        A.dbg_stage[((size_t)a * P.Hmax + h) * P.Nmax + n] = c;
      }
    }
    if (DBG && live) atomicAdd(A.dbg_pairs + 4 * a, pairs);
    if (SURM) {
      // one atomic per counter and item, after every wave's last count
      __syncthreads();
      if (tid == 0) {
#pragma unroll
        for (int c2 = 0; c2 < 5; ++c2)
          if (L.sur[c2]) atomicAdd(A.sur_counts + kSurCounters * a + c2, (unsigned long long)L.sur[c2]);
      }
    }
    if (DBG && lane == 0) {
      atomicAdd(A.dbg_pairs + 4 * a + 1, (unsigned long long)set_passes);
      atomicAdd(A.dbg_pairs + 4 * a + 2, (unsigned long long)set_refines);
      atomicAdd(A.dbg_pairs + 4 * a + 3, (unsigned long long)self_refines);
    }
  }
}

// ---------------------------------------------------------------------------
// Sense + Shift for every arm (runs on the caller's input pointers, so it is
// launched outside the captured graph).
__global__ __launch_bounds__(256) void k_sense(SenseArgs A) {
  __shared__ float s_mu[kMaxArms * kMaxH * kMaxDof];
  // the read side of the board and the arms' sizes, loaded together up front
  __shared__ float s_bdist[kMaxArms], s_dnow[kMaxArms];
  __shared__ int s_bvalid[kMaxArms], s_S[kMaxArms], s_H[kMaxArms];
  const int tid = threadIdx.x;
  const Params& P = *A.P;
  StepState& SS = *A.ss;
  const int nA = P.A;
  if (tid < nA) {
    s_bvalid[tid] = A.meta->valid[0][tid];
    s_bdist[tid] = A.meta->dist[0][tid];
    s_S[tid] = A.arms[tid].S;
    s_H[tid] = A.arms[tid].H;
  }
  for (int i = tid; i < nA * 21; i += blockDim.x) A.st_state[i] = A.state[i];
  for (int i = tid; i < nA * 7; i += blockDim.x) A.st_goal[i] = A.goal[i];
  for (int i = tid; i < A.n_obs * 4; i += blockDim.x) A.st_obs[i] = A.obstacles[i];
  for (int i = tid; i < nA * P.Hmax * 7; i += blockDim.x) s_mu[i] = A.mu[i];
  __syncthreads();
  // Shift: mu_h <- mu_{h+1}, the last step keeps its value.
  for (int i = tid; i < nA * P.Hmax * 7; i += blockDim.x) {
    const int a = i / (P.Hmax * 7), r = i % (P.Hmax * 7), h = r / 7;
    const int H = A.arms[a].H;
    if (h + 1 < H) A.mu[i] = s_mu[i + 7];
  }
  // The adapted covariances and their factors shift with the means: each
  // (arm, entry) column belongs to one thread of a block-stride loop (8 arms
  // hold 448 columns, more than the block's threads) and moves its steps in
  // increasing order.
  if (P.cov) {
    for (int col = tid; col < nA * 2 * kTri; col += blockDim.x) {
      const int a = col / (2 * kTri), e = col % (2 * kTri);
      float* m = (e < kTri ? A.sig : A.chol) + (size_t)a * P.Hmax * kTri + e % kTri;
      const int H = A.arms[a].H;
      for (int h = 0; h + 1 < H; ++h) m[(size_t)h * kTri] = m[(size_t)(h + 1) * kTri];
    }
  }
  if (tid < nA) {
    const int a = tid;
    const DevArm* arm = A.arms + a;
    float q[8];
    for (int j = 0; j < 7; ++j) q[j] = A.state[(a * 7 + j) * 3];
    q[7] = 0.f;
    Frame F[7];
    forward_kinematics(F, arm, q);
    float ex, ey, ez;
    frame_point(F[6], arm->tool[0], arm->tool[1], arm->tool[2], ex, ey, ez);
    const float* g = A.goal + a * 7;
    const float dx = ex - g[0], dy = ey - g[1], dz = ez - g[2];
    const float dnow = sqrtf(fmaf_(dx, dx, fmaf_(dy, dy, dz * dz)));
    SS.dist_now[a] = dnow;
    s_dnow[a] = dnow;
    // Goal rotation from the (normalised) quaternion w, x, y, z.
    float w = g[3], x = g[4], y = g[5], z = g[6];
    const float inv = 1.0f / sqrtf(fmaf_(w, w, fmaf_(x, x, fmaf_(y, y, z * z))));
    w *= inv; x *= inv; y *= inv; z *= inv;
    float* R = A.goalR + a * 9;
    R[0] = 1.f - 2.f * (y * y + z * z); R[1] = 2.f * (x * y - w * z); R[2] = 2.f * (x * z + w * y);
    R[3] = 2.f * (x * y + w * z); R[4] = 1.f - 2.f * (x * x + z * z); R[5] = 2.f * (y * z - w * x);
    R[6] = 2.f * (x * z - w * y); R[7] = 2.f * (y * z + w * x); R[8] = 1.f - 2.f * (x * x + y * y);
  }
  if (tid == 0) {
    SS.t = A.t;
    SS.n_obs = A.n_obs;
    SS.u_out = A.u_out;
  }
  __syncthreads();
  // Priority factors against every published neighbour (Eq. 10), one thread
  // of wave 0 per (arm a, neighbour i), and the per-arm neighbour table in
  // increasing i (each entry's slot is the count of published neighbours
  // before it, from a ballot over the arm's 8 lanes).
  static_assert(kMaxArms * kMaxArms <= kWave, "the (arm, neighbour) threads form one wave");
  if (tid < kMaxArms * kMaxArms) {
    const int a = tid / kMaxArms, i = tid % kMaxArms;
    const bool in = a < nA && i < nA;
    const bool act = in && i != a && s_bvalid[i] != 0;
    float al = 0.f;
    if (act) {
      const float da = fmaxf(s_dnow[a], P.dist_floor);
      const float di = fmaxf(s_bdist[i], P.dist_floor);
      al = fminf(fmaxf(powf(da / di, P.tau), P.prio_min), P.prio_max);
    }
    if (in) SS.alpha[a][i] = al;
    const unsigned row = (unsigned)(__ballot(act) >> (kMaxArms * a)) & 0xFFu;
    if (act) {
      Nb nb;
      nb.arm = i;
      nb.S = s_S[i];
      nb.H = s_H[i];
      nb.pad = 0;
      nb.alpha = al;
      nb.pad1 = nb.pad2 = nb.pad3 = 0.f;
      SS.nb[a][__popc(row & ((1u << i) - 1u))] = nb;
    }
    if (in && i == 0) SS.nb_count[a] = __popc(row);
  }
}

// ---------------------------------------------------------------------------
// Eq. 1 totals, Eq. 2 weights and PickBest for one arm per block.
// (value, index) minimum with ties to the lower index.
__device__ __forceinline__ void argmin_merge(float& v, int& i, float v2, int i2) {
  if (v2 < v || (v2 == v && i2 < i)) {
    v = v2;
    i = i2;
  }
}

// Eq. 1 totals, one thread per rollout of every arm: C_n = sum_h gamma^h
// C_{n,h} as one FMA chain in step order, so the value does not depend on the
// rollout kernel's horizon tiling.
// Eq. 1 total of rollout n of arm a: the stage costs weighted by gamma^h,
// one FMA chain in step order.
__device__ __forceinline__ float rollout_total(const ReduceArgs& A, const Params& P, int a, int H, int n) {
  const float* stage = A.partial + (size_t)a * kMaxH * P.Nmax + n;
  float c = 0.f;
#pragma unroll 8
  for (int h = 0; h < H; ++h) c = fmaf_(P.gpow[h], stage[(size_t)h * P.Nmax], c);
  return c;
}

__global__ __launch_bounds__(256) void k_total(ReduceArgs A) {
  const int a = blockIdx.y;
  const int n = blockIdx.x * 256 + threadIdx.x;
  const DevArm* arm = A.arms + a;
  if (n >= arm->N) return;
  A.cost[(size_t)a * A.P->Nmax + n] = rollout_total(A, *A.P, a, arm->H, n);
}

// with_total: the block first forms its arm's Eq. 1 totals itself (small
// problems, where a separate k_total launch costs more than the work).
__global__ __launch_bounds__(1024) void k_softmax(ReduceArgs A, int with_total) {
  // Reductions: shuffles inside each wave, then the 16 wave results in a
  // fixed order (4 barriers in all).
  constexpr int kWaves = 1024 / kWave;
  __shared__ float s_v[kWaves];
  __shared__ int s_i[kWaves];
  __shared__ float s_bcast[2];
  __shared__ int s_nstar;
  const int a = blockIdx.x, tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  const Params& P = *A.P;
  const DevArm* arm = A.arms + a;
  const int N = arm->N;
  float* cost = A.cost + (size_t)a * P.Nmax;
  float best = 3.4e38f;
  int bi = 0x7fffffff;
  for (int n = tid; n < N; n += blockDim.x) {
    float c;
    if (with_total) {
      c = rollout_total(A, P, a, arm->H, n);
      cost[n] = c;  // read back below by the same thread only
    } else {
      c = cost[n];
    }
    if (c < best) { best = c; bi = n; }
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1)
    argmin_merge(best, bi, __shfl_xor(best, off), __shfl_xor(bi, off));
  if (lane == 0) {
    s_v[wv] = best;
    s_i[wv] = bi;
  }
  __syncthreads();
  if (tid == 0) {
    float v = s_v[0];
    int i = s_i[0];
    for (int k = 1; k < kWaves; ++k) argmin_merge(v, i, s_v[k], s_i[k]);
    s_bcast[0] = v;
    // All-NaN costs leave no minimum; fall back to rollout 0 so every index stays in range.
    s_nstar = i < N ? i : 0;
  }
  __syncthreads();
  const float m = s_bcast[0];
  const int nstar = s_nstar;
  const float inv_lambda = 1.0f / P.lambda;
  float z = 0.f;
  for (int n = tid; n < N; n += blockDim.x) z += expf(-(cost[n] - m) * inv_lambda);
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) z += __shfl_xor(z, off);
  if (lane == 0) s_v[wv] = z;
  __syncthreads();
  if (tid == 0) {
    float zs = s_v[0];
    for (int k = 1; k < kWaves; ++k) zs += s_v[k];
    s_bcast[1] = zs;
  }
  __syncthreads();
  const float zinv = 1.0f / s_bcast[1];
  float* w = A.w + (size_t)a * P.Nmax;
  for (int n = tid; n < N; n += blockDim.x) w[n] = expf(-(cost[n] - m) * inv_lambda) * zinv;
  if (tid < 7) {
    // U* into the staged copy and straight into the caller's array of this
    // step (its address came with Sense, outside the captured graph)
    const float* eps = A.eps + arm->eps_off;
    const float u = A.mu[(size_t)a * P.Hmax * 7 + tid] + eps[(size_t)tid * arm->Npad + nstar];
    A.u_out[a * 7 + tid] = u;
    float* uo = A.ss->u_out;
    if (uo) uo[a * 7 + tid] = u;
  }
  if (tid == 0) A.argmin[a] = nstar;
}

// Manipulability term of Eq. 5 for every rollout step: the rollout's joints
// (the iteration's noise, integrated as in the rollout kernel), the end-effector
// point by the same walking frame, the geometric Jacobian (column k = (z_k x
// (p_ee - o_k), z_k) from frame k), J J^T and its Cholesky factor, whose
// pivot product is sqrt(det(J J^T)); C_manip = max(0, 1 - that / thresh).
__global__ __launch_bounds__(kWave) void k_manip(const DevArm* __restrict__ arms, const Params* __restrict__ Pp,
                                                 const StepState* __restrict__ ssp, const float* __restrict__ mu_all,
                                                 const float* __restrict__ state, const float* __restrict__ eps,
                                                 float* __restrict__ out) {
  const Params& P = *Pp;
  const int a = blockIdx.y;
  const DevArm* arm = arms + a;
  const int n = blockIdx.x * kWave + threadIdx.x;
  if (n >= arm->Npad) return;
  const float* mu = mu_all + (size_t)a * P.Hmax * 7;
  float q[8], qd[8];
  for (int j = 0; j < 7; ++j) {
    q[j] = state[(a * 7 + j) * 3 + 0];
    qd[j] = state[(a * 7 + j) * 3 + 1];
  }
  q[7] = qd[7] = 0.f;
  for (int h = 0; h < arm->H; ++h) {
    float z[7];
    for (int j = 0; j < 7; ++j) z[j] = eps[arm->eps_off + ((size_t)h * 7 + j) * arm->Npad + n];
    for (int j = 0; j < 7; ++j) {
      const float u = z[j] + mu[h * 7 + j];
      qd[j] = fmaf_(P.dt, u, qd[j]);
      q[j] = fmaf_(P.dt, qd[j], q[j]);
    }
    Chain C;
    chain_angles(C, arm, q);
    Frame W;
    frame_base(W, arm);
    for (int k = 0; k < 7; ++k) walk(W, arm, C, k);
    float ee[3];
    frame_point(W, arm->tool[0], arm->tool[1], arm->tool[2], ee[0], ee[1], ee[2]);
    float G[21];  // J J^T, packed lower triangle of a 6x6
    for (int e = 0; e < 21; ++e) G[e] = 0.f;
    frame_base(W, arm);
    for (int k = 0; k < 7; ++k) {
      walk(W, arm, C, k);
      const float rx = ee[0] - W.t[0], ry = ee[1] - W.t[1], rz = ee[2] - W.t[2];
      float col[6];
      col[0] = W.z[1] * rz - W.z[2] * ry;
      col[1] = W.z[2] * rx - W.z[0] * rz;
      col[2] = W.z[0] * ry - W.z[1] * rx;
      col[3] = W.z[0];
      col[4] = W.z[1];
      col[5] = W.z[2];
      for (int i = 0; i < 6; ++i)
        for (int j = 0; j <= i; ++j) G[i * (i + 1) / 2 + j] = fmaf_(col[i], col[j], G[i * (i + 1) / 2 + j]);
    }
    float L[21], vol = 1.f;
    for (int j = 0; j < 6; ++j) {
      float d = G[j * (j + 1) / 2 + j];
      for (int m = 0; m < j; ++m) d -= L[j * (j + 1) / 2 + m] * L[j * (j + 1) / 2 + m];
      if (!(d > 0.f)) {
        vol = 0.f;
        break;
      }
      const float ljj = sqrtf(d);
      L[j * (j + 1) / 2 + j] = ljj;
      vol *= ljj;
      for (int i = j + 1; i < 6; ++i) {
        float v = G[i * (i + 1) / 2 + j];
        for (int m = 0; m < j; ++m) v -= L[i * (i + 1) / 2 + m] * L[j * (j + 1) / 2 + m];
        L[i * (i + 1) / 2 + j] = v / ljj;
      }
    }
    out[((size_t)a * P.Hmax + h) * P.Nmax + n] = fmaxf(0.f, 1.f - vol / P.manip_thresh);
  }
}

// SampleControls: the iteration's noise of every (arm, step, rollout) (see
// noise_at).  One thread per (arm, step, rollout), so the launch is wide
// whatever the horizon.
__global__ __launch_bounds__(kNoiseThreads) void k_noise(const DevArm* __restrict__ arms,
                                                         const Params* __restrict__ Pp,
                                                         const StepState* __restrict__ ssp,
                                                         const float* __restrict__ chol, float* __restrict__ eps,
                                                         int k) {
  noise_at(arms, *Pp, ssp->t, chol, eps, k, blockIdx.z, blockIdx.y, blockIdx.x * kNoiseThreads + threadIdx.x);
}

// Eq. 3 (weighted mean, and with covariance adaptation the weighted second
// moments), split over (chunk of 1024 rollouts, step, arm) so that the noise
// stream is read by enough workgroups to keep HBM busy.  Each thread reads
// four consecutive rollouts of the 7 noise rows (16-byte loads); the block
// reduces its sums with wave shuffles and then across its 4 waves in a fixed
// order and stores them as the chunk's partial.  k_wmean_fin adds the
// partials in chunk order (the result does not depend on the launch) and
// applies Eq. 4.
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__global__ __launch_bounds__(256) void k_wmean(ReduceArgs A) {
  __shared__ float s_w[4][kWmeanSums];
  const int chunk = blockIdx.x, h = blockIdx.y, a = blockIdx.z, tid = threadIdx.x;
  const int lane = tid & (kWave - 1), wv = tid / kWave;
  const Params& P = *A.P;
  const DevArm* arm = A.arms + a;
  const int N = arm->N, Npad = arm->Npad;
  const int nchunks = (N + kWmeanChunk - 1) / kWmeanChunk;
  if (h >= arm->H || chunk >= nchunks) return;
  const bool cov = P.cov != 0;
  const int nsum = cov ? kWmeanSums : 7;
  const int n0 = chunk * kWmeanChunk + 4 * tid;
  float s[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  float s2[kTri];
#pragma unroll
  for (int e = 0; e < kTri; ++e) s2[e] = 0.f;
  if (n0 < N) {
    // Npad is a multiple of 64 and the arm's block starts 64-float aligned,
    // so the four rollouts n0..n0+3 (< Npad) form one aligned 16-byte load;
    // rollouts from N on carry no weight.
    float4 w4 = *reinterpret_cast<const float4*>(A.w + (size_t)a * P.Nmax + n0);
    float wn[4] = {w4.x, w4.y, w4.z, w4.w};
    float en[4][7];
    const float* eps = A.eps + arm->eps_off + (size_t)h * 7 * Npad + n0;
#pragma unroll
    for (int j = 0; j < 7; ++j) {
      const float4 e4 = *reinterpret_cast<const float4*>(eps + (size_t)j * Npad);
      en[0][j] = e4.x;
      en[1][j] = e4.y;
      en[2][j] = e4.z;
      en[3][j] = e4.w;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (n0 + r >= N) {
        wn[r] = 0.f;
#pragma unroll
        for (int j = 0; j < 7; ++j) en[r][j] = 0.f;
      }
#pragma unroll
      for (int j = 0; j < 7; ++j) s[j] = fmaf_(wn[r], en[r][j], s[j]);
      if (cov) {
#pragma unroll
        for (int j = 0; j < 7; ++j) {
          const float we = wn[r] * en[r][j];
#pragma unroll
          for (int m = 0; m <= j; ++m) s2[tri7(j, m)] = fmaf_(we, en[r][m], s2[tri7(j, m)]);
        }
      }
    }
  }
#pragma unroll
  for (int j = 0; j < 7; ++j) {
    const float v = wave_sum(s[j]);
    if (lane == 0) s_w[wv][j] = v;
  }
  if (cov) {
#pragma unroll
    for (int e = 0; e < kTri; ++e) {
      const float v = wave_sum(s2[e]);
      if (lane == 0) s_w[wv][7 + e] = v;
    }
  }
  __syncthreads();
  if (tid < nsum)
    A.wpart[((((size_t)a * P.Hmax + h) * kWmeanMaxChunks) + chunk) * kWmeanSums + tid] =
        ((s_w[0][tid] + s_w[1][tid]) + s_w[2][tid]) + s_w[3][tid];
}

// Eq. 4 for one (arm a, step h) from the chunk totals t[0..6] (the weighted
// noise sums) and, with covariance adaptation, t[7..34] (the weighted second
// moments): the mean update for joint j (one thread per joint), and Eq. 3's
// weighted covariance, its EMA and the floored Cholesky factor (one thread).
__device__ __forceinline__ float mean_update(const ReduceArgs& A, const Params& P, int a, int h, int j,
                                             const float* t) {
  float* mu = A.mu + ((size_t)a * P.Hmax + h) * 7 + j;
  const float m0 = *mu;
  const float mt = m0 + t[j];
  const float m1 = fmaf_(P.alpha_mu, mt, (1.0f - P.alpha_mu) * m0);
  *mu = m1;
  return m1;
}

__device__ __forceinline__ void cov_update(const ReduceArgs& A, const Params& P, int a, int h, const float* t) {
  // Eq. 3: Sigma~ = sum_n w_n (U_n - mu~)(U_n - mu~)^T = sum_n w_n eps eps^T - ebar ebar^T
  // (U_n - mu~ = eps_n - ebar, ebar = sum_n w_n eps_n); Eq. 4: EMA; then the
  // Cholesky factor, pivots floored at sigma_floor^2.
  float* sg = A.sig + ((size_t)a * P.Hmax + h) * kTri;
  float* L = A.chol + ((size_t)a * P.Hmax + h) * kTri;
  float S[kTri], Lc[kTri];
  for (int j = 0; j < 7; ++j)
    for (int m = 0; m <= j; ++m) {
      const float st = t[7 + tri7(j, m)] - t[j] * t[m];
      S[tri7(j, m)] = fmaf_(P.alpha_sigma, st, (1.0f - P.alpha_sigma) * sg[tri7(j, m)]);
    }
  const float f2 = P.sigma_floor * P.sigma_floor;
  for (int j = 0; j < 7; ++j) {
    float d = S[tri7(j, j)];
    for (int m = 0; m < j; ++m) d -= Lc[tri7(j, m)] * Lc[tri7(j, m)];
    const float ljj = sqrtf(fmaxf(d, f2));
    Lc[tri7(j, j)] = ljj;
    for (int i = j + 1; i < 7; ++i) {
      float v = S[tri7(i, j)];
      for (int m = 0; m < j; ++m) v -= Lc[tri7(i, m)] * Lc[tri7(j, m)];
      Lc[tri7(i, j)] = v / ljj;
    }
  }
  for (int e = 0; e < kTri; ++e) {
    sg[e] = S[e];
    L[e] = Lc[e];
  }
}

// The chunk partials of one (arm, step) added in chunk order.
__device__ __forceinline__ float chunk_total(const ReduceArgs& A, const Params& P, int a, int h, int nchunks, int e) {
  const float* part = A.wpart + (((size_t)a * P.Hmax + h) * kWmeanMaxChunks) * kWmeanSums + e;
  // every chunk's partial is loaded before the sum (one memory round trip),
  // then added in chunk order
  float v[kWmeanMaxChunks];
#pragma unroll
  for (int c2 = 0; c2 < kWmeanMaxChunks; ++c2) v[c2] = c2 < nchunks ? part[(size_t)c2 * kWmeanSums] : 0.f;
  float t = v[0];
#pragma unroll
  for (int c2 = 1; c2 < kWmeanMaxChunks; ++c2)
    if (c2 < nchunks) t += v[c2];
  return t;
}

// Between optimisation iterations (K > 1): the totals of every (arm, step)
// and Eq. 4; after the last iteration k_toplan does the same.
__global__ __launch_bounds__(64) void k_wmean_fin(ReduceArgs A) {
  __shared__ float s_tot[kWmeanSums];
  const int h = blockIdx.x, a = blockIdx.y, tid = threadIdx.x;
  const Params& P = *A.P;
  const DevArm* arm = A.arms + a;
  if (h >= arm->H) return;
  const int nchunks = (arm->N + kWmeanChunk - 1) / kWmeanChunk;
  const bool cov = P.cov != 0;
  const int nsum = cov ? kWmeanSums : 7;
  if (tid < nsum) s_tot[tid] = chunk_total(A, P, a, h, nchunks, tid);
  __syncthreads();
  if (tid < 7) (void)mean_update(A, P, a, h, tid, s_tot);
  if (cov && tid == 32) cov_update(A, P, a, h, s_tot);
}

// ToPlan (one 256-thread block per arm): first the last iteration's
// weighted-mean totals and Eq. 4 (when `fin`), then the updated means
// integrated from the current state (one thread per joint), the link frames
// of every step (one thread per step, into LDS), and the plan spheres and
// planned joints of every (step, sphere) in parallel, into the board's write
// side.
constexpr int kToplanThreads = 256;
__global__ __launch_bounds__(kToplanThreads) void k_toplan(ReduceArgs A, int fin) {
  __shared__ float s_tot[kMaxH][kWmeanSums];
  __shared__ float s_mu[kMaxH * 7];
  __shared__ float s_q[kMaxH][8];
  __shared__ Frame s_F[kMaxH][7];
  __shared__ float4 s_slot[kMaxSpheres];
  __shared__ int s_src[kMaxSpheres], s_body[kMaxSpheres];
  const int a = blockIdx.x, tid = threadIdx.x;
  const Params& P = *A.P;
  const DevArm* arm = A.arms + a;
  const int H = arm->H;
  const int slots = kLayoutSlots[arm->layout];
  // the sensed joint of thread j < 7, loaded while the totals come in
  float q0 = 0.f, qd0 = 0.f;
  if (tid < 7) {
    q0 = A.st_state[(a * 7 + tid) * 3 + 0];
    qd0 = A.st_state[(a * 7 + tid) * 3 + 1];
  }
  // The sphere table for the plan spheres below (read after the barriers).
  for (int e = tid; e < slots; e += kToplanThreads) {
    s_slot[e] = reinterpret_cast<const float4*>(arm->slot)[e];
    s_src[e] = arm->slot_src[e];
    int b = 0;
    while (e >= kLayoutStart[arm->layout][b + 1]) ++b;
    s_body[e] = b;
  }
  // The arm's means (updated here after the last iteration) in LDS for the
  // integration below.
  if (fin) {
    const int nchunks = (arm->N + kWmeanChunk - 1) / kWmeanChunk;
    const bool cov = P.cov != 0;
    const int nsum = cov ? kWmeanSums : 7;
    for (int e = tid; e < H * nsum; e += kToplanThreads) s_tot[e / nsum][e % nsum] = chunk_total(A, P, a, e / nsum, nchunks, e % nsum);
    __syncthreads();
    for (int e = tid; e < H * 7; e += kToplanThreads) s_mu[e] = mean_update(A, P, a, e / 7, e % 7, s_tot[e / 7]);
    if (cov)
      for (int h = tid; h < H; h += kToplanThreads) cov_update(A, P, a, h, s_tot[h]);
  } else {
    for (int e = tid; e < H * 7; e += kToplanThreads) s_mu[e] = A.mu[(size_t)a * P.Hmax * 7 + e];
  }
  __syncthreads();
  if (tid < 7) {
    // One thread per joint (the joints integrate independently).
    const int j = tid;
    float q = q0, qd = qd0;
    for (int h = 0; h < H; ++h) {
      if (P.plan_mode == 0) {
        qd = fmaf_(P.dt, s_mu[h * 7 + j], qd);
        q = fmaf_(P.dt, qd, q);
      }
      // plan_mode 1 (the S_d ablation): the current configuration at every step
      s_q[h][j] = q;
    }
  }
  __syncthreads();
  for (int h = tid; h < H; h += kToplanThreads) {
    float q[8];
    for (int j = 0; j < 7; ++j) q[j] = s_q[h][j];
    q[7] = 0.f;
    Frame F[7];
    forward_kinematics(F, arm, q);
    for (int k = 0; k < 7; ++k) s_F[h][k] = F[k];
  }
  __syncthreads();
  // Spheres in the arm's slot order (the hand is rigid with the last link),
  // written to their user positions.
  float4* out = reinterpret_cast<float4*>(A.plan_write) + (size_t)a * P.Hmax * P.Smax;
  for (int e = tid; e < H * slots; e += kToplanThreads) {
    const int h = e / slots, jslot = e % slots;
    const int src = s_src[jslot];
    if (src < 0) continue;
    const int b = s_body[jslot];
    const float4 p = s_slot[jslot];
    float x, y, z;
    frame_point(s_F[h][b < 7 ? b : 6], p.x, p.y, p.z, x, y, z);
    out[(size_t)h * P.Smax + src] = make_float4(x, y, z, p.w);
  }
  for (int e = tid; e < H * 7; e += kToplanThreads)
    A.planq_write[((size_t)a * P.Hmax + e / 7) * 7 + e % 7] = s_q[e / 7][e % 7];
  if (tid == 0) {
    A.meta->dist[1][a] = A.ss->dist_now[a];
    A.meta->valid[1][a] = 1;
  }
}

// Publish: copy the masked arms' written plans to the read side, each arm's
// plan split over kPublishSplit blocks.
constexpr int kPublishSplit = 8;
__global__ __launch_bounds__(256) void k_publish(PublishArgs A) {
  const int a = blockIdx.x, part = blockIdx.y;
  if (!((A.mask >> a) & 1u)) return;
  if (!A.meta->valid[1][a]) return;
  const size_t n = (size_t)A.Hmax * A.Smax, nq = (size_t)A.Hmax * 7;
  const float4* src = reinterpret_cast<const float4*>(A.plan_write) + a * n;
  float4* dst = reinterpret_cast<float4*>(A.plan_read) + a * n;
  for (size_t i = part * 256 + threadIdx.x; i < n; i += 256 * kPublishSplit) dst[i] = src[i];
  for (size_t i = part * 256 + threadIdx.x; i < nq; i += 256 * kPublishSplit)
    A.planq_read[a * nq + i] = A.planq_write[a * nq + i];
  if (part == 0 && threadIdx.x == 0) {
    A.meta->dist[0][a] = A.meta->dist[1][a];
    A.meta->valid[0][a] = 1;
  }
}

__global__ void k_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t c0 = ctr[4 * i], c1 = ctr[4 * i + 1], c2 = ctr[4 * i + 2], c3 = ctr[4 * i + 3];
  philox4x32_10(c0, c1, c2, c3, key[2 * i], key[2 * i + 1]);
  out[4 * i] = c0;
  out[4 * i + 1] = c1;
  out[4 * i + 2] = c2;
  out[4 * i + 3] = c3;
}

// Plant stand-in: one step of the rollout dynamics under u.
__global__ void k_sim_execute(float* state, const float* u, int n, float dt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float acc = u[i];
  const float v = fmaf_(dt, acc, state[3 * i + 1]);
  state[3 * i + 0] = fmaf_(dt, v, state[3 * i + 0]);
  state[3 * i + 1] = v;
  state[3 * i + 2] = acc;
}

// Strided 3-D copy of floats (debug capture, board access, plan transpose):
// dst[i0*d0 + i1*d1 + i2*d2] = src[i0*s0 + i1*s1 + i2*s2].
__global__ void k_copy3d(const float* src, long long s0, long long s1, long long s2, float* dst,
                         long long d0, long long d1, long long d2, int n0, int n1, int n2) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long total = (long long)n0 * n1 * n2;
  if (i >= total) return;
  const long long i2 = i % n2, r = i / n2, i1 = r % n1, i0 = r / n1;
  dst[i0 * d0 + i1 * d1 + i2 * d2] = src[i0 * s0 + i1 * s1 + i2 * s2];
}

__global__ void k_set_meta(BoardMeta* meta, int arm, float dist, int valid) {
  meta->dist[0][arm] = dist;
  meta->valid[0][arm] = valid;
}

// ---------------------------------------------------------------------------
// Launchers.
template <int LAY, bool DBG, int SURM, int WPB>
static hipError_t launch_rollout_t(const RolloutArgs& A, int grid, hipStream_t s) {
  hipLaunchKernelGGL((k_rollout<LAY, DBG, SURM, WPB>), dim3(grid), dim3(kWave * WPB), 0, s, A.arms, A.P, A.ss,
                     A.items, A.mu, A.state, A.goal, A.goalR, A.obs, A.plan_read, A);
  return hipGetLastError();
}

template <int LAY, bool DBG, int SURM>
static hipError_t launch_rollout_w(const RolloutArgs& A, int waves, int grid, hipStream_t s) {
  switch (waves) {
    case 1: return launch_rollout_t<LAY, DBG, SURM, 1>(A, grid, s);
    case 2: return launch_rollout_t<LAY, DBG, SURM, 2>(A, grid, s);
    case 4: return launch_rollout_t<LAY, DBG, SURM, 4>(A, grid, s);
    default: return hipErrorInvalidValue;
  }
}

template <int LAY, bool DBG>
static hipError_t launch_rollout_s(const RolloutArgs& A, int waves, int grid, hipStream_t s) {
  if (!A.learned) return launch_rollout_w<LAY, DBG, 0>(A, waves, grid, s);
  return A.audit ? launch_rollout_w<LAY, DBG, 2>(A, waves, grid, s) : launch_rollout_w<LAY, DBG, 1>(A, waves, grid, s);
}

// The learned-distance variants (A.learned set; audited or not) are separate
// instantiations so that the exact kernel carries none of their bookkeeping.
hipError_t launch_rollout(const RolloutArgs& A, int layout, bool debug, int waves, int grid, hipStream_t s) {
  if (layout == 0)
    return debug ? launch_rollout_s<0, true>(A, waves, grid, s) : launch_rollout_s<0, false>(A, waves, grid, s);
  return debug ? launch_rollout_s<1, true>(A, waves, grid, s) : launch_rollout_s<1, false>(A, waves, grid, s);
}

hipError_t launch_sense(const SenseArgs& A, hipStream_t s) {
  hipLaunchKernelGGL(k_sense, dim3(1), dim3(256), 0, s, A);
  return hipGetLastError();
}

hipError_t launch_softmax(const ReduceArgs& A, int n_arms, int nmax, int hmax, hipStream_t s) {
  // Up to 64 stage costs per thread of the 1024-thread block the totals go
  // into the softmax launch; beyond that a launch of their own, one thread
  // per rollout, reads them at full width.
  const int with_total = (long long)nmax * hmax <= 64 * 1024 ? 1 : 0;
  if (!with_total) {
    hipLaunchKernelGGL(k_total, dim3((nmax + 255) / 256, n_arms), dim3(256), 0, s, A);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_softmax, dim3(n_arms), dim3(1024), 0, s, A, with_total);
  return hipGetLastError();
}

hipError_t launch_wmean(const ReduceArgs& A, int n_arms, int hmax, int nmax, bool fin, hipStream_t s) {
  const int chunks = (nmax + kWmeanChunk - 1) / kWmeanChunk;
  hipLaunchKernelGGL(k_wmean, dim3(chunks, hmax, n_arms), dim3(256), 0, s, A);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess || !fin) return e;
  hipLaunchKernelGGL(k_wmean_fin, dim3(hmax, n_arms), dim3(64), 0, s, A);
  return hipGetLastError();
}

hipError_t launch_toplan(const ReduceArgs& A, int n_arms, bool fin, hipStream_t s) {
  hipLaunchKernelGGL(k_toplan, dim3(n_arms), dim3(kToplanThreads), 0, s, A, fin ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_publish(const PublishArgs& A, int n_arms, hipStream_t s) {
  hipLaunchKernelGGL(k_publish, dim3(n_arms, kPublishSplit), dim3(256), 0, s, A);
  return hipGetLastError();
}

hipError_t launch_manip(const DevArm* arms, const Params* P, const StepState* ss, const float* mu, const float* state,
                        const float* eps, int n_arms, int npad_max, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_manip, dim3((npad_max + kWave - 1) / kWave, n_arms), dim3(kWave), 0, s, arms, P, ss, mu, state,
                     eps, out);
  return hipGetLastError();
}

hipError_t launch_noise(const DevArm* arms, const Params* P, const StepState* ss, const float* chol, float* eps, int k,
                        int n_arms, int hmax, int npad_max, hipStream_t s) {
  hipLaunchKernelGGL(k_noise, dim3((npad_max + kNoiseThreads - 1) / kNoiseThreads, hmax, n_arms), dim3(kNoiseThreads),
                     0, s, arms, P, ss, chol, eps, k);
  return hipGetLastError();
}

hipError_t launch_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_philox, dim3((n + 255) / 256), dim3(256), 0, s, ctr, key, out, n);
  return hipGetLastError();
}

hipError_t launch_sim_execute(float* state, const float* u, int n, float dt, hipStream_t s) {
  hipLaunchKernelGGL(k_sim_execute, dim3((n + 63) / 64), dim3(64), 0, s, state, u, n, dt);
  return hipGetLastError();
}

hipError_t launch_copy3d(const float* src, long long s0, long long s1, long long s2, float* dst,
                         long long d0, long long d1, long long d2, int n0, int n1, int n2, hipStream_t s) {
  const long long total = (long long)n0 * n1 * n2;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy3d, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, src, s0, s1, s2, dst,
                     d0, d1, d2, n0, n1, n2);
  return hipGetLastError();
}

hipError_t launch_set_meta(BoardMeta* meta, int arm, float dist, int valid, hipStream_t s) {
  hipLaunchKernelGGL(k_set_meta, dim3(1), dim3(1), 0, s, meta, arm, dist, valid);
  return hipGetLastError();
}

}  // namespace mrs
