// Host runtime of the MR-STORM step library: validation, HBM layout, the
// plan board, launch-shape tuning and hipGraph capture, and the C-ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"
#include "mrstorm.h"
#include "surrogate.hpp"

using namespace mrs;

// Device-side tables (the per-step powers of gamma, the LDS copy of the
// neighbours' planned joints in the inference kernel) are sized for the
// largest valid problem.
static_assert(kMaxH >= MPC_MAX_HORIZON && kMaxArms >= MPC_MAX_ARMS, "device tables cover every valid problem");
static_assert(kWmeanMaxChunks * kWmeanChunk >= MPC_MAX_ROLLOUTS, "weighted-mean partials cover every rollout count");

static thread_local std::string g_last_error;

// Working memory of mpc_surrogate_predict_noalloc: the bfloat16 input rows
// and two ping-pong bfloat16 activation buffers of MPC_PREDICT_NOALLOC_MAX
// queries.  One copy per GPU for the life of the process; host code reaches
// it only through the address hipGetSymbolAddress gives on that device.
constexpr size_t kNaQueries = MPC_PREDICT_NOALLOC_MAX;
constexpr size_t kNaX16Bytes = (kNaQueries * 17 * sizeof(uint16_t) + 255) / 256 * 256;
constexpr size_t kNaActBytes = kNaQueries * 256 * sizeof(uint16_t);
constexpr size_t kNaBytes = kNaX16Bytes + 2 * kNaActBytes;
static __device__ __align__(256) unsigned char scratch[kNaBytes];

// Per-device address of `scratch`, taken once per device with that device
// current (each GPU holds its own copy at its own address).
constexpr int kNaMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kNaMaxDevices] = {};

static hipError_t scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kNaMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// (start, end) HIP event pairs recorded around launches while profiling.
struct EventLog {
  std::vector<hipEvent_t> ev;
  size_t used = 0;
  // Records the start event; returns the end event to record after the launch.
  hipError_t begin(hipStream_t s, hipEvent_t* end) {
    while (ev.size() < used + 2) {
      hipEvent_t e;
      hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) return r;
      ev.push_back(e);
    }
    hipError_t r = hipEventRecord(ev[used], s);
    if (r != hipSuccess) return r;
    *end = ev[used + 1];
    used += 2;
    return hipSuccess;
  }
  // Sum of the recorded durations (ms) and their count; clears the record.
  hipError_t read(double* total_ms, int* n) {
    double tot = 0.0;
    for (size_t i = 0; i + 1 < used; i += 2) {
      float ms = 0.f;
      hipError_t r = hipEventElapsedTime(&ms, ev[i], ev[i + 1]);
      if (r != hipSuccess) return r;
      tot += ms;
    }
    *total_ms = tot;
    *n = (int)(used / 2);
    used = 0;
    return hipSuccess;
  }
  void destroy() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    ev.clear();
  }
};

struct mpc_ctx {
  int A = 0, Hmax = 0, Smax = 0, Nmax = 0, layout = 0;
  hipStream_t stream = nullptr;
  void* na_scratch = nullptr;          // this device's copy of `scratch` (allocation-free prediction)
  Params P{};
  std::vector<DevArm> harms;
  DevArm* d_arms = nullptr;
  Params* d_P = nullptr;
  StepState* d_ss = nullptr;
  BoardMeta* d_meta = nullptr;
  float* mu = nullptr;
  float* eps = nullptr;
  float* manip = nullptr;              // [A][Hmax][Nmax] C_manip of the iteration (w_manip > 0)
  float* sig = nullptr;                // [A][Hmax][28] adapted covariances (packed lower triangles)
  float* chol = nullptr;               // their Cholesky factors
  float* wpart = nullptr;              // weighted-mean chunk partials [A][Hmax][kWmeanMaxChunks][35]
  float* partial = nullptr;
  float* cost = nullptr;
  float* w = nullptr;
  float* st_state = nullptr;
  float* st_goal = nullptr;
  float* st_goalR = nullptr;
  float* st_obs = nullptr;
  float* plan[2] = {nullptr, nullptr};
  float* planq[2] = {nullptr, nullptr};
  float* u_stage = nullptr;
  int* argmin = nullptr;
  Item* d_items = nullptr;
  size_t items_cap = 0;
  int n_items = 0;
  int h_tile = 0, grid = 0, waves = 1;  // launch shape: horizon tile, workgroups, 64-rollout waves per workgroup
  int force_tile = 0, force_grid = 0, force_waves = 0;
  int pair_cull = 1;                   // 0: every body bound is unbounded (no pair is culled)
  unsigned long long* tune_counts = nullptr;  // learned-distance counters of tuner replays [A][kSurCounters]
  bool tuned = false;
  int n_published = 0;                 // arms whose plan has been published at least once
  std::vector<char> published;
  int untuned_steps = 0;
  hipGraphExec_t gexec = nullptr;
  bool debug = false;
  float* dbg_q = nullptr;
  float* dbg_qd = nullptr;
  float* dbg_sph = nullptr;
  float* dbg_stage = nullptr;
  unsigned long long* dbg_pairs = nullptr;
  uint32_t t = 0;
  bool stepped = false;
  bool profile = false;
  EventLog prof_roll;                   // bracketed rollout launches
  EventLog prof_infer;                  // bracketed learned-distance inference launches
  // learned arm-pair distance
  int collision_mode = 0;
  bool sur_ready = false;              // trained or set parameters present
  bool sur_audit = false;
  SurModel hmodel{};
  SurModel* d_model = nullptr;
  float* sur_p = nullptr;              // FP32 master parameters
  float* sur_m = nullptr;              // Adam moments
  float* sur_v = nullptr;
  float* sur_g = nullptr;              // gradient
  uint16_t* sur_p16 = nullptr;         // bfloat16 copy
  uint16_t* sur_F = nullptr;           // own-joint feature rows [A][Hmax][Nmax][8] (bfloat16)
  uint8_t* sur_skip = nullptr;         // decisions of live queries [A][A][Hmax][Nmax] (debug capture)
  float* sur_pred = nullptr;           // their predictions (debug capture)
  uint8_t* sur_screen = nullptr;       // groups that need no prediction [A][A][Hmax]
  // dropped 64-rollout checks per group, two control steps [2][A][A][Hmax]
  // (parity of the step counter); kHistNone = no history
  unsigned* sur_hist = nullptr;
  bool hist_stale = true;
  int* sur_grp = nullptr;              // first inference descriptor of each group [A][A][Hmax] (-1: none)
  int* sur_count = nullptr;            // descriptors of the step
  uint32_t* sur_nbrec = nullptr;       // neighbour records of the inference [A][A][Hmax][kNbrRec]
  float* sur_y = nullptr;              // predictions in descriptor order [items][32]
  bool sur_bufs = false;               // every learned-distance step buffer allocated
  unsigned long long* sur_counts = nullptr;  // [A][kSurCounters]
  SurItem* d_sur_items = nullptr;
  int n_sur_items = 0;
  int sur_grid = 0;
  std::string err;
  std::vector<void*> allocations;
};

static int fail(mpc_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  g_last_error = msg;
  return code;
}

#define HIPCHK(c, x)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (x);                                                                   \
    if (e_ != hipSuccess) return fail((c), MPC_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <class T>
static int dalloc(mpc_ctx* c, T** p, size_t count) {
  void* q = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc(&q, count * sizeof(T));
  if (e != hipSuccess) return fail(c, MPC_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  c->allocations.push_back(q);  // freed by mpc_destroy, also when the fill below fails
  e = hipMemset(q, 0, count * sizeof(T));
  if (e != hipSuccess) return fail(c, MPC_EHIP, std::string("hipMemset: ") + hipGetErrorString(e));
  *p = static_cast<T*>(q);
  return MPC_OK;
}

static bool finite_all(const float* p, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

// ---------------------------------------------------------------------------
static int build_arm(mpc_ctx* c, const mpc_arm_desc& d, int layout, DevArm& o) {
  memset(&o, 0, sizeof(o));
  o.dof = d.dof;
  o.S = d.n_spheres;
  o.N = d.n_rollouts;
  o.H = d.horizon;
  o.Npad = (d.n_rollouts + kWave - 1) / kWave * kWave;
  o.layout = layout;
  for (int k = 0; k < 7; ++k) {
    o.a[k] = d.dh[4 * k + 0];
    o.cal[k] = (float)std::cos((double)d.dh[4 * k + 1]);
    o.sal[k] = (float)std::sin((double)d.dh[4 * k + 1]);
    o.d[k] = d.dh[4 * k + 2];
    o.off[k] = d.dh[4 * k + 3];
    o.qlo[k] = d.q_lim[2 * k];
    o.qhi[k] = d.q_lim[2 * k + 1];
    o.qdmax[k] = d.qd_max[k];
  }
  o.base[0] = d.base[0];
  o.base[1] = d.base[1];
  o.base[2] = d.base[2];
  o.base[3] = d.base[3];  // yaw (the learned distance's canonical frame)
  o.cyaw = (float)std::cos((double)d.base[3]);
  o.syaw = (float)std::sin((double)d.base[3]);
  o.tool[0] = d.tool[0];
  o.tool[1] = d.tool[1];
  o.tool[2] = d.tool[2];
  for (int s = 0; s < kMaxSpheres; ++s) {
    o.slot_src[s] = -1;
    o.slot[s][0] = o.slot[s][1] = o.slot[s][2] = 0.f;
    o.slot[s][3] = -1.f;  // parked
  }
  int fill[kBodies] = {0};
  for (int s = 0; s < d.n_spheres; ++s) {
    const int b = d.sphere_link[s];
    const int slot = kLayoutStart[layout][b] + fill[b]++;
    for (int i = 0; i < 4; ++i) {
      o.slot[slot][i] = d.spheres[4 * s + i];
      o.usph[s][i] = d.spheres[4 * s + i];
    }
    o.slot_src[slot] = s;
    o.link[s] = b;
  }
  // Body bounding spheres for the kernels' pair culls: the middle of the
  // centres' box, the largest centre offset from it plus the largest radius,
  // with 1e-4 m for the FP32 forward kinematics (the frames stay orthonormal
  // to about 1e-6, and offsets are at most 1.5 m).
  for (int b = 0; b < kBodies; ++b) {
    double lo[3] = {1e30, 1e30, 1e30}, hi[3] = {-1e30, -1e30, -1e30}, rmax = 0.0;
    int cnt = 0;
    for (int sl = kLayoutStart[layout][b]; sl < kLayoutStart[layout][b + 1]; ++sl) {
      if (o.slot_src[sl] < 0) continue;
      ++cnt;
      for (int i = 0; i < 3; ++i) {
        lo[i] = std::min(lo[i], (double)o.slot[sl][i]);
        hi[i] = std::max(hi[i], (double)o.slot[sl][i]);
      }
      rmax = std::max(rmax, (double)o.slot[sl][3]);
    }
    if (cnt == 0) {
      o.bnd[b][0] = o.bnd[b][1] = o.bnd[b][2] = 0.f;
      o.bnd[b][3] = -1.f;
      continue;
    }
    float ctr[3];
    for (int i = 0; i < 3; ++i) ctr[i] = (float)(0.5 * (lo[i] + hi[i]));
    double rho = 0.0;
    for (int sl = kLayoutStart[layout][b]; sl < kLayoutStart[layout][b + 1]; ++sl) {
      if (o.slot_src[sl] < 0) continue;
      double d2 = 0.0;
      for (int i = 0; i < 3; ++i) d2 += ((double)o.slot[sl][i] - ctr[i]) * ((double)o.slot[sl][i] - ctr[i]);
      rho = std::max(rho, std::sqrt(d2));
    }
    for (int i = 0; i < 3; ++i) o.bnd[b][i] = ctr[i];
    o.bnd[b][3] = std::nextafter((float)(rho + rmax + 1e-4), 1e30f);
  }
  // Half-body bounding spheres (the first (C+1)/2 slots of the body, then the
  // rest): middle of the centres' box, largest centre offset plus radius.
  for (int b = 0; b < kBodies; ++b) {
    const int s0 = kLayoutStart[layout][b], cnt = kLayoutCount[layout][b], mid = s0 + (cnt + 1) / 2;
    for (int half = 0; half < 2; ++half) {
      const int a0 = half ? mid : s0, a1 = half ? s0 + cnt : mid;
      double lo[3] = {1e30, 1e30, 1e30}, hi[3] = {-1e30, -1e30, -1e30};
      int n = 0;
      for (int sl = a0; sl < a1; ++sl) {
        if (o.slot_src[sl] < 0) continue;
        ++n;
        for (int i = 0; i < 3; ++i) {
          lo[i] = std::min(lo[i], (double)o.slot[sl][i]);
          hi[i] = std::max(hi[i], (double)o.slot[sl][i]);
        }
      }
      float* hb = o.hb[b][half];
      if (n == 0) {
        hb[0] = hb[1] = hb[2] = 0.f;
        hb[3] = -1.f;
        continue;
      }
      for (int i = 0; i < 3; ++i) hb[i] = (float)(0.5 * (lo[i] + hi[i]));
      double rad = 0.0;
      for (int sl = a0; sl < a1; ++sl) {
        if (o.slot_src[sl] < 0) continue;
        double d2 = 0.0;
        for (int i = 0; i < 3; ++i) d2 += ((double)o.slot[sl][i] - hb[i]) * ((double)o.slot[sl][i] - hb[i]);
        rad = std::max(rad, std::sqrt(d2) + (double)o.slot[sl][3]);
      }
      hb[3] = std::nextafter((float)(rad + 1e-4), 1e30f);
    }
  }
  (void)c;
  return MPC_OK;
}

static int validate_arm(mpc_ctx* c, const mpc_arm_desc& d, int i, int counts[kBodies]) {
  char buf[160];
  auto bad = [&](const char* what) {
    snprintf(buf, sizeof(buf), "arm %d: %s", i, what);
    return fail(c, MPC_EINVAL, buf);
  };
  if (d.dof != 7) {
    snprintf(buf, sizeof(buf), "arm %d: dof %d not supported (this build runs 7-DoF chains)", i, d.dof);
    return fail(c, MPC_EUNSUPPORTED, buf);
  }
  if (d.n_spheres < 1 || d.n_spheres > MPC_MAX_SPHERES) return bad("n_spheres out of range");
  if (d.n_rollouts < 1 || d.n_rollouts > MPC_MAX_ROLLOUTS) return bad("n_rollouts out of range");
  if (d.horizon < 1 || d.horizon > MPC_MAX_HORIZON) return bad("horizon out of range");
  if (!d.dh || !d.q_lim || !d.qd_max || !d.spheres || !d.sphere_link) return bad("null table");
  if (!finite_all(d.dh, 28) || !finite_all(d.q_lim, 14) || !finite_all(d.qd_max, 7) ||
      !finite_all(d.spheres, 4 * d.n_spheres) || !finite_all(d.base, 4) || !finite_all(d.tool, 3))
    return bad("non-finite value");
  for (int k = 0; k < kBodies; ++k) counts[k] = 0;
  for (int s = 0; s < d.n_spheres; ++s) {
    const int b = d.sphere_link[s];
    if (b < 0 || b > 7) return bad("sphere_link outside 0..7");
    if (++counts[b] > MPC_MAX_SPHERES_PER_BODY) return bad("more than 8 spheres on one body");
    if (!(d.spheres[4 * s + 3] >= 0.f) || d.spheres[4 * s + 3] > 1.f) return bad("sphere radius outside [0, 1]");
    for (int k = 0; k < 3; ++k)
      if (std::fabs(d.spheres[4 * s + k]) > 1.5f) return bad("sphere centre more than 1.5 m from its link");
  }
  for (int k = 0; k < 7; ++k) {
    if (std::fabs(d.dh[4 * k]) > 1.5f || std::fabs(d.dh[4 * k + 2]) > 1.5f) return bad("link length above 1.5 m");
    if (!(d.q_lim[2 * k] <= d.q_lim[2 * k + 1])) return bad("joint limits reversed");
  }
  // The squared-gap filter is sized for world coordinates within 6 m of the
  // origin: the base within 3 m, every point of the chain within 2.6 m of its
  // base.  Each joint origin lies sqrt(a^2 + d^2) past the previous one, and a
  // sphere centre or the tool point lies at most its offset from its frame's
  // origin, so the sum of the link spacings, the tool offset and the largest
  // sphere offset bounds the reach.
  double reach = 0.0, off = 0.0;
  for (int k = 0; k < 7; ++k) reach += std::hypot((double)d.dh[4 * k], (double)d.dh[4 * k + 2]);
  for (int s = 0; s < d.n_spheres; ++s)
    off = std::max(off, std::sqrt((double)d.spheres[4 * s] * d.spheres[4 * s] +
                                  (double)d.spheres[4 * s + 1] * d.spheres[4 * s + 1] +
                                  (double)d.spheres[4 * s + 2] * d.spheres[4 * s + 2]));
  reach += off + std::sqrt((double)d.tool[0] * d.tool[0] + (double)d.tool[1] * d.tool[1] +
                           (double)d.tool[2] * d.tool[2]);
  if (reach > 2.6) return bad("chain reach (link spacings + tool + largest sphere offset) above 2.6 m");
  if (std::sqrt(d.base[0] * d.base[0] + d.base[1] * d.base[1] + d.base[2] * d.base[2]) > 3.f)
    return bad("base more than 3 m from the world origin");
  return MPC_OK;
}

extern "C" int mpc_init(const mpc_arm_desc* arms, int n_arms, const mpc_params* p, void* hip_stream,
                        mpc_ctx** out) {
  if (!out) return fail(nullptr, MPC_EINVAL, "out is NULL");
  *out = nullptr;
  if (!arms || !p) return fail(nullptr, MPC_EINVAL, "arms or params is NULL");
  if (n_arms < 1 || n_arms > MPC_MAX_ARMS) return fail(nullptr, MPC_EINVAL, "n_arms outside 1..8");
  // Host-side validation first (no device needed), then the device.
  const float pf[] = {p->dt, p->sigma, p->lambda, p->gamma, p->alpha_mu, p->w_pose, p->w_rot,
                      p->w_stop, p->w_joint, p->w_coll, p->w_dyn, p->buf_env, p->buf_self,
                      p->buf_dyn, p->tau, p->prio_min, p->prio_max, p->dist_floor, p->joint_margin};
  if (!finite_all(pf, (int)(sizeof(pf) / sizeof(float)))) return fail(nullptr, MPC_EINVAL, "non-finite parameter");
  if (!(p->lambda > 0.f) || !(p->dt > 0.f) || !(p->sigma >= 0.f) || !(p->alpha_mu >= 0.f && p->alpha_mu <= 1.f) ||
      !(p->buf_env > 0.f && p->buf_self > 0.f && p->buf_dyn > 0.f) || !(p->prio_min <= p->prio_max) ||
      !(p->dist_floor > 0.f))
    return fail(nullptr, MPC_EINVAL, "parameter out of range");
  if (p->iters < 1 || p->iters > 8) return fail(nullptr, MPC_EINVAL, "iters outside 1..8");
  if (p->max_obstacles < 0 || p->max_obstacles > MPC_MAX_OBSTACLES)
    return fail(nullptr, MPC_EINVAL, "max_obstacles outside 0..64");
  if (p->collision_mode != 0 && p->collision_mode != 1) return fail(nullptr, MPC_EINVAL, "collision_mode must be 0 or 1");
  if (!(p->alpha_sigma >= 0.f && p->alpha_sigma <= 1.f)) return fail(nullptr, MPC_EINVAL, "alpha_sigma outside [0, 1]");
  if (!(p->sigma_floor > 0.f && p->sigma_floor < 1e3f)) return fail(nullptr, MPC_EINVAL, "sigma_floor must be positive");
  if (p->plan_mode != 0 && p->plan_mode != 1) return fail(nullptr, MPC_EINVAL, "plan_mode must be 0 or 1");
  if (!(p->w_manip >= 0.f && p->w_manip < 1e30f) || !(p->manip_thresh > 0.f && p->manip_thresh < 1e30f))
    return fail(nullptr, MPC_EINVAL, "w_manip must be >= 0 and manip_thresh > 0");
  // The learned distance may drop a check only when its prediction is at
  // least the margin, so a margin below B would hide gaps the hinge sees.
  // 0 means "B itself"; checked here whatever the mode, since the mode can be
  // switched later.
  if (!(p->surrogate_margin == 0.f || p->surrogate_margin >= p->buf_dyn))
    return fail(nullptr, MPC_EINVAL, "surrogate_margin must be 0 (= buf_dyn) or at least buf_dyn");
  if (!(p->surrogate_screen >= 0.f && p->surrogate_screen < 10.f))
    return fail(nullptr, MPC_EINVAL, "surrogate_screen outside [0, 10) m");
  if (!(p->surrogate_probe == 0 || (p->surrogate_probe >= 2 && p->surrogate_probe <= 1000)))
    return fail(nullptr, MPC_EINVAL, "surrogate_probe must be 0 or in [2, 1000]");
  if (!(p->surrogate_min_drop >= 0.f && p->surrogate_min_drop < 1.f))
    return fail(nullptr, MPC_EINVAL, "surrogate_min_drop outside [0, 1)");
  if (p->pair_cull != 0 && p->pair_cull != 1) return fail(nullptr, MPC_EINVAL, "pair_cull must be 0 or 1");
  bool all52 = true;
  for (int i = 0; i < n_arms; ++i) {
    int counts[kBodies];
    const int rc = validate_arm(nullptr, arms[i], i, counts);
    if (rc != MPC_OK) return rc;
    for (int b = 0; b < kBodies; ++b) all52 = all52 && counts[b] == kLayoutCount[0][b];
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
    return fail(nullptr, MPC_EHIP, "no HIP device available");
  int dev = 0;
  (void)hipGetDevice(&dev);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return fail(nullptr, MPC_EHIP, "hipGetDeviceProperties failed");
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(nullptr, MPC_EHIP, std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950");

  void* na_scratch = nullptr;
  {
    const hipError_t e = scratch_address(dev, &na_scratch);
    if (e != hipSuccess)
      return fail(nullptr, MPC_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  }

  mpc_ctx* c = new mpc_ctx();
  c->A = n_arms;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->na_scratch = na_scratch;
  for (int i = 0; i < n_arms; ++i) {
    c->Hmax = std::max(c->Hmax, arms[i].horizon);
    c->Smax = std::max(c->Smax, arms[i].n_spheres);
    c->Nmax = std::max(c->Nmax, (arms[i].n_rollouts + kWave - 1) / kWave * kWave);
  }
  c->layout = all52 ? 0 : 1;
  c->harms.resize(n_arms);
  long long eps_off = 0;
  c->pair_cull = p->pair_cull;
  for (int i = 0; i < n_arms; ++i) {
    build_arm(c, arms[i], c->layout, c->harms[i]);
    if (!c->pair_cull) {
      // Every body and half-body bound reaches every group (1e18 m; squares
      // stay finite in FP32), so the kernels' cull keeps every sphere pair:
      // the all-pairs check.
      for (int b = 0; b < kBodies; ++b) {
        if (c->harms[i].bnd[b][3] >= 0.f) c->harms[i].bnd[b][3] = 1.0e18f;
        for (int half = 0; half < 2; ++half)
          if (c->harms[i].hb[b][half][3] >= 0.f) c->harms[i].hb[b][half][3] = 1.0e18f;
      }
    }
    c->harms[i].eps_off = eps_off;
    eps_off += (long long)arms[i].horizon * 7 * c->harms[i].Npad;
  }
  Params& P = c->P;
  P.dt = p->dt; P.sigma = p->sigma; P.lambda = p->lambda; P.gamma = p->gamma; P.alpha_mu = p->alpha_mu;
  P.w_pose = p->w_pose; P.w_rot = p->w_rot; P.w_stop = p->w_stop; P.w_joint = p->w_joint;
  P.w_coll = p->w_coll; P.w_dyn = p->w_dyn; P.buf_env = p->buf_env; P.buf_self = p->buf_self;
  P.buf_dyn = p->buf_dyn; P.tau = p->tau; P.prio_min = p->prio_min; P.prio_max = p->prio_max;
  P.dist_floor = p->dist_floor; P.joint_margin = p->joint_margin;
  P.alpha_sigma = p->alpha_sigma; P.sigma_floor = p->sigma_floor;
  P.plan_mode = p->plan_mode; P.cov = p->alpha_sigma > 0.f ? 1 : 0;
  P.w_manip = p->w_manip; P.manip_thresh = p->manip_thresh;
  P.seed_lo = (uint32_t)(p->seed & 0xffffffffull);
  P.seed_hi = (uint32_t)(p->seed >> 32);
  P.iters = p->iters; P.A = n_arms; P.dof = 7; P.Hmax = c->Hmax; P.Smax = c->Smax; P.Nmax = c->Nmax;
  P.max_obs = p->max_obstacles;
  for (int h = 0; h < kMaxH; ++h) P.gpow[h] = (float)std::pow((double)p->gamma, (double)h);

  int rc = MPC_OK;
  const size_t A = n_arms, H = c->Hmax, S = c->Smax, N = c->Nmax;
  if ((rc = dalloc(c, &c->d_arms, A)) || (rc = dalloc(c, &c->d_P, 1)) || (rc = dalloc(c, &c->d_ss, 1)) ||
      (rc = dalloc(c, &c->d_meta, 1)) || (rc = dalloc(c, &c->mu, A * H * 7)) ||
      (rc = dalloc(c, &c->eps, (size_t)eps_off)) || (rc = dalloc(c, &c->partial, A * kMaxH * N)) ||
      (rc = dalloc(c, &c->cost, A * N)) || (rc = dalloc(c, &c->w, A * N)) ||
      (rc = dalloc(c, &c->st_state, A * 21)) || (rc = dalloc(c, &c->st_goal, A * 7)) ||
      (rc = dalloc(c, &c->st_goalR, A * 9)) || (rc = dalloc(c, &c->st_obs, (size_t)kMaxObs * 4)) ||
      (rc = dalloc(c, &c->plan[0], A * H * S * 4)) || (rc = dalloc(c, &c->plan[1], A * H * S * 4)) ||
      (rc = dalloc(c, &c->planq[0], A * H * 7)) || (rc = dalloc(c, &c->planq[1], A * H * 7)) ||
      (rc = dalloc(c, &c->u_stage, A * 7)) || (rc = dalloc(c, &c->argmin, A)) ||
      (rc = dalloc(c, &c->sig, A * H * kTri)) || (rc = dalloc(c, &c->chol, A * H * kTri)) ||
      (rc = dalloc(c, &c->wpart, A * H * kWmeanMaxChunks * kWmeanSums)) ||
      (p->w_manip > 0.f && (rc = dalloc(c, &c->manip, A * H * N)))) {
    g_last_error = c->err;
    mpc_destroy(c);
    return rc;
  }
  // Sigma_h = sigma^2 I and its factor sigma I (set directly, not factorised,
  // so that without adaptation the noise is exactly sigma z).
  std::vector<float> sig0(A * H * kTri, 0.f), chol0(A * H * kTri, 0.f);
  for (size_t i = 0; i < A * H; ++i)
    for (int j = 0; j < 7; ++j) {
      sig0[i * kTri + tri7(j, j)] = p->sigma * p->sigma;
      chol0[i * kTri + tri7(j, j)] = p->sigma;
    }
  if (hipMemcpy(c->d_arms, c->harms.data(), A * sizeof(DevArm), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->d_P, &c->P, sizeof(Params), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->sig, sig0.data(), sig0.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->chol, chol0.data(), chol0.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
    fail(c, MPC_EHIP, "upload of arm tables failed");
    mpc_destroy(c);
    return MPC_EHIP;
  }
  // Learned-distance model state: joint normalisation of the (shared) arm
  // model, parameters and the per-step buffers.
  c->collision_mode = p->collision_mode;
  for (int j = 0; j < 7; ++j) {
    const double lo = arms[0].q_lim[2 * j], hi = arms[0].q_lim[2 * j + 1];
    c->hmodel.mid[j] = (float)(0.5 * (lo + hi));
    c->hmodel.inv_half[j] = (float)(hi > lo ? 2.0 / (hi - lo) : 1.0);
  }
  c->hmodel.margin = p->surrogate_margin > 0.f ? p->surrogate_margin : p->buf_dyn;
  c->hmodel.screen = p->surrogate_screen;
  c->hmodel.probe = p->surrogate_probe;
  c->hmodel.min_drop = p->surrogate_min_drop;
  if ((rc = dalloc(c, &c->d_model, 1)) || (rc = dalloc(c, &c->sur_p, (size_t)kMlpParams)) ||
      (rc = dalloc(c, &c->sur_m, (size_t)kMlpParams)) || (rc = dalloc(c, &c->sur_v, (size_t)kMlpParams)) ||
      (rc = dalloc(c, &c->sur_g, (size_t)kMlpParams)) || (rc = dalloc(c, &c->sur_p16, (size_t)kMlpParams)) ||
      (rc = dalloc(c, &c->sur_counts, kSurCounters * A))) {
    g_last_error = c->err;
    mpc_destroy(c);
    return rc;
  }
  if (hipMemcpy(c->d_model, &c->hmodel, sizeof(SurModel), hipMemcpyHostToDevice) != hipSuccess) {
    fail(c, MPC_EHIP, "upload of the distance model failed");
    mpc_destroy(c);
    return MPC_EHIP;
  }
  *out = c;
  return MPC_OK;
}

extern "C" void mpc_destroy(mpc_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  c->prof_roll.destroy();
  c->prof_infer.destroy();
  for (void* p : c->allocations) (void)hipFree(p);
  delete c;
}

extern "C" const char* mpc_last_error(const mpc_ctx* c) {
  return c ? c->err.c_str() : g_last_error.c_str();
}

extern "C" int mpc_sync(mpc_ctx* c) {
  if (!c) return MPC_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return MPC_OK;
}

// ---------------------------------------------------------------------------
// Work items of the rollout launch for a horizon tile T and W waves per
// workgroup: every arm's blocks of 64 W rollouts times its ceil(H/T) tiles,
// heaviest (longest tile) first.
static void build_items(const mpc_ctx* c, int T, int W, std::vector<Item>& items) {
  items.clear();
  for (int a = 0; a < c->A; ++a) {
    const DevArm& arm = c->harms[a];
    const int blocks = arm.Npad / (kWave * W);
    for (int h0 = 0; h0 < arm.H; h0 += T)
      for (int b = 0; b < blocks; ++b) items.push_back(Item{a, b, h0, std::min(arm.H, h0 + T)});
  }
  std::stable_sort(items.begin(), items.end(),
                   [](const Item& x, const Item& y) { return (x.h1 - x.h0) > (y.h1 - y.h0); });
}

// W waves per workgroup fit when every arm's padded rollout count is a
// multiple of 64 W (no wave of an item past an arm's rollouts).
static bool waves_fit(const mpc_ctx* c, int W) {
  if (W != 1 && W != 2 && W != 4) return false;
  for (const DevArm& arm : c->harms)
    if (arm.Npad % (kWave * W) != 0) return false;
  return true;
}

// Launch shapes the tuner chose, per problem shape and device, for the
// lifetime of the process: a context with the same shape on the same device
// starts from the cached choice instead of timing candidates again.
struct TuneChoice {
  int T, grid, waves;
};
static std::mutex g_tune_mu;
static std::map<std::vector<long long>, TuneChoice> g_tune_cache;

static std::vector<long long> tune_key(const mpc_ctx* c) {
  int dev = -1;
  (void)hipGetDevice(&dev);
  std::vector<long long> k = {dev, c->layout, c->collision_mode, c->sur_audit ? 1 : 0, c->P.cov,
                              c->manip ? 1 : 0, c->P.max_obs, c->A, c->pair_cull};
  for (const DevArm& arm : c->harms) {
    k.push_back(arm.N);
    k.push_back(arm.H);
    k.push_back(arm.S);
  }
  return k;
}

static RolloutArgs rollout_args(const mpc_ctx* c, int k) {
  RolloutArgs R{};
  R.arms = c->d_arms;
  R.P = c->d_P;
  R.ss = c->d_ss;
  R.items = c->d_items;
  R.n_items = c->n_items;
  R.k = k;
  R.mu = c->mu;
  R.eps = c->eps;
  R.partial = c->partial;
  R.state = c->st_state;
  R.goal = c->st_goal;
  R.goalR = c->st_goalR;
  R.obs = c->st_obs;
  R.plan_read = c->plan[0];
  R.dbg_q = c->dbg_q;
  R.dbg_qd = c->dbg_qd;
  R.dbg_sph = c->dbg_sph;
  R.dbg_stage = c->dbg_stage;
  R.dbg_pairs = c->dbg_pairs;
  R.learned = c->collision_mode == 1 ? 1 : 0;
  R.audit = c->sur_audit ? 1 : 0;
  R.sur_y = c->sur_y;
  R.sur_grp = c->sur_grp;
  R.sur_F = c->sur_F;
  R.sur_rec = c->sur_nbrec;
  R.sur_margin = c->hmodel.margin;
  R.sur_counts = c->sur_counts;
  R.sur_hist = c->sur_hist;
  R.dbg_pred = c->sur_pred;
  R.dbg_skip = c->sur_skip;
  R.manip = c->manip;
  return R;
}

static ReduceArgs reduce_args(const mpc_ctx* c) {
  ReduceArgs R{};
  R.arms = c->d_arms;
  R.P = c->d_P;
  R.ss = c->d_ss;
  R.partial = c->partial;
  R.cost = c->cost;
  R.w = c->w;
  R.eps = c->eps;
  R.mu = c->mu;
  R.u_out = c->u_stage;
  R.argmin = c->argmin;
  R.st_state = c->st_state;
  R.plan_write = c->plan[1];
  R.planq_write = c->planq[1];
  R.meta = c->d_meta;
  R.sig = c->sig;
  R.chol = c->chol;
  R.wpart = c->wpart;
  return R;
}

static int set_items(mpc_ctx* c, int T, int W) {
  std::vector<Item> items;
  build_items(c, T, W, items);
  if (items.size() > c->items_cap) {
    Item* p = nullptr;
    HIPCHK(c, hipMalloc(&p, items.size() * sizeof(Item)));
    c->allocations.push_back(p);
    c->d_items = p;
    c->items_cap = items.size();
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(c->d_items, items.data(), items.size() * sizeof(Item), hipMemcpyHostToDevice));
  c->n_items = (int)items.size();
  c->h_tile = T;
  c->waves = W;
  return MPC_OK;
}

static int enqueue_learned_prelude(mpc_ctx* c, int k, bool debug, unsigned long long* counts);

// Noise of iteration k: sigma z, or L_h z with the adapted covariance; in
// collision mode 1 the same launch screens the learned distance's groups.
static hipError_t enqueue_noise(mpc_ctx* c, int k) {
  const float* chol = c->P.cov ? c->chol : nullptr;
  if (c->collision_mode == 1)
    return launch_noise_screen(c->d_arms, c->d_P, c->d_ss, chol, c->eps, k, c->A, c->Hmax, c->Nmax, c->d_model,
                               c->d_meta, c->mu, c->st_state, c->plan[0], c->sur_screen, c->sur_hist, c->stream);
  return launch_noise(c->d_arms, c->d_P, c->d_ss, chol, c->eps, k, c->A, c->Hmax, c->Nmax, c->stream);
}

// Launch-shape tuner: times the rollout launch for every candidate number of
// waves per workgroup, horizon tile and grid size on the live inputs of the
// first representative step and keeps the fastest; the choice is cached per
// problem shape and device.  In collision mode 1 the candidates run on this
// step's skip decisions, and their counts go to a scratch row, not to the
// context's counters.
static int tune(mpc_ctx* c) {
  const std::vector<long long> key = tune_key(c);
  const bool forced = c->force_tile > 0 || c->force_grid > 0 || c->force_waves > 0;
  if (!forced) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto hit = g_tune_cache.find(key);
    if (hit != g_tune_cache.end()) {
      const TuneChoice ch = hit->second;
      int rc = set_items(c, ch.T, ch.waves);
      if (rc) return rc;
      c->grid = std::min(ch.grid, c->n_items);
      c->tuned = true;
      return MPC_OK;
    }
  }
  std::vector<int> waves;
  if (c->force_waves > 0) {
    waves.push_back(c->force_waves);
  } else {
    for (int W : {1, 2, 4})
      if (waves_fit(c, W)) waves.push_back(W);
  }
  std::vector<int> tiles;
  if (c->force_tile > 0) {
    tiles.push_back(std::min(c->force_tile, c->Hmax));
  } else {
    for (int T : {1, 2, 4, 5, 8, 10, 16, 20, 32, 64})
      if (T <= c->Hmax) tiles.push_back(T);
    if (std::find(tiles.begin(), tiles.end(), c->Hmax) == tiles.end()) tiles.push_back(c->Hmax);
  }
  if (c->collision_mode == 1 && !c->tune_counts) {
    int rc = dalloc(c, &c->tune_counts, (size_t)kSurCounters * c->A);
    if (rc) return rc;
  }
  HIPCHK(c, enqueue_noise(c, 0));
  if (c->collision_mode == 1) {
    int rc = enqueue_learned_prelude(c, 0, false, c->tune_counts);
    if (rc) return rc;
  }
  hipEvent_t e0, e1;
  HIPCHK(c, hipEventCreate(&e0));
  HIPCHK(c, hipEventCreate(&e1));
  float best_ms = 1e30f;
  int best_T = tiles[0], best_grid = 0, best_W = waves[0];
  for (int W : waves) {
    for (int T : tiles) {
      int rc = set_items(c, T, W);
      if (rc) return rc;
      std::vector<int> grids;
      if (c->force_grid > 0) {
        grids.push_back(std::min(c->force_grid, c->n_items));
      } else {
        grids.push_back(c->n_items);
        for (int g : {1024, 2048, 4096})
          if (g / W < c->n_items) grids.push_back(g / W);
      }
      for (int g : grids) {
        RolloutArgs R = rollout_args(c, 0);
        if (R.sur_counts) R.sur_counts = c->tune_counts;
        R.sur_hist = nullptr;  // replays leave the drop history alone
        HIPCHK(c, launch_rollout(R, c->layout, false, W, g, c->stream));
        HIPCHK(c, hipEventRecord(e0, c->stream));
        for (int r = 0; r < 3; ++r) HIPCHK(c, launch_rollout(R, c->layout, false, W, g, c->stream));
        HIPCHK(c, hipEventRecord(e1, c->stream));
        HIPCHK(c, hipEventSynchronize(e1));
        float ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
        if (ms < best_ms) {
          best_ms = ms;
          best_T = T;
          best_grid = g;
          best_W = W;
        }
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  int rc = set_items(c, best_T, best_W);
  if (rc) return rc;
  c->grid = best_grid;
  c->tuned = true;
  if (!forced) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = TuneChoice{best_T, best_grid, best_W};
  }
  return MPC_OK;
}

// Learned distance before each rollout launch of iteration k (after the
// noise launch, which also screened the groups): own-joint features of every
// rollout step, the neighbour records and the inference descriptors (one
// launch), then the network's prediction of every query that needs one;
// the rollout kernel takes the skip decisions from the predictions and
// counts the queries.  In a debug step the capture buffers start cleared.
static int enqueue_learned_prelude(mpc_ctx* c, int k, bool debug, unsigned long long* counts) {
  (void)k;
  if (debug) {
    const size_t n = (size_t)c->A * c->A * c->Hmax * c->Nmax;
    HIPCHK(c, hipMemsetAsync(c->sur_skip, 0, n, c->stream));
    HIPCHK(c, hipMemsetAsync(c->sur_pred, 0, n * sizeof(float), c->stream));
  }
  HIPCHK(c, launch_sur_states(c->d_arms, c->d_P, c->d_model, c->mu, c->st_state, c->eps, c->A, c->Nmax, c->Hmax,
                              c->sur_F, c->d_meta, c->planq[0], c->sur_nbrec, c->sur_screen, c->d_sur_items,
                              c->sur_grp, c->sur_count, counts, c->stream));
  SurInferArgs I{};
  I.P = c->d_P;
  I.model = c->d_model;
  I.W16 = c->sur_p16;
  I.P32 = c->sur_p;
  I.F = c->sur_F;
  I.nbrec = c->sur_nbrec;
  I.items = c->d_sur_items;
  I.count = c->sur_count;
  I.y = c->sur_y;
  hipEvent_t ei = nullptr;
  if (c->profile) HIPCHK(c, c->prof_infer.begin(c->stream, &ei));
  HIPCHK(c, launch_sur_infer(I, c->sur_grid, c->stream));
  if (ei) HIPCHK(c, hipEventRecord(ei, c->stream));
  return MPC_OK;
}

// The per-step device work after Sense: K x {rollout, softmax/act, weighted
// mean + update}, then ToPlan.
static int enqueue_body(mpc_ctx* c, bool debug) {
  ReduceArgs Rr = reduce_args(c);
  for (int k = 0; k < c->P.iters; ++k) {
    RolloutArgs R = rollout_args(c, k);
    HIPCHK(c, enqueue_noise(c, k));
    if (c->manip)
      HIPCHK(c, launch_manip(c->d_arms, c->d_P, c->d_ss, c->mu, c->st_state, c->eps, c->A, c->Nmax, c->manip,
                             c->stream));
    if (c->collision_mode == 1) {
      int rc = enqueue_learned_prelude(c, k, debug, c->sur_counts);
      if (rc) return rc;
    }
    hipEvent_t e1 = nullptr;
    if (c->profile) HIPCHK(c, c->prof_roll.begin(c->stream, &e1));
    HIPCHK(c, launch_rollout(R, c->layout, debug, c->waves, c->grid, c->stream));
    if (e1) HIPCHK(c, hipEventRecord(e1, c->stream));
    HIPCHK(c, launch_softmax(Rr, c->A, c->Nmax, c->Hmax, c->stream));
    // Between iterations the totals and Eq. 4 run on their own; after the
    // last one ToPlan applies them first.
    HIPCHK(c, launch_wmean(Rr, c->A, c->Hmax, c->Nmax, k + 1 < c->P.iters, c->stream));
  }
  HIPCHK(c, launch_toplan(Rr, c->A, true, c->stream));
  return MPC_OK;
}

// Per-step buffers of the learned distance and its work items: every
// (arm, neighbour, step within both horizons, 32-rollout block).
static int ensure_sur_buffers(mpc_ctx* c) {
  if (c->sur_bufs) return MPC_OK;
  // A call that failed part-way leaves its buffers to mpc_destroy and starts over.
  const size_t A = c->A, H = c->Hmax, N = c->Nmax;
  int rc;
  if ((rc = dalloc(c, &c->sur_F, A * H * N * 8)) || (rc = dalloc(c, &c->sur_skip, A * A * H * N)) ||
      (rc = dalloc(c, &c->sur_pred, A * A * H * N)) || (rc = dalloc(c, &c->sur_nbrec, A * A * H * kNbrRec)) ||
      (rc = dalloc(c, &c->sur_screen, A * A * H)) || (rc = dalloc(c, &c->sur_grp, A * A * H)) ||
      (rc = dalloc(c, &c->sur_count, 1)) || (rc = dalloc(c, &c->sur_hist, 2 * A * A * H)))
    return rc;
  c->hist_stale = true;
  // Room for the descriptors of every (arm, neighbour, step within both
  // horizons, 32-rollout block), the step's are written by k_sur_states.
  long long n_items = 0;
  for (int a = 0; a < c->A; ++a)
    for (int i = 0; i < c->A; ++i)
      if (i != a) n_items += (long long)std::min(c->harms[a].H, c->harms[i].H) * (c->harms[a].Npad / 32);
  c->n_sur_items = (int)n_items;
  if (n_items > 0 &&
      ((rc = dalloc(c, &c->d_sur_items, (size_t)n_items)) || (rc = dalloc(c, &c->sur_y, (size_t)n_items * 32))))
    return rc;
  // One inference block per compute unit (its LDS and registers fill one).
  int dev = 0, n_cu = 0;
  HIPCHK(c, hipGetDevice(&dev));
  HIPCHK(c, hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
  c->sur_grid = std::max(1, std::min(c->n_sur_items, std::max(n_cu, 1)));
  c->sur_bufs = true;
  return MPC_OK;
}

static int capture_graph(mpc_ctx* c) {
  if (c->gexec) {
    (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
  }
  if (c->stream == nullptr) return MPC_OK;  // the null stream cannot be captured
  hipGraph_t g = nullptr;
  HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  int rc = enqueue_body(c, false);
  hipError_t e = hipStreamEndCapture(c->stream, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(c, MPC_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(c, MPC_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  return MPC_OK;
}

extern "C" int mpc_step(mpc_ctx* c, const float* state, const float* goal, const float* obstacles,
                        int n_obstacles, float* u_out) {
  if (!c) return MPC_EINVAL;
  if (!state || !goal || !u_out) return fail(c, MPC_EINVAL, "state, goal and u_out must be device pointers");
  if (n_obstacles < 0 || n_obstacles > c->P.max_obs)
    return fail(c, MPC_EINVAL, "n_obstacles outside [0, max_obstacles]");
  if (n_obstacles > 0 && !obstacles) return fail(c, MPC_EINVAL, "obstacles is NULL");
  if (c->collision_mode == 1) {
    if (!c->sur_ready) return fail(c, MPC_ESTATE, "collision mode 1 needs trained or set distance-model parameters");
    const int rc0 = ensure_sur_buffers(c);
    if (rc0) return rc0;
    if (c->hist_stale) {
      // No drop history yet: every group runs the network on its next step
      // (outside the captured step body).
      const std::vector<unsigned> none((size_t)2 * c->A * c->A * c->Hmax, kHistNone);
      HIPCHK(c, hipMemcpyAsync(c->sur_hist, none.data(), none.size() * sizeof(unsigned), hipMemcpyHostToDevice,
                               c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
      c->hist_stale = false;
    }
  }
  SenseArgs S{};
  S.arms = c->d_arms;
  S.P = c->d_P;
  S.ss = c->d_ss;
  S.meta = c->d_meta;
  S.state = state;
  S.goal = goal;
  S.obstacles = obstacles;
  S.n_obs = n_obstacles;
  S.t = c->t;
  S.u_out = u_out;
  S.st_state = c->st_state;
  S.st_goal = c->st_goal;
  S.st_obs = c->st_obs;
  S.goalR = c->st_goalR;
  S.mu = c->mu;
  S.sig = c->sig;
  S.chol = c->chol;
  HIPCHK(c, launch_sense(S, c->stream));
  int rc;
  if (!c->tuned) {
    // Tune on a representative step: once every arm's plan is visible to the
    // others (or after a few steps if the caller never publishes them all).
    const bool representative = c->A == 1 || c->n_published == c->A || c->untuned_steps >= 3;
    if (representative) {
      if ((rc = tune(c))) return rc;
      if ((rc = capture_graph(c))) return rc;
    } else {
      if (c->n_items == 0) {
        const int T = c->force_tile > 0 ? std::min(c->force_tile, c->Hmax) : std::min(4, c->Hmax);
        if ((rc = set_items(c, T, c->force_waves > 0 ? c->force_waves : 1))) return rc;
      }
      c->grid = c->force_grid > 0 ? std::min(c->force_grid, c->n_items) : c->n_items;
      ++c->untuned_steps;
    }
  }
  if (c->debug) {
    HIPCHK(c, hipMemsetAsync(c->dbg_pairs, 0, sizeof(unsigned long long) * 4 * c->A, c->stream));
    if ((rc = enqueue_body(c, true))) return rc;
  } else if (c->gexec && !c->profile) {
    HIPCHK(c, hipGraphLaunch(c->gexec, c->stream));
  } else {
    if ((rc = enqueue_body(c, false))) return rc;
  }
  c->t += 1;
  c->stepped = true;
  return MPC_OK;
}

extern "C" int mpc_share_plans(mpc_ctx* c, const unsigned char* mask) {
  if (!c) return MPC_EINVAL;
  PublishArgs P{};
  P.plan_write = c->plan[1];
  P.planq_write = c->planq[1];
  P.plan_read = c->plan[0];
  P.planq_read = c->planq[0];
  P.meta = c->d_meta;
  P.Hmax = c->Hmax;
  P.Smax = c->Smax;
  uint32_t m = 0;
  if (c->published.empty()) c->published.assign(c->A, 0);
  for (int a = 0; a < c->A; ++a)
    if (!mask || mask[a]) {
      m |= 1u << a;
      if (c->stepped && !c->published[a]) {
        c->published[a] = 1;
        ++c->n_published;
      }
    }
  P.mask = m;
  HIPCHK(c, launch_publish(P, c->A, c->stream));
  return MPC_OK;
}

extern "C" int mpc_get_plan(mpc_ctx* c, int arm, float* plan, float* plan_q, float* mean) {
  if (!c) return MPC_EINVAL;
  if (arm < 0 || arm >= c->A) return fail(c, MPC_EINVAL, "arm out of range");
  if (!c->stepped) return fail(c, MPC_ESTATE, "no plan before the first mpc_step");
  const DevArm& d = c->harms[arm];
  const long long H = c->Hmax, S = c->Smax;
  if (plan) {
    const float* src = c->plan[1] + (size_t)arm * H * S * 4;
    // src [h][s][c] -> dst [s][c][h]
    HIPCHK(c, launch_copy3d(src, 4, 1, S * 4, plan, 4LL * d.H, d.H, 1, d.S, 4, d.H, c->stream));
  }
  if (plan_q)
    HIPCHK(c, hipMemcpyAsync(plan_q, c->planq[1] + (size_t)arm * H * 7, sizeof(float) * d.H * 7,
                             hipMemcpyDeviceToDevice, c->stream));
  if (mean)
    HIPCHK(c, hipMemcpyAsync(mean, c->mu + (size_t)arm * H * 7, sizeof(float) * d.H * 7,
                             hipMemcpyDeviceToDevice, c->stream));
  return MPC_OK;
}

// ---------------------------------------------------------------------------
extern "C" int mpc_debug_enable(mpc_ctx* c, int on) {
  if (!c) return MPC_EINVAL;
  if (on && !c->dbg_pairs) {  // allocated last: set only when every capture buffer is
    const size_t A = c->A, N = c->Nmax, H = c->Hmax, S = c->Smax;
    int rc;
    if ((rc = dalloc(c, &c->dbg_q, A * N * H * 7)) || (rc = dalloc(c, &c->dbg_qd, A * N * H * 7)) ||
        (rc = dalloc(c, &c->dbg_sph, A * N * H * S * 4)) || (rc = dalloc(c, &c->dbg_stage, A * H * N)) ||
        (rc = dalloc(c, &c->dbg_pairs, 4 * A)))
      return rc;
  }
  c->debug = on != 0;
  return MPC_OK;
}

extern "C" int mpc_debug_get(mpc_ctx* c, int what, int arm, void* dev_out) {
  if (!c) return MPC_EINVAL;
  if (arm < 0 || arm >= c->A || !dev_out) return fail(c, MPC_EINVAL, "bad arm or output");
  const DevArm& d = c->harms[arm];
  const long long N = c->Nmax, H = c->Hmax, S = c->Smax;
  float* out = static_cast<float*>(dev_out);
  const bool needs_dbg = what == MPC_DBG_Q || what == MPC_DBG_QD || what == MPC_DBG_SPHERES ||
                         what == MPC_DBG_STAGE_COST || what == MPC_DBG_PAIRS || what == MPC_DBG_PASSES;
  if (needs_dbg && !c->dbg_pairs) return fail(c, MPC_ESTATE, "debug capture is off");
  switch (what) {
    case MPC_DBG_NOISE:
      HIPCHK(c, launch_copy3d(c->eps + d.eps_off, d.Npad, 1, 0, out, d.N, 1, 0, d.H * 7, d.N, 1, c->stream));
      break;
    case MPC_DBG_Q:
    case MPC_DBG_QD: {
      const float* src = (what == MPC_DBG_Q ? c->dbg_q : c->dbg_qd) + (size_t)arm * N * H * 7;
      HIPCHK(c, launch_copy3d(src, H * 7, 1, 0, out, d.H * 7LL, 1, 0, d.N, d.H * 7, 1, c->stream));
      break;
    }
    case MPC_DBG_SPHERES: {
      const float* src = c->dbg_sph + (size_t)arm * N * H * S * 4;
      HIPCHK(c, launch_copy3d(src, H * S * 4, S * 4, 1, out, (long long)d.H * d.S * 4, d.S * 4LL, 1, d.N, d.H,
                              d.S * 4, c->stream));
      break;
    }
    case MPC_DBG_STAGE_COST:
      HIPCHK(c, launch_copy3d(c->dbg_stage + (size_t)arm * H * N, N, 1, 0, out, d.N, 1, 0, d.H, d.N, 1, c->stream));
      break;
    case MPC_DBG_COST:
      HIPCHK(c, hipMemcpyAsync(out, c->cost + (size_t)arm * N, sizeof(float) * d.N, hipMemcpyDeviceToDevice, c->stream));
      break;
    case MPC_DBG_WEIGHTS:
      HIPCHK(c, hipMemcpyAsync(out, c->w + (size_t)arm * N, sizeof(float) * d.N, hipMemcpyDeviceToDevice, c->stream));
      break;
    case MPC_DBG_MEAN:
      HIPCHK(c, hipMemcpyAsync(out, c->mu + (size_t)arm * H * 7, sizeof(float) * d.H * 7, hipMemcpyDeviceToDevice, c->stream));
      break;
    case MPC_DBG_ALPHA:
      HIPCHK(c, hipMemcpyAsync(out, &c->d_ss->alpha[arm][0], sizeof(float) * c->A, hipMemcpyDeviceToDevice, c->stream));
      break;
    case MPC_DBG_DIST:
      HIPCHK(c, hipMemcpyAsync(out, &c->d_ss->dist_now[arm], sizeof(float), hipMemcpyDeviceToDevice, c->stream));
      break;
    case MPC_DBG_PAIRS:
      HIPCHK(c, hipMemcpyAsync(out, c->dbg_pairs + 4 * arm, sizeof(unsigned long long), hipMemcpyDeviceToDevice, c->stream));
      break;
    case MPC_DBG_PRED:
      if (!c->sur_pred) return fail(c, MPC_ESTATE, "no learned-distance step has run");
      HIPCHK(c, launch_copy3d(c->sur_pred + (size_t)arm * c->A * H * N, H * N, N, 1, out, (long long)d.H * d.N, d.N,
                              1, c->A, d.H, d.N, c->stream));
      break;
    case MPC_DBG_PASSES:
      HIPCHK(c, hipMemcpyAsync(out, c->dbg_pairs + 4 * arm + 1, 3 * sizeof(unsigned long long),
                               hipMemcpyDeviceToDevice, c->stream));
      break;
    case MPC_DBG_ARGMIN:
      HIPCHK(c, hipMemcpyAsync(out, c->argmin + arm, sizeof(int), hipMemcpyDeviceToDevice, c->stream));
      break;
    case MPC_DBG_SKIP:
      if (!c->sur_skip) return fail(c, MPC_ESTATE, "no learned-distance step has run");
      for (int i = 0; i < c->A; ++i)
        HIPCHK(c, hipMemcpy2DAsync(static_cast<uint8_t*>(dev_out) + (size_t)i * d.H * d.N, d.N,
                                   c->sur_skip + ((size_t)arm * c->A + i) * H * N, N, d.N, d.H,
                                   hipMemcpyDeviceToDevice, c->stream));
      break;
    case MPC_DBG_SIGMA:
    case MPC_DBG_CHOL:
      HIPCHK(c, hipMemcpyAsync(out, (what == MPC_DBG_SIGMA ? c->sig : c->chol) + (size_t)arm * H * kTri,
                               sizeof(float) * d.H * kTri, hipMemcpyDeviceToDevice, c->stream));
      break;
    default:
      return fail(c, MPC_EINVAL, "unknown debug quantity");
  }
  return MPC_OK;
}

extern "C" int mpc_get_board(mpc_ctx* c, int arm, float* plan, float* plan_q, float* dist, int* valid) {
  if (!c) return MPC_EINVAL;
  if (arm < 0 || arm >= c->A) return fail(c, MPC_EINVAL, "arm out of range");
  const DevArm& d = c->harms[arm];
  const long long H = c->Hmax, S = c->Smax;
  if (plan)
    HIPCHK(c, launch_copy3d(c->plan[0] + (size_t)arm * H * S * 4, S * 4, 1, 0, plan, d.S * 4LL, 1, 0, d.H, d.S * 4, 1,
                            c->stream));
  if (plan_q)
    HIPCHK(c, hipMemcpyAsync(plan_q, c->planq[0] + (size_t)arm * H * 7, sizeof(float) * d.H * 7,
                             hipMemcpyDeviceToDevice, c->stream));
  if (dist || valid) {
    BoardMeta m;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(&m, c->d_meta, sizeof(m), hipMemcpyDeviceToHost));
    if (dist) *dist = m.dist[0][arm];
    if (valid) *valid = m.valid[0][arm];
  }
  return MPC_OK;
}

extern "C" int mpc_set_board(mpc_ctx* c, int arm, const float* plan, const float* plan_q, float dist, int valid) {
  if (!c) return MPC_EINVAL;
  if (arm < 0 || arm >= c->A) return fail(c, MPC_EINVAL, "arm out of range");
  if (!std::isfinite(dist)) return fail(c, MPC_EINVAL, "non-finite distance");
  const DevArm& d = c->harms[arm];
  const long long H = c->Hmax, S = c->Smax;
  if (plan)
    HIPCHK(c, launch_copy3d(plan, d.S * 4LL, 1, 0, c->plan[0] + (size_t)arm * H * S * 4, S * 4, 1, 0, d.H, d.S * 4, 1,
                            c->stream));
  if (plan_q)
    HIPCHK(c, hipMemcpyAsync(c->planq[0] + (size_t)arm * H * 7, plan_q, sizeof(float) * d.H * 7,
                             hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, launch_set_meta(c->d_meta, arm, dist, valid ? 1 : 0, c->stream));
  return MPC_OK;
}

extern "C" int mpc_set_mean(mpc_ctx* c, int arm, const float* mean) {
  if (!c) return MPC_EINVAL;
  if (arm < 0 || arm >= c->A || !mean) return fail(c, MPC_EINVAL, "bad arm or mean");
  HIPCHK(c, hipMemcpyAsync(c->mu + (size_t)arm * c->Hmax * 7, mean, sizeof(float) * c->harms[arm].H * 7,
                           hipMemcpyDeviceToDevice, c->stream));
  return MPC_OK;
}

extern "C" int mpc_get_step(const mpc_ctx* c, unsigned int* t) {
  if (!c || !t) return MPC_EINVAL;
  *t = c->t;
  return MPC_OK;
}

extern "C" int mpc_set_step(mpc_ctx* c, unsigned int t) {
  if (!c) return MPC_EINVAL;
  c->t = t;
  return MPC_OK;
}

extern "C" int mpc_sim_execute(mpc_ctx* c, float* state, const float* u) {
  if (!c) return MPC_EINVAL;
  if (!state || !u) return fail(c, MPC_EINVAL, "null state or command");
  HIPCHK(c, launch_sim_execute(state, u, c->A * 7, c->P.dt, c->stream));
  return MPC_OK;
}

extern "C" int mpc_get_tuning(const mpc_ctx* c, int* rollouts_per_block, int* h_tile, int* grid) {
  if (!c) return MPC_EINVAL;
  if (rollouts_per_block) *rollouts_per_block = kWave * c->waves;
  if (h_tile) *h_tile = c->h_tile;
  if (grid) *grid = c->grid;
  return c->n_items > 0 ? MPC_OK : MPC_ESTATE;
}

extern "C" int mpc_set_tuning(mpc_ctx* c, int rollouts_per_block, int h_tile, int grid) {
  if (!c) return MPC_EINVAL;
  if (rollouts_per_block != 0 && rollouts_per_block != kWave && rollouts_per_block != 2 * kWave &&
      rollouts_per_block != 4 * kWave)
    return fail(c, MPC_EUNSUPPORTED, "rollouts per block must be 64, 128 or 256 (0 = tuned)");
  if (rollouts_per_block != 0 && !waves_fit(c, rollouts_per_block / kWave))
    return fail(c, MPC_EINVAL, "every arm's rollout count, padded to 64, must be a multiple of rollouts_per_block");
  if (h_tile < 0 || grid < 0) return fail(c, MPC_EINVAL, "negative tuning value");
  c->force_tile = h_tile;
  c->force_grid = grid;
  c->force_waves = rollouts_per_block / kWave;
  c->tuned = false;
  c->n_items = 0;
  return MPC_OK;
}

extern "C" int mpc_profile_enable(mpc_ctx* c, int on) {
  if (!c) return MPC_EINVAL;
  c->profile = on != 0;
  return MPC_OK;
}

extern "C" int mpc_profile_read(mpc_ctx* c, double* total_ms, int* launches) {
  if (!c || !total_ms || !launches) return MPC_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, c->prof_roll.read(total_ms, launches));
  return MPC_OK;
}

extern "C" int mpc_profile_read_surrogate(mpc_ctx* c, double* total_ms, int* launches) {
  if (!c || !total_ms || !launches) return MPC_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, c->prof_infer.read(total_ms, launches));
  return MPC_OK;
}

extern "C" int mpc_philox(const unsigned int* ctr, const unsigned int* key, unsigned int* out, int n,
                          void* hip_stream) {
  if (n < 0 || (n > 0 && (!ctr || !key || !out))) return fail(nullptr, MPC_EINVAL, "bad philox arguments");
  hipError_t e = launch_philox(ctr, key, out, n, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return fail(nullptr, MPC_EHIP, hipGetErrorString(e));
  return MPC_OK;
}

// ---------------------------------------------------------------------------
// Learned arm-pair distance: exact distance, features, training, parameters.

static int check_shared_model(mpc_ctx* c) {
  for (int a = 0; a < c->A; ++a) {
    const DevArm& x = c->harms[a];
    const DevArm& y = c->harms[0];
    if (x.a[0] != 0.f || x.sal[0] != 0.f)
      return fail(c, MPC_EUNSUPPORTED, "the learned distance needs a first joint about the base z axis");
    if (memcmp(x.a, y.a, sizeof(x.a)) || memcmp(x.cal, y.cal, sizeof(x.cal)) || memcmp(x.sal, y.sal, sizeof(x.sal)) ||
        memcmp(x.d, y.d, sizeof(x.d)) || memcmp(x.off, y.off, sizeof(x.off)) ||
        memcmp(x.slot, y.slot, sizeof(x.slot)) || memcmp(x.qlo, y.qlo, sizeof(x.qlo)) ||
        memcmp(x.qhi, y.qhi, sizeof(x.qhi)))
      return fail(c, MPC_EUNSUPPORTED, "the learned distance needs every arm to be the same model");
  }
  return MPC_OK;
}

extern "C" int mpc_pair_distance(mpc_ctx* c, int arm_i, int arm_j, const float* q_i, const float* q_j, int m,
                                 float* rho) {
  if (!c) return MPC_EINVAL;
  if (arm_i < 0 || arm_i >= c->A || arm_j < 0 || arm_j >= c->A || m < 0 || (m > 0 && (!q_i || !q_j || !rho)))
    return fail(c, MPC_EINVAL, "bad pair-distance arguments");
  HIPCHK(c, launch_pair_distance(c->layout, c->d_arms, arm_i, arm_j, q_i, q_j, m, rho, c->stream));
  return MPC_OK;
}

extern "C" int mpc_pair_features(mpc_ctx* c, int arm_i, int arm_j, const float* q_i, const float* q_j, int m,
                                 float* features) {
  if (!c) return MPC_EINVAL;
  if (arm_i < 0 || arm_i >= c->A || arm_j < 0 || arm_j >= c->A || m < 0 || (m > 0 && (!q_i || !q_j || !features)))
    return fail(c, MPC_EINVAL, "bad feature arguments");
  HIPCHK(c, launch_features(c->d_arms, c->d_model, arm_i, arm_j, q_i, q_j, m, features, c->stream));
  return MPC_OK;
}

// Scratch of one forward + backward pass over a batch of B samples.
struct MlpScratch {
  size_t B = 0;
  float *Z[3] = {nullptr, nullptr, nullptr}, *y = nullptr, *dy = nullptr, *dZ = nullptr, *loss = nullptr;
  uint16_t *A16[3] = {nullptr, nullptr, nullptr}, *dy16 = nullptr, *dZ16 = nullptr, *X16 = nullptr;
  std::vector<void*> mem;
  ~MlpScratch() {
    for (void* p : mem) (void)hipFree(p);
  }
  template <class T>
  hipError_t get(T** p, size_t n) {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, (n ? n : 1) * sizeof(T));
    if (e == hipSuccess) {
      mem.push_back(q);
      *p = static_cast<T*>(q);
    }
    return e;
  }
  hipError_t alloc(size_t b) {
    B = b;
    hipError_t e = hipSuccess;
    for (int l = 0; l < 3 && e == hipSuccess; ++l) {
      e = get(&Z[l], B * kHid);
      if (e == hipSuccess) e = get(&A16[l], B * kHid);
    }
    if (e == hipSuccess) e = get(&y, B);
    if (e == hipSuccess) e = get(&dy, B);
    if (e == hipSuccess) e = get(&dy16, B);
    if (e == hipSuccess) e = get(&dZ, B * kHid);
    if (e == hipSuccess) e = get(&dZ16, B * kHid);
    if (e == hipSuccess) e = get(&loss, 1);
    if (e == hipSuccess) e = get(&X16, B * kFeat);
    return e;
  }
};

static GemmArgs gemm(int M, int N, int K, const uint16_t* A, int lda, int ta, const uint16_t* B, int ldb, int tb) {
  GemmArgs g{};
  g.M = M; g.N = N; g.K = K;
  g.A = A; g.lda = lda; g.transA = ta;
  g.B = B; g.ldb = ldb; g.transB = tb;
  return g;
}

// Forward pass of B samples (X16 [B][17]) with the bfloat16 parameters:
// Z_l = bf(A_{l-1}) bf(W_l)^T + b_l, A_l = bf(relu(Z_l)), y = Z_4.
static hipError_t mlp_forward(mpc_ctx* c, MlpScratch& S, const uint16_t* X16, int B) {
  const uint16_t* in = X16;
  int K = kFeat;
  for (int l = 0; l < 3; ++l) {
    GemmArgs g = gemm(B, kHid, K, in, K, 0, c->sur_p16 + mlp_w_off(l), K, 1);
    g.bias = c->sur_p + mlp_b_off(l);
    g.C32 = S.Z[l]; g.ldc = kHid;
    g.C16 = S.A16[l]; g.ldc16 = kHid; g.relu = 1;
    hipError_t e = launch_gemm_bf16(g, c->stream);
    if (e != hipSuccess) return e;
    in = S.A16[l];
    K = kHid;
  }
  GemmArgs g = gemm(B, 1, kHid, in, kHid, 0, c->sur_p16 + mlp_w_off(3), kHid, 1);
  g.bias = c->sur_p + mlp_b_off(3);
  g.C32 = S.y; g.ldc = 1;
  return launch_gemm_bf16(g, c->stream);
}

// Backward pass into c->sur_g (after mlp_forward and the loss):
// dW_l = bf(dZ_l)^T bf(A_{l-1}), db_l = sum dZ_l, dZ_{l-1} = (bf(dZ_l) bf(W_l)) * [Z_{l-1} > 0].
static hipError_t mlp_backward(mpc_ctx* c, MlpScratch& S, const uint16_t* X16, int B) {
  hipError_t e;
  // output layer
  GemmArgs g = gemm(1, kHid, B, S.dy16, 1, 1, S.A16[2], kHid, 0);
  g.C32 = c->sur_g + mlp_w_off(3); g.ldc = kHid;
  if ((e = launch_gemm_bf16(g, c->stream)) != hipSuccess) return e;
  if ((e = launch_colsum(S.dy, B, 1, c->sur_g + mlp_b_off(3), c->stream)) != hipSuccess) return e;
  g = gemm(B, kHid, 1, S.dy16, 1, 0, c->sur_p16 + mlp_w_off(3), kHid, 0);
  g.mask = S.Z[2]; g.ldm = kHid;
  g.C32 = S.dZ; g.ldc = kHid; g.C16 = S.dZ16; g.ldc16 = kHid;
  if ((e = launch_gemm_bf16(g, c->stream)) != hipSuccess) return e;
  for (int l = 2; l >= 0; --l) {
    const uint16_t* in = l > 0 ? S.A16[l - 1] : X16;
    const int K = l > 0 ? kHid : kFeat;
    g = gemm(kHid, K, B, S.dZ16, kHid, 1, in, K, 0);
    g.C32 = c->sur_g + mlp_w_off(l); g.ldc = K;
    if ((e = launch_gemm_bf16(g, c->stream)) != hipSuccess) return e;
    if ((e = launch_colsum(S.dZ, B, kHid, c->sur_g + mlp_b_off(l), c->stream)) != hipSuccess) return e;
    if (l > 0) {
      // dZ16 is read by this product and rewritten by it: stage through dZ first.
      g = gemm(B, kHid, kHid, S.dZ16, kHid, 0, c->sur_p16 + mlp_w_off(l), kHid, 0);
      g.mask = S.Z[l - 1]; g.ldm = kHid;
      g.C32 = S.dZ; g.ldc = kHid;
      if ((e = launch_gemm_bf16(g, c->stream)) != hipSuccess) return e;
      if ((e = launch_f32_to_bf16(S.dZ, S.dZ16, (long long)B * kHid, c->stream)) != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

extern "C" int mpc_surrogate_grad(mpc_ctx* c, const float* features, const float* targets, int B, float over_w,
                                  float near_w, float near_band, float* grad, float* loss) {
  if (!c) return MPC_EINVAL;
  if (B < 1 || !features || !targets || !grad) return fail(c, MPC_EINVAL, "bad gradient arguments");
  MlpScratch S;
  HIPCHK(c, S.alloc((size_t)B));
  HIPCHK(c, launch_f32_to_bf16(features, S.X16, (long long)B * kFeat, c->stream));
  HIPCHK(c, hipMemsetAsync(S.loss, 0, sizeof(float), c->stream));
  HIPCHK(c, launch_params_to_bf16(c->sur_p, c->sur_p16, kMlpParams, c->stream));
  HIPCHK(c, mlp_forward(c, S, S.X16, B));
  HIPCHK(c, launch_loss(S.y, targets, B, over_w, near_w, near_band, S.dy, S.dy16, S.loss, c->stream));
  HIPCHK(c, mlp_backward(c, S, S.X16, B));
  HIPCHK(c, hipMemcpyAsync(grad, c->sur_g, sizeof(float) * kMlpParams, hipMemcpyDeviceToDevice, c->stream));
  float l = 0.f;
  HIPCHK(c, hipMemcpyAsync(&l, S.loss, sizeof(float), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (loss) *loss = l;
  return MPC_OK;
}

extern "C" int mpc_surrogate_predict(mpc_ctx* c, const float* features, int m, float* y) {
  if (!c) return MPC_EINVAL;
  if (m < 0 || (m > 0 && (!features || !y))) return fail(c, MPC_EINVAL, "bad prediction arguments");
  const int chunk = 65536;
  MlpScratch S;
  HIPCHK(c, S.alloc((size_t)std::min(m, chunk)));
  HIPCHK(c, launch_params_to_bf16(c->sur_p, c->sur_p16, kMlpParams, c->stream));
  for (int m0 = 0; m0 < m; m0 += chunk) {
    const int b = std::min(chunk, m - m0);
    HIPCHK(c, launch_f32_to_bf16(features + (size_t)m0 * kFeat, S.X16, (long long)b * kFeat, c->stream));
    HIPCHK(c, mlp_forward(c, S, S.X16, b));
    HIPCHK(c, hipMemcpyAsync(y + m0, S.y, sizeof(float) * b, hipMemcpyDeviceToDevice, c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return MPC_OK;
}

extern "C" int mpc_surrogate_predict_noalloc(mpc_ctx* c, const float* features, int m, float* y) {
  if (!c) return MPC_EINVAL;
  if (m < 0 || (m > 0 && (!features || !y))) return fail(c, MPC_EINVAL, "bad prediction arguments");
  if (m > MPC_PREDICT_NOALLOC_MAX)
    return fail(c, MPC_EINVAL, "m above MPC_PREDICT_NOALLOC_MAX (" + std::to_string(MPC_PREDICT_NOALLOC_MAX) +
                                   "): the fixed working memory holds that many queries");
  if (m == 0) return MPC_OK;
  if (!c->na_scratch) return fail(c, MPC_ESTATE, "no working memory on this device");
  unsigned char* base = static_cast<unsigned char*>(c->na_scratch);
  uint16_t* X16 = reinterpret_cast<uint16_t*>(base);
  uint16_t* act[2] = {reinterpret_cast<uint16_t*>(base + kNaX16Bytes),
                      reinterpret_cast<uint16_t*>(base + kNaX16Bytes + kNaActBytes)};
  // The forward pass of mpc_surrogate_predict (same kernels, same bfloat16
  // dataflow) with the hidden activations ping-ponging through the fixed
  // buffers and the output written straight to y.
  HIPCHK(c, launch_f32_to_bf16(features, X16, (long long)m * kFeat, c->stream));
  const uint16_t* in = X16;
  int K = kFeat;
  for (int l = 0; l < 3; ++l) {
    GemmArgs g = gemm(m, kHid, K, in, K, 0, c->sur_p16 + mlp_w_off(l), K, 1);
    g.bias = c->sur_p + mlp_b_off(l);
    g.C16 = act[l & 1]; g.ldc16 = kHid; g.relu = 1;
    HIPCHK(c, launch_gemm_bf16(g, c->stream));
    in = act[l & 1];
    K = kHid;
  }
  GemmArgs g = gemm(m, 1, kHid, in, kHid, 0, c->sur_p16 + mlp_w_off(3), kHid, 1);
  g.bias = c->sur_p + mlp_b_off(3);
  g.C32 = y; g.ldc = 1;
  HIPCHK(c, launch_gemm_bf16(g, c->stream));
  return MPC_OK;
}

extern "C" int mpc_surrogate_get_params(mpc_ctx* c, float* params) {
  if (!c || !params) return MPC_EINVAL;
  HIPCHK(c, hipMemcpyAsync(params, c->sur_p, sizeof(float) * kMlpParams, hipMemcpyDeviceToDevice, c->stream));
  return MPC_OK;
}

extern "C" int mpc_surrogate_set_params(mpc_ctx* c, const float* params) {
  if (!c || !params) return MPC_EINVAL;
  int rc = check_shared_model(c);
  if (rc) return rc;
  HIPCHK(c, hipMemcpyAsync(c->sur_p, params, sizeof(float) * kMlpParams, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, launch_params_to_bf16(c->sur_p, c->sur_p16, kMlpParams, c->stream));
  c->sur_ready = true;
  c->hist_stale = true;
  return MPC_OK;
}

extern "C" int mpc_surrogate_train(mpc_ctx* c, const mpc_train_params* tp, mpc_train_report* rep) {
  if (!c || !tp) return MPC_EINVAL;
  if (c->A < 2) return fail(c, MPC_EINVAL, "the learned distance needs at least two arms");
  if (tp->samples < 1024 || tp->batch < 64 || tp->batch > 65536 || tp->epochs < 1 ||
      !(tp->val_fraction >= 0.f && tp->val_fraction < 0.5f) || !(tp->lr > 0.f) ||
      !(tp->lr_final > 0.f && tp->lr_final <= tp->lr) || !(tp->near_weight >= 0.f) ||
      !(tp->target_floor < tp->target_clip))
    return fail(c, MPC_EINVAL, "bad training parameters");
  int rc = check_shared_model(c);
  if (rc) return rc;
  hipEvent_t e0, e1;
  HIPCHK(c, hipEventCreate(&e0));
  HIPCHK(c, hipEventCreate(&e1));
  HIPCHK(c, hipEventRecord(e0, c->stream));
  const int M = tp->samples;
  const int n_val = (int)(M * tp->val_fraction);
  const int n_train = M - n_val;
  const int B = tp->batch;
  // Training set: every directed arm pair of this context, joints uniform in the limits.
  std::vector<int> pairs;
  for (int a = 0; a < c->A; ++a)
    for (int i = 0; i < c->A; ++i)
      if (i != a) {
        pairs.push_back(a);
        pairs.push_back(i);
      }
  MlpScratch S;
  HIPCHK(c, S.alloc((size_t)B));
  uint16_t* X16 = nullptr;
  float* T = nullptr;
  int* d_pairs = nullptr;
  HIPCHK(c, S.get(&X16, (size_t)M * kFeat));
  HIPCHK(c, S.get(&T, (size_t)M));
  HIPCHK(c, S.get(&d_pairs, pairs.size()));
  HIPCHK(c, hipMemcpy(d_pairs, pairs.data(), pairs.size() * sizeof(int), hipMemcpyHostToDevice));
  const uint32_t slo = (uint32_t)(tp->seed & 0xffffffffull), shi = (uint32_t)(tp->seed >> 32);
  for (int m0 = 0; m0 < M; m0 += (1 << 20)) {
    const int n = std::min(1 << 20, M - m0);
    HIPCHK(c, launch_sur_sample_layout(c->layout, c->d_arms, c->d_model, d_pairs, (int)pairs.size() / 2, slo, shi,
                                       m0, n, tp->target_clip, tp->target_floor, X16 + (size_t)m0 * kFeat, T + m0,
                                       nullptr, c->stream));
  }
  // Parameters uniform in +-1/sqrt(fan_in), zero Adam moments.
  HIPCHK(c, launch_init_params(c->sur_p, slo ^ 0x9E3779B9u, shi, c->stream));
  HIPCHK(c, hipMemsetAsync(c->sur_m, 0, sizeof(float) * kMlpParams, c->stream));
  HIPCHK(c, hipMemsetAsync(c->sur_v, 0, sizeof(float) * kMlpParams, c->stream));
  HIPCHK(c, launch_params_to_bf16(c->sur_p, c->sur_p16, kMlpParams, c->stream));
  long long step = 0;
  float last_loss = 0.f;
  const int nb = n_train / B;
  for (int ep = 0; ep < tp->epochs; ++ep) {
    HIPCHK(c, hipMemsetAsync(S.loss, 0, sizeof(float), c->stream));
    for (int b = 0; b < nb; ++b) {
      const uint16_t* xb = X16 + (size_t)b * B * kFeat;
      HIPCHK(c, mlp_forward(c, S, xb, B));
      HIPCHK(c, launch_loss(S.y, T + (size_t)b * B, B, tp->over_weight, tp->near_weight, tp->near_band, S.dy, S.dy16,
                            S.loss, c->stream));
      HIPCHK(c, mlp_backward(c, S, xb, B));
      ++step;
      // step size: cosine from lr to lr_final over the run
      const double total = (double)tp->epochs * nb;
      const double cw = 0.5 * (1.0 + std::cos(M_PI * (double)(step - 1) / total));
      const float lr_t = (float)(tp->lr_final + (tp->lr - tp->lr_final) * cw);
      HIPCHK(c, launch_adam(c->sur_p, c->sur_m, c->sur_v, c->sur_g, kMlpParams, lr_t, tp->beta1, tp->beta2,
                            tp->adam_eps, (int)std::min<long long>(step, 1 << 30), c->stream));
      HIPCHK(c, launch_params_to_bf16(c->sur_p, c->sur_p16, kMlpParams, c->stream));
    }
    float l = 0.f;
    HIPCHK(c, hipMemcpyAsync(&l, S.loss, sizeof(float), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    last_loss = nb > 0 ? l / nb : 0.f;
  }
  // Held-out error of the trained network (same bfloat16 dataflow), and the
  // skip decision at the context's margin: share of samples predicted at or
  // beyond it, share of colliding samples (target < 0) among them, largest
  // over-prediction of a sample whose target is below the margin.
  float mae = 0.f, rmse = 0.f, p99 = 0.f, max_over = 0.f, min_err = 0.f;
  float skip_rate = 0.f, miss_rate = 0.f, max_over_near = 0.f;
  const float margin = c->hmodel.margin;
  if (n_val > 0) {
    std::vector<float> pred(n_val), tgt(n_val);
    float* yv = nullptr;
    HIPCHK(c, S.get(&yv, (size_t)n_val));
    for (int m0 = 0; m0 < n_val; m0 += B) {
      const int b = std::min(B, n_val - m0);
      HIPCHK(c, mlp_forward(c, S, X16 + (size_t)(n_train + m0) * kFeat, b));
      HIPCHK(c, hipMemcpyAsync(yv + m0, S.y, sizeof(float) * b, hipMemcpyDeviceToDevice, c->stream));
    }
    HIPCHK(c, hipMemcpyAsync(pred.data(), yv, sizeof(float) * n_val, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(tgt.data(), T + n_train, sizeof(float) * n_val, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    std::vector<float> ae(n_val);
    double s1 = 0.0, s2 = 0.0;
    long long n_skip = 0, n_coll = 0, n_miss = 0;
    for (int i = 0; i < n_val; ++i) {
      const float e = pred[i] - tgt[i];
      ae[i] = std::fabs(e);
      s1 += ae[i];
      s2 += (double)e * e;
      max_over = std::max(max_over, e);
      min_err = std::min(min_err, e);
      const bool skip = pred[i] >= margin;
      n_skip += skip;
      if (tgt[i] < 0.f) {
        ++n_coll;
        n_miss += skip;
      }
      if (tgt[i] < margin) max_over_near = std::max(max_over_near, e);
    }
    skip_rate = (float)((double)n_skip / n_val);
    miss_rate = n_coll ? (float)((double)n_miss / n_coll) : 0.f;
    std::sort(ae.begin(), ae.end());
    mae = (float)(s1 / n_val);
    rmse = (float)std::sqrt(s2 / n_val);
    p99 = ae[(size_t)(0.99 * (n_val - 1))];
  }
  HIPCHK(c, hipEventRecord(e1, c->stream));
  HIPCHK(c, hipEventSynchronize(e1));
  float ms = 0.f;
  HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->sur_ready = true;
  c->hist_stale = true;
  if (rep) {
    rep->final_loss = last_loss;
    rep->val_mae = mae;
    rep->val_rmse = rmse;
    rep->val_p99 = p99;
    rep->val_max_over = max_over;
    rep->val_min_err = min_err;
    rep->val_skip_rate = skip_rate;
    rep->val_miss_rate = miss_rate;
    rep->val_max_over_near = max_over_near;
    rep->steps = step;
    rep->seconds = ms * 1e-3f;
  }
  return MPC_OK;
}

extern "C" int mpc_surrogate_samples(mpc_ctx* c, unsigned long long seed, long long first, int m, float clip,
                                     float floor, float* features, float* targets, float* joints) {
  if (!c) return MPC_EINVAL;
  if (c->A < 2 || m < 0 || (m > 0 && (!features || !targets)))
    return fail(c, MPC_EINVAL, "bad sample arguments");
  int rc = check_shared_model(c);
  if (rc) return rc;
  std::vector<int> pairs;
  for (int a = 0; a < c->A; ++a)
    for (int i = 0; i < c->A; ++i)
      if (i != a) {
        pairs.push_back(a);
        pairs.push_back(i);
      }
  MlpScratch S;
  int* d_pairs = nullptr;
  uint16_t* X16 = nullptr;
  HIPCHK(c, S.get(&d_pairs, pairs.size()));
  HIPCHK(c, S.get(&X16, (size_t)m * kFeat));
  HIPCHK(c, hipMemcpy(d_pairs, pairs.data(), pairs.size() * sizeof(int), hipMemcpyHostToDevice));
  HIPCHK(c, launch_sur_sample_layout(c->layout, c->d_arms, c->d_model, d_pairs, (int)pairs.size() / 2,
                                     (uint32_t)(seed & 0xffffffffull), (uint32_t)(seed >> 32), first, m, clip, floor,
                                     X16, targets, joints, c->stream));
  // features back to FP32 (they are exactly the bfloat16 values the network sees)
  std::vector<uint16_t> h((size_t)m * kFeat);
  std::vector<float> f((size_t)m * kFeat);
  HIPCHK(c, hipMemcpyAsync(h.data(), X16, h.size() * 2, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (size_t i = 0; i < h.size(); ++i) {
    const uint32_t u = (uint32_t)h[i] << 16;
    memcpy(&f[i], &u, 4);
  }
  HIPCHK(c, hipMemcpy(features, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice));
  return MPC_OK;
}

extern "C" int mpc_surrogate_adam(mpc_ctx* c, const float* grad, float lr, float b1, float b2, float eps, int step) {
  if (!c) return MPC_EINVAL;
  if (!grad || step < 1 || !(lr > 0.f) || !(b1 >= 0.f && b1 < 1.f) || !(b2 >= 0.f && b2 < 1.f) || !(eps >= 0.f))
    return fail(c, MPC_EINVAL, "bad Adam arguments");
  if (step == 1) {
    HIPCHK(c, hipMemsetAsync(c->sur_m, 0, sizeof(float) * kMlpParams, c->stream));
    HIPCHK(c, hipMemsetAsync(c->sur_v, 0, sizeof(float) * kMlpParams, c->stream));
  }
  HIPCHK(c, launch_adam(c->sur_p, c->sur_m, c->sur_v, grad, kMlpParams, lr, b1, b2, eps, step, c->stream));
  HIPCHK(c, launch_params_to_bf16(c->sur_p, c->sur_p16, kMlpParams, c->stream));
  c->hist_stale = true;  // a changed network starts without drop history
  return MPC_OK;
}

extern "C" int mpc_set_collision_mode(mpc_ctx* c, int mode) {
  if (!c) return MPC_EINVAL;
  if (mode != 0 && mode != 1) return fail(c, MPC_EINVAL, "mode must be 0 or 1");
  if (mode == 1) {
    int rc = check_shared_model(c);
    if (rc) return rc;
    if (!(c->hmodel.margin >= c->P.buf_dyn))
      return fail(c, MPC_EINVAL, "surrogate_margin must be at least buf_dyn");
  }
  if (mode != c->collision_mode) {
    c->collision_mode = mode;
    c->tuned = false;  // re-tune and re-capture for the new step body
    c->n_items = 0;
    c->hist_stale = true;
  }
  return MPC_OK;
}

extern "C" int mpc_surrogate_audit(mpc_ctx* c, int on) {
  if (!c) return MPC_EINVAL;
  if ((on != 0) != c->sur_audit) {
    c->sur_audit = on != 0;
    c->tuned = false;
    c->n_items = 0;
  }
  return MPC_OK;
}

extern "C" int mpc_surrogate_stats(mpc_ctx* c, unsigned long long* out, int reset) {
  if (!c || !out) return MPC_EINVAL;
  std::vector<unsigned long long> h(kSurCounters * c->A);
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(h.data(), c->sur_counts, h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost));
  for (int k = 0; k < kSurCounters; ++k) {
    out[k] = 0;
    for (int a = 0; a < c->A; ++a) out[k] += h[kSurCounters * a + k];
  }
  if (reset) HIPCHK(c, hipMemset(c->sur_counts, 0, h.size() * sizeof(unsigned long long)));
  return MPC_OK;
}
