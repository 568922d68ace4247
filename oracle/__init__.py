"""ctypes binding of the FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Imported by the tests, by ``__graft_entry__.smoke()`` and by the
CPU-baseline leg of ``bench.py``; never by the product package.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC = os.path.join(_HERE, "mrstorm_oracle.c")

MAX_DOF, MAX_SPHERES, MAX_ARMS = 8, 64, 16


def build(force: bool = True) -> str:
    """Compile the oracle with the host C compiler (no contraction, no
    fast-math, so every operation is the IEEE double operation written)."""
    if force or not os.path.exists(LIB_PATH):
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-o", LIB_PATH, SRC, "-lm"]
        subprocess.run(cmd, check=True)
    return LIB_PATH


class OrcArm(C.Structure):
    _fields_ = [("dof", C.c_int), ("n_spheres", C.c_int), ("n_rollouts", C.c_int),
                ("horizon", C.c_int),
                ("dh", C.c_double * 4 * MAX_DOF), ("qlim", C.c_double * 2 * MAX_DOF),
                ("qdmax", C.c_double * MAX_DOF), ("spheres", C.c_double * 4 * MAX_SPHERES),
                ("link", C.c_int * MAX_SPHERES), ("base", C.c_double * 4),
                ("tool", C.c_double * 3)]


class OrcParams(C.Structure):
    _fields_ = [(n, C.c_double) for n in (
        "dt", "sigma", "lam", "gamma", "alpha_mu", "w_pose", "w_rot", "w_stop", "w_joint",
        "w_coll", "w_dyn", "buf_env", "buf_self", "buf_dyn", "tau", "prio_min", "prio_max",
        "dist_floor", "joint_margin")] + [("seed", C.c_ulonglong), ("iters", C.c_int),
                                          ("plan_mode", C.c_int), ("alpha_sigma", C.c_double),
                                          ("sigma_floor", C.c_double), ("w_manip", C.c_double),
                                          ("manip_thresh", C.c_double)]


_lib = None
_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_up = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        L.orc_philox4x32_10.argtypes = [_up, _up, _up]
        L.orc_normals.argtypes = [C.c_ulonglong, C.c_int, C.c_uint32, C.c_int, C.c_int, C.c_int,
                                  C.c_int, _dp]
        L.orc_integrate.argtypes = [C.c_int, C.c_int, C.c_double, _dp, _dp, _dp, _dp, _dp]
        L.orc_fk.argtypes = [C.POINTER(OrcArm), _dp, _dp]
        L.orc_spheres.argtypes = [C.POINTER(OrcArm), _dp, _dp]
        L.orc_ee_pose.argtypes = [C.POINTER(OrcArm), _dp, _dp]
        L.orc_quat_to_rot.argtypes = [_dp, _dp]
        L.orc_sphere_rho.argtypes = [_dp, _dp]
        L.orc_sphere_rho.restype = C.c_double
        L.orc_rho_sets.argtypes = [_dp, C.c_int, _dp, C.c_int]
        L.orc_rho_sets.restype = C.c_double
        L.orc_rho_self.argtypes = [_dp, _ip, C.c_int]
        L.orc_rho_self.restype = C.c_double
        L.orc_hinge.argtypes = [C.c_double, C.c_double]
        L.orc_hinge.restype = C.c_double
        L.orc_pose_cost.argtypes = [_dp, _dp, C.c_double]
        L.orc_pose_cost.restype = C.c_double
        L.orc_stop_cost.argtypes = [C.POINTER(OrcArm), C.c_int, C.c_int, _dp]
        L.orc_stop_cost.restype = C.c_double
        L.orc_joint_cost.argtypes = [C.POINTER(OrcArm), _dp, C.c_double]
        L.orc_joint_cost.restype = C.c_double
        L.orc_priority.argtypes = [C.c_double] * 6
        L.orc_priority.restype = C.c_double
        L.orc_total_cost.argtypes = [C.c_int, C.c_double, _dp]
        L.orc_total_cost.restype = C.c_double
        L.orc_weights.argtypes = [C.c_int, C.c_double, _dp, _dp]
        L.orc_weighted_mean.argtypes = [C.c_int, C.c_int, C.c_int, _dp, _dp, _dp]
        L.orc_ema.argtypes = [C.c_int, C.c_int, C.c_double, _dp, _dp]
        L.orc_weighted_cov.argtypes = [C.c_int, C.c_int, C.c_int, _dp, _dp, _dp, _dp]
        L.orc_cholesky_floor.argtypes = [C.c_int, _dp, C.c_double, _dp]
        L.orc_jacobian.argtypes = [C.c_void_p, _dp, _dp]
        L.orc_manip_cost.argtypes = [C.c_void_p, _dp, C.c_double]
        L.orc_manip_cost.restype = C.c_double
        L.orc_get_sigma.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]
        L.orc_argmin.argtypes = [C.c_int, _dp]
        L.orc_argmin.restype = C.c_int
        L.orc_shift.argtypes = [C.c_int, C.c_int, _dp]
        L.orc_pair_count.argtypes = [C.c_int, C.c_int, C.c_int, _ip, C.c_int]
        L.orc_pair_count.restype = C.c_longlong
        L.orc_stage_costs_batch.argtypes = [
            C.POINTER(OrcArm), C.POINTER(OrcParams), C.c_int, C.c_int, _dp, _dp, _dp, _dp, _dp,
            C.c_int, _dp, C.c_int, C.c_int, C.c_int, _ip, _ip, _ip, _dp, _dp, C.c_void_p]
        L.orc_create.argtypes = [C.POINTER(OrcArm), C.c_int, C.POINTER(OrcParams)]
        L.orc_create.restype = C.c_void_p
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_share_plans.argtypes = [C.c_void_p, C.c_void_p]
        L.orc_step.argtypes = [C.c_void_p, _dp, _dp, _dp, C.c_int, _dp]
        L.orc_set_rollout_window.argtypes = [C.c_void_p, C.c_int, C.c_int]
        L.orc_get_mean.argtypes = [C.c_void_p, C.c_int, _dp]
        L.orc_set_mean.argtypes = [C.c_void_p, C.c_int, _dp]
        L.orc_get_plan.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p,
                                   C.POINTER(C.c_double), C.POINTER(C.c_int)]
        L.orc_set_plan.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_double, C.c_int]
        L.orc_get_costs.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_get_noise.argtypes = [C.c_void_p, C.c_int, _dp]
        L.orc_get_alpha.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_get_step.argtypes = [C.c_void_p]
        L.orc_get_step.restype = C.c_uint32
        L.orc_set_step.argtypes = [C.c_void_p, C.c_uint32]
        L.orc_arm_pair_rho.argtypes = [C.POINTER(OrcArm), _dp, C.POINTER(OrcArm), _dp]
        L.orc_arm_pair_rho.restype = C.c_double
        L.orc_mlp_param_count.argtypes = [C.c_int, _ip]
        L.orc_mlp_param_count.restype = C.c_longlong
        L.orc_mlp_forward.argtypes = [C.c_int, _ip, _dp, C.c_int, _dp, _dp]
        L.orc_mlp_loss_grad.argtypes = [C.c_int, _ip, _dp, C.c_int, _dp, _dp, C.c_double, C.c_double, C.c_double,
                                        _dp]
        L.orc_mlp_loss_grad.restype = C.c_double
        L.orc_adam.argtypes = [C.c_longlong, _dp, _dp, _dp, _dp, C.c_double, C.c_double,
                               C.c_double, C.c_double, C.c_int]
        L.orc_bf16.argtypes = [C.c_double]
        L.orc_bf16.restype = C.c_double
        L.orc_mlp_loss_grad_bf16.argtypes = [C.c_int, _ip, _dp, C.c_int, _dp, _dp, C.c_double, C.c_double,
                                             C.c_double, _dp]
        L.orc_mlp_loss_grad_bf16.restype = C.c_double
        L.orc_pair_features.argtypes = [C.POINTER(OrcArm), _dp, C.POINTER(OrcArm), _dp, _dp]
        L.orc_mlp_forward_bf16.argtypes = [C.c_int, _ip, _dp, C.c_int, _dp, _dp]
        _lib = L
    return _lib


def _f64(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def make_arm(arm) -> OrcArm:
    """Oracle arm descriptor from a scenes.Arm (FP32 values widened exactly)."""
    o = OrcArm()
    d, S = arm.dof, arm.n_spheres
    o.dof, o.n_spheres, o.n_rollouts, o.horizon = d, S, arm.n_rollouts, arm.horizon
    for k in range(d):
        for i in range(4):
            o.dh[k][i] = float(arm.dh[k, i])
        o.qlim[k][0], o.qlim[k][1] = float(arm.q_lim[k, 0]), float(arm.q_lim[k, 1])
        o.qdmax[k] = float(arm.qd_max[k])
    for s in range(S):
        for i in range(4):
            o.spheres[s][i] = float(arm.spheres[s, i])
        o.link[s] = int(arm.sphere_link[s])
    for i in range(4):
        o.base[i] = float(arm.base[i])
    for i in range(3):
        o.tool[i] = float(arm.tool[i])
    return o


def make_params(p: dict) -> OrcParams:
    o = OrcParams()
    for name, _ in OrcParams._fields_:
        if name in ("seed", "iters", "plan_mode"):
            continue
        setattr(o, name, float(np.float32(p[name])))
    o.seed = int(p["seed"])
    o.iters = int(p["iters"])
    o.plan_mode = int(p.get("plan_mode", 0))
    return o


# ---------------------------------------------------------------- wrappers
def philox(ctr, key):
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(np.asarray(ctr, dtype=np.uint32), np.asarray(key, dtype=np.uint32), out)
    return out


def normals(seed, arm, t, k, n, h, dof):
    z = np.zeros(dof)
    lib().orc_normals(seed, arm, t, k, n, h, dof, z)
    return z


def integrate(q0, qd0, U, dt):
    U = _f64(U)
    H, d = U.shape
    q, qd = np.zeros((H, d)), np.zeros((H, d))
    lib().orc_integrate(d, H, dt, _f64(q0), _f64(qd0), U, q, qd)
    return q, qd


def fk(oarm: OrcArm, q):
    fr = np.zeros((oarm.dof + 1, 4, 4))
    lib().orc_fk(C.byref(oarm), _f64(q), fr)
    return fr


def spheres(oarm: OrcArm, q):
    out = np.zeros((oarm.n_spheres, 4))
    lib().orc_spheres(C.byref(oarm), _f64(q), out)
    return out


def ee_pose(oarm: OrcArm, q):
    T = np.zeros((4, 4))
    lib().orc_ee_pose(C.byref(oarm), _f64(q), T)
    return T


def quat_to_rot(q):
    R = np.zeros((3, 3))
    lib().orc_quat_to_rot(_f64(q), R)
    return R


def sphere_rho(a, b):
    return lib().orc_sphere_rho(_f64(a), _f64(b))


def rho_sets(A, B):
    A, B = _f64(A).reshape(-1, 4), _f64(B).reshape(-1, 4)
    return lib().orc_rho_sets(A, A.shape[0], B, B.shape[0])


def rho_self(c, link):
    c = _f64(c).reshape(-1, 4)
    return lib().orc_rho_self(c, np.ascontiguousarray(link, dtype=np.int32), c.shape[0])


def hinge(rho, B):
    return lib().orc_hinge(rho, B)


def pose_cost(T, goal, w_rot):
    return lib().orc_pose_cost(_f64(T), _f64(goal), w_rot)


def stop_cost(oarm, H, h, qd):
    return lib().orc_stop_cost(C.byref(oarm), H, h, _f64(qd))


def joint_cost(oarm, q, margin):
    return lib().orc_joint_cost(C.byref(oarm), _f64(q), margin)


def priority(d_own, d_other, tau, floor_, pmin, pmax):
    return lib().orc_priority(d_own, d_other, tau, floor_, pmin, pmax)


def total_cost(stage, gamma):
    stage = _f64(stage)
    return lib().orc_total_cost(stage.shape[0], gamma, stage)


def weights(C_, lam):
    C_ = _f64(C_)
    w = np.zeros_like(C_)
    lib().orc_weights(C_.shape[0], lam, C_, w)
    return w


def weighted_mean(w, U):
    U = _f64(U)
    N, H, d = U.shape
    mt = np.zeros((H, d))
    lib().orc_weighted_mean(N, H, d, _f64(w), U, mt)
    return mt


def weighted_cov(w, U, mt):
    U = _f64(U)
    N, H, d = U.shape
    out = np.zeros((H, d, d))
    lib().orc_weighted_cov(N, H, d, _f64(w), U, _f64(mt), out)
    return out


def jacobian(oarm, q):
    J = np.zeros((6, oarm.dof))
    lib().orc_jacobian(C.byref(oarm), _f64(q), J)
    return J


def manip_cost(oarm, q, thresh):
    return lib().orc_manip_cost(C.byref(oarm), _f64(q), float(thresh))


def cholesky_floor(S, floor_var):
    S = _f64(S)
    d = S.shape[0]
    L = np.zeros((d, d))
    lib().orc_cholesky_floor(d, S, float(floor_var), L)
    return L


def ema(mu, mt, a):
    mu = _f64(mu).copy()
    H, d = mu.shape
    lib().orc_ema(H, d, a, _f64(mt), mu)
    return mu


def argmin(C_):
    C_ = _f64(C_)
    return lib().orc_argmin(C_.shape[0], C_)


def shift(mu):
    mu = _f64(mu).copy()
    H, d = mu.shape
    lib().orc_shift(H, d, mu)
    return mu


def pair_count(H, N, S_own, S_nb):
    S_nb = np.ascontiguousarray(S_nb, dtype=np.int32)
    return lib().orc_pair_count(H, N, S_own, S_nb, S_nb.shape[0])


def stage_costs_batch(oarm, oparams, q, qd, sph, goal, obs, plans, nb_S, nb_H, nb_valid,
                      alpha_row, want_terms=False):
    """q, qd: [N][H][d]; sph: [N][H][S][4]; plans: [n_nb][Hmax][Smax][4].
    Returns stage costs [H][N] (and terms [H][N][8]: pose, stop, joint, coll,
    self, dyn, total, manip)."""
    q, qd, sph = _f64(q), _f64(qd), _f64(sph)
    N, H, _ = q.shape
    obs = _f64(obs).reshape(-1, 4)
    if obs.shape[0] == 0:
        obs = np.zeros((1, 4))
        n_obs = 0
    else:
        n_obs = obs.shape[0]
    plans = _f64(plans)
    if plans.size == 0:
        plans = np.zeros((1, 1, 1, 4))
    n_nb = len(nb_S)
    out = np.zeros((H, N))
    terms = np.zeros((H, N, 8)) if want_terms else None
    lib().orc_stage_costs_batch(
        C.byref(oarm), C.byref(oparams), N, H, q, qd, sph, _f64(goal), obs, n_obs, plans, n_nb,
        plans.shape[1], plans.shape[2], np.ascontiguousarray(nb_S, dtype=np.int32) if n_nb else np.zeros(1, np.int32),
        np.ascontiguousarray(nb_H, dtype=np.int32) if n_nb else np.zeros(1, np.int32),
        np.ascontiguousarray(nb_valid, dtype=np.int32) if n_nb else np.zeros(1, np.int32),
        _f64(alpha_row) if n_nb else np.zeros(1), out,
        terms.ctypes.data_as(C.c_void_p) if want_terms else None)
    return (out, terms) if want_terms else out


def arm_pair_rho(oa, qa, ob, qb):
    return lib().orc_arm_pair_rho(C.byref(oa), _f64(qa), C.byref(ob), _f64(qb))


def mlp_param_count(widths):
    w = np.ascontiguousarray(widths, dtype=np.int32)
    return lib().orc_mlp_param_count(len(widths) - 1, w)


def mlp_forward(widths, params, x):
    w = np.ascontiguousarray(widths, dtype=np.int32)
    x = _f64(x)
    y = np.zeros((x.shape[0], widths[-1]))
    lib().orc_mlp_forward(len(widths) - 1, w, _f64(params), x.shape[0], x, y)
    return y


def mlp_loss_grad(widths, params, x, t, over_w, near_w=0.0, near_band=0.0):
    w = np.ascontiguousarray(widths, dtype=np.int32)
    x = _f64(x)
    g = np.zeros(mlp_param_count(widths))
    loss = lib().orc_mlp_loss_grad(len(widths) - 1, w, _f64(params), x.shape[0], x, _f64(t),
                                   over_w, near_w, near_band, g)
    return loss, g


def bf16(x):
    return lib().orc_bf16(float(x))


def mlp_forward_bf16(widths, params, x):
    w = np.ascontiguousarray(widths, dtype=np.int32)
    x = _f64(x)
    y = np.zeros((x.shape[0], widths[-1]))
    lib().orc_mlp_forward_bf16(len(widths) - 1, w, _f64(params), x.shape[0], x, y)
    return y


def mlp_loss_grad_bf16(widths, params, x, t, over_w, near_w=0.0, near_band=0.0):
    w = np.ascontiguousarray(widths, dtype=np.int32)
    x = _f64(x)
    g = np.zeros(mlp_param_count(widths))
    loss = lib().orc_mlp_loss_grad_bf16(len(widths) - 1, w, _f64(params), x.shape[0], x, _f64(t),
                                        over_w, near_w, near_band, g)
    return loss, g


def pair_features(oa, qa, oi, qi):
    f = np.zeros(17)
    lib().orc_pair_features(C.byref(oa), _f64(qa), C.byref(oi), _f64(qi), f)
    return f


def adam(p, m, v, g, lr, b1, b2, eps, step):
    lib().orc_adam(p.size, p, m, v, _f64(g), lr, b1, b2, eps, step)


class Controller:
    """Full oracle controller over all arms of a scene (Alg. 1 per arm)."""

    def __init__(self, scene_arms, params: dict):
        self.arms = [make_arm(a) for a in scene_arms]
        self.params = make_params(params)
        arr = (OrcArm * len(self.arms))(*self.arms)
        self._arr = arr
        self.h = lib().orc_create(arr, len(self.arms), C.byref(self.params))
        if not self.h:
            raise ValueError("orc_create failed")
        self.A = len(self.arms)
        self.d = scene_arms[0].dof
        self.Hmax = max(a.horizon for a in scene_arms)
        self.Smax = max(a.n_spheres for a in scene_arms)
        self.Nmax = max(a.n_rollouts for a in scene_arms)

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_destroy(self.h)
            self.h = None

    def share_plans(self, mask=None):
        if mask is None:
            lib().orc_share_plans(self.h, None)
        else:
            m = np.ascontiguousarray(mask, dtype=np.uint8)
            lib().orc_share_plans(self.h, m.ctypes.data_as(C.c_void_p))

    def step(self, state, goal, obstacles):
        obs = _f64(obstacles).reshape(-1, 4)
        n_obs = obs.shape[0]
        if n_obs == 0:
            obs = np.zeros((1, 4))
        u = np.zeros((self.A, self.d))
        lib().orc_step(self.h, _f64(state), _f64(goal), obs, n_obs, u)
        return u

    def set_window(self, lo, hi):
        lib().orc_set_rollout_window(self.h, lo, hi)

    def mean(self, a):
        mu = np.zeros((self.Hmax, self.d))
        lib().orc_get_mean(self.h, a, mu)
        return mu

    def set_mean(self, a, mu):
        lib().orc_set_mean(self.h, a, _f64(mu))

    def sigma(self, a):
        """(covariances, Cholesky factors) of arm a, [Hmax][d][d] each."""
        H, d = self.Hmax, self.d
        sig, chol = np.zeros((H, d, d)), np.zeros((H, d, d))
        lib().orc_get_sigma(self.h, a, sig.ctypes.data_as(C.c_void_p), chol.ctypes.data_as(C.c_void_p))
        return sig, chol

    def plan(self, a, side=0):
        p = np.zeros((self.Hmax, self.Smax, 4))
        pq = np.zeros((self.Hmax, self.d))
        dist, valid = C.c_double(), C.c_int()
        lib().orc_get_plan(self.h, a, side, p.ctypes.data_as(C.c_void_p),
                           pq.ctypes.data_as(C.c_void_p), C.byref(dist), C.byref(valid))
        return p, pq, dist.value, valid.value

    def set_plan(self, a, plan, plan_q, dist, valid):
        p = _f64(plan)
        pq = _f64(plan_q)
        lib().orc_set_plan(self.h, a, p.ctypes.data_as(C.c_void_p), pq.ctypes.data_as(C.c_void_p),
                           dist, valid)

    def costs(self, a):
        tot = np.zeros(self.Nmax)
        st = np.zeros((self.Hmax, self.Nmax))
        w = np.zeros(self.Nmax)
        lib().orc_get_costs(self.h, a, tot.ctypes.data_as(C.c_void_p),
                            st.ctypes.data_as(C.c_void_p), w.ctypes.data_as(C.c_void_p))
        return tot, st, w

    def noise(self, a):
        e = np.zeros((self.Nmax, self.Hmax, self.d))
        lib().orc_get_noise(self.h, a, e)
        return e

    def alpha(self):
        al = np.zeros((self.A, self.A))
        dn = np.zeros(self.A)
        lib().orc_get_alpha(self.h, al.ctypes.data_as(C.c_void_p), dn.ctypes.data_as(C.c_void_p))
        return al, dn

    @property
    def t(self):
        return lib().orc_get_step(self.h)

    @t.setter
    def t(self, v):
        lib().orc_set_step(self.h, v)
