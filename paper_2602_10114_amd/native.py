"""ctypes binding of libmrstorm.so (the C-ABI in include/mrstorm.h).

Argument marshalling only: every step of the control step runs in the HIP
library.  PyTorch is used for device memory and streams.  There is no
fallback: if the library is missing or no gfx950 device is present the calls
raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmrstorm.so")

MPC_OK, MPC_EINVAL, MPC_ENOMEM, MPC_EHIP, MPC_ESTATE, MPC_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
DBG = dict(NOISE=0, Q=1, QD=2, SPHERES=3, STAGE_COST=4, COST=5, WEIGHTS=6, MEAN=7, ALPHA=8,
           DIST=9, PAIRS=10, ARGMIN=11, PASSES=12, PRED=13, SIGMA=14, CHOL=15, SKIP=16)
EXPORTS = ["mpc_init", "mpc_share_plans", "mpc_step", "mpc_get_plan", "mpc_destroy",
           "mpc_last_error", "mpc_sync", "mpc_debug_enable", "mpc_debug_get", "mpc_get_board",
           "mpc_set_board", "mpc_set_mean", "mpc_get_step", "mpc_set_step", "mpc_sim_execute",
           "mpc_get_tuning", "mpc_set_tuning", "mpc_philox", "mpc_profile_enable",
           "mpc_profile_read", "mpc_pair_distance", "mpc_pair_features", "mpc_surrogate_samples",
           "mpc_surrogate_train", "mpc_surrogate_get_params", "mpc_surrogate_set_params",
           "mpc_surrogate_predict", "mpc_surrogate_grad", "mpc_set_collision_mode",
           "mpc_surrogate_audit", "mpc_surrogate_stats", "mpc_profile_read_surrogate",
           "mpc_surrogate_adam", "mpc_surrogate_predict_noalloc"]
MLP_WIDTHS = [17, 256, 256, 256, 1]
PREDICT_NOALLOC_MAX = 4096   # MPC_PREDICT_NOALLOC_MAX
MLP_PARAMS = 136449
# Default training recipe of the learned distance: 2M exact-kernel samples,
# Adam; the loss weighs over-prediction (the unsafe direction) 256x and
# samples within 0.15 m of contact 5x, with targets clipped to [-0.1, 0.5] m.
TRAINING_RECIPE = dict(samples=2_000_000, epochs=40, batch=4096, lr=1e-3, over_weight=256.0, near_weight=4.0,
                       near_band=0.15, target_floor=-0.1, target_clip=0.5, val_fraction=0.05, seed=7)


class MpcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class MpcArmDesc(C.Structure):
    _fields_ = [("dof", C.c_int), ("n_spheres", C.c_int), ("n_rollouts", C.c_int), ("horizon", C.c_int),
                ("dh", C.POINTER(C.c_float)), ("q_lim", C.POINTER(C.c_float)),
                ("qd_max", C.POINTER(C.c_float)), ("spheres", C.POINTER(C.c_float)),
                ("sphere_link", C.POINTER(C.c_int)), ("base", C.c_float * 4), ("tool", C.c_float * 3)]


class MpcTrainParams(C.Structure):
    _fields_ = [("samples", C.c_int), ("epochs", C.c_int), ("batch", C.c_int), ("lr", C.c_float),
                ("beta1", C.c_float), ("beta2", C.c_float), ("adam_eps", C.c_float),
                ("over_weight", C.c_float), ("target_clip", C.c_float), ("val_fraction", C.c_float),
                ("seed", C.c_ulonglong), ("lr_final", C.c_float), ("near_weight", C.c_float),
                ("near_band", C.c_float), ("target_floor", C.c_float)]


class MpcTrainReport(C.Structure):
    _fields_ = [("final_loss", C.c_float), ("val_mae", C.c_float), ("val_rmse", C.c_float),
                ("val_p99", C.c_float), ("val_max_over", C.c_float), ("val_min_err", C.c_float),
                ("steps", C.c_longlong), ("seconds", C.c_float), ("val_skip_rate", C.c_float),
                ("val_miss_rate", C.c_float), ("val_max_over_near", C.c_float)]


class MpcParams(C.Structure):
    _fields_ = [("dt", C.c_float), ("sigma", C.c_float), ("lam", C.c_float), ("gamma", C.c_float),
                ("alpha_mu", C.c_float), ("iters", C.c_int),
                ("w_pose", C.c_float), ("w_rot", C.c_float), ("w_stop", C.c_float),
                ("w_joint", C.c_float), ("w_coll", C.c_float), ("w_dyn", C.c_float),
                ("buf_env", C.c_float), ("buf_self", C.c_float), ("buf_dyn", C.c_float),
                ("tau", C.c_float), ("prio_min", C.c_float), ("prio_max", C.c_float),
                ("dist_floor", C.c_float), ("joint_margin", C.c_float), ("seed", C.c_ulonglong),
                ("max_obstacles", C.c_int), ("collision_mode", C.c_int),
                ("surrogate_margin", C.c_float), ("alpha_sigma", C.c_float), ("sigma_floor", C.c_float),
                ("plan_mode", C.c_int), ("w_manip", C.c_float), ("manip_thresh", C.c_float),
                ("surrogate_screen", C.c_float), ("surrogate_probe", C.c_int),
                ("surrogate_min_drop", C.c_float), ("pair_cull", C.c_int)]


_lib = None


def lib():
    """Load the built library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, ip, fp = C.c_void_p, C.c_int, C.c_float
        L.mpc_init.argtypes = [C.POINTER(MpcArmDesc), ip, C.POINTER(MpcParams), vp, C.POINTER(vp)]
        L.mpc_share_plans.argtypes = [vp, vp]
        L.mpc_step.argtypes = [vp, vp, vp, vp, ip, vp]
        L.mpc_get_plan.argtypes = [vp, ip, vp, vp, vp]
        L.mpc_destroy.argtypes = [vp]
        L.mpc_destroy.restype = None
        L.mpc_last_error.argtypes = [vp]
        L.mpc_last_error.restype = C.c_char_p
        L.mpc_sync.argtypes = [vp]
        L.mpc_debug_enable.argtypes = [vp, ip]
        L.mpc_debug_get.argtypes = [vp, ip, ip, vp]
        L.mpc_get_board.argtypes = [vp, ip, vp, vp, C.POINTER(fp), C.POINTER(ip)]
        L.mpc_set_board.argtypes = [vp, ip, vp, vp, fp, ip]
        L.mpc_set_mean.argtypes = [vp, ip, vp]
        L.mpc_get_step.argtypes = [vp, C.POINTER(C.c_uint)]
        L.mpc_set_step.argtypes = [vp, C.c_uint]
        L.mpc_sim_execute.argtypes = [vp, vp, vp]
        L.mpc_get_tuning.argtypes = [vp, C.POINTER(ip), C.POINTER(ip), C.POINTER(ip)]
        L.mpc_set_tuning.argtypes = [vp, ip, ip, ip]
        L.mpc_philox.argtypes = [vp, vp, vp, ip, vp]
        L.mpc_pair_distance.argtypes = [vp, ip, ip, vp, vp, ip, vp]
        L.mpc_pair_features.argtypes = [vp, ip, ip, vp, vp, ip, vp]
        L.mpc_surrogate_samples.argtypes = [vp, C.c_ulonglong, C.c_longlong, ip, fp, fp, vp, vp, vp]
        L.mpc_surrogate_train.argtypes = [vp, C.POINTER(MpcTrainParams), C.POINTER(MpcTrainReport)]
        L.mpc_surrogate_get_params.argtypes = [vp, vp]
        L.mpc_surrogate_set_params.argtypes = [vp, vp]
        L.mpc_surrogate_predict.argtypes = [vp, vp, ip, vp]
        L.mpc_surrogate_grad.argtypes = [vp, vp, vp, ip, fp, fp, fp, vp, C.POINTER(fp)]
        L.mpc_surrogate_adam.argtypes = [vp, vp, fp, fp, fp, fp, ip]
        L.mpc_surrogate_predict_noalloc.argtypes = [vp, vp, ip, vp]
        L.mpc_set_collision_mode.argtypes = [vp, ip]
        L.mpc_surrogate_audit.argtypes = [vp, ip]
        L.mpc_surrogate_stats.argtypes = [vp, vp, ip]
        L.mpc_profile_enable.argtypes = [vp, ip]
        L.mpc_profile_read.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(ip)]
        L.mpc_profile_read_surrogate.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(ip)]
        _lib = L
    return _lib


def _check(rc, ctx=None):
    if rc != MPC_OK:
        msg = lib().mpc_last_error(ctx).decode()
        raise MpcError(rc, msg)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def params_struct(p: dict) -> MpcParams:
    s = MpcParams()
    for name, _ in MpcParams._fields_:
        if name in ("iters", "max_obstacles", "collision_mode", "plan_mode"):
            setattr(s, name, int(p[name]))
        elif name == "surrogate_probe":
            s.surrogate_probe = int(p.get("surrogate_probe", 0))
        elif name == "surrogate_min_drop":
            s.surrogate_min_drop = float(p.get("surrogate_min_drop", 0.0))
        elif name == "pair_cull":
            s.pair_cull = int(p.get("pair_cull", 1))
        elif name == "seed":
            s.seed = int(p["seed"])
        else:
            setattr(s, name, float(p[name]))
    return s


def arm_descs(arms):
    """C descriptors of scenes.Arm records, and the host tables they point at
    (keep them alive until mpc_init returns)."""
    keep = []
    descs = (MpcArmDesc * len(arms))()
    for i, a in enumerate(arms):
        tabs = [np.ascontiguousarray(a.dh, np.float32), np.ascontiguousarray(a.q_lim, np.float32),
                np.ascontiguousarray(a.qd_max, np.float32), np.ascontiguousarray(a.spheres, np.float32),
                np.ascontiguousarray(a.sphere_link, np.int32)]
        keep.append(tabs)
        d = descs[i]
        d.dof, d.n_spheres, d.n_rollouts, d.horizon = a.dof, a.n_spheres, a.n_rollouts, a.horizon
        d.dh = tabs[0].ctypes.data_as(C.POINTER(C.c_float))
        d.q_lim = tabs[1].ctypes.data_as(C.POINTER(C.c_float))
        d.qd_max = tabs[2].ctypes.data_as(C.POINTER(C.c_float))
        d.spheres = tabs[3].ctypes.data_as(C.POINTER(C.c_float))
        d.sphere_link = tabs[4].ctypes.data_as(C.POINTER(C.c_int))
        for k in range(4):
            d.base[k] = float(a.base[k])
        for k in range(3):
            d.tool[k] = float(a.tool[k])
    return descs, keep


class Controller:
    """One context for every arm of a scene.  `arms` are scenes.Arm records;
    `stream` a torch.cuda.Stream (default: the current stream)."""

    def __init__(self, arms, params: dict, stream=None):
        import torch
        self.torch = torch
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.A = len(arms)
        self.arms = arms
        descs, self._keep = arm_descs(arms)
        self.params = params_struct(params)
        h = C.c_void_p()
        _check(lib().mpc_init(descs, self.A, C.byref(self.params), C.c_void_p(self.stream.cuda_stream),
                              C.byref(h)))
        self.h = h
        self._keep = None
        self.dev = torch.device("cuda", torch.cuda.current_device())

    def close(self):
        if getattr(self, "h", None):
            lib().mpc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _f32(self, x):
        t = self.torch
        if isinstance(x, t.Tensor):
            assert x.is_cuda and x.dtype == t.float32 and x.is_contiguous()
            return x
        return t.as_tensor(np.ascontiguousarray(x, np.float32), device=self.dev)

    def step(self, state, goal, obstacles, u_out=None):
        state, goal = self._f32(state), self._f32(goal)
        obstacles = self._f32(obstacles).reshape(-1, 4) if obstacles is not None else None
        n_obs = 0 if obstacles is None else int(obstacles.shape[0])
        if u_out is None:
            u_out = self.torch.empty((self.A, 7), dtype=self.torch.float32, device=self.dev)
        _check(lib().mpc_step(self.h, _ptr(state), _ptr(goal), _ptr(obstacles) if n_obs else None, n_obs,
                              _ptr(u_out)), self.h)
        return u_out

    def share_plans(self, mask=None):
        if mask is None:
            _check(lib().mpc_share_plans(self.h, None), self.h)
        else:
            m = (C.c_ubyte * self.A)(*[1 if x else 0 for x in mask])
            _check(lib().mpc_share_plans(self.h, C.cast(m, C.c_void_p)), self.h)

    def get_plan(self, arm):
        a = self.arms[arm]
        t = self.torch
        plan = t.empty((a.n_spheres, 4, a.horizon), dtype=t.float32, device=self.dev)
        pq = t.empty((a.horizon, 7), dtype=t.float32, device=self.dev)
        mean = t.empty((a.horizon, 7), dtype=t.float32, device=self.dev)
        _check(lib().mpc_get_plan(self.h, arm, _ptr(plan), _ptr(pq), _ptr(mean)), self.h)
        return plan, pq, mean

    def sync(self):
        _check(lib().mpc_sync(self.h), self.h)

    def debug_enable(self, on=True):
        _check(lib().mpc_debug_enable(self.h, 1 if on else 0), self.h)

    def debug_get(self, what, arm):
        a = self.arms[arm]
        N, H, S = a.n_rollouts, a.horizon, a.n_spheres
        t = self.torch
        shapes = dict(NOISE=(H, 7, N), Q=(N, H, 7), QD=(N, H, 7), SPHERES=(N, H, S, 4),
                      STAGE_COST=(H, N), COST=(N,), WEIGHTS=(N,), MEAN=(H, 7), ALPHA=(self.A,),
                      DIST=(1,), PAIRS=(1,), ARGMIN=(1,), PASSES=(3,), PRED=(self.A, H, N),
                      SIGMA=(H, 28), CHOL=(H, 28), SKIP=(self.A, H, N))
        dtype = dict(PAIRS=t.int64, ARGMIN=t.int32, PASSES=t.int64, SKIP=t.uint8).get(what, t.float32)
        out = t.empty(shapes[what], dtype=dtype, device=self.dev)
        _check(lib().mpc_debug_get(self.h, DBG[what], arm, _ptr(out)), self.h)
        return out

    def get_board(self, arm):
        a = self.arms[arm]
        t = self.torch
        plan = t.empty((a.horizon, a.n_spheres, 4), dtype=t.float32, device=self.dev)
        pq = t.empty((a.horizon, 7), dtype=t.float32, device=self.dev)
        dist, valid = C.c_float(), C.c_int()
        _check(lib().mpc_get_board(self.h, arm, _ptr(plan), _ptr(pq), C.byref(dist), C.byref(valid)), self.h)
        return plan, pq, dist.value, valid.value

    def set_board(self, arm, plan, plan_q, dist, valid):
        plan = self._f32(plan) if plan is not None else None
        plan_q = self._f32(plan_q) if plan_q is not None else None
        _check(lib().mpc_set_board(self.h, arm, _ptr(plan), _ptr(plan_q), float(dist), int(valid)), self.h)

    def set_mean(self, arm, mean):
        mean = self._f32(mean)
        _check(lib().mpc_set_mean(self.h, arm, _ptr(mean)), self.h)

    @property
    def t(self):
        v = C.c_uint()
        _check(lib().mpc_get_step(self.h, C.byref(v)), self.h)
        return v.value

    @t.setter
    def t(self, v):
        _check(lib().mpc_set_step(self.h, int(v)), self.h)

    def sim_execute(self, state, u):
        _check(lib().mpc_sim_execute(self.h, _ptr(state), _ptr(u)), self.h)

    def tuning(self):
        r, h, g = C.c_int(), C.c_int(), C.c_int()
        _check(lib().mpc_get_tuning(self.h, C.byref(r), C.byref(h), C.byref(g)), self.h)
        return r.value, h.value, g.value

    def set_tuning(self, rollouts_per_block=0, h_tile=0, grid=0):
        _check(lib().mpc_set_tuning(self.h, rollouts_per_block, h_tile, grid), self.h)


    def profile_enable(self, on=True):
        _check(lib().mpc_profile_enable(self.h, 1 if on else 0), self.h)

    def profile_read(self):
        """(total ms, launches) of the rollout kernels bracketed since the last read."""
        ms, n = C.c_double(), C.c_int()
        _check(lib().mpc_profile_read(self.h, C.byref(ms), C.byref(n)), self.h)
        return ms.value, n.value

    def profile_read_surrogate(self):
        """(total ms, launches) of the learned-distance inference kernels bracketed since the last read."""
        ms, n = C.c_double(), C.c_int()
        _check(lib().mpc_profile_read_surrogate(self.h, C.byref(ms), C.byref(n)), self.h)
        return ms.value, n.value


    # ---- learned arm-pair distance ----
    def pair_distance(self, arm_i, arm_j, q_i, q_j):
        q_i, q_j = self._f32(q_i), self._f32(q_j)
        m = int(q_i.shape[0])
        out = self.torch.empty(m, dtype=self.torch.float32, device=self.dev)
        _check(lib().mpc_pair_distance(self.h, arm_i, arm_j, _ptr(q_i), _ptr(q_j), m, _ptr(out)), self.h)
        return out

    def pair_features(self, arm_i, arm_j, q_i, q_j):
        q_i, q_j = self._f32(q_i), self._f32(q_j)
        m = int(q_i.shape[0])
        out = self.torch.empty((m, 17), dtype=self.torch.float32, device=self.dev)
        _check(lib().mpc_pair_features(self.h, arm_i, arm_j, _ptr(q_i), _ptr(q_j), m, _ptr(out)), self.h)
        return out

    def surrogate_samples(self, seed, first, m, clip=0.5, floor=-1e30):
        t = self.torch
        f = t.empty((m, 17), dtype=t.float32, device=self.dev)
        y = t.empty(m, dtype=t.float32, device=self.dev)
        q = t.empty((m, 14), dtype=t.float32, device=self.dev)
        _check(lib().mpc_surrogate_samples(self.h, int(seed), int(first), m, float(clip), float(floor), _ptr(f),
                                           _ptr(y), _ptr(q)), self.h)
        return f, y, q

    def surrogate_train(self, samples=2_000_000, epochs=10, batch=4096, lr=1e-3, beta1=0.9, beta2=0.999,
                        adam_eps=1e-8, over_weight=4.0, target_clip=0.5, val_fraction=0.05, seed=7,
                        lr_final=None, near_weight=0.0, near_band=0.0, target_floor=-1e30):
        tp = MpcTrainParams(samples, epochs, batch, lr, beta1, beta2, adam_eps, over_weight, target_clip,
                            val_fraction, seed, lr if lr_final is None else lr_final, near_weight, near_band,
                            target_floor)
        rep = MpcTrainReport()
        _check(lib().mpc_surrogate_train(self.h, C.byref(tp), C.byref(rep)), self.h)
        return {k: getattr(rep, k) for k, _ in MpcTrainReport._fields_}

    def surrogate_params(self):
        out = self.torch.empty(MLP_PARAMS, dtype=self.torch.float32, device=self.dev)
        _check(lib().mpc_surrogate_get_params(self.h, _ptr(out)), self.h)
        return out

    def set_surrogate_params(self, params):
        params = self._f32(params)
        _check(lib().mpc_surrogate_set_params(self.h, _ptr(params)), self.h)

    def surrogate_predict(self, features):
        features = self._f32(features)
        m = int(features.shape[0])
        out = self.torch.empty(m, dtype=self.torch.float32, device=self.dev)
        _check(lib().mpc_surrogate_predict(self.h, _ptr(features), m, _ptr(out)), self.h)
        return out

    def surrogate_grad(self, features, targets, over_weight=4.0, near_weight=0.0, near_band=0.0):
        features, targets = self._f32(features), self._f32(targets)
        g = self.torch.empty(MLP_PARAMS, dtype=self.torch.float32, device=self.dev)
        loss = C.c_float()
        _check(lib().mpc_surrogate_grad(self.h, _ptr(features), _ptr(targets), int(features.shape[0]),
                                        float(over_weight), float(near_weight), float(near_band), _ptr(g),
                                        C.byref(loss)), self.h)
        return g, loss.value

    def surrogate_adam(self, grad, lr, beta1=0.9, beta2=0.999, eps=1e-8, step=1):
        grad = self._f32(grad)
        _check(lib().mpc_surrogate_adam(self.h, _ptr(grad), float(lr), float(beta1), float(beta2), float(eps),
                                        int(step)), self.h)

    def set_collision_mode(self, mode):
        _check(lib().mpc_set_collision_mode(self.h, int(mode)), self.h)

    def surrogate_audit(self, on=True):
        _check(lib().mpc_surrogate_audit(self.h, 1 if on else 0), self.h)

    def surrogate_stats(self, reset=False):
        out = (C.c_ulonglong * 6)()
        _check(lib().mpc_surrogate_stats(self.h, C.cast(out, C.c_void_p), 1 if reset else 0), self.h)
        return dict(zip(["queries", "predicted_far", "waves_skipped", "misses", "missed_collisions",
                         "network_rows"], [int(x) for x in out]))


def philox(ctr, key, stream=None):
    """Device Philox4x32-10 on torch int32 tensors ctr [n][4], key [n][2]."""
    import torch
    n = ctr.shape[0]
    out = torch.empty((n, 4), dtype=torch.int32, device=ctr.device)
    s = stream if stream is not None else torch.cuda.current_stream()
    _check(lib().mpc_philox(_ptr(ctr), _ptr(key), _ptr(out), n, C.c_void_p(s.cuda_stream)))
    return out
