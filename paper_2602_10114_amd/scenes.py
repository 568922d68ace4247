"""Seeded synthetic inputs for the multi-arm MPC step.

This module only draws numbers: arm tables, base placements, start states,
goals, obstacle spheres and their straight-line motion.  It holds none of the
controller's arithmetic (no integration, kinematics, distances or costs), so
the HIP path and the CPU oracle can both be fed from it without sharing any
of the method.

The paper's robots (UR5e, Unitree G1), its IsaacSim scenes and its datasets
are not available; these scenes stand in for them with the shapes of the
benchmark configurations: a Franka-like 7-DoF arm described in modified
(Craig) Denavit-Hartenberg form, a collision-sphere tiling per link as in the
sphere-tiling description of Sec. IV-A, arm counts and layouts of 1, 2, 4 and
8 arms, and the reaching-task conventions of Sec. V-A (goals reset on a 5 cm
arrival or after one second; "hard" goals drawn in the shared centre).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

F32 = np.float32

# Modified DH rows (a_{k-1}, alpha_{k-1}, d_k, theta_offset_k) of a
# Panda-scale 7-DoF arm: 0.333 m shoulder height, 0.316 m upper arm,
# 0.384 m forearm, 0.0825 m elbow offsets, 0.088 m wrist offset.
FRANKA_LIKE_DH = np.array([
    [0.0, 0.0, 0.333, 0.0],
    [0.0, -math.pi / 2, 0.0, 0.0],
    [0.0, math.pi / 2, 0.316, 0.0],
    [0.0825, math.pi / 2, 0.0, 0.0],
    [-0.0825, -math.pi / 2, 0.384, 0.0],
    [0.0, math.pi / 2, 0.0, 0.0],
    [0.088, math.pi / 2, 0.0, 0.0],
], dtype=np.float64)

FRANKA_LIKE_QLIM = np.array([
    [-2.8973, 2.8973], [-1.7628, 1.7628], [-2.8973, 2.8973],
    [-3.0718, -0.0698], [-2.8973, 2.8973], [-0.0175, 3.7525],
    [-2.8973, 2.8973]], dtype=np.float64)

FRANKA_LIKE_QDMAX = np.array([2.175, 2.175, 2.175, 2.175, 2.61, 2.61, 2.61])

# End-effector point in the last link frame (flange 0.107 m + hand 0.143 m).
FRANKA_LIKE_TOOL = np.array([0.0, 0.0, 0.25])
# Start posture: a tucked "ready" pose inside the joint limits.
FRANKA_LIKE_READY = np.array([0.0, -0.785, 0.0, -2.356, 0.0, 1.571, 0.785])

# Body b (0..6) is rigid with link frame b+1; body 7 is the hand, rigid with
# the last link frame.  Each body's spheres sit evenly along a segment given
# in that body's frame (builder-chosen to follow the link geometry).
_BODY_SEGMENTS = [
    ((0.0, 0.0, -0.30), (0.0, 0.0, -0.10)),     # shoulder column
    ((0.0, 0.0, 0.0), (0.0, -0.15, 0.0)),       # shoulder
    ((0.0, 0.0, -0.18), (0.0, 0.0, -0.06)),     # upper arm
    ((0.0, 0.0, 0.0), (-0.0825, 0.19, 0.0)),    # elbow
    ((0.0, 0.0, -0.28), (0.0, 0.0, -0.15)),     # forearm
    ((0.0, 0.0, 0.0), (0.06, 0.0, 0.0)),        # wrist
    ((0.0, 0.0, 0.0), (0.0, 0.0, 0.107)),       # flange
]
# Hand: four spheres along the axis, four on the finger pads.
_HAND_POINTS = [
    (0.0, 0.0, 0.16), (0.0, 0.0, 0.19), (0.0, 0.0, 0.22), (0.0, 0.0, 0.25),
    (0.0, 0.05, 0.18), (0.0, -0.05, 0.18), (0.0, 0.04, 0.23), (0.0, -0.04, 0.23),
]

LAYOUT_52 = (4, 6, 6, 6, 8, 6, 8, 8)
LAYOUT_64 = (8, 8, 8, 8, 8, 8, 8, 8)


@dataclasses.dataclass
class Arm:
    dh: np.ndarray            # [d][4] f32
    q_lim: np.ndarray         # [d][2] f32
    qd_max: np.ndarray        # [d] f32
    spheres: np.ndarray       # [S][4] f32, link-frame centre + radius
    sphere_link: np.ndarray   # [S] int32, body index 0..d (d = hand)
    base: np.ndarray          # [4] f32: x, y, z, yaw
    tool: np.ndarray          # [3] f32
    n_rollouts: int
    horizon: int

    @property
    def dof(self) -> int:
        return int(self.dh.shape[0])

    @property
    def n_spheres(self) -> int:
        return int(self.spheres.shape[0])


def default_params(**over) -> dict:
    """Controller parameters.  w_dyn, buf_dyn and tau follow the paper's
    standard variant (Sec. V-A, variant M); K=1 is its M_fast setting."""
    p = dict(dt=0.02, sigma=0.3, lam=0.05, gamma=0.99, alpha_mu=1.0, iters=1,
             w_pose=1.0, w_rot=0.1, w_stop=1.0, w_joint=10.0, w_coll=5000.0,
             w_dyn=5000.0, buf_env=0.03, buf_self=0.03, buf_dyn=0.03,
             tau=3.0, prio_min=0.5, prio_max=2.0, dist_floor=1e-3,
             joint_margin=0.05, seed=0, max_obstacles=32,
             collision_mode=0, surrogate_margin=0.05,
             alpha_sigma=0.0, sigma_floor=1e-3, plan_mode=0,
             w_manip=0.0, manip_thresh=0.1, surrogate_screen=0.0, surrogate_probe=0,
             surrogate_min_drop=0.0, pair_cull=1)
    p.update(over)
    return p


def franka_like_arm(rng: np.random.Generator, layout=LAYOUT_52, base=(0, 0, 0, 0),
                    n_rollouts=64, horizon=20) -> Arm:
    """A 7-DoF arm with len(layout) bodies; layout[b] spheres on body b,
    radii U(0.04, 0.08) m."""
    centres, links = [], []
    for b, cnt in enumerate(layout):
        if b < 7:
            p0, p1 = (np.array(x) for x in _BODY_SEGMENTS[b])
            for i in range(cnt):
                f = (i + 0.5) / cnt
                centres.append(p0 + f * (p1 - p0))
                links.append(b)
        else:
            pts = _HAND_POINTS[:cnt]
            for pt in pts:
                centres.append(np.array(pt))
                links.append(7)
    radii = rng.uniform(0.04, 0.08, size=len(centres))
    sph = np.concatenate([np.array(centres), radii[:, None]], axis=1)
    return Arm(dh=FRANKA_LIKE_DH.astype(F32), q_lim=FRANKA_LIKE_QLIM.astype(F32),
               qd_max=FRANKA_LIKE_QDMAX.astype(F32), spheres=sph.astype(F32),
               sphere_link=np.array(links, dtype=np.int32),
               base=np.array(base, dtype=F32), tool=FRANKA_LIKE_TOOL.astype(F32),
               n_rollouts=int(n_rollouts), horizon=int(horizon))


def random_quaternion(rng) -> np.ndarray:
    """Uniform unit quaternion, (w, x, y, z) order, w >= 0."""
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    if q[0] < 0:
        q = -q
    return q


def start_state(rng, arm: Arm) -> np.ndarray:
    """[d][3] joint state (theta, theta_dot, theta_ddot): the ready pose
    perturbed by U(-0.2, 0.2) rad, at rest."""
    q = FRANKA_LIKE_READY[:arm.dof] + rng.uniform(-0.2, 0.2, size=arm.dof)
    st = np.zeros((arm.dof, 3))
    st[:, 0] = q
    return st.astype(F32)


def _goal_in_box(rng, lo, hi) -> np.ndarray:
    p = rng.uniform(lo, hi)
    return np.concatenate([p, random_quaternion(rng)]).astype(F32)


@dataclasses.dataclass
class Scene:
    name: str
    arms: list
    params: dict
    state: np.ndarray        # [A][d][3]
    goal: np.ndarray         # [A][7]
    obstacles: np.ndarray    # [O][4]
    obstacle_vel: np.ndarray  # [O][3]
    box_lo: np.ndarray        # obstacle / goal region
    box_hi: np.ndarray
    goal_lo: np.ndarray       # [A][3]
    goal_hi: np.ndarray
    steps: int
    seed: int

    @property
    def n_arms(self) -> int:
        return len(self.arms)

    def rollout_steps(self) -> int:
        return sum(a.n_rollouts * a.horizon for a in self.arms) * int(self.params["iters"])


def _moving_obstacles(rng, n, lo, hi, rmin=0.05, rmax=0.10):
    pos = rng.uniform(lo, hi, size=(n, 3))
    rad = rng.uniform(rmin, rmax, size=(n, 1))
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    speed = rng.uniform(0.05, 0.3, size=(n, 1))
    return (np.concatenate([pos, rad], axis=1).astype(F32), (d * speed).astype(F32))


def make_scene(config: int, seed: int | None = None, **param_over) -> Scene:
    """The five benchmark scenes (1-arm smoke, 2 facing arms, 4 uneven arms,
    4 arms for the learned distance, 8 arms in two rows)."""
    seed = {1: 1001, 2: 1002, 3: 1003, 4: 1004, 5: 1005}[config] if seed is None else seed
    rng = np.random.default_rng(seed)
    params = default_params(seed=seed, **param_over)
    layout = LAYOUT_64 if config == 5 else LAYOUT_52
    sphere_rng = np.random.default_rng(seed + 7)
    if config == 1:
        bases = [(0.0, 0.0, 0.0, 0.0)]
        nh = [(64, 20)]
        steps = 1
    elif config == 2:
        bases = [(-0.4, 0.0, 0.0, 0.0), (0.4, 0.0, 0.0, math.pi)]
        nh = [(512, 30)] * 2
        steps = 200
    elif config in (3, 4):
        c = 0.6
        bases = [(-c, -c, 0.0, math.pi / 4), (c, -c, 0.0, 3 * math.pi / 4),
                 (c, c, 0.0, -3 * math.pi / 4), (-c, c, 0.0, -math.pi / 4)]
        nh = [(256, 20), (512, 30), (768, 30), (1024, 40)] if config == 3 else [(1024, 30)] * 4
        steps = 500 if config == 3 else 10000
        if config == 4:
            params["collision_mode"] = param_over.get("collision_mode", 1)
    elif config == 5:
        # Rows 1.0 m apart, so that the perturbed ready poses of facing arms
        # start clear of each other (0.18 m at the closest pair).
        xs = (-0.75, -0.25, 0.25, 0.75)
        bases = [(x, -0.5, 0.0, math.pi / 2) for x in xs] + [(x, 0.5, 0.0, -math.pi / 2) for x in xs]
        nh = [(4096, 40)] * 8
        steps = 1000
        params["collision_mode"] = param_over.get("collision_mode", 1)
    else:
        raise ValueError(config)
    # One arm template per scene (same radii on every arm, as identical robots).
    template = franka_like_arm(sphere_rng, layout)
    arms = []
    for b, (n, h) in zip(bases, nh):
        arms.append(dataclasses.replace(template, base=np.array(b, dtype=F32),
                                        n_rollouts=n, horizon=h))
    state = np.stack([start_state(rng, a) for a in arms])
    A = len(arms)
    goal_lo = np.zeros((A, 3))
    goal_hi = np.zeros((A, 3))
    for i, a in enumerate(arms):
        bx, by = float(a.base[0]), float(a.base[1])
        if config == 1:
            goal_lo[i], goal_hi[i] = (bx + 0.3, by - 0.3, 0.2), (bx + 0.6, by + 0.3, 0.6)
        elif config == 2:
            goal_lo[i], goal_hi[i] = (-0.15, -0.3, 0.2), (0.15, 0.3, 0.6)
        elif config in (3, 4):
            goal_lo[i], goal_hi[i] = (-0.3, -0.3, 0.2), (0.3, 0.3, 0.6)
        else:
            goal_lo[i], goal_hi[i] = (bx - 0.25, -0.2, 0.2), (bx + 0.25, 0.2, 0.6)
    goal = np.stack([_goal_in_box(rng, goal_lo[i], goal_hi[i]) for i in range(A)])
    if config == 1:
        shoulder = np.array([0.0, 0.0, 0.333])
        mid = 0.5 * (shoulder + goal[0, :3].astype(np.float64))
        obstacles = np.array([[*mid, 0.08]], dtype=F32)
        vel = np.zeros((1, 3), dtype=F32)
        box_lo, box_hi = np.array([-1.0, -1.0, 0.0]), np.array([1.0, 1.0, 1.0])
    elif config == 2:
        obstacles = np.zeros((0, 4), dtype=F32)
        vel = np.zeros((0, 3), dtype=F32)
        box_lo, box_hi = np.array([-0.6, -0.6, 0.0]), np.array([0.6, 0.6, 0.9])
    elif config in (3, 4):
        box_lo, box_hi = np.array([-0.6, -0.6, 0.1]), np.array([0.6, 0.6, 0.8])
        obstacles, vel = _moving_obstacles(rng, 8, box_lo, box_hi)
    else:
        box_lo, box_hi = np.array([-1.0, -0.45, 0.1]), np.array([1.0, 0.45, 0.8])
        obstacles, vel = _moving_obstacles(rng, 20, box_lo, box_hi)
    return Scene(name=f"cfg{config}", arms=arms, params=params, state=state, goal=goal,
                 obstacles=obstacles, obstacle_vel=vel, box_lo=box_lo, box_hi=box_hi,
                 goal_lo=goal_lo, goal_hi=goal_hi, steps=steps, seed=seed)


def move_obstacles(scene: Scene, dt: float) -> None:
    """Advance obstacle centres along straight lines, reflecting off the
    region's walls (positions are updated between control steps only)."""
    if scene.obstacles.shape[0] == 0:
        return
    p = scene.obstacles[:, :3].astype(np.float64) + dt * scene.obstacle_vel.astype(np.float64)
    v = scene.obstacle_vel.astype(np.float64)
    lo, hi = scene.box_lo, scene.box_hi
    over, under = p > hi, p < lo
    p = np.where(over, 2 * hi - p, p)
    p = np.where(under, 2 * lo - p, p)
    v = np.where(over | under, -v, v)
    scene.obstacles[:, :3] = p.astype(F32)
    scene.obstacle_vel[:] = v.astype(F32)


def reset_goals(scene: Scene, rng, dist_to_goal, age, tol=0.05, max_age=50) -> np.ndarray:
    """Reaching-task goal resets: a new goal once an arm is within `tol` of
    its goal or after `max_age` control steps.  Returns the reset mask."""
    mask = (np.asarray(dist_to_goal) < tol) | (np.asarray(age) >= max_age)
    for i in np.nonzero(mask)[0]:
        scene.goal[i] = _goal_in_box(rng, scene.goal_lo[i], scene.goal_hi[i])
    return mask


def random_plan_inputs(rng, arm: Arm, n, scale=1.0):
    """Random joint configurations uniform within the joint limits, [n][d]."""
    lo, hi = arm.q_lim[:, 0].astype(np.float64), arm.q_lim[:, 1].astype(np.float64)
    return (lo + (hi - lo) * rng.uniform(size=(n, arm.dof)) * scale).astype(F32)
