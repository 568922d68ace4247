"""Pins of the FP64 CPU oracle against facts fixed by the paper and by
mathematics: published known-answer vectors, closed forms, invariants,
special cases that reduce to textbook or library routines, and brute force.
None of these re-type the oracle's own formulas."""
import math
import os

import numpy as np
import pytest
from scipy import stats
from scipy.spatial.distance import cdist
from scipy.spatial.transform import Rotation

from paper_2602_10114_amd import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _arm(layout=scenes.LAYOUT_52, seed=3, **kw):
    return scenes.franka_like_arm(np.random.default_rng(seed), layout, **kw)


# ----------------------------------------------------------------- noise
def test_philox_known_answers(orc):
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = orc.philox(v[0:4], v[4:6])
        assert list(out) == v[6:10]


def test_normals_distribution(orc):
    """Kolmogorov-Smirnov against scipy's normal CDF, moments within 5 sigma
    of their sampling error, and no correlation between joints or steps."""
    d, n = 7, 3000
    z = np.array([orc.normals(1234, 1, 5, 0, i, h, d) for i in range(n) for h in (0, 3)])
    flat = z.ravel()
    m = flat.size
    assert abs(flat.mean()) < 5 / math.sqrt(m)
    assert abs(flat.var() - 1) < 5 * math.sqrt(2 / m)
    assert stats.kstest(flat, "norm").pvalue > 1e-3
    c = np.corrcoef(z.T)
    assert np.abs(c - np.eye(d)).max() < 5 / math.sqrt(z.shape[0])


def test_normals_distinct_streams(orc):
    """Different arm, step, iteration, rollout or horizon index give
    different draws; the same index gives the same draw."""
    base = orc.normals(7, 0, 0, 0, 0, 0, 7)
    assert np.array_equal(base, orc.normals(7, 0, 0, 0, 0, 0, 7))
    for args in [(7, 1, 0, 0, 0, 0), (7, 0, 1, 0, 0, 0), (7, 0, 0, 1, 0, 0),
                 (7, 0, 0, 0, 1, 0), (7, 0, 0, 0, 0, 1), (8, 0, 0, 0, 0, 0)]:
        assert not np.allclose(base, orc.normals(*args, 7))


# ------------------------------------------------------------- dynamics
def test_integrate_constant_acceleration_closed_form(orc):
    rng = np.random.default_rng(0)
    d, H, dt = 7, 25, 0.02
    q0, qd0, a = rng.normal(size=d), rng.normal(size=d), rng.normal(size=d)
    q, qd = orc.integrate(q0, qd0, np.tile(a, (H, 1)), dt)
    h = np.arange(1, H + 1)[:, None]
    np.testing.assert_allclose(qd, qd0 + a * dt * h, atol=1e-12)
    np.testing.assert_allclose(q, q0 + h * dt * qd0 + a * dt * dt * h * (h + 1) / 2, atol=1e-12)


# ------------------------------------------------------------ kinematics
def _two_link():
    arm = _arm()
    dh = np.zeros((2, 4), np.float32)
    dh[0] = (0, 0, 0.5, 0)
    dh[1] = (0.3, np.float32(math.pi / 2), 0.1, 0)
    return scenes.Arm(dh=dh, q_lim=arm.q_lim[:2], qd_max=arm.qd_max[:2],
                      spheres=np.array([[0, 0, 0, 0.05], [0.1, 0, 0, 0.05]], np.float32),
                      sphere_link=np.array([0, 1], np.int32), base=np.zeros(4, np.float32),
                      tool=np.zeros(3, np.float32), n_rollouts=1, horizon=1)


def _golden_fk():
    out = {}
    for l in open(os.path.join(GOLDEN, "fk_hand_derived.txt")):
        if l.strip() and not l.startswith("#"):
            f = l.split()
            out[f[0]] = np.array([float(x) for x in f[1:]])
    return out


def test_fk_hand_derived_two_link(orc):
    g = _golden_fk()
    oa = orc.make_arm(_two_link())
    for name in ("two_link_q00", "two_link_q90"):
        v = g[name]
        fr = orc.fk(oa, v[0:2])
        # alpha = pi/2 is rounded to FP32 in the table, hence 1e-7.
        np.testing.assert_allclose(fr[1][:3, 3], v[2:5], atol=1e-7)
        np.testing.assert_allclose(fr[1][:3, :3].ravel(), v[5:14], atol=1e-7)


def test_fk_franka_like_zero_pose(orc):
    g = _golden_fk()
    arm = _arm()
    oa = orc.make_arm(arm)
    fr = orc.fk(oa, np.zeros(7))
    np.testing.assert_allclose(fr[6][:3, 3], g["franka_like_q0_frame7"], atol=1e-6)
    flange = fr[6][:3, 3] + 0.107 * fr[6][:3, 2]
    np.testing.assert_allclose(flange, g["franka_like_q0_flange"], atol=1e-6)


def test_ee_pose_franka_like_zero_pose_with_tool(orc):
    """The end-effector point (Eq. 5's pose term) at the classic zero pose:
    the tool's 0.25 m along the last frame's z axis, which points down, and
    the last frame's orientation diag(1, -1, -1), both multiplied out by hand
    (golden file)."""
    g = _golden_fk()["franka_like_q0_ee"]
    arm = _arm()
    np.testing.assert_array_equal(arm.tool, np.array([0, 0, 0.25], np.float32))
    T = orc.ee_pose(orc.make_arm(arm), np.zeros(7))
    np.testing.assert_allclose(T[:3, 3], g[0:3], atol=1e-6)
    np.testing.assert_allclose(T[:3, :3].ravel(), g[3:12], atol=1e-6)
    np.testing.assert_allclose(T[3], [0, 0, 0, 1])


def _two_link_offsets(p):
    """The two-link arm with one sphere on each body and the tool, all at the
    same offset p off the frames' axes."""
    arm = _two_link()
    sph = np.array([[p[0], p[1], p[2], 0.05], [p[0], p[1], p[2], 0.07]], np.float32)
    return scenes.Arm(**{**arm.__dict__, "spheres": sph, "tool": np.array(p, np.float32)})


def test_offsets_off_the_axes_rotate_with_their_frame(orc):
    """A sphere centre and the tool point at an offset that is not along any
    frame axis, on frames whose rotations are not symmetric (golden file, by
    hand): catches a transposed rotation, which the norm-preservation pin
    cannot see."""
    g = _golden_fk()
    arm = _two_link_offsets((0.1, 0.2, 0.3))
    oa = orc.make_arm(arm)
    q = np.array([math.pi / 2, 0.0])
    sph = orc.spheres(oa, q)
    np.testing.assert_allclose(sph[0, :3], g["two_link_q90_offset_on_frame1"], atol=1e-7)
    np.testing.assert_allclose(sph[1, :3], g["two_link_q90_offset_on_frame2"], atol=1e-7)
    assert sph[0, 3] == float(np.float32(0.05)) and sph[1, 3] == float(np.float32(0.07))
    # the tool point rides on the last frame (frame 2 here)
    T = orc.ee_pose(oa, q)
    np.testing.assert_allclose(T[:3, 3], g["two_link_q90_offset_on_frame2"], atol=1e-7)


def test_fk_orthonormal_and_spacing(orc):
    arm = _arm()
    oa = orc.make_arm(arm)
    rng = np.random.default_rng(1)
    dh = arm.dh.astype(np.float64)
    for _ in range(20):
        q = scenes.random_plan_inputs(rng, arm, 1)[0].astype(np.float64)
        fr = orc.fk(oa, q)
        for k in range(8):
            R = fr[k][:3, :3]
            np.testing.assert_allclose(R.T @ R, np.eye(3), atol=1e-12)
            assert abs(np.linalg.det(R) - 1) < 1e-12
            np.testing.assert_allclose(fr[k][3], [0, 0, 0, 1])
        # origin of frame k+1 sits sqrt(a^2 + d^2) from frame k's origin
        for k in range(6):
            gap = np.linalg.norm(fr[k + 1][:3, 3] - fr[k][:3, 3])
            assert abs(gap - math.hypot(dh[k + 1, 0], dh[k + 1, 2])) < 1e-12


def test_fk_planar_chain_textbook(orc):
    """All twists, offsets and d zero: joint origins follow
    x_k = sum_i a_i cos(q_1 + ... + q_{i-1}), y likewise with sin."""
    a = np.array([0.0, 0.4, 0.3, 0.25, 0.2], np.float32)
    dh = np.zeros((5, 4), np.float32)
    dh[:, 0] = a
    arm = scenes.Arm(dh=dh, q_lim=np.zeros((5, 2), np.float32), qd_max=np.ones(5, np.float32),
                     spheres=np.zeros((1, 4), np.float32), sphere_link=np.zeros(1, np.int32),
                     base=np.zeros(4, np.float32), tool=np.zeros(3, np.float32),
                     n_rollouts=1, horizon=1)
    oa = orc.make_arm(arm)
    q = np.array([0.3, -0.7, 1.1, 0.2, -0.4])
    fr = orc.fk(oa, q)
    ang = np.concatenate([[0.0], np.cumsum(q)])
    for k in range(5):
        x = sum(float(a[i]) * math.cos(ang[i]) for i in range(k + 1))
        y = sum(float(a[i]) * math.sin(ang[i]) for i in range(k + 1))
        np.testing.assert_allclose(fr[k][:2, 3], [x, y], atol=1e-12)
        assert abs(math.atan2(fr[k][1, 0], fr[k][0, 0]) -
                   math.atan2(math.sin(ang[k + 1]), math.cos(ang[k + 1]))) < 1e-12


def test_fk_base_yaw_equals_first_joint(orc):
    arm = _arm()
    rng = np.random.default_rng(2)
    q = scenes.random_plan_inputs(rng, arm, 1)[0].astype(np.float64)
    psi = 0.7
    yawed = scenes.Arm(**{**arm.__dict__, "base": np.array([0.1, -0.2, 0.05, psi], np.float32)})
    plain = scenes.Arm(**{**arm.__dict__, "base": np.array([0.1, -0.2, 0.05, 0.0], np.float32)})
    q2 = q.copy()
    q2[0] += float(np.float32(psi))
    np.testing.assert_allclose(orc.fk(orc.make_arm(yawed), q), orc.fk(orc.make_arm(plain), q2), atol=1e-12)


def test_spheres_keep_body_offsets(orc):
    arm = _arm()
    oa = orc.make_arm(arm)
    q = scenes.random_plan_inputs(np.random.default_rng(4), arm, 1)[0]
    fr = orc.fk(oa, q)
    sph = orc.spheres(oa, q)
    for s in range(arm.n_spheres):
        t = fr[arm.sphere_link[s]][:3, 3]
        assert abs(np.linalg.norm(sph[s, :3] - t) - np.linalg.norm(arm.spheres[s, :3].astype(np.float64))) < 1e-12
        assert sph[s, 3] == float(arm.spheres[s, 3])


# ------------------------------------------------------------- distances
def test_two_sphere_closed_form(orc):
    assert abs(orc.sphere_rho([0, 0, 0, 0.1], [0.5, 0, 0, 0.2]) - 0.2) < 1e-15
    assert abs(orc.sphere_rho([1, 2, 3, 0.3], [1, 2, 3.1, 0.2]) + 0.4) < 1e-12


def test_set_distance_brute_force_and_invariance(orc):
    rng = np.random.default_rng(5)
    for _ in range(50):
        na, nb = rng.integers(1, 5, size=2)
        A = np.concatenate([rng.normal(size=(na, 3)), rng.uniform(0.01, 0.2, (na, 1))], 1)
        B = np.concatenate([rng.normal(size=(nb, 3)), rng.uniform(0.01, 0.2, (nb, 1))], 1)
        brute = (cdist(A[:, :3], B[:, :3]) - A[:, 3:4] - B[:, 3][None, :]).min()
        assert abs(orc.rho_sets(A, B) - brute) < 1e-12
        assert abs(orc.rho_sets(B, A) - brute) < 1e-12
        R = Rotation.random(random_state=int(rng.integers(1 << 30))).as_matrix()
        t = rng.normal(size=3)
        A2, B2 = A.copy(), B.copy()
        A2[:, :3] = A[:, :3] @ R.T + t
        B2[:, :3] = B[:, :3] @ R.T + t
        assert abs(orc.rho_sets(A2, B2) - brute) < 1e-12


def test_self_pairs_skip_adjacent_bodies(orc):
    c = np.array([[0, 0, 0, 0.1], [0.05, 0, 0, 0.1], [0.5, 0, 0, 0.1]], float)
    # bodies 0,1 overlap but are adjacent; the surfaces of 0 and 2 are 0.3 apart.
    assert abs(orc.rho_self(c, [0, 1, 2]) - 0.3) < 1e-12
    assert orc.rho_self(c, [0, 1, 1]) == math.inf


def test_hinge_special_values(orc):
    B = 0.03
    assert orc.hinge(B, B) == 0.0 and orc.hinge(0.5, B) == 0.0
    assert orc.hinge(0.0, B) == 1.0 and orc.hinge(-0.2, B) == 1.0
    assert abs(orc.hinge(B / 2, B) - 0.5) < 1e-15
    assert orc.hinge(math.inf, B) == 0.0


# --------------------------------------------------------------- costs
def test_pose_rotation_term_matches_quaternion_inner_product(orc):
    """(3 - tr(Rg^T R)) / 4 = 1 - <q, g>^2, with the quaternions taken from
    scipy's independent rotation code."""
    rng = np.random.default_rng(6)
    for _ in range(20):
        Rm = Rotation.random(random_state=int(rng.integers(1 << 30)))
        T = np.eye(4)
        T[:3, :3] = Rm.as_matrix()
        T[:3, 3] = rng.normal(size=3)
        g = np.concatenate([T[:3, 3] + [0.3, 0, 0], scenes.random_quaternion(rng)])
        qx, qy, qz, qw = Rm.as_quat()
        ip = qw * g[3] + qx * g[4] + qy * g[5] + qz * g[6]
        expected = 0.3 + 0.1 * (1 - ip * ip)
        assert abs(orc.pose_cost(T, g, 0.1) - expected) < 1e-12
    # reached goal -> zero
    T = np.eye(4)
    T[:3, :3] = Rotation.from_euler("xyz", [0.2, -0.4, 1.0]).as_matrix()
    x, y, z, w = Rotation.from_matrix(T[:3, :3]).as_quat()
    assert abs(orc.pose_cost(T, [0, 0, 0, w, x, y, z], 0.1)) < 1e-14


def test_quat_rotation_matches_scipy(orc):
    rng = np.random.default_rng(7)
    for _ in range(10):
        q = scenes.random_quaternion(rng)
        R = orc.quat_to_rot(q * 1.7)  # normalised internally
        np.testing.assert_allclose(R, Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix(), atol=1e-12)


def test_stop_and_joint_special_cases(orc):
    arm = _arm()
    oa = orc.make_arm(arm)
    H = 10
    qd = np.array([0.5, -0.5, 0, 0, 0, 0, 0.1])
    # last step: nothing may move
    assert abs(orc.stop_cost(oa, H, H - 1, qd) - np.abs(qd).sum()) < 1e-14
    # first step: limits are 0.9 qd_max > |qd|
    assert orc.stop_cost(oa, H, 0, qd) == 0.0
    mid = arm.q_lim.astype(np.float64).mean(1)
    mid[3] = -1.5
    assert orc.joint_cost(oa, mid, 0.05) == 0.0
    q = mid.copy()
    q[0] = float(arm.q_lim[0, 0]) - 0.1
    assert abs(orc.joint_cost(oa, q, 0.05) - 0.15) < 1e-12


def test_priority_properties(orc):
    assert orc.priority(0.4, 0.1, 0.0, 1e-3, 0.5, 2.0) == 1.0
    for da, db in [(0.3, 0.2), (0.05, 0.4), (0.7, 0.69)]:
        p1 = orc.priority(da, db, 3.0, 1e-3, 0.0, 1e300)
        p2 = orc.priority(db, da, 3.0, 1e-3, 0.0, 1e300)
        assert abs(p1 * p2 - 1) < 1e-12
        # the arm nearer its goal carries the smaller weight
        assert (p1 < 1) == (da < db)
    assert orc.priority(0.9, 0.1, 3.0, 1e-3, 0.5, 2.0) == 2.0
    assert orc.priority(0.0, 0.0, 3.0, 1e-3, 0.5, 2.0) == 1.0


# -------------------------------------------------------------- update
def test_weights_properties(orc):
    rng = np.random.default_rng(8)
    C = rng.normal(size=200) * 3 + 1e4
    w = orc.weights(C, 0.05)
    assert abs(w.sum() - 1) < 1e-12
    np.testing.assert_allclose(orc.weights(C + 123.0, 0.05), w, rtol=1e-9, atol=1e-300)
    np.testing.assert_allclose(orc.weights(C, 1e30), np.full(200, 1 / 200), rtol=1e-12)
    w0 = orc.weights(C, 1e-30)
    assert w0[np.argmin(C)] == 1.0 and w0.sum() == 1.0


def test_update_limits(orc):
    rng = np.random.default_rng(9)
    N, H, d = 64, 6, 7
    U = rng.normal(size=(N, H, d))
    C = rng.uniform(size=N)
    np.testing.assert_allclose(orc.weighted_mean(orc.weights(C, 1e30), U), U.mean(0), atol=1e-12)
    np.testing.assert_allclose(orc.weighted_mean(orc.weights(C, 1e-30), U), U[np.argmin(C)], atol=0)
    np.testing.assert_allclose(orc.weighted_mean(orc.weights(C[:1], 0.05), U[:1]), U[0], atol=0)
    mu = rng.normal(size=(H, d))
    np.testing.assert_array_equal(orc.ema(mu, U[0], 0.0), mu)
    np.testing.assert_array_equal(orc.ema(mu, U[0], 1.0), U[0])
    s = mu
    for _ in range(H):
        s = orc.shift(s)
    np.testing.assert_array_equal(s, np.tile(mu[-1], (H, 1)))
    assert orc.argmin(np.array([3.0, 1.0, 1.0, 2.0])) == 1


def test_weighted_covariance_limits(orc):
    """Eq. 3's covariance: uniform weights give numpy's population covariance
    of the samples; one dominant rollout gives zero; a pair with weights
    (p, 1-p) gives p(1-p) (a-b)(a-b)^T."""
    rng = np.random.default_rng(31)
    N, H, d = 200, 3, 7
    U = rng.normal(size=(N, H, d)) * rng.uniform(0.1, 2.0, size=d)
    w = np.full(N, 1.0 / N)
    S = orc.weighted_cov(w, U, orc.weighted_mean(w, U))
    for h in range(H):
        np.testing.assert_allclose(S[h], np.cov(U[:, h, :].T, bias=True), atol=1e-12)
    w1 = np.zeros(N)
    w1[17] = 1.0
    np.testing.assert_allclose(orc.weighted_cov(w1, U, orc.weighted_mean(w1, U)), 0.0, atol=1e-15)
    p = 0.3
    w2 = np.zeros(N)
    w2[3], w2[8] = p, 1 - p
    dlt = U[3] - U[8]
    S2 = orc.weighted_cov(w2, U, orc.weighted_mean(w2, U))
    for h in range(H):
        np.testing.assert_allclose(S2[h], p * (1 - p) * np.outer(dlt[h], dlt[h]), atol=1e-12)


def test_cholesky_floor(orc):
    """Factor of an SPD matrix equals numpy's; a singular matrix gets its
    pivots floored (L L^T = S + the floor on the null direction)."""
    rng = np.random.default_rng(32)
    M = rng.normal(size=(7, 7))
    S = M @ M.T + 0.1 * np.eye(7)
    np.testing.assert_allclose(orc.cholesky_floor(S, 1e-12), np.linalg.cholesky(S), atol=1e-12)
    v = rng.normal(size=7)
    Z = np.outer(v, v)                      # rank one: pivots 2..7 vanish
    L = orc.cholesky_floor(Z, 1e-6)
    assert abs(L[0, 0] - abs(v[0])) < 1e-12
    np.testing.assert_allclose(np.diag(L)[1:], 1e-3, rtol=1e-9)
    np.testing.assert_allclose((L @ L.T)[:, 0], Z[:, 0], atol=1e-12)


def test_covariance_adaptation_in_the_controller(orc):
    """alpha_Sigma = 0 keeps Sigma = sigma^2 I; alpha_Sigma = 1 at infinite
    temperature makes Sigma_h the population covariance of the step's
    controls (numpy), its factor numpy's Cholesky; the next step's noise then
    has that covariance (sampling pin over 4096 rollouts, 5 standard errors)."""
    sc = scenes.make_scene(1)
    sc.arms[0].n_rollouts = 4096
    sc.arms[0].horizon = 4
    sig = float(np.float32(0.3))
    c0 = orc.Controller(sc.arms, {**sc.params, "alpha_sigma": 0.0})
    c0.step(sc.state, sc.goal, sc.obstacles)
    S0, L0 = c0.sigma(0)
    for h in range(4):
        np.testing.assert_array_equal(S0[h], sig * sig * np.eye(7))
        np.testing.assert_array_equal(L0[h], sig * np.eye(7))
    ctl = orc.Controller(sc.arms, {**sc.params, "alpha_sigma": 1.0, "lam": 1e30})
    ctl.step(sc.state, sc.goal, sc.obstacles)
    eps = ctl.noise(0)                       # [N][H][d]; U = mu + eps with mu = 0 here
    S, L = ctl.sigma(0)
    for h in range(4):
        ref = np.cov(eps[:, h, :].T, bias=True)
        np.testing.assert_allclose(S[h], ref, atol=1e-12)
        np.testing.assert_allclose(L[h], np.linalg.cholesky(ref), atol=1e-10)
    ctl.step(sc.state, sc.goal, sc.obstacles)
    eps2 = ctl.noise(0)
    for h in range(3):                       # step h uses Sigma_{h+1} after the shift
        Sh = S[h + 1]
        emp = np.cov(eps2[:, h, :].T, bias=True)
        se = np.sqrt((np.outer(np.diag(Sh), np.diag(Sh)) + Sh ** 2) / 4096)
        assert np.all(np.abs(emp - Sh) < 5 * se + 1e-12)


def test_static_plans_are_current_spheres(orc):
    """plan_mode 1 (the S_d ablation): every published step holds the
    spheres of the arm's current configuration."""
    sc = scenes.make_scene(2, plan_mode=1)
    for a in sc.arms:
        a.n_rollouts = 16
    ctl = orc.Controller(sc.arms, sc.params)
    ctl.step(sc.state, sc.goal, sc.obstacles)
    ctl.share_plans()
    for a in range(2):
        p, pq, _, valid = ctl.plan(a, 0)
        ref = orc.spheres(ctl.arms[a], sc.state[a, :, 0].astype(np.float64))
        assert valid == 1
        for h in range(sc.arms[a].horizon):
            np.testing.assert_allclose(p[h, :sc.arms[a].n_spheres], ref, atol=1e-12)
            np.testing.assert_allclose(pq[h], sc.state[a, :, 0], atol=1e-7)


def _fd_jacobian(orc, oa, q, h=1e-6):
    """Jacobian by central differences of the forward kinematics: linear rows
    from the end-effector point, angular rows from R(q+h) R(q-h)^T."""
    J = np.zeros((6, 7))
    for k in range(7):
        qp, qm = q.copy(), q.copy()
        qp[k] += h
        qm[k] -= h
        Tp, Tm = orc.ee_pose(oa, qp), orc.ee_pose(oa, qm)
        J[:3, k] = (Tp[:3, 3] - Tm[:3, 3]) / (2 * h)
        W = Tp[:3, :3] @ Tm[:3, :3].T
        J[3:, k] = np.array([W[2, 1] - W[1, 2], W[0, 2] - W[2, 0], W[1, 0] - W[0, 1]]) / (4 * h)
    return J


def test_jacobian_and_manipulability(orc):
    """C_manip's Jacobian against central differences of the kinematics, its
    cost against numpy's determinant; the zero configuration (joint axes 1
    and 3, 5 and 7 aligned) is singular; the threshold limits."""
    oa = orc.make_arm(_arm())
    rng = np.random.default_rng(41)
    lo, hi = _arm().q_lim[:, 0].astype(np.float64), _arm().q_lim[:, 1].astype(np.float64)
    for _ in range(5):
        q = rng.uniform(lo, hi)
        J = orc.jacobian(oa, q)
        Jf = _fd_jacobian(orc, oa, q)
        np.testing.assert_allclose(J, Jf, atol=1e-7)
        m = np.sqrt(max(np.linalg.det(Jf @ Jf.T), 0.0))
        assert abs(orc.manip_cost(oa, q, 0.1) - max(0.0, 1.0 - m / 0.1)) < 1e-6
        assert orc.manip_cost(oa, q, 1e-9) == 0.0
    assert abs(orc.manip_cost(oa, np.zeros(7), 0.1) - 1.0) < 1e-6


def test_total_cost_geometric(orc):
    # constant stage cost c: sum_{h<H} gamma^h c = c (1 - gamma^H) / (1 - gamma)
    g, H = 0.99, 30
    assert abs(orc.total_cost(np.full(H, 2.5), g) - 2.5 * (1 - g ** H) / (1 - g)) < 1e-12
    assert orc.total_cost(np.arange(5.0), 1.0) == 10.0


# --------------------------------------------------------- full controller
def _scene_controller(orc, cfg, **over):
    sc = scenes.make_scene(cfg, **over)
    return sc, orc.Controller(sc.arms, sc.params)


def test_step_act_consistency_at_zero_temperature(orc):
    """lambda -> 0 with alpha_mu = 1: the new mean's first step is the
    executed command (both pick the minimum-cost rollout)."""
    sc, ctl = _scene_controller(orc, 1, lam=1e-30)
    u = ctl.step(sc.state, sc.goal, sc.obstacles)
    mu = ctl.mean(0)
    np.testing.assert_allclose(mu[0], u[0], atol=1e-15)


def test_step_costs_match_stage_function(orc):
    """The controller's stage costs equal the stage function applied to the
    rollouts rebuilt from its own noise (integration + FK done here through
    the primitive functions)."""
    sc, ctl = _scene_controller(orc, 1)
    arm = sc.arms[0]
    arm.n_rollouts = 8
    sc.arms[0] = arm
    ctl = orc.Controller(sc.arms, sc.params)
    ctl.step(sc.state, sc.goal, sc.obstacles)
    eps = ctl.noise(0)[:8, :arm.horizon]
    tot, st, w = ctl.costs(0)
    oa = orc.make_arm(arm)
    H, d = arm.horizon, arm.dof
    q0 = sc.state[0, :, 0].astype(np.float64)
    qd0 = sc.state[0, :, 1].astype(np.float64)
    qs, qds, sphs = [], [], []
    for n in range(8):
        q, qd = orc.integrate(q0, qd0, eps[n], float(np.float32(0.02)))
        qs.append(q)
        qds.append(qd)
        sphs.append(np.stack([orc.spheres(oa, q[h]) for h in range(H)]))
    prm = orc.make_params(sc.params)
    stage = orc.stage_costs_batch(oa, prm, np.stack(qs), np.stack(qds), np.stack(sphs), sc.goal[0],
                                  sc.obstacles, np.zeros((0,)), [], [], [], [])
    np.testing.assert_allclose(stage, st[:H, :8], rtol=1e-12)
    for n in range(8):
        assert abs(orc.total_cost(stage[:, n], float(np.float32(0.99))) - tot[n]) < 1e-9


def test_unpublished_neighbours_are_ignored(orc):
    """Without a publish, the second arm's plan never enters the first arm's
    cost: the costs equal those of a run where w_dyn = 0."""
    sc, ctl = _scene_controller(orc, 2)
    for a in sc.arms:
        a.n_rollouts = 16
        a.horizon = 8
    ctl = orc.Controller(sc.arms, sc.params)
    ctl0 = orc.Controller(sc.arms, {**sc.params, "w_dyn": 0.0})
    for _ in range(2):
        ctl.step(sc.state, sc.goal, sc.obstacles)
        ctl0.step(sc.state, sc.goal, sc.obstacles)
    np.testing.assert_array_equal(ctl.costs(0)[0], ctl0.costs(0)[0])
    # after a publish the plans do enter (the arms start 1 cm apart)
    ctl.share_plans()
    ctl0.share_plans()
    ctl.step(sc.state, sc.goal, sc.obstacles)
    ctl0.step(sc.state, sc.goal, sc.obstacles)
    assert np.any(ctl.costs(0)[0] != ctl0.costs(0)[0])
    assert ctl.alpha()[0][0, 1] > 0


def test_cost_weights_scale_linearly(orc):
    sc = scenes.make_scene(2)
    arm = sc.arms[0]
    oa = orc.make_arm(arm)
    rng = np.random.default_rng(10)
    q = scenes.random_plan_inputs(rng, arm, 6).reshape(2, 3, 7).astype(np.float64)
    qd = rng.normal(size=q.shape)
    sph = np.stack([[orc.spheres(oa, q[n, h]) for h in range(3)] for n in range(2)])
    other = orc.make_arm(sc.arms[1])
    plan = np.stack([orc.spheres(other, q[1, h]) for h in range(3)])[None]
    args = (q, qd, sph, sc.goal[0], np.array([[0.2, 0, 0.4, 0.1]]), plan, [52], [3], [1], [1.3])
    p1 = orc.make_params(sc.params)
    over = {k: sc.params[k] * 3 for k in ("w_pose", "w_stop", "w_joint", "w_coll", "w_dyn")}
    p3 = orc.make_params({**sc.params, **over})
    c1 = orc.stage_costs_batch(oa, p1, *args)
    c3 = orc.stage_costs_batch(oa, p3, *args)
    np.testing.assert_allclose(c3, 3 * c1, rtol=1e-12)


def test_pair_count_formula(orc):
    assert orc.pair_count(40, 4096, 64, [64] * 7) == 40 * 4096 * 64 * 448


# --------------------------------------------------- learned arm-pair part
def test_arm_pair_rho_is_set_distance(orc):
    sc = scenes.make_scene(2)
    a, b = (orc.make_arm(x) for x in sc.arms)
    rng = np.random.default_rng(11)
    for _ in range(5):
        qa, qb = (scenes.random_plan_inputs(rng, sc.arms[0], 1)[0] for _ in range(2))
        r = orc.arm_pair_rho(a, qa, b, qb)
        sa, sb = orc.spheres(a, qa), orc.spheres(b, qb)
        brute = (cdist(sa[:, :3], sb[:, :3]) - sa[:, 3:4] - sb[:, 3][None, :]).min()
        assert abs(r - brute) < 1e-12
        assert abs(orc.arm_pair_rho(b, qb, a, qa) - r) < 1e-12


def test_mlp_forward_hand_computed(orc):
    # 2 -> 2 -> 1: W0 = [[1, -1], [2, 0.5]], b0 = [0, -1]; W1 = [[1, 3]], b1 = [0.5]
    params = np.array([1, -1, 2, 0.5, 0, -1, 1, 3, 0.5], float)
    x = np.array([[1.0, 2.0], [-1.0, 0.0]])
    # x0: z = [-1, 2] -> relu [0, 2] -> 6.5; x1: z = [-1, -3] -> 0 -> 0.5
    np.testing.assert_allclose(orc.mlp_forward([2, 2, 1], params, x)[:, 0], [6.5, 0.5])


def test_mlp_gradient_finite_difference(orc):
    widths = [5, 7, 6, 1]
    rng = np.random.default_rng(12)
    n = orc.mlp_param_count(widths)
    p = rng.normal(size=n) * 0.5
    x = rng.normal(size=(9, 5))
    t = rng.normal(size=9)
    loss, g = orc.mlp_loss_grad(widths, p, x, t, 4.0)
    h = 1e-6
    for i in range(n):
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (orc.mlp_loss_grad(widths, pp, x, t, 4.0)[0] - orc.mlp_loss_grad(widths, pm, x, t, 4.0)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i]))
    y = orc.mlp_forward(widths, p, x)[:, 0]
    e = y - t
    assert abs(loss - np.mean(e * e + 4.0 * np.maximum(e, 0) ** 2)) < 1e-12


def test_mlp_near_weighted_loss(orc):
    """Samples whose target lies below the band count (1 + near_w) times: the
    loss and gradient equal those of the unweighted loss over a batch in which
    each such sample is repeated 1 + near_w times (rescaled to the batch size);
    finite differences agree with the gradient."""
    widths = [4, 6, 1]
    rng = np.random.default_rng(21)
    n = orc.mlp_param_count(widths)
    p = rng.normal(size=n) * 0.5
    x = rng.normal(size=(6, 4))
    t = np.array([-0.2, 0.01, 0.3, 0.04, 0.6, -0.05])
    band, near_w = 0.05, 2.0
    loss, g = orc.mlp_loss_grad(widths, p, x, t, 4.0, near_w, band)
    rep = np.concatenate([np.repeat(np.arange(6)[t < band], 3), np.arange(6)[t >= band]])
    l_rep, g_rep = orc.mlp_loss_grad(widths, p, x[rep], t[rep], 4.0)
    scale = len(rep) / 6.0
    assert abs(loss - l_rep * scale) < 1e-12
    np.testing.assert_allclose(g, g_rep * scale, rtol=1e-12, atol=1e-14)
    h = 1e-6
    for i in range(0, n, 3):
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (orc.mlp_loss_grad(widths, pp, x, t, 4.0, near_w, band)[0]
              - orc.mlp_loss_grad(widths, pm, x, t, 4.0, near_w, band)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i]))
    # the reduced-precision dataflow applies the same weights
    lb, _ = orc.mlp_loss_grad_bf16(widths, p, x, t, 4.0, near_w, band)
    lb0, _ = orc.mlp_loss_grad_bf16(widths, p, x, t, 4.0)
    assert lb > lb0


def test_adam_first_step_is_signed_lr(orc):
    p = np.array([1.0, -2.0, 0.5])
    m, v = np.zeros(3), np.zeros(3)
    g = np.array([0.3, -4.0, 1e-3])
    orc.adam(p, m, v, g, 0.01, 0.9, 0.999, 1e-12, 1)
    np.testing.assert_allclose(p, [0.99, -1.99, 0.49], atol=1e-8)


def test_adam_bias_correction_constant_gradient(orc):
    """With a constant gradient the bias-corrected moments equal g and g^2 at
    every step (m_t = (1 - b1^t) g, v_t = (1 - b2^t) g^2), so with eps = 0
    each step moves every parameter by exactly lr against the gradient's
    sign: after 3 steps, 3 lr."""
    p0 = np.array([1.0, -2.0, 0.5, 3.0])
    g = np.array([0.3, -4.0, 1e-3, -7.5])
    p, m, v = p0.copy(), np.zeros(4), np.zeros(4)
    for t in (1, 2, 3):
        orc.adam(p, m, v, g, 0.01, 0.9, 0.999, 0.0, t)
        np.testing.assert_allclose(p, p0 - t * 0.01 * np.sign(g), rtol=0, atol=1e-14)


def test_adam_two_steps_by_hand(orc):
    """g = +1 then -1 with b1 = 1/2, b2 = 3/4, eps = 0, worked by hand:
    step 1: m = 1/2, v = 1/4, m^ = 1, v^ = 1 -> p -= lr;
    step 2: m = 1/4 - 1/2 = -1/4, v = 3/16 + 1/4 = 7/16, m^ = -1/4 / (3/4) = -1/3,
    v^ = (7/16) / (7/16) = 1 -> p += lr/3; total -2 lr / 3."""
    p, m, v = np.array([0.0]), np.zeros(1), np.zeros(1)
    orc.adam(p, m, v, np.array([1.0]), 0.03, 0.5, 0.75, 0.0, 1)
    assert abs(p[0] + 0.03) < 1e-15
    orc.adam(p, m, v, np.array([-1.0]), 0.03, 0.5, 0.75, 0.0, 2)
    assert abs(m[0] + 0.25) < 1e-15 and abs(v[0] - 7 / 16) < 1e-15
    assert abs(p[0] + 0.02) < 1e-15


def test_bf16_rounding_matches_torch(orc):
    """Round-to-nearest-even bfloat16 against torch's own conversion."""
    import torch
    rng = np.random.default_rng(13)
    xs = np.concatenate([rng.normal(size=2000) * 10 ** rng.uniform(-6, 6, size=2000),
                         [1 + 2 ** -8, 1 + 3 * 2 ** -8, -1 - 2 ** -8, 0.0, 3.14159265]]).astype(np.float32)
    ref = torch.from_numpy(xs).to(torch.bfloat16).to(torch.float64).numpy()
    got = np.array([orc.bf16(float(x)) for x in xs])
    np.testing.assert_array_equal(got, ref)


def test_bf16_gradient_exact_when_nothing_rounds(orc):
    """A linear layer with small integer weights, inputs and targets: every
    product operand is bfloat16-exact, so the reduced-precision gradient
    equals the FP64 one exactly; with non-representable operands it does not."""
    widths = [3, 1]
    p = np.array([1.0, -1.0, 0.0, 2.0])
    x = np.array([[1.0, 0.0, -1.0], [1.0, 1.0, 1.0]])
    t = np.array([1.0, -2.0])
    l1, g1 = orc.mlp_loss_grad(widths, p, x, t, 4.0)
    l2, g2 = orc.mlp_loss_grad_bf16(widths, p, x, t, 4.0)
    assert l1 == l2
    np.testing.assert_array_equal(g1, g2)
    _, g3 = orc.mlp_loss_grad(widths, p + 1e-3, x * 1.001, t, 4.0)
    _, g4 = orc.mlp_loss_grad_bf16(widths, p + 1e-3, x * 1.001, t, 4.0)
    assert np.any(g3 != g4)


def test_bf16_forward_exact_when_nothing_rounds(orc):
    """Small integer weights, inputs and biases keep every product operand and
    hidden activation bfloat16-exact: the reduced-precision forward equals the
    hand-computed 2-2-1 network exactly."""
    params = np.array([1, -1, 2, 0.5, 0, -1, 1, 3, 0.5], float)
    x = np.array([[1.0, 2.0], [-1.0, 0.0]])
    np.testing.assert_array_equal(orc.mlp_forward_bf16([2, 2, 1], params, x)[:, 0], [6.5, 0.5])


def test_bf16_forward_rounds_each_operand(orc):
    """Each rounding point of the dataflow on a 1-1-1 chain (W0, b0, W1, b1):
    an input of 1 + 2^-9 enters as 1 and so does a weight of 1 + 2^-9 (the
    bfloat16 spacing at 1 is 2^-7); a hidden activation 1 + 2^-7 + 2^-9 leaves
    as 1 + 2^-7; a bias is added unrounded; a negative hidden value is cut to
    0 while the output may be negative."""
    def f(p, x):
        return orc.mlp_forward_bf16([1, 1, 1], np.array(p, float), np.array([[x]], float))[0, 0]
    e9, e7 = 2.0 ** -9, 2.0 ** -7
    assert f([1, 0, 1, 0], 1 + e9) == 1.0
    assert f([1 + e9, 0, 1, 0], 1.0) == 1.0
    assert f([1 + e7, e9, 1, 0], 1.0) == 1 + e7
    assert f([1, 0, 1, 2.0 ** -20], 1.0) == 1 + 2.0 ** -20
    assert f([1, -2, 1, -0.25], 1.0) == -0.25
    # the plain forward keeps the digits the reduced one drops
    assert orc.mlp_forward([1, 1, 1], np.array([1 + e7, e9, 1, 0.0]), np.array([[1.0]]))[0, 0] == 1 + e7 + e9


def test_bf16_backward_rounds_each_operand(orc):
    """Each rounding point of the reduced-precision backward on a 1-1-1 chain,
    worked by hand (bfloat16 keeps 8 significant bits: spacing 2^-7 at 1).
    x = 1 + 2^-10, W0 = 1, b0 = 2^-10, W1 = 1 + 2^-7 + 2^-10, b1 = 0,
    t = 1/2 + 3 2^-10, squared error only:
      a0 = bf(x) = 1; z1 = 1 + 2^-10, a1 = bf(z1) = 1; y = bf(W1) a1 = 1 + 2^-7;
      dy = 2 (y - t) = 1 + 2^-7 + 2^-9, bf(dy) = 1 + 2^-7;
      db1 = dy (unrounded)                   = 1 + 2^-7 + 2^-9
      dW1 = bf(dy) a1                        = 1 + 2^-7
      dZ1 = bf(W1) bf(dy) = (1 + 2^-7)^2     = 1 + 2^-6 + 2^-14 (z1 > 0)
      db0 = dZ1 (unrounded)                  = 1 + 2^-6 + 2^-14
      dW0 = bf(dZ1) a0                       = 1 + 2^-6.
    Dropping any one rounding (or rounding a bias gradient, or using the
    unrounded input or activation) changes one of the four values."""
    e = lambda k: 2.0 ** -k
    params = np.array([1.0, e(10), 1 + e(7) + e(10), 0.0])
    x = np.array([[1 + e(10)]])
    t = np.array([0.5 + 3 * e(10)])
    loss, g = orc.mlp_loss_grad_bf16([1, 1, 1], params, x, t, 0.0)
    assert loss == (0.5 + 5 * e(10)) ** 2
    np.testing.assert_array_equal(g, [1 + e(6), 1 + e(6) + e(14), 1 + e(7), 1 + e(7) + e(9)])
    # a negative hidden pre-activation stops the gradient below the ReLU
    params[1] = -2.0
    loss, g = orc.mlp_loss_grad_bf16([1, 1, 1], params, x, t, 0.0)
    assert loss == t[0] ** 2
    np.testing.assert_array_equal(g, [0.0, 0.0, 0.0, -2 * t[0]])


def test_bf16_forward_is_the_training_dataflow_forward(orc):
    """The training dataflow's loss at target 0 without the asymmetric or
    near weights is the batch mean of y^2, with y its own forward pass; the
    standalone forward gives the same y.  Both stay within the bfloat16
    operand error of the FP64 network."""
    widths = [17, 32, 32, 1]
    rng = np.random.default_rng(23)
    p = rng.normal(size=orc.mlp_param_count(widths)) * 0.3
    x = rng.uniform(-1, 1, size=(40, 17))
    y = orc.mlp_forward_bf16(widths, p, x)[:, 0]
    loss, _ = orc.mlp_loss_grad_bf16(widths, p, x, np.zeros(40), 0.0)
    assert abs(loss - np.mean(y * y)) <= 1e-12 * max(1.0, loss)
    y64 = orc.mlp_forward(widths, p, x)[:, 0]
    assert np.linalg.norm(y - y64) / np.linalg.norm(y64) < 3e-2
    assert np.any(y != y64)


def test_bf16_gradient_close_to_fp64(orc):
    widths = [17, 32, 32, 1]
    rng = np.random.default_rng(15)
    n = orc.mlp_param_count(widths)
    p = rng.normal(size=n) * 0.3
    x = rng.uniform(-1, 1, size=(64, 17))
    t = rng.uniform(-0.1, 0.5, size=64)
    _, g1 = orc.mlp_loss_grad(widths, p, x, t, 4.0)
    _, g2 = orc.mlp_loss_grad_bf16(widths, p, x, t, 4.0)
    assert np.linalg.norm(g2 - g1) / np.linalg.norm(g1) < 3e-2


def test_pair_features_reproduce_the_distance(orc):
    """The canonical frame of the features preserves the exact distance: both
    arms rebuilt from the features alone (own arm at the origin, the other at
    the feature offset with its yaw folded into its first joint) are exactly
    as far apart as in the world."""
    sc = scenes.make_scene(5, collision_mode=0)
    rng = np.random.default_rng(16)
    for a, i in [(0, 4), (1, 2), (6, 3), (7, 0)]:
        A, I = sc.arms[a], sc.arms[i]
        qa = scenes.random_plan_inputs(rng, A, 1)[0].astype(np.float64)
        qi = scenes.random_plan_inputs(rng, I, 1)[0].astype(np.float64)
        f = orc.pair_features(orc.make_arm(A), qa, orc.make_arm(I), qi)
        lo, hi = A.q_lim[:, 0].astype(np.float64), A.q_lim[:, 1].astype(np.float64)
        mid, half = (lo + hi) / 2, (hi - lo) / 2
        np.testing.assert_allclose(mid + half * f[:7], qa, atol=1e-12)
        qi2 = np.concatenate([[f[7] * math.pi], mid[1:] + half[1:] * f[8:14]])
        A0 = scenes.Arm(**{**A.__dict__, "base": np.zeros(4, np.float32)})
        I0 = scenes.Arm(**{**I.__dict__, "base": np.array([0, 0, 0, 0], np.float32)})
        oa0, oi0 = orc.make_arm(A0), orc.make_arm(I0)
        oi0.base[0], oi0.base[1], oi0.base[2] = f[14], f[15], f[16]
        world = orc.arm_pair_rho(orc.make_arm(A), qa, orc.make_arm(I), qi)
        canon = orc.arm_pair_rho(oa0, qa, oi0, qi2)
        assert abs(world - canon) < 1e-9
        assert -1 <= f[7] < 1
