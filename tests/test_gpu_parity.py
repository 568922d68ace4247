"""GPU parity of the HIP control step against the FP64 CPU oracle, through
the C-ABI.  Tolerances (FP32 GPU vs FP64 oracle):
  noise eps             1e-6 absolute (sigma * 2e-6 on the normals, rounded up)
  sphere centres        1e-5 m, end to end
  stage / rollout costs 1e-4 relative with floor max(|C|, 1), stage-isolated
                        (the oracle's cost stage is fed the GPU's FP32 joint
                        states, spheres, plans and priority factors)
  updated means         1e-5 absolute, stage-isolated (oracle update fed the
                        GPU's FP32 costs and noise)
  plans                 1e-5 m (oracle ToPlan fed the GPU's updated means)
Integer and index results (Philox words, argmin, query counts) are exact.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2602_10114_amd import native, scenes
from helpers import Capture, f32, oracle_stage, read_boards, rel_err, small_scene

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    native.lib()
    yield


def _obs(sc):
    return sc.obstacles if sc.obstacles.shape[0] else None


# --------------------------------------------------------------------- noise
def test_philox_bitwise():
    _say("case: philox 4096 random counters")
    rng = np.random.default_rng(0)
    ctr = rng.integers(0, 2**32, size=(4096, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2**32, size=(4096, 2), dtype=np.uint64).astype(np.uint32)
    ctr[0], key[0] = 0, 0
    out = native.philox(torch.from_numpy(ctr.view(np.int32)).cuda(), torch.from_numpy(key.view(np.int32)).cuda())
    got = out.cpu().numpy().view(np.uint32)
    for i in range(0, 4096, 97):
        assert list(got[i]) == list(oracle.philox(ctr[i], key[i]))
    assert list(got[0]) == [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]


# ------------------------------------------------------------ single arm
@pytest.fixture(scope="module")
def cfg1_ragged():
    _say("case: one-arm scene, N=100 (ragged tail), H=20, one step with capture")
    sc = small_scene(1, n=100)
    ctl = native.Controller(sc.arms, sc.params)
    ctl.debug_enable(True)
    u = ctl.step(sc.state, sc.goal, sc.obstacles).cpu().numpy()
    ctl.sync()
    cap = Capture(ctl, 0)
    plan, pq, mean = (x.cpu().numpy().astype(np.float64) for x in ctl.get_plan(0))
    yield sc, ctl, cap, u, plan, pq
    ctl.close()


def test_noise_matches_oracle(cfg1_ragged):
    sc, _, cap, _, _, _ = cfg1_ragged
    p = sc.params
    N, H = sc.arms[0].n_rollouts, sc.arms[0].horizon
    err = 0.0
    for n in range(N):
        for h in range(H):
            z = oracle.normals(p["seed"], 0, 0, 0, n, h, 7)
            err = max(err, np.abs(cap.eps[h, :, n] - f32(p["sigma"]) * z).max())
    assert err < 1e-6, err


def test_spheres_end_to_end(cfg1_ragged):
    sc, _, cap, _, _, _ = cfg1_ragged
    p, arm = sc.params, sc.arms[0]
    oa = oracle.make_arm(arm)
    st = sc.state[0].astype(np.float64)
    err = 0.0
    for n in list(range(0, arm.n_rollouts, 9)) + [arm.n_rollouts - 1]:
        U = np.stack([f32(p["sigma"]) * oracle.normals(p["seed"], 0, 0, 0, n, h, 7) for h in range(arm.horizon)])
        q, qd = oracle.integrate(st[:, 0], st[:, 1], U, f32(p["dt"]))
        np.testing.assert_allclose(cap.q[n], q, atol=2e-6)
        np.testing.assert_allclose(cap.qd[n], qd, atol=2e-6)
        for h in range(arm.horizon):
            err = max(err, np.abs(oracle.spheres(oa, q[h]) - cap.sph[n, h]).max())
    assert err < 1e-5, err


def test_stage_costs_stage_isolated(cfg1_ragged):
    sc, ctl, cap, _, _, _ = cfg1_ragged
    boards = read_boards(ctl, sc)
    ref = oracle_stage(sc, 0, cap, sc.obstacles, boards)
    assert rel_err(cap.stage, ref) < 1e-4
    tot = np.array([oracle.total_cost(cap.stage[:, n], f32(sc.params["gamma"])) for n in range(cap.stage.shape[1])])
    assert rel_err(cap.cost, tot) < 1e-5


def test_update_and_act_stage_isolated(cfg1_ragged):
    sc, _, cap, u, _, _ = cfg1_ragged
    lam = f32(sc.params["lam"])
    w = oracle.weights(cap.cost, lam)
    np.testing.assert_allclose(cap.w, w, atol=1e-6, rtol=1e-4)
    U = np.transpose(cap.eps, (2, 0, 1))  # the means were zero before this step
    mt = oracle.weighted_mean(w, U)
    assert np.abs(cap.mu - mt).max() < 1e-5
    n_star = oracle.argmin(cap.cost)
    assert cap.argmin == n_star
    assert np.abs(u[0] - U[n_star, 0]).max() < 1e-6


def test_plan_stage_isolated(cfg1_ragged):
    sc, _, cap, _, plan, pq = cfg1_ragged
    arm = sc.arms[0]
    oa = oracle.make_arm(arm)
    st = sc.state[0].astype(np.float64)
    q, _ = oracle.integrate(st[:, 0], st[:, 1], cap.mu, f32(sc.params["dt"]))
    assert np.abs(pq - q).max() < 2e-6
    for h in range(arm.horizon):
        s = oracle.spheres(oa, q[h])
        assert np.abs(plan[:, :, h] - s).max() < 1e-5


# -------------------------------------------------------------- many arms
def _run_multi(sc, steps, publish=True, debug_last=True, stream=None):
    ctl = native.Controller(sc.arms, sc.params, stream=stream)
    caps, boards, us = None, None, None
    for t in range(steps):
        last = t == steps - 1
        if last and debug_last:
            ctl.debug_enable(True)
            ctl.sync()
            boards = read_boards(ctl, sc)
        u = ctl.step(sc.state, sc.goal, _obs(sc))
        if publish:
            ctl.share_plans()
        us = u
    ctl.sync()
    if debug_last:
        caps = [Capture(ctl, a) for a in range(sc.n_arms)]
    return ctl, caps, boards, us.cpu().numpy()


def test_two_arms_plan_sharing():
    _say("case: two facing arms, N=128, H=12, 3 steps with plan sharing")
    sc = small_scene(2, n=128, h=12)
    ctl, caps, boards, u = _run_multi(sc, 3)
    for a in range(2):
        assert boards[1 - a][1] == 1
        ref = oracle_stage(sc, a, caps[a], sc.obstacles, boards)
        assert rel_err(caps[a].stage, ref) < 1e-4
        # priority factor from the GPU's distance and the published one
        d_other = boards[1 - a][2]
        al = oracle.priority(caps[a].dist, d_other, f32(3.0), f32(1e-3), f32(0.5), f32(2.0))
        assert abs(caps[a].alpha[1 - a] - al) < 1e-5 * max(1.0, al)
    # the coordination term is live in this scene (arms start ~1 cm apart)
    assert any((c.stage > 100).any() for c in caps)
    ctl.close()


def test_uneven_batch_and_counter():
    _say("case: four uneven arms, ragged N (64,100,128,192), H (8,12,12,16), 3 steps")
    sc = small_scene(3, n=[64, 100, 128, 192], h=[8, 12, 12, 16])
    ctl, caps, boards, u = _run_multi(sc, 3)
    for a in range(4):
        ref = oracle_stage(sc, a, caps[a], sc.obstacles, boards)
        assert rel_err(caps[a].stage, ref) < 1e-4, a
        # Sec. IV-A complexity: H N N_S sum_i N_S^(i) queries, counted over the
        # steps each neighbour's (shorter) horizon reaches.
        arm = sc.arms[a]
        expect = sum(arm.n_rollouts * arm.n_spheres * sum(sc.arms[i].n_spheres for i in range(4)
                                                          if i != a and h < sc.arms[i].horizon and boards[i][1])
                     for h in range(arm.horizon))
        assert caps[a].pairs == expect
    ctl.close()


def test_wide_rollout_spread_keeps_every_near_pair():
    """The pair cull decides once per wave of 64 rollouts, with one bounding
    sphere per body widened by the wave's spread.  With a large sampling
    sigma the rollouts of a wave fan out (a neighbour's plan within the
    buffer in some lanes, clear of it in others); every stage cost must still
    equal the oracle's all-pairs one."""
    spread = mixed = 0
    for cfg, n, h in ((2, 128, 12), (3, [64, 128, 128, 192], [8, 12, 12, 16])):
        _say(f"case: config {cfg} with sigma 4.0, N={n}, H={h}, 3 steps with plan sharing")
        sc = small_scene(cfg, n=n, h=h, sigma=4.0)
        ctl, caps, boards, _ = _run_multi(sc, 3)
        B = sc.params["buf_dyn"]
        for a in range(sc.n_arms):
            ref = oracle_stage(sc, a, caps[a], sc.obstacles, boards)
            assert rel_err(caps[a].stage, ref) < 1e-4, (cfg, a)
            sph = caps[a].sph  # [N][H][S][4]
            N, H = sph.shape[0], sph.shape[1]
            # each lane's smallest gap to any neighbour plan sphere, per step
            gap = np.full((N, H), np.inf)
            for i in range(sc.n_arms):
                if i == a or not boards[i][1]:
                    continue
                plan = boards[i][0]  # [H_i][S_i][4]
                for hh in range(min(H, plan.shape[0])):
                    d = np.linalg.norm(sph[:, hh, :, None, :3] - plan[None, hh, None, :, :3], axis=3)
                    g = d - sph[:, hh, :, None, 3] - plan[None, hh, None, :, 3]
                    gap[:, hh] = np.minimum(gap[:, hh], g.min(axis=(1, 2)))
            for w0 in range(0, N - 63, 64):
                c = sph[w0:w0 + 64, -1, :, :3]
                spread = max(spread, float(np.linalg.norm(c - c[0], axis=2).max()))
                near = gap[w0:w0 + 64] < B  # [64][H]
                mixed += int((near.any(axis=0) & ~near.all(axis=0)).sum())
        ctl.close()
    # the waves did fan out, and at some steps held lanes within the buffer
    # beside lanes clear of it
    assert spread > 0.1
    assert mixed > 0


def _closed_loop(sc, steps, setup=None):
    """Controls of `steps` closed-loop steps (Publish, step, plant) and the
    final plans, as host arrays; `setup(ctl)` runs after init."""
    import torch
    ctl = native.Controller(sc.arms, sc.params)
    if setup is not None:
        setup(ctl)
    state = torch.as_tensor(sc.state.astype(np.float32), device="cuda").contiguous()
    us = []
    for _ in range(steps):
        ctl.share_plans()
        u = ctl.step(state, sc.goal, _obs(sc))
        ctl.sim_execute(state, u)
        us.append(u.cpu().numpy().copy())
    ctl.sync()
    plans = [ctl.get_plan(a)[0].cpu().numpy().copy() for a in range(sc.n_arms)]
    stats = ctl.surrogate_stats() if setup is not None else None
    ctl.close()
    return np.stack(us), plans, stats


def test_pair_cull_changes_no_bit():
    """The bounding-sphere cull of sphere pairs (pair_cull 1) against every
    pair through the filter (pair_cull 0): closed-loop controls and plans
    bitwise equal, on scenes where the coordination, obstacle and self terms
    are live (two facing arms 1 cm apart, also with sigma 4 so the waves fan
    out; four uneven arms with obstacles; eight arms of 64 spheres)."""
    cases = ((2, 128, 12, {}), (2, 128, 12, {"sigma": 4.0}), (3, [64, 100, 128, 192], [8, 12, 12, 16], {}),
             (5, 128, 10, {}))
    for cfg, n, h, over in cases:
        _say(f"case: config {cfg} {over} N={n} H={h}, 6 closed-loop steps with pair_cull 1 and 0")
        (u1, p1, _), (u0, p0, _) = [_closed_loop(small_scene(cfg, n=n, h=h, pair_cull=cull, collision_mode=0,
                                                             **over), 6) for cull in (1, 0)]
        assert np.array_equal(u1.view(np.uint32), u0.view(np.uint32)), cfg
        for a, b in zip(p1, p0):
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), cfg


def test_unpublished_neighbours_ignored():
    _say("case: two facing arms without publish")
    sc = small_scene(2, n=64, h=10)
    ctl, caps, boards, _ = _run_multi(sc, 2, publish=False)
    for a in range(2):
        assert caps[a].alpha[1 - a] == 0.0
        assert caps[a].pairs == 0
    ctl.close()
    sc0 = small_scene(2, n=64, h=10, w_dyn=0.0)
    ctl0, caps0, _, _ = _run_multi(sc0, 2, publish=True)
    for a in range(2):
        np.testing.assert_array_equal(caps[a].stage, caps0[a].stage)
    ctl0.close()


def test_fault_injected_plan():
    _say("case: injected neighbour plan through the board")
    sc = small_scene(2, n=64, h=10)
    ctl = native.Controller(sc.arms, sc.params)
    ctl.step(sc.state, sc.goal, None)
    ctl.sync()
    # put arm 1's plan right on top of arm 0's current spheres
    oa = oracle.make_arm(sc.arms[0])
    s0 = oracle.spheres(oa, sc.state[0, :, 0].astype(np.float64))
    fake = np.repeat(s0[None], 10, axis=0).astype(np.float32)
    ctl.set_board(1, fake, np.zeros((10, 7), np.float32), 0.5, 1)
    ctl.debug_enable(True)
    boards = read_boards(ctl, sc)
    ctl.step(sc.state, sc.goal, None)
    ctl.sync()
    cap = Capture(ctl, 0)
    ref = oracle_stage(sc, 0, cap, sc.obstacles, boards)
    assert rel_err(cap.stage, ref) < 1e-4
    assert cap.stage.min() > 5000 * 0.5 * 0.9  # every rollout overlaps the injected plan
    ctl.close()


def test_update_second_step_and_shift():
    _say("case: one-arm scene, two steps, update stage-isolated on the shifted means")
    sc = small_scene(1, n=128, alpha_mu=0.5)
    ctl = native.Controller(sc.arms, sc.params)
    ctl.step(sc.state, sc.goal, sc.obstacles)
    ctl.sync()
    mu1 = ctl.get_plan(0)[2].cpu().numpy().astype(np.float64)
    ctl.debug_enable(True)
    u = ctl.step(sc.state, sc.goal, sc.obstacles).cpu().numpy()
    ctl.sync()
    cap = Capture(ctl, 0)
    mu_prev = oracle.shift(mu1)
    U = mu_prev[None] + np.transpose(cap.eps, (2, 0, 1))
    w = oracle.weights(cap.cost, f32(sc.params["lam"]))
    mt = oracle.weighted_mean(w, U)
    new = oracle.ema(mu_prev, mt, f32(0.5))
    assert np.abs(cap.mu - new).max() < 1e-5
    n_star = oracle.argmin(cap.cost)
    assert np.abs(u[0] - U[n_star, 0]).max() < 1e-6
    ctl.close()


def test_graph_path_bitwise_equals_capture_path():
    _say("case: graph-captured production kernel vs capturing kernel, four uneven arms")
    sc = small_scene(3, n=[64, 100, 128, 192], h=[8, 12, 12, 16])
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        c1, _, _, u1 = _run_multi(sc, 3, debug_last=False, stream=s)
        c2, _, _, u2 = _run_multi(sc, 3, debug_last=True, stream=s)
        m1 = [c1.get_plan(a)[2].cpu().numpy() for a in range(4)]
        m2 = [c2.get_plan(a)[2].cpu().numpy() for a in range(4)]
    s.synchronize()
    np.testing.assert_array_equal(u1, u2)
    for a in range(4):
        np.testing.assert_array_equal(m1[a], m2[a])
    c1.close()
    c2.close()


def test_deterministic_repeat():
    _say("case: repeat run bitwise, two facing arms")
    sc = small_scene(2, n=256, h=16)
    outs = []
    for _ in range(2):
        ctl, _, _, u = _run_multi(sc, 4, debug_last=False)
        outs.append((u, [ctl.get_plan(a)[2].cpu().numpy() for a in range(2)]))
        ctl.close()
    np.testing.assert_array_equal(outs[0][0], outs[1][0])
    for a in range(2):
        np.testing.assert_array_equal(outs[0][1][a], outs[1][1][a])


def test_tiles_do_not_change_results():
    """Every launch shape gives bitwise the same stage costs, totals,
    weights, means and actions: horizon tiles 1, 3 and H, and 1, 2 or 4
    waves (64, 128 or 256 rollouts) per workgroup sharing one staged copy of
    the step's sets (rollout counts 256, 200, 512, 460: ragged last waves),
    two steps with plan sharing so the neighbour sets are live."""
    _say("case: forced launch shapes (waves per workgroup x horizon tile) give identical results")
    sc = small_scene(3, n=[256, 200, 512, 460], h=[8, 12, 12, 16])
    res = []
    for W, T in ((1, 1), (1, 3), (1, 16), (2, 3), (2, 16), (4, 1), (4, 5), (4, 16)):
        ctl = native.Controller(sc.arms, sc.params)
        ctl.set_tuning(64 * W, T, 0)
        ctl.step(sc.state, sc.goal, sc.obstacles)
        ctl.share_plans()
        ctl.debug_enable(True)
        u = ctl.step(sc.state, sc.goal, sc.obstacles).cpu().numpy()
        ctl.sync()
        res.append((u, [[ctl.debug_get(k, a).cpu().numpy() for k in ("STAGE_COST", "COST", "WEIGHTS", "MEAN", "PAIRS")]
                        for a in range(4)]))
        assert ctl.tuning()[:2] == (64 * W, T)
        ctl.close()
    for u, r in res[1:]:
        np.testing.assert_array_equal(u, res[0][0])
        for a in range(4):
            for x, x0 in zip(r[a], res[0][1][a]):
                np.testing.assert_array_equal(x, x0)
    # a workgroup may not reach past an arm's padded rollouts
    bad = small_scene(3, n=[64, 100, 128, 192], h=[8, 12, 12, 16])
    ctl = native.Controller(bad.arms, bad.params)
    with pytest.raises(native.MpcError) as e:
        ctl.set_tuning(128, 0, 0)
    assert e.value.code == native.MPC_EINVAL
    with pytest.raises(native.MpcError) as e:
        ctl.set_tuning(96, 0, 0)
    assert e.value.code == native.MPC_EUNSUPPORTED
    ctl.close()


def test_tuner_choice_is_cached_per_shape():
    """The tuner's launch shape is kept per problem shape and device: a second
    context with the same shape starts from the same choice."""
    _say("case: tuner cache, four uneven arms")
    sc = small_scene(3, n=[256, 200, 512, 460], h=[8, 12, 12, 16])
    shapes = []
    for _ in range(2):
        ctl = native.Controller(sc.arms, sc.params)
        for _ in range(2):
            ctl.step(sc.state, sc.goal, sc.obstacles)
            ctl.share_plans()
        ctl.sync()
        shapes.append(ctl.tuning())
        ctl.close()
    _say(f"  tuned launch shapes {shapes}")
    assert shapes[0] == shapes[1]
    assert shapes[0][0] in (64, 128, 256)


# ------------------------------------------------------------- edge cases
def test_single_rollout_and_single_step_horizon():
    _say("case: N=1, H=1")
    sc = small_scene(1, n=1, h=1)
    ctl = native.Controller(sc.arms, sc.params)
    ctl.debug_enable(True)
    u = ctl.step(sc.state, sc.goal, sc.obstacles).cpu().numpy()
    ctl.sync()
    cap = Capture(ctl, 0)
    assert cap.w[0] == 1.0
    np.testing.assert_allclose(cap.mu[0], cap.eps[0, :, 0], atol=1e-7)
    np.testing.assert_allclose(u[0], cap.eps[0, :, 0], atol=1e-7)
    boards = read_boards(ctl, sc)
    assert rel_err(cap.stage, oracle_stage(sc, 0, cap, sc.obstacles, boards)) < 1e-4
    ctl.close()


def test_no_obstacles_and_errors():
    _say("case: zero obstacles, argument errors")
    sc = small_scene(1, n=64, h=6)
    ctl = native.Controller(sc.arms, sc.params)
    ctl.debug_enable(True)
    ctl.step(sc.state, sc.goal, None)
    ctl.sync()
    cap = Capture(ctl, 0)
    assert rel_err(cap.stage, oracle_stage(sc, 0, cap, np.zeros((0, 4)), read_boards(ctl, sc))) < 1e-4
    too_many = np.zeros((sc.params["max_obstacles"] + 1, 4), np.float32)
    with pytest.raises(native.MpcError) as e:
        ctl.step(sc.state, sc.goal, too_many)
    assert e.value.code == native.MPC_EINVAL
    buf = torch.empty(4096, device="cuda")
    assert native.lib().mpc_get_plan(ctl.h, 5, native._ptr(buf), None, None) == native.MPC_EINVAL
    assert native.lib().mpc_debug_get(ctl.h, 99, 0, native._ptr(buf)) == native.MPC_EINVAL
    ctl.close()
    fresh = native.Controller(sc.arms, sc.params)
    with pytest.raises(native.MpcError) as e:
        fresh.get_plan(0)
    assert e.value.code == native.MPC_ESTATE
    fresh.close()
    bad = small_scene(1, n=64, h=6)
    bad.arms[0].horizon = 65
    with pytest.raises(native.MpcError) as e:
        native.Controller(bad.arms, bad.params)
    assert e.value.code == native.MPC_EINVAL


def test_padded_sphere_layout():
    _say("case: 64-sphere layout (8 per body), 2 arms")
    sc = scenes.make_scene(5, collision_mode=0)
    sc.arms = sc.arms[:2]
    sc.arms[1] = scenes.dataclasses.replace(sc.arms[1], base=np.array([-0.75, 0.4, 0.0, -np.pi / 2], np.float32))
    for a in sc.arms:
        a.n_rollouts, a.horizon = 64, 8
    sc.state, sc.goal = sc.state[:2], sc.goal[:2]
    ctl, caps, boards, _ = _run_multi(sc, 2)
    for a in range(2):
        assert rel_err(caps[a].stage, oracle_stage(sc, a, caps[a], sc.obstacles, boards)) < 1e-4
    ctl.close()


def test_mixed_layout_arms():
    _say("case: arms with 52 and 40 spheres (padded layout for both)")
    sc = small_scene(2, n=64, h=8)
    a1 = sc.arms[1]
    keep = np.arange(a1.n_spheres) % 4 != 3
    sc.arms[1] = scenes.dataclasses.replace(a1, spheres=a1.spheres[keep], sphere_link=a1.sphere_link[keep])
    ctl, caps, boards, _ = _run_multi(sc, 2)
    for a in range(2):
        assert rel_err(caps[a].stage, oracle_stage(sc, a, caps[a], sc.obstacles, boards)) < 1e-4
    ctl.close()


def _end_to_end(sc, steps, obstacles):
    """GPU and full oracle controller from their own noise for `steps` steps
    with plan sharing; per arm the largest relative total-cost gap (floor 1),
    the largest mean gap and max|U| of the last step."""
    ctl = native.Controller(sc.arms, sc.params)
    orc = oracle.Controller(sc.arms, sc.params)
    for t in range(steps):
        ctl.debug_enable(t == steps - 1)
        ctl.step(sc.state, sc.goal, obstacles)
        orc.step(sc.state, sc.goal, obstacles if obstacles is not None else np.zeros((0, 4), np.float32))
        ctl.share_plans()
        orc.share_plans()
    ctl.sync()
    out = []
    for a in range(sc.n_arms):
        N, H = sc.arms[a].n_rollouts, sc.arms[a].horizon
        cap = Capture(ctl, a, want_spheres=False)
        tot, _, _ = orc.costs(a)
        mu_o = orc.mean(a)[:H]
        rel = rel_err(cap.cost, tot[:N])
        U = np.abs(np.transpose(cap.eps, (2, 0, 1))).max() + np.abs(mu_o).max()
        out.append((rel, np.abs(cap.mu - mu_o).max(), U, np.abs(tot[:N]).max()))
    ctl.close()
    return out


def test_end_to_end_costs_and_means_fixed_tolerance():
    """End to end (the oracle draws its own FP64 noise and runs its own
    controller) on a scene whose hinges stay clear of their buffers (one arm,
    no obstacle): total costs within 1e-4 relative (floor 1), then the means
    within the softmax conditioning bound evaluated at that limit,
    max|U| * 1e-4 max(|C|, 1) / lambda -- a fixed bound, not one widened by
    the measured cost gap."""
    _say("case: end to end vs the full oracle controller, one arm, 128 rollouts x 16 steps, 3 steps")
    sc = small_scene(1, n=128, h=16)
    lam = f32(sc.params["lam"])
    for rel, dmu, U, cmax in _end_to_end(sc, 3, None):
        _say(f"  total costs: max relative gap {rel:.2e}; means: max gap {dmu:.2e}")
        assert rel < 1e-4
        assert dmu <= U * 1e-4 * max(cmax, 1.0) / lam


def test_end_to_end_report_with_live_coordination():
    """Report only (not a gate): with the two arms about 1 cm apart, the
    coordination hinge's slope w_dyn / B = 1.7e5 per metre turns the FP32
    rounding of a sphere centre (1e-7 m) into cost gaps far above 1e-4, so
    end-to-end parity is not a property of an FP32 implementation here; the
    stage-isolated tests above are the gate.  Prints the measured gaps."""
    _say("case: end to end, two facing arms with live coordination, 3 steps (report)")
    sc = small_scene(2, n=64, h=10)
    for a, (rel, dmu, U, _) in enumerate(_end_to_end(sc, 3, None)):
        _say(f"  arm {a}: total costs max relative gap {rel:.2e}; means max gap {dmu:.2e} (max|U| {U:.2f})")
        assert np.isfinite(rel) and np.isfinite(dmu)


# -------------------------------------------------------- Sense and Publish
def test_sense_distance_to_goal_against_oracle():
    """Sense (Eq. 10's distance to goal): the end-effector point of each arm's
    sensed joints against its goal position, end to end against the oracle's
    kinematics, 1e-5 m, on the eight arms of the 64-sphere workload."""
    _say("case: Sense distance to goal, 8 arms")
    sc = scenes.make_scene(5, collision_mode=0)
    for a in sc.arms:
        a.n_rollouts, a.horizon = 64, 4
    ctl = native.Controller(sc.arms, sc.params)
    ctl.step(sc.state, sc.goal, sc.obstacles)
    ctl.sync()
    for a in range(sc.n_arms):
        T = oracle.ee_pose(oracle.make_arm(sc.arms[a]), sc.state[a, :, 0].astype(np.float64))
        ref = np.linalg.norm(T[:3, 3] - sc.goal[a, :3].astype(np.float64))
        got = float(ctl.debug_get("DIST", a)[0])
        assert abs(got - ref) < 1e-5, (a, got, ref)
    ctl.close()


def test_publish_copies_the_written_plan():
    """Publish: after mpc_share_plans the read side of every arm's board holds
    exactly what ToPlan wrote (the plan in the paper's layout, transposed;
    the planned joints; the distance to goal sensed at that step; valid),
    and that plan matches the oracle's ToPlan on the GPU's updated means
    (1e-5 m, joints 2e-6)."""
    _say("case: publish, 3 arms with ragged rollouts and horizons")
    sc = small_scene(3, n=[64, 100, 128, 192], h=[8, 12, 12, 16])
    sc.arms, sc.state, sc.goal = sc.arms[:3], sc.state[:3], sc.goal[:3]
    ctl = native.Controller(sc.arms, sc.params)
    ctl.step(sc.state, sc.goal, _obs(sc))
    ctl.sync()
    for a in range(3):
        assert ctl.get_board(a)[3] == 0        # nothing published yet
    dist = [float(ctl.debug_get("DIST", a)[0]) for a in range(3)]
    ctl.share_plans()
    ctl.sync()
    for a in range(3):
        arm = sc.arms[a]
        plan, pq, mean = (x.cpu().numpy() for x in ctl.get_plan(a))        # [S][4][H], [H][7], [H][7]
        bplan, bpq, bdist, bvalid = ctl.get_board(a)
        bplan, bpq = bplan.cpu().numpy(), bpq.cpu().numpy()                 # [H][S][4], [H][7]
        assert bvalid == 1
        np.testing.assert_array_equal(bplan, np.transpose(plan, (2, 0, 1)))
        np.testing.assert_array_equal(bpq, pq)
        assert np.float32(bdist) == np.float32(dist[a])
        st = sc.state[a].astype(np.float64)
        q, _ = oracle.integrate(st[:, 0], st[:, 1], mean.astype(np.float64), f32(sc.params["dt"]))
        assert np.abs(bpq - q).max() < 2e-6
        oa = oracle.make_arm(arm)
        for h in range(arm.horizon):
            assert np.abs(bplan[h] - oracle.spheres(oa, q[h])).max() < 1e-5
    ctl.close()


def test_masked_publish_hides_the_withheld_arm():
    """A withheld arm stays invisible (Sec. IV-C: plans that were not
    published are ignored).  Three arms step; only arms 0 and 2 publish.  At
    the next step no arm sees arm 1 (priority factor 0, no distance queries
    against it), and the stage costs of arms 0 and 2 equal the oracle's with
    arm 1 inactive and the other arm's plan taken from what its ToPlan wrote
    (board inputs built without reading the board's read side).  The oracle controller with the same mask agrees on the flags
    and priority factors, and its costs equal those of an oracle controller
    that published every arm and then marked arm 1 invalid.  A second, full
    publish then makes arm 1 visible on the GPU."""
    _say("case: masked publish, 3 arms, arm 1 withheld")
    sc = small_scene(3, n=[64, 100, 128, 192], h=[8, 12, 12, 16])
    sc.arms, sc.state, sc.goal = sc.arms[:3], sc.state[:3], sc.goal[:3]
    mask = np.array([1, 0, 1], np.uint8)
    ctl = native.Controller(sc.arms, sc.params)
    ctl.step(sc.state, sc.goal, _obs(sc))
    ctl.sync()
    dist1 = [float(ctl.debug_get("DIST", a)[0]) for a in range(3)]
    # what ToPlan wrote (pinned to the oracle's ToPlan by the publish test)
    written = [np.transpose(ctl.get_plan(a)[0].cpu().numpy().astype(np.float64), (2, 0, 1)) for a in range(3)]
    ctl.share_plans(mask)
    ctl.debug_enable(True)
    ctl.step(sc.state, sc.goal, _obs(sc))
    ctl.sync()
    assert [ctl.get_board(a)[3] for a in range(3)] == [1, 0, 1]
    # board inputs built without the read side: the written plans, the mask's
    # validity and the distances sensed at step 1
    boards = [(written[i], int(mask[i]), dist1[i]) for i in range(3)]
    for a in (0, 2):
        cap = Capture(ctl, a)
        assert cap.alpha[1] == 0.0
        o = 2 - a
        al = oracle.priority(cap.dist, dist1[o], f32(3.0), f32(1e-3), f32(0.5), f32(2.0))
        assert abs(cap.alpha[o] - al) < 1e-5 * max(1.0, al)
        arm = sc.arms[a]
        expect = sum(arm.n_rollouts * arm.n_spheres * sc.arms[o].n_spheres
                     for h in range(arm.horizon) if h < sc.arms[o].horizon)
        assert cap.pairs == expect
        ref = oracle_stage(sc, a, cap, sc.obstacles, boards)
        assert rel_err(cap.stage, ref) < 1e-4
    # the oracle controller with the same mask
    orc = oracle.Controller(sc.arms, sc.params)
    orc.step(sc.state, sc.goal, sc.obstacles)
    orc.share_plans(mask)
    assert [orc.plan(i, 0)[3] for i in range(3)] == [1, 0, 1]
    orc.step(sc.state, sc.goal, sc.obstacles)
    al_o, _ = orc.alpha()
    assert al_o[0, 1] == 0.0 and al_o[2, 1] == 0.0 and al_o[0, 2] > 0.0
    orc2 = oracle.Controller(sc.arms, sc.params)
    orc2.step(sc.state, sc.goal, sc.obstacles)
    orc2.share_plans()
    p1, pq1, d1, _ = orc2.plan(1, 0)
    orc2.set_plan(1, p1, pq1, d1, 0)
    orc2.step(sc.state, sc.goal, sc.obstacles)
    for a in (0, 2):
        np.testing.assert_array_equal(orc.costs(a)[1], orc2.costs(a)[1])
    # full publish: arm 1 becomes visible at the next step
    ctl.share_plans()
    ctl.step(sc.state, sc.goal, _obs(sc))
    ctl.sync()
    assert ctl.get_board(1)[3] == 1
    assert float(ctl.debug_get("ALPHA", 0)[1]) > 0.0
    ctl.close()


@pytest.mark.parametrize("config", [1, 5])
def test_obstacles_at_the_buffer_edge_of_small_spheres(config):
    """The set filter gives every sphere of a body the body's largest radius;
    the pairs it must still catch are those of a body's smaller spheres right
    at the buffer edge.  Per body, one obstacle (r = 2 cm) sits at a gap of
    exactly B from a sphere at least 1 cm smaller than the body's largest, in
    a direction that leaves every other sphere of the arm at least 2 mm
    beyond the buffer at the start pose, so the sampled rollouts fall on both
    sides of the edge.  Stage costs match the oracle in every run, and the
    obstacle term is on for some rollout steps and off for others."""
    _say(f"case: an obstacle at the buffer edge of a small sphere of each body, arm of config {config}")
    sc = small_scene(config, n=128, h=10, collision_mode=0)
    sc.arms, sc.state, sc.goal = sc.arms[:1], sc.state[:1], sc.goal[:1]
    arm = sc.arms[0]
    sph = oracle.spheres(oracle.make_arm(arm), sc.state[0, :, 0].astype(np.float64))
    links = np.asarray(arm.sphere_link)
    B, r_obs = f32(sc.params["buf_env"]), 0.02

    def run(obstacles):
        ctl = native.Controller(sc.arms, sc.params)
        ctl.debug_enable(True)
        ctl.step(sc.state, sc.goal, obstacles)
        ctl.sync()
        cap = Capture(ctl, 0, want_spheres=obstacles is not None)
        if obstacles is not None:
            ref = oracle_stage(sc, 0, cap, obstacles, read_boards(ctl, sc))
            assert rel_err(cap.stage, ref) < 1e-4
        ctl.close()
        return cap.stage

    def placement(j):
        for d in dirs:
            p = sph[j, :3] + d * (sph[j, 3] + r_obs + B)
            gaps = np.linalg.norm(sph[:, :3] - p, axis=1) - sph[:, 3] - r_obs
            if np.all(np.delete(gaps, j) >= B + 0.002):
                return p
        return None

    i = np.arange(1024) + 0.5
    zs = 1.0 - 2.0 * i / 1024
    ang = np.pi * (1 + 5 ** 0.5) * i
    dirs = np.stack([np.sqrt(1 - zs * zs) * np.cos(ang), np.sqrt(1 - zs * zs) * np.sin(ang), zs], axis=1)
    free = run(None)
    on, off, placed = 0, 0, 0
    for b in sorted(set(links.tolist())):
        idx = np.nonzero(links == b)[0]
        small = [j for j in idx[np.argsort(sph[idx, 3])] if sph[j, 3] <= sph[idx, 3].max() - 0.01]
        p = next((x for x in map(placement, small) if x is not None), None)
        if p is None:
            continue
        placed += 1
        env = run(np.array([[*p, r_obs]], np.float32)) - free
        on += int(np.sum(env > 0))
        off += int(np.sum(env == 0))
    _say(f"  bodies with an obstacle placed: {placed}; rollout steps with the obstacle term on / off: {on} / {off}")
    assert placed >= 3
    assert on > 0 and off > 0
