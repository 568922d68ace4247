"""Throughput of the batched MR-STORM control step on one MI355X.

Workload: 8 arms in two facing rows of 4 (0.5 m pitch), 4096 rollouts x 40
horizon steps per arm, 64 collision spheres per arm, 20 moving obstacle
spheres, every arm scored against the 7 published neighbour plans (exact
coordination distances).  One step = Publish + mpc_step (Sense, Shift,
sampling, dynamics, kinematics, scoring, update, ToPlan, PickBest) + the
plant stand-in, on inputs already resident in HBM; obstacle positions for
every step are precomputed and uploaded before the timed region.

Prints one JSON line: rollout-steps/s, p50/p99 step latency, the roofline of
the fused rollout kernel (FP32 ALU bound, achieved algorithmic TFLOP/s over
its HIP-event-timed launches) and the CPU oracle baseline.  With the learned
arm-pair distance (unless --no-surrogate): the network trained on this
workload's arms, the same steps with the exact check only below the margin
(throughput, latency, speedup, share of exact checks skipped), and on the
4-arm scene the same comparison plus an audited closed loop of --audit-steps
steps that counts every query the network passed whose exact distance was
below the buffer or below zero.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2602_10114_amd import scenes  # noqa: E402  (seeded inputs; no GPU use at import)

METRIC = "rollout-steps/s (arms×rollouts×horizon) + p50/p99 step latency, exact vs surrogate"
FP32_PEAK_TFLOPS = 157.3  # MI355X FP32 vector, 256 CUs at 2.4 GHz
BF16_PEAK_TFLOPS = 2500.0  # MI355X dense bfloat16 MFMA
KERNEL_SOURCES = ["paper_2602_10114_amd/csrc/kernels.hip", "paper_2602_10114_amd/csrc/device.hpp",
                  "paper_2602_10114_amd/csrc/common.hpp"]
# HBM bytes per k_rollout launch on this workload, by waves per workgroup,
# from rocprofv3 FETCH_SIZE and WRITE_SIZE passes, each scaled by the same
# counter's reading for a 256 MiB device copy (fetch x2.000, write x1.000);
# valid only for the kernel sources with this digest (see
# profiles/k_rollout_cfg5_exact.md).
TRAFFIC = {"sources_sha256": "9ff49b4953348398",
           "bytes_per_launch": {1: 48041000, 2: 105265000, 4: 76774000}}


def traffic_bytes(waves):
    """HBM bytes per rollout launch of the instantiation with `waves` waves
    per workgroup from the recorded counters, or None when the kernel sources
    changed since they were taken (stale counters are never reported)."""
    if TRAFFIC["sources_sha256"] != sources_digest():
        return None
    return TRAFFIC["bytes_per_launch"].get(waves)


def sources_digest():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def summarize(trace_dir, fetch_dir, write_dir, steps):
    """Text summary of rocprofv3 output of `bench.py --steps <steps>`: per-kernel
    durations over the steady-state launches (the last 2*steps rollout
    launches: the timed and the event-bracketed passes) and HBM bytes per
    dispatch from the FETCH_SIZE / WRITE_SIZE passes scaled by the copy
    kernel's reading."""
    import csv
    import glob
    from collections import defaultdict
    out = []
    by = defaultdict(list)
    if trace_dir:
        tr = glob.glob(os.path.join(trace_dir, "*kernel_trace.csv"))[0]
        for r in csv.DictReader(open(tr)):
            name = r["Kernel_Name"].split("(")[0]
            by[name].append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
        out.append(f"kernel trace: {tr}")
        out.append(f"{'kernel':44s} {'calls':>6s} {'steady calls':>12s} {'steady avg us':>14s} {'min us':>9s} {'max us':>9s}")
    for name, v in sorted(by.items(), key=lambda kv: -sum(d for _, d in kv[1])):
        v.sort()
        steady = [d for _, d in v[-2 * steps:]] if "k_rollout" in name else [d for _, d in v[-steps:]]
        out.append(f"{name[:44]:44s} {len(v):6d} {len(steady):12d} {np.mean(steady) / 1e3:14.2f} "
                   f"{min(steady) / 1e3:9.2f} {max(steady) / 1e3:9.2f}")
    res = {}
    if fetch_dir and write_dir:
        for tag, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
            f = glob.glob(os.path.join(d, "*counter_collection.csv"))[0]
            rows = list(csv.DictReader(open(f)))
            per = defaultdict(list)
            for r in rows:
                if r["Counter_Name"] == tag:
                    per[r["Kernel_Name"].split("(")[0]].append((int(r["Dispatch_Id"]), float(r["Counter_Value"])))
            copy = max(per["__amd_rocclr_copyBuffer"], key=lambda x: x[1])[1]
            factor = (256 * 1024) / copy
            out.append(f"{tag}: {f}; 256 MiB copy reads {copy:.1f} KiB -> scale x{factor:.3f}")
            for name, v in sorted(per.items()):
                if name.startswith("mrs::") or "k_rollout" in name:
                    v.sort()
                    kib = v[-1][1]
                    res.setdefault(name, {})[tag] = kib * factor * 1024
                    out.append(f"  {name[:44]:44s} last dispatch {kib:12.1f} KiB -> {kib * factor * 1024 / 1e6:10.3f} MB")
        out.append("HBM bytes per dispatch (scaled FETCH + WRITE):")
        for name, v in res.items():
            out.append(f"  {name[:44]:44s} {(v.get('FETCH_SIZE', 0) + v.get('WRITE_SIZE', 0)) / 1e6:10.3f} MB")
    out.append(f"kernel sources sha256[:16] at summary time: {sources_digest()}")
    return "\n".join(out)


def summarize_pmc(pmc_dir):
    """Text summary of a rocprofv3 --pmc pass (CSV, each counter already summed
    over its instances): per kernel, the counters of its last dispatch and the
    MFMA busy share SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE / 8 XCDs x 1024
    SIMDs), GRBM_GUI_ACTIVE being the sum of the 8 XCDs' active cycles, and,
    where the VALU counters were taken, the active-lane share, the issue rates
    per SIMD and clock and the FP32 operations the instruction counts imply."""
    import csv
    import glob
    from collections import defaultdict
    f = glob.glob(os.path.join(pmc_dir, "*counter_collection.csv"))[0]
    per = defaultdict(lambda: defaultdict(dict))
    dur = {}
    for r in csv.DictReader(open(f)):
        per[r["Kernel_Name"].split("(")[0]][int(r["Dispatch_Id"])][r["Counter_Name"]] = float(r["Counter_Value"])
        if r.get("End_Timestamp"):
            dur[int(r["Dispatch_Id"])] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
    out = [f"counter collection: {f}"]
    for name, disp in sorted(per.items()):
        vals = disp[max(disp)]
        t = dur.get(max(disp), 0.0)
        out.append(f"{name[:60]} (dispatches {len(disp)}, last: {t * 1e6:.1f} us):")
        for c in sorted(vals):
            out.append(f"  {c:28s} {vals[c]:16.6g}")
        if "SQ_VALU_MFMA_BUSY_CYCLES" in vals and vals.get("GRBM_GUI_ACTIVE"):
            share = vals["SQ_VALU_MFMA_BUSY_CYCLES"] / (vals["GRBM_GUI_ACTIVE"] / 8 * 1024)
            out.append(f"  MFMA busy share             {share:16.4f}")
        if vals.get("SQ_ACTIVE_INST_VALU") and vals.get("SQ_THREAD_CYCLES_VALU"):
            util = vals["SQ_THREAD_CYCLES_VALU"] / (vals["SQ_ACTIVE_INST_VALU"] * 64)
            out.append(f"  VALU active-lane share      {util:16.4f}")
        # Clock cycles of the dispatch: the busy cycles of one XCD
        # (GRBM_GUI_ACTIVE sums the 8), else the duration at 2.4 GHz.
        cyc = vals["GRBM_GUI_ACTIVE"] / 8 if vals.get("GRBM_GUI_ACTIVE") else t * 2.4e9
        if vals.get("SQ_INSTS_VALU") and cyc > 0:
            # wave-level VALU instructions per SIMD per clock (1024 SIMDs);
            # non-packed FP32 FMA on 16 lanes caps FMAs at 0.25
            rate = vals["SQ_INSTS_VALU"] / (1024 * cyc)
            out.append(f"  VALU wave-insts/SIMD-cycle  {rate:16.4f}")
        if "SQ_INSTS_VALU_FMA_F32" in vals:
            ops = 64 * (2 * vals["SQ_INSTS_VALU_FMA_F32"] + vals.get("SQ_INSTS_VALU_ADD_F32", 0)
                        + vals.get("SQ_INSTS_VALU_MUL_F32", 0) + vals.get("SQ_INSTS_VALU_TRANS_F32", 0))
            out.append(f"  FP32 VALU ops (64 lanes)    {ops:16.6g}")
            if cyc > 0:
                out.append(f"  FP32 VALU TFLOP/s at 2.4 GHz {ops / (cyc / 2.4e9) / 1e12:15.4f}")
                fma = vals["SQ_INSTS_VALU_FMA_F32"] / (1024 * cyc)
                out.append(f"  FMA wave-insts/SIMD-cycle   {fma:16.4f}")
            if vals.get("SQ_INSTS_VALU"):
                share = (vals["SQ_INSTS_VALU_FMA_F32"] + vals.get("SQ_INSTS_VALU_ADD_F32", 0)
                         + vals.get("SQ_INSTS_VALU_MUL_F32", 0) + vals.get("SQ_INSTS_VALU_TRANS_F32", 0)) / vals["SQ_INSTS_VALU"]
                out.append(f"  FP32 share of VALU insts    {share:16.4f}")
    return "\n".join(out)


WMEAN_SIZES = (4096, 8192, 16384)


def summarize_sizes(trace_dir):
    """The weighted mean's launch time per problem size from a trace of
    `bench.py --wmean-sizes`: the launches of each size are told apart by
    their grid (one block per 1024-rollout chunk, step and arm), the median
    of each size is taken, and the bytes it reads (the noise of every arm,
    step and joint) give its rate and the marginal rate between sizes."""
    import csv
    import glob
    from collections import defaultdict
    tr = glob.glob(os.path.join(trace_dir, "*kernel_trace.csv"))[0]
    by = defaultdict(list)
    for r in csv.DictReader(open(tr)):
        if "k_wmean" in r["Kernel_Name"] and "fin" not in r["Kernel_Name"]:
            blocks = int(r["Grid_Size_X"]) // int(r["Workgroup_Size_X"])
            by[blocks].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    out = [f"kernel trace: {tr}", f"{'rollouts/arm':>12s} {'MB read':>8s} {'launches':>8s} {'median us':>10s} {'TB/s':>6s}"]
    prev = None
    for n in WMEAN_SIZES:
        blocks = -(-n // 1024)
        v = sorted(by.get(blocks, []))
        if not v:
            continue
        t = v[len(v) // 2] / 1e3
        mb = 8 * 40 * 7 * n * 4 / 1e6
        line = f"{n:12d} {mb:8.1f} {len(v):8d} {t:10.2f} {mb / t:6.2f}"
        if prev:
            line += f"   marginal {(mb - prev[0]) / (t - prev[1]):.2f} TB/s"
        out.append(line)
        prev = (mb, t)
    return "\n".join(out)


def algorithmic_flops_per_step(scene, active_neighbours=True):
    """Algorithmic work of one rollout launch: 11 FLOP per sphere pair (3 sub,
    5 for the dot product, sqrt, minus radii, min) plus the per rollout-step
    base 4d (sampling and integration) + 8*63 (frame composition) + 18 S
    (sphere placement) + 30 (pose) + 7 d (stop and joint limits)."""
    total = 0
    d = 7
    O = scene.obstacles.shape[0]
    for a, arm in enumerate(scene.arms):
        L = arm.sphere_link
        S = arm.n_spheres
        self_pairs = int(sum(1 for s in range(S) for t in range(s + 1, S) if abs(int(L[s]) - int(L[t])) >= 2))
        base = 4 * d + 8 * 63 + 18 * S + 30 + 7 * d
        for h in range(arm.horizon):
            dyn = 0
            if active_neighbours:
                dyn = sum(S * b.n_spheres for i, b in enumerate(scene.arms) if i != a and h < b.horizon)
            total += arm.n_rollouts * (11 * (self_pairs + S * O + dyn) + base)
    return total * int(scene.params["iters"])


def _oracle_window_step(args):
    """One control step of the oracle on rollouts [lo, hi) of every arm, after
    an untimed step that publishes plans; returns (start, end) wall times."""
    config, lo, hi = args
    import oracle
    scene = scenes.make_scene(config, collision_mode=0)
    orc = oracle.Controller(scene.arms, scene.params)
    orc.set_window(0, 1)
    orc.step(scene.state, scene.goal, scene.obstacles)
    orc.share_plans()
    orc.set_window(lo, hi)
    t0 = time.time()
    orc.step(scene.state, scene.goal, scene.obstacles)
    return t0, time.time()


def host_info():
    """The host the CPU baseline runs on: logical CPUs the OS reports, the
    CPUs this process may use, and the CPU model."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "cpu_model": model}


def cpu_baseline(scene):
    """The FP64 oracle, as it stands, on the host cores, on bounded samples of
    one control step: (1) one thread on the first 320 rollouts of every arm;
    (2) the first 640 rollouts of every arm split over worker processes, one
    per core this process may use, at most 16,
    each running the unmodified oracle on a disjoint rollout window; value =
    rollout-steps / wall time of (2).  The host's CPU count and model are
    recorded with it."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    window = 320
    t0, t1 = _oracle_window_step((5, 0, window))
    rs1 = window * sum(a.horizon for a in scene.arms)
    single = {"value": rs1 / (t1 - t0), "cores": 1,
              "sample": f"first {window} of 4096 rollouts of every arm, {t1 - t0:.1f} s"}
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    N = 640
    bounds = [(5, N * i // cores, N * (i + 1) // cores) for i in range(cores)]
    # (a worker that dies raises BrokenProcessPool here rather than hanging)
    with ProcessPoolExecutor(max_workers=cores, mp_context=mp.get_context("spawn")) as ex:
        spans = list(ex.map(_oracle_window_step, bounds, timeout=600))
    wall = max(e for _, e in spans) - min(b for b, _ in spans)
    rs = N * sum(a.horizon for a in scene.arms)
    return {"value": rs / wall, "unit": "rollout-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"one control step of all 8 arms restricted to their first {N} of 4096 rollouts "
                      f"({rs} rollout-steps, FP64), split into {cores} rollout windows run by {cores} "
                      f"processes in {wall:.1f} s",
            "host": host_info(), "single_thread": single}


def obstacle_track(scene, n):
    """Obstacle positions for n consecutive control steps (scene is advanced)."""
    out = []
    for _ in range(n):
        out.append(scene.obstacles.copy())
        scenes.move_obstacles(scene, float(scene.params["dt"]))
    return np.stack(out)


# Closed-loop control steps of each benchmark workload, keyed by the scene
# number of scenes.make_scene; the one-arm workload is a single control step,
# timed here over 200 repetitions.
CONFIG_STEPS = {1: 200, 2: 200, 3: 500, 4: 1000, 5: 1000}


def goal_schedule(scene, steps, goal_age=50):
    """Goals of `steps` consecutive control steps, [steps][A][7]: each arm's
    goal re-drawn every goal_age steps (one second at dt = 0.02 s, the
    reaching task's time-out of Sec. V-A), staggered over the arms."""
    A = scene.n_arms
    rng = np.random.default_rng(scene.seed + 99)
    age = np.arange(A) * (goal_age // A)
    out = []
    for _ in range(steps):
        m = scenes.reset_goals(scene, rng, np.full(A, np.inf), age, max_age=goal_age)
        age = np.where(m, 0, age + 1)
        out.append(scene.goal.copy())
    return np.stack(out)


def latency_leg(config, steps, dev, stream, params=None, warmup=10, screen=0.0, probe=0, min_drop=0.0):
    """The workload's own closed loop (Publish + mpc_step + plant) for
    `steps` control steps after `warmup`, goals re-drawn every second and
    obstacles moving, every input resident in HBM (goal and obstacle
    sequences uploaded beforehand): per-step HIP-event latency p50 / p99 and
    the rollout-steps/s of the mean step.  params: learned distance on."""
    import torch
    from paper_2602_10114_amd import native
    sc = scenes.make_scene(config, collision_mode=0)
    goals = torch.as_tensor(goal_schedule(scenes.make_scene(config, collision_mode=0), warmup + steps), device=dev)
    obs = None
    if sc.obstacles.shape[0]:
        obs = torch.as_tensor(obstacle_track(scenes.make_scene(config, collision_mode=0), warmup + steps), device=dev)
    ctl = native.Controller(sc.arms, {**sc.params, "surrogate_screen": screen, "surrogate_probe": probe,
                                      "surrogate_min_drop": min_drop}, stream=stream)
    if params is not None:
        ctl.set_surrogate_params(params)
        ctl.set_collision_mode(1)
    with torch.cuda.stream(stream):
        state = torch.as_tensor(sc.state, device=dev).contiguous()
        u = torch.zeros((sc.n_arms, 7), dtype=torch.float32, device=dev)

        def one(k):
            ctl.share_plans()
            ctl.step(state, goals[k], obs[k] if obs is not None else None, u_out=u)
            ctl.sim_execute(state, u)

        for k in range(warmup):
            one(k)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        for i in range(steps):
            ev[i][0].record(stream)
            one(warmup + i)
            ev[i][1].record(stream)
        stream.synchronize()
    lat = np.array([a.elapsed_time(b) for a, b in ev])
    tuning = list(ctl.tuning())
    stats = ctl.surrogate_stats() if params is not None else None
    ctl.close()
    out = {"config": config, "mode": "learned" if params is not None else "exact", "steps": steps,
           "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
           "mean_ms": float(lat.mean()), "max_ms": float(lat.max()),
           "rollout_steps_per_s": sc.rollout_steps() / (lat.mean() * 1e-3), "tuning": tuning}
    if stats is not None:
        q = max(stats["queries"], 1)
        out.update({"screen_m": screen, "probe": probe, "min_drop": min_drop,
                    "exact_checks_skipped": stats["waves_skipped"] * 64 / q,
                    "queries_through_network": stats["network_rows"] / q})
    return out


def timed_loop(ctl, scene, stream, steps, warmup, mode, dev, replay=None):
    """Closed-loop control steps (Publish + mpc_step + plant) on inputs resident
    in HBM; returns wall seconds of the timed steps, per-step latencies (ms)
    from HIP events, and the rollout-kernel event time per launch.  The
    rollout launches are timed with HIP events around each launch, which
    turns the step's graph off, so in a leg of their own: with `replay` (a
    function of the chosen tuning that returns a fresh controller) the same
    warm-up and timed steps again from the same start, so the events time the
    launches of the timed steps themselves; without it the next `steps`
    steps of the loop."""
    import torch
    A = scene.n_arms
    obs = torch.as_tensor(obstacle_track(scene, warmup + 2 * steps), device=dev)
    with torch.cuda.stream(stream):
        state = torch.as_tensor(scene.state, device=dev).contiguous()
        goal = torch.as_tensor(scene.goal, device=dev).contiguous()
        u = torch.zeros((A, 7), dtype=torch.float32, device=dev)
        ctl.set_collision_mode(mode)
        k = 0

        def one_step(c):
            nonlocal k
            c.share_plans()
            c.step(state, goal, obs[k], u_out=u)
            c.sim_execute(state, u)
            k += 1

        for _ in range(warmup):
            one_step(ctl)
        stream.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        ctl.surrogate_stats(reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            ev[i][0].record(stream)
            one_step(ctl)
            ev[i][1].record(stream)
        stream.synchronize()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        stats = ctl.surrogate_stats()
        lat = np.array([a.elapsed_time(b) for a, b in ev])
        pc = ctl
        if replay is not None:
            pc = replay(ctl.tuning())
            pc.set_collision_mode(mode)
            state.copy_(torch.as_tensor(scene.state, device=dev))
            u.zero_()
            k = 0
            for _ in range(warmup):
                one_step(pc)
        pc.profile_enable(True)
        for i in range(steps):
            one_step(pc)
        ms_roll, n_roll = pc.profile_read()
        ms_inf, n_inf = pc.profile_read_surrogate()
        pc.profile_enable(False)
        stream.synchronize()
        if pc is not ctl:
            pc.close()
    stats["infer_ms"] = ms_inf / n_inf if n_inf else None
    return wall, lat, ms_roll / max(n_roll, 1), stats


def audit_run(scene, params, steps, dev, goal_age=50, screen=0.0, probe=0, min_drop=0.0):
    """Closed loop with goals reset every goal_age steps (staggered per arm)
    so that the arms keep crossing the shared workspace.  With params: the
    learned distance, audited (the dropped checks are also computed exactly):
    counts of dropped queries whose exact distance is below buf_dyn (misses)
    or below zero (missed collisions).  Without: the exact controller on the
    same goal sequence.  Both report the smallest exact gap between the arms
    as executed."""
    import torch
    from paper_2602_10114_amd import native
    A = scene.n_arms
    rng = np.random.default_rng(scene.seed + 99)
    ctl = native.Controller(scene.arms, {**scene.params, "collision_mode": 0, "surrogate_screen": screen,
                                         "surrogate_probe": probe, "surrogate_min_drop": min_drop})
    if params is not None:
        ctl.set_surrogate_params(params)
        ctl.set_collision_mode(1)
        ctl.surrogate_audit(True)
    state = torch.as_tensor(scene.state, device=dev).contiguous()
    goal = torch.as_tensor(scene.goal, device=dev).contiguous()
    u = torch.zeros((A, 7), dtype=torch.float32, device=dev)
    age = np.arange(A) * (goal_age // A)
    qs = torch.empty((steps, A, 7), dtype=torch.float32, device=dev)
    t0 = time.perf_counter()
    for k in range(steps):
        m = scenes.reset_goals(scene, rng, np.full(A, np.inf), age, max_age=goal_age)
        age = np.where(m, 0, age + 1)
        if m.any():
            goal.copy_(torch.as_tensor(scene.goal))
        ctl.share_plans()
        ctl.step(state, goal, scene.obstacles, u_out=u)
        ctl.sim_execute(state, u)
        qs[k].copy_(state[:, :, 0])
        scenes.move_obstacles(scene, float(scene.params["dt"]))
        if (k + 1) % 2000 == 0:
            print(f"bench: audit step {k + 1}/{steps}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = ctl.surrogate_stats()
    gap, first = np.inf, None
    for i in range(A):
        for j in range(i + 1, A):
            gij = ctl.pair_distance(i, j, qs[:, i].contiguous(), qs[:, j].contiguous()).cpu().numpy()
            gap = min(gap, float(gij.min()))
            neg = np.nonzero(gij < 0)[0]
            if neg.size and (first is None or neg[0] < first["step"]):
                first = {"step": int(neg[0]), "arms": [i, j], "gap_m": float(gij[neg[0]])}
    ctl.close()
    return {"steps": steps, "queries": st["queries"], "predicted_far": st["predicted_far"],
            "misses_below_buffer": st["misses"], "missed_collisions": st["missed_collisions"],
            "executed_min_arm_gap_m": gap, "first_executed_contact": first, "seconds": wall}


def ablation_run(variant, steps, dev, seed=None):
    """Closed loop on the two facing arms (0.8 m apart, goals drawn in the
    shared middle region): MR-STORM (tau = 3, shared plans), M_tau (tau = 0:
    no priority) or S_d (no plans: each arm sees the other's current spheres
    as a static obstacle).  Goals are re-drawn when reached (5 cm) or after
    150 steps (3 s).  Returns goals reached and their mean time, steps where
    both arms are stalled away from their goals (joint speed below 0.05
    rad/s, more than 10 cm from the goal: the livelock signature), and the
    smallest executed gap after the first step (the start pose is shared)."""
    import torch
    from paper_2602_10114_amd import native
    over = {"M": {}, "M_tau": {"tau": 0.0}, "S_d": {"plan_mode": 1}}[variant]
    sc = scenes.make_scene(2, seed=seed, collision_mode=0, **over)
    A = sc.n_arms
    rng = np.random.default_rng(sc.seed + 7)
    ctl = native.Controller(sc.arms, sc.params)
    state = torch.as_tensor(sc.state, device=dev).contiguous()
    u = torch.zeros((A, 7), dtype=torch.float32, device=dev)
    age = np.zeros(A, dtype=int)
    reached, stalled, t_reach = 0, 0, []
    qs = torch.empty((steps, A, 7), dtype=torch.float32, device=dev)
    for k in range(steps):
        ctl.share_plans()
        ctl.step(state, sc.goal, None, u_out=u)
        ctl.sim_execute(state, u)
        qs[k].copy_(state[:, :, 0])
        dist = np.array([float(ctl.debug_get("DIST", a)[0]) for a in range(A)])
        speed = state[:, :, 1].abs().max(dim=1).values.cpu().numpy()
        if np.all((speed < 0.05) & (dist > 0.10)):
            stalled += 1
        m = scenes.reset_goals(sc, rng, dist, age, tol=0.05, max_age=150)
        hit = m & (dist < 0.05)
        reached += int(np.sum(hit))
        t_reach += [int(age[a]) + 1 for a in np.nonzero(hit)[0]]
        age = np.where(m, 0, age + 1)
    gaps = ctl.pair_distance(0, 1, qs[:, 0].contiguous(), qs[:, 1].contiguous())
    ctl.close()
    return {"goals_reached": reached, "steps_to_goal": t_reach,
            "stalled_steps": stalled, "executed_min_arm_gap_m": float(gaps[1:].min()),
            "start_gap_m": float(gaps[0]), "steps": steps}


def ablation(steps, seeds, dev):
    """The three variants over the same scene seeds (start poses, goal
    sequences, sphere radii): goals per seed, their total, the pooled mean
    time to goal, stalled steps and the smallest executed gap."""
    base = scenes.make_scene(2).seed
    seed_list = [base + 100 * i for i in range(seeds)]
    out = {"seeds": seed_list, "steps_per_seed": steps}
    for v in ("M", "M_tau", "S_d"):
        runs = [ablation_run(v, steps, dev, seed=sd) for sd in seed_list]
        t = [x for r in runs for x in r["steps_to_goal"]]
        out[v] = {"goals_per_seed": [r["goals_reached"] for r in runs],
                  "goals_total": int(sum(r["goals_reached"] for r in runs)),
                  "mean_steps_to_goal": float(np.mean(t)) if t else None,
                  "stalled_steps": int(sum(r["stalled_steps"] for r in runs)),
                  "executed_min_arm_gap_m": min(r["executed_min_arm_gap_m"] for r in runs),
                  "start_gap_m": min(r["start_gap_m"] for r in runs)}
    return out


def fig1_run(variant, steps, dev, seed, goal=(0.0, 0.0, 0.35)):
    """The livelock scenario of Fig. 1 (Sec. IV-B): two arms facing each
    other 0.8 m apart reach for the same goal point between them, tool
    pointing down.  An arm that arrives (5 cm) then leaves for a waiting
    point beside its own base, which frees the goal for the other.  Per
    step: each arm's distance to its goal; "withdrawals" are steps at which
    both arms, both more than 10 cm from the shared goal, move away from it
    by more than 1 mm (the retreat of Fig. 1 D.1), counted as episodes of
    consecutive such steps; "stalled" steps have both arms slow (joint speed
    below 0.05 rad/s) and away from their goals."""
    import torch
    from paper_2602_10114_amd import native
    over = {"M": {}, "M_tau": {"tau": 0.0}, "S_d": {"plan_mode": 1}}[variant]
    sc = scenes.make_scene(2, seed=seed, collision_mode=0, **over)
    down = np.array([0.0, 1.0, 0.0, 0.0], np.float32)          # w, x, y, z: tool along -z
    shared = np.concatenate([np.array(goal, np.float32), down])
    wait = [np.concatenate([np.array([-0.35, 0.35, 0.5], np.float32), down]),
            np.concatenate([np.array([0.35, -0.35, 0.5], np.float32), down])]
    goals = np.stack([shared, shared]).astype(np.float32)
    ctl = native.Controller(sc.arms, sc.params)
    state = torch.as_tensor(sc.state, device=dev).contiguous()
    g = torch.as_tensor(goals, device=dev).contiguous()
    u = torch.zeros((2, 7), dtype=torch.float32, device=dev)
    reached = [None, None]
    prev = None
    withdraw_steps = withdraw_episodes = stalled = 0
    in_episode = False
    qs = torch.empty((steps, 2, 7), dtype=torch.float32, device=dev)
    for k in range(steps):
        ctl.share_plans()
        ctl.step(state, g, None, u_out=u)
        ctl.sim_execute(state, u)
        qs[k].copy_(state[:, :, 0])
        dist = np.array([float(ctl.debug_get("DIST", a)[0]) for a in range(2)])
        speed = state[:, :, 1].abs().max(dim=1).values.cpu().numpy()
        to_shared = [dist[a] if reached[a] is None else np.inf for a in range(2)]
        if prev is not None and reached[0] is None and reached[1] is None:
            back = all(to_shared[a] > 0.10 and dist[a] > prev[a] + 1e-3 for a in range(2))
            withdraw_steps += back
            withdraw_episodes += back and not in_episode
            in_episode = back
        if np.all((speed < 0.05) & (dist > 0.10)):
            stalled += 1
        for a in range(2):
            if reached[a] is None and dist[a] < 0.05:
                reached[a] = k + 1
                goals[a] = wait[a]
                g.copy_(torch.as_tensor(goals))
        prev = dist
        if reached[0] is not None and reached[1] is not None:
            break
    gaps = ctl.pair_distance(0, 1, qs[:k + 1, 0].contiguous(), qs[:k + 1, 1].contiguous())
    ctl.close()
    order = sorted(r for r in reached if r is not None)
    return {"first_arrival": order[0] if order else None, "both_arrived": order[1] if len(order) == 2 else None,
            "withdraw_steps": withdraw_steps, "withdraw_episodes": withdraw_episodes, "stalled_steps": stalled,
            "executed_min_arm_gap_m": float(gaps[1:].min()), "steps_run": k + 1}


def fig1(steps, seeds, dev):
    """Fig. 1's shared-goal scenario over several scene seeds (start poses,
    noise) for MR-STORM (tau = 3), M_tau (tau = 0) and S_d (no plans)."""
    base = scenes.make_scene(2).seed
    seed_list = [base + 100 * i for i in range(seeds)]
    out = {"seeds": seed_list, "max_steps": steps}
    for v in ("M", "M_tau", "S_d"):
        runs = [fig1_run(v, steps, dev, sd) for sd in seed_list]
        out[v] = {"runs": runs,
                  "both_arrived": sum(r["both_arrived"] is not None for r in runs),
                  "mean_first_arrival": float(np.mean([r["first_arrival"] for r in runs if r["first_arrival"]]))
                  if any(r["first_arrival"] for r in runs) else None,
                  "withdraw_episodes": int(sum(r["withdraw_episodes"] for r in runs)),
                  "withdraw_steps": int(sum(r["withdraw_steps"] for r in runs)),
                  "stalled_steps": int(sum(r["stalled_steps"] for r in runs)),
                  "executed_min_arm_gap_m": min(r["executed_min_arm_gap_m"] for r in runs)}
    m, mt = out["M"], out["M_tau"]
    out["priority_resolves_livelock"] = bool(m["withdraw_episodes"] < mt["withdraw_episodes"] and
                                             m["both_arrived"] >= mt["both_arrived"])
    return out


SCREEN_SWEEP = (0.0, 0.1, 0.2, 0.3, 0.4, 0.6)
# Drop-history screen of the learned legs: a group that dropped at most a
# share min_drop of its checks in the last control step skips the network,
# re-probed every 8th step; min_drop is picked from MIN_DROP_SWEEP on the
# first 300 steps of the workload's closed loop (goals re-drawn).
SURROGATE_PROBE = 8
MIN_DROP_SWEEP = (0.0, 0.25, 0.5, 0.75)


def min_drop_sweep(config, params, screen, dev, stream, steps=300):
    """Mean learned step time (ms) of the closed loop with goals re-drawn
    for each min_drop of MIN_DROP_SWEEP; returns the sweep and the fastest."""
    out = {m: latency_leg(config, steps, dev, stream, params=params, screen=screen, probe=SURROGATE_PROBE,
                          min_drop=m)["mean_ms"] for m in MIN_DROP_SWEEP}
    return out, min(out, key=out.get)


def screen_sweep(config, params, stream, dev, steps, warmup, probe=SURROGATE_PROBE, pair_cull=1):
    """Learned step time (ms) for each screen distance of SCREEN_SWEEP (the
    mean-rollout distance below which an arm-neighbour-step group skips the
    network and is checked exactly); returns the sweep and the fastest."""
    from paper_2602_10114_amd import native
    out = {}
    for tau in SCREEN_SWEEP:
        sc = scenes.make_scene(config, collision_mode=0)
        ctl = native.Controller(sc.arms, {**sc.params, "surrogate_screen": tau, "surrogate_probe": probe,
                                          "pair_cull": pair_cull}, stream=stream)
        ctl.set_surrogate_params(params)
        w, _, _, _ = timed_loop(ctl, sc, stream, steps, warmup, 1, dev)
        ctl.close()
        out[tau] = 1e3 * w / steps
    return out, min(out, key=out.get)


def all_pairs_leg(out, params, md5, stream, dev, args):
    """The 8-arm exact and learned steps with the pair cull off (every sphere
    pair through the filter, as in the paper's exact check), the screen
    distance swept for that setting; adds out["surrogate"]["all_pairs"]."""
    from paper_2602_10114_amd import native
    sweep3, tau3 = screen_sweep(5, params, stream, dev, max(5, args.steps // 2), args.warmup, pair_cull=0)
    scene3 = scenes.make_scene(5, collision_mode=0)
    ctl3 = native.Controller(scene3.arms, {**scene3.params, "collision_mode": 0, "surrogate_screen": tau3,
                                           "surrogate_probe": SURROGATE_PROBE, "surrogate_min_drop": md5,
                                           "pair_cull": 0}, stream=stream)
    ctl3.set_surrogate_params(params)
    w3e, _, roll3e, _ = timed_loop(ctl3, scenes.make_scene(5, collision_mode=0), stream, args.steps,
                                   args.warmup, 0, dev)
    w3l, _, roll3l, _ = timed_loop(ctl3, scenes.make_scene(5, collision_mode=0), stream, args.steps,
                                   args.warmup, 1, dev)
    ctl3.close()
    out["surrogate"]["all_pairs"] = {
        "exact_ms_per_step": 1e3 * w3e / args.steps, "learned_ms_per_step": 1e3 * w3l / args.steps,
        "speedup_vs_exact": w3e / w3l, "exact_rollout_kernel_ms": roll3e,
        "learned_rollout_kernel_ms": roll3l, "screen_m": tau3,
        "screen_sweep_ms": {str(k): v for k, v in sweep3.items()}}
    print(f"bench: pair cull off: exact {1e3 * w3e / args.steps:.3f} ms, learned {1e3 * w3l / args.steps:.3f} ms",
          file=sys.stderr, flush=True)


def train_surrogate(scene):
    from paper_2602_10114_amd import native
    ctl = native.Controller(scene.arms, {**scene.params, "collision_mode": 0})
    rep = ctl.surrogate_train(**native.TRAINING_RECIPE)
    params = ctl.surrogate_params().clone()
    ctl.close()
    return params, rep


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the learned-distance legs")
    ap.add_argument("--audit-steps", type=int, default=10000,
                    help="closed-loop steps of the audited learned-distance runs on the 8-arm and 4-arm scenes "
                         "(0: skip)")
    ap.add_argument("--no-latency", action="store_true",
                    help="skip the per-workload latency legs (each workload's own closed-loop step count)")
    ap.add_argument("--fig1-steps", type=int, default=600,
                    help="step limit of each run of the Fig. 1 shared-goal scenario (0: skip)")
    ap.add_argument("--fig1-seeds", type=int, default=5)
    ap.add_argument("--ablation-steps", type=int, default=1500,
                    help="closed-loop steps of each variant of the two-arm ablation (0: skip)")
    ap.add_argument("--ablation-seeds", type=int, default=5,
                    help="scene seeds of the two-arm ablation (start poses, goals, noise)")
    ap.add_argument("--summarize", nargs=3, metavar=("TRACE_DIR", "FETCH_DIR", "WRITE_DIR"),
                    help="print a summary of rocprofv3 output of a bench run and exit")
    ap.add_argument("--summarize-pmc", metavar="PMC_DIR",
                    help="print a summary of a rocprofv3 --pmc pass (per-kernel counters, MFMA busy share) and exit")
    ap.add_argument("--no-all-pairs", action="store_true",
                    help="skip the legs with the pair cull off (the all-pairs check)")
    ap.add_argument("--tuning", metavar="R,T,G",
                    help="exact leg: fix the rollout launch (rollouts per workgroup, horizon tile, grid) "
                         "instead of tuning it, e.g. for counter runs at the tuner's usual pick")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (reference kernel for HBM byte counters) and "
                         "a plain sum over the weighted mean's bytes (read-only reference rate)")
    ap.add_argument("--screen", type=float, default=None,
                    help="learned legs: this screen distance instead of the sweep")
    ap.add_argument("--min-drop", type=float, default=None,
                    help="learned legs: this drop-history share instead of the sweep")
    ap.add_argument("--no-4arm", action="store_true", help="skip the 4-arm learned-distance legs")
    ap.add_argument("--wmean-sizes", action="store_true",
                    help="also run the 8-arm workload at 8192 and 16384 rollouts per arm (weighted-mean size sweep)")
    ap.add_argument("--summarize-sizes", metavar="TRACE_DIR",
                    help="print the weighted mean's launch time per size from a trace of --wmean-sizes and exit")
    args = ap.parse_args()
    if args.summarize:
        print(summarize(*args.summarize, steps=args.steps))
        return
    if args.summarize_pmc:
        print(summarize_pmc(args.summarize_pmc))
        return
    if args.summarize_sizes:
        print(summarize_sizes(args.summarize_sizes))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the multi-GPU plan all-gather "
                                   "is a design, not a runnable path (--gpus 1)"}))
        sys.exit(2)

    import torch
    from paper_2602_10114_amd import native

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    stream = torch.cuda.Stream()
    scene = scenes.make_scene(5, collision_mode=0)
    ctl = native.Controller(scene.arms, scene.params, stream=stream)
    if args.tuning:
        ctl.set_tuning(*[int(x) for x in args.tuning.split(",")])

    def fresh(tuning):
        c = native.Controller(scene.arms, scene.params, stream=stream)
        c.set_tuning(*tuning)
        return c

    wall, lat, roll_ms, _ = timed_loop(ctl, scene, stream, args.steps, args.warmup, 0, dev, replay=fresh)
    tuning = list(ctl.tuning())
    print(f"bench: exact {args.steps} steps in {wall:.3f} s, tuning {tuning}", file=sys.stderr, flush=True)
    scene = scenes.make_scene(5, collision_mode=0)
    rs_per_step = scene.rollout_steps()
    flops = algorithmic_flops_per_step(scene)
    achieved = flops / (roll_ms * 1e-3) / 1e12
    out = {
        "metric": METRIC,
        "value": rs_per_step / (wall / args.steps),
        "unit": "rollout-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "8 arms (two facing rows of 4, 0.5 m pitch) x 4096 rollouts x 40 steps, "
                               "64 spheres/arm, 20 moving obstacles, exact coordination distances, K=1",
                   "arms": scene.n_arms, "rollouts": 4096, "horizon": 40, "spheres": 64, "obstacles": 20,
                   "mode": "exact", "tuning": tuning},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "mean": float(lat.mean())},
        "roofline": {"kernel": "k_rollout", "bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS,
                     "traffic": traffic_bytes(tuning[0] // 64),
                     "kernel_ms": roll_ms, "algorithmic_flop_per_launch": flops,
                     "note": "the model counts 11 FLOP for every sphere pair; the bounding-sphere cull "
                             "evaluates only the pairs that can be within the buffer, so the algorithmic "
                             "rate exceeds the peak (frac > 1)"},
    }
    if not args.no_surrogate:
        # Learned arm-pair distance on the same workload: exact check only
        # below the margin, same inputs and step count.
        params, rep = train_surrogate(scenes.make_scene(5, collision_mode=0))
        print(f"bench: surrogate trained in {rep['seconds']:.1f} s", file=sys.stderr, flush=True)
        if args.screen is None:
            sweep5, tau5 = screen_sweep(5, params, stream, dev, max(5, args.steps // 2), args.warmup)
            print(f"bench: screen sweep {sweep5} -> {tau5}", file=sys.stderr, flush=True)
        else:
            sweep5, tau5 = {}, args.screen
        if args.min_drop is None:
            drops5, md5 = min_drop_sweep(5, params, tau5, dev, stream)
            print(f"bench: min_drop sweep {drops5} -> {md5}", file=sys.stderr, flush=True)
        else:
            drops5, md5 = {}, args.min_drop
        scene = scenes.make_scene(5, collision_mode=0)
        learned_params = {**scene.params, "collision_mode": 0, "surrogate_screen": tau5,
                          "surrogate_probe": SURROGATE_PROBE, "surrogate_min_drop": md5}

        def fresh_learned(tuning=None):
            c = native.Controller(scene.arms, learned_params, stream=stream)
            c.set_surrogate_params(params)
            if tuning is not None:
                c.set_tuning(*tuning)
            return c

        ctl2 = fresh_learned()
        w2, lat2, roll2, st = timed_loop(ctl2, scene, stream, args.steps, args.warmup, 1, dev,
                                         replay=fresh_learned)
        ctl2.close()
        q = max(st["queries"], 1)
        # Inference roofline: every query row the network runs (the screened
        # groups' queries run none) costs its multiply-adds
        # (17*256 + 2*256*256 + 256) x 2 FLOP.
        rows_per_launch = st["network_rows"] / args.steps
        mlp_flops = rows_per_launch * 2 * (17 * 256 + 2 * 256 * 256 + 256)
        inf_ach = mlp_flops / (st["infer_ms"] * 1e-3) / 1e12
        out["surrogate"] = {
            "value": rs_per_step / (w2 / args.steps), "unit": "rollout-steps/s",
            "ms_per_step": 1e3 * w2 / args.steps, "speedup_vs_exact": wall / w2,
            "latency_ms": {"p50": float(np.percentile(lat2, 50)), "p99": float(np.percentile(lat2, 99))},
            "rollout_kernel_ms": roll2, "queries_predicted_far": st["predicted_far"] / q,
            "queries_through_network": st["network_rows"] / q,
            "roofline": {"kernel": "k_sur_infer", "bound": "mfma", "achieved": inf_ach, "peak": BF16_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": inf_ach / BF16_PEAK_TFLOPS, "traffic": None,
                         "kernel_ms": st["infer_ms"], "algorithmic_flop_per_launch": mlp_flops},
            "exact_checks_skipped": st["waves_skipped"] * 64 / q,
            "screen_m": tau5, "probe": SURROGATE_PROBE, "min_drop": md5,
            "screen_sweep_ms": {str(k): v for k, v in sweep5.items()},
            "min_drop_sweep_mean_ms": {str(k): v for k, v in drops5.items()},
            "train": {k: (round(v, 5) if isinstance(v, float) else v) for k, v in rep.items()},
            "recipe": native.TRAINING_RECIPE,
        }
        # The paper's exact check has no broad phase: the same two steps with
        # the pair cull off (every sphere pair through the filter), on the
        # same inputs and network, the screen distance swept again for it.
        if not args.no_all_pairs:
            all_pairs_leg(out, params, md5, stream, dev, args)
        if args.audit_steps > 0:
            # The same 8-arm workload, audited: goals re-drawn every second so
            # the arms keep crossing, every dropped check also computed exactly.
            aud5 = audit_run(scenes.make_scene(5, collision_mode=0), params, args.audit_steps, dev, screen=tau5,
                             probe=SURROGATE_PROBE, min_drop=md5)
            aud5_exact = audit_run(scenes.make_scene(5, collision_mode=0), None, args.audit_steps, dev)
            out["surrogate"]["audit"] = aud5
            out["surrogate"]["audited_dynamics"] = {
                "learned_s": aud5["seconds"], "exact_s": aud5_exact["seconds"],
                "exact_executed_min_arm_gap_m": aud5_exact["executed_min_arm_gap_m"],
                "exact_first_executed_contact": aud5_exact["first_executed_contact"]}
        if not args.no_latency:
            out["surrogate"]["latency_1000"] = latency_leg(5, CONFIG_STEPS[5], dev, stream, params=params,
                                                           screen=tau5, probe=SURROGATE_PROBE, min_drop=md5)
            out["surrogate"]["latency_1000_no_history"] = latency_leg(5, CONFIG_STEPS[5], dev, stream,
                                                                      params=params, screen=tau5)
    if not args.no_surrogate and not args.no_4arm:
        # The 4-arm workload with its own network: exact vs learned step,
        # then the audit.
        sc4 = scenes.make_scene(4, collision_mode=0)
        p4, rep4 = train_surrogate(scenes.make_scene(4, collision_mode=0))
        if args.screen is None:
            sweep4, tau4 = screen_sweep(4, p4, stream, dev, max(5, args.steps // 2), args.warmup)
        else:
            sweep4, tau4 = {}, args.screen
        if args.min_drop is None:
            drops4, md4 = min_drop_sweep(4, p4, tau4, dev, stream)
        else:
            drops4, md4 = {}, args.min_drop
        ctl4 = native.Controller(sc4.arms, {**sc4.params, "collision_mode": 0, "surrogate_screen": tau4,
                                            "surrogate_probe": SURROGATE_PROBE, "surrogate_min_drop": md4},
                                 stream=stream)
        ctl4.set_surrogate_params(p4)
        w4e, _, _, _ = timed_loop(ctl4, scenes.make_scene(4, collision_mode=0), stream, args.steps,
                                  args.warmup, 0, dev)
        w4l, lat4, _, st4 = timed_loop(ctl4, scenes.make_scene(4, collision_mode=0), stream, args.steps,
                                       args.warmup, 1, dev)
        ctl4.close()
        aud = aud_exact = None
        if args.audit_steps > 0:
            aud = audit_run(sc4, p4, args.audit_steps, dev, screen=tau4, probe=SURROGATE_PROBE, min_drop=md4)
            aud_exact = audit_run(scenes.make_scene(4, collision_mode=0), None, args.audit_steps, dev)
        out["surrogate_4arm"] = {
            "workload": "4 arms on a 1.2 m square, 1024 rollouts x 30 steps each, 8 moving obstacles",
            "exact_ms_per_step": 1e3 * w4e / args.steps, "surrogate_ms_per_step": 1e3 * w4l / args.steps,
            "speedup_vs_exact": w4e / w4l,
            "exact_checks_skipped": st4["waves_skipped"] * 64 / max(st4["queries"], 1),
            "screen_m": tau4, "probe": SURROGATE_PROBE, "min_drop": md4,
            "screen_sweep_ms": {str(k): v for k, v in sweep4.items()},
            "min_drop_sweep_mean_ms": {str(k): v for k, v in drops4.items()},
            "train": {k: (round(v, 5) if isinstance(v, float) else v) for k, v in rep4.items()},
        }
        if aud is not None:
            out["surrogate_4arm"].update({
                "audit": aud,
                "audited_dynamics": {"learned_s": aud["seconds"], "exact_s": aud_exact["seconds"]},
                "exact_same_goals": {"executed_min_arm_gap_m": aud_exact["executed_min_arm_gap_m"],
                                     "first_executed_contact": aud_exact["first_executed_contact"],
                                     "seconds": aud_exact["seconds"]}})
        if not args.no_latency:
            out["surrogate_4arm"]["latency_1000"] = latency_leg(4, CONFIG_STEPS[4], dev, stream, params=p4,
                                                                screen=tau4, probe=SURROGATE_PROBE, min_drop=md4)
            out["surrogate_4arm"]["latency_1000_no_history"] = latency_leg(4, CONFIG_STEPS[4], dev, stream,
                                                                           params=p4, screen=tau4)
    if not args.no_latency:
        # Every workload's own closed loop (exact distances): configs 1-5.
        out["latency"] = {f"config{c}": latency_leg(c, CONFIG_STEPS[c], dev, stream) for c in (1, 2, 3, 4, 5)}
    if args.fig1_steps > 0:
        out["fig1_shared_goal"] = fig1(args.fig1_steps, args.fig1_seeds, dev)
    if args.ablation_steps > 0:
        out["ablation_2arm"] = ablation(args.ablation_steps, args.ablation_seeds, dev)
    if args.calibrate_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        # a plain read-only reduction over as many bytes as the weighted
        # mean reads on this workload (the noise of every arm, step, joint)
        n_eps = sum(a.n_rollouts * a.horizon for a in scenes.make_scene(5, collision_mode=0).arms) * 7
        for _ in range(3):
            red = src[:n_eps].sum()
        torch.cuda.synchronize()
        del red
        out["copy_calibration_bytes"] = src.numel() * 4
        out["reduction_reference_bytes"] = n_eps * 4
    if args.wmean_sizes:
        # The same 8-arm workload at 2x and 4x the rollouts (the weighted
        # mean then reads 73.4 and 146.8 MB): a few closed-loop steps each,
        # for a kernel trace of the weighted mean against its size.
        for n in WMEAN_SIZES[1:]:
            sc = scenes.make_scene(5, collision_mode=0)
            for a in sc.arms:
                a.n_rollouts = n
            c = native.Controller(sc.arms, sc.params, stream=stream)
            timed_loop(c, sc, stream, 5, 3, 0, dev)
            c.close()
        out["wmean_sizes"] = list(WMEAN_SIZES)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(scenes.make_scene(5, collision_mode=0))
    ctl.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
