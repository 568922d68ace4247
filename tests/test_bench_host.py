"""Host logic of the benchmark (CPU only): the algorithmic work model, the
counter summaries and the guard that ties the recorded HBM traffic to the
kernel sources it was measured on."""
import csv
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2602_10114_amd import scenes  # noqa: E402


def _self_pairs(arm):
    L = [int(x) for x in arm.sphere_link]
    return sum(1 for s in range(len(L)) for t in range(s + 1, len(L)) if abs(L[s] - L[t]) >= 2)


def test_self_pair_counts_of_the_two_sphere_tables():
    # Sphere pairs on bodies at least two apart: 872 for the 52-sphere
    # table, 1344 for the 64-sphere one (8 spheres on each of 8 bodies:
    # 64 * 63 / 2 minus 8 * 28 same-body pairs minus 7 * 64 adjacent ones).
    assert _self_pairs(scenes.make_scene(1).arms[0]) == 872
    assert _self_pairs(scenes.make_scene(5).arms[0]) == 64 * 63 // 2 - 8 * 28 - 7 * 64 == 1344


def test_algorithmic_work_by_hand():
    # One arm, 52 spheres, one obstacle, 64 rollouts x 20 steps:
    # 11 FLOP x (872 self + 52 obstacle pairs) + 4*7 + 8*63 + 18*52 + 30 + 7*7.
    per_step = 11 * (872 + 52) + (4 * 7 + 8 * 63 + 18 * 52 + 30 + 7 * 7)
    assert bench.algorithmic_flops_per_step(scenes.make_scene(1)) == 64 * 20 * per_step == 14_990_080
    # Eight arms of 64 spheres, 20 obstacles, 7 neighbour plans each:
    # 346,019 FLOP per rollout step, 4096 x 40 rollout steps per arm.
    per_step5 = 11 * (1344 + 64 * 20 + 7 * 64 * 64) + (4 * 7 + 8 * 63 + 18 * 64 + 30 + 7 * 7)
    assert per_step5 == 346_019
    assert bench.algorithmic_flops_per_step(scenes.make_scene(5)) == 8 * 4096 * 40 * per_step5


def test_recorded_traffic_is_reported_only_for_its_kernel_sources(monkeypatch):
    # The HBM bytes in the bench line are measured counters, valid only for
    # the sources they were taken on: with the digest of the current sources
    # they are reported, after any edit to those sources they are not.
    assert set(bench.TRAFFIC["bytes_per_launch"]) == {1, 2, 4}
    assert all(v > 0 for v in bench.TRAFFIC["bytes_per_launch"].values())
    monkeypatch.setitem(bench.TRAFFIC, "sources_sha256", bench.sources_digest())
    for w in (1, 2, 4):
        assert bench.traffic_bytes(w) == bench.TRAFFIC["bytes_per_launch"][w]
    monkeypatch.setitem(bench.TRAFFIC, "sources_sha256", "0" * 16)
    assert bench.traffic_bytes(1) is None


def _write_counters(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value",
                                          "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_counter_summary_rates(tmp_path):
    # Two dispatches of one kernel; the summary reads the last one.  With
    # GRBM_GUI_ACTIVE summed over 8 XCDs, one XCD ran 8e6 cycles.
    cyc = 8.0e6
    last = {"GRBM_GUI_ACTIVE": 8 * cyc, "SQ_INSTS_VALU": 0.3 * 1024 * cyc,
            "SQ_INSTS_VALU_FMA_F32": 0.2 * 1024 * cyc, "SQ_INSTS_VALU_ADD_F32": 0.05 * 1024 * cyc,
            "SQ_ACTIVE_INST_VALU": 1000.0, "SQ_THREAD_CYCLES_VALU": 1000.0 * 64 * 0.75,
            "SQ_VALU_MFMA_BUSY_CYCLES": 0.5 * 1024 * cyc}
    rows = []
    for d, scale in ((1, 0.5), (2, 1.0)):
        for k, v in last.items():
            rows.append({"Dispatch_Id": d, "Kernel_Name": "mrs::k_probe(args)", "Counter_Name": k,
                         "Counter_Value": v * scale, "Start_Timestamp": 0, "End_Timestamp": 3_000_000})
    _write_counters(tmp_path / "p_counter_collection.csv", rows)
    out = bench.summarize_pmc(str(tmp_path))
    vals = {}
    for line in out.splitlines():
        parts = line.strip().rsplit(None, 1)
        if len(parts) == 2:
            try:
                vals[parts[0].strip()] = float(parts[1])
            except ValueError:
                pass
    assert "dispatches 2" in out
    assert vals["VALU wave-insts/SIMD-cycle"] == pytest.approx(0.3, abs=1e-4)
    assert vals["FMA wave-insts/SIMD-cycle"] == pytest.approx(0.2, abs=1e-4)
    assert vals["VALU active-lane share"] == pytest.approx(0.75, abs=1e-4)
    assert vals["MFMA busy share"] == pytest.approx(0.5, abs=1e-4)
    assert vals["FP32 share of VALU insts"] == pytest.approx(0.25 / 0.3, abs=1e-4)
    # FP32 operations: 64 lanes x (2 per FMA + 1 per add)
    assert vals["FP32 VALU ops (64 lanes)"] == pytest.approx(64 * (2 * 0.2 + 0.05) * 1024 * cyc, rel=1e-5)


def test_weighted_mean_size_summary(tmp_path):
    # Launches of three sizes told apart by their grid (one 256-thread block
    # per 1024-rollout chunk); medians 8, 12 and 20 us for 36.7, 73.4 and
    # 146.8 MB of noise; other kernels and the between-iterations kernel are
    # ignored.
    fields = ["Kernel_Name", "Start_Timestamp", "End_Timestamp", "Workgroup_Size_X", "Grid_Size_X"]
    rows = []
    for chunks, us in ((4, (7.0, 8.0, 9.0)), (8, (12.0, 11.0, 13.0)), (16, (20.0, 19.0, 30.0))):
        for t in us:
            rows.append({"Kernel_Name": "mrs::k_wmean(mrs::ReduceArgs)", "Start_Timestamp": 0,
                         "End_Timestamp": int(t * 1000), "Workgroup_Size_X": 256, "Grid_Size_X": 256 * chunks})
    rows.append({"Kernel_Name": "mrs::k_wmean_fin(mrs::ReduceArgs)", "Start_Timestamp": 0, "End_Timestamp": 999000,
                 "Workgroup_Size_X": 64, "Grid_Size_X": 256})
    rows.append({"Kernel_Name": "mrs::k_total(mrs::ReduceArgs)", "Start_Timestamp": 0, "End_Timestamp": 5000,
                 "Workgroup_Size_X": 256, "Grid_Size_X": 1024})
    with open(tmp_path / "t_kernel_trace.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        for r in rows:
            w.writerow(r)
    out = bench.summarize_sizes(str(tmp_path)).splitlines()
    table = [line.split() for line in out[2:]]
    assert [int(r[0]) for r in table] == [4096, 8192, 16384]
    assert [float(r[3]) for r in table] == [8.0, 12.0, 20.0]
    mb = [8 * 40 * 7 * n * 4 / 1e6 for n in (4096, 8192, 16384)]
    assert float(table[0][4]) == pytest.approx(mb[0] / 8.0, abs=0.01)
    # marginal rate between the last two sizes: 73.4 MB in 8 us
    assert out[-1].endswith(f"marginal {(mb[2] - mb[1]) / 8.0:.2f} TB/s")
