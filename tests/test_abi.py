"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every entry point the header declares, the ctypes structures match the C
layout, and init fails loudly without a gfx950 device."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2602_10114_amd import native, scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mrstorm.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(mpc_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = native.lib()
    names = _declared()
    assert "mpc_init" in names and "mpc_step" in names and "mpc_share_plans" in names
    for n in names:
        assert hasattr(L, n), n
    assert sorted(native.EXPORTS) == names


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "mrstorm.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu\\n", sizeof(mpc_arm_desc), offsetof(mpc_arm_desc, sphere_link),
         offsetof(mpc_arm_desc, base), offsetof(mpc_arm_desc, tool), sizeof(mpc_params));
  printf("%zu %zu %zu %zu %zu %zu %zu %zu\\n", offsetof(mpc_params, iters), offsetof(mpc_params, seed),
         offsetof(mpc_params, collision_mode), offsetof(mpc_params, surrogate_margin),
         offsetof(mpc_params, surrogate_screen), offsetof(mpc_params, surrogate_probe),
         offsetof(mpc_params, surrogate_min_drop), offsetof(mpc_params, pair_cull));
  printf("%zu %zu %zu %zu\\n", sizeof(mpc_train_params), offsetof(mpc_train_params, seed),
         offsetof(mpc_train_params, lr_final), offsetof(mpc_train_params, target_floor));
  printf("%zu %zu %zu\\n", sizeof(mpc_train_report), offsetof(mpc_train_report, steps),
         offsetof(mpc_train_report, val_max_over_near));
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    A, P = native.MpcArmDesc, native.MpcParams
    T, R = native.MpcTrainParams, native.MpcTrainReport
    expect = [C.sizeof(A), A.sphere_link.offset, A.base.offset, A.tool.offset, C.sizeof(P),
              P.iters.offset, P.seed.offset, P.collision_mode.offset, P.surrogate_margin.offset,
              P.surrogate_screen.offset, P.surrogate_probe.offset, P.surrogate_min_drop.offset,
              P.pair_cull.offset,
              C.sizeof(T), T.seed.offset, T.lr_final.offset, T.target_floor.offset,
              C.sizeof(R), R.steps.offset, R.val_max_over_near.offset]
    assert [int(x) for x in out] == expect


def test_init_without_gpu_fails_loudly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    L = native.lib()
    sc = scenes.make_scene(1)
    descs, keep = native.arm_descs(sc.arms)
    prm = native.params_struct(sc.params)
    h = C.c_void_p()
    rc = L.mpc_init(descs, 1, C.byref(prm), None, C.byref(h))
    assert rc == native.MPC_EHIP
    assert b"device" in L.mpc_last_error(None)
    assert not h.value


def _init_rc(arms, params):
    descs, keep = native.arm_descs(arms)
    prm = native.params_struct(params)
    h = C.c_void_p()
    rc = native.lib().mpc_init(descs, len(arms), C.byref(prm), None, C.byref(h))
    assert not h.value
    return rc, native.lib().mpc_last_error(None).decode()


def test_descriptor_and_parameter_errors_need_no_device():
    """Arm descriptors and parameters are validated on the host before any
    device call, so every rejection below is the same with or without a GPU."""
    sc = scenes.make_scene(2)
    # the learned distance's margin must not hide gaps inside the buffer B
    rc, msg = _init_rc(sc.arms, {**sc.params, "surrogate_margin": 0.02, "buf_dyn": 0.03})
    assert rc == native.MPC_EINVAL and "surrogate_margin" in msg
    rc, msg = _init_rc(sc.arms, {**sc.params, "surrogate_margin": 0.02, "buf_dyn": 0.03, "collision_mode": 0})
    assert rc == native.MPC_EINVAL
    # a chain whose reach exceeds the range the FP32 filter is sized for:
    # each link of the table at most 1.5 m, their sum above 2.6 m
    long = scenes.dataclasses.replace(sc.arms[0], dh=sc.arms[0].dh.copy())
    long.dh[:, 2] = 0.45
    rc, msg = _init_rc([long, sc.arms[1]], sc.params)
    assert rc == native.MPC_EINVAL and "reach" in msg
    # a tool point far off the flange counts towards the reach as well
    tool = scenes.dataclasses.replace(sc.arms[0], tool=np.array([0.0, 0.0, 1.4], np.float32))
    rc, msg = _init_rc([tool, sc.arms[1]], sc.params)
    assert rc == native.MPC_EINVAL and "reach" in msg
    # the drop-history screen's probe period: 0 (off) or 2..1000 steps
    for bad in (1, -1, 1001):
        rc, msg = _init_rc(sc.arms, {**sc.params, "surrogate_probe": bad})
        assert rc == native.MPC_EINVAL and "surrogate_probe" in msg
    for bad in (-0.1, 1.0, float("nan")):
        rc, msg = _init_rc(sc.arms, {**sc.params, "surrogate_min_drop": bad})
        assert rc == native.MPC_EINVAL and "surrogate_min_drop" in msg
    # the pair cull is on (1) or off (0)
    for bad in (-1, 2):
        rc, msg = _init_rc(sc.arms, {**sc.params, "pair_cull": bad})
        assert rc == native.MPC_EINVAL and "pair_cull" in msg
    # only 7-DoF chains are built
    six = scenes.dataclasses.replace(sc.arms[0], dh=sc.arms[0].dh[:6], q_lim=sc.arms[0].q_lim[:6],
                                     qd_max=sc.arms[0].qd_max[:6])
    rc, msg = _init_rc([six, sc.arms[1]], sc.params)
    assert rc == native.MPC_EUNSUPPORTED


def test_bad_arguments_rejected_before_device_use():
    L = native.lib()
    h = C.c_void_p()
    assert L.mpc_init(None, 1, None, None, C.byref(h)) == native.MPC_EINVAL
    assert L.mpc_step(None, None, None, None, 0, None) == native.MPC_EINVAL
    assert L.mpc_share_plans(None, None) == native.MPC_EINVAL
    assert L.mpc_philox(None, None, None, -1, None) == native.MPC_EINVAL
