"""The synthetic benchmark scenes start collision-free: every pair of arms is
apart at the sensed start pose (exact sphere-set distance of the oracle,
Sec. IV-A's sphere model), so any contact in a closed loop comes from the
controller, not from the scene's set-up."""
import numpy as np
import pytest

import oracle
from paper_2602_10114_amd import scenes


@pytest.mark.parametrize("config", [2, 3, 4, 5])
def test_start_poses_are_clear(config):
    sc = scenes.make_scene(config, collision_mode=0)
    oas = [oracle.make_arm(a) for a in sc.arms]
    q = sc.state[:, :, 0].astype(np.float64)
    gaps = [oracle.arm_pair_rho(oas[a], q[a], oas[b], q[b])
            for a in range(sc.n_arms) for b in range(a + 1, sc.n_arms)]
    assert min(gaps) > 0.0, f"config {config}: arms start in contact ({min(gaps):.4f} m)"
