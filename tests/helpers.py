"""Shared helpers of the GPU parity tests: run the HIP path with capture on,
then evaluate the oracle's stages on the HIP path's own upstream values."""
import numpy as np

import oracle
from paper_2602_10114_amd import scenes

F = np.float32


def f32(x):
    return float(np.float32(x))


def small_scene(config, n=None, h=None, seed=None, **over):
    sc = scenes.make_scene(config, seed=seed, **over)
    for i, a in enumerate(sc.arms):
        if n is not None:
            a.n_rollouts = n[i] if isinstance(n, (list, tuple)) else n
        if h is not None:
            a.horizon = h[i] if isinstance(h, (list, tuple)) else h
    return sc


class Capture:
    """Per-arm capture of one GPU step (host float64 copies)."""

    def __init__(self, ctl, arm, want_spheres=True):
        g = lambda k: ctl.debug_get(k, arm).cpu().numpy()
        self.eps = g("NOISE").astype(np.float64)            # [H][7][N]
        self.q = g("Q").astype(np.float64)                  # [N][H][7]
        self.qd = g("QD").astype(np.float64)
        self.sph = g("SPHERES").astype(np.float64) if want_spheres else None
        self.stage = g("STAGE_COST").astype(np.float64)     # [H][N]
        self.cost = g("COST").astype(np.float64)
        self.w = g("WEIGHTS").astype(np.float64)
        self.mu = g("MEAN").astype(np.float64)
        self.alpha = g("ALPHA").astype(np.float64)
        self.dist = float(g("DIST")[0])
        self.pairs = int(g("PAIRS")[0])
        self.argmin = int(g("ARGMIN")[0])


def board_inputs(ctl, sc, arm, boards=None):
    """Neighbour plans as the arm saw them at Sense (read side, before the
    step's publish), in the oracle's batch layout."""
    A = sc.n_arms
    Hm = max(a.horizon for a in sc.arms)
    Sm = max(a.n_spheres for a in sc.arms)
    nbs = [i for i in range(A) if i != arm]
    plans = np.zeros((max(len(nbs), 1), Hm, Sm, 4))
    nb_S, nb_H, nb_valid = [], [], []
    for m, i in enumerate(nbs):
        if boards is not None:
            plan, valid = boards[i]
        else:
            p, _, _, valid = ctl.get_board(i)
            plan = p.cpu().numpy()
        a = sc.arms[i]
        plans[m, :a.horizon, :a.n_spheres] = plan
        nb_S.append(a.n_spheres)
        nb_H.append(a.horizon)
        nb_valid.append(int(valid))
    return nbs, plans, nb_S, nb_H, nb_valid


def read_boards(ctl, sc):
    out = []
    for i in range(sc.n_arms):
        p, _, dist, valid = ctl.get_board(i)
        out.append((p.cpu().numpy().astype(np.float64), valid, dist))
    return out


def oracle_stage(sc, arm, cap, obstacles, boards, rows=None):
    """Oracle stage costs [H][N] on the GPU's own q, qd, spheres, plans, alpha."""
    a = sc.arms[arm]
    oa = oracle.make_arm(a)
    prm = oracle.make_params(sc.params)
    nbs, plans, nb_S, nb_H, nb_valid = board_inputs(None, sc, arm, [(b[0], b[1]) for b in boards])
    alpha_row = [cap.alpha[i] for i in nbs]
    q, qd, sph = cap.q, cap.qd, cap.sph
    if rows is not None:
        q, qd, sph = q[rows], qd[rows], sph[rows]
    return oracle.stage_costs_batch(oa, prm, q, qd, sph, sc.goal[arm], obstacles, plans if nbs else np.zeros(0),
                                    nb_S, nb_H, nb_valid, alpha_row)


def rel_err(a, b, floor=1.0):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float((np.abs(a - b) / np.maximum(np.abs(b), floor)).max()) if a.size else 0.0
