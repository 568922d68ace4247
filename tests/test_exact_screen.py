"""Host check of the screen the rollout kernel's exact pass applies before
forming FP64 gaps (Eq. 6 distance, exact mode): per staged sphere, one pass
over the candidates computes FP32 gaps and marks those below
min(best, B, smallest FP32 gap so far) + 1e-4 m; only marked candidates get
an FP64 gap.  Whenever the FP64 minimum over all candidates is below
min(best, B), the minimum over the marked ones equals it, so the hinge
max(0, 1 - max(0, d)/B) and the tests d < B, d < 0 are unchanged."""
import numpy as np


def screened_min(own, r_own, p, r_p, best, B):
    g32 = (np.sqrt(((own - p.astype(np.float32)) ** 2).sum(axis=1, dtype=np.float32), dtype=np.float32)
           - r_own - np.float32(r_p))
    lim = min(best, B)
    m32 = np.float32(3.0e38)
    for j, g in enumerate(g32):
        m32 = min(m32, g)
        if float(g) < min(lim, float(m32)) + 1.0e-4:
            d = ((own[j].astype(np.float64) - p.astype(np.float64)) ** 2).sum()
            best = min(best, np.sqrt(d) - float(r_own[j]) - float(r_p))
    return best


def test_screen_keeps_the_minimum_below_the_buffer():
    rng = np.random.default_rng(3)
    B = 0.03
    for trial in range(4000):
        n = int(rng.integers(1, 9))
        centre = rng.uniform(-2.5, 2.5, 3)
        own = (centre + rng.normal(scale=0.05, size=(n, 3))).astype(np.float32)
        r_own = rng.uniform(0.02, 0.08, n).astype(np.float32)
        p = (centre + rng.normal(scale=0.05, size=3)).astype(np.float32)
        r_p = np.float32(rng.uniform(0.02, 0.08))
        best = float(rng.choice([1.0e300, rng.uniform(-0.05, 0.05)]))
        full = min(best, min(np.sqrt(((own[j].astype(np.float64) - p.astype(np.float64)) ** 2).sum())
                             - float(r_own[j]) - float(r_p) for j in range(n)))
        got = screened_min(own, r_own, p, r_p, best, B)
        if full < min(best, B):
            assert got == full, (trial, got, full)
        else:
            assert got >= min(best, B) or got == full
        hinge = lambda d: max(0.0, 1.0 - max(0.0, d) / B)
        assert hinge(got) == hinge(full) and (got < B) == (full < B) and (got < 0) == (full < 0)
