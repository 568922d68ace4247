"""The allocation-free prediction entry point (for callers that cannot
allocate) against the allocating one, through the C-ABI: two calls in a
row, the second with fewer queries, each bitwise equal to
mpc_surrogate_predict on the same inputs (same kernels and bfloat16
dataflow); sizes beyond the fixed working memory are rejected."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2602_10114_amd import native
from helpers import small_scene

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _params(seed):
    W = native.MLP_WIDTHS
    rng = np.random.default_rng(seed)
    p = np.zeros(native.MLP_PARAMS, np.float32)
    o = 0
    for l in range(len(W) - 1):
        nw = W[l + 1] * W[l]
        p[o:o + nw] = rng.uniform(-1, 1, nw) * math.sqrt(6 / W[l])
        p[o + nw:o + nw + W[l + 1]] = rng.normal(size=W[l + 1]) * 0.05
        o += nw + W[l + 1]
    return p


def test_noalloc_prediction_equals_allocating_prediction():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    _say("case: allocation-free prediction, 4096 then 1000 queries, against mpc_surrogate_predict")
    sc = small_scene(2, n=64, h=4)
    ctl = native.Controller(sc.arms, sc.params)
    ctl.set_surrogate_params(_params(5))
    L = native.lib()
    rng = np.random.default_rng(6)
    for m in (native.PREDICT_NOALLOC_MAX, 1000):
        feats = torch.from_numpy(rng.uniform(-1.2, 1.2, size=(m, 17)).astype(np.float32)).cuda()
        ref = ctl.surrogate_predict(feats)
        y = torch.full((m + 8,), float("nan"), dtype=torch.float32, device="cuda")
        rc = L.mpc_surrogate_predict_noalloc(ctl.h, native._ptr(feats), m, native._ptr(y))
        assert rc == native.MPC_OK, L.mpc_last_error(ctl.h)
        ctl.sync()
        got, want = y[:m].cpu().numpy(), ref.cpu().numpy()
        _say(f"  m = {m}: max |diff| {np.abs(got - want).max():.3g}")
        np.testing.assert_array_equal(got, want)
        assert torch.isnan(y[m:]).all()          # nothing written past m
    big = torch.zeros((native.PREDICT_NOALLOC_MAX + 1, 17), dtype=torch.float32, device="cuda")
    out = torch.zeros(native.PREDICT_NOALLOC_MAX + 1, dtype=torch.float32, device="cuda")
    rc = L.mpc_surrogate_predict_noalloc(ctl.h, native._ptr(big), native.PREDICT_NOALLOC_MAX + 1, native._ptr(out))
    assert rc == native.MPC_EINVAL
    assert b"MPC_PREDICT_NOALLOC_MAX" in L.mpc_last_error(ctl.h)
    assert L.mpc_surrogate_predict_noalloc(ctl.h, None, 0, None) == native.MPC_OK
    ctl.close()
