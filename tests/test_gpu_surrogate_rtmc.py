"""The learned surrogate, trained on RTMC yields, against RTMC on held-out foams.

Reduced scale (the full experiment -- 1024 training foams, 256 held-out foams
evaluated at 1e5 primaries per point -- is `python -m paper_1806_00205_amd.surrogate`).
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1806_00205_amd as rt
    c = rt.Context(0)
    yield c
    c.close()


def test_surrogate_beats_rtmc_at_matched_error(ctx):
    """160 training foams of 64^3-96^3 (10240 RTMC yields), 24 held-out foams
    judged by RTMC on the 25-point grid: the held-out mean absolute yield
    error is within the 0.02 target (observed 0.0158; training and tracing are
    deterministic, so is this figure)."""
    from paper_1806_00205_amd.surrogate import run_experiment
    res, model = run_experiment(ctx, n_train=160, points_per_foam=64, n_test=24, train_primaries=20000,
                                eval_primaries=50000, steps=3000, seed=1, log=lambda s: None, sizes=(64, 80, 96),
                                workers=16)
    # held-out foams never seen in training: absolute yield error
    assert res["mae"] <= 0.02, res
    # what the network gains over tracing at the same error
    assert res["gain"] > 50, res
    assert res["in_support_frac"] == 1.0


def test_fallback_outside_training_support(ctx):
    from paper_1806_00205_amd.surrogate import Surrogate
    rng = np.random.default_rng(0)
    F = rng.normal(size=(512, 8))
    y = F[:, 0] * 0.1
    s = Surrogate(ctx, seed=2)
    s.fit(F, y, steps=50, batch=256)
    inside = F[:4]
    outside = F[:4] + 100.0
    calls = []
    yy, ok = s.predict_or_trace(np.concatenate([inside, outside]), lambda i: calls.append(i) or -1.0)
    assert list(ok) == [True] * 4 + [False] * 4
    assert calls == [4, 5, 6, 7] and np.all(yy[4:] == -1.0) and np.all(np.isfinite(yy[:4]))
    assert math.isfinite(float(yy[0]))
