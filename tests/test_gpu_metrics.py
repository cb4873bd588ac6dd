"""mc_rms_w (Sec. 2.7, Eq. RMSw, and Table S1's unweighted and log-ratio variants)
on the GPU against the oracle's definitions, on seeded profiles that include
depths the metrics must skip (zero, negative, infinite or NaN values)."""
from __future__ import annotations

import numpy as np
import pytest
import torch

from oracle import estimators as est
from paper_2604_13929_amd import photonmc as pm

pytestmark = pytest.mark.gpu


def banner(msg):
    print(f"[gpu] {msg}", flush=True)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pm.load()


@pytest.mark.parametrize("n", [1, 7, 256, 257, 4099])
def test_rms_w_matches_oracle(n):
    banner(f"mc_rms_w, {n} depths")
    rng = np.random.default_rng(n)
    q = np.exp(-rng.random(n) * 8.0) * 3.0
    p = q * np.exp(rng.normal(0.0, 0.3, n))
    if n > 4:
        q[1], p[2], q[3] = 0.0, -0.5, np.inf
        p[4] = np.nan
    got = pm.rms_w(p, q)
    assert got["weighted"] == pytest.approx(est.rms_w(p, q), rel=1e-12)
    assert got["unweighted"] == pytest.approx(est.rms_unweighted(p, q), rel=1e-12)
    assert got["log"] == pytest.approx(est.rms_log(p, q), rel=1e-12)


def test_rms_w_of_identical_profiles_and_of_no_valid_depth():
    banner("mc_rms_w edge cases")
    q = np.linspace(1.0, 2.0, 33)
    assert pm.rms_w(q, q) == {"weighted": 0.0, "unweighted": 0.0, "log": 0.0}
    z = pm.rms_w(np.ones(5), np.zeros(5))
    assert all(np.isnan(v) for v in z.values())
    # a profile that is zero where the reference is positive: no log term, the others defined
    r = pm.rms_w(np.zeros(4), np.ones(4))
    assert r["weighted"] == 1.0 and r["unweighted"] == 1.0 and np.isnan(r["log"])
