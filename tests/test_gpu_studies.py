"""Parity at the parameter settings the studies sweep (shrink ratio k, significance level alpha_F,
lower-bound exponent alpha, initial radius r1), and the study harness end to end."""
import dataclasses
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_04411_amd import hk
    hk.lib()
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def _with(w, **kw):
    return dataclasses.replace(w, params=dataclasses.replace(w.params, **kw))


@pytest.mark.parametrize("k,alpha_f,alpha", [(0.5, 0.05, 0.75), (0.9, 0.05, 0.75), (0.7, 0.01, 0.75),
                                             (0.7, 0.2, 0.75), (0.6, 0.1, 0.5), (0.8, 0.05, 0.95)])
def test_box_parity_at_study_settings(k, alpha_f, alpha):
    from tests import gpu_parity as GP
    from workloads import generators as G
    w = _with(G.box_scene(seed=5, res=32, J=120_000, n_iter=6), k=k, alpha_f=alpha_f, alpha=alpha)
    rep = GP.run_parity(w, 6)
    assert rep.shrinks > 0


@pytest.mark.parametrize("r1", [0.025, 0.1])
def test_plane_parity_at_study_radii(r1):
    from tests import gpu_parity as GP
    from workloads import generators as G
    w = G.config0(seed=9, n_side=24, J=80_000, n_iter=5, r1=r1)
    GP.run_parity(w, 5)


def test_study_harness_small():
    """The sweep at a small size: radii stay within [r_min, r1], every MSE is finite, and a stricter
    significance level keeps larger radii (fewer rejections)."""
    from paper_2504_04411_amd import studies
    res = studies.run(res=24, J=60_000, iters=10, seed=3, workers=1,
                      settings={"alpha_f": [0.01, 0.3], "k": [0.5]})
    rows = {(r["parameter"], r["value"]): r for r in res["rows"]}
    assert res["marks"] == [8, 10]
    for r in res["rows"]:
        assert all(math.isfinite(v) for v in r["mse"].values())
        assert r["radius_max"] <= np.float32(r["r1"])
        assert r["radius_min"] >= 0.001 * r["r1"] * 0.999
    assert rows[("alpha_f", 0.01)]["radius_mean"] > rows[("alpha_f", 0.3)]["radius_mean"]
