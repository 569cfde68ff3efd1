"""The GPR of libgadi (host code, gadi_gpr_*) against the float64 oracle
(oracle/gpr.py): the same grid point is chosen, the linear mean, the
hyperparameters, the log marginal likelihood and the predictions agree; the
retraining loop adds each prediction before the next size.  No GPU work."""
import numpy as np
import pytest

from oracle import gpr as ogpr

gadi = pytest.importorskip("paper_2501_04229_amd")
from paper_2501_04229_amd.predictor import gpr  # noqa: E402


@pytest.mark.parametrize("seed,m", [(1, 5), (2, 7), (3, 12), (4, 2)])
def test_fit_and_predict_match_the_oracle(seed, m):
    rng = np.random.default_rng(seed)
    x = np.sort(rng.uniform(3.0, 5.0, m))
    y = -1.2 + 0.1 * x + 0.05 * np.sin(3.0 * x) + 0.01 * rng.normal(size=m)
    g = gpr.GPR(x, y)
    ref = ogpr.fit(x, y)
    p = g.params()
    assert abs(p["b0"] - ref["b0"]) <= 1e-12 * max(1, abs(ref["b0"])) and abs(p["b1"] - ref["b1"]) <= 1e-12
    assert p["ell"] == pytest.approx(ref["ell"], rel=1e-12)
    assert p["sf2"] == pytest.approx(ref["sf2"], rel=1e-8)
    assert p["sn2"] == pytest.approx(ref["sn2"], rel=1e-8)
    assert p["lml"] == pytest.approx(ref["lml"], rel=1e-9, abs=1e-9)
    xq = np.linspace(2.0, 8.0, 25)
    mu, sd = g.predict(xq)
    mu_r, sd_r = ogpr.predict(ref, xq)
    assert np.allclose(mu, mu_r, rtol=1e-9, atol=1e-10)
    assert np.allclose(sd, sd_r, rtol=1e-6, atol=1e-7)


def test_single_point_and_constant_inputs():
    g = gpr.GPR(np.array([4.0]), np.array([-1.0]))
    mu, sd = g.predict(np.array([4.0, 6.0]))
    assert np.allclose(mu, -1.0)
    g = gpr.GPR(np.array([4.0, 4.0, 4.0]), np.array([-1.0, -1.2, -1.1]))
    assert g.params()["b1"] == 0.0
    assert np.allclose(g.predict(np.array([4.0]))[0], ogpr.predict(ogpr.fit([4.0] * 3, [-1.0, -1.2, -1.1]), [4.0])[0])


def test_argument_checks():
    with pytest.raises(gadi.GadiError):
        gpr.GPR(np.array([]), np.array([]))
    with pytest.raises(gadi.GadiError):
        gpr.GPR(np.array([1.0, np.nan]), np.array([0.0, 1.0]))
    with pytest.raises(ValueError):
        gpr.GPR(np.array([1.0, 2.0]), np.array([0.0]))
    with pytest.raises(gadi.GadiError):
        gpr.GPR(np.arange(257.0), np.zeros(257))


def test_retraining_adds_each_prediction():
    sizes = [8, 12, 16, 24]
    alphas = [0.2, 0.15, 0.12, 0.1]
    out = gpr.predict_alpha(sizes, alphas, [64, 32], retrain=True)
    assert [o[0] for o in out] == [32, 64]
    xs = list(np.log2(sizes))
    ys = list(np.log10(alphas))
    m32, _ = ogpr.predict(ogpr.fit(xs, ys), [5.0])
    assert out[0][1] == pytest.approx(10 ** m32[0], rel=1e-9)
    m64, _ = ogpr.predict(ogpr.fit(xs + [5.0], ys + [m32[0]]), [6.0])
    assert out[1][1] == pytest.approx(10 ** m64[0], rel=1e-9)


def test_dichotomy_search_on_known_costs():
    """The search of Section 3.3's training-set generation on costs with a known minimiser:
    a smooth bowl, an integer-valued (flat) bowl, failures beyond a threshold, and all-failed."""
    import math
    from paper_2501_04229_amd.predictor.gpr import dichotomy_search
    u, v, ev = dichotomy_search(lambda u: (u - 0.37) ** 2)
    assert abs(u - 0.37) <= 0.08 and ev <= 7 + 2 * 10
    u, v, _ = dichotomy_search(lambda u: math.floor(40 * abs(u + 0.9)))
    assert abs(u + 0.9) <= 0.08 and v <= math.floor(40 * 0.08)
    u, v, _ = dichotomy_search(lambda u: math.inf if u < -0.4 else (u + 0.3) ** 2)
    assert abs(u + 0.3) <= 0.1
    u, v, _ = dichotomy_search(lambda u: math.inf)
    assert math.isnan(u) and v == math.inf
