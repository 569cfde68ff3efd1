"""Pins of the GPR oracle (Section 3.3: alpha regressed on the problem size), CPU only.

G1  for fixed hyperparameters the posterior mean and latent standard deviation
    equal scikit-learn's GaussianProcessRegressor (constant x RBF kernel, noise
    on the training diagonal, no optimiser);
G2  the log marginal likelihood equals scikit-learn's for the same kernel, and
    the profiled sf2 is its maximiser along sf2;
G3  exactly linear data: the fit is the line (b0, b1) and the GP part is negligible;
G4  near-noise-free posterior interpolates the training residuals;
G5  the grid search returns the best grid point (brute force over the grid
    with scikit-learn's likelihood);
G6  a kernel with the 1/2 of its exponent dropped fails G1 (the pin catches
    that mistake).
"""
import numpy as np
import pytest
from sklearn.gaussian_process import GaussianProcessRegressor
from sklearn.gaussian_process.kernels import RBF, ConstantKernel

from oracle import gpr


def _data(seed, m=9):
    rng = np.random.default_rng(seed)
    x = np.sort(rng.uniform(3.0, 5.0, m))
    y = -1.2 + 0.1 * x + 0.05 * np.sin(3.0 * x) + 0.01 * rng.normal(size=m)
    return x, y


def _sk(x, e, ell, sf2, sn2):
    k = ConstantKernel(sf2, constant_value_bounds="fixed") * RBF(ell, length_scale_bounds="fixed")
    return GaussianProcessRegressor(kernel=k, alpha=sn2, optimizer=None, normalize_y=False).fit(x[:, None], e)


@pytest.mark.parametrize("ell,sf2,sn2", [(0.5, 0.01, 1e-4), (2.0, 0.3, 1e-6), (0.2, 1.0, 0.1)])
def test_g1_posterior_matches_sklearn(ell, sf2, sn2):
    x, y = _data(1)
    e = y - y.mean()
    xq = np.linspace(2.5, 7.0, 17)
    mu, sd = gpr.posterior(x, e, xq, ell, sf2, sn2)
    m2, s2 = _sk(x, e, ell, sf2, sn2).predict(xq[:, None], return_std=True)
    assert np.allclose(mu, m2, rtol=1e-9, atol=1e-12)
    assert np.allclose(sd, s2, rtol=1e-7, atol=1e-9)


@pytest.mark.parametrize("ell,sf2,sn2", [(0.5, 0.01, 1e-4), (1.5, 0.2, 1e-3)])
def test_g2_marginal_likelihood_and_profile(ell, sf2, sn2):
    x, y = _data(2)
    e = y - y.mean()
    ref = _sk(x, e, ell, sf2, sn2).log_marginal_likelihood_value_
    assert abs(gpr.log_marginal(x, e, ell, sf2, sn2) - ref) <= 1e-9 * max(1.0, abs(ref))
    eta = 1e-3
    s_hat = gpr.profiled_sf2(x, e, ell, eta)
    best = gpr.log_marginal(x, e, ell, s_hat, eta * s_hat)
    for f in (0.8, 0.95, 1.05, 1.25):
        assert gpr.log_marginal(x, e, ell, f * s_hat, eta * f * s_hat) < best


def test_g3_linear_data():
    x = np.array([3.0, 3.5, 4.0, 4.5, 5.0])
    y = 2.0 + 3.0 * x
    m = gpr.fit(x, y)
    assert abs(m["b0"] - 2.0) < 1e-12 and abs(m["b1"] - 3.0) < 1e-12
    mu, sd = gpr.predict(m, np.array([0.0, 7.0]))
    # the residuals are rounding noise: whatever GP is fitted to them is negligible
    assert np.allclose(mu, [2.0, 23.0], atol=1e-11) and np.all(sd < 1e-10)


def test_g4_interpolation():
    x, y = _data(3)
    e = y - y.mean()
    mu, sd = gpr.posterior(x, e, x, 0.4, 0.05, 1e-12)
    assert np.allclose(mu, e, atol=1e-6)
    assert np.all(sd < 1e-4)


def test_g5_grid_search_is_the_best_grid_point():
    x, y = _data(4, m=7)
    m = gpr.fit(x, y)
    e = m["e"]
    s = np.ptp(x)
    best = -np.inf
    for ell in s * np.logspace(-1, 1, 25):
        for eta in np.logspace(-6, 0, 13):
            # profiled sf2 through scikit-learn: maximise over a fine sf2 scan around the closed form
            sf = gpr.profiled_sf2(x, e, ell, eta)
            best = max(best, _sk(x, e, ell, sf, eta * sf).log_marginal_likelihood_value_)
    assert abs(m["lml"] - best) <= 1e-9 * max(1.0, abs(best))


def test_g6_planted_kernel_mistake_fails_g1():
    x, y = _data(5)
    e = y - y.mean()
    xq = np.linspace(3.0, 5.0, 5)
    ell, sf2, sn2 = 0.5, 0.02, 1e-4
    good = gpr.rbf
    try:
        gpr.rbf = lambda a, b, l, s=1.0: s * np.exp(-((np.asarray(a, float)[:, None] - np.asarray(b, float)[None, :]) ** 2) / (l * l))
        mu, _ = gpr.posterior(x, e, xq, ell, sf2, sn2)
    finally:
        gpr.rbf = good
    m2 = _sk(x, e, ell, sf2, sn2).predict(xq[:, None])
    assert not np.allclose(mu, m2, rtol=1e-6, atol=1e-9)
