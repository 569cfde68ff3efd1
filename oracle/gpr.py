"""Gaussian-process regression of alpha on the problem size -- TEST INFRASTRUCTURE ONLY.

Section 3.3 predicts the splitting parameter of a large system from the best
parameters of small systems of the same structure by Gaussian-process
regression (GPR) on the size.  The model here, written from the textbook
definitions (Rasmussen and Williams, Gaussian Processes for Machine Learning,
2006: the posterior of Section 2.2 and the marginal likelihood of Section
2.3):

    y(x) = b0 + b1 x + f(x) + e,   f ~ GP(0, k),   e ~ N(0, sn2),
    k(x, x') = sf2 exp(-(x - x')^2 / (2 ell^2)),

with the linear mean fitted by least squares and the GP fitted to its
residuals (no GP when every residual is at most 1e-12 max(1, max |y|): the
data are a line up to rounding).  Hyperparameters maximise the log marginal likelihood of the
residuals over ell in 25 log-spaced values in [0.1 s, 10 s] (s = spread of x,
1 if zero) and eta = sn2 / sf2 in 13 log-spaced values in [1e-6, 1], with sf2
at its maximiser for each (ell, eta); the first grid point wins ties.
Predictions are the latent mean and standard deviation (the noise is not
added; the uncertainty of the linear mean is not added either).
"""
from __future__ import annotations

import numpy as np

ELL_POINTS = 25
ETA_POINTS = 13


def linear_mean(x, y):
    """Least-squares b0, b1 (b1 = 0 when all x are equal)."""
    x = np.asarray(x, float)
    y = np.asarray(y, float)
    if np.ptp(x) == 0.0:
        return float(np.mean(y)), 0.0
    X = np.stack([np.ones_like(x), x], axis=1)
    coef, *_ = np.linalg.lstsq(X, y, rcond=None)
    return float(coef[0]), float(coef[1])


def rbf(a, b, ell, sf2=1.0):
    a = np.asarray(a, float)[:, None]
    b = np.asarray(b, float)[None, :]
    return sf2 * np.exp(-((a - b) ** 2) / (2.0 * ell * ell))


def log_marginal(x, e, ell, sf2, sn2):
    """log p(e | x) = -1/2 e^T K^-1 e - 1/2 log det K - m/2 log(2 pi), K = k(x, x) + sn2 I."""
    m = len(x)
    K = rbf(x, x, ell, sf2) + sn2 * np.eye(m)
    sign, logdet = np.linalg.slogdet(K)
    if sign <= 0:
        return -np.inf
    return float(-0.5 * e @ np.linalg.solve(K, e) - 0.5 * logdet - 0.5 * m * np.log(2.0 * np.pi))


def profiled_sf2(x, e, ell, eta):
    """The sf2 that maximises log_marginal(x, e, ell, sf2, eta sf2): e^T Kt^-1 e / m, Kt = K / sf2."""
    Kt = rbf(x, x, ell) + eta * np.eye(len(x))
    return float(e @ np.linalg.solve(Kt, e) / len(x))


def posterior(x, e, xq, ell, sf2, sn2):
    """GP posterior mean and latent standard deviation at xq given residual data (x, e)."""
    K = rbf(x, x, ell, sf2) + sn2 * np.eye(len(x))
    ks = rbf(xq, x, ell, sf2)
    mean = ks @ np.linalg.solve(K, e)
    var = sf2 - np.einsum("ij,ji->i", ks, np.linalg.solve(K, ks.T))
    return mean, np.sqrt(np.maximum(var, 0.0))


def fit(x, y):
    """Returns dict(b0, b1, ell, sf2, sn2, lml, x, e) by the grid rule of the module docstring."""
    x = np.asarray(x, float)
    y = np.asarray(y, float)
    b0, b1 = linear_mean(x, y)
    e = y - b0 - b1 * x
    s = float(np.ptp(x)) or 1.0
    out = {"b0": b0, "b1": b1, "x": x, "e": e}
    if np.max(np.abs(e)) <= 1e-12 * max(1.0, float(np.max(np.abs(y)))):
        out.update(ell=s, sf2=0.0, sn2=0.0, lml=np.inf)
        return out
    best = None
    for ell in s * np.logspace(-1.0, 1.0, ELL_POINTS):
        for eta in np.logspace(-6.0, 0.0, ETA_POINTS):
            sf2 = profiled_sf2(x, e, ell, eta)
            if not sf2 > 0.0:
                continue
            lml = log_marginal(x, e, ell, sf2, eta * sf2)
            if best is None or lml > best[0]:
                best = (lml, ell, sf2, eta * sf2)
    out.update(lml=best[0], ell=best[1], sf2=best[2], sn2=best[3])
    return out


def predict(model, xq):
    """Latent mean and standard deviation at xq."""
    xq = np.asarray(xq, float)
    lin = model["b0"] + model["b1"] * xq
    if model["sf2"] == 0.0:
        return lin, np.zeros_like(xq)
    mu, sd = posterior(model["x"], model["e"], xq, model["ell"], model["sf2"], model["sn2"])
    return lin + mu, sd
