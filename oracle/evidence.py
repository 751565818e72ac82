"""Reference values of the model evidence, used to pin the sampler.

The paper never estimates the evidence; it is the standard by-product of an
SMC sampler (the product over steps of the mean incremental weight), and it
makes the whole tempered sampler checkable against numbers computed without
any sampling:

  * k = 1 with a N(a, b^2) prior: Z_beta = int p0(mu) L(mu)^beta dmu is a
    Gaussian integral in closed form for every beta.
  * k = 2, small n, N(0, s0^2) prior: Z = sum over all 2^n allocations z of
    prod_j w_{z_j} prod_i G(S_i(z)), where G(S) is the conjugate normal
    marginal likelihood of the observations allocated to one component.
  * k = 2: the same Z by trapezoidal quadrature of p0(mu1) p0(mu2) L(mu1, mu2)
    over a fine 2-D grid, using the oracle's own likelihood and prior.

The second and third agree only if the likelihood, the prior and their
normalising constants are all right, which is why they are compared.
"""

from __future__ import annotations

import math

import numpy as np

from .gmm import Model, log_prior, per_datum_loglik


def log_z_tempered_k1(y, sigma2, beta, prior_a=0.0, prior_b=10.0) -> float:
    """log int N(mu; a, b^2) L(mu)^beta dmu for a single-component model.

    With ybar, S = sum (y - ybar)^2 and v = sigma2 / (beta n):
      log Z = -(n beta / 2) log(2 pi sigma2) - beta S / (2 sigma2)
              + (1/2) log(v / (v + b^2)) - (ybar - a)^2 / (2 (v + b^2)).
    """
    y = np.asarray(y, dtype=np.float64)
    n = y.size
    if beta == 0.0:
        return 0.0
    ybar = float(np.mean(y))
    S = float(np.sum((y - ybar) ** 2))
    v = sigma2 / (beta * n)
    b2 = prior_b * prior_b
    return (-0.5 * n * beta * math.log(2.0 * math.pi * sigma2) - beta * S / (2.0 * sigma2)
            + 0.5 * math.log(v / (v + b2)) - (ybar - prior_a) ** 2 / (2.0 * (v + b2)))


def posterior_k1(y, sigma2, beta, prior_a=0.0, prior_b=10.0):
    """Mean and variance of the tempered single-component posterior p0 L^beta."""
    y = np.asarray(y, dtype=np.float64)
    prec = 1.0 / prior_b ** 2 + beta * y.size / sigma2
    mean = (prior_a / prior_b ** 2 + beta * float(np.sum(y)) / sigma2) / prec
    return mean, 1.0 / prec


def _log_g(m, sy, syy, sigma2, s0):
    """Conjugate marginal log-likelihood of m observations with sum sy and sum
    of squares syy under mu ~ N(0, s0^2), y | mu ~ N(mu, sigma2)."""
    s02 = s0 * s0
    return (-0.5 * m * math.log(2.0 * math.pi * sigma2)
            - 0.5 * np.log1p(m * s02 / sigma2)
            - (syy - s02 * sy * sy / (sigma2 + m * s02)) / (2.0 * sigma2))


def log_z_enumerate_k2(y, sigma2, s0=10.0, w=(0.5, 0.5)) -> float:
    """Exact log-evidence of a two-component model by enumerating all 2^n
    allocations (n <= 22), each weighted by prod_j w_{z_j}."""
    y = np.asarray(y, dtype=np.float64)
    n = y.size
    if n > 22:
        raise ValueError("enumeration is limited to n <= 22")
    codes = np.arange(1 << n, dtype=np.int64)
    bits = ((codes[:, None] >> np.arange(n)[None, :]) & 1).astype(np.float64)  # 1: component 2
    m2 = bits.sum(axis=1)
    m1 = n - m2
    sy_all, syy_all = float(y.sum()), float((y * y).sum())
    sy2 = bits @ y
    syy2 = bits @ (y * y)
    sy1 = sy_all - sy2
    syy1 = syy_all - syy2
    terms = (m1 * math.log(w[0]) + m2 * math.log(w[1])
             + _log_g(m1, sy1, syy1, sigma2, s0) + _log_g(m2, sy2, syy2, sigma2, s0))
    mx = float(terms.max())
    return mx + math.log(float(np.sum(np.exp(terms - mx))))


def log_z_quadrature_k2(y, sigma2, s0=10.0, lo=-12.0, hi=12.0, h=0.02) -> float:
    """log-evidence of the two-component model by the trapezoidal rule on a
    square grid, integrand p0(mu1) p0(mu2) L(mu1, mu2) from the oracle's own
    likelihood and prior."""
    model = Model.equal_weights(2, 1, sigma2, prior="gauss", prior_a=0.0, prior_b=s0)
    g = np.arange(lo, hi + 0.5 * h, h)
    G = g.size
    wts = np.full(G, h)
    wts[0] = wts[-1] = 0.5 * h
    logs = np.empty((G, G))
    for r in range(G):
        theta = np.vstack([np.full(G, g[r]), g])                  # mu1 = g[r], mu2 = grid
        logs[r] = per_datum_loglik(theta, y, model).sum(axis=1) + log_prior(theta, model)
    mx = float(logs.max())
    return mx + math.log(float(np.sum(np.exp(logs - mx) * wts[:, None] * wts[None, :])))
