"""Gaussian-mixture log-likelihood and log-priors, plain FP64 definitions.

Mixture Modelling section of the paper: observations y_1..y_n are i.i.d. from
sum_i w_i f(y | mu_i, sigma_i) with known k, weights and variance; the
likelihood of the data is the product over observations. Here f is the
d-variate normal with covariance sigma2 * I (d = 1 in the paper), so

    l(mu) = sum_j log sum_i w_i (2 pi sigma2)^(-d/2) exp(-||y_j - mu_i||^2 / (2 sigma2)).

Each datum's inner sum is evaluated as a max-shifted log-sum-exp in FP64 and
the squared distance is formed directly from the differences (never by
expanding the square). The data are the float32 observations widened to FP64,
exactly the values the GPU reads, so a comparison measures only arithmetic.

Parameter layout: theta is [k*d][N] (component-major structure of arrays),
entry (i*d + c, p) = coordinate c of mean i of particle p.

Priors: the paper's uniform prior on the hypercube [-10, 10]^k, and the
N(a, b^2) prior on every coordinate used by the scaled workloads. Both are
normalised densities, because the log-evidence needs them.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Sequence

import numpy as np


@dataclasses.dataclass(frozen=True)
class Model:
    k: int
    d: int
    sigma2: float
    log_w: Sequence[float]
    prior: str = "gauss"        # "gauss": N(prior_a, prior_b^2); "box": U[prior_a, prior_b]
    prior_a: float = 0.0
    prior_b: float = 10.0

    @staticmethod
    def equal_weights(k, d, sigma2, **kw):
        return Model(k=k, d=d, sigma2=sigma2, log_w=tuple([math.log(1.0 / k)] * k), **kw)


def _as_2d_data(y, d):
    y = np.asarray(y)
    return y.astype(np.float64).reshape(-1, d)


def per_datum_loglik(theta, y, model: Model) -> np.ndarray:
    """log p(y_j | mu_p) for every particle p and datum j, shape (N, n)."""
    k, d = model.k, model.d
    theta = np.asarray(theta, dtype=np.float64)
    N = theta.shape[1]
    Y = _as_2d_data(y, d)                                   # (n, d)
    mu = theta.reshape(k, d, N)                             # (k, d, N)
    log_w = np.asarray(model.log_w, dtype=np.float64)
    # squared distance ||y_j - mu_{p,i}||^2 formed from the differences
    diff = Y[None, :, None, :] - np.transpose(mu, (2, 0, 1))[:, None, :, :]   # (N, n, k, d)
    sq = np.sum(diff * diff, axis=-1)                       # (N, n, k)
    a = log_w[None, None, :] - sq / (2.0 * model.sigma2)    # log w_i + log kernel
    m = np.max(a, axis=-1)
    lse = m + np.log(np.sum(np.exp(a - m[..., None]), axis=-1))
    return lse - 0.5 * d * math.log(2.0 * math.pi * model.sigma2)


def loglik(theta, y, model: Model, chunk_elems: int = 1 << 22) -> np.ndarray:
    """Per-particle log-likelihood l(mu_p) = sum_j log p(y_j | mu_p), shape (N,)."""
    theta = np.asarray(theta, dtype=np.float64)
    N = theta.shape[1]
    n = np.asarray(y).reshape(-1, model.d).shape[0]
    step = max(1, chunk_elems // max(1, n * model.k * model.d))
    out = np.empty(N, dtype=np.float64)
    for s in range(0, N, step):
        out[s:s + step] = per_datum_loglik(theta[:, s:s + step], y, model).sum(axis=1)
    return out


def log_prior(theta, model: Model) -> np.ndarray:
    """Normalised log prior density of each particle, shape (N,)."""
    theta = np.asarray(theta, dtype=np.float64)
    kd = model.k * model.d
    if model.prior == "gauss":
        a, b = model.prior_a, model.prior_b
        z = theta - a
        return np.sum(-0.5 * math.log(2.0 * math.pi * b * b) - (z * z) / (2.0 * b * b), axis=0)
    if model.prior == "box":
        lo, hi = model.prior_a, model.prior_b
        inside = np.all((theta >= lo) & (theta <= hi), axis=0)
        return np.where(inside, -kd * math.log(hi - lo), -np.inf)
    raise ValueError(model.prior)
