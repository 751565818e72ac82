"""Bootstrap particle filter for the factor stochastic-volatility model, plain
FP64 (TEST INFRASTRUCTURE, like the rest of this package).

Factor Stochastic Volatility subsection: latent x_t (K factors' log-variances)
with x_t ~ N(Phi x_{t-1}, U), x_0 = 0, and observations
y_t | x_t ~ N(0, B diag(exp(x_t)) B^T + Psi). Sequential Monte Carlo subsection:
particles are propagated by the transition, weighted by the observation
density, and resampled from the empirical CDF of the weights when the
effective sample size falls below ess_frac * N.

Readings (listed in the design notes): the filter starts from x_0 = 0 for every
particle; resampling is systematic with the ESS < N/2 rule of the SMC sampler;
the transition noise of particle p at time t is the Philox normals of stream
(p, 0, t, PROP, 0); the filtered mean and standard deviation at time t are the
weighted moments before resampling; the log-likelihood estimate is
sum_t log sum_p W_p^{(t-1)} g(y_t | x_t^p).
"""

from __future__ import annotations

import math

import numpy as np

from . import philox as px
from .smc import reweight, resample_offset, systematic_resample


def arrays(model):
    return (np.asarray(model.B, dtype=np.float64), np.asarray(model.psi, dtype=np.float64),
            np.asarray(model.phi, dtype=np.float64), np.asarray(model.U, dtype=np.float64))


def obs_cov(model, x):
    """Sigma_p = B diag(exp(x_p)) B^T + diag(psi) for every particle: [N][M][M]."""
    B, psi, _, _ = arrays(model)
    h = np.exp(np.asarray(x, dtype=np.float64)).T            # [N][K]
    return np.einsum("ak,nk,bk->nab", B, h, B) + np.diag(psi)[None]


def log_obs_density(model, y_t, x):
    """log N(y_t; 0, Sigma_p) for every particle (library slogdet and solve)."""
    S = obs_cov(model, x)
    m = S.shape[-1]
    sign, logdet = np.linalg.slogdet(S)
    yb = np.broadcast_to(np.asarray(y_t, dtype=np.float64), S.shape[:-1])
    v = np.linalg.solve(S, yb[..., None])[..., 0]
    quad = np.einsum("na,na->n", v, yb)
    return -0.5 * m * math.log(2.0 * math.pi) - 0.5 * logdet - 0.5 * quad


def propagate(model, x, seed, t):
    """x_t = Phi x_{t-1} + chol(U) z, z = the Philox normals of stream (p, 0, t, PROP, 0)."""
    _, _, phi, U = arrays(model)
    K, N = x.shape
    z = px.normals(seed, np.arange(N, dtype=np.uint64), t, px.PROP, 0, K)
    return phi[:, None] * x + np.linalg.cholesky(U) @ z


def particle_filter(y, model, N, seed, ess_frac=0.5):
    """Run the filter over y [T][M]. Returns dict(loglik, loglik_inc [T], mean [T][K],
    sd [T][K], ess [T], resampled [T], x, logw, x_end, logw_end): x, logw are the
    final population before its resampling, x_end, logw_end after it."""
    y = np.asarray(y, dtype=np.float64)
    T = y.shape[0]
    K = model.k
    x = np.zeros((K, N))
    logw = np.zeros(N)
    out = dict(loglik_inc=[], mean=[], sd=[], ess=[], resampled=[])
    for t in range(1, T + 1):
        x = propagate(model, x, seed, t)
        lg = log_obs_density(model, y[t - 1], x)
        logw, W, inc, e = reweight(logw, lg, 1.0)
        mean = x @ W
        sd = np.sqrt(np.maximum((x * x) @ W - mean * mean, 0.0))
        out["loglik_inc"].append(inc)
        out["mean"].append(mean)
        out["sd"].append(sd)
        out["ess"].append(e)
        fire = bool(e < ess_frac * N)
        out["resampled"].append(fire)
        if t == T:
            out["x"], out["logw"] = x.copy(), logw.copy()
        if fire:
            idx = systematic_resample(W, resample_offset(seed, t))
            x = x[:, idx]
            logw = np.zeros(N)
    out["x_end"], out["logw_end"] = x, logw             # after the last step's resampling
    out["loglik"] = float(np.sum(out["loglik_inc"]))
    for key in ("loglik_inc", "ess"):
        out[key] = np.asarray(out[key])
    out["mean"] = np.asarray(out["mean"])
    out["sd"] = np.asarray(out["sd"])
    out["resampled"] = np.asarray(out["resampled"])
    return out


def grid_loglik_scalar(y, b, psi, phi, u, half_width=8.0, points=4001):
    """Exact-up-to-quadrature log p(y_1:T) of the scalar model (K = M = 1):
    x_t ~ N(phi x_{t-1}, u), x_0 = 0, y_t ~ N(0, b^2 exp(x_t) + psi), by a
    deterministic grid filter (trapezoid rule on a uniform grid)."""
    g = np.linspace(-half_width, half_width, points)
    h = g[1] - g[0]
    w = np.full(points, h)
    w[0] = w[-1] = h / 2
    trans = np.exp(-0.5 * (g[:, None] - phi * g[None, :]) ** 2 / u) / math.sqrt(2 * math.pi * u)
    pred = np.exp(-0.5 * g ** 2 / u) / math.sqrt(2 * math.pi * u)     # p(x_1), x_0 = 0
    total = 0.0
    for t, yt in enumerate(np.asarray(y, dtype=np.float64).ravel()):
        if t > 0:
            pred = trans @ (w * filt)
        var = b * b * np.exp(g) + psi
        like = np.exp(-0.5 * yt * yt / var) / np.sqrt(2 * math.pi * var)
        joint = pred * like
        py = float(np.sum(w * joint))
        total += math.log(py)
        filt = joint / py
    return total
