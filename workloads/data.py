"""Seeded input generators (numpy PCG64; not the method's own random numbers)."""

from __future__ import annotations

from typing import Optional, Sequence

import numpy as np

from .configs import WorkloadConfig


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def make_mixture_data(n: int, means: np.ndarray, sigma2: float, seed: int,
                      weights: Optional[Sequence[float]] = None) -> np.ndarray:
    """n observations from sum_i w_i N(mu_i, sigma2 I), rounded to float32.

    ``means`` has shape (k,) for 1-D data or (k, d). Returns shape (n,) for 1-D
    and (n, d) row-major otherwise.
    """
    means = np.asarray(means, dtype=np.float64)
    one_d = means.ndim == 1
    mu = means.reshape(means.shape[0], -1)
    k, d = mu.shape
    rng = _rng(seed)
    p = None if weights is None else np.asarray(weights, dtype=np.float64)
    z = rng.choice(k, size=n, p=p)
    y = mu[z] + np.sqrt(sigma2) * rng.standard_normal((n, d))
    y = y.astype(np.float32)
    return y.reshape(n) if one_d else y


def true_means_for(cfg: WorkloadConfig) -> np.ndarray:
    if cfg.true_means is not None:
        mu = np.asarray(cfg.true_means, dtype=np.float64)
        return mu if cfg.d == 1 else mu.reshape(cfg.k, cfg.d)
    rng = _rng(cfg.data_seed + 1_000_003)
    mu = cfg.true_mean_sd * rng.standard_normal((cfg.k, cfg.d))
    return mu.reshape(cfg.k) if cfg.d == 1 else mu


def make_data(cfg: WorkloadConfig) -> np.ndarray:
    """The workload's observations (float32; shape (n,) or (n, d))."""
    return make_mixture_data(cfg.n, true_means_for(cfg), cfg.sigma2, cfg.data_seed)


def beta_schedule(T: int, kind: str) -> np.ndarray:
    """Inverse temperatures beta_0..beta_T in FP64, computed once on the host.

    "linear": t/T; "quadratic": (t/T)^2 (the paper's cooling schedule with
    T = 200). Both sides of every comparison receive this same array.
    """
    t = np.arange(T + 1, dtype=np.float64)
    if kind == "linear":
        b = t / T
    elif kind == "quadratic":
        b = (t * t) / float(T * T)
    else:
        raise ValueError(kind)
    b[0] = 0.0
    b[-1] = 1.0
    return b


def pt_betas(M: int, power: int = 4) -> np.ndarray:
    """Parallel-tempering ladder beta_i = (i/M)^power, i = 1..M (index i-1)."""
    i = np.arange(1, M + 1, dtype=np.float64)
    b = (i / M) ** power
    b[-1] = 1.0
    return b


def theta_prior_draws(N: int, k: int, d: int, seed: int, a: float = 0.0,
                      b: float = 10.0) -> np.ndarray:
    """Probe parameters drawn from N(a, b^2), layout [k*d][N] (component-major SoA)."""
    rng = _rng(seed)
    return (a + b * rng.standard_normal((k * d, N))).astype(np.float64)


def theta_near_posterior(N: int, true_means: np.ndarray, seed: int,
                         jitter: float = 0.1) -> np.ndarray:
    """Probe parameters near a posterior mode: a random relabelling of the true
    means plus N(0, jitter^2) noise, layout [k*d][N]."""
    mu = np.asarray(true_means, dtype=np.float64)
    mu = mu.reshape(mu.shape[0], -1)
    k, d = mu.shape
    rng = _rng(seed)
    perm = np.argsort(rng.random((N, k)), axis=1)          # one relabelling per particle
    out = mu[perm].reshape(N, k * d).T.copy()              # [k*d][N]
    out += jitter * rng.standard_normal(out.shape)
    return out


def lognormal_logw(N: int, seed: int, spread: float = 3.0) -> np.ndarray:
    """Unnormalised log-weights with log-normal spread, for reweight/resample probes."""
    rng = _rng(seed)
    return spread * rng.standard_normal(N)
