"""Factor stochastic-volatility model and simulated observations (Factor
Stochastic Volatility subsection): the paper's parameters and a seeded draw of
the latent path and the observations. Inputs only; none of the filter."""

from __future__ import annotations

import dataclasses
from typing import Tuple

import numpy as np


@dataclasses.dataclass(frozen=True)
class FsvModel:
    """y_t ~ N(0, B diag(exp(x_t)) B^T + diag(psi)), x_t ~ N(diag(phi) x_{t-1}, U)."""
    B: Tuple[Tuple[float, ...], ...]     # M x K factor loadings (zero above the diagonal)
    psi: Tuple[float, ...]               # M idiosyncratic variances
    phi: Tuple[float, ...]               # K autoregression coefficients
    U: Tuple[Tuple[float, ...], ...]     # K x K innovation covariance

    @property
    def m(self) -> int:
        return len(self.psi)

    @property
    def k(self) -> int:
        return len(self.phi)


PAPER_FSV = FsvModel(
    B=((1.0, 0.0, 0.0), (0.5, 1.0, 0.0), (0.5, 0.5, 1.0), (0.2, 0.6, 0.3), (0.8, 0.7, 0.5)),
    psi=(0.5,) * 5,
    phi=(0.9,) * 3,
    U=((0.5, 0.2, 0.1), (0.2, 0.5, 0.2), (0.1, 0.2, 0.5)))


def simulate(model: FsvModel, T: int, seed: int):
    """x_0 = 0; for t = 1..T: x_t = Phi x_{t-1} + chol(U) e_t, f_t ~ N(0, diag(exp(x_t))),
    y_t = B f_t + sqrt(psi) * eta_t. Returns (x [T+1][K], y [T][M]) in FP64."""
    rng = np.random.Generator(np.random.PCG64(seed))
    B = np.asarray(model.B)
    L = np.linalg.cholesky(np.asarray(model.U))
    phi = np.asarray(model.phi)
    psi = np.asarray(model.psi)
    x = np.zeros((T + 1, model.k))
    y = np.zeros((T, model.m))
    for t in range(1, T + 1):
        x[t] = phi * x[t - 1] + L @ rng.standard_normal(model.k)
        f = np.exp(0.5 * x[t]) * rng.standard_normal(model.k)
        y[t - 1] = B @ f + np.sqrt(psi) * rng.standard_normal(model.m)
    return x, y
