"""Pins for the factor stochastic-volatility particle filter oracle (Factor
Stochastic Volatility subsection; Sequential Monte Carlo subsection)."""

import dataclasses
import math

import numpy as np
import pytest
from scipy import integrate, stats

from oracle import fsv
from workloads.fsv import PAPER_FSV, FsvModel, simulate


def test_observation_density_matches_scipy():
    rng = np.random.default_rng(1)
    x = rng.normal(scale=1.5, size=(3, 7))
    y = rng.normal(size=5)
    got = fsv.log_obs_density(PAPER_FSV, y, x)
    B, psi = np.asarray(PAPER_FSV.B), np.asarray(PAPER_FSV.psi)
    for p in range(7):
        S = B @ np.diag(np.exp(x[:, p])) @ B.T + np.diag(psi)
        assert abs(got[p] - stats.multivariate_normal(mean=np.zeros(5), cov=S).logpdf(y)) < 1e-12


def test_no_transition_noise_gives_the_closed_form():
    """With U -> 0 every particle stays at x = 0, so each increment is
    log N(y_t; 0, B B^T + Psi) exactly and no resampling happens."""
    model = dataclasses.replace(PAPER_FSV, U=tuple(tuple(1e-30 * (i == j) for j in range(3))
                                                   for i in range(3)))
    _, y = simulate(PAPER_FSV, 12, 4)
    r = fsv.particle_filter(y, model, 64, 2)
    B, psi = np.asarray(PAPER_FSV.B), np.asarray(PAPER_FSV.psi)
    S = B @ B.T + np.diag(psi)
    want = sum(stats.multivariate_normal(mean=np.zeros(5), cov=S).logpdf(yt) for yt in y)
    assert abs(r["loglik"] - want) < 1e-9
    assert not r["resampled"].any()
    assert np.max(np.abs(r["mean"])) < 1e-12


def test_grid_filter_matches_adaptive_quadrature():
    """phi = 0 makes the steps independent: p(y_t) = int N(y_t; 0, b^2 e^x + psi) N(x; 0, u) dx,
    integrated by scipy's adaptive quadrature."""
    b, psi, u = 1.3, 0.4, 0.7
    y = np.array([0.3, -1.7, 2.4, 0.05])
    want = 0.0
    for yt in y:
        f = lambda x: (stats.norm.pdf(yt, scale=math.sqrt(b * b * math.exp(x) + psi))
                       * stats.norm.pdf(x, scale=math.sqrt(u)))
        want += math.log(integrate.quad(f, -12, 12, epsabs=1e-14, epsrel=1e-12)[0])
    got = fsv.grid_loglik_scalar(y, b, psi, 0.0, u)
    assert abs(got - want) < 1e-8


@pytest.mark.slow
def test_particle_filter_loglik_agrees_with_grid_filter():
    """Scalar model (K = M = 1): the particle-filter log-likelihood over 8 seeds
    agrees with the deterministic grid filter within 4 standard errors."""
    model = FsvModel(B=((1.1,),), psi=(0.5,), phi=(0.9,), U=((0.5,),))
    _, y = simulate(model, 20, 9)
    exact = fsv.grid_loglik_scalar(y[:, 0], 1.1, 0.5, 0.9, 0.5)
    z = np.array([fsv.particle_filter(y, model, 1 << 14, s)["loglik"] for s in range(8)])
    se = z.std(ddof=1) / math.sqrt(z.size)
    assert abs(z.mean() - exact) < 4 * se + 1e-3


def test_one_step_transition_covariance():
    """After one step from x_0 = 0 the particles are N(0, U) draws."""
    x = fsv.propagate(PAPER_FSV, np.zeros((3, 1 << 16)), 5, 1)
    C = np.cov(x)
    assert np.max(np.abs(C - np.asarray(PAPER_FSV.U))) < 0.02
    assert np.max(np.abs(x.mean(axis=1))) < 0.01


def test_filter_tracks_the_simulated_path():
    x, y = simulate(PAPER_FSV, 200, 7)
    r = fsv.particle_filter(y, PAPER_FSV, 2048, 3)
    for c in range(3):
        assert np.corrcoef(r["mean"][:, c], x[1:, c])[0, 1] > 0.4
    assert 0 < r["resampled"].sum() < 200
    assert np.all(r["sd"] > 0)
