"""Pins for the log-evidence references and the oracle SMC sampler built on them."""

import math

import numpy as np
import pytest

from oracle import evidence, gmm, smc
from oracle.gmm import Model
from workloads import beta_schedule, make_mixture_data


def _k2_data():
    return make_mixture_data(20, np.array([-2.0, 2.0]), 0.55, seed=7)


def test_k2_enumeration_matches_2d_quadrature():
    y = _k2_data()
    a = evidence.log_z_enumerate_k2(y, 0.55)
    b = evidence.log_z_quadrature_k2(y, 0.55)
    assert abs(a - b) < 1e-8


def test_k1_closed_form_matches_quadrature():
    y = make_mixture_data(30, np.array([1.0]), 0.55, seed=4)
    m = Model.equal_weights(1, 1, 0.55)
    g = np.arange(-40.0, 40.0, 0.002)
    l = gmm.loglik(g[None, :], y, m)
    lp = gmm.log_prior(g[None, :], m)
    for beta in (0.01, 0.3, 1.0):
        v = beta * l + lp
        mx = v.max()
        q = mx + math.log(np.trapezoid(np.exp(v - mx), g))
        assert abs(q - evidence.log_z_tempered_k1(y, 0.55, beta)) < 1e-8


def _smc_logz(y, model, betas, N, seeds, n_moves=2):
    return np.array([smc.smc_run(y, model, betas, N, 0.5, n_moves, seed=s)["logZ"] for s in seeds])


@pytest.mark.slow
def test_smc_logz_k1_closed_form():
    y = make_mixture_data(100, np.array([1.5]), 0.55, seed=12)
    m = Model.equal_weights(1, 1, 0.55)
    betas = beta_schedule(30, "quadratic")
    z = _smc_logz(y, m, betas, 4096, range(6))
    exact = evidence.log_z_tempered_k1(y, 0.55, 1.0)
    se = z.std(ddof=1) / math.sqrt(z.size)
    assert abs(z.mean() - exact) < 4 * se + 0.02


@pytest.mark.slow
def test_smc_logz_k2_exact_enumeration():
    y = _k2_data()
    m = Model.equal_weights(2, 1, 0.55)
    betas = beta_schedule(40, "quadratic")
    z = _smc_logz(y, m, betas, 8192, range(6))
    exact = evidence.log_z_enumerate_k2(y, 0.55)
    se = z.std(ddof=1) / math.sqrt(z.size)
    assert abs(z.mean() - exact) < 4 * se + 0.02


def test_single_step_smc_is_importance_sampling_from_prior():
    """beta 0 -> 1 in one step with no resampling and no move: the estimate is
    log of the mean likelihood of the prior draws."""
    y = make_mixture_data(10, np.array([-1.0, 1.0]), 0.55, seed=2)
    m = Model.equal_weights(2, 1, 0.55)
    out = smc.smc_run(y, m, np.array([0.0, 1.0]), 512, 0.5, 0, seed=3, resample=False)
    th = smc.prior_init(m, 512, 3)
    l = gmm.loglik(th, y, m)
    mx = l.max()
    assert abs(out["logZ"] - (mx + math.log(np.mean(np.exp(l - mx))))) < 1e-10
