"""Pins for the oracle's mixture log-likelihood and priors."""

import json
import math
import os

import numpy as np
from scipy import stats

from oracle import gmm, smc
from oracle.gmm import Model
from workloads import make_mixture_data, theta_prior_draws, theta_near_posterior

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _model(k=4, d=1, sigma2=0.55, **kw):
    return Model.equal_weights(k, d, sigma2, **kw)


def test_permutation_invariance_1d():
    """Relabelling the components leaves the likelihood unchanged (k! symmetric modes)."""
    y = make_mixture_data(200, np.array([-3.0, 0.0, 3.0, 6.0]), 0.55, seed=11)
    m = _model()
    th = np.vstack([theta_prior_draws(64, 4, 1, seed=3),
                    ])
    th = np.hstack([th, theta_near_posterior(64, np.array([-3.0, 0.0, 3.0, 6.0]), seed=4)])
    base = gmm.loglik(th, y, m)
    rng = np.random.default_rng(0)
    for _ in range(5):
        perm = rng.permutation(4)
        np.testing.assert_allclose(gmm.loglik(th[perm], y, m), base, rtol=1e-13, atol=0)


def test_permutation_invariance_ddim():
    mu = np.random.default_rng(1).normal(0, 3, size=(3, 2))
    y = make_mixture_data(50, mu, 1.0, seed=5)
    m = _model(k=3, d=2, sigma2=1.0)
    th = theta_prior_draws(16, 3, 2, seed=8)
    base = gmm.loglik(th, y, m)
    perm = [2, 0, 1]
    thp = th.reshape(3, 2, -1)[perm].reshape(6, -1)
    np.testing.assert_allclose(gmm.loglik(thp, y, m), base, rtol=1e-13)


def test_k1_closed_form():
    y = make_mixture_data(300, np.array([1.0]), 0.7, seed=2).astype(np.float64)
    mu = np.array([[-4.0, 0.3, 1.1, 25.0]])
    got = gmm.loglik(mu, y, _model(k=1, sigma2=0.7))
    want = np.array([-0.5 * y.size * math.log(2 * math.pi * 0.7)
                     - np.sum((y - m) ** 2) / (2 * 0.7) for m in mu[0]])
    np.testing.assert_allclose(got, want, rtol=1e-12)


def test_equal_means_reduce_to_one_component():
    y = make_mixture_data(100, np.array([-3.0, 0.0, 3.0, 6.0]), 0.55, seed=1)
    mus = np.array([-2.0, 0.5, 7.0])
    th = np.tile(mus, (4, 1))
    got = gmm.loglik(th, y, _model())
    want = gmm.loglik(mus[None, :], y, _model(k=1))
    np.testing.assert_allclose(got, want, rtol=1e-13)


def test_tiny_n_direct_product_of_densities():
    """Brute force: log of the product of mixture densities from scipy's normal pdf."""
    y = np.array([-1.25, 0.5, 3.0, 6.5], dtype=np.float32)
    th = np.array([[-3.0, 1.0], [0.0, 2.0], [3.0, -9.0], [6.0, 4.5]])
    w = np.array([0.1, 0.2, 0.3, 0.4])
    m = Model(k=4, d=1, sigma2=0.55, log_w=tuple(np.log(w)))
    got = gmm.loglik(th, y, m)
    for p in range(2):
        dens = [np.sum(w * stats.norm.pdf(float(yy), loc=th[:, p], scale=math.sqrt(0.55)))
                for yy in y]
        assert abs(got[p] - math.log(np.prod(dens))) <= 1e-12 * abs(got[p])


def test_tiny_n_direct_product_ddim():
    rng = np.random.default_rng(3)
    k, d = 3, 4
    y = rng.normal(size=(3, d)).astype(np.float32)
    th = rng.normal(size=(k * d, 2))
    m = _model(k=k, d=d, sigma2=1.3)
    got = gmm.loglik(th, y, m)
    for p in range(2):
        mu = th[:, p].reshape(k, d)
        dens = [np.mean([stats.multivariate_normal.pdf(yy.astype(np.float64), mean=mu[i],
                                                       cov=1.3 * np.eye(d)) for i in range(k)])
                for yy in y]
        assert abs(got[p] - math.log(np.prod(dens))) <= 1e-12 * abs(got[p])


def test_ddim_identity_covariance_factorises_for_k1():
    rng = np.random.default_rng(4)
    d = 5
    y = rng.normal(size=(40, d)).astype(np.float32)
    mu = rng.normal(size=(d, 3))
    got = gmm.loglik(mu, y, _model(k=1, d=d, sigma2=0.8))
    want = sum(gmm.loglik(mu[c:c + 1], y[:, c], _model(k=1, d=1, sigma2=0.8)) for c in range(d))
    np.testing.assert_allclose(got, want, rtol=1e-12)


def test_is_worked_example_second_moment():
    """The importance-sampling example's target density, written as a one-datum
    mixture likelihood, integrates x^2 to the closed-form 1.875."""
    g = json.load(open(os.path.join(GOLD, "is_example.json")))
    m = Model(k=2, d=1, sigma2=g["variance"], log_w=tuple(np.log(g["weights"])))
    th = np.array(g["means"])[:, None]
    xs = np.linspace(-12.0, 12.0, 48001)
    dens = np.array([math.exp(gmm.loglik(th, np.array([x], dtype=np.float64), m)[0]) for x in xs[::40]])
    h = xs[40] - xs[0]
    x = xs[::40]
    # trapezoid over a smooth, rapidly decaying integrand
    val = h * (np.sum(x * x * dens) - 0.5 * (x[0] ** 2 * dens[0] + x[-1] ** 2 * dens[-1]))
    mass = h * (np.sum(dens) - 0.5 * (dens[0] + dens[-1]))
    assert abs(mass - 1.0) < 1e-10
    assert abs(val - g["second_moment"]) < 1e-10


def test_paper_model_symmetry_count():
    g = json.load(open(os.path.join(GOLD, "paper_model.json")))
    assert math.factorial(g["k"]) == g["n_modes"]
    h = sum(1.0 / i for i in range(1, g["n_modes"] + 1))
    assert round(g["n_modes"] * h) == g["coupon_collector_expectation_approx"]
    # every relabelling of the true means gives the same likelihood
    y = make_mixture_data(g["m"], np.array(g["true_means"]), g["sigma"] ** 2, seed=1)
    m = Model(k=4, d=1, sigma2=g["sigma"] ** 2, log_w=tuple(np.log(g["weights"])),
              prior="box", prior_a=g["prior_box"][0], prior_b=g["prior_box"][1])
    import itertools
    perms = np.array(list(itertools.permutations(g["true_means"]))).T
    assert perms.shape[1] == g["n_modes"]
    l = gmm.loglik(perms, y, m)
    assert np.ptp(l) <= 1e-12 * abs(l[0])


def test_log_prior_gauss_matches_scipy():
    th = theta_prior_draws(10, 4, 1, seed=9)
    m = _model(prior="gauss", prior_a=1.0, prior_b=10.0)
    want = stats.norm.logpdf(th, loc=1.0, scale=10.0).sum(axis=0)
    np.testing.assert_allclose(gmm.log_prior(th, m), want, rtol=1e-13)


def test_log_prior_box():
    m = _model(prior="box", prior_a=-10.0, prior_b=10.0)
    th = np.array([[0.0, 9.9, 10.5], [1.0, -10.0, 0.0], [2.0, 0.0, 0.0], [3.0, 0.0, 0.0]])
    lp = gmm.log_prior(th, m)
    assert lp[0] == lp[1] == -4 * math.log(20.0)
    assert lp[2] == -np.inf


def test_prior_draws_have_prior_moments():
    m = _model(prior="gauss", prior_a=0.0, prior_b=10.0)
    th = smc.prior_init(m, 1 << 15, seed=31)
    assert abs(th.mean()) < 4 * 10.0 / math.sqrt(th.size)
    assert abs(th.std() - 10.0) < 0.1
    mb = _model(prior="box", prior_a=-10.0, prior_b=10.0)
    tb = smc.prior_init(mb, 1 << 15, seed=31)
    assert tb.min() > -10.0 and tb.max() < 10.0
    assert abs(tb.var() - 400.0 / 12.0) < 0.5
