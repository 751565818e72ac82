"""Pins for the oracle's stratified and multinomial resampling and the 53-bit
uniform map (Sequential Monte Carlo subsection: resampling draws the new
population from the empirical CDF of the weights)."""

import math

import numpy as np
import pytest

from oracle import philox as px
from oracle import smc
from oracle.gmm import Model
from workloads import beta_schedule, lognormal_logw, make_mixture_data


def test_u01_53_map():
    assert px.u01_53(0, 0) == 0.0
    assert px.u01_53(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0 ** -53
    assert px.u01_53(1, 0) == 2.0 ** -32
    assert px.u01_53(0, 1 << 11) == 2.0 ** -53
    assert px.u01_53(0, (1 << 11) - 1) == 0.0          # the low 11 bits are dropped
    w = np.arange(0, 1 << 32, 65537, dtype=np.uint64)
    u = px.u01_53(w, w)
    assert np.all(np.diff(u) > 0) and np.all(u < 1.0)


def test_stratified_points_one_per_stratum():
    for N in (1, 7, 1000, 4096):
        U = smc.resample_points(N, "stratified", 5, 3)
        i = np.arange(N)
        assert np.all(U >= i / N) and np.all(U < (i + 1) / N)


@pytest.mark.parametrize("N", [1, 2, 1024, 1 << 16])
def test_uniform_weights_closed_forms(N):
    """N a power of two and W = 1/N: C_j = (j+1)/N exactly, so stratified
    resampling is the identity and multinomial gives floor(N u_i)."""
    W = np.full(N, 1.0 / N)
    assert np.array_equal(smc.resample_indices(W, "stratified", 9, 2), np.arange(N, dtype=np.int32))
    u = smc.per_index_uniforms(9, 2, N, "multinomial")
    assert np.array_equal(smc.resample_indices(W, "multinomial", 9, 2),
                          np.floor(u * N).astype(np.int32))


@pytest.mark.parametrize("scheme", smc.SCHEMES)
def test_one_hot_and_zero_weights(scheme):
    W = np.zeros(333)
    W[100] = 1.0
    assert np.all(smc.resample_indices(W, scheme, 1, 1) == 100)
    W = smc.normalise(lognormal_logw(500, seed=4))
    W[::3] = 0.0
    W /= W.sum()
    idx = smc.resample_indices(W, scheme, 2, 7)
    assert np.all(W[idx] > 0.0)


def test_stratified_counts_within_two_of_expectation():
    for N, seed in ((1000, 1), (4096, 2)):
        W = smc.normalise(lognormal_logw(N, seed=seed))
        for step in range(5):
            idx = smc.resample_indices(W, "stratified", seed, step)
            assert np.all(np.diff(idx) >= 0)
            counts = np.bincount(idx, minlength=N)
            assert np.all(np.abs(counts - N * W) < 2.0 + 1e-9)


@pytest.mark.parametrize("scheme", ["stratified", "multinomial"])
def test_counts_are_unbiased(scheme):
    """E[count_j] = N W_j: the mean over R independent steps is within 5
    standard errors of N W_j (multinomial variance bounds the stratified one)."""
    N, R = 16, 4000
    W = smc.normalise(np.log(np.arange(1, N + 1, dtype=np.float64)))
    counts = np.zeros(N)
    for step in range(R):
        counts += np.bincount(smc.resample_indices(W, scheme, 77, step), minlength=N)
    mean = counts / R
    se = np.sqrt(N * W * (1 - W) / R)
    assert np.all(np.abs(mean - N * W) < 5 * se + 1e-12)


def test_multinomial_count_variance():
    """Multinomial counts have variance N W (1 - W)."""
    N, R = 8, 6000
    W = np.array([0.3, 0.2, 0.15, 0.1, 0.1, 0.08, 0.05, 0.02])
    c = np.array([np.bincount(smc.resample_indices(W, "multinomial", 3, s), minlength=N)
                  for s in range(R)], dtype=np.float64)
    var = c.var(axis=0, ddof=1)
    want = N * W * (1 - W)
    # the sample variance of R draws has relative sd about sqrt(2/R) (plus kurtosis)
    assert np.all(np.abs(var / want - 1.0) < 0.12)


@pytest.mark.parametrize("scheme", smc.SCHEMES)
def test_search_matches_exact_rational_bruteforce(scheme):
    rng = np.random.default_rng(23)
    for trial in range(300):
        N = int(rng.integers(1, 9))
        raw = rng.exponential(size=N) * (rng.random(N) < 0.8)
        if raw.sum() == 0:
            raw[0] = 1.0
        W = raw / raw.sum()
        U = smc.resample_points(N, scheme, trial, 5)
        assert np.array_equal(smc.search_cdf(W, U), smc.search_bruteforce(W, U)), (W, U)


def test_systematic_scheme_is_the_systematic_resampler():
    W = smc.normalise(lognormal_logw(2049, seed=8))
    assert np.array_equal(smc.resample_indices(W, "systematic", 4, 6),
                          smc.systematic_resample(W, smc.resample_offset(4, 6)))


@pytest.mark.slow
@pytest.mark.parametrize("scheme", ["stratified", "multinomial"])
def test_smc_logz_k1_closed_form_other_schemes(scheme):
    """The SMC sampler's log-evidence with stratified or multinomial resampling
    agrees with the k = 1 closed form (conjugate Gaussian) within 4 SE."""
    from oracle import evidence
    y = make_mixture_data(100, np.array([1.5]), 0.55, seed=12)
    m = Model.equal_weights(1, 1, 0.55)
    betas = beta_schedule(30, "quadratic")
    z = np.array([smc.smc_run(y, m, betas, 4096, 0.5, 2, seed=s, scheme=scheme)["logZ"]
                  for s in range(6)])
    exact = evidence.log_z_tempered_k1(y, 0.55, 1.0)
    se = z.std(ddof=1) / math.sqrt(z.size)
    assert abs(z.mean() - exact) < 4 * se + 0.02
