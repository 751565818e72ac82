"""Pins for the oracle's reweighting, normalisation, ESS and systematic resampling."""

import math
from fractions import Fraction

import numpy as np
import pytest
from hypothesis import example, given, settings, strategies as st

from oracle import evidence, gmm, smc
from oracle.gmm import Model
from workloads import lognormal_logw, make_mixture_data

EPS = 2.0 ** -52


# ------------------------------------------------------------------ weights

def test_normalised_weights_sum_to_one():
    for N in (1, 7, 1024, 100003):
        W = smc.normalise(lognormal_logw(N, seed=N))
        assert abs(W.sum() - 1.0) <= N * EPS


def test_ess_special_cases():
    for N in (1, 2, 64, 1 << 16):
        assert smc.ess(np.full(N, 1.0 / N)) == N          # exact for powers of two
    W = np.zeros(1000)
    W[17] = 1.0
    assert smc.ess(W) == 1.0
    W = smc.normalise(lognormal_logw(5000, seed=3))
    e = smc.ess(W)
    assert 1.0 <= e <= 5000.0


def test_reweight_is_shift_invariant():
    logw = lognormal_logw(4096, seed=5)
    l = -1000.0 + 10.0 * lognormal_logw(4096, seed=6)
    a = smc.reweight(logw, l, 0.03)
    b = smc.reweight(logw + 123.456, l, 0.03)
    np.testing.assert_allclose(a[1], b[1], rtol=1e-12, atol=1e-300)
    assert abs(a[2] - b[2]) < 1e-9
    assert abs(a[3] - b[3]) < 1e-9 * a[3]


def test_reweight_increment_is_log_mean_incremental_weight():
    """With equal weights the increment is log((1/N) sum exp(dbeta l))."""
    N = 1000
    l = np.linspace(-50.0, -10.0, N)
    _, W, inc, _ = smc.reweight(np.zeros(N), l, 0.5)
    want = math.log(np.mean(np.exp(0.5 * l)))
    assert abs(inc - want) < 1e-12
    np.testing.assert_allclose(W, np.exp(0.5 * l) / np.sum(np.exp(0.5 * l)), rtol=1e-12)


def test_reweight_increment_matches_closed_form_ratio_k1():
    """k = 1: under exact draws from pi_{beta0}, the increment estimates
    log Z_{beta1} - log Z_{beta0} (closed form), within Monte Carlo error."""
    y = make_mixture_data(100, np.array([1.5]), 0.55, seed=21)
    m = Model.equal_weights(1, 1, 0.55)
    b0, b1 = 0.2, 0.25
    mean, var = evidence.posterior_k1(y, 0.55, b0)
    rng = np.random.default_rng(0)
    th = rng.normal(mean, math.sqrt(var), size=(1, 1 << 16))
    l = gmm.loglik(th, y, m)
    _, W, inc, _ = smc.reweight(np.zeros(th.shape[1]), l, b1 - b0)
    want = evidence.log_z_tempered_k1(y, 0.55, b1) - evidence.log_z_tempered_k1(y, 0.55, b0)
    # delta-method standard error of the log of a sample mean
    r = np.exp((b1 - b0) * l - np.max((b1 - b0) * l))
    se = np.std(r) / (np.mean(r) * math.sqrt(r.size))
    assert abs(inc - want) < 5 * se + 1e-9


def test_normalise_rejects_degenerate_input():
    with pytest.raises(FloatingPointError):
        smc.normalise(np.full(4, -np.inf))
    with pytest.raises(FloatingPointError):
        smc.normalise(np.array([0.0, np.nan]))


# --------------------------------------------------------------- resampling

def test_correctly_rounded_prefix_matches_fsum():
    import math as _m
    W = smc.normalise(lognormal_logw(300, seed=8, spread=6.0))
    C = smc.prefix_sums_correctly_rounded(W)
    for j in range(W.size):
        assert C[j] == _m.fsum(W[: j + 1])


def _check_systematic_invariants(W, idx):
    N = W.size
    assert idx.dtype == np.int32 and idx.size == N
    assert np.all(np.diff(idx) >= 0)
    counts = np.bincount(idx, minlength=N)
    assert counts.sum() == N
    NW = N * W
    lo = np.floor(NW - 1e-9)
    hi = np.ceil(NW + 1e-9)
    assert np.all(counts >= lo) and np.all(counts <= hi)
    assert np.all(counts[W == 0.0] == 0)


def test_systematic_counts_floor_ceil():
    for N, seed in ((1000, 1), (4096, 2), (65536, 3)):
        W = smc.normalise(lognormal_logw(N, seed=seed))
        for u in (0.0, 0.3, 0.999999):
            _check_systematic_invariants(W, smc.systematic_resample(W, u))


def test_systematic_uniform_power_of_two_is_identity():
    for N in (1, 2, 1024, 1 << 17):
        idx = smc.systematic_resample(np.full(N, 1.0 / N), 0.5)
        assert np.array_equal(idx, np.arange(N, dtype=np.int32))


def test_systematic_one_hot_is_constant():
    W = np.zeros(777)
    W[300] = 1.0
    for u in (0.0, 0.5, 1.0 - 2 ** -32):
        assert np.all(smc.systematic_resample(W, u) == 300)


def test_systematic_bruteforce_small_n():
    rng = np.random.default_rng(17)
    for trial in range(400):
        N = int(rng.integers(1, 9))
        raw = rng.exponential(size=N) * (rng.random(N) < 0.8)
        if raw.sum() == 0:
            raw[0] = 1.0
        W = raw / raw.sum()
        u = float(rng.integers(0, 2 ** 32)) * 2.0 ** -32
        assert np.array_equal(smc.systematic_resample(W, u),
                              smc.systematic_resample_bruteforce(W, u)), (W, u)


def _rounding_ties(W, u):
    """Positions i whose U_i lies between an exact prefix sum and its correctly
    rounded FP64 value (inclusive). The sampler compares U with the rounded
    prefixes, so only there may it differ from the exact-rational brute force."""
    N = len(W)
    exact, acc = [], Fraction(0)
    for w in W:
        acc += Fraction(float(w))
        exact.append(acc)
    bands = [(min(c, Fraction(float(c))), max(c, Fraction(float(c)))) for c in exact]
    out = set()
    for i in range(N):
        Ui = (i + Fraction(float(u))) / N
        if any(lo <= Ui <= hi for lo, hi in bands):
            out.add(i)
    return out


@settings(max_examples=60, deadline=None)
@given(st.lists(st.one_of(st.just(0.0), st.floats(1e-300, 1e3)), min_size=1, max_size=64),
       st.integers(0, 2 ** 32 - 1))
@example([0.0, 1.0, 1e-300, 1.0], 0)      # U_2 = 0.5 equals C_1 exactly; C_2 rounds to 0.5
def test_systematic_property(raw, r):
    raw = np.asarray(raw)
    if raw.sum() == 0.0:
        raw[0] = 1.0
    W = raw / raw.sum()
    u = r * 2.0 ** -32
    idx = smc.systematic_resample(W, u)
    _check_systematic_invariants(W, idx)
    brute = smc.systematic_resample_bruteforce(W, u)
    ties = _rounding_ties(W, u)
    for i in range(len(W)):
        if i not in ties:
            assert idx[i] == brute[i], (i, W, u)
