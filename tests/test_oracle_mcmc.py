"""Pins for the oracle's random-walk MH move and exchange move."""

import itertools
import math

import numpy as np

from oracle import evidence, gmm, smc
from oracle.gmm import Model
from workloads import make_mixture_data, pt_betas


def test_rwmh_leaves_k1_tempered_posterior_invariant():
    """Start from exact draws of p0 L^beta (Gaussian for k = 1); after RW-MH
    moves the mean and variance still match the closed form."""
    y = make_mixture_data(50, np.array([2.0]), 0.55, seed=3)
    m = Model.equal_weights(1, 1, 0.55)
    beta = 0.3
    mean, var = evidence.posterior_k1(y, 0.55, beta)
    rng = np.random.default_rng(5)
    N = 1 << 15
    th = rng.normal(mean, math.sqrt(var), size=(1, N))
    l = gmm.loglik(th, y, m)
    acc = 0
    for mv in range(4):
        th, l, a = smc.rwmh_move(th, l, y, m, beta, 0.5, seed=77, step=1, move=mv)
        acc += a.sum()
    assert 0.05 < acc / (4 * N) < 0.95
    se_mean = math.sqrt(var / N)
    assert abs(th.mean() - mean) < 5 * se_mean * 3        # moves correlate draws mildly
    assert abs(th.var() / var - 1.0) < 5 * math.sqrt(2.0 / N) * 3


def test_rwmh_drifts_away_from_wrong_distribution():
    """Counter-check: started off-target, the sampler moves toward the posterior
    (a sign error in log alpha would push it away)."""
    y = make_mixture_data(50, np.array([2.0]), 0.55, seed=3)
    m = Model.equal_weights(1, 1, 0.55)
    mean, var = evidence.posterior_k1(y, 0.55, 1.0)
    th = np.full((1, 4096), mean + 2.0)
    l = gmm.loglik(th, y, m)
    for mv in range(150):
        th, l, _ = smc.rwmh_move(th, l, y, m, 1.0, 0.15, seed=1, step=2, move=mv)
    assert abs(th.mean() - mean) < 0.1


def test_exchange_log_alpha_properties():
    assert smc.exchange_log_alpha(0.3, 0.3, -5.0, -100.0) == 0.0
    for ba, bb, la, lb in ((0.1, 0.4, -10.0, -3.0), (0.9, 0.2, -1e4, -5e3)):
        # the reverse move (states already swapped) has the reciprocal ratio
        assert smc.exchange_log_alpha(ba, bb, la, lb) + smc.exchange_log_alpha(ba, bb, lb, la) == 0.0
        # relabelling the pair does not change the ratio
        assert smc.exchange_log_alpha(ba, bb, la, lb) == smc.exchange_log_alpha(bb, ba, lb, la)


def test_exchange_detailed_balance_discrete_target():
    """Two chains on a 3-state space with targets pi_b(x) ~ exp(b * E(x)): the
    exchange kernel built from exchange_log_alpha leaves the product target
    invariant (its transition matrix has it as a stationary vector)."""
    E = np.array([-1.0, -4.0, -0.2])
    ba, bb = 0.25, 1.0
    pa = np.exp(ba * E) / np.exp(ba * E).sum()
    pb = np.exp(bb * E) / np.exp(bb * E).sum()
    states = list(itertools.product(range(3), range(3)))
    P = np.zeros((9, 9))
    for s, (xa, xb) in enumerate(states):
        la = smc.exchange_log_alpha(ba, bb, E[xa], E[xb])
        acc = min(1.0, math.exp(la))
        t = states.index((xb, xa))
        P[s, t] += acc
        P[s, s] += 1.0 - acc
    pi = np.array([pa[xa] * pb[xb] for xa, xb in states])
    np.testing.assert_allclose(pi @ P, pi, atol=1e-15)


def test_exchange_pairs_partitions():
    assert smc.exchange_pairs(6, 0, False) == [(0, 1), (2, 3), (4, 5)]
    assert smc.exchange_pairs(6, 1, False) == [(1, 2), (3, 4)]
    assert smc.exchange_pairs(6, 1, True) == [(1, 2), (3, 4), (5, 0)]
    assert smc.exchange_pairs(7, 0, False) == [(0, 1), (2, 3), (4, 5)]
    # pairs are disjoint
    for M in (2, 5, 8, 9):
        for par in (0, 1):
            flat = [i for p in smc.exchange_pairs(M, par, True) for i in p]
            assert len(flat) == len(set(flat))


def test_pt_exchange_equal_betas_always_swap():
    M = 8
    th = np.arange(4 * M, dtype=np.float64).reshape(4, M)
    l = -np.arange(M, dtype=np.float64)
    th2, l2, n = smc.pt_exchange(th, l, np.full(M, 0.5), 0, False, seed=3, it=0)
    assert n == M // 2
    assert np.array_equal(l2, l.reshape(-1, 2)[:, ::-1].reshape(-1))
    assert np.array_equal(th2[:, 0], th[:, 1])


def test_pt_run_small_moves_hot_chain_between_modes():
    """A short population-MCMC run on a 2-component posterior: the beta = 1 chain
    ends near a mode (log-likelihood close to the best one)."""
    mu = np.array([-2.0, 2.0])
    y = make_mixture_data(40, mu, 0.55, seed=9)
    m = Model.equal_weights(2, 1, 0.55)
    betas = pt_betas(16, power=2)
    out = smc.pt_run(y, m, betas, 200, 0.5, seed=5)
    lbest = gmm.loglik(mu[:, None], y, m)[0]
    assert out["l"][-1] > lbest - 15.0
    assert out["swaps"] > 0


# ---------------------------------------------------------------------------
# The prior term of the Metropolis ratio. Under a strong prior, or at beta = 0
# where the prior is the whole target, a move that drops log p0(theta') -
# log p0(theta) or flips its sign leaves the target at once; these checks start
# from exact draws of the target (particles are independent chains, so after the
# moves they are still independent exact draws and the standard errors are the
# plain ones) and fail for either mistake (shown below by planting each one).

def _moments_off(th, mean, var, z=5.0):
    """Reasons the particle cloud's mean or variance is more than z standard
    errors from (mean, var); empty if both agree."""
    N = th.size
    out = []
    if abs(th.mean() - mean) > z * math.sqrt(var / N):
        out.append(f"mean {th.mean():.5f} vs {mean:.5f}")
    if abs(th.var() / var - 1.0) > z * math.sqrt(2.0 / N):
        out.append(f"variance {th.var():.5f} vs {var:.5f}")
    return out


def _check_strong_gauss_prior():
    """k = 1, prior N(1, 0.2^2), beta = 0.01, n = 50: the prior precision (25)
    is about 27 times the tempered likelihood's (0.91). Start from exact draws
    of p0 L^beta (closed form); after 12 moves the draws keep its moments."""
    y = make_mixture_data(50, np.array([2.0]), 0.55, seed=3)
    m = Model.equal_weights(1, 1, 0.55, prior="gauss", prior_a=1.0, prior_b=0.2)
    beta = 0.01
    mean, var = evidence.posterior_k1(y, 0.55, beta, prior_a=1.0, prior_b=0.2)
    rng = np.random.default_rng(11)
    N = 1 << 14
    th = rng.normal(mean, math.sqrt(var), size=(1, N))
    l = gmm.loglik(th, y, m)
    acc = 0
    for mv in range(12):
        th, l, a = smc.rwmh_move(th, l, y, m, beta, 0.3, seed=21, step=4, move=mv)
        acc += int(a.sum())
    out = _moments_off(th[0], mean, var)
    if not 0.2 < acc / (12 * N) < 0.8:
        out.append(f"acceptance {acc / (12 * N):.3f}")
    return out


def _check_beta0_gauss_prior():
    """beta = 0: the target is the prior N(3, 2^2) on each of the k = 4 means.
    Prior draws moved 20 times keep mean 3 and variance 4 in every coordinate."""
    y = make_mixture_data(50, np.array([-3.0, 0.0, 3.0, 6.0]), 0.55, seed=4)
    m = Model.equal_weights(4, 1, 0.55, prior="gauss", prior_a=3.0, prior_b=2.0)
    N = 1 << 14
    th = smc.prior_init(m, N, seed=31)
    l = gmm.loglik(th, y, m)
    for mv in range(20):
        th, l, _ = smc.rwmh_move(th, l, y, m, 0.0, 1.0, seed=32, step=1, move=mv)
    out = []
    for c in range(4):
        out += [f"coordinate {c}: {r}" for r in _moments_off(th[c], 3.0, 4.0)]
    return out


def _check_beta0_box_prior():
    """beta = 0 under the paper's box prior U[-10, 10]^4: uniform draws moved 20
    times with sd 3 never leave the box and keep the uniform's moments."""
    y = make_mixture_data(50, np.array([-3.0, 0.0, 3.0, 6.0]), 0.3025, seed=5)
    m = Model.equal_weights(4, 1, 0.3025, prior="box", prior_a=-10.0, prior_b=10.0)
    N = 1 << 14
    th = smc.prior_init(m, N, seed=41)
    l = gmm.loglik(th, y, m)
    for mv in range(20):
        th, l, _ = smc.rwmh_move(th, l, y, m, 0.0, 3.0, seed=42, step=1, move=mv)
    out = []
    if np.any(np.abs(th) > 10.0):
        out.append(f"{int(np.sum(np.any(np.abs(th) > 10.0, axis=0)))} particles left the box")
    for c in range(4):
        out += [f"coordinate {c}: {r}" for r in _moments_off(th[c], 0.0, 400.0 / 12.0)]
    return out


_PRIOR_CHECKS = (_check_strong_gauss_prior, _check_beta0_gauss_prior, _check_beta0_box_prior)


def test_rwmh_prior_term_strong_prior_and_beta0():
    for check in _PRIOR_CHECKS:
        assert check() == [], check.__name__


def test_rwmh_prior_term_checks_catch_planted_mistakes(monkeypatch):
    """Each planted mistake in the oracle's prior term (dropped, or with its sign
    flipped) makes every one of the three checks above fail."""
    planted = {
        "dropped": lambda beta, l_cur, l_prop, lp_cur, lp_prop: beta * (l_prop - l_cur),
        "sign flipped": lambda beta, l_cur, l_prop, lp_cur, lp_prop:
            beta * (l_prop - l_cur) - (lp_prop - lp_cur),
    }
    for name, wrong in planted.items():
        with monkeypatch.context() as mp, np.errstate(invalid="ignore"):
            # (outside the box both priors are -inf: the flipped term is NaN there)
            mp.setattr(smc, "rwmh_log_alpha", wrong)
            for check in _PRIOR_CHECKS:
                assert check() != [], (name, check.__name__)


def test_sampled_step_equals_whole_step_columns():
    """The oracle's step with moves on a sample of positions gives exactly the
    sampled columns of the whole step (with and without resampling)."""
    y = make_mixture_data(60, np.array([-3.0, 0.0, 3.0, 6.0]), 0.55, seed=8)
    m = Model.equal_weights(4, 1, 0.55)
    N = 700
    th = smc.prior_init(m, N, seed=9)
    l = gmm.loglik(th, y, m)
    betas = np.array([0.0, 0.002, 0.01, 0.05])
    sample = np.array([0, 5, 77, 300, 699, 5])
    lw = np.zeros(N)
    fired = []
    for t in (1, 2, 3):
        a = smc.smc_step(th, l, lw, y, m, betas, t, 0.5, 2, 12)
        fired.append(a[5]["resampled"])
        b = smc.smc_step_sampled(th, l, lw, y, m, betas, t, 0.5, 2, 12, sample)
        assert np.array_equal(a[0][:, sample], b[0]) and np.array_equal(a[1][sample], b[1])
        assert np.array_equal(a[2], b[2]) and a[4] == b[4]
        assert a[5]["resampled"] == b[5]["resampled"]
        for am, bm in zip(a[5]["accepted"], b[5]["accepted"]):
            assert np.array_equal(am[sample], bm)
        th, l, lw = a[0], a[1], a[2]
    assert any(fired) and not all(fired), fired


def test_pt_iteration_pairs_equal_whole_iteration_columns():
    """The oracle's population-MCMC iteration restricted to sampled pairs gives
    exactly those chains' columns of the whole iteration (move, then exchange),
    for both partitions and the wrap pair."""
    y = make_mixture_data(40, np.array([-3.0, 0.0, 3.0, 6.0]), 0.3025, seed=2)
    m = Model.equal_weights(4, 1, 0.3025, prior="box", prior_a=-10.0, prior_b=10.0)
    M = 64
    betas = pt_betas(M, 2)
    th = smc.prior_init(m, M, seed=5)
    l = gmm.loglik(th, y, m)
    for it, wrap in ((0, False), (1, False), (3, True)):
        parity = it & 1
        th1, l1, _ = smc.rwmh_move(th, l, y, m, betas, 1.0, 13, it, 0)
        th1, l1, nsw = smc.pt_exchange(th1, l1, betas, parity, wrap, 13, it)
        pairs = smc.exchange_pairs(M, parity, wrap)
        pick = [pairs[0], pairs[len(pairs) // 2], pairs[-1]]
        ths, ls, chains = smc.pt_iteration_pairs(th, l, y, m, betas, it, 1.0, 13, pick)
        assert np.array_equal(ths, th1[:, chains]) and np.array_equal(ls, l1[chains])
        assert nsw > 0
        th, l = th1, l1
