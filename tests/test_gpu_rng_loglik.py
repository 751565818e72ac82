"""GPU parity: Philox words, Box-Muller normals, prior draws and the mixture
log-likelihood against the FP64 oracle."""

import math

import numpy as np
import pytest
import torch

from gpu_common import announce, oracle_model, rel_err
from oracle import gmm as ogmm
from oracle import philox as opx
from oracle import smc as osmc
from workloads import (CONFIGS, make_data, make_mixture_data, theta_near_posterior,
                       theta_prior_draws)
from workloads.data import true_means_for

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-6       # per-particle relative error bound for the FP32 likelihood
FP64_TOL = 1e-12


@pytest.fixture(scope="module")
def smc():
    import paper_0905_2441_amd as smc
    return smc


@pytest.fixture(scope="module")
def ctx(smc):
    return smc.Context(0)


def test_philox_words_bit_identical(smc):
    for (seed, count, block, step, purpose, move) in ((0, 1, 0, 0, 1, 0),
                                                      (123456789012345, 1 << 20, 3, 77, 2, 5),
                                                      (2 ** 64 - 1, 4097, 0, 2 ** 32 - 1, 4, 0)):
        announce(f"philox seed={seed} count={count}")
        got = smc.smc_rng_words(seed, count, block, step, purpose, move)
        torch.cuda.synchronize()
        g = got.cpu().numpy().view(np.uint32).astype(np.uint64)
        w = opx.words(seed, np.arange(count, dtype=np.uint64), block, step, purpose, move)
        ref = np.stack(w, axis=1)
        assert np.array_equal(g, ref)


def test_box_muller_normals_match(smc):
    announce("normals")
    count, per = 1 << 16, 7
    got = smc.smc_rng_normals(42, count, per, 9, "prop", 3).cpu().numpy()
    ref = opx.normals(42, np.arange(count, dtype=np.uint64), 9, opx.PROP, 3, per)
    assert np.max(np.abs(got - ref)) < 1e-13


@pytest.mark.parametrize("prior", ["gauss", "box"])
def test_prior_init_matches(smc, ctx, prior):
    announce(f"prior {prior}")
    g = smc.Gmm.equal_weights(4, 1, 0.55, prior=prior,
                              prior_a=0.0 if prior == "gauss" else -10.0, prior_b=10.0)
    th = smc.smc_prior_init(ctx, g, 3000, 77).cpu().numpy()
    ref = osmc.prior_init(oracle_model(g), 3000, 77)
    assert np.max(np.abs(th - ref)) < 1e-12


def _check_loglik(smc, ctx, g, y, theta, prec, tol):
    got = smc.smc_loglik(ctx, g, torch.as_tensor(y).cuda(), torch.as_tensor(theta).cuda(), prec)
    ctx.check()
    ref = ogmm.loglik(theta, y, oracle_model(g))
    err = rel_err(got.cpu().numpy(), ref)
    assert err.max() <= tol, (prec, float(err.max()))
    return err


@pytest.mark.parametrize("prec,tol", [("fp32", FP32_TOL), ("fp64", FP64_TOL)])
@pytest.mark.parametrize("n,N", [(100, 1024), (1000, 777), (37, 65), (1, 3), (5000, 200)])
def test_loglik_1d_parity(smc, ctx, prec, tol, n, N):
    announce(f"loglik 1d {prec} n={n} N={N}")
    mu = np.array([-3.0, 0.0, 3.0, 6.0])
    y = make_mixture_data(n, mu, 0.55, seed=n)
    g = smc.Gmm.equal_weights(4, 1, 0.55)
    th = np.hstack([theta_prior_draws(N // 2, 4, 1, seed=N),
                    theta_near_posterior(N - N // 2, mu, seed=N + 1)])
    _check_loglik(smc, ctx, g, y, th, prec, tol)


@pytest.mark.parametrize("k", [1, 2, 3, 5, 6, 7, 8])
@pytest.mark.parametrize("prec,tol", [("fp32", FP32_TOL), ("fp64", FP64_TOL)])
def test_loglik_1d_every_k(smc, ctx, k, prec, tol):
    announce(f"loglik k={k} {prec}")
    rng = np.random.default_rng(k)
    mu = np.sort(rng.uniform(-8, 8, size=k))
    w = rng.dirichlet(np.ones(k))
    y = make_mixture_data(333, mu, 0.4, seed=k, weights=w)
    g = smc.Gmm(k=k, d=1, sigma2=0.4, log_w=tuple(np.log(w)))
    th = np.hstack([theta_prior_draws(100, k, 1, seed=k), theta_near_posterior(91, mu, seed=k)])
    _check_loglik(smc, ctx, g, y, th, prec, tol)


@pytest.mark.parametrize("k", [1, 2, 4, 8])
@pytest.mark.parametrize("prec,tol", [("fp32", FP32_TOL), ("fp64", FP64_TOL)])
def test_loglik_ddim_parity(smc, ctx, k, prec, tol):
    announce(f"loglik d=8 k={k} {prec}")
    rng = np.random.default_rng(10 + k)
    mu = 3.0 * rng.standard_normal((k, 8))
    y = make_mixture_data(700, mu, 1.0, seed=k)
    g = smc.Gmm.equal_weights(k, 8, 1.0)
    th = np.hstack([theta_prior_draws(70, k, 8, seed=k), theta_near_posterior(60, mu, seed=k)])
    _check_loglik(smc, ctx, g, y, th, prec, tol)


@pytest.mark.parametrize("k", [1, 2, 4, 8])
@pytest.mark.parametrize("n,N", [(700, 130), (7, 5), (1000, 1)])
def test_loglik_ddim_mfma_parity(smc, ctx, k, n, N):
    """The split-BF16 MFMA form of the d = 8 likelihood is within the FP32 bound."""
    announce(f"loglik mfma d=8 k={k} n={n} N={N}")
    rng = np.random.default_rng(20 + k)
    mu = 3.0 * rng.standard_normal((k, 8))
    y = make_mixture_data(n, mu, 1.0, seed=k + n)
    g = smc.Gmm.equal_weights(k, 8, 1.0)
    th = np.hstack([theta_prior_draws(N - N // 2, k, 8, seed=k), theta_near_posterior(N // 2, mu, seed=k)])
    _check_loglik(smc, ctx, g, y, th, "bf16x3", FP32_TOL)


def test_loglik_ddim_mfma_headline_size_sampled(smc, ctx):
    """d = 8, k = 8 at the full workload size (n = 65536, N = 16384), sampled particles."""
    cfg = CONFIGS["gmm8d_k8_n65536_N16384"]
    announce("loglik mfma headline size")
    y = make_data(cfg)
    mu = true_means_for(cfg)
    N = cfg.N
    th = np.hstack([theta_prior_draws(N // 2, 8, 8, seed=5), theta_near_posterior(N // 2, mu, seed=6)])
    g = smc.Gmm.equal_weights(8, 8, cfg.sigma2)
    got = smc.smc_loglik(ctx, g, torch.as_tensor(y).cuda(), torch.as_tensor(th).cuda(), "bf16x3")
    got = got.cpu().numpy()
    sample = np.unique(np.concatenate([np.arange(0, N, 1021), [N - 1, N // 2, N // 2 + 1]]))
    ref = ogmm.loglik(th[:, sample], y, oracle_model(g), chunk_elems=1 << 24)
    assert rel_err(got[sample], ref).max() <= FP32_TOL
    assert np.all(np.isfinite(got))


@pytest.mark.parametrize("slices", [1, 2, 5, 16])
def test_loglik_slice_counts(smc, ctx, slices):
    """Every split of the data over waves gives the oracle's value."""
    announce(f"loglik slices={slices}")
    mu = np.array([-3.0, 0.0, 3.0, 6.0])
    y = make_mixture_data(999, mu, 0.55, seed=3)
    g = smc.Gmm.equal_weights(4, 1, 0.55)
    th = theta_near_posterior(300, mu, seed=4)
    ctx.set_slices(slices)
    try:
        _check_loglik(smc, ctx, g, y, th, "fp32", FP32_TOL)
        _check_loglik(smc, ctx, g, y, th, "fp64", FP64_TOL)
    finally:
        ctx.set_slices(0)


def test_loglik_headline_size_sampled(smc, ctx):
    """At the headline size (n = 1000, N = 131072) compare a sample of particles."""
    cfg = CONFIGS["gmm1d_k4_n1000_N131072"]
    announce("loglik headline size")
    y = make_data(cfg)
    mu = true_means_for(cfg)
    N = cfg.N
    th = np.hstack([theta_prior_draws(N // 2, 4, 1, seed=5), theta_near_posterior(N // 2, mu, seed=6)])
    g = smc.Gmm.equal_weights(4, 1, cfg.sigma2)
    yt = torch.as_tensor(y).cuda()
    tt = torch.as_tensor(th).cuda()
    sample = np.unique(np.concatenate([np.arange(0, N, 509), [N - 1]]))
    for prec, tol in (("fp32", FP32_TOL), ("fp64", FP64_TOL)):
        got = smc.smc_loglik(ctx, g, yt, tt, prec).cpu().numpy()
        ref = ogmm.loglik(th[:, sample], y, oracle_model(g))
        assert rel_err(got[sample], ref).max() <= tol
        assert np.all(np.isfinite(got))


def test_loglik_long_data_fp32(smc, ctx):
    """n = 10^5 observations (the longest data of the batched workload)."""
    announce("loglik n=1e5")
    mu = np.array([-3.0, 0.0, 3.0, 6.0])
    y = make_mixture_data(100000, mu, 0.55, seed=8)
    g = smc.Gmm.equal_weights(4, 1, 0.55)
    th = np.hstack([theta_prior_draws(64, 4, 1, seed=8), theta_near_posterior(64, mu, seed=9)])
    _check_loglik(smc, ctx, g, y, th, "fp32", FP32_TOL)


@pytest.mark.parametrize("case", ["unnormalised_weights", "interleaved", "outlier_block",
                                  "far_tile", "d8_outlier_block"])
def test_loglik_fp32_direct_and_shifted_forms(smc, ctx, case):
    """The FP32 likelihood takes a direct form (no per-datum max shift) for
    waves near the data and the shifted form otherwise, switching mid-slice
    at a block of data far from every component; every mix agrees with the
    oracle: weights of total mass 4 (shifted only), near and far particles
    interleaved lane by lane, near particles whose data hold a block of
    outliers at +40, one far tile among near ones, and the same outliers in
    d = 8 (VALU and MFMA forms)."""
    announce(f"loglik fp32 forms {case}")
    mu = np.array([-3.0, 0.0, 3.0, 6.0])
    n, N = 1000, 640
    y = make_mixture_data(n, mu, 0.55, seed=31)
    near = theta_near_posterior(N, mu, seed=32)
    far = theta_prior_draws(N, 4, 1, seed=33)
    g = smc.Gmm.equal_weights(4, 1, 0.55)
    th = near
    if case == "unnormalised_weights":
        g = smc.Gmm(k=4, d=1, sigma2=0.55, log_w=(0.0, 0.0, 0.0, 0.0))
        th = np.hstack([near[:, : N // 2], far[:, N // 2:]])
    elif case == "interleaved":
        th = np.where(np.arange(N) % 7 == 3, far, near)
    elif case == "outlier_block":
        y = y.copy()
        y[480:520] = 40.0 + np.arange(40, dtype=np.float32) * 0.01
    elif case == "far_tile":
        th = near.copy()
        th[:, 128:192] = far[:, 128:192]
    elif case == "d8_outlier_block":
        rng = np.random.default_rng(34)
        mu8 = 3.0 * rng.standard_normal((4, 8))
        y = make_mixture_data(600, mu8, 1.0, seed=35)
        y[300:340] += 40.0
        g = smc.Gmm.equal_weights(4, 8, 1.0)
        th = theta_near_posterior(200, mu8, seed=36)
    precs = ("fp32", "bf16x3") if case.startswith("d8") else ("fp32",)
    for slices in (0, 3):
        ctx.set_slices(slices)
        try:
            for prec in precs:
                _check_loglik(smc, ctx, g, y, th, prec, FP32_TOL)
        finally:
            ctx.set_slices(0)


@pytest.mark.parametrize("case", ["sorted_near", "sorted_far", "sorted_mixed", "sorted_k1",
                                  "sorted_k2", "sorted_k3", "sorted_k8", "unsorted",
                                  "sorted_outliers", "wide_clusters", "zero_weights",
                                  "slice_63", "slice_65", "slice_127", "slice_128", "slice_129",
                                  "slice_191", "slice_192", "slice_193", "slice_200", "slice_256",
                                  "slice_255", "slice_257", "slice_320", "slice_384",
                                  "slice_512", "slice_520", "pairs_then_single",
                                  "clusters_at_crossings"])
def test_loglik_fp32_pivot_form(smc, ctx, case):
    """The FP32 pivot form (1-D data, windows of 64 data, each particle's
    largest component at the window's midpoint as its pivot) at 4 slices:
    on ascending data near and far particles and every k take it (k = 1
    leaves only the pivot's own terms); unordered data, windows that span
    far-apart clusters or hold a jump to outliers at +40 are refused for some
    or all particles and go through the plain forms; components of zero
    weight never become pivots; slices of 63 to 520 data sit on either side
    of the shortest slice the form takes (128), of a window's length (64) and
    of a pair of windows (two windows share one choice of pivots while no
    particle's bound over both passes the limit; a wide second window ends the
    pairs for the rest of the slice), with partial last windows and pairs;
    tight clusters of data straddle the points where two components'
    densities cross. Every case agrees with the oracle."""
    announce(f"loglik fp32 pivot {case}")
    mu = np.array([-3.0, 0.0, 3.0, 6.0])
    g = smc.Gmm.equal_weights(4, 1, 0.55)
    n = 1000
    y = make_mixture_data(n, mu, 0.55, seed=43)
    th = theta_near_posterior(500, mu, seed=42)
    if case == "sorted_far":
        th = theta_prior_draws(500, 4, 1, seed=45)
    elif case == "sorted_mixed":
        far = theta_prior_draws(500, 4, 1, seed=45)
        th = np.where(np.arange(500) % 5 == 2, far, th)
    elif case.startswith("sorted_k"):
        k = int(case[len("sorted_k"):])
        mu = np.linspace(-4.0, 7.0, k) if k > 1 else np.array([1.5])
        g = smc.Gmm.equal_weights(k, 1, 0.55)
        y = make_mixture_data(n, mu, 0.55, seed=46 + k)
        th = np.hstack([theta_near_posterior(300, mu, seed=47), theta_prior_draws(200, k, 1, 48)])
    elif case == "sorted_outliers":
        y = y.copy()
        y[-40:] = 40.0 + np.arange(40, dtype=np.float32) * 0.01
    elif case == "wide_clusters":
        mu = np.array([-30.0, -10.0, 10.0, 30.0])
        y = make_mixture_data(n, mu, 0.55, seed=49)
        th = np.hstack([theta_near_posterior(300, mu, seed=50), theta_prior_draws(200, 4, 1, 51)])
    elif case == "zero_weights":
        g = smc.Gmm(k=4, d=1, sigma2=0.55,
                    log_w=(math.log(0.5), float("-inf"), math.log(0.5), float("-inf")))
        y = make_mixture_data(n, np.array([-3.0, 3.0]), 0.55, seed=52)
    elif case.startswith("slice_"):
        per = int(case.split("_")[1])
        y = make_mixture_data(4 * per, mu, 0.55, seed=per)
    elif case == "pairs_then_single":
        # 4 slices of 250 sorted data; the fourth slice's last 40 data jump to
        # +40, so its second pair is refused and its windows go one at a time
        y = np.sort(make_mixture_data(n, mu, 0.55, seed=53))
        y[-40:] = 40.0 + np.arange(40, dtype=np.float32) * 0.01
    elif case == "clusters_at_crossings":
        # 4 slices of 256 sorted data, each two tight clusters of 128 data 5
        # apart; in the first two slices the clusters straddle the point where
        # two components' densities cross (-1.5, 4.5), and each pair of
        # windows holds one cluster
        rng = np.random.default_rng(54)
        y = np.concatenate([c + 0.3 * rng.random(128)
                            for c in (-4.0, 1.0, 2.0, 7.0, 8.0, 13.0, 14.0, 19.0)])
        y = y.astype(np.float32)
    if case != "unsorted":
        y = np.sort(y)
    ctx.set_slices(4)
    try:
        _check_loglik(smc, ctx, g, y, th, "fp32", FP32_TOL)
    finally:
        ctx.set_slices(0)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_loglik_nan_raises_status(smc, ctx, prec):
    announce(f"loglik NaN status {prec}")
    g = smc.Gmm.equal_weights(4, 1, 0.55)
    y = torch.tensor([0.0, float("nan"), 1.0] + [0.5] * 30, dtype=torch.float32).cuda()
    th = torch.zeros((4, 64), dtype=torch.float64).cuda()
    smc.smc_loglik(ctx, g, y, th, prec)
    with pytest.raises(smc.SmcError):
        ctx.check()
    ctx.check()  # cleared


def test_argument_errors(smc, ctx):
    g = smc.Gmm.equal_weights(4, 1, 0.55)
    y = torch.zeros(10, dtype=torch.float32).cuda()
    th = torch.zeros((3, 8), dtype=torch.float64).cuda()
    with pytest.raises(ValueError):
        smc.smc_loglik(ctx, g, y, th, "fp32")
    bad = smc.Gmm(k=9, d=1, sigma2=1.0, log_w=tuple([0.0] * 9))
    with pytest.raises(Exception):
        smc.smc_loglik(ctx, bad, y, torch.zeros((9, 8), dtype=torch.float64).cuda(), "fp32")
    g3 = smc.Gmm.equal_weights(3, 8, 1.0)   # (k=3, d=8) is not compiled
    with pytest.raises(smc.SmcError):
        smc.smc_loglik(ctx, g3, torch.zeros((10, 8), dtype=torch.float32).cuda(),
                       torch.zeros((24, 8), dtype=torch.float64).cuda(), "fp32")
