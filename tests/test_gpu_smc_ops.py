"""GPU parity: reweight / LSE / ESS, systematic resampling, RW-MH move and the
exchange move against the FP64 oracle on the same inputs."""

import math

import numpy as np
import pytest
import torch

from gpu_common import announce, oracle_model, rel_err
from oracle import gmm as ogmm
from oracle import philox as opx
from oracle import smc as osmc
from workloads import (CONFIGS, lognormal_logw, make_data, make_mixture_data, pt_betas,
                       theta_near_posterior, theta_prior_draws)
from workloads.data import true_means_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def smc():
    import paper_0905_2441_amd as smc
    return smc


@pytest.fixture(scope="module")
def ctx(smc):
    return smc.Context(0)


def _cuda(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype).cuda()


# ------------------------------------------------------------------ reweight / ESS

@pytest.mark.parametrize("N", [1, 5, 1000, 4097, 131072, 1 << 20])
def test_reweight_matches_oracle(smc, ctx, N):
    announce(f"reweight N={N}")
    logw0 = lognormal_logw(N, seed=N, spread=2.0)
    l = -500.0 + 30.0 * lognormal_logw(N, seed=N + 1)
    dbeta = 0.0123
    lw = _cuda(logw0)
    W = torch.empty(N, dtype=torch.float64).cuda()
    logZ = torch.full((1,), 1.5, dtype=torch.float64).cuda()
    ess = torch.zeros(1, dtype=torch.float64).cuda()
    smc.smc_reweight(ctx, lw, _cuda(l), dbeta, W=W, logZ=logZ, ess=ess)
    ctx.check()
    lw_ref, W_ref, inc_ref, ess_ref = osmc.reweight(logw0, l, dbeta)
    assert np.array_equal(lw.cpu().numpy(), lw_ref)                 # one mul + one add each
    assert np.max(np.abs(W.cpu().numpy() - W_ref)) <= 1e-14
    assert abs(logZ.item() - (1.5 + inc_ref)) <= 1e-12 * max(1.0, abs(inc_ref))
    assert abs(ess.item() - ess_ref) <= 1e-12 * ess_ref
    # standalone ESS of the oracle's weights
    e2 = torch.zeros(1, dtype=torch.float64).cuda()
    smc.smc_ess(ctx, _cuda(W_ref), e2)
    assert abs(e2.item() - osmc.ess(W_ref)) <= 1e-12 * ess_ref


def test_reweight_special_cases(smc, ctx):
    announce("reweight special")
    N = 1 << 12
    W = torch.empty(N, dtype=torch.float64).cuda()
    ess = torch.zeros(1, dtype=torch.float64).cuda()
    smc.smc_reweight(ctx, _cuda(np.zeros(N)), _cuda(np.full(N, -3.0)), 0.5, W=W, ess=ess)
    assert ess.item() == N
    assert np.all(W.cpu().numpy() == 1.0 / N)
    lw = np.full(N, -np.inf)
    lw[17] = 0.0
    smc.smc_reweight(ctx, _cuda(lw), _cuda(np.zeros(N)), 0.1, W=W, ess=ess)
    assert ess.item() == 1.0
    ctx.check()
    smc.smc_reweight(ctx, _cuda(np.full(N, -np.inf)), _cuda(np.zeros(N)), 0.1, W=W, ess=ess)
    with pytest.raises(smc.SmcError):
        ctx.check()


# ------------------------------------------------------------------ resampling

def _resample_gpu(smc, ctx, W, u, theta=None, l=None):
    N = W.size
    idx = torch.empty(N, dtype=torch.int32).cuda()
    kw = {}
    if theta is not None:
        kw.update(theta_in=_cuda(theta), theta_out=torch.empty(theta.shape, dtype=torch.float64).cuda(),
                  l_in=_cuda(l), l_out=torch.empty(N, dtype=torch.float64).cuda())
    smc.smc_resample_systematic(ctx, _cuda(W), seed=0, step=0,
                                u_override=_cuda(np.array([u])), idx=idx, **kw)
    return idx, kw


@pytest.mark.parametrize("N", [1, 2, 7, 1000, 2049, 131072, (1 << 20) - 1, 1 << 20,
                               (1 << 21) + 12345, (1 << 22) + 4321])
def test_resample_bit_exact(smc, ctx, N):
    announce(f"resample N={N}")
    W = osmc.normalise(lognormal_logw(N, seed=N + 5, spread=3.0))
    rng = np.random.default_rng(N)
    for trial in range(2):
        u = float(rng.integers(0, 2 ** 32)) * 2.0 ** -32
        idx, _ = _resample_gpu(smc, ctx, W, u)
        ref = osmc.systematic_resample(W, u)
        assert np.array_equal(idx.cpu().numpy(), ref)


def test_resample_degenerate_weights(smc, ctx):
    announce("resample degenerate")
    N = 5000
    for W in (np.full(N, 1.0 / N), np.eye(1, N, 4321).ravel(),
              np.where(np.arange(N) % 3 == 0, 1.0, 0.0) / (N // 3 + 1)):
        W = W / W.sum()
        for u in (0.0, 0.5, 1.0 - 2.0 ** -32):
            idx, _ = _resample_gpu(smc, ctx, W, u)
            assert np.array_equal(idx.cpu().numpy(), osmc.systematic_resample(W, u))


def test_resample_gather_and_predicate(smc, ctx):
    announce("resample gather")
    N, kd = 3000, 4
    W = osmc.normalise(lognormal_logw(N, seed=1))
    theta = np.random.default_rng(0).normal(size=(kd, N))
    l = np.random.default_rng(1).normal(size=N)
    idx, kw = _resample_gpu(smc, ctx, W, 0.25, theta, l)
    ref = osmc.systematic_resample(W, 0.25)
    assert np.array_equal(kw["theta_out"].cpu().numpy(), theta[:, ref])
    assert np.array_equal(kw["l_out"].cpu().numpy(), l[ref])
    # ESS predicate: not fired -> identity and copies
    idx2 = torch.empty(N, dtype=torch.int32).cuda()
    th_out = torch.empty((kd, N), dtype=torch.float64).cuda()
    ess = _cuda(np.array([osmc.ess(W)]))
    smc.smc_resample_systematic(ctx, _cuda(W), 3, 4, ess=ess, ess_threshold=1.0, idx=idx2,
                                theta_in=_cuda(theta), theta_out=th_out)
    assert np.array_equal(idx2.cpu().numpy(), np.arange(N))
    assert np.array_equal(th_out.cpu().numpy(), theta)
    # fired, with the offset drawn from the Philox stream of (seed, step)
    smc.smc_resample_systematic(ctx, _cuda(W), 3, 4, ess=ess, ess_threshold=float(N), idx=idx2)
    assert np.array_equal(idx2.cpu().numpy(), osmc.systematic_resample(W, osmc.resample_offset(3, 4)))


@pytest.mark.parametrize("N", [1, 7, 1000, 2049, 131072, 1 << 20, (1 << 21) + 12345,
                               (1 << 22) + 4321])
@pytest.mark.parametrize("scheme", ["stratified", "multinomial", "systematic"])
def test_resample_schemes_bit_exact(smc, ctx, scheme, N):
    """Every scheme's indices equal the oracle's bit for bit when the GPU is fed
    the oracle's weights; the points come from each side's own Philox. From
    N = 2^22 on a workgroup of the sorted schemes' search takes 2048 points."""
    announce(f"resample {scheme} N={N}")
    W = osmc.normalise(lognormal_logw(N, seed=N % 97))
    idx = torch.empty(N, dtype=torch.int32).cuda()
    for step in (1, 5):
        smc.smc_resample(ctx, _cuda(W), scheme, 21, step, idx=idx)
        assert np.array_equal(idx.cpu().numpy(), osmc.resample_indices(W, scheme, 21, step))


@pytest.mark.parametrize("scheme", ["systematic", "stratified"])
def test_resample_sorted_points_large_n_degenerate_gather_predicate(smc, ctx, scheme):
    """Past 2^20 particles (a ragged last chunk of the CDF): equal weights, one
    particle holding all the weight (first, inside, last), every third
    particle, zero weight on the last thousand, the gather with the logw
    reset, and an unfired predicate (identity and copies)."""
    N, kd = (1 << 20) + 77, 2
    announce(f"resample sorted large N {scheme}")
    cases = [np.full(N, 1.0 / N), np.eye(1, N, 0).ravel(), np.eye(1, N, 654321).ravel(),
             np.eye(1, N, N - 1).ravel(), np.where(np.arange(N) % 3 == 0, 1.0, 0.0),
             np.where(np.arange(N) < N - 1000, 1.0, 0.0),
             # sparse weight: every wave's points span thousands of particles
             np.where(np.arange(N) % 4099 == 17, 1.0, 0.0)]
    idx = torch.empty(N, dtype=torch.int32).cuda()
    for W in cases:
        W = W / W.sum()
        smc.smc_resample(ctx, _cuda(W), scheme, 6, 3, idx=idx)
        assert np.array_equal(idx.cpu().numpy(), osmc.resample_indices(W, scheme, 6, 3))
    W = osmc.normalise(lognormal_logw(N, seed=4, spread=3.0))
    rng = np.random.default_rng(2)
    theta = rng.normal(size=(kd, N))
    l = rng.normal(size=N)
    th_out = torch.empty((kd, N), dtype=torch.float64).cuda()
    l_out = torch.empty(N, dtype=torch.float64).cuda()
    logw = _cuda(np.ones(N))
    smc.smc_resample(ctx, _cuda(W), scheme, 8, 2, idx=idx, theta_in=_cuda(theta),
                     theta_out=th_out, l_in=_cuda(l), l_out=l_out, logw=logw)
    ref = osmc.resample_indices(W, scheme, 8, 2)
    assert np.array_equal(idx.cpu().numpy(), ref)
    assert np.array_equal(th_out.cpu().numpy(), theta[:, ref])
    assert np.array_equal(l_out.cpu().numpy(), l[ref])
    assert np.all(logw.cpu().numpy() == 0.0)
    if scheme == "systematic":
        ess = _cuda(np.array([osmc.ess(W)]))
        th2 = torch.empty((kd, N), dtype=torch.float64).cuda()
        smc.smc_resample_systematic(ctx, _cuda(W), 3, 4, ess=ess, ess_threshold=1.0, idx=idx,
                                    theta_in=_cuda(theta), theta_out=th2)
        assert np.array_equal(idx.cpu().numpy(), np.arange(N))
        assert np.array_equal(th2.cpu().numpy(), theta)
        for u in (0.0, 1.0 - 2.0 ** -32):
            ii, _ = _resample_gpu(smc, ctx, W, u)
            assert np.array_equal(ii.cpu().numpy(), osmc.systematic_resample(W, u))


@pytest.mark.parametrize("scheme", ["stratified", "multinomial"])
def test_resample_schemes_degenerate_and_gather(smc, ctx, scheme):
    announce(f"resample {scheme} degenerate + gather")
    N, kd = 5000, 4
    for W in (np.full(N, 1.0 / N), np.eye(1, N, 4321).ravel(),
              np.where(np.arange(N) % 3 == 0, 1.0, 0.0) / (N // 3 + 1)):
        W = W / W.sum()
        idx = torch.empty(N, dtype=torch.int32).cuda()
        smc.smc_resample(ctx, _cuda(W), scheme, 4, 9, idx=idx)
        assert np.array_equal(idx.cpu().numpy(), osmc.resample_indices(W, scheme, 4, 9))
    W = osmc.normalise(lognormal_logw(N, seed=3))
    theta = np.random.default_rng(0).normal(size=(kd, N))
    l = np.random.default_rng(1).normal(size=N)
    th_out = torch.empty((kd, N), dtype=torch.float64).cuda()
    l_out = torch.empty(N, dtype=torch.float64).cuda()
    logw = _cuda(np.ones(N))
    smc.smc_resample(ctx, _cuda(W), scheme, 8, 2, theta_in=_cuda(theta), theta_out=th_out,
                     l_in=_cuda(l), l_out=l_out, logw=logw)
    ref = osmc.resample_indices(W, scheme, 8, 2)
    assert np.array_equal(th_out.cpu().numpy(), theta[:, ref])
    assert np.array_equal(l_out.cpu().numpy(), l[ref])
    assert np.all(logw.cpu().numpy() == 0.0)
    th = _cuda(theta)
    with pytest.raises(smc.SmcError):                       # aliasing is refused
        smc.smc_resample(ctx, _cuda(W), "systematic", 8, 2, theta_in=th, theta_out=th)
    with pytest.raises(KeyError):
        smc.smc_resample(ctx, _cuda(W), "residual", 8, 2)


# ------------------------------------------------------------------ RW-MH move

@pytest.mark.parametrize("slices", [0, 40, 128])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_rwmh_move_matches_oracle(smc, ctx, prec, slices):
    """slices 40 and 128 spread each 64-particle tile over 3 and 8 workgroups
    (partials in scratch, decision in a second kernel)."""
    announce(f"rwmh {prec} slices={slices}")
    mu = np.array([-3.0, 0.0, 3.0, 6.0])
    y = make_mixture_data(200, mu, 0.55, seed=2)
    g = smc.Gmm.equal_weights(4, 1, 0.55)
    om = oracle_model(g)
    N = 4000
    th = np.hstack([theta_prior_draws(N // 2, 4, 1, seed=3), theta_near_posterior(N // 2, mu, seed=4)])
    l = ogmm.loglik(th, y, om)
    tt, lt = _cuda(th), _cuda(l)
    acc = torch.zeros(1, dtype=torch.int64).cuda()
    beta = 0.37
    ctx.set_slices(slices)
    try:
        smc.smc_rwmh_move(ctx, g, _cuda(y, torch.float32), tt, lt, beta, 0.5, seed=11, step=6,
                          move=2, prec=prec, n_accept=acc)
        ctx.check()
    finally:
        ctx.set_slices(0)
    th_ref, l_ref, a_ref = osmc.rwmh_move(th, l, y, om, beta, 0.5, 11, 6, 2)
    got_th, got_l = tt.cpu().numpy(), lt.cpu().numpy()
    a_got = np.any(got_th != th, axis=0)
    flips = int(np.sum(a_got != a_ref))
    if prec == "fp64":
        assert flips == 0
    else:
        assert flips <= 2          # FP32 log-likelihood error can flip a near-tie decision
    same = a_got == a_ref
    assert acc.item() == int(a_got.sum())
    assert np.max(np.abs(got_th[:, same] - th_ref[:, same])) <= 1e-13 * 30
    tol = 1e-12 if prec == "fp64" else 1e-6
    assert rel_err(got_l[same], l_ref[same]).max() <= tol


def test_rwmh_per_chain_beta_and_box_prior(smc, ctx):
    announce("rwmh beta_vec box")
    mu = np.array([-2.0, 2.0])
    y = make_mixture_data(80, mu, 0.3, seed=5)
    g = smc.Gmm.equal_weights(2, 1, 0.3, prior="box", prior_a=-10.0, prior_b=10.0)
    om = oracle_model(g)
    M = 512
    betas = pt_betas(M, 4)
    th = osmc.prior_init(om, M, 9)
    th[:, :5] = 9.95                           # proposals near the edge leave the box
    l = ogmm.loglik(th, y, om)
    tt, lt = _cuda(th), _cuda(l)
    smc.smc_rwmh_move(ctx, g, _cuda(y, torch.float32), tt, lt, 0.0, 1.0, seed=5, step=1,
                      prec="fp64", beta_vec=_cuda(betas))
    th_ref, l_ref, a_ref = osmc.rwmh_move(th, l, y, om, betas, 1.0, 5, 1, 0)
    assert np.max(np.abs(tt.cpu().numpy() - th_ref)) <= 1e-12
    assert rel_err(lt.cpu().numpy(), l_ref).max() <= 1e-12
    assert np.all(tt.cpu().numpy() <= 10.0) and np.all(tt.cpu().numpy() >= -10.0)


def test_fp32_shifted_form_counter(smc, ctx):
    """The device counter of the FP32 move's per-datum forms. On data in their
    generated (unordered) order the pivot form refuses every window: a move of
    prior draws (far from the data) then takes the plain shifted form for
    every full block of 8 observations of every wave's slice, and a move of
    particles near a posterior mode stays in the plain direct form. On the
    same data in ascending order the near particles take the pivot form
    throughout, with fewer than 2.5 of their three other components on
    average (the rest fall below 2^-25 over a window), and the prior draws
    take it in most windows. FP64 moves do not count. (Four slices whose boundaries fall on multiples of 8: 248, 248, 248
    and 256 observations, all in full blocks.)"""
    announce("fp32 form counter")
    mu = np.array([-3.0, 0.0, 3.0, 6.0])
    n, N = 1000, 4096
    y_np = make_mixture_data(n, mu, 0.55, seed=2)
    g = smc.Gmm.equal_weights(4, 1, 0.55)
    tiles = N // 64
    prior = theta_prior_draws(N, 4, 1, seed=3)
    near = theta_near_posterior(N, mu, seed=4, jitter=0.1)
    ctx.set_slices(4)
    try:
        for name, y_in, th_np, prec, want in (
                ("prior", y_np, prior, "fp32", lambda c: c == tiles * n),
                ("near", y_np, near, "fp32", lambda c: c == 0),
                ("prior fp64", y_np, prior, "fp64", lambda c: c == 0),
                ("prior sorted", np.sort(y_np), prior, "fp32", lambda c: 0 < c < tiles * n // 2),
                ("near sorted", np.sort(y_np), near, "fp32", lambda c: c == 0)):
            y = _cuda(y_in, torch.float32)
            th = _cuda(th_np)
            l = torch.empty(N, dtype=torch.float64, device="cuda")
            smc.smc_loglik(ctx, g, y, th, prec, out=l)
            ctx.fp32_form_counts(reset=True)
            smc.smc_rwmh_move(ctx, g, y, th, l, 0.5, 0.5, seed=5, step=1, prec=prec)
            ctx.check()
            fc = ctx.fp32_form_counts(reset=True)
            got = fc["shifted"]
            assert want(got), (name, fc)
            # every pair of a 1-D FP32 move is in the pivot form, the plain
            # shifted form or the plain direct form; the pivot form evaluates
            # at most k - 1 other components per pair
            assert fc["shifted"] + fc["pivot"] <= tiles * n, (name, fc)
            assert fc["pivot_terms"] <= 3 * fc["pivot"], (name, fc)
            if name == "near sorted":
                assert fc["pivot"] == tiles * n and fc["pivot_terms"] < 2.5 * fc["pivot"], fc
            if prec == "fp64" or name in ("prior", "near"):
                assert fc["pivot"] == 0 and fc["pivot_terms"] == 0, (name, fc)
    finally:
        ctx.set_slices(0)


def _order_keys(v):
    """Sign-magnitude order keys of FP32 values (the order smc_sort_data defines)."""
    b = np.ascontiguousarray(v, dtype=np.float32).view(np.int32).astype(np.int64)
    return np.where(b >= 0, b, b ^ 0x7FFFFFFF)


@pytest.mark.parametrize("n", [0, 1, 2, 3, 100, 4095, 4096, 4097, 10000, 65537, (1 << 20) + 3])
def test_sort_data_matches_key_order(smc, n):
    """smc_sort_data gives the bits of numpy's sort of the values' order keys,
    with NaNs of both signs, infinities, signed zeros and many ties, and leaves
    the array's neighbours untouched."""
    announce(f"sort n={n}")
    rng = np.random.default_rng(n + 17)
    v = rng.standard_normal(n).astype(np.float32)
    if n >= 10:
        v[rng.integers(0, n, n // 10)] = np.float32(1.5)                 # ties
        special = np.array([np.nan, -np.nan, np.inf, -np.inf, 0.0, -0.0], dtype=np.float32)
        v[rng.integers(0, n, 6)] = special
        v[n // 2] = np.frombuffer(np.uint32(0xFFC00001).tobytes(), dtype=np.float32)[0]
    buf = np.full(n + 8, 7.25, dtype=np.float32)
    buf[4:4 + n] = v
    t = _cuda(buf, torch.float32)
    smc.smc_sort_data(t[4:4 + n])
    torch.cuda.synchronize()
    got = t.cpu().numpy()
    want = np.sort(_order_keys(v), kind="stable")
    assert np.array_equal(_order_keys(got[4:4 + n]), want)
    assert np.all(got[:4] == 7.25) and np.all(got[4 + n:] == 7.25)


def test_sort_data_rejects_bad_sizes(smc):
    from paper_0905_2441_amd import _lib
    lib = _lib.load()
    assert lib.smc_sort_data(None, -1, None) == _lib.SMC_ERR_INVALID_ARG
    assert lib.smc_sort_data(None, 5, None) == _lib.SMC_ERR_INVALID_ARG
    assert lib.smc_sort_data(None, (1 << 30) + 1, None) == _lib.SMC_ERR_INVALID_ARG
    assert lib.smc_sort_data(None, 0, None) == _lib.SMC_OK


def test_samplers_hold_sorted_data(smc, ctx):
    """The 1-D samplers sort their own device copy of the data (each batched
    run's data apart); d > 1 data keep their order."""
    announce("samplers sort data")
    mu = np.array([-3.0, 0.0, 3.0, 6.0])
    y = make_mixture_data(777, mu, 0.55, seed=61)
    g = smc.Gmm.equal_weights(4, 1, 0.55)
    s = smc.SMCSampler(ctx, g, y, 128, np.linspace(0.0, 1.0, 5), 0.5, 1, 3)
    s.stream.synchronize()
    assert np.array_equal(s.y.cpu().numpy(), np.sort(y))
    assert not np.array_equal(y, np.sort(y))                              # the caller's copy
    p = smc.PTSampler(ctx, g, y, np.linspace(0.1, 1.0, 8), 0.5, 3)
    p.stream.synchronize()
    assert np.array_equal(p.y.cpu().numpy(), np.sort(y))
    datas = [make_mixture_data(n, mu, 0.55, seed=n) for n in (50, 300, 4100)]
    b = smc.BatchSampler(ctx, g, datas, [64, 64, 64], [1, 2, 3], np.linspace(0.0, 1.0, 4), 0.5, 1)
    b.stream.synchronize()
    assert np.array_equal(b.y.cpu().numpy(), np.concatenate([np.sort(d) for d in datas]))
    y8 = make_mixture_data(100, 3.0 * np.ones((2, 8)), 1.0, seed=62)
    s8 = smc.SMCSampler(ctx, smc.Gmm.equal_weights(2, 8, 1.0), y8, 64,
                        np.linspace(0.0, 1.0, 3), 0.5, 1, 3)
    s8.stream.synchronize()
    assert np.array_equal(s8.y.cpu().numpy(), y8)


def test_launch_table_selects_slices(smc, ctx):
    """A matching launch rule gives the same bits as the same explicit slice
    count; a non-matching rule leaves the built-in choice; bad rules raise."""
    announce("launch table")
    mu = np.array([-3.0, 0.0, 3.0, 6.0])
    y = _cuda(make_mixture_data(200, mu, 0.55, seed=2), torch.float32)
    g = smc.Gmm.equal_weights(4, 1, 0.55)
    th0 = _cuda(theta_prior_draws(4000, 4, 1, seed=3))
    l0 = torch.zeros(4000, dtype=torch.float64, device="cuda")

    def run():
        th, l = th0.clone(), l0.clone()
        smc.smc_loglik(ctx, g, y, th, "fp32", out=l)
        smc.smc_rwmh_move(ctx, g, y, th, l, 0.5, 0.5, seed=3, step=2, prec="fp32")
        torch.cuda.synchronize()
        return th.cpu().numpy(), l.cpu().numpy()

    base = run()
    ctx.set_slices(40)
    try:
        forced = run()
    finally:
        ctx.set_slices(0)
    rule = dict(k=4, d=1, prec="fp32", slices=40, n_lo=100, n_hi=300, N_lo=1, N_hi=5000)
    try:
        ctx.set_launch_table([rule])
        tabled = run()
        ctx.set_launch_table([dict(rule, n_lo=201)])
        missed = run()
        with pytest.raises(smc.SmcError):
            ctx.set_launch_table([dict(rule, slices=129)])
        with pytest.raises(smc.SmcError):
            ctx.set_launch_table([dict(rule, N_lo=6000)])
        # a batch rule (persistent batched move) is not a per-call rule, and
        # its slices must divide the workgroup's 8 waves
        ctx.set_launch_table([dict(rule, kind="batch", slices=4)])
        batch_only = run()
        with pytest.raises(smc.SmcError):
            ctx.set_launch_table([dict(rule, kind="batch", slices=3)])
        with pytest.raises(smc.SmcError):
            ctx.set_launch_table([dict(rule, kind="batch", slices=16)])
    finally:
        ctx.set_launch_table([])
    assert all(np.array_equal(a, b) for a, b in zip(batch_only, base))
    assert all(np.array_equal(a, b) for a, b in zip(tabled, forced))
    assert all(np.array_equal(a, b) for a, b in zip(missed, base))
    assert not np.array_equal(forced[1], base[1])          # the slicing changed the sums


def test_autotune_shapes(smc, ctx):
    """The tuner times every candidate of a 1-D and a d-dim shape and its rules
    install in the launch table."""
    announce("autotune")
    from paper_0905_2441_amd import autotune
    shapes = [(4, 1, 300, 2000, "fp32"), (8, 8, 256, 512, "bf16x3"), (2, 8, 200, 300, "fp64")]
    try:
        rules = autotune.make_rules(ctx, shapes, reps=2)
        ctx.set_launch_table(rules)
    finally:
        ctx.set_launch_table([])
    for (k, d, n, N, prec), r in zip(shapes, rules):
        assert r["slices"] in autotune.candidates(n, N, prec)
        assert set(r["ms"]) == {str(t) for t in autotune.candidates(n, N, prec)}
        assert r["n_lo"] <= n <= r["n_hi"] and r["N_lo"] <= N <= r["N_hi"]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_rwmh_move_pt_size_sampled(smc, ctx, prec):
    """One move of 8192 chains at their own temperatures over n = 10000 data (the
    population-MCMC workload, automatic launch shape: 4 workgroups per tile),
    checked against the oracle's move on 256 sampled chains. Each chain's move
    depends only on its own state and counter, so the sample is exact."""
    announce(f"rwmh pt-size sampled {prec}")
    mu = np.array([-3.0, 0.0, 3.0, 6.0])
    n, M, kd = 10000, 8192, 4
    y = make_mixture_data(n, mu, 0.55, seed=21)
    g = smc.Gmm.equal_weights(4, 1, 0.55)
    om = oracle_model(g)
    betas = pt_betas(M, 4)
    th = np.hstack([theta_prior_draws(M // 2, 4, 1, seed=22), theta_near_posterior(M // 2, mu, seed=23)])
    rng = np.random.default_rng(24)
    idx = np.unique(np.concatenate([np.arange(64), rng.choice(M, 128, replace=False),
                                    np.arange(M - 64, M)]))
    l = np.full(M, -1.0e4)
    l[idx] = ogmm.loglik(th[:, idx], y, om)
    tt, lt = _cuda(th), _cuda(l)
    sd, seed, step, move = 0.05, 31, 9, 0
    smc.smc_rwmh_move(ctx, g, _cuda(y, torch.float32), tt, lt, 0.0, sd, seed=seed, step=step,
                      move=move, prec=prec, beta_vec=_cuda(betas))
    ctx.check()
    uidx = idx.astype(np.uint64)
    prop = th[:, idx] + sd * opx.normals(seed, uidx, step, opx.PROP, move, kd)
    l_prop = ogmm.loglik(prop, y, om)
    la = osmc.rwmh_log_alpha(betas[idx], l[idx], l_prop, ogmm.log_prior(th[:, idx], om),
                             ogmm.log_prior(prop, om))
    acc_ref = (la >= 0.0) | (np.log(opx.uniforms_open(seed, uidx, step, opx.ACC, move)) < la)
    got_th, got_l = tt.cpu().numpy()[:, idx], lt.cpu().numpy()[idx]
    acc_got = np.any(got_th != th[:, idx], axis=0)
    flips = int(np.sum(acc_got != acc_ref))
    assert flips == 0 if prec == "fp64" else flips <= 2
    assert 10 < int(acc_ref.sum()) < idx.size - 10          # both outcomes occur
    same = acc_got == acc_ref
    want_th = np.where(acc_ref, prop, th[:, idx])
    want_l = np.where(acc_ref, l_prop, l[idx])
    assert np.max(np.abs(got_th[:, same] - want_th[:, same])) <= 1e-12
    tol = 1e-12 if prec == "fp64" else 1e-6
    assert rel_err(got_l[same], want_l[same]).max() <= tol


@pytest.mark.parametrize("prec,it", [("fp32", 11), ("fp64", 12)])
def test_pt_iteration_workload_size_sampled(smc, ctx, prec, it):
    """One population-MCMC iteration of the 8192-chain workload (n = 10^4) in
    the benchmark's launch shape (32 slices: each tile over two workgroups, so
    the moves' decisions and the exchanges run in one kernel), checked on 40
    sampled pairs of the iteration's partition: both chains' moves, then the
    pair's exchange, against the oracle. A pair depends only on its own two
    chains, so the sample is exact."""
    cfg = CONFIGS["pt_k4_n10000_M8192"]
    announce(f"pt iteration workload size {prec} it={it}")
    y = make_data(cfg)
    M, kd = cfg.N, 4
    mu = np.array(cfg.true_means)
    betas = pt_betas(M, 4)
    g = smc.Gmm.equal_weights(4, 1, cfg.sigma2)
    om = oracle_model(g)
    th = np.hstack([theta_prior_draws(M // 4, 4, 1, seed=61),
                    theta_near_posterior(M - M // 4, mu, seed=62, jitter=0.3)])
    parity = it & 1
    rng = np.random.default_rng(63)
    npairs = (M - parity) // 2                 # pairs (parity + 2q, parity + 2q + 1)
    leads = parity + 2 * np.unique(np.concatenate([[0, npairs - 1],
                                                   rng.choice(npairs, 38, replace=False)]))
    chains = np.unique(np.concatenate([leads, leads + 1]))
    l = np.full(M, -1.0e6)
    l[chains] = ogmm.loglik(th[:, chains], y, om)
    tt, lt = _cuda(th), _cuda(l)
    itd = torch.full((1,), it, dtype=torch.int32).cuda()
    sd, seed = cfg.step_sd, 71
    ctx.set_slices(32)
    try:
        smc.pt_iteration(ctx, g, _cuda(y, torch.float32), tt, lt, _cuda(betas), itd, sd, seed,
                         0, False, prec)
        ctx.check()
    finally:
        ctx.set_slices(0)
    assert itd.item() == it + 1
    # the oracle: moves of the sampled chains, then their pairs' exchanges
    uc = chains.astype(np.uint64)
    prop = th[:, chains] + sd * opx.normals(seed, uc, it, opx.PROP, 0, kd)
    l_prop = ogmm.loglik(prop, y, om)
    la = osmc.rwmh_log_alpha(betas[chains], l[chains], l_prop, ogmm.log_prior(th[:, chains], om),
                             ogmm.log_prior(prop, om))
    acc = (la >= 0.0) | (np.log(opx.uniforms_open(seed, uc, it, opx.ACC, 0)) < la)
    ref_th = th.copy()
    ref_l = l.copy()
    ref_th[:, chains] = np.where(acc, prop, th[:, chains])
    ref_l[chains] = np.where(acc, l_prop, l[chains])
    swapped = 0
    for a in leads:
        b = a + 1
        lx = osmc.exchange_log_alpha(betas[a], betas[b], ref_l[a], ref_l[b])
        u = float(opx.uniforms_open(seed, int(a), it, opx.EXCH, 0))
        if lx >= 0.0 or np.log(u) < lx:
            ref_th[:, [a, b]] = ref_th[:, [b, a]]
            ref_l[a], ref_l[b] = ref_l[b], ref_l[a]
            swapped += 1
    got_th, got_l = tt.cpu().numpy(), lt.cpu().numpy()
    same = np.all(np.abs(got_th[:, chains] - ref_th[:, chains]) <= 1e-12, axis=0)
    assert int(np.sum(~same)) <= (0 if prec == "fp64" else 4)
    tol = 1e-12 if prec == "fp64" else 1e-6
    assert rel_err(got_l[chains][same], ref_l[chains][same]).max() <= tol
    assert 0 < int(acc.sum()) < chains.size and swapped > 0


# ------------------------------------------------------------------ exchange

@pytest.mark.parametrize("M,parity,wrap", [(8192, 0, False), (8192, 1, False), (64, 1, True),
                                           (7, 0, False), (7, 1, True), (2, 0, False)])
def test_exchange_matches_oracle(smc, ctx, M, parity, wrap):
    announce(f"exchange M={M} parity={parity} wrap={wrap}")
    rng = np.random.default_rng(M + parity)
    betas = pt_betas(M, 4)
    th = rng.normal(size=(4, M))
    l = -1000.0 + 50.0 * rng.normal(size=M)
    tt, lt = _cuda(th), _cuda(l)
    ns = torch.zeros(1, dtype=torch.int32).cuda()
    smc.pt_exchange(ctx, tt, lt, _cuda(betas), parity, wrap, seed=17, iteration=33, n_swap=ns)
    th_ref, l_ref, n_ref = osmc.pt_exchange(th, l, betas, parity, wrap, 17, 33)
    assert np.array_equal(lt.cpu().numpy(), l_ref)
    assert np.array_equal(tt.cpu().numpy(), th_ref)
    assert ns.item() == n_ref


# ------------------------------------------------------------------ several PT iterations

@pytest.mark.parametrize("k,d,prec,M,slices,parity,wrap,iters", [
    (4, 1, "fp32", 1024, 1, 0, False, 6),      # 16 tiles: the largest population at k*d = 4
    (4, 1, "fp64", 100, 8, 1, True, 9),        # ragged tile, random parity with the wrap pair
    (7, 1, "fp64", 576, 1, 1, True, 5),        # k*d = 7: 576 chains in LDS
    (2, 8, "fp32", 256, 4, 0, False, 4),       # k*d = 16: 256 chains
    (1, 1, "fp32", 2, 16, 1, False, 11),       # two chains, 16 slices of one tile
    (4, 1, "fp32", 1025, 0, 0, False, 3),      # past the single-workgroup form
    # one launch per iteration with the exchange deferred (odd and even counts)
    (4, 1, "fp32", 1025, 4, 1, True, 3),
    (4, 1, "fp64", 2048, 2, 1, True, 4),
    (2, 8, "fp32", 700, 2, 0, False, 5),
    (1, 1, "fp64", 1500, 8, 1, True, 1),
])
def test_pt_iterations_equal_single_iterations(smc, ctx, k, d, prec, M, slices, parity, wrap,
                                               iters):
    """pt_iterations(n) leaves exactly the state, counter and tallies of n
    pt_iteration calls with the same launch shape (both sum a tile's slices in
    the same order, so even FP32 agrees bit for bit): the single-workgroup
    form for populations that fit, else one launch per iteration with the
    exchange deferred into the next launch."""
    announce(f"pt_iterations k={k} d={d} {prec} M={M} slices={slices} parity={parity}")
    rng = np.random.default_rng(M + 7 * k)
    mu = rng.uniform(-4.0, 6.0, size=(k, d)) if d > 1 else np.linspace(-3.0, 6.0, k)
    y = make_mixture_data(700, mu, 0.55, seed=M)
    g = smc.Gmm.equal_weights(k, d, 0.55)
    om = oracle_model(g)
    betas = pt_betas(M, 4)
    th = theta_prior_draws(M, k, d, seed=M + 1)
    l = ogmm.loglik(th, y, om)
    yd = _cuda(y, torch.float32)
    bd = _cuda(betas)
    outs = []
    ctx.set_slices(slices)
    ctx.set_pt_single_workgroup(1)
    try:
        for fused in (True, False):
            tt, lt = _cuda(th), _cuda(l)
            it = torch.full((1,), 5, dtype=torch.int32).cuda()
            na = torch.zeros(1, dtype=torch.int64).cuda()
            ns = torch.zeros(1, dtype=torch.int32).cuda()
            if fused:
                smc.pt_iterations(ctx, g, yd, tt, lt, bd, it, iters, 0.3, 41, parity, wrap, prec,
                                  na, ns)
            else:
                for _ in range(iters):
                    smc.pt_iteration(ctx, g, yd, tt, lt, bd, it, 0.3, 41, parity, wrap, prec,
                                     na, ns)
            ctx.check()
            outs.append((tt.cpu().numpy(), lt.cpu().numpy(), it.item(), na.item(), ns.item()))
    finally:
        ctx.set_slices(0)
        ctx.set_pt_single_workgroup(0)
    (t1, l1, i1, a1, s1), (t2, l2, i2, a2, s2) = outs
    assert i1 == i2 == 5 + iters
    assert np.array_equal(t1, t2) and np.array_equal(l1, l2)
    assert (a1, s1) == (a2, s2)
    assert 0 < a1 < M * iters          # moves both accepted and rejected
    if M > 2:
        assert s1 > 0


def test_pt_iterations_matches_oracle_and_rejects_bad_count(smc, ctx):
    """Twenty iterations of 300 chains against the oracle's population MCMC
    run (FP64, alternating parity) in each of pt_iterations' forms (one
    single-workgroup launch; automatic; per iteration), and n_iters < 1 or an
    unknown mode refused."""
    mu = np.array([-3.0, 0.0, 3.0, 6.0])
    y = make_mixture_data(250, mu, 0.55, seed=12)
    M, iters = 300, 20
    betas = pt_betas(M, 4)
    g = smc.Gmm.equal_weights(4, 1, 0.55)
    om = oracle_model(g)
    ref = osmc.pt_run(y, om, betas, iters, 0.5, 88, parity_mode="alternate", wrap=False)
    try:
        for mode in (1, 0, -1):
            announce(f"pt_iterations oracle M=300 mode={mode}")
            ctx.set_pt_single_workgroup(mode)
            s = smc.PTSampler(ctx, g, y, betas, 0.5, seed=88, parity_mode=0, wrap=False,
                              prec="fp64")
            s.init()
            smc.pt_iterations(ctx, g, s.y, s.theta, s.loglik, s.beta, s.it, iters, 0.5, 88, 0,
                              False, "fp64", s.n_accept, s.n_swap, stream=s.stream)
            s.stream.synchronize()
            ctx.check()
            assert s.it.item() == iters
            assert s.n_swap.item() == ref["swaps"]
            assert s.n_accept.item() == ref["accepted"]
            assert np.max(np.abs(s.theta.cpu().numpy() - ref["theta"])) <= 1e-9
            assert rel_err(s.loglik.cpu().numpy(), ref["l"]).max() <= 1e-10
    finally:
        ctx.set_pt_single_workgroup(0)
    with pytest.raises(smc.SmcError):
        smc.pt_iterations(ctx, g, s.y, s.theta, s.loglik, s.beta, s.it, 0, 0.5, 88)
    with pytest.raises(smc.SmcError):
        ctx.set_pt_single_workgroup(2)


def test_rwmh_move_ddim_workload_size_sampled(smc, ctx):
    """One MFMA move of the d = 8, k = 8 workload at its full size (N = 16384,
    n = 65536), checked against the oracle's move on 96 sampled particles (each
    particle's move depends only on its own state and counter)."""
    cfg = CONFIGS["gmm8d_k8_n65536_N16384"]
    announce("rwmh d=8 workload size sampled")
    y = make_data(cfg)
    mu = true_means_for(cfg)
    N, kd = cfg.N, 64
    th = np.hstack([theta_prior_draws(N // 2, 8, 8, seed=41), theta_near_posterior(N // 2, mu, seed=42)])
    g = smc.Gmm.equal_weights(8, 8, cfg.sigma2)
    om = oracle_model(g)
    rng = np.random.default_rng(43)
    idx = np.unique(np.concatenate([np.arange(16), rng.choice(N, 64, replace=False),
                                    np.arange(N - 16, N)]))
    l = np.full(N, -1.0e6)
    l[idx] = ogmm.loglik(th[:, idx], y, om, chunk_elems=1 << 24)
    tt, lt = _cuda(th), _cuda(l)
    sd, seed, step, move, beta = 0.02, 51, 7, 0, 0.9
    smc.smc_rwmh_move(ctx, g, _cuda(y, torch.float32), tt, lt, beta, sd, seed=seed, step=step,
                      move=move, prec="bf16x3")
    ctx.check()
    uidx = idx.astype(np.uint64)
    prop = th[:, idx] + sd * opx.normals(seed, uidx, step, opx.PROP, move, kd)
    l_prop = ogmm.loglik(prop, y, om, chunk_elems=1 << 24)
    la = osmc.rwmh_log_alpha(np.full(idx.size, beta), l[idx], l_prop,
                             ogmm.log_prior(th[:, idx], om), ogmm.log_prior(prop, om))
    acc_ref = (la >= 0.0) | (np.log(opx.uniforms_open(seed, uidx, step, opx.ACC, move)) < la)
    got_th, got_l = tt.cpu().numpy()[:, idx], lt.cpu().numpy()[idx]
    acc_got = np.any(got_th != th[:, idx], axis=0)
    assert int(np.sum(acc_got != acc_ref)) <= 2
    assert 5 < int(acc_ref.sum()) < idx.size - 5            # both outcomes occur
    same = acc_got == acc_ref
    want_th = np.where(acc_ref, prop, th[:, idx])
    want_l = np.where(acc_ref, l_prop, l[idx])
    assert np.max(np.abs(got_th[:, same] - want_th[:, same])) <= 1e-12
    assert rel_err(got_l[same], want_l[same]).max() <= 1e-6


@pytest.mark.parametrize("prec", ["bf16x3", "fp64"])
def test_rwmh_move_ddim_matches_oracle(smc, ctx, prec):
    """d = 8, k = 4 move: MFMA form (and the FP64 VALU form) against the oracle."""
    announce(f"rwmh d=8 {prec}")
    rng = np.random.default_rng(3)
    mu = 3.0 * rng.standard_normal((4, 8))
    y = make_mixture_data(500, mu, 1.0, seed=7)
    g = smc.Gmm.equal_weights(4, 8, 1.0)
    om = oracle_model(g)
    N = 600
    th = np.hstack([theta_prior_draws(N // 2, 4, 8, seed=3), theta_near_posterior(N // 2, mu, seed=4)])
    l = ogmm.loglik(th, y, om)
    tt, lt = _cuda(th), _cuda(l)
    acc = torch.zeros(1, dtype=torch.int64).cuda()
    smc.smc_rwmh_move(ctx, g, _cuda(y, torch.float32), tt, lt, 0.8, 0.05, seed=21, step=4,
                      move=1, prec=prec, n_accept=acc)
    ctx.check()
    th_ref, l_ref, a_ref = osmc.rwmh_move(th, l, y, om, 0.8, 0.05, 21, 4, 1)
    got_th, got_l = tt.cpu().numpy(), lt.cpu().numpy()
    a_got = np.any(got_th != th, axis=0)
    flips = int(np.sum(a_got != a_ref))
    assert flips <= (0 if prec == "fp64" else 2)
    assert 0 < a_got.sum() < N
    same = a_got == a_ref
    assert acc.item() == int(a_got.sum())
    assert np.max(np.abs(got_th[:, same] - th_ref[:, same])) <= 1e-12
    tol = 1e-12 if prec == "fp64" else 1e-6
    assert rel_err(got_l[same], l_ref[same]).max() <= tol
