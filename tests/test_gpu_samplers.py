"""GPU parity of whole runs under matched randomness: the tempered SMC sampler
(small workload, FP64 and FP32) and population MCMC, eager and graph-replayed."""

import numpy as np
import pytest
import torch

from gpu_common import announce, loglik_threads, oracle_model, rel_err, replay_positions
from oracle import gmm as ogmm
from oracle import smc as osmc
from workloads import CONFIGS, beta_schedule, make_data, pt_betas, make_mixture_data

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def smc():
    import paper_0905_2441_amd as smc
    return smc


@pytest.fixture(scope="module")
def ctx(smc):
    return smc.Context(0)


@pytest.fixture(scope="module")
def small():
    cfg = CONFIGS["gmm1d_k4_n100_N1024"]
    y = make_data(cfg)
    betas = beta_schedule(cfg.T, cfg.schedule)
    return cfg, y, betas


@pytest.fixture(scope="module")
def small_oracle(small):
    cfg, y, betas = small
    from oracle.gmm import Model
    om = Model.equal_weights(cfg.k, cfg.d, cfg.sigma2, prior=cfg.prior, prior_a=cfg.prior_a,
                             prior_b=cfg.prior_b)
    return osmc.smc_run(y, om, betas, cfg.N, cfg.step_sd, cfg.n_moves, cfg.run_seed,
                        ess_frac=cfg.ess_frac)


def _sampler(smc, ctx, cfg, y, betas, prec):
    g = smc.Gmm.equal_weights(cfg.k, cfg.d, cfg.sigma2, prior=cfg.prior, prior_a=cfg.prior_a,
                              prior_b=cfg.prior_b)
    return smc.SMCSampler(ctx, g, y, cfg.N, betas, cfg.step_sd, cfg.n_moves, cfg.run_seed,
                          ess_frac=cfg.ess_frac, prec=prec)


@pytest.mark.parametrize("graph,steps_per_call,slices", [(False, 1, 0), (True, 1, 0),
                                                         (False, 10, 4), (True, 7, 4)])
def test_smc_small_fp64_matches_oracle(smc, ctx, small, small_oracle, graph, steps_per_call,
                                       slices):
    """Single steps, and chains of 10 or 7 steps per smc_steps call (4 slices:
    one workgroup per tile, so each move also makes the next step's reweight;
    7 leaves a ragged last group), eager and replayed, equal the oracle."""
    cfg, y, betas = small
    announce(f"smc small fp64 graph={graph} steps/call={steps_per_call} slices={slices}")
    s = _sampler(smc, ctx, cfg, y, betas, "fp64")
    ctx.set_slices(slices)
    try:
        r = s.run(graph=graph, steps_per_graph=steps_per_call)
    finally:
        ctx.set_slices(0)
    ref = small_oracle
    assert r["t"] == cfg.T + 1
    assert r["resamples"] == int(np.sum(ref["trace"]["resampled"]))
    assert abs(r["logZ"] - ref["logZ"]) <= 1e-3
    assert np.max(np.abs(r["theta"] - ref["theta"])) <= 1e-9
    assert rel_err(r["l"], ref["l"]).max() <= 1e-10
    assert r["accepted"] == int(np.sum(ref["trace"]["accepted"]))
    assert np.max(np.abs(r["W"] - ref["W"])) <= 1e-14
    assert np.max(np.abs(r["logw"] - ref["logw"])) <= 1e-9


@pytest.mark.parametrize("scheme", ["stratified", "multinomial"])
def test_smc_other_schemes_match_oracle(smc, ctx, small, scheme):
    """The small FP64 run with stratified or multinomial resampling (chosen by
    the context setting, searched inside the first move) equals the oracle's."""
    cfg, y, betas = small
    announce(f"smc small fp64 {scheme}")
    from oracle.gmm import Model
    om = Model.equal_weights(cfg.k, cfg.d, cfg.sigma2, prior=cfg.prior, prior_a=cfg.prior_a,
                             prior_b=cfg.prior_b)
    ref = osmc.smc_run(y, om, betas, cfg.N, cfg.step_sd, cfg.n_moves, cfg.run_seed,
                       ess_frac=cfg.ess_frac, scheme=scheme)
    g = smc.Gmm.equal_weights(cfg.k, cfg.d, cfg.sigma2, prior=cfg.prior, prior_a=cfg.prior_a,
                              prior_b=cfg.prior_b)
    s = smc.SMCSampler(ctx, g, y, cfg.N, betas, cfg.step_sd, cfg.n_moves, cfg.run_seed,
                       ess_frac=cfg.ess_frac, prec="fp64", scheme=scheme)
    try:
        r = s.run(graph=True)
    finally:
        ctx.set_resampling("systematic")
    assert r["resamples"] == int(np.sum(ref["trace"]["resampled"])) > 0
    assert r["accepted"] == int(np.sum(ref["trace"]["accepted"]))
    assert np.max(np.abs(r["theta"] - ref["theta"])) <= 1e-9
    assert rel_err(r["l"], ref["l"]).max() <= 1e-10
    assert abs(r["logZ"] - ref["logZ"]) <= 1e-3


@pytest.mark.parametrize("slices", [0, 40])
def test_smc_paper_mode_ten_moves_match_oracle(smc, ctx, slices):
    """The paper's sampler settings (box prior, sigma = 0.55 as a scale, ten
    N(0, I) moves per step) over 30 steps, FP64: with one workgroup per tile the
    ten moves run in one launch (states in LDS); slices = 40 spreads each tile
    over three workgroups and launches the moves one by one. Both equal the
    oracle."""
    from workloads.configs import paper_mode
    announce(f"smc paper mode ten moves slices={slices}")
    cfg = paper_mode(512)
    y = make_data(cfg)
    betas = beta_schedule(30, "quadratic")
    g = smc.Gmm.equal_weights(cfg.k, cfg.d, cfg.sigma2, prior=cfg.prior, prior_a=cfg.prior_a,
                              prior_b=cfg.prior_b)
    om = oracle_model(g)
    ref = osmc.smc_run(y, om, betas, cfg.N, cfg.step_sd, cfg.n_moves, cfg.run_seed,
                       ess_frac=cfg.ess_frac)
    ctx.set_slices(slices)
    try:
        s = smc.SMCSampler(ctx, g, y, cfg.N, betas, cfg.step_sd, cfg.n_moves, cfg.run_seed,
                           ess_frac=cfg.ess_frac, prec="fp64")
        r = s.run(graph=True, steps_per_graph=10)
    finally:
        ctx.set_slices(0)
    assert r["resamples"] == int(np.sum(ref["trace"]["resampled"])) > 0
    assert r["accepted"] == int(np.sum(ref["trace"]["accepted"]))
    assert np.max(np.abs(r["theta"] - ref["theta"])) <= 1e-9
    assert rel_err(r["l"], ref["l"]).max() <= 1e-10
    assert np.max(np.abs(r["W"] - ref["W"])) <= 1e-14
    assert abs(r["logZ"] - ref["logZ"]) <= 1e-3


def test_smc_split_tiles_match_oracle(smc, ctx, small, small_oracle):
    """The small run with each tile's data spread over 3 workgroups per move
    (42 slices of 2-3 observations); the fused ancestor search then runs in every
    workgroup and the decision kernel reads group 0's ancestors."""
    cfg, y, betas = small
    announce("smc small fp64 split tiles")
    ctx.set_slices(40)
    try:
        r = _sampler(smc, ctx, cfg, y, betas, "fp64").run(graph=True)
    finally:
        ctx.set_slices(0)
    ref = small_oracle
    assert r["resamples"] == int(np.sum(ref["trace"]["resampled"]))
    assert r["accepted"] == int(np.sum(ref["trace"]["accepted"]))
    assert np.max(np.abs(r["theta"] - ref["theta"])) <= 1e-9
    assert rel_err(r["l"], ref["l"]).max() <= 1e-10
    assert np.max(np.abs(r["W"] - ref["W"])) <= 1e-14


@pytest.mark.parametrize("n_moves,ess_frac", [(0, 0.5), (3, 0.5), (1, 0.0), (2, 1.0)])
def test_smc_step_variants_match_oracle(smc, ctx, small, n_moves, ess_frac):
    """No moves (pure reweight/resample), several moves per step, no resampling
    (annealed importance sampling), and resampling at every step."""
    cfg, y, betas = small
    announce(f"smc variants moves={n_moves} ess_frac={ess_frac}")
    from oracle.gmm import Model
    om = Model.equal_weights(cfg.k, cfg.d, cfg.sigma2)
    N = 300
    g = smc.Gmm.equal_weights(cfg.k, cfg.d, cfg.sigma2)
    s = smc.SMCSampler(ctx, g, y, N, betas[:13], cfg.step_sd, n_moves, 77, ess_frac=ess_frac,
                       prec="fp64")
    r = s.run(graph=True)
    ref = osmc.smc_run(y, om, betas[:13], N, cfg.step_sd, n_moves, 77, ess_frac=ess_frac,
                       resample=ess_frac > 0.0)
    assert r["resamples"] == int(np.sum(ref["trace"]["resampled"]))
    assert abs(r["logZ"] - ref["logZ"]) <= 1e-9 * max(1.0, abs(ref["logZ"]))
    assert np.max(np.abs(r["theta"] - ref["theta"])) <= 1e-9
    assert np.max(np.abs(r["W"] - ref["W"])) <= 1e-14


def test_smc_graph_replay_is_bit_identical_to_eager(smc, ctx, small):
    cfg, y, betas = small
    announce("smc graph vs eager")
    a = _sampler(smc, ctx, cfg, y, betas, "fp32").run(graph=False)
    b = _sampler(smc, ctx, cfg, y, betas, "fp32").run(graph=True)
    assert a["logZ"] == b["logZ"]
    assert np.array_equal(a["theta"], b["theta"])
    for spg in (2, 7, 10):              # several steps in one smc_steps call / graph
        for slices in (0, 4):           # split tiles (plain steps) and fused reweights
            ctx.set_slices(slices)
            try:
                c = _sampler(smc, ctx, cfg, y, betas, "fp32").run(graph=True, steps_per_graph=spg)
                d = _sampler(smc, ctx, cfg, y, betas, "fp32").run(graph=False, steps_per_graph=spg)
            finally:
                ctx.set_slices(0)
            assert c["logZ"] == d["logZ"] and np.array_equal(c["theta"], d["theta"])
            assert np.array_equal(c["W"], d["W"]) and c["t"] == d["t"] == cfg.T + 1
            # other slicings round each datum's FP32 term differently (the
            # expanded forms centre each slice's data on its own midrange):
            # log Z moves by at most the largest change of a particle's
            # log-likelihood, each within the FP32 form's 1e-6 relative bound
            assert abs(c["logZ"] - a["logZ"]) <= 1e-6 * max(1.0, abs(a["logZ"]))
            assert c["resamples"] == a["resamples"]
    # repeated replays of the same sampler give the same answer again
    s = _sampler(smc, ctx, cfg, y, betas, "fp32")
    c = s.run(graph=True)
    d = s.run(graph=True)
    assert c["logZ"] == d["logZ"] and np.array_equal(c["theta"], d["theta"])


def test_graphs_captured_before_scratch_growth_stay_valid(smc, small, small_oracle):
    """Graphs of both step directions are captured on a fresh context, then a
    larger reservation regrows its scratch (VALU and MFMA forms) to new
    addresses. The context keeps the superseded scratch, so replaying the old
    graphs still runs the small FP64 run exactly as the oracle does."""
    cfg, y, betas = small
    announce("graphs replayed after the context scratch grew")
    c2 = smc.Context(0)
    s = _sampler(smc, c2, cfg, y, betas, "fp64")
    try:
        s.capture(0, 1)
        s.capture(1, 1)
        c2.reserve(1 << 20, 8, 1 << 16)
        r = s.run(graph=True)
    finally:
        for g in s.graphs.values():
            g.close()
        s.graphs.clear()
        s.stream.synchronize()
        c2.close()
    ref = small_oracle
    assert r["resamples"] == int(np.sum(ref["trace"]["resampled"]))
    assert r["accepted"] == int(np.sum(ref["trace"]["accepted"]))
    assert np.max(np.abs(r["theta"] - ref["theta"])) <= 1e-9
    assert abs(r["logZ"] - ref["logZ"]) <= 1e-3


def _snapshot(s):
    s.stream.synchronize()
    return (s.theta.cpu().numpy().copy(), s.loglik.cpu().numpy().copy(),
            s.logw.cpu().numpy().copy(), float(s.stats[0].item()))


def test_smc_small_fp32_stepwise_replay(smc, ctx, small):
    """FP32 run checked step by step: the oracle takes every step from the GPU's
    own state, so reweight/ESS/resampling must agree to FP64 rounding and the
    moves may differ only by FP32 near-tie accept flips, which are counted."""
    cfg, y, betas = small
    announce("smc small fp32 stepwise")
    from oracle.gmm import Model
    om = Model.equal_weights(cfg.k, cfg.d, cfg.sigma2, prior=cfg.prior, prior_a=cfg.prior_a,
                             prior_b=cfg.prior_b)
    s = _sampler(smc, ctx, cfg, y, betas, "fp32")
    s.init()
    th, l, lw, z = _snapshot(s)
    l_ref0 = ogmm.loglik(th, y, om)
    assert rel_err(l, l_ref0).max() <= 1e-6
    flips = decisions = 0
    sum_gpu = sum_ref = 0.0
    for t in range(1, cfg.T + 1):
        s.step(graph=False)
        th1, l1, lw1, z1 = _snapshot(s)
        rth, rl, rlw, _, inc, info = osmc.smc_step(th, l, lw, y, om, betas, t, cfg.step_sd,
                                                   cfg.n_moves, cfg.run_seed, cfg.ess_frac)
        assert abs((z1 - z) - inc) <= 1e-10 * max(1.0, abs(inc))
        assert np.array_equal(lw1, rlw) or np.max(np.abs(lw1 - rlw)) <= 1e-12
        same = np.all(th1 == rth, axis=0) | np.all(np.abs(th1 - rth) <= 1e-12, axis=0)
        flips += int(np.sum(~same))
        decisions += cfg.N * cfg.n_moves
        assert rel_err(l1[same], rl[same]).max() <= 1e-6
        sum_gpu += z1 - z
        sum_ref += inc
        th, l, lw, z = th1, l1, lw1, z1
    assert flips <= max(3, decisions // 1000), flips
    assert abs(sum_gpu - sum_ref) <= 1e-3
    print(f"fp32 flipped decisions: {flips} of {decisions}")


@pytest.mark.parametrize("workload,prec,slices,n_steps,start", [
    ("gmm1d_k4_n100_N1024", "fp64", 4, 7, 0),
    ("gmm1d_k4_n100_N1024", "fp64", 0, 6, 0),            # split tiles: plain steps
    ("gmm1d_k4_n1000_N131072", "fp32", 4, 10, 0),
    ("gmm1d_k4_n1000_N131072", "fp32", 4, 100, 0),         # the benchmark's whole-run chain
    ("gmm1d_k4_n1000_N131072", "fp64", 8, 5, 45),
    ("ragged_N150017_n200", "fp32", 4, 6, 0),            # 2345 tile partials, last tile of 1
    ("paper_smc_N4000", "fp64", 2, 9, 0),                # ten moves per step in one launch
    ("paper_smc_N4000", "fp32", 4, 8, 100)])
def test_smc_steps_equal_single_steps(smc, ctx, workload, prec, slices, n_steps, start):
    """smc_steps(n) against n smc_step calls from the same state: with one
    workgroup per tile and all of a step's moves in one launch (one move, or the
    paper's ten at k*d <= 16) every step's last move but the final one also
    makes the next step's reweight, so weights, ESS and evidence may differ in
    the last bits; populations, resampling decisions and accept counts are equal."""
    if workload == "ragged_N150017_n200":
        import dataclasses
        cfg = dataclasses.replace(CONFIGS["gmm1d_k4_n1000_N131072"], N=150017, n=200)
    elif workload == "paper_smc_N4000":
        from workloads.configs import paper_mode
        cfg = paper_mode(4000)
    else:
        cfg = CONFIGS[workload]
    announce(f"smc_steps {workload} {prec} slices={slices} n={n_steps} from t={start + 1}")
    y = make_data(cfg)
    betas = beta_schedule(cfg.T, cfg.schedule)
    s1 = _sampler(smc, ctx, cfg, y, betas, prec)
    s2 = _sampler(smc, ctx, cfg, y, betas, prec)
    ctx.set_slices(slices)
    try:
        # the two samplers share the context's scratch: one after the other
        for s, chained in ((s1, True), (s2, False)):
            s.init()
            s.advance(start, graph=False)
            if chained:
                s.step(graph=False, steps=n_steps)
            else:
                for _ in range(n_steps):
                    s.step(graph=False)
            s.stream.synchronize()
            ctx.check(s.stream)
    finally:
        ctx.set_slices(0)
    st1, st2 = s1.stats.cpu().numpy(), s2.stats.cpu().numpy()
    assert s1.t.item() == s2.t.item() == start + n_steps + 1
    assert st1[2] == st2[2]                                   # resampling steps
    assert abs(st1[0] - st2[0]) <= 1e-10 * max(1.0, abs(st2[0]))
    assert abs(st1[1] - st2[1]) <= 1e-10 * st2[1]
    assert s1.n_accept.item() == s2.n_accept.item()
    assert np.array_equal(s1.theta.cpu().numpy(), s2.theta.cpu().numpy())
    assert np.array_equal(s1.loglik.cpu().numpy(), s2.loglik.cpu().numpy())
    lw1, lw2 = s1.logw.cpu().numpy(), s2.logw.cpu().numpy()
    assert np.max(np.abs(lw1 - lw2)) <= 1e-12 * max(1.0, np.abs(lw2).max())
    assert rel_err(s1.W.cpu().numpy(), s2.W.cpu().numpy()).max() <= 1e-12


def test_smc_steps_rejects_bad_arguments(smc, ctx, small):
    """A step count below one, or one population (or log-likelihood array)
    passed as both buffers: an error and nothing enqueued (counter, weights and
    populations unchanged)."""
    cfg, y, betas = small
    announce("smc_steps argument errors")
    s = _sampler(smc, ctx, cfg, y, betas, "fp64")
    s.init()
    s.stream.synchronize()
    before = (s.t.item(), s.logw.cpu().numpy().copy(), s.thetas[0].cpu().numpy().copy())
    a, b = s.thetas, s.logliks
    common = dict(n_accept=s.n_accept, stream=s.stream)
    args = lambda ta, la, tb, lb, n_steps: (ctx, s.model, s.y, ta, la, tb, lb, s.logw, s.W,
                                            s.beta, s.t, n_steps, s.step_sd, 1, s.seed,
                                            s.ess_frac, "fp64", s.stats)
    for bad in (args(a[0], b[0], a[1], b[1], 0), args(a[0], b[0], a[1], b[1], -3),
                args(a[0], b[0], a[0], b[1], 4), args(a[0], b[0], a[1], b[0], 4)):
        with pytest.raises(smc.SmcError):
            smc.smc_steps(*bad, **common)
    s.stream.synchronize()
    assert s.t.item() == before[0]
    assert np.array_equal(s.logw.cpu().numpy(), before[1])
    assert np.array_equal(s.thetas[0].cpu().numpy(), before[2])


@pytest.mark.parametrize("prec,slices", [("fp32", 4), ("fp64", 8)])
def test_headline_size_steps_from_gpu_state(smc, ctx, prec, slices):
    """At the headline size (N = 131072, n = 1000) in the launch shape the
    benchmark times (4 slices per tile in FP32, 8 in FP64): the first step
    whose ESS test fires (reweight, correctly rounded CDF, ancestor search
    fused into the move) and a step near the posterior (t = 30, the direct FP32
    form) are each checked against the oracle's step taken from the GPU's own
    state. FP64 must agree in every decision; FP32 may flip near-tie accepts,
    which are counted."""
    cfg = CONFIGS["gmm1d_k4_n1000_N131072"]
    announce(f"headline-size steps {prec} slices={slices}")
    y = make_data(cfg)
    betas = beta_schedule(cfg.T, cfg.schedule)
    from oracle.gmm import Model
    om = Model.equal_weights(cfg.k, cfg.d, cfg.sigma2)
    s = _sampler(smc, ctx, cfg, y, betas, prec)
    ctx.set_slices(slices)
    try:
        s.init()
        prev = _snapshot(s)
        fired_at = None
        for t in range(1, 30):
            s.step(graph=False)
            s.stream.synchronize()
            if s.stats[2].item() > 0:
                fired_at = t
                break
            prev = _snapshot(s)
        assert fired_at is not None, "no resampling in the first 29 steps"
        checks = [(fired_at, prev, _snapshot(s))]
        s.advance(29 - fired_at, graph=True)
        before = _snapshot(s)
        s.step(graph=False)
        checks.append((30, before, _snapshot(s)))
    finally:
        ctx.set_slices(0)
    tol_l = 1e-6 if prec == "fp32" else 1e-10
    for t, (th, l, lw, z), (th1, l1, lw1, z1) in checks:
        rth, rl, rlw, _, inc, info = osmc.smc_step(th, l, lw, y, om, betas, t, cfg.step_sd,
                                                   cfg.n_moves, cfg.run_seed, cfg.ess_frac)
        assert info["resampled"] == (t == fired_at), t
        assert abs((z1 - z) - inc) <= 1e-10 * max(1.0, abs(inc))
        assert np.max(np.abs(lw1 - rlw)) <= 1e-12
        same = np.all(np.abs(th1 - rth) <= 1e-12, axis=0)
        flips = int(np.sum(~same))
        assert flips <= (0 if prec == "fp64" else cfg.N // 1000), (t, flips)
        assert rel_err(l1[same], rl[same]).max() <= tol_l
        print(f"{prec} step {t}: resampled={info['resampled']} flips={flips}")


def _full_state(s):
    s.stream.synchronize()
    st = s.stats.cpu().numpy()
    return dict(theta=s.theta.cpu().numpy().copy(), l=s.loglik.cpu().numpy().copy(),
                logw=s.logw.cpu().numpy().copy(), logZ=float(st[0]), resamples=int(st[2]),
                accepted=int(s.n_accept.cpu().item()))


def test_headline_fp32_run_replayed_by_oracle(smc, ctx):
    """The benchmark's FP32 run (N = 131072, n = 1000, 100 steps, 4 slices per
    tile) in replay mode.
    (1) The whole run as one 100-step chain in one graph replay, as timed.
    (2) The same run as alternating one-step and nine-step chains (one graph
        replay each), keeping the state before and after every step
        t = 10k + 1; its final population equals (1)'s and its evidence
        agrees to 1e-9.
    (3) The oracle takes each kept step from the GPU's state before it:
        - the GPU's FP32 log-likelihoods of all N particles are within 1e-6 of
          the oracle's FP64 values on the same parameters;
        - from the GPU's log-likelihoods the oracle gives the GPU's evidence
          increment (1e-10 relative), log-weights (1e-12) and resampling
          decision; on about 4200 sampled positions the moved particles equal
          the oracle's except FP32 near-tie accept flips (at most one per
          thousand decisions) and their log-likelihoods agree to 1e-6;
        - from the oracle's FP64 log-likelihoods the increments move by the
          FP32 likelihood error only: summed over the ten steps, the GPU's
          increments are within 1e-3 of the oracle's."""
    cfg = CONFIGS["gmm1d_k4_n1000_N131072"]
    y = make_data(cfg)
    betas = beta_schedule(cfg.T, cfg.schedule)
    from oracle.gmm import Model
    om = Model.equal_weights(cfg.k, cfg.d, cfg.sigma2)
    ctx.set_slices(4)
    try:
        announce("headline fp32: 100-step chain in one graph")
        a = _sampler(smc, ctx, cfg, y, betas, "fp32")
        a.run(graph=True, steps_per_graph=cfg.T)
        whole = _full_state(a)
        announce("headline fp32: chains of 1 and 9 steps with saved states")
        b = _sampler(smc, ctx, cfg, y, betas, "fp32")
        b.init()
        kept = []
        for k in range(cfg.T // 10):
            before = _full_state(b)
            b.step(graph=True, steps=1)
            kept.append((10 * k + 1, before, _full_state(b)))
            b.step(graph=True, steps=9)
        split = _full_state(b)
        ctx.check(b.stream)
    finally:
        ctx.set_slices(0)
    assert whole["resamples"] == split["resamples"] > 0
    assert whole["accepted"] == split["accepted"]
    assert np.array_equal(whole["theta"], split["theta"])
    assert np.array_equal(whole["l"], split["l"])
    assert abs(whole["logZ"] - split["logZ"]) <= 1e-9 * max(1.0, abs(whole["logZ"]))
    flips = decisions = 0
    drift = []
    for t, s0, s1 in kept:
        l_o = loglik_threads(s0["theta"], y, om)
        assert rel_err(s0["l"], l_o).max() <= 1e-6, t
        pos = replay_positions(cfg.N, 4096, seed=t)
        rth, rl, rlw, _, inc, info = osmc.smc_step_sampled(
            s0["theta"], s0["l"], s0["logw"], y, om, betas, t, cfg.step_sd, cfg.n_moves,
            cfg.run_seed, pos, cfg.ess_frac)
        inc_gpu = s1["logZ"] - s0["logZ"]
        assert info["resampled"] == (s1["resamples"] == s0["resamples"] + 1), t
        assert abs(inc_gpu - inc) <= 1e-10 * max(1.0, abs(inc)), t
        assert np.max(np.abs(s1["logw"] - rlw)) <= 1e-12, t
        same = np.all(np.abs(s1["theta"][:, pos] - rth) <= 1e-12, axis=0)
        flips += int(np.sum(~same))
        decisions += pos.size * cfg.n_moves
        assert rel_err(s1["l"][pos][same], rl[same]).max() <= 1e-6, t
        inc_fp64 = osmc.reweight(s0["logw"], l_o, betas[t] - betas[t - 1])[2]
        drift.append(inc_gpu - inc_fp64)
        print(f"step {t}: resampled={info['resampled']} increment {inc_gpu:.9f} "
              f"(oracle on FP64 l: {inc_fp64:.9f}) flips={int(np.sum(~same))}")
    assert flips <= max(3, decisions // 1000), flips
    assert abs(sum(drift)) <= 1e-3 and max(abs(x) for x in drift) <= 1e-4, drift
    print(f"summed increment error {sum(drift):.3e}; flips {flips} of {decisions}")


@pytest.mark.parametrize("slices,iters_per_graph,fused", [(0, 1, False), (24, 7, False),
                                                          (0, 7, True), (3, 25, True)])
def test_pt_matches_oracle(smc, ctx, slices, iters_per_graph, fused):
    """slices = 24 spreads each tile over 2 workgroups; 7 iterations per graph
    leave a ragged last graph (25 = 3 * 7 + 4); fused runs each graph's
    iterations in one single-workgroup launch."""
    announce(f"pt small fp64 slices={slices} iters_per_graph={iters_per_graph} fused={fused}")
    mu = np.array([-3.0, 0.0, 3.0, 6.0])
    y = make_mixture_data(300, mu, 0.55, seed=3)
    M, iters = 128, 25
    betas = pt_betas(M, 4)
    g = smc.Gmm.equal_weights(4, 1, 0.55)
    om = oracle_model(g)
    ctx.set_slices(slices)
    ctx.set_pt_single_workgroup(1 if fused else 0)
    try:
        s = smc.PTSampler(ctx, g, y, betas, 0.5, seed=103, parity_mode=0, wrap=False, prec="fp64",
                          fused_iterations=fused)
        r = s.run(iters, graph=True, iters_per_graph=iters_per_graph)
    finally:
        ctx.set_slices(0)
        ctx.set_pt_single_workgroup(0)
    ref = osmc.pt_run(y, om, betas, iters, 0.5, 103, parity_mode="alternate", wrap=False)
    assert r["it"] == iters
    assert r["swaps"] == ref["swaps"]
    assert r["accepted"] == ref["accepted"]
    assert np.max(np.abs(r["theta"] - ref["theta"])) <= 1e-9
    assert rel_err(r["l"], ref["l"]).max() <= 1e-10


@pytest.mark.parametrize("M,iters,iters_per_graph,parity_mode,wrap",
                         [(600, 15, 7, 0, False), (640, 16, 8, 1, True), (1001, 9, 9, 1, True)])
def test_pt_deferred_exchange_graphs_match_oracle(smc, ctx, M, iters, iters_per_graph,
                                                  parity_mode, wrap):
    """Populations past the single-workgroup form, one launch per iteration
    with the exchange deferred, captured in graphs of odd and even iteration
    counts (so the population ends in either buffer), in FP64 against the
    oracle's run."""
    announce(f"pt deferred M={M} iters={iters}/{iters_per_graph} parity={parity_mode} wrap={wrap}")
    mu = np.array([-3.0, 0.0, 3.0, 6.0])
    y = make_mixture_data(100, mu, 0.3025, seed=5)
    betas = pt_betas(M, 2)
    g = smc.Gmm.equal_weights(4, 1, 0.3025, prior="box", prior_a=-10.0, prior_b=10.0)
    om = oracle_model(g)
    ctx.set_slices(4)
    try:
        s = smc.PTSampler(ctx, g, y, betas, 1.0, seed=17, parity_mode=parity_mode, wrap=wrap,
                          prec="fp64")
        r = s.run(iters, graph=True, iters_per_graph=iters_per_graph)
    finally:
        ctx.set_slices(0)
    ref = osmc.pt_run(y, om, betas, iters, 1.0, 17,
                      parity_mode="random" if parity_mode else "alternate", wrap=wrap)
    assert r["it"] == iters
    assert r["swaps"] == ref["swaps"]
    assert r["accepted"] == ref["accepted"]
    assert np.max(np.abs(r["theta"] - ref["theta"])) <= 1e-9
    assert rel_err(r["l"], ref["l"]).max() <= 1e-10


@pytest.mark.parametrize("M,slices,fused", [(32, 0, False), (32, 40, False), (33, 24, False),
                                            (32, 0, True), (33, 5, True)])
def test_pt_paper_mode_random_parity_wrap(smc, ctx, M, slices, fused):
    """Random parity with the wrap pair; slices > 16 run the moves' decisions and
    the exchanges in one kernel (pairs, the wrap pair, and for odd M the
    unpaired chain 0)."""
    announce(f"pt paper mode M={M} slices={slices} fused={fused}")
    mu = np.array([-3.0, 0.0, 3.0, 6.0])
    y = make_mixture_data(100, mu, 0.3025, seed=1)
    iters = 15
    betas = pt_betas(M, 2)
    g = smc.Gmm.equal_weights(4, 1, 0.3025, prior="box", prior_a=-10.0, prior_b=10.0)
    om = oracle_model(g)
    ctx.set_slices(slices)
    try:
        s = smc.PTSampler(ctx, g, y, betas, 1.0, seed=7, parity_mode=1, wrap=True, prec="fp64",
                          fused_iterations=fused)
        r = s.run(iters, graph=False)
    finally:
        ctx.set_slices(0)
    ref = osmc.pt_run(y, om, betas, iters, 1.0, 7, parity_mode="random", wrap=True)
    assert r["swaps"] == ref["swaps"]
    assert r["accepted"] == ref["accepted"]
    if slices == 0 and not fused:
        # the beta = 1 chain recorded after every iteration, as the oracle records it
        s = smc.PTSampler(ctx, g, y, betas, 1.0, seed=7, parity_mode=1, wrap=True, prec="fp64",
                          record_chain=M - 1, record_iters=iters)
        rr = s.run(iters, graph=True, iters_per_graph=4)
        ref2 = osmc.pt_run(y, om, betas, iters, 1.0, 7, parity_mode="random", wrap=True,
                           record_chain=M - 1)
        assert np.max(np.abs(rr["chain"] - ref2["chain"])) <= 1e-9
    assert np.max(np.abs(r["theta"] - ref["theta"])) <= 1e-9


def _batch_inputs():
    rng = np.random.default_rng(44)
    specs = [(1000, 700), (40, 63), (1, 5), (333, 256), (100, 1), (5000, 130)]
    datas, Ns, seeds = [], [], []
    for r, (n, N) in enumerate(specs):
        mu = rng.uniform(-6, 9, size=4)
        datas.append(make_mixture_data(n, mu, 0.55, seed=900 + r))
        Ns.append(N)
        seeds.append(5000 + r)
    return datas, Ns, seeds


@pytest.mark.parametrize("graph,scheme", [(False, "systematic"), (True, "systematic"),
                                          (True, "multinomial")])
def test_batched_runs_match_oracle_fp64(smc, ctx, graph, scheme):
    """Every run of a batch equals the oracle's sampler run alone with its own seed."""
    announce(f"batched fp64 graph={graph} {scheme}")
    datas, Ns, seeds = _batch_inputs()
    betas = beta_schedule(12, "quadratic")
    g = smc.Gmm.equal_weights(4, 1, 0.55)
    om = oracle_model(g)
    b = smc.BatchSampler(ctx, g, datas, Ns, seeds, betas, 0.5, 1, ess_frac=0.5, prec="fp64",
                         scheme=scheme)
    try:
        r = b.run(graph=graph)
    finally:
        ctx.set_resampling("systematic")
    assert r["t"] == 13
    acc_total = 0
    for i in range(len(Ns)):
        ref = osmc.smc_run(datas[i], om, betas, Ns[i], 0.5, 1, seeds[i], ess_frac=0.5,
                           scheme=scheme)
        assert r["resamples"][i] == int(np.sum(ref["trace"]["resampled"])), i
        assert abs(r["logZ"][i] - ref["logZ"]) <= 1e-9 * max(1.0, abs(ref["logZ"])), i
        assert np.max(np.abs(r["theta"][i] - ref["theta"])) <= 1e-9, i
        assert rel_err(r["l"][i], ref["l"]).max() <= 1e-10, i
        acc_total += int(np.sum(ref["trace"]["accepted"]))
    assert r["accepted"] == acc_total


# launch tables of the batched move: the built-in rule, and one that gives
# short-data runs a single wave per tile and long-data runs two
BATCH_TABLES = {
    "built-in": [],
    "one-two": [dict(k=4, d=1, prec="any", kind="batch", slices=1, n_lo=1, n_hi=999,
                     N_lo=1, N_hi=1 << 30),
                dict(k=4, d=1, prec="any", kind="batch", slices=2, n_lo=1000, n_hi=1 << 30,
                     N_lo=1, N_hi=1 << 30)],
}


@pytest.mark.parametrize("table", sorted(BATCH_TABLES))
def test_batched_full_workload_sampled_runs(smc, ctx, table):
    """The benchmark's whole 256-run batch (n log-uniform in 1e2..1e5, N in
    1024..65536) advanced three graph-replayed FP64 steps, under two launch
    tables of the persistent move; the four cheapest runs and one with long
    data (N = 1024, n nearest 2e4), checked one by one, equal the oracle's runs
    alone over the same three steps."""
    from workloads.configs import BATCHED, batched_runs
    announce(f"batched full workload, sampled runs, table {table}")
    runs = batched_runs(256)
    datas = [make_mixture_data(x.n, x.true_means, BATCHED["sigma2"], x.data_seed) for x in runs]
    g = smc.Gmm.equal_weights(4, 1, BATCHED["sigma2"])
    om = oracle_model(g)
    betas = beta_schedule(BATCHED["T"], BATCHED["schedule"])
    ctx.set_launch_table(BATCH_TABLES[table])
    try:
        b = smc.BatchSampler(ctx, g, datas, [x.N for x in runs], [x.run_seed for x in runs],
                             betas, BATCHED["step_sd"], BATCHED["n_moves"],
                             ess_frac=BATCHED["ess_frac"], prec="fp64")
    finally:
        ctx.set_launch_table([])
    r = b.run(graph=True, steps=3)
    assert r["t"] == 4
    order = np.argsort([x.N * x.n for x in runs])
    long_data = min((x for x in runs if x.N == 1024), key=lambda x: abs(x.n - 20000)).index
    for i in list(order[:4]) + [long_data]:
        x = runs[i]
        ref = osmc.smc_run(datas[i], om, betas[:4], x.N, BATCHED["step_sd"], BATCHED["n_moves"],
                           x.run_seed, ess_frac=BATCHED["ess_frac"])
        assert r["resamples"][i] == int(np.sum(ref["trace"]["resampled"])), i
        assert abs(r["logZ"][i] - ref["logZ"]) <= 1e-9 * max(1.0, abs(ref["logZ"])), i
        assert np.max(np.abs(r["theta"][i] - ref["theta"])) <= 1e-9, i
        assert rel_err(r["l"][i], ref["l"]).max() <= 1e-10, i


def _batch_state(b):
    b.stream.synchronize()
    return dict(theta=b.theta.cpu().numpy().copy(), l=b.loglik.cpu().numpy().copy(),
                logw=b.logw.cpu().numpy().copy(),
                stats=b.stats.cpu().numpy().reshape(b.R, 4).copy())


def _run_view(b, st, r):
    """Run r's (theta [kd][N_r], l, logw, logZ, resamples) from a batch state."""
    kd, N, a = b.model.kd, b.Ns[r], int(b.p_off[r])
    return (st["theta"][kd * a:kd * (a + N)].reshape(kd, N), st["l"][a:a + N],
            st["logw"][a:a + N], float(st["stats"][r, 0]), int(st["stats"][r, 2]))


def _replay_batched(b, states, runs, datas, om, betas, max_evals):
    """Each listed run's steps taken by the oracle from the GPU's state before
    each step (replay mode); moves on all particles, or on sampled positions
    when the run is large. Returns (flips, decisions)."""
    flips = decisions = 0
    for r in runs:
        y = datas[r]
        N, n = b.Ns[r], b.ns[r]
        pos = np.arange(N) if N * n <= max_evals else replay_positions(N, 512, seed=r)
        th0, l0, _, _, _ = _run_view(b, states[0], r)
        assert rel_err(l0[pos], ogmm.loglik(th0[:, pos], y, om)).max() <= 1e-6, r
        for t in range(1, len(states)):
            th0, l0, lw0, z0, c0 = _run_view(b, states[t - 1], r)
            th1, l1, lw1, z1, c1 = _run_view(b, states[t], r)
            rth, rl, rlw, _, inc, info = osmc.smc_step_sampled(
                th0, l0, lw0, y, om, betas, t, b.step_sd, b.n_moves, b.seeds[r], pos,
                b.ess_frac)
            assert info["resampled"] == (c1 == c0 + 1), (r, t)
            assert abs((z1 - z0) - inc) <= 1e-10 * max(1.0, abs(inc)), (r, t)
            assert np.max(np.abs(lw1 - rlw)) <= 1e-12, (r, t)
            same = np.all(np.abs(th1[:, pos] - rth) <= 1e-12, axis=0)
            flips += int(np.sum(~same))
            decisions += pos.size * b.n_moves
            if same.any():
                assert rel_err(l1[pos][same], rl[same]).max() <= 1e-6, (r, t)
    return flips, decisions


def test_batched_fp32_runs_replayed_by_oracle(smc, ctx):
    """Six uneven FP32 runs with two moves per step, one graph replay per step:
    replaying the whole batch gives the same results, and every step of every
    run, taken by the oracle from the GPU's state before it, gives the GPU's
    evidence increment, log-weights and decision, and its population except
    FP32 near-tie accept flips (at most one per thousand decisions)."""
    announce("batched fp32 two moves, replay mode")
    datas, Ns, seeds = _batch_inputs()
    betas = beta_schedule(8, "linear")
    g = smc.Gmm.equal_weights(4, 1, 0.55)
    om = oracle_model(g)
    b = smc.BatchSampler(ctx, g, datas, Ns, seeds, betas, 0.5, 2, ess_frac=0.5, prec="fp32")
    r1 = b.run(graph=True)
    b.init()
    states = [_batch_state(b)]
    for _ in range(b.T):
        b.capture().launch()
        states.append(_batch_state(b))
    ctx.check(b.stream)
    assert np.array_equal(states[-1]["stats"][:, 0], r1["logZ"])
    flips, decisions = _replay_batched(b, states, range(b.R), datas, om, betas, 10 ** 9)
    assert flips <= max(3, decisions // 1000), (flips, decisions)
    print(f"batched fp32 flips {flips} of {decisions}")


def test_batched_full_workload_fp32_replayed_by_oracle(smc, ctx):
    """The benchmark's whole 256-run batch in FP32 (the benchmarked form),
    three graph-replayed steps with the state kept after each. The oracle
    replays seven runs step by step from the GPU's state: the four cheapest,
    one with long data (N = 1024, n nearest 2e4), the largest N with the
    shortest data and the largest N x n (moves on 512 sampled positions where
    N x n exceeds 2e7). Increments to 1e-10 relative, log-weights to 1e-12,
    decisions equal, flips at most one per thousand decisions, and the
    log-likelihoods of unflipped particles to 1e-6."""
    from workloads.configs import BATCHED, batched_runs
    announce("batched full workload fp32, replay mode")
    runs = batched_runs(256)
    datas = [make_mixture_data(x.n, x.true_means, BATCHED["sigma2"], x.data_seed) for x in runs]
    g = smc.Gmm.equal_weights(4, 1, BATCHED["sigma2"])
    om = oracle_model(g)
    betas = beta_schedule(BATCHED["T"], BATCHED["schedule"])
    b = smc.BatchSampler(ctx, g, datas, [x.N for x in runs], [x.run_seed for x in runs], betas,
                         BATCHED["step_sd"], BATCHED["n_moves"], ess_frac=BATCHED["ess_frac"],
                         prec="fp32")
    b.init()
    states = [_batch_state(b)]
    for _ in range(3):
        b.capture().launch()
        states.append(_batch_state(b))
    ctx.check(b.stream)
    order = list(np.argsort([x.N * x.n for x in runs]))
    long_data = min((x for x in runs if x.N == 1024), key=lambda x: abs(x.n - 20000)).index
    big_N = min((x for x in runs if x.N == 65536), key=lambda x: x.n).index
    picked = list(dict.fromkeys(order[:4] + [long_data, big_N, order[-1]]))
    flips, decisions = _replay_batched(b, states, picked, datas, om, betas, 2 * 10 ** 7)
    assert flips <= max(3, decisions // 1000), (flips, decisions)
    print(f"batched full workload fp32: runs {picked}, flips {flips} of {decisions}")
