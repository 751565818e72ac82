#!/usr/bin/env python3
"""Throughput of the tempered-SMC hot path on one MI355X.

A step is one whole tempering step of the SMC sampler (incremental reweight,
log-sum-exp normalisation, ESS, ESS-triggered systematic resampling, one
RW-MH move whose proposal log-likelihood is the mixture likelihood over all
observations) on the headline workload: 1-D k = 4 mixture, n = 1000
observations, N = 131072 particles, 100 quadratic tempering steps. The step
is device-driven (step index, temperature and resampling decision live in
device memory), so ten consecutive steps are captured in one hipGraph and
replayed; inputs are resident in HBM.

value = particle x datum log-likelihood evaluations per second over whole
steps (FP32 path). The same run times the plain FP64 GPU form and reports the
FP32/FP64 step-time ratio, the dominant kernel's roofline position (its
average launch time from HIP events on its own stream) and the FP64 CPU
oracle on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps 100] [--warmup 5]
"""

from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "gmm1d_k4_n1000_N131072"
OTHER_WORKLOADS = ("gmm1d_k4_n100_N1024", "pt_k4_n10000_M8192", "gmm8d_k8_n65536_N16384",
                   "batched_256runs", "probes", "paper_tables", "fsv_pf")

# The paper's running times on its GTX 280 in seconds (tables of running times
# in the SMC Sampler and Population-Based MCMC subsections): context for the
# paper-mode runs, not a target.
PAPER_GTX280_S = {
    "smc": {8192: 0.597, 16384: 1.114, 32768: 2.114, 65536: 4.270, 131072: 8.075,
            262144: 16.219},
    "pt": {8: 1.083, 32: 1.098, 128: 1.100, 512: 1.235, 2048: 1.427, 8192: 2.323,
           32768: 7.729, 131072: 28.349},
    # factor stochastic-volatility particle filter, T = 200 (Factor Stochastic Volatility)
    "fsv": {8192: 0.082, 16384: 0.144, 32768: 0.249, 65536: 0.465, 131072: 0.929},
}

# Issue-slot model of gfx950: 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz =
# 3.93e13 non-packed FP32 VALU lane-operations per second (one wave64 VALU
# instruction per SIMD every 4 cycles). The hardware exp2 (v_exp_f32) holds the
# VALU for two of those issue slots (counters: SQ_ACTIVE_INST_VALU -
# SQ_INSTS_VALU = SQ_INSTS_VALU_TRANS_F32), so the time bound of an evaluation
# charges each exp2 two slots and every other instruction one; `frac` is that
# bound over the measured time. The roofline also reports the fraction with
# exp2 charged one slot (a looser bound) and the counter-measured VALU-busy
# share. (The part clocks at about 2.47 GHz under this load, so a fraction
# against the nominal 2.4 GHz can pass 1.)
PEAK_LANE_OPS = 256 * 64 * 2.4e9
TRANS_SLOTS = 2.0
HBM_PEAK_GBS = 8000.0

# HBM traffic of the dominant kernel (the FP32 move at the headline shape, the
# standalone launches timed below) from two rocprofv3 --pmc runs of this same
# command: FETCH_SIZE and WRITE_SIZE in KiB per dispatch, averaged over those
# launches, each scaled by what the counter reads for a plain 256 MiB device
# copy (FETCH_SIZE reads half the copied bytes, WRITE_SIZE all of them). The
# figures belong to the kernel sources whose SHA-256 is recorded; after any
# change to them the traffic is reported as null until it is measured again.
MOVE_COUNTERS = {
    "sources_sha256": "c937fe5f0e5ec4ec3b5f99af64c4d1b7a994521e962a05889036e595eef654a4",
    # the launch shape the counters were taken at (data slices per 64-particle
    # tile, and so waves per launch); figures apply only to a timed move of that
    # shape. The standalone moves run from the population after `steps` timed
    # steps, whose acceptance rate sets the bytes written.
    "slices": 4, "waves": 8192, "steps": 20,
    "fetch_kib": 2726.4, "fetch_scale": 2.0,
    "write_kib": 1921.0, "write_scale": 1.0,
    "summary": "profiles/k_rwmh_fp32_gmm1d_k4_n1000_N131072_hbm_counters.txt",
    # SQ_ACTIVE_INST_VALU x 4 cycles / (1024 SIMDs x GRBM_GUI_ACTIVE / 8 XCDs) of the
    # same launches: the share of SIMD cycles the VALU pipeline was issuing
    # (profiles/k_rwmh_fp32_gmm1d_k4_n1000_N131072_valu_counters.txt)
    "valu_busy": 0.751,
}


# the files the move kernel is compiled from (with the compiler flags of build.py)
MOVE_SOURCES = ("gmm_kernels.hip", "gmm_common.hpp", "exchange.hpp", "internal.hpp",
                "philox.hpp", "wave.hpp", "dd.hpp", "cdf_search.hpp", "reduce.hpp",
                "../../include/smc.h")


def kernel_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_0905_2441_amd", "csrc")
    for name in MOVE_SOURCES:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    # and the compiler flags (the CXXFLAGS assignment of the build script)
    import re
    with open(os.path.join(ROOT, "paper_0905_2441_amd", "build.py")) as f:
        flags = re.search(r"^CXXFLAGS = \[.*?\]", f.read(), flags=re.S | re.M)
    h.update(flags.group(0).encode() if flags else b"?")
    return h.hexdigest()


def counters_apply(slices) -> bool:
    """Whether the recorded counters belong to the timed move: same kernel
    sources (and flags) and the same launch shape."""
    c = MOVE_COUNTERS
    return c["sources_sha256"] == kernel_sources_sha256() and slices == c["slices"]


def move_valu_busy(slices):
    """Counter-measured VALU-busy share of the dominant kernel, or None if the
    counters were taken on other kernel sources or another launch shape."""
    c = MOVE_COUNTERS
    return c["valu_busy"] if counters_apply(slices) else None


def move_traffic(slices, steps):
    """HBM bytes per launch of the dominant kernel, or None if the counters were
    taken on other kernel sources, another launch shape or after another number
    of steps (another population, so another acceptance rate)."""
    c = MOVE_COUNTERS
    if c["fetch_kib"] is None or not counters_apply(slices) or steps != c["steps"]:
        return None
    return 1024.0 * (c["fetch_kib"] * c["fetch_scale"] + c["write_kib"] * c["write_scale"])
STEPS_PER_GRAPH = 50    # tempering steps (filter steps, PT iterations) per hipGraph replay
# measured best groupings that differ from it: the headline's whole 100-step run
# in one replay (per step 90.1 us against 92.6 at 50 and 95.5 at 10 on one box);
# the small run's 25 us steps in replays of 10 (39-41 us per step at 50)
GRAPH_STEPS = {"gmm1d_k4_n1000_N131072": 100, "gmm1d_k4_n100_N1024": 10}
PT_ITERS_PER_GRAPH = 64  # population-MCMC iterations per replay in the paper's runs


def ops_per_eval(k: int, form: str = "pivot") -> float:
    """Algorithmic VALU issue slots of one particle x datum evaluation in an
    FP32 form for 1-D data (exp2 counted as TRANS_SLOTS slots):
    pivot (the form the samplers' data in ascending order take): per
    component other than the particle's pivot one FMA (its exponent offset,
    linear in the datum) and one exp2; per datum k-2 adds and one FMA into the
    running product: 2k - 2 VALU + k - 1 transcendental (12 slots for k = 4;
    9 with exp2 at one). The pivot's own terms come per window of 64 data from
    sums the wave shares, outside the per-datum count.
    direct (plain form, waves near the data): per component two FMAs and one
    exp2; per datum k-1 adds and the product update: 3k VALU + k
    transcendental (20 slots for k = 4).
    shifted (plain form, waves holding a particle far from the data): per
    component two FMAs, a shift subtract and the exp2; per datum the maximum
    (v_max3 folds two comparisons), k-1 adds, the product update and the block
    sum of maxima: 4k + ceil((k-1)/2) + 1 VALU + k transcendental (27 slots for
    k = 4)."""
    if form == "pivot":
        return 2.0 * k - 2.0 + TRANS_SLOTS * (k - 1)
    if form == "direct":
        return 3.0 * k + TRANS_SLOTS * k
    return 4.0 * k + (k // 2) + 1.0 + TRANS_SLOTS * k


def trans_per_eval(k: int, form: str = "pivot") -> int:
    """exp2 instructions per evaluation in the form of ops_per_eval."""
    return k - 1 if form == "pivot" else k


def form_shares(fc, pairs):
    """Shares of (observation, tile) pairs by FP32 form from the device form
    counters, and the pivot form's mean number of other components evaluated
    per pair (it leaves out those below 2^-25 over a window for the whole
    wave)."""
    piv, sh = fc["pivot"] / pairs, fc["shifted"] / pairs
    return {"pivot": piv, "direct": max(0.0, 1.0 - piv - sh), "shifted": sh,
            "pivot_terms_mean": fc["pivot_terms"] / fc["pivot"] if fc["pivot"] else 0.0}


def ops_mix(k: int, forms, trans: float = TRANS_SLOTS) -> float:
    """Algorithmic issue slots per evaluation for a measured mix of forms: the
    pivot form at its measured mean of m other components (per datum m FMAs,
    m exp2, m - 1 adds and one FMA into the product: (2 + trans) m), the plain
    direct and shifted forms as in ops_per_eval."""
    def plain(form):
        return ops_per_eval(k, form) - (TRANS_SLOTS - trans) * trans_per_eval(k, form)
    return (forms["pivot"] * (2.0 + trans) * forms["pivot_terms_mean"]
            + forms["direct"] * plain("direct") + forms["shifted"] * plain("shifted"))


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(cfg, y, betas, budget_s=12.0):
    """The FP64 oracle on a bounded sample: whole tempering steps of the same
    workload (same n, data, schedule) on fewer particles, timed on host cores."""
    from oracle import gmm as ogmm
    from oracle import smc as osmc
    from oracle.gmm import Model
    import numpy as np
    om = Model.equal_weights(cfg.k, cfg.d, cfg.sigma2, prior=cfg.prior, prior_a=cfg.prior_a,
                             prior_b=cfg.prior_b)
    Ns = 4096
    theta = osmc.prior_init(om, Ns, cfg.run_seed)
    l = ogmm.loglik(theta, y, om)
    logw = np.zeros(Ns)
    t = 1
    steps = 0
    t0 = time.perf_counter()
    while True:
        theta, l, logw, _, _, _ = osmc.smc_step(theta, l, logw, y, om, betas, t, cfg.step_sd,
                                                cfg.n_moves, cfg.run_seed, cfg.ess_frac)
        steps += 1
        t = min(t + 1, cfg.T)
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    evals = steps * Ns * cfg.n * cfg.n_moves
    cpu = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {
        "value": evals / dt,
        "unit": "evals/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"{steps} whole tempering steps (reweight, ESS, resampling, RW-MH move) "
                   f"of the {cfg.name} workload on {Ns} particles (n = {cfg.n}), {dt:.1f} s, "
                   f"NumPy FP64 single-threaded on {cpu}; "
                   f"{len(os.sched_getaffinity(0))} host cores visible"),
        "ms_per_step_scaled_to_N": dt / steps * 1e3 * cfg.N / Ns,
    }


# ---------------------------------------------------------------------------
# The oracle leg: the FP64 CPU oracle timed on a bounded sample (cpu_baseline)
# and the error of the measured GPU results against it (oracle_error). This is
# the only part of the benchmark that runs the oracle; --no-cpu-baseline skips it.

LOGLIK_SAMPLE = 512         # particles whose log-likelihood the oracle recomputes
REPLAY_SAMPLE = 4096        # positions whose moves a replayed step checks


def _oracle_model(k, d, sigma2, prior="gauss", prior_a=0.0, prior_b=10.0):
    from oracle.gmm import Model
    return Model.equal_weights(k, d, sigma2, prior=prior, prior_a=prior_a, prior_b=prior_b)


def _positions(N, count, seed):
    import numpy as np
    if N <= count:
        return np.arange(N)
    return np.sort(np.random.default_rng(seed).choice(N, size=count, replace=False))


def _oracle_loglik(theta, y, om, workers=8):
    """The oracle's log-likelihood of every column, columns split over threads."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    from oracle import gmm as ogmm
    parts = np.array_split(np.arange(theta.shape[1]), workers)
    with ThreadPoolExecutor(max_workers=workers) as ex:
        return np.concatenate(list(ex.map(lambda ix: ogmm.loglik(theta[:, ix], y, om), parts)))


def loglik_error(theta, l, y, om, count=LOGLIK_SAMPLE, seed=0):
    """Largest relative error of the GPU log-likelihoods `l` of parameters
    `theta` against the oracle's, over `count` sampled particles."""
    import numpy as np
    from oracle import gmm as ogmm
    pos = _positions(theta.shape[1], count, seed)
    ref = ogmm.loglik(theta[:, pos], y, om)
    return float(np.max(np.abs(l[pos] - ref) / np.abs(ref)))


def _sampler_state(s):
    s.stream.synchronize()
    st = s.stats.cpu().numpy()
    return dict(theta=s.theta.cpu().numpy(), l=s.loglik.cpu().numpy(), logw=s.logw.cpu().numpy(),
                logZ=float(st[0]), resamples=int(st[2]))


def replay_step(t, s0, s1, y, om, betas, step_sd, n_moves, seed, ess_frac, count, fp64_l):
    """Tempering step t taken by the oracle from the GPU's state s0 and compared
    with the GPU's result s1 (replay mode): the evidence increment, log-weights
    and decision over the whole population, the moves on `count` sampled
    positions (FP32 near-tie accept flips counted), and with fp64_l the
    increment from the oracle's FP64 log-likelihoods of the same particles."""
    import numpy as np
    from oracle import smc as osmc
    pos = _positions(s0["l"].size, count, seed=t)
    rth, rl, rlw, _, inc, info = osmc.smc_step_sampled(
        s0["theta"], s0["l"], s0["logw"], y, om, betas, t, step_sd, n_moves, seed, pos, ess_frac)
    inc_gpu = s1["logZ"] - s0["logZ"]
    same = np.all(np.abs(s1["theta"][:, pos] - rth) <= 1e-12, axis=0)
    out = {"t": t, "resampled": bool(info["resampled"]),
           "decision_equal": bool(info["resampled"] == (s1["resamples"] > s0["resamples"])),
           "logZ_increment": inc_gpu,
           "logZ_increment_abs_err": abs(inc_gpu - inc),
           "logw_max_abs_err": float(np.max(np.abs(s1["logw"] - rlw))),
           "flips": int(np.sum(~same)), "decisions": int(pos.size * n_moves),
           "moved_loglik_max_rel_err": float(np.max(np.abs(s1["l"][pos][same] - rl[same])
                                                    / np.abs(rl[same]))) if same.any() else None}
    if fp64_l:
        l_o = _oracle_loglik(s0["theta"], y, om)
        out["loglik_all_max_rel_err"] = float(np.max(np.abs(s0["l"] - l_o) / np.abs(l_o)))
        inc_o = osmc.reweight(s0["logw"], l_o, betas[t] - betas[t - 1])[2]
        out["logZ_increment_abs_err_fp64_l"] = abs(inc_gpu - inc_o)
    return out


def headline_oracle_error(smc, ctx, cfg, g, y, betas, runs):
    """oracle_error of the headline line: the final populations of the timed
    runs (log-likelihoods of sampled particles against the oracle's) and two
    steps of a fresh FP32 run replayed by the oracle from the GPU's state: the
    first step that resamples and the step at t = T/2."""
    om = _oracle_model(cfg.k, cfg.d, cfg.sigma2, cfg.prior, cfg.prior_a, cfg.prior_b)
    out = {"against": "FP64 CPU oracle (oracle/), same inputs and random streams",
           "final_population_loglik_max_rel_err": {
               p: loglik_error(r["theta"], r["l"], y, om) for p, r in runs.items()},
           "loglik_sample": LOGLIK_SAMPLE}
    s = smc.SMCSampler(ctx, g, y, cfg.N, betas, cfg.step_sd, cfg.n_moves, cfg.run_seed,
                       ess_frac=cfg.ess_frac, prec="fp32")
    s.init()
    replays = []
    before, done, mid = _sampler_state(s), 0, cfg.T // 2
    while done < mid - 1:
        s.step(graph=False)
        done += 1
        after = _sampler_state(s)
        if after["resamples"] > before["resamples"]:
            replays.append(replay_step(done, before, after, y, om, betas, cfg.step_sd,
                                       cfg.n_moves, cfg.run_seed, cfg.ess_frac, REPLAY_SAMPLE,
                                       True))
            break
        before = after
    if mid - 1 - done > 0:
        s.advance(mid - 1 - done, graph=True, steps_per_graph=cfg.T)
    before = _sampler_state(s)
    s.step(graph=False)
    replays.append(replay_step(mid, before, _sampler_state(s), y, om, betas, cfg.step_sd,
                               cfg.n_moves, cfg.run_seed, cfg.ess_frac, REPLAY_SAMPLE, True))
    ctx.check(s.stream)
    out["replayed_steps_fp32"] = replays
    out["bounds"] = {"loglik_rel": 1e-6, "logZ_abs": 1e-3, "flips_per_decision": 1e-3}
    return out


def small_run_oracle_error(smc, ctx, cfg, g, y, betas, prec):
    """The oracle-sized run in full: a fresh GPU run of all T steps (ten steps
    per graph replay) against the oracle's run with the same seeds."""
    import numpy as np
    from oracle import smc as osmc
    om = _oracle_model(cfg.k, cfg.d, cfg.sigma2, cfg.prior, cfg.prior_a, cfg.prior_b)
    s = smc.SMCSampler(ctx, g, y, cfg.N, betas, cfg.step_sd, cfg.n_moves, cfg.run_seed,
                       ess_frac=cfg.ess_frac, prec=prec)
    r = s.run(graph=True, steps_per_graph=10)
    ref = osmc.smc_run(y, om, betas, cfg.N, cfg.step_sd, cfg.n_moves, cfg.run_seed,
                       ess_frac=cfg.ess_frac)
    return {"against": "the oracle's whole run (same seeds)",
            "logZ_abs_err": abs(r["logZ"] - ref["logZ"]),
            "theta_max_abs_err": float(np.max(np.abs(r["theta"] - ref["theta"]))),
            "loglik_max_rel_err": float(np.max(np.abs(r["l"] - ref["l"]) / np.abs(ref["l"]))),
            "W_max_abs_err": float(np.max(np.abs(r["W"] - ref["W"]))),
            "resamples": [r["resamples"], int(np.sum(ref["trace"]["resampled"]))],
            "accepted": [r["accepted"], int(np.sum(ref["trace"]["accepted"]))]}


def pt_oracle_error(smc, ctx, cfg, g, y, prec, final, pairs=40, it=10):
    """Population MCMC: the timed run's final chains (log-likelihoods of sampled
    chains against the oracle's) and iteration `it` of a fresh run replayed by
    the oracle from the GPU's state on sampled pairs of its partition (both
    chains' moves, then the pair's exchange: exact for a sample of pairs)."""
    import numpy as np
    from oracle import smc as osmc
    from workloads import pt_betas
    om = _oracle_model(cfg.k, cfg.d, cfg.sigma2, cfg.prior, cfg.prior_a, cfg.prior_b)
    betas = pt_betas(cfg.N, 4)
    s = smc.PTSampler(ctx, g, y, betas, cfg.step_sd, cfg.run_seed, parity_mode=0, wrap=False,
                      prec=prec)
    s.init()
    s.advance(it, graph=True, iters_per_graph=it)
    r0 = s.results()
    s.advance(1, graph=False)
    r1 = s.results()
    ctx.check(s.stream)
    all_pairs = osmc.exchange_pairs(cfg.N, it & 1, False)
    rng = np.random.default_rng(it)
    pick = [all_pairs[0], all_pairs[-1]] + [all_pairs[i] for i in
                                            rng.choice(len(all_pairs), pairs, replace=False)]
    th, ll, chains = osmc.pt_iteration_pairs(r0["theta"], r0["l"], y, om, betas, it,
                                             cfg.step_sd, cfg.run_seed, pick)
    same = np.all(np.abs(r1["theta"][:, chains] - th) <= 1e-12, axis=0)
    return {"against": "FP64 CPU oracle (oracle/), same inputs and random streams",
            "final_population_loglik_max_rel_err": loglik_error(final["theta"], final["l"], y,
                                                                om),
            "loglik_sample": LOGLIK_SAMPLE,
            "replayed_iteration": {
                "it": it, "chains": int(chains.size), "flips": int(np.sum(~same)),
                "loglik_max_rel_err": float(np.max(np.abs(r1["l"][chains][same] - ll[same])
                                                   / np.abs(ll[same])))}}


def ddim_oracle_error(y, cfg, res, count=128):
    """d-dimensional mixture: each precision's final population (its own
    log-likelihoods) against the oracle on `count` sampled particles."""
    import numpy as np
    om = _oracle_model(cfg.k, cfg.d, cfg.sigma2, cfg.prior, cfg.prior_a, cfg.prior_b)
    out = {"against": "FP64 CPU oracle (oracle/), same inputs", "loglik_sample": count,
           "final_population_loglik_max_rel_err": {}}
    for p, r in res.items():
        pos = _positions(r["theta"].shape[1], count, seed=1)
        ref = _oracle_loglik(r["theta"][:, pos], y, om)
        out["final_population_loglik_max_rel_err"][p] = float(
            np.max(np.abs(r["l"][pos] - ref) / np.abs(ref)))
    return out


def batched_oracle_error(b, datas, betas, final, replay_state, replay_runs, per_run=64):
    """Batched runs: the timed final populations (sampled particles of every
    eighth run against the oracle) and one further step replayed by the oracle
    from the GPU's state for a few runs (moves on sampled positions)."""
    import numpy as np
    from oracle import smc as osmc
    om = _oracle_model(b.model.k, b.model.d, b.model.sigma2)
    kd = b.model.kd
    worst = 0.0
    for r in range(0, b.R, 8):
        a, N = int(b.p_off[r]), b.Ns[r]
        th = final["theta"][kd * a:kd * (a + N)].reshape(kd, N)
        worst = max(worst, loglik_error(th, final["l"][a:a + N], datas[r], om, per_run, seed=r))
    t, s0, s1 = replay_state
    steps = []
    for r in replay_runs:
        a, N = int(b.p_off[r]), b.Ns[r]
        view = lambda st: dict(theta=st["theta"][kd * a:kd * (a + N)].reshape(kd, N),
                               l=st["l"][a:a + N], logw=st["logw"][a:a + N],
                               logZ=float(st["stats"][r, 0]), resamples=int(st["stats"][r, 2]))
        rep = replay_step(t, view(s0), view(s1), datas[r], om, betas, b.step_sd, b.n_moves,
                          b.seeds[r], b.ess_frac, 256, False)
        rep["run"] = int(r)
        steps.append(rep)
    return {"against": "FP64 CPU oracle (oracle/), same inputs and random streams",
            "final_population_loglik_max_rel_err": worst,
            "loglik_sample": f"{per_run} particles of each of {len(range(0, b.R, 8))} runs",
            "replayed_step": steps}


def time_pt(smc, torch, ctx, cfg, g, y, prec, steps, warmup):
    """Population-MCMC iterations (one RW-MH move per chain, then exchanges),
    STEPS_PER_GRAPH iterations per hipGraph replay."""
    from workloads import pt_betas
    betas = pt_betas(cfg.N, 4)
    s = smc.PTSampler(ctx, g, y, betas, cfg.step_sd, cfg.run_seed, parity_mode=0, wrap=False,
                      prec=prec)
    u = min(STEPS_PER_GRAPH, steps)
    s.init()
    s.advance(warmup, graph=True, iters_per_graph=u)
    s.init()
    s.advance(steps, graph=True, iters_per_graph=u)    # the timed sequence's graphs captured
    s.stream.synchronize()
    s.init()
    s.stream.synchronize()
    t0 = time.perf_counter()
    s.advance(steps, graph=True, iters_per_graph=u)
    s.stream.synchronize()
    t1 = time.perf_counter()
    ctx.check(s.stream)
    r = s.results()
    return dict(ms_per_step=(t1 - t0) * 1e3 / steps, swaps=r["swaps"], accepted=r["accepted"],
                theta=r["theta"], l=r["l"])


def tune(ctx, cfg, precs, no_tune, fixed=None):
    """Pick the launch shape (data slices per 64-particle tile) of each precision
    with the package's autotuner (timed moves of this exact shape) and install
    it in the context's launch table; {prec: {"slices", "ms_per_move"}}.
    fixed = {prec: slices} installs those shapes instead of tuning them."""
    fixed = fixed or {}
    out = {}
    rules = []
    for p in precs:
        if p in fixed:
            rules.append(dict(k=cfg.k, d=cfg.d, prec=p, slices=fixed[p], n_lo=cfg.n, n_hi=cfg.n,
                              N_lo=cfg.N, N_hi=cfg.N))
            out[p] = {"slices": fixed[p], "chosen": "fixed"}
    tuned = [p for p in precs if p not in fixed]
    if no_tune:
        out.update({p: {"slices": "built-in"} for p in tuned})
    elif tuned:
        from paper_0905_2441_amd import autotune
        got = autotune.make_rules(ctx, [(cfg.k, cfg.d, cfg.n, cfg.N, p) for p in tuned],
                                  reps=10, exact=True, log=log)
        rules += got
        out.update({r["prec"]: {"slices": r["slices"], "ms_per_move": r["ms"][str(r["slices"])],
                                "ms_by_slices": r["ms"]} for r in got})
    ctx.set_launch_table(rules)
    return out


def moves_of_steps(smc, torch, ctx, cfg, g, s, betas, prec, steps):
    """Average time (ms) of the moves of the timed steps on their own: the run is
    taken again from the prior one step at a time, each step's input population
    is copied before the step, and then the step's move (same temperature and
    random streams) is launched on every copy back to back between two HIP
    events on the sampler's stream. A step that resampled moved its ancestors
    rather than this copy, at the same cost per particle."""
    s.init()
    copies = []
    for t in range(1, steps + 1):
        with torch.cuda.stream(s.stream):
            copies.append((min(t, cfg.T), s.theta.clone(), s.loglik.clone()))
        s.step(graph=False)
    s.stream.synchronize()

    def move(c):
        t, th, l = c
        smc.smc_rwmh_move(ctx, g, s.y, th, l, float(betas[t]), cfg.step_sd, cfg.run_seed, t, 0,
                          prec, stream=s.stream)

    move(tuple(x.clone() if hasattr(x, "clone") else x for x in copies[0]))   # warm, untimed
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s.stream)
    for c in copies:
        move(c)
    e1.record(s.stream)
    e1.synchronize()
    ctx.check(s.stream)
    del copies
    return e0.elapsed_time(e1) / steps


def time_precision(smc, torch, ctx, cfg, g, y, betas, prec, steps, warmup):
    s = smc.SMCSampler(ctx, g, y, cfg.N, betas, cfg.step_sd, cfg.n_moves, cfg.run_seed,
                       ess_frac=cfg.ess_frac, prec=prec)
    u = min(STEPS_PER_GRAPH, steps)
    s.init()
    s.advance(warmup, graph=True, steps_per_graph=u)
    s.init()
    s.advance(steps, graph=True, steps_per_graph=u)    # the timed sequence's graphs captured
    s.stream.synchronize()
    s.init()                               # a fresh run from the prior for the timed steps
    s.stream.synchronize()
    ctx.fp32_form_counts(reset=True)
    t0 = time.perf_counter()
    s.advance(steps, graph=True, steps_per_graph=u)
    s.stream.synchronize()
    t1 = time.perf_counter()
    ctx.check(s.stream)
    # the timed steps' moves: (observation, tile) pairs in the shifted form
    step_pairs = steps * cfg.n_moves * ((cfg.N + 63) // 64) * cfg.n
    forms_steps = form_shares(ctx.fp32_form_counts(reset=True), step_pairs)
    res = s.results()          # the timed run's final population (before the kernel timing)
    ms_step = (t1 - t0) * 1e3 / steps
    # the dominant kernel alone: the RW-MH move (proposal + likelihood + accept)
    # launched back to back, timed with HIP events recorded on the stream it
    # runs on (an event pair around every launch would add its own overhead)
    reps = max(10, steps)
    acc = torch.zeros(1, dtype=torch.int64, device="cuda")
    ctx.fp32_form_counts(reset=True)
    kern_ms = time_launches(torch, s.stream, lambda i: smc.smc_rwmh_move(
        ctx, g, s.y, s.theta, s.loglik, 1.0, cfg.step_sd, cfg.run_seed, cfg.T + 1 + i, 0, prec,
        n_accept=acc, stream=s.stream), reps)
    ctx.check(s.stream)
    accept_rate = acc.item() / ((reps + 1) * cfg.N)
    forms = None
    if prec == "fp32":
        # the (observation, tile) pairs of the reps + 1 launches (one untimed)
        pairs = (reps + 1) * ((cfg.N + 63) // 64) * cfg.n
        forms = form_shares(ctx.fp32_form_counts(reset=True), pairs)
    move_steps_ms = moves_of_steps(smc, torch, ctx, cfg, g, s, betas, prec, steps)
    return dict(ms_per_step=ms_step, kernel_ms=kern_ms, forms=forms,
                accept_rate=accept_rate, move_steps_ms=move_steps_ms,
                forms_steps=forms_steps if prec == "fp32" else None,
                resamples=res["resamples"],
                accepted=res["accepted"], logZ=res["logZ"], theta=res["theta"], l=res["l"],
                t=res["t"])


def main():
    global STEPS_PER_GRAPH
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle leg (CPU baseline and the error against the oracle)")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--steps-per-graph", type=int, default=None,
                    help="tempering steps (filter steps, PT iterations) per hipGraph replay "
                         f"(default: {GRAPH_STEPS} by workload, else {STEPS_PER_GRAPH})")
    ap.add_argument("--no-tune", action="store_true",
                    help="use the built-in launch shape instead of autotuning it first")
    ap.add_argument("--slices", type=int, default=None,
                    help="fix the FP32 move's data slices per tile (headline) instead of tuning")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a device copy of known size (HBM counter calibration)")
    ap.add_argument("--workload", default=WORKLOAD, choices=(WORKLOAD,) + OTHER_WORKLOADS,
                    help="the headline workload (default) or another measured configuration")
    args = ap.parse_args()
    STEPS_PER_GRAPH = max(1, int(args.steps_per_graph if args.steps_per_graph is not None
                                 else GRAPH_STEPS.get(args.workload, STEPS_PER_GRAPH)))
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs as a single process on one GPU", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_0905_2441_amd as smc
    from workloads import CONFIGS, beta_schedule, make_data

    if args.copy_calibration:
        return copy_calibration()
    if args.workload != WORKLOAD:
        return other_workload(args)
    cfg = CONFIGS[WORKLOAD]
    y = make_data(cfg)
    betas = beta_schedule(cfg.T, cfg.schedule)
    torch.cuda.set_device(0)
    ctx = smc.Context(0)
    g = smc.Gmm.equal_weights(cfg.k, cfg.d, cfg.sigma2, prior=cfg.prior, prior_a=cfg.prior_a,
                              prior_b=cfg.prior_b)
    evals_per_step = cfg.N * cfg.n * cfg.n_moves
    launch = tune(ctx, cfg, ["fp32"] + ([] if args.no_fp64 else ["fp64"]), args.no_tune,
                  fixed={"fp32": args.slices} if args.slices else None)
    slices32 = launch["fp32"]["slices"]

    log(f"[bench] {WORKLOAD}: fp32 {args.steps} steps after {args.warmup} warm-up")
    r32 = time_precision(smc, torch, ctx, cfg, g, y, betas, "fp32", args.steps, args.warmup)
    log(f"[bench] fp32 {r32['ms_per_step']:.4f} ms/step, move kernel {r32['kernel_ms']:.4f} ms")
    r64 = None
    if not args.no_fp64:
        r64 = time_precision(smc, torch, ctx, cfg, g, y, betas, "fp64", args.steps, args.warmup)
        log(f"[bench] fp64 {r64['ms_per_step']:.4f} ms/step, move kernel {r64['kernel_ms']:.4f} ms")

    kern_evals = evals_per_step / (r32["kernel_ms"] * 1e-3)
    ops = ops_mix(cfg.k, r32["forms"])
    achieved = kern_evals * ops
    roofline = {
        "bound": "alu",
        "achieved": achieved / 1e12,
        "peak": PEAK_LANE_OPS / 1e12,
        "unit": "Tlane-op/s",
        "frac": achieved / PEAK_LANE_OPS,
        "traffic": move_traffic(slices32, args.steps),
        # read theta, l (40 B) per particle, write theta, l (40 B) per accepted one
        "traffic_algorithmic": cfg.N * 40.0 * (1.0 + r32["accept_rate"]),
        "traffic_unit": "bytes per launch",
        "kernel": "k_rwmh<4,1,FP32> (proposal + likelihood + accept)",
        # issue slots per evaluation at the timed launches' measured form mix
        # (device form counters: pivot form at its mean number of other
        # components, exp2 at two slots)
        "ops_per_eval": ops,
        "forms": r32["forms"],
        "forms_timed_steps": r32["forms_steps"],
        # the same launches against the pivot form with all k - 1 other
        # components (12 slots for k = 4), and with exp2 charged one slot
        "frac_dense_pivot": kern_evals * ops_per_eval(cfg.k) / PEAK_LANE_OPS,
        "frac_exp_one_slot": kern_evals * ops_mix(cfg.k, r32["forms"], 1.0) / PEAK_LANE_OPS,
        "valu_busy_measured": move_valu_busy(slices32),
        "counters": {"slices": MOVE_COUNTERS["slices"], "waves": MOVE_COUNTERS["waves"],
                     "apply_to_timed_shape": counters_apply(slices32)},
        "kernel_ms": r32["kernel_ms"],
        "kernel_evals_per_s": kern_evals,
        "accept_rate": r32["accept_rate"],
        "launch_slices": slices32,
    }
    cpu = oracle_error = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        cpu = cpu_baseline(cfg, y, betas)
        log(f"[bench] oracle {cpu['value']:.3e} evals/s")
        log("[bench] error of the measured runs against the oracle ...")
        oracle_error = headline_oracle_error(
            smc, ctx, cfg, g, y, betas, {"fp32": r32, **({"fp64": r64} if r64 else {})})
        log(f"[bench] oracle error: {json.dumps(oracle_error)}")

    value = evals_per_step / (r32["ms_per_step"] * 1e-3)
    out = {
        "metric": "particle×datum loglik evals/s; ms per SMC tempering step, FP32/batched vs FP64",
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "k": cfg.k, "d": cfg.d, "n": cfg.n, "N": cfg.N,
                   "T": cfg.T, "schedule": "(t/T)^2", "moves_per_step": cfg.n_moves,
                   "ess_threshold": "N/2", "graph": f"{min(STEPS_PER_GRAPH, args.steps)} tempering steps per hipGraph replay",
                   "launch": launch},
        "fp64_ms_per_step": r64["ms_per_step"] if r64 else None,
        "fp32_over_fp64_speedup": (r64["ms_per_step"] / r32["ms_per_step"]) if r64 else None,
        "fp64_move_kernel_ms": r64["kernel_ms"] if r64 else None,
        # the timed steps' moves launched alone on each step's input population,
        # and what the step spends besides (k_step_mid, the chain's first
        # reweight pass, launch gaps)
        "step_split": {"ms_per_step": r32["ms_per_step"],
                       "move_ms": r32["move_steps_ms"],
                       "other_ms": r32["ms_per_step"] - r32["move_steps_ms"],
                       "other_share": 1.0 - r32["move_steps_ms"] / r32["ms_per_step"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "oracle_error": oracle_error,
    }
    print(json.dumps(out), flush=True)


def time_batched(smc, torch, ctx, prec, steps, warmup, R=256, keep_state=False,
                 tune_batch=True):
    """256 independent 1-D k = 4 runs (n log-uniform in [100, 1e5], N in
    {1024, ..., 65536}) advanced by one graph-replayed batched step."""
    from workloads import beta_schedule, make_mixture_data
    from workloads.configs import BATCHED, batched_runs
    runs = batched_runs(R)
    datas = [make_mixture_data(r.n, r.true_means, BATCHED["sigma2"], r.data_seed) for r in runs]
    g = smc.Gmm.equal_weights(4, 1, BATCHED["sigma2"])
    betas = beta_schedule(BATCHED["T"], BATCHED["schedule"])
    table = None
    if tune_batch:
        # per range of n, the waves per tile of the persistent move (untimed)
        from paper_0905_2441_amd import autotune
        table = autotune.tune_batched(ctx, g, datas, [r.N for r in runs],
                                      [r.run_seed for r in runs], betas, BATCHED["step_sd"],
                                      BATCHED["n_moves"], BATCHED["ess_frac"], prec, log=log)
        ctx.set_launch_table(table)
    b = smc.BatchSampler(ctx, g, datas, [r.N for r in runs], [r.run_seed for r in runs], betas,
                         BATCHED["step_sd"], BATCHED["n_moves"], ess_frac=BATCHED["ess_frac"],
                         prec=prec)
    b.init()
    graph = b.capture()
    for _ in range(warmup):
        graph.launch()
    b.stream.synchronize()
    b.init()
    b.stream.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        graph.launch()
    b.stream.synchronize()
    t1 = time.perf_counter()
    ctx.check(b.stream)
    evals = sum(r.N * r.n for r in runs) * BATCHED["n_moves"]
    out = dict(ms_per_step=(t1 - t0) * 1e3 / steps, evals_per_step=evals, R=R,
               N_total=sum(r.N for r in runs), n_total=sum(r.n for r in runs),
               launch_table=table)
    if keep_state:
        # the timed run's final state, then one more (untimed) step with the
        # states around it, for the oracle leg
        def state():
            b.stream.synchronize()
            return dict(theta=b.theta.cpu().numpy(), l=b.loglik.cpu().numpy(),
                        logw=b.logw.cpu().numpy(),
                        stats=b.stats.cpu().numpy().reshape(b.R, 4).copy())
        t = min(int(b.t.cpu().item()), b.T)
        s0 = state()
        graph.launch()
        out.update(sampler=b, datas=datas, betas=betas, final=s0, replay=(t, s0, state()))
        ctx.check(b.stream)
    return out


def copy_calibration(nbytes=1 << 28, reps=4):
    """A plain device-to-device copy of `nbytes` (read nbytes, write nbytes), the
    reference for scaling the HBM byte counters of a profiled run."""
    import torch
    torch.cuda.set_device(0)
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "reps": reps}), flush=True)


def time_launches(torch, stream, fn, reps):
    """Average device time (ms) of fn(i), i = 0..reps-1, enqueued back to back
    on `stream` between two HIP events recorded on that stream (after one
    untimed call)."""
    fn(0)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(reps):
        fn(i)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def probes(smc, torch, ctx, reps):
    """Roofline probes away from launch latency: the FP32 likelihood at
    N = 2^20, n = 4096 (issue-slot bound), and the reweight (+ W) and the
    systematic resampling with gather at N = 2^17, 2^20, 2^24 with log-normal
    weights (sigma = 3) (HBM bound, algorithmic bytes 40 and 100 per particle
    at k*d = 4)."""
    import numpy as np
    from workloads import lognormal_logw, make_mixture_data, theta_prior_draws
    s = torch.cuda.Stream()
    out = {}
    g = smc.Gmm.equal_weights(4, 1, 0.55)
    N, n = 1 << 20, 4096
    with torch.cuda.stream(s):
        y = torch.as_tensor(make_mixture_data(n, np.array([-3.0, 0.0, 3.0, 6.0]), 0.55, 7)).cuda()
        smc.smc_sort_data(y, stream=s)
        th = torch.as_tensor(theta_prior_draws(N, 4, 1, seed=8)).cuda()
        l = torch.empty(N, dtype=torch.float64, device="cuda")
    ms = time_launches(torch, s, lambda i: smc.smc_loglik(ctx, g, y, th, "fp32", out=l, stream=s),
                       reps)
    evals = N * n / (ms * 1e-3)
    out["loglik_fp32_N1048576_n4096"] = {
        "us": ms * 1e3, "evals_per_s": evals,
        "form": "pivot (prior draws, far from the data; data in ascending order)",
        # against the pivot form with all 3 other components (12 slots)
        "frac_issue_slots_dense_pivot": evals * ops_per_eval(4, "pivot") / PEAK_LANE_OPS}
    del th, l
    for logN in (17, 20, 24):
        N = 1 << logN
        with torch.cuda.stream(s):
            logw0 = torch.as_tensor(lognormal_logw(N, seed=logN)).cuda()
            logw = logw0.clone()
            l = torch.as_tensor(lognormal_logw(N, seed=logN + 100)).cuda()
            W = torch.empty_like(logw)
            lz = torch.zeros(1, dtype=torch.float64, device="cuda")
            ess = torch.zeros(1, dtype=torch.float64, device="cuda")
        ctx.reserve(N, 4)
        rw = time_launches(torch, s, lambda i: smc.smc_reweight(ctx, logw, l, 1e-3, W=W, logZ=lz,
                                                              ess=ess, stream=s), reps)
        with torch.cuda.stream(s):
            th_in = torch.randn((4, N), dtype=torch.float64, device="cuda")
            th_out = torch.empty_like(th_in)
            l_out = torch.empty_like(l)
            idx = torch.empty(N, dtype=torch.int32, device="cuda")
            lw2 = torch.empty_like(logw)
            smc.smc_reweight(ctx, logw0.clone(), torch.zeros_like(l), 0.0, W=W, stream=s)
        rs = time_launches(torch, s, lambda i: smc.smc_resample_systematic(
            ctx, W, 11, 3, idx=idx, theta_in=th_in, theta_out=th_out, l_in=l, l_out=l_out,
            logw=lw2, stream=s), reps)
        ctx.check(s)
        out[f"reweight_N{N}"] = {"us": rw * 1e3, "GBps": 40.0 * N / (rw * 1e-3) / 1e9,
                                 "frac_hbm": 40.0 * N / (rw * 1e-3) / 1e9 / HBM_PEAK_GBS}
        out[f"resample_gather_N{N}"] = {"us": rs * 1e3, "GBps": 100.0 * N / (rs * 1e-3) / 1e9,
                                        "frac_hbm": 100.0 * N / (rs * 1e-3) / 1e9 / HBM_PEAK_GBS}
        del th_in, th_out, l_out, idx, lw2, logw, logw0, l, W
    return out


def paper_tables(smc, torch, ctx):
    """The paper's own SMC-sampler and population-MCMC runs, whole runs timed
    end to end (prior draws, initial likelihoods, every step; FP32 likelihood):
    uniform prior on [-10, 10]^4, sigma = 0.55 as a scale, m = 100 observations,
    N(0, I) random walk. SMC: 200 steps of (t/200)^2, 10 moves per step, ESS < N/2
    resampling. Population MCMC: beta_i = (i/M)^2, random parity with the wrap
    pair, 8192 iterations, 64 per graph replay (small populations run a
    replay's iterations in one single-workgroup launch). Each shape's launch is
    autotuned first (untimed)."""
    import numpy as np
    from paper_0905_2441_amd import autotune
    from workloads import beta_schedule, make_data, pt_betas
    from workloads.configs import paper_mode
    out = {"smc": {}, "pt": {}}
    for N in sorted(PAPER_GTX280_S["smc"]):
        cfg = paper_mode(N)
        y = make_data(cfg)
        betas = beta_schedule(cfg.T, cfg.schedule)
        g = smc.Gmm.equal_weights(cfg.k, cfg.d, cfg.sigma2, prior=cfg.prior, prior_a=cfg.prior_a,
                                  prior_b=cfg.prior_b)
        ctx.set_launch_table(autotune.make_rules(ctx, [(cfg.k, cfg.d, cfg.n, N, "fp32")], reps=10,
                                                 exact=True))
        s = smc.SMCSampler(ctx, g, y, N, betas, cfg.step_sd, cfg.n_moves, cfg.run_seed,
                           ess_frac=cfg.ess_frac, prec="fp32")
        s.run(graph=True, steps_per_graph=STEPS_PER_GRAPH)          # capture and warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.init()
        s.advance(cfg.T, graph=True, steps_per_graph=STEPS_PER_GRAPH)
        s.stream.synchronize()
        dt = time.perf_counter() - t0
        r = s.results()
        census = smc.mode_census(r["theta"], r["W"])
        shares = np.array(list(census.values()))
        out["smc"][N] = {"s": dt, "gtx280_s": PAPER_GTX280_S["smc"][N],
                         "speedup_vs_gtx280": PAPER_GTX280_S["smc"][N] / dt,
                         "evals_per_s": cfg.T * cfg.n_moves * N * cfg.n / dt,
                         "resamples": r["resamples"], "log_Z": r["logZ"],
                         "modes_with_1pct": int(np.sum(shares >= 0.01)),
                         "largest_mode_share": float(shares.max())}
        log(f"[bench] paper SMC N={N}: {dt * 1e3:.1f} ms "
            f"({PAPER_GTX280_S['smc'][N] / dt:.0f}x the GTX 280)")
    cfg = paper_mode(8192)
    y = make_data(cfg)
    g = smc.Gmm.equal_weights(cfg.k, cfg.d, cfg.sigma2, prior=cfg.prior, prior_a=cfg.prior_a,
                              prior_b=cfg.prior_b)
    iters = 8192
    for M in sorted(PAPER_GTX280_S["pt"]):
        ctx.set_launch_table(autotune.make_rules(ctx, [(cfg.k, cfg.d, cfg.n, M, "fp32")], reps=10,
                                                 exact=True))
        s = smc.PTSampler(ctx, g, y, pt_betas(M, 2), cfg.step_sd, 301, parity_mode=1, wrap=True,
                          prec="fp32")
        s.run(2 * PT_ITERS_PER_GRAPH, graph=True, iters_per_graph=PT_ITERS_PER_GRAPH)  # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.init()
        s.advance(iters, graph=True, iters_per_graph=PT_ITERS_PER_GRAPH)
        s.stream.synchronize()
        dt = time.perf_counter() - t0
        r = s.results()
        out["pt"][M] = {"s": dt, "gtx280_s": PAPER_GTX280_S["pt"][M],
                        "speedup_vs_gtx280": PAPER_GTX280_S["pt"][M] / dt,
                        "evals_per_s": iters * M * cfg.n / dt, "swaps": r["swaps"]}
        if M <= 2048:
            # untimed: a longer run recording the beta = 1 chain after every
            # iteration, for the iterations it takes to visit all 24 modes
            long = 8 * iters
            s = smc.PTSampler(ctx, g, y, pt_betas(M, 2), cfg.step_sd, 301, parity_mode=1,
                              wrap=True, prec="fp32", record_chain=M - 1, record_iters=long)
            rr = s.run(long, graph=True, iters_per_graph=STEPS_PER_GRAPH)
            out["pt"][M]["traversal_iters"] = smc.traversal_time(rr["chain"])
            out["pt"][M]["traversal_run"] = long
        log(f"[bench] paper PT M={M}: {dt * 1e3:.1f} ms "
            f"({PAPER_GTX280_S['pt'][M] / dt:.0f}x the GTX 280)")
    ctx.set_launch_table([])
    return out


def fsv_runs(smc, torch, ctx):
    """The paper's particle filter for the factor stochastic-volatility model:
    m = 5, k = 3, T = 200 simulated observations, FP64, whole runs timed end to end
    at the paper's N and at 2^20 (ten filter steps per graph)."""
    from workloads.fsv import PAPER_FSV, simulate
    _, y = simulate(PAPER_FSV, 200, 7)
    out = {}
    for N in sorted(PAPER_GTX280_S["fsv"]) + [1 << 20]:
        f = smc.FSVFilter(ctx, PAPER_FSV, y, N, seed=3)
        f.run(graph=True, steps_per_graph=STEPS_PER_GRAPH)             # capture and warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        f.init()
        f.advance(f.T, graph=True, steps_per_graph=STEPS_PER_GRAPH)
        f.stream.synchronize()
        dt = time.perf_counter() - t0
        r = f.results()
        ref = PAPER_GTX280_S["fsv"].get(N)
        out[N] = {"s": dt, "us_per_step": dt / f.T * 1e6, "particle_steps_per_s": N * f.T / dt,
                  "loglik": r["loglik"], "resamples": r["resamples"],
                  "gtx280_s": ref, "speedup_vs_gtx280": (ref / dt) if ref else None}
        log(f"[bench] fsv N={N}: {dt * 1e3:.2f} ms" + (f" ({ref / dt:.0f}x the GTX 280)" if ref else ""))
    return out


def other_workload(args):
    """Secondary measurements (same JSON shape, no CPU baseline)."""
    import torch
    import paper_0905_2441_amd as smc
    from workloads import CONFIGS, beta_schedule, make_data

    if args.workload == "fsv_pf":
        torch.cuda.set_device(0)
        ctx = smc.Context(0)
        r = fsv_runs(smc, torch, ctx)
        out = {"metric": "whole-run seconds of the factor stochastic-volatility particle filter",
               "n_gpus": 1, "data": "synthetic", "dtype": "f64",
               "config": {"workload": "fsv_pf", "m": 5, "k": 3, "T": 200}, "fsv": r}
        print(json.dumps(out), flush=True)
        return

    if args.workload == "paper_tables":
        torch.cuda.set_device(0)
        ctx = smc.Context(0)
        r = paper_tables(smc, torch, ctx)
        out = {"metric": "whole-run seconds of the paper's SMC-sampler and population-MCMC runs",
               "n_gpus": 1, "data": "synthetic", "dtype": "f32",
               "config": {"workload": "paper_tables"}, "paper_tables": r}
        print(json.dumps(out), flush=True)
        return

    if args.workload == "probes":
        torch.cuda.set_device(0)
        ctx = smc.Context(0)
        r = probes(smc, torch, ctx, max(10, args.steps))
        out = {"metric": "roofline probes (kernel time per call; algorithmic evals or bytes)",
               "n_gpus": 1, "steps": max(10, args.steps), "warmup": 1, "data": "synthetic",
               "config": {"workload": "probes"}, "probes": r}
        print(json.dumps(out), flush=True)
        return

    if args.workload == "batched_256runs":
        torch.cuda.set_device(0)
        ctx = smc.Context(0)
        r = time_batched(smc, torch, ctx, "fp32", args.steps, args.warmup,
                         keep_state=not args.no_cpu_baseline, tune_batch=not args.no_tune)
        oracle_error = None
        if not args.no_cpu_baseline:
            log("[bench] error of the batched runs against the oracle ...")
            b = r["sampler"]
            order = sorted(range(b.R), key=lambda i: b.Ns[i] * b.ns[i])
            big = max(range(b.R), key=lambda i: b.Ns[i] * b.ns[i])
            oracle_error = batched_oracle_error(b, r["datas"], r["betas"], r["final"],
                                                r["replay"], order[:3] + [big])
            log(f"[bench] oracle error: {json.dumps(oracle_error)}")
            del r["sampler"], b
        r64 = time_batched(smc, torch, ctx, "fp64", max(2, args.steps // 5), 1,
                           tune_batch=not args.no_tune)
        out = {"metric": "particle×datum loglik evals/s; ms per SMC tempering step, FP32/batched vs FP64",
               "value": r["evals_per_step"] / (r["ms_per_step"] * 1e-3), "unit": "evals/s",
               "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
               "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak",
               "vs_baseline": None, "dtype": "f32", "data": "synthetic",
               "config": {"workload": "batched_256runs", "R": r["R"], "N_total": r["N_total"],
                          "n_total": r["n_total"], "evals_per_step": r["evals_per_step"],
                          "launch": {"fp32": r["launch_table"] or "built-in",
                                     "fp64": r64["launch_table"] or "built-in"}},
               "fp64_ms_per_step": r64["ms_per_step"],
               "fp32_over_fp64_speedup": r64["ms_per_step"] / r["ms_per_step"],
               "oracle_error": oracle_error}
        print(json.dumps(out), flush=True)
        return

    cfg = CONFIGS[args.workload]
    y = make_data(cfg)
    torch.cuda.set_device(0)
    ctx = smc.Context(0)
    g = smc.Gmm.equal_weights(cfg.k, cfg.d, cfg.sigma2, prior=cfg.prior, prior_a=cfg.prior_a,
                              prior_b=cfg.prior_b)
    evals = cfg.N * cfg.n * cfg.n_moves
    out = {"metric": "particle×datum loglik evals/s; ms per SMC tempering step, FP32/batched vs FP64",
           "unit": "evals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "data": "synthetic",
           "config": {"workload": cfg.name, "k": cfg.k, "d": cfg.d, "n": cfg.n, "N": cfg.N}}
    if cfg.sampler == "pt":
        out["config"]["launch"] = tune(ctx, cfg, ["fp32", "fp64"], args.no_tune)
        r = time_pt(smc, torch, ctx, cfg, g, y, "fp32", args.steps, args.warmup)
        r64 = time_pt(smc, torch, ctx, cfg, g, y, "fp64", max(5, args.steps // 5), 2)
        out.update(value=evals / (r["ms_per_step"] * 1e-3), ms_per_step=r["ms_per_step"],
                   dtype="f32", fp64_ms_per_step=r64["ms_per_step"],
                   fp32_over_fp64_speedup=r64["ms_per_step"] / r["ms_per_step"],
                   swaps=r["swaps"], accepted=r["accepted"])
        out["config"]["step"] = "one PT iteration: RW-MH per chain + exchanges (alternating parity)"
        if not args.no_cpu_baseline:
            log("[bench] error of the population-MCMC run against the oracle ...")
            out["oracle_error"] = pt_oracle_error(smc, ctx, cfg, g, y, "fp32", r)
            log(f"[bench] oracle error: {json.dumps(out['oracle_error'])}")
    else:
        betas = beta_schedule(cfg.T, cfg.schedule)
        precs = list(cfg.precisions)
        if cfg.d > 1 and "fp32" not in precs:
            precs.append("fp32")
        res = {}
        out["config"]["launch"] = tune(ctx, cfg, precs, args.no_tune)
        for prec in precs:
            steps = args.steps if prec != "fp64" else max(5, args.steps // 5)
            res[prec] = time_precision(smc, torch, ctx, cfg, g, y, betas, prec, steps, args.warmup)
            log(f"[bench] {cfg.name} {prec}: {res[prec]['ms_per_step']:.4f} ms/step, "
                f"move kernels {res[prec]['kernel_ms']:.4f} ms")
        fast = precs[0]
        out.update(value=evals / (res[fast]["ms_per_step"] * 1e-3),
                   ms_per_step=res[fast]["ms_per_step"], dtype={"fp64": "f64", "fp32": "f32",
                                                               "bf16x3": "bf16x3+f32"}[fast],
                   per_precision={p: {"ms_per_step": r["ms_per_step"], "move_ms": r["kernel_ms"],
                                      "move_evals_per_s": evals / (r["kernel_ms"] * 1e-3)}
                                  for p, r in res.items()})
        if "fp64" in res and fast != "fp64":
            out["fp64_ms_per_step"] = res["fp64"]["ms_per_step"]
            out["fast_over_fp64_speedup"] = res["fp64"]["ms_per_step"] / res[fast]["ms_per_step"]
        if not args.no_cpu_baseline:
            log(f"[bench] error of the {cfg.name} runs against the oracle ...")
            if cfg.d > 1:
                out["oracle_error"] = ddim_oracle_error(y, cfg, res)
            else:
                out["oracle_error"] = small_run_oracle_error(smc, ctx, cfg, g, y, betas, fast)
            log(f"[bench] oracle error: {json.dumps(out['oracle_error'])}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
